"""Pins of the oracle's kernel SVM trainer (Exp. 6, Sec. 5).

* closed forms: two training points, where the maximiser of the penalised
  dual is known by hand for both label patterns and both sides of the box;
* an independent optimiser: the fixed point of the projected gradient ascent
  equals the maximiser found by scipy's L-BFGS-B from objective values alone
  (finite-difference gradients), so a wrong term or sign in the trainer's
  gradient moves the fixed point away;
* the objective against a brute-force double loop over kernel_eval;
* the step: 1 / (largest eigenvalue of K + beta n) from LAPACK;
* the KKT structure of the result: at the maximiser every free support
  vector has the same y_i - (K v)_i, namely beta sum(v), so the bias equals
  beta sum(v) and f(x_i) = y_i on the free support vectors;
* the stopping rule's limits (max_iter = 0, tol = 0).
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from paper_2203_14832_amd.workloads import svm_dataset


def dense_apply(orc, P, kind, h=1.0):
    return lambda v: orc.direct(P, v, kind, h)


def dense_matrix(orc, P, kind, h=1.0):
    n = P.shape[0]
    return np.column_stack([orc.direct(P, np.eye(n)[:, j], kind, h) for j in range(n)])


@pytest.mark.parametrize("lam", [10.0, 0.5])
@pytest.mark.parametrize("kind", ["exp_r", "gauss"])
def test_two_points_opposite_labels(orc, kind, lam):
    # y = (1, -1): by symmetry a_1 = a_2 = a, sum a y = 0, and
    # L = 2a - (1 - k) a^2 with k = K(x_1, x_2), so a = min(1 / (1 - k), lam)
    P = np.array([[0.0, 0.0], [0.8, 0.0]])
    y = np.array([1.0, -1.0])
    k = orc.kernel_eval(kind, P[0], P[1], 1.0)
    a, b, it, eta = orc.svm_train(dense_apply(orc, P, kind), y, lam=lam, beta=1.0, tol=1e-15, max_iter=100000)
    want = min(1.0 / (1.0 - k), lam)
    assert np.allclose(a, want, rtol=1e-12, atol=0), (a, want)
    f = orc.svm_decision(dense_apply(orc, P, kind), y, a, b)
    if want < lam:
        # both are free support vectors on the margin, no bias
        assert abs(b) <= 1e-12
        assert np.allclose(f, y, atol=1e-12)
    else:
        assert b == 0.0   # no free support vector
        assert np.all(f * y > 0)


@pytest.mark.parametrize("beta", [1.0, 0.25])
def test_two_points_equal_labels(orc, beta):
    # y = (1, 1): a_1 = a_2 = a and L = 2a - (1 + k) a^2 - 2 beta a^2, so
    # a = 1 / (1 + k + 2 beta): pins the penalty term, its sign and factor
    P = np.array([[0.0, 0.0], [0.0, 0.6]])
    y = np.array([1.0, 1.0])
    k = orc.kernel_eval("exp_r", P[0], P[1], 1.0)
    a, b, _, _ = orc.svm_train(dense_apply(orc, P, "exp_r"), y, lam=5.0, beta=beta, tol=1e-15, max_iter=100000)
    want = 1.0 / (1.0 + k + 2.0 * beta)
    assert np.allclose(a, want, rtol=1e-12, atol=0), (a, want)
    # the bias is beta sum(v) at the maximiser
    assert abs(b - beta * 2.0 * want) <= 1e-12


def test_objective_brute_force(orc):
    rng = np.random.default_rng(5)
    P = rng.uniform(-1.4, 1.4, (7, 2))
    y = np.where(rng.uniform(size=7) < 0.5, 1.0, -1.0)
    a = rng.uniform(0, 1, 7)
    beta = 0.7
    K = dense_matrix(orc, P, "exp_r")
    s = 0.0
    for i in range(7):
        for j in range(7):
            s += orc.kernel_eval("exp_r", P[i], P[j], 1.0) * y[i] * y[j] * a[i] * a[j]
    c = sum(a[j] * y[j] for j in range(7))
    want = sum(a) - 0.5 * s - 0.5 * beta * c * c
    assert abs(orc.svm_objective(K, y, a, beta) - want) <= 1e-13 * abs(want)


@pytest.mark.parametrize("kind", ["exp_r", "gauss"])
@pytest.mark.parametrize("beta", [1.0, 0.1])
def test_fixed_point_is_the_bounded_maximiser(orc, kind, beta):
    P, y, _, _ = svm_dataset(60, 2, "disk")
    n = P.shape[0]
    K = dense_matrix(orc, P, kind)
    a, b, it, eta = orc.svm_train(dense_apply(orc, P, kind), y, lam=1.0, beta=beta, tol=1e-13, max_iter=100000)
    assert it < 100000
    r = minimize(lambda al: -orc.svm_objective(K, y, al, beta), np.zeros(n), method="L-BFGS-B",
                 bounds=[(0.0, 1.0)] * n, options=dict(ftol=1e-15, gtol=1e-12, maxfun=200000, maxiter=100000))
    # the same maximiser (strictly concave: K + beta y y^T is positive
    # definite), up to L-BFGS-B's finite-difference accuracy
    assert np.abs(r.x - a).max() <= 1e-4
    La, Lr = orc.svm_objective(K, y, a, beta), -r.fun
    assert La >= Lr - 1e-10 * abs(Lr)
    # some free support vectors and some at each bound: the box is active
    free = (a > 0) & (a < 1.0)
    assert free.sum() >= 3 and (a == 0).sum() >= 3


@pytest.mark.parametrize("beta", [1.0, 0.1])
def test_bias_is_penalty_times_constraint_residual(orc, beta):
    P, y, _, _ = svm_dataset(80, 2, "wave")
    ap = dense_apply(orc, P, "gauss")
    a, b, it, _ = orc.svm_train(ap, y, lam=1.0, beta=beta, tol=1e-14, max_iter=200000)
    v = y * a
    kv = ap(v)
    free = (a > 0) & (a < 1.0)
    assert free.sum() >= 3
    # KKT of a free coordinate: 1 - y_i (K v)_i - beta sum(v) y_i = 0
    assert np.ptp(y[free] - kv[free]) <= 1e-8
    assert abs(b - beta * v.sum()) <= 1e-8
    f = orc.svm_decision(ap, y, a, b)
    assert np.allclose(f[free], y[free], atol=1e-8)
    # bound coordinates: the gradient points out of the box
    g = 1.0 - y * kv - beta * v.sum() * y
    assert np.all(g[a == 0.0] <= 1e-8) and np.all(g[a == 1.0] >= -1e-8)


@pytest.mark.parametrize("kind", ["exp_r", "gauss"])
def test_step_size_is_inverse_lipschitz_bound(orc, kind):
    P, y, _, _ = svm_dataset(120, 2, "disk")
    n = P.shape[0]
    lmax = np.linalg.eigvalsh(dense_matrix(orc, P, kind))[-1]
    eta = orc.svm_step_size(dense_apply(orc, P, kind), n, 0.5)
    assert abs(eta - 1.0 / (lmax + 0.5 * n)) <= 1e-10 * eta


def test_stopping_limits(orc):
    P, y, _, _ = svm_dataset(40, 2, "disk")
    ap = dense_apply(orc, P, "exp_r")
    a, b, it, _ = orc.svm_train(ap, y, max_iter=0)
    assert it == 0 and not a.any() and b == 0.0
    a, b, it, _ = orc.svm_train(ap, y, tol=0.0, max_iter=37)
    assert it == 37
    # one step from zero: alpha = clip(eta * 1, 0, lam) everywhere
    a, _, it, eta = orc.svm_train(ap, y, max_iter=1)
    assert it == 1 and np.all(a == min(eta, 1.0))


@pytest.mark.parametrize("kind,rule", [("exp_r", "disk"), ("gauss", "wave")])
def test_held_out_accuracy(orc, kind, rule):
    # the classifier separates the synthetic classes of Exp. 6 (the paper
    # reports 95.9-100 % per class on its own data)
    P, y, Q, yq = svm_dataset(1500, 2, rule)
    a, b, it, _ = orc.svm_train(dense_apply(orc, P, kind), y, lam=1.0, beta=1.0, tol=1e-6, max_iter=1000)
    f = orc.svm_decision(lambda v: orc.direct2(Q, P, v, kind), y, a, b)
    acc = np.mean(np.sign(f) == yq)
    assert acc >= 0.9, acc
