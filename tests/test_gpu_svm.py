"""GPU parity of the kernel SVM of Exp. 6 (Sec. 5): ``nnca_svm_train`` and
``nnca_svm_decision`` through the C ABI against the oracle's trainer.

* the same step count of projected gradient ascent from zero with the same
  step gives the same iterate (every entry to 1e-10 of the box bound), the
  same free support vectors and the same bias; the step the library picks
  (power method) equals the oracle's;
* the decision function at the held-out points (a general handle, targets
  = test points, sources = training points) and at the training points
  (the symmetric handle) equals the oracle's;
* at the paper's 2D size (M = 5625, 85 % for training) the trainer stops
  by its rule and classifies the held-out points; repeated runs are bit
  identical; the mixed form tracks the FP64 one;
* argument errors.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_14832_amd import nnca  # noqa: E402
from paper_2203_14832_amd.workloads import svm_dataset  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# the two 2D datasets of Exp. 6: "Matern" exp(-r) and the Gaussian exp(-r^2)
DATASETS = [("exp_r", "disk"), ("gauss", "wave")]
TOL = 1e-10   # ACA tolerance of the parity problems
LAM, BETA = 1.0, 1.0


@pytest.mark.parametrize("kind,rule", DATASETS)
def test_train_and_decision_parity(orc, kind, rule):
    P, y, Q, yq = svm_dataset(3000, 2, rule)
    n = P.shape[0]
    print("svm parity", kind, rule, n, Q.shape[0], flush=True)
    O = orc.H2(orc.Tree(P, 64), kind, TOL)
    eta = orc.svm_step_size(O.matvec, n, BETA)
    a_o, b_o, it_o, _ = orc.svm_train(O.matvec, y, LAM, BETA, eta, tol=0.0, max_iter=300)
    OG = orc.H2General(orc.Tree2(Q, P, 64), kind, TOL)
    f_o = orc.svm_decision(OG.matvec, y, a_o, b_o)
    ft_o = orc.svm_decision(O.matvec, y, a_o, b_o)

    G = nnca.H2Matrix(P, kind, TOL, 64)
    a_g, b_g, it_g, eta_g = G.svm_train(y, LAM, BETA, eta=eta, tol=0.0, max_iter=300)
    a_g = a_g.cpu().numpy()
    assert it_g == it_o == 300 and eta_g == eta
    assert np.abs(a_g - a_o).max() <= 1e-10 * LAM
    free_o = (a_o > 0) & (a_o < LAM)
    np.testing.assert_array_equal((a_g > 0) & (a_g < LAM), free_o)
    assert free_o.sum() >= 10 and (a_o == 0).sum() >= 10
    assert abs(b_g - b_o) <= 1e-10
    GG = nnca.H2General(Q, P, kind, TOL, 64)
    f_g = GG.svm_decision(y, a_g, b_g).cpu().numpy()
    assert np.abs(f_g - f_o).max() <= 1e-9 * max(1.0, np.abs(f_o).max())
    ft_g = G.svm_decision(y, a_g, b_g).cpu().numpy()
    assert np.abs(ft_g - ft_o).max() <= 1e-9 * max(1.0, np.abs(ft_o).max())
    # the library's own step: the power method on its H2 operator
    _, _, it0, eta_auto = G.svm_train(y, LAM, BETA, eta=0.0, max_iter=0)
    assert it0 == 0 and abs(eta_auto - eta) <= 1e-9 * eta


@pytest.mark.parametrize("kind,rule", DATASETS)
def test_paper_size_converges_and_classifies(kind, rule):
    # M = 5625 points of Exp. 6 in 2D, 85 % for training
    P, y, Q, yq = svm_dataset(5625, 2, rule)
    print("svm paper size", kind, rule, P.shape[0], flush=True)
    G = nnca.H2Matrix(P, kind, 1e-8, 64)
    a, b, it, eta = G.svm_train(y, LAM, BETA, tol=1e-4, max_iter=20000)
    assert it < 20000
    a2, b2, it2, _ = G.svm_train(y, LAM, BETA, tol=1e-4, max_iter=20000)
    assert it2 == it and b2 == b and torch.equal(a, a2)
    GG = nnca.H2General(Q, P, kind, 1e-8, 64)
    f = GG.svm_decision(y, a, b).cpu().numpy()
    acc = [np.mean(np.sign(f[yq == c]) == c) for c in (1.0, -1.0)]
    print("accuracy per class", acc, "steps", it)
    assert min(acc) >= 0.9, acc
    # mixed-precision products track the FP64 ones
    am, bm, _, _ = G.svm_train(y, LAM, BETA, eta=eta, tol=0.0, max_iter=300, precision="mixed")
    a3, b3, _, _ = G.svm_train(y, LAM, BETA, eta=eta, tol=0.0, max_iter=300)
    assert (am - a3).abs().max().item() <= 1e-5 * LAM


def test_small_and_warm_start(orc):
    # a single leaf (dense near field only) and a warm start from a given
    # iterate: 7 + 5 steps equal 12
    P, y, _, _ = svm_dataset(40, 2, "disk")
    ap = lambda v: orc.direct(P, v, "exp_r")
    eta = orc.svm_step_size(ap, P.shape[0], BETA)
    a_o, b_o, _, _ = orc.svm_train(ap, y, LAM, BETA, eta, tol=0.0, max_iter=12)
    G = nnca.H2Matrix(P, "exp_r", 1e-10, 64)
    a7, _, _, _ = G.svm_train(y, LAM, BETA, eta=eta, tol=0.0, max_iter=7)
    a12, b12, it, _ = G.svm_train(y, LAM, BETA, eta=eta, tol=0.0, max_iter=5, alpha0=a7)
    assert it == 5
    assert np.abs(a12.cpu().numpy() - a_o).max() <= 1e-12
    assert abs(b12 - b_o) <= 1e-12


def test_argument_errors():
    P, y, Q, _ = svm_dataset(200, 2, "disk")
    G = nnca.H2Matrix(P, "exp_r", 1e-8, 64)
    for kw in (dict(lam=0.0), dict(lam=float("inf")), dict(beta=-1.0), dict(tol=-1.0), dict(max_iter=-1),
               dict(eta=float("nan"))):
        with pytest.raises(nnca.NncaError) as e:
            G.svm_train(y, **kw)
        assert e.value.status == 1, kw
    yd = torch.tensor(y, device="cuda")
    L = nnca.lib()
    # alpha aliasing y
    st = L.nnca_svm_train(G._h, C.c_void_p(yd.data_ptr()), C.c_void_p(yd.data_ptr()), 1.0, 1.0, 0.0, 1e-8, 10, 0,
                          None, None, None, None)
    assert st == 1
    GG = nnca.H2General(Q, P, "exp_r", 1e-8, 64)
    with pytest.raises(nnca.NncaError) as e:
        GG.svm_train(np.ones(Q.shape[0]))
    assert e.value.status == 4   # training needs the symmetric handle
    f = torch.zeros(Q.shape[0], dtype=torch.float64, device="cuda")
    st = L.nnca_svm_decision(GG._h, C.c_void_p(yd.data_ptr()), C.c_void_p(yd.data_ptr()), float("nan"),
                             C.c_void_p(f.data_ptr()), 0, None)
    assert st == 1
