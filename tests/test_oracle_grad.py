"""Pins of the oracle's length-scale derivative (Gaussian kernel, pivots
frozen) against what the definitions fix:

* the frozen re-evaluation C_B(h) = K_h(t~, J) K_h(I, J)^{-1} (a dense solve
  with partial pivoting) reproduces, at the build's own h, the operators the
  ACA by-products gave (Remark in Sec. 2.3.2) -- two different computations;
* the forward-mode derivative equals central finite differences of the
  frozen-pivot matvec (step 1e-4, FP64), and a Richardson-extrapolated
  difference to ~1e-9, tight enough that dropping the transfer-operator term
  dC_B (planted here, in the oracle) fails;
* the dense derivative sum_ij g_i x_j dK/dh equals torch autograd of
  g^T A(h) x in float64, and the H2 derivative approaches it as the ACA
  tolerance falls.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_14832_amd import workloads as W

H0 = 0.5


def _problem(n, leaf, tol, seed_offset=0):
    pts, x = W.workload("c4", n=n, nrhs=1, seed_offset=seed_offset)
    g = np.random.default_rng(77 + seed_offset).standard_normal(n)
    T = oracle.Tree(pts, leaf)
    H = oracle.H2(T, "gauss", tol, h=H0)
    return pts, x[:, 0], g, T, H


def _loss(H, h, x, g):
    return float(g @ H.frozen(h).matvec(x))


def _fd(H, x, g, d):
    return (_loss(H, H0 + d, x, g) - _loss(H, H0 - d, x, g)) / (2 * d)


@pytest.fixture(scope="module")
def small():
    return _problem(3000, 32, 1e-6)


def test_frozen_at_same_h_reproduces_build(small):
    pts, x, g, T, H = small
    F = H.frozen(H0)
    for l in range(H.lmin, T.kappa + 1):
        for b in range(0, T.ncell(l), max(1, T.ncell(l) // 7)):
            a, c = H.cell(l, b), F.cell(l, b)
            assert np.array_equal(a["piv"], c["piv"])
            if a["k"] == 0:
                continue
            scale = max(1.0, np.abs(a["C"]).max())
            assert np.abs(a["C"] - c["C"]).max() <= 1e-9 * scale, (l, b)
    y0, y1 = H.matvec(x), F.matvec(x)
    assert np.linalg.norm(y1 - y0) <= 1e-12 * np.linalg.norm(y0)


def test_frozen_changes_with_h(small):
    pts, x, g, T, H = small
    y0 = H.matvec(x)
    y1 = H.frozen(H0 * 1.1).matvec(x)
    assert np.linalg.norm(y1 - y0) > 1e-2 * np.linalg.norm(y0)
    ref = oracle.direct(pts, x, "gauss", h=H0 * 1.1)
    assert np.linalg.norm(y1 - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", [(3000, 32, 1e-6, 0), (4000, 64, 1e-6, 1), (2500, 16, 1e-8, 2)])
def test_grad_matches_central_differences(case):
    n, leaf, tol, so = case
    pts, x, g, T, H = _problem(n, leaf, tol, so)
    gr = H.grad_h(x, g)
    fd = _fd(H, x, g, 1e-4)
    # truncation error of the central difference is (d^2/6) L''' ; for
    # h = 0.5 and these point sets it stays below 1e-6 relative at d = 1e-4
    assert abs(gr - fd) <= 1e-6 * abs(fd)


def test_grad_richardson_detects_each_term(small):
    pts, x, g, T, H = small
    d = 1e-4
    f1, f2 = _fd(H, x, g, d), _fd(H, x, g, d / 2)
    rich = (4 * f2 - f1) / 3        # O(d^4) truncation
    gr = H.grad_h(x, g)
    tol = 1e-8 * abs(rich)
    assert abs(gr - rich) <= tol
    # planted mistakes: drop one term at a time (near field, M2L blocks,
    # transfer operators) -- every one must be visible to this pin
    for parts in (6, 5, 3):
        assert abs(H.grad_h(x, g, parts) - rich) > 100 * tol, parts
    # the three terms add up
    s = sum(H.grad_h(x, g, p) for p in (1, 2, 4))
    assert abs(s - gr) <= 1e-12 * sum(abs(H.grad_h(x, g, p)) for p in (1, 2, 4))


def test_dense_grad_equals_autograd():
    rng = np.random.default_rng(5)
    n = 400
    pts = W.draw_points("mixture", n, 3, rng)
    x, g = rng.standard_normal(n), rng.standard_normal(n)
    P = torch.tensor(pts, dtype=torch.float64)
    h = torch.tensor(H0, dtype=torch.float64, requires_grad=True)
    r2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    L = torch.tensor(g) @ (torch.exp(-r2 / h ** 2) @ torch.tensor(x))
    L.backward()
    ref = float(h.grad)
    got = oracle.dense_grad_h(pts, x, g, H0)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_grad_approaches_dense_as_tol_falls():
    pts, x, g, T, _ = _problem(3000, 32, 1e-6)
    dense = oracle.dense_grad_h(pts, x, g, H0)
    errs = []
    for tol in (1e-3, 1e-5, 1e-7, 1e-9):
        H = oracle.H2(T, "gauss", tol, h=H0)
        errs.append(abs(H.grad_h(x, g) - dense) / abs(dense))
    assert errs[-1] <= 1e-8
    assert errs[0] > errs[-1] * 100
    assert all(b <= a * 1.5 for a, b in zip(errs, errs[1:])), errs


def test_grad_rejects_other_kernels():
    pts, x = W.workload("c2", n=500, nrhs=1)
    T = oracle.Tree(pts, 32)
    H = oracle.H2(T, "inv_r", 1e-6)
    assert np.isnan(H.grad_h(x[:, 0], x[:, 0]))
    with pytest.raises(ValueError):
        H.frozen(0.5)
