"""Pins of the regularised kernels of Exp. 1-4 (Sec. 5) in the oracle, and of
the H2 matvec with them on the tensor-product Chebyshev grids of Exp. 2 and 4:
* the method's kernel (project-written log, IEEE sqrt and division) against
  the closed forms with the C library at chosen radii, both branches;
* continuity at r = a (both branches give 1) and K(0) = 0;
* the H2 product against the direct sum, error falling with the tolerance;
  tol = 0 reproduces the dense product."""
import math

import numpy as np
import pytest

from paper_2203_14832_amd.workloads import chebyshev_grid

A = 1e-4


def k1(r, a=A):
    return 0.0 if r == 0 else (r * (math.log(r) - 1) / (a * (math.log(a) - 1)) if r < a else math.log(r) / math.log(a))


def k2(r, a=A):
    return 0.0 if r == 0 else (r / a if r < a else a / r)


@pytest.mark.parametrize("kind,f,d", [("log_reg", k1, 2), ("inv_reg", k2, 2), ("inv_reg", k2, 3)])
def test_regularised_kernel_values(orc, kind, f, d):
    rng = np.random.default_rng(60)
    for r in [0.0, 1e-7, 3e-5, 0.999 * A, A, 1.001 * A, 2e-4, 0.01, 0.5, 1.7]:
        u = rng.standard_normal(d)
        u /= np.linalg.norm(u)
        x = rng.uniform(-1, 1, d)
        y = x + r * u
        rr = float(np.linalg.norm(y - x))
        got = orc.kernel_eval(kind, x, y, A)
        assert got == pytest.approx(f(rr), rel=2e-13, abs=1e-300), (kind, r)
    # continuity at r = a: both branches give 1
    x = np.zeros(d)
    y = np.zeros(d)
    y[0] = A
    assert orc.kernel_eval(kind, x, y, A) == pytest.approx(1.0, rel=1e-15)
    assert orc.kernel_eval(kind, x, x, A) == 0.0


@pytest.mark.parametrize("kind,d,n_axis,leaf", [("log_reg", 2, 48, 32), ("inv_reg", 3, 13, 32)])
def test_chebyshev_h2_against_direct(orc, kind, d, n_axis, leaf):
    p = chebyshev_grid(n_axis, d)
    x = np.random.default_rng(61).standard_normal(p.shape[0])
    yd = orc.direct(p, x, kind, A)
    T = orc.Tree(p, leaf)
    errs = []
    for tol in (1e-3, 1e-5, 1e-7, 1e-9):
        y = orc.H2(T, kind, tol, h=A).matvec(x)
        errs.append(np.linalg.norm(y - yd) / np.linalg.norm(yd))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-7
    y0 = orc.H2(T, kind, 0.0, h=A).matvec(x)
    assert np.linalg.norm(y0 - yd) <= 1e-10 * np.linalg.norm(yd)
