"""Pins of the oracle's restarted GMRES (the solver of the integral-equation
experiment, Exp. 5 of Sec. 5): it is checked against a direct dense solve,
against the exact termination of Krylov methods on an operator whose
minimal polynomial has degree three, and on the Nystrom system built with
the oracle's own H2 matvec."""
import numpy as np
import pytest

from paper_2203_14832_amd.workloads import nystrom_grid


def test_dense_against_direct_solve(orc):
    rng = np.random.default_rng(50)
    n = 80
    M = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, it, rr = orc.gmres(lambda v: M @ v, b, tol=1e-12, restart=n)
    xs = np.linalg.solve(M, b)
    assert rr <= 1e-12 and it <= n
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    # restarted: more applications, the same solution
    x5, it5, rr5 = orc.gmres(lambda v: M @ v, b, tol=1e-12, restart=5, max_iter=2000)
    assert rr5 <= 1e-12 and it5 >= it
    assert np.linalg.norm(x5 - xs) <= 1e-10 * np.linalg.norm(xs)


def test_exact_termination(orc):
    # I + (rank 2): the minimal polynomial has degree 3, so full GMRES
    # reaches the solution in at most three applications
    rng = np.random.default_rng(51)
    n = 200
    Uu, Vv = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
    M = np.eye(n) + Uu @ Vv.T / n
    b = rng.standard_normal(n)
    x, it, rr = orc.gmres(lambda v: M @ v, b, tol=1e-13, restart=50)
    assert it <= 3 and rr <= 1e-12


def test_zero_rhs_and_iteration_cap(orc):
    M = np.diag(np.arange(1.0, 51.0))
    x, it, rr = orc.gmres(lambda v: M @ v, np.zeros(50))
    assert it == 0 and not x.any()
    x, it, rr = orc.gmres(lambda v: M @ v, np.ones(50), tol=1e-14, max_iter=4, restart=10)
    assert it == 4 and rr > 1e-14


def test_nystrom_with_oracle_h2(orc):
    # (I + w A~) sigma = f with f formed by the same operator: GMRES recovers
    # sigma to about the tolerance times the conditioning
    p, w, sigma = nystrom_grid(8)
    T = orc.Tree(p, 16)
    H = orc.H2(T, "inv_r", 1e-9)
    op = lambda v: v + w * H.matvec(v)
    f = op(sigma)
    x, it, rr = orc.gmres(op, f, tol=1e-10, restart=30)
    assert rr <= 1e-10 and it <= 30
    assert np.linalg.norm(x - sigma) <= 1e-8 * np.linalg.norm(sigma)
    # the H2 operator agrees with the dense Nystrom operator to the ACA tolerance
    fd = sigma + w * orc.direct(p, sigma, "inv_r")
    assert np.linalg.norm(f - fd) <= 1e-7 * np.linalg.norm(fd)
