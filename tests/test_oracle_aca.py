"""Pins of the oracle's partially pivoted ACA (Sec. 2.2.1) and of the
transfer operators taken from its by-products (Remark in Sec. 2.3.2).

* an independent formulation: ACA on the explicit residual matrix;
* exact cases: a block of known rank, tol = 0;
* invariants of cross approximation: interpolation of the pivot rows and
  columns, triangular factors, identity rows of the transfer operator;
* the transfer operator equals A(:, J) A(I, J)^{-1} computed by LAPACK;
* the error is never below the SVD optimum of the same rank (Eckart-Young)
  and stays within a small multiple of tol on well-separated blocks;
* rank bounds on well-separated 1/r blocks from the multipole expansion.
"""
import math

import numpy as np
import pytest


def dense(kind, P, Q, h=1.0):
    diff = P[:, None, :] - Q[None, :, :]
    r2 = (diff ** 2).sum(-1)
    if kind == "inv_r":
        return np.where(r2 > 0, 1 / np.sqrt(np.where(r2 > 0, r2, 1)), 0.0)
    if kind == "log_r":
        return np.where(r2 > 0, 0.5 * np.log(np.where(r2 > 0, r2, 1)), 0.0)
    if kind == "gauss":
        return np.exp(-r2 / (h * h))
    if kind == "poly2":
        return (1 + P @ Q.T) ** 2
    raise ValueError(kind)


def aca_explicit(A, tol):
    """Partially pivoted ACA written on the explicit residual matrix."""
    m, n = A.shape
    R = A.copy()
    ru, cu = np.zeros(m, bool), np.zeros(n, bool)
    I, J, us, vs = [], [], [], []
    nrm2 = 0.0
    i = 0
    while len(I) < min(m, n):
        row = np.where(cu, 0.0, R[i])
        if np.abs(row).max() == 0.0:
            ru[i] = True
            free = np.where(~ru)[0]
            if free.size == 0:
                break
            i = int(free[0])
            continue
        j = int(np.argmax(np.abs(row)))
        v = row / row[j]
        u = np.where(ru, 0.0, R[:, j])
        R = R - np.outer(u, v)
        ru[i] = True
        cu[j] = True
        nrm2 = nrm2 + 2 * sum((u @ ul) * (vl @ v) for ul, vl in zip(us, vs)) + (u @ u) * (v @ v)
        I.append(i); J.append(j); us.append(u); vs.append(v)
        if np.linalg.norm(u) * np.linalg.norm(v) <= tol * np.sqrt(max(nrm2, 0.0)):
            break
        if len(I) == min(m, n):
            break
        cand = np.where(ru, -1.0, np.abs(u))
        i = int(np.argmax(cand))
        if cand[i] < 0:
            break
    return np.array(I), np.array(J), np.array(us).T, np.array(vs)


def clusters(rng, d, m, n, sep):
    P = rng.uniform(-0.5, 0.5, (m, d))
    Q = rng.uniform(-0.5, 0.5, (n, d))
    Q[:, 0] += sep
    return P, Q


@pytest.mark.parametrize("kind,d,sep,tol", [("inv_r", 3, 2.5, 1e-6), ("inv_r", 2, 3.0, 1e-9),
                                            ("log_r", 2, 2.5, 1e-8), ("gauss", 3, 1.0, 1e-7)])
def test_matches_explicit_residual_formulation(orc, kind, d, sep, tol):
    rng = np.random.default_rng(0)
    P, Q = clusters(rng, d, 70, 90, sep)
    I, J, U, V, Cm = orc.aca_block(P, Q, kind, tol, h=0.7)
    # the same kernel entries as the oracle (its kernel functions have pins
    # of their own), so that only the ACA logic is compared
    A = np.array([[orc.kernel_eval(kind, p, q, 0.7) for q in Q] for p in P])
    assert np.abs(A - dense(kind, P, Q, 0.7)).max() <= 1e-14 * np.abs(A).max()
    I2, J2, U2, V2 = aca_explicit(A, tol)
    assert list(I) == list(I2) and list(J) == list(J2)
    assert np.abs(U - U2).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(V - V2).max() <= 1e-13


def test_known_rank_block(orc):
    # (1 + x.y)^2 in 3D spans the 10 monomials of degree <= 2: rank 10
    rng = np.random.default_rng(1)
    P, Q = rng.uniform(-1, 1, (60, 3)), rng.uniform(-1, 1, (80, 3))
    I, J, U, V, Cm = orc.aca_block(P, Q, "poly2", 1e-10)
    A = dense("poly2", P, Q)
    assert len(I) <= 11
    assert np.linalg.norm(A - U @ V) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("kind,d", [("gauss", 3), ("inv_r", 3), ("log_r", 2)])
def test_zero_tolerance_is_exact(orc, kind, d):
    rng = np.random.default_rng(2)
    P, Q = rng.uniform(-1, 1, (25, d)), rng.uniform(-1, 1, (40, d))
    I, J, U, V, Cm = orc.aca_block(P, Q, kind, 0.0, h=0.3)
    A = dense(kind, P, Q, 0.3)
    assert len(I) == 25
    assert np.linalg.norm(A - U @ V) <= 1e-12 * np.linalg.norm(A)
    # full row rank: every row is a pivot, the operator is a permutation
    assert sorted(I) == list(range(25))
    perm = np.zeros((25, 25))
    perm[I, np.arange(25)] = 1.0
    np.testing.assert_array_equal(Cm, perm)


@pytest.mark.parametrize("kind,d,sep", [("inv_r", 3, 2.0), ("log_r", 2, 2.0), ("gauss", 2, 0.5)])
def test_cross_invariants_and_transfer_operator(orc, kind, d, sep):
    rng = np.random.default_rng(3)
    P, Q = clusters(rng, d, 50, 120, sep)
    tol = 1e-8
    I, J, U, V, Cm = orc.aca_block(P, Q, kind, tol, h=0.5)
    A = dense(kind, P, Q, 0.5)
    k = len(I)
    Ak = U @ V
    scale = np.abs(A).max()
    # interpolation of the pivot rows and columns
    assert np.abs(Ak[I] - A[I]).max() <= 1e-12 * scale
    assert np.abs(Ak[:, J] - A[:, J]).max() <= 1e-12 * scale
    # L = U(I,:) lower triangular, V(:,J) unit upper triangular -- exactly
    L = U[I]
    assert (np.triu(L, 1) == 0).all()
    VJ = V[:, J]
    assert (np.tril(VJ, -1) == 0).all() and (np.diag(VJ) == 1).all()
    # transfer operator: identity rows at the pivots, and A(:,J) A(I,J)^{-1}
    np.testing.assert_array_equal(Cm[I], np.eye(k))
    ref = np.linalg.solve(A[np.ix_(I, J)].T, A[:, J].T).T
    cond = np.linalg.cond(A[np.ix_(I, J)])
    assert np.abs(Cm - ref).max() <= 1e-15 * cond * max(1.0, np.abs(ref).max()) * 10


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7, 1e-9])
def test_error_between_svd_optimum_and_tolerance(orc, tol):
    rng = np.random.default_rng(4)
    P, Q = clusters(rng, 3, 80, 200, 2.5)
    I, J, U, V, Cm = orc.aca_block(P, Q, "inv_r", tol)
    A = dense("inv_r", P, Q)
    k = len(I)
    err = np.linalg.norm(A - U @ V)
    s = np.linalg.svd(A, compute_uv=False)
    assert err >= np.sqrt((s[k:] ** 2).sum()) * (1 - 1e-9)
    assert err <= 10 * tol * np.linalg.norm(A)


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_rank_bound_well_separated(orc, tol):
    # Clusters in balls of radius a, centres D apart: the multipole expansion
    # of 1/r truncated at order p has (p+1)^2 terms and relative error
    # ~ rho^(p+1), rho = 2a/(D-a); ACA (not optimal) gets a little slack.
    rng = np.random.default_rng(5)
    a, D = 0.5, 3.0
    def ball(n):
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        return v * a * rng.uniform(0, 1, (n, 1)) ** (1 / 3)
    P, Q = ball(300), ball(300) + np.array([D, 0, 0])
    I, J, U, V, Cm = orc.aca_block(P, Q, "inv_r", tol)
    rho = 2 * a / (D - a)
    p = math.ceil(math.log(tol) / math.log(rho))
    assert len(I) <= (p + 1) ** 2 + 4
    assert len(I) <= min(P.shape[0], Q.shape[0])


def test_zero_rows_and_exhaustion(orc):
    # All column points coincide with the first row point: row 0 is exactly
    # zero (K = 0 at r = 0) and is skipped without a cross; the block is then
    # exactly rank one, every later residual row is exactly zero and the
    # rows run out with k = 1, even at tol = 0.
    rng = np.random.default_rng(6)
    q = np.array([0.1, 0.2, 0.3])
    P = np.vstack([q, rng.uniform(2, 3, (9, 3))])
    Q = np.tile(q, (30, 1))
    I, J, U, V, Cm = orc.aca_block(P, Q, "inv_r", 0.0)
    A = dense("inv_r", P, Q)
    assert list(I) == [1] and list(J) == [0]
    np.testing.assert_array_equal(U @ V, A)
    Q = rng.uniform(-1, 1, (30, 3)) + np.array([3.0, 0, 0])
    # fewer columns than rows: the rank stops at n
    I, J, U, V, Cm = orc.aca_block(rng.uniform(-1, 1, (20, 3)), Q[:4], "inv_r", 0.0)
    assert len(I) == 4
