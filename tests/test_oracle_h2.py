"""Pins of the oracle's NNCA build and H2 matvec (Sec. 2.3, 3, 4, 5).

* reductions to the plain definition: a single leaf (kappa = 0) and tol = 0
  give the dense product;
* brute force: the H2 product against the dense direct sum, and the error
  falling with the ACA tolerance decade by decade (Sec. 5, Exp. 1-2);
* structure: the nested candidate sets of Sec. 2.3.2 (non-leaf rows are the
  children's pivots, far-field pivots come from the interaction-list region),
  identity rows of the transfer operators, permutations at full rank;
* symmetry of the symmetric case (Sec. 5), adjoint, linearity.
"""
import numpy as np
import pytest

from paper_2203_14832_amd.workloads import workload


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def build(orc, p, kind, tol, leaf, eta2=None, h=1.0, policy=1):
    T = orc.Tree(p, leaf, eta2=eta2)
    return T, orc.H2(T, kind, tol, h=h, policy=policy)


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 3), ("exp_r", 2)])
def test_single_leaf_is_dense(orc, kind, d):
    rng = np.random.default_rng(0)
    p, x = rng.uniform(-1, 1, (300, d)), rng.standard_normal(300)
    T, H = build(orc, p, kind, 1e-6, leaf=300, h=0.5)
    assert T.kappa == 0
    assert rel(H.matvec(x), orc.direct(p, x, kind, 0.5)) <= 1e-14


@pytest.mark.parametrize("kind,d,n", [("inv_r", 3, 3000), ("log_r", 2, 2000), ("gauss", 3, 2500),
                                      ("exp_r", 2, 2000)])
def test_zero_tolerance_is_dense(orc, kind, d, n):
    rng = np.random.default_rng(1)
    p, x = rng.uniform(-1, 1, (n, d)), rng.standard_normal(n)
    T, H = build(orc, p, kind, 0.0, leaf=16, h=0.5)
    assert T.kappa >= 3
    assert rel(H.matvec(x), orc.direct(p, x, kind, 0.5)) <= 1e-10


def test_c1_workload_against_direct_sum(orc):
    p, x = workload("c1")
    T, H = build(orc, p, "log_r", 1e-8, leaf=64)
    assert T.kappa == 4 and H.lmin == 2
    y = H.matvec(x[:, 0])
    assert rel(y, orc.direct(p, x[:, 0], "log_r")) <= 1e-6


@pytest.mark.parametrize("kind,d,n,leaf", [("log_r", 2, 4096, 32), ("inv_r", 3, 8192, 32), ("exp_r", 2, 4096, 32)])
def test_error_falls_with_tolerance(orc, kind, d, n, leaf):
    rng = np.random.default_rng(2)
    p, x = rng.uniform(-1, 1, (n, d)), rng.standard_normal(n)
    yd = orc.direct(p, x, kind)
    T = orc.Tree(p, leaf)
    errs = [rel(orc.H2(T, kind, tol).matvec(x), yd) for tol in 10.0 ** -np.arange(2, 11, 2)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-8


def _far_region_points(T, H, l, b):
    """Candidate far-field points of cell b at level l (Sec. 2.3.2 step 1)."""
    order = T.order()
    cells = T.cells(l)
    ptr, idx = T.lists(l, "il")
    out = set()
    for e in idx[ptr[b]:ptr[b + 1]]:
        if l == T.kappa:
            f, k = cells["first"][e], cells["count"][e]
            out |= set(order[f:f + k].tolist())
        else:
            ch = np.where(T.cells(l + 1)["parent"] == e)[0]
            for c in ch:
                out |= set(H.cell(l + 1, c)["piv"].tolist())
    return out


@pytest.mark.parametrize("eta2", [None, (2, 1)])
def test_nested_pivot_structure(orc, eta2):
    rng = np.random.default_rng(3)
    p = rng.uniform(-1, 1, (6000, 3))
    T, H = build(orc, p, "inv_r", 1e-6, leaf=20, eta2=eta2)
    order = T.order()
    for l in range(H.lmin, T.kappa + 1):
        cells = T.cells(l)
        for b in range(0, T.ncell(l), max(1, T.ncell(l) // 40)):
            c = H.cell(l, b)
            if l == T.kappa:
                f, k = cells["first"][b], cells["count"][b]
                assert list(c["tt"]) == list(order[f:f + k])
            else:
                ch = np.where(T.cells(l + 1)["parent"] == b)[0]
                assert list(c["tt"]) == [v for cc in ch for v in H.cell(l + 1, cc)["piv"]]
            assert c["k"] <= c["m"]
            assert set(c["piv"]) <= set(c["tt"])
            assert len(set(c["piv"])) == c["k"]
            if not c["passthrough"]:
                assert c["k"] <= c["n"]
                assert set(c["colpts"]) <= _far_region_points(T, H, l, b)
            pos = [list(c["tt"]).index(v) for v in c["piv"]]
            np.testing.assert_array_equal(c["C"][pos], np.eye(c["k"]))
            if c["k"] == c["m"]:
                assert ((c["C"] == 0) | (c["C"] == 1)).all()


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 2)])
def test_symmetry_adjoint_linearity(orc, kind, d):
    rng = np.random.default_rng(4)
    p = rng.uniform(-1, 1, (3000, d))
    T, H = build(orc, p, kind, 1e-5, leaf=24, h=0.4)
    X = rng.standard_normal((3000, 3))
    Y = H.matvec(X)
    for c in range(3):
        np.testing.assert_array_equal(Y[:, c], H.matvec(X[:, c]))
    np.testing.assert_array_equal(H.matvec(X, adjoint=True), Y)
    a = X[:, 0] @ Y[:, 1]
    b = Y[:, 0] @ X[:, 1]
    assert abs(a - b) <= 1e-12 * (abs(a) + np.linalg.norm(Y) * np.linalg.norm(X))


def test_literal_sqrt2_and_passthrough_policy(orc):
    rng = np.random.default_rng(5)
    p, x = rng.uniform(-1, 1, (5000, 3)), rng.standard_normal(5000)
    yd = orc.direct(p, x, "inv_r")
    T, H = build(orc, p, "inv_r", 1e-7, leaf=16, eta2=(2, 1))
    assert rel(H.matvec(x), yd) <= 1e-5
    T, H = build(orc, p, "inv_r", 1e-7, leaf=16, policy=0)
    assert rel(H.matvec(x), yd) <= 1e-5


def test_clustered_points_gaussian(orc):
    p, x = workload("c4", n=6000)
    T, H = build(orc, p, "gauss", 1e-8, leaf=32, h=0.5)
    assert rel(H.matvec(x[:, 0]), orc.direct(p, x[:, 0], "gauss", 0.5)) <= 1e-6


def test_degenerate_inputs(orc):
    rng = np.random.default_rng(6)
    # one point
    T, H = build(orc, np.zeros((1, 3)), "inv_r", 1e-6, leaf=1)
    assert H.matvec(np.array([2.0]))[0] == 0.0
    # all points identical: K = 0 everywhere for 1/r, K = 1 for the Gaussian
    p = np.ones((40, 3))
    x = rng.standard_normal(40)
    T, H = build(orc, p, "inv_r", 1e-6, leaf=4)
    np.testing.assert_array_equal(H.matvec(x), np.zeros(40))
    T, H = build(orc, p, "gauss", 1e-6, leaf=4)
    assert rel(H.matvec(x), np.full(40, x.sum())) <= 1e-14
    # many duplicates in an otherwise random set
    p = rng.uniform(-1, 1, (2000, 3))
    p[100:160] = p[7]
    x = rng.standard_normal(2000)
    T, H = build(orc, p, "inv_r", 1e-8, leaf=16)
    assert T.kappa == 20
    assert rel(H.matvec(x), orc.direct(p, x, "inv_r")) <= 1e-6


def _brute_interactions(T, H, eta2=None):
    """Interaction counts recomputed without the oracle's lists: every pair of
    same-level cells is classified from its integer cell coordinates by the
    admissibility test of Sec. 2.2 (adjacency for eta^2 = d); a pair of
    level l >= lmin is a transverse block iff it is admissible and its
    parents are not (Table 1); a pair of leaves is a near-field block iff it
    is not admissible."""
    d = T.d
    num, den = (d, 1) if eta2 is None else eta2

    def adm(coord):
        g = np.maximum(np.abs(coord[:, None, :] - coord[None, :, :]) - 1, 0)
        return d * den <= num * (g * g).sum(-1)

    far = [0] * (T.kappa + 1)
    for l in range(H.lmin, T.kappa + 1):
        cl = T.cells(l)
        k = np.array([H.cell(l, b)["k"] for b in range(T.ncell(l))], np.int64)
        a = adm(cl["coord"])
        if l > 0:
            pa = adm(T.cells(l - 1)["coord"])
            par = cl["parent"]
            a &= ~pa[par[:, None], par[None, :]]
        far[l] = int((np.outer(k, k) * a).sum())
    leaf = T.cells(T.kappa)
    cnt = leaf["count"].astype(np.int64)
    near = int((np.outer(cnt, cnt) * ~adm(leaf["coord"])).sum())
    return far, near


@pytest.mark.parametrize("kind,d,n,leaf,tol,eta2", [("inv_r", 3, 4000, 16, 1e-4, None),
                                                    ("log_r", 2, 3000, 12, 1e-6, None),
                                                    ("inv_r", 3, 2500, 12, 1e-5, (2, 1))])
def test_interaction_counts_brute_force(orc, kind, d, n, leaf, tol, eta2):
    # the counts behind the throughput figures, per level, against a
    # recount from cell coordinates and the oracle's ranks
    rng = np.random.default_rng(40)
    p = rng.uniform(-1, 1, (n, d))
    T, H = build(orc, p, kind, tol, leaf, eta2=eta2)
    far, near = _brute_interactions(T, H, eta2)
    assert H.interactions_by_level() == far
    assert H.interactions() == (sum(far), near)
    assert sum(far) > 0 and near > 0


def test_interaction_counts_cover_all_pairs(orc):
    # tol = 0 keeps every cell at full rank (k_B = |B|), so the transverse and
    # near-field blocks together cover every ordered pair exactly once (Sec. 3):
    # their interaction counts add up to N^2
    rng = np.random.default_rng(41)
    n = 3000
    p = rng.uniform(-1, 1, (n, 3))
    T, H = build(orc, p, "inv_r", 0.0, leaf=16)
    for l in range(H.lmin, T.kappa + 1):
        cl = T.cells(l)
        for b in range(T.ncell(l)):
            assert H.cell(l, b)["k"] == cl["count"][b]
    far, near = H.interactions()
    assert far + near == n * n
