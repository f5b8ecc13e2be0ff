"""Pins of the oracle's general case, targets P != sources Q (Sec. 2.1, 2.3).

* reduction: with Q = P every pivot, operator and product equals the
  symmetric one-ACA oracle of Sec. 5 bit for bit;
* plain definition: a single leaf and tol = 0 give the dense product
  sum_j K(p_i, q_j) x_j, and the error falls with the ACA tolerance;
* the operators are the formulas of Sec. 2.3.1, re-derived from the pivots
  with a library solve: U_B = A(t^B, s^{B,i}) A(t^{B,i}, s^{B,i})^{-1},
  V_B^T = A(t^{B,o}, s^{B,o})^{-1} A(t^{B,o}, s^B), and the translations
  C_{B_c B}, T_{B B_c}; the low-rank form of an admissible leaf block;
* structure: the depth rule counts P and Q separately, candidate sets are
  nested (Sec. 2.3.2), far-field pivots come from the interaction list;
* coverage: the transverse and near-field blocks cover P x Q exactly once;
* transposition: the product of (Q, P) is the adjoint of that of (P, Q),
  and <A~ x, g> = <x, A~^T g>.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def two_sets(rng, np_, nq, d, shift=0.3):
    """Sources uniform in [-1,1]^d, targets in a shifted, scaled cube that
    overlaps them partly: cells with only targets, only sources, or both."""
    Q = rng.uniform(-1, 1, (nq, d))
    P = rng.uniform(-1, 1, (np_, d)) * 0.8 + shift
    return P, Q


def dense(P, Q, kind, h=1.0):
    r = cdist(P, Q)
    with np.errstate(divide="ignore"):
        if kind == "inv_r":
            K = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
        elif kind == "log_r":
            K = np.where(r > 0, np.log(np.where(r > 0, r, 1.0)), 0.0)
        else:
            K = np.exp(-(r / h) ** 2)
    return K


def K_of(orc, kind, A, B, h=1.0):
    return np.array([[orc.kernel_eval(kind, a, b, h) for b in B] for a in A])


def test_direct2_is_the_dense_product(orc):
    rng = np.random.default_rng(50)
    for kind, d in [("inv_r", 3), ("log_r", 2), ("gauss", 3)]:
        P, Q = two_sets(rng, 700, 500, d)
        Q[:3] = P[:3]                       # coincident pairs: K = 0 (1/r, log)
        x = rng.standard_normal(500)
        assert rel(orc.direct2(P, Q, x, kind, 0.5), dense(P, Q, kind, 0.5) @ x) <= 1e-13


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 3)])
def test_same_sets_reduce_to_the_symmetric_case(orc, kind, d):
    rng = np.random.default_rng(51)
    p, x = rng.uniform(-1, 1, (4000, d)), rng.standard_normal(4000)
    T = orc.Tree(p, 32)
    H = orc.H2(T, kind, 1e-6, h=0.5)
    T2 = orc.Tree2(p, p.copy(), 32)
    G = orc.H2General(T2, kind, 1e-6, h=0.5)
    assert T2.kappa == T.kappa and G.lmin == H.lmin
    for l in range(H.lmin, T.kappa + 1):
        for b in range(T.ncell(l)):
            c = H.cell(l, b)
            for half in ("in", "out"):
                g = G.cell(half, l, b)
                assert np.array_equal(g["piv"], c["piv"]) and np.array_equal(g["C"], c["C"])
                assert g["passthrough"] == c["passthrough"]
                if not c["passthrough"]:
                    assert np.array_equal(g["colpts"], c["colpts"])
    ys = H.matvec(x)
    assert np.array_equal(G.matvec(x), ys)
    assert np.array_equal(G.matvec(x, adjoint=True), ys)
    assert G.interactions() == H.interactions()


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 3)])
def test_single_leaf_is_dense(orc, kind, d):
    rng = np.random.default_rng(52)
    P, Q = two_sets(rng, 300, 200, d)
    x = rng.standard_normal(200)
    T = orc.Tree2(P, Q, 300)
    assert T.kappa == 0
    G = orc.H2General(T, kind, 1e-6, h=0.5)
    assert rel(G.matvec(x), orc.direct2(P, Q, x, kind, 0.5)) <= 1e-14


@pytest.mark.parametrize("kind,d,np_,nq", [("inv_r", 3, 3000, 2000), ("log_r", 2, 1500, 2500),
                                           ("gauss", 3, 2500, 1800)])
def test_zero_tolerance_is_dense_and_covers_every_pair(orc, kind, d, np_, nq):
    rng = np.random.default_rng(53)
    P, Q = two_sets(rng, np_, nq, d)
    x, g = rng.standard_normal(nq), rng.standard_normal(np_)
    T = orc.Tree2(P, Q, 16)
    assert T.kappa >= 3
    G = orc.H2General(T, kind, 0.0, h=0.5)
    assert rel(G.matvec(x), orc.direct2(P, Q, x, kind, 0.5)) <= 1e-10
    assert rel(G.matvec(g, adjoint=True), orc.direct2(Q, P, g, kind, 0.5)) <= 1e-10
    # full rank everywhere: the transverse and near blocks cover P x Q once
    far, near = G.interactions()
    assert far + near == np_ * nq
    for l in range(G.lmin, T.kappa + 1):
        nt, ns = T.counts(l)
        for b in range(T.ncell(l)):
            assert G.cell("in", l, b)["k"] == nt[b]
            assert G.cell("out", l, b)["k"] == ns[b]


@pytest.mark.parametrize("kind,d,np_,nq", [("log_r", 2, 3000, 4096), ("inv_r", 3, 6000, 8192)])
@pytest.mark.parametrize("layout,final", [("shifted", 1e-7), ("same_region", 1e-9)])
def test_error_falls_with_tolerance(orc, kind, d, np_, nq, layout, final):
    # targets drawn over the sources' region converge like the symmetric
    # case; targets that overlap the sources only partly leave some cells
    # with few targets in their interaction list, whose outgoing pivots then
    # see little of the far field, and converge more slowly
    rng = np.random.default_rng(54)
    P, Q = two_sets(rng, np_, nq, d)
    if layout == "same_region":
        P = rng.uniform(-1, 1, (np_, d))
    x = rng.standard_normal(nq)
    yd = orc.direct2(P, Q, x, kind)
    T = orc.Tree2(P, Q, 32)
    errs = [rel(orc.H2General(T, kind, tol).matvec(x), yd) for tol in 10.0 ** -np.arange(2, 11, 2)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < final


def test_depth_counts_targets_and_sources_separately(orc):
    rng = np.random.default_rng(55)
    # many targets in one corner, sources spread out: the targets set the depth
    Q = rng.uniform(-1, 1, (500, 2))
    P = rng.uniform(0.5, 1.0, (3000, 2))
    nu = 40
    T = orc.Tree2(P, Q, nu)
    nt, ns = T.counts(T.kappa)
    assert nt.max() <= nu and ns.max() <= nu
    Tc = orc.Tree(np.vstack([P, Q]), nu)     # the union's total count is stricter
    assert Tc.kappa >= T.kappa
    # one level up some cell holds more than nu of one set
    nt1, ns1 = T.counts(T.kappa - 1)
    assert max(nt1.max(), ns1.max()) > nu


def test_operators_are_the_formulas_of_the_nested_bases(orc):
    rng = np.random.default_rng(56)
    kind = "inv_r"
    P, Q = two_sets(rng, 2500, 2000, 3)
    T = orc.Tree2(P, Q, 24)
    G = orc.H2General(T, kind, 1e-7)
    kap = T.kappa
    cells = T.cells(kap)
    order = T.order()
    checked = 0
    for l in range(G.lmin, kap + 1):
        nt, ns = T.counts(l)
        for b in range(T.ncell(l)):
            gi, go = G.cell("in", l, b), G.cell("out", l, b)
            if gi["passthrough"] or go["passthrough"] or gi["k"] == 0 or go["k"] == 0:
                continue
            tI, sI = gi["piv"], gi["colpts"]           # t^{B,i} (P), s^{B,i} (Q)
            sO, tO = go["piv"], go["colpts"]           # s^{B,o} (Q), t^{B,o} (P)
            # rows of the candidate sets: own targets / own sources
            Kin = K_of(orc, kind, P[tI], Q[sI])
            Kout = K_of(orc, kind, P[tO], Q[sO])
            Ui = K_of(orc, kind, P[gi["tt"]], Q[sI]) @ np.linalg.inv(Kin)
            Vo = (np.linalg.solve(Kout, K_of(orc, kind, P[tO], Q[go["tt"]]))).T
            ci = np.linalg.cond(Kin) * 1e-15
            co = np.linalg.cond(Kout) * 1e-15
            assert np.abs(gi["C"] - Ui).max() <= max(ci, 1e-12) * max(1.0, np.abs(Ui).max()) * 10
            assert np.abs(go["C"] - Vo).max() <= max(co, 1e-12) * max(1.0, np.abs(Vo).max()) * 10
            # identity rows at the pivots (cross interpolation)
            pos_i = [list(gi["tt"]).index(t) for t in tI]
            pos_o = [list(go["tt"]).index(s) for s in sO]
            assert np.array_equal(gi["C"][pos_i], np.eye(gi["k"]))
            assert np.array_equal(go["C"][pos_o], np.eye(go["k"]))
            if l == kap:
                # a leaf's candidate rows are its own points of each set
                f, c = cells["first"][b], cells["count"][b]
                mine = order[f:f + c]
                assert sorted(gi["tt"]) == sorted(int(z) for z in mine if z < T.np)
                assert sorted(go["tt"]) == sorted(int(z) - T.np for z in mine if z >= T.np)
            checked += 1
    assert checked > 50


def test_candidates_are_nested_and_far_pivots_lie_in_the_interaction_list(orc):
    rng = np.random.default_rng(57)
    P, Q = two_sets(rng, 3000, 2500, 2)
    T = orc.Tree2(P, Q, 16)
    G = orc.H2General(T, "log_r", 1e-8)
    for l in range(G.lmin, T.kappa):
        ch = T.cells(l + 1)["parent"]
        ptr, idx = T.lists(l, "il")
        for b in range(T.ncell(l)):
            kids = np.where(ch == b)[0]
            gi, go = G.cell("in", l, b), G.cell("out", l, b)
            assert np.array_equal(gi["tt"], np.concatenate([G.cell("in", l + 1, c)["piv"] for c in kids]))
            assert np.array_equal(go["tt"], np.concatenate([G.cell("out", l + 1, c)["piv"] for c in kids]))
            ilk = [c for e in idx[ptr[b]:ptr[b + 1]] for c in np.where(ch == e)[0]]
            far_q = set(int(v) for c in ilk for v in G.cell("out", l + 1, c)["piv"])
            far_p = set(int(v) for c in ilk for v in G.cell("in", l + 1, c)["piv"])
            assert gi["n"] == sum(G.cell("out", l + 1, c)["k"] for c in ilk)
            assert go["n"] == sum(G.cell("in", l + 1, c)["k"] for c in ilk)
            if not gi["passthrough"]:
                assert set(gi["colpts"].tolist()) <= far_q
            if not go["passthrough"]:
                assert set(go["colpts"].tolist()) <= far_p


def test_low_rank_form_of_an_admissible_leaf_block(orc):
    # A(t^X, s^Y) ~ U_X S_{X,Y} V_Y^T with S = A(t^{X,i}, s^{Y,o}) (eq. NCA)
    rng = np.random.default_rng(58)
    kind = "inv_r"
    P, Q = two_sets(rng, 4000, 4000, 3, shift=0.1)
    T = orc.Tree2(P, Q, 32)
    G = orc.H2General(T, kind, 1e-8)
    kap = T.kappa
    cells = T.cells(kap)
    order = T.order()
    ptr, idx = T.lists(kap, "il")
    worst, done = 0.0, 0
    for X in range(T.ncell(kap)):
        for Y in idx[ptr[X]:ptr[X + 1]][:3]:
            gi, go = G.cell("in", kap, X), G.cell("out", kap, Y)
            if gi["m"] == 0 or go["m"] == 0:
                continue
            A = K_of(orc, kind, P[gi["tt"]], Q[go["tt"]])
            S = K_of(orc, kind, P[gi["piv"]], Q[go["piv"]])
            worst = max(worst, rel(gi["C"] @ S @ go["C"].T, A))
            done += 1
        if done > 60:
            break
    assert done > 30 and worst < 1e-5


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("log_r", 2), ("gauss", 3)])
def test_swapping_the_sets_transposes_the_product(orc, kind, d):
    rng = np.random.default_rng(59)
    P, Q = two_sets(rng, 3000, 2200, d)
    x, g = rng.standard_normal(2200), rng.standard_normal(3000)
    Ga = orc.H2General(orc.Tree2(P, Q, 32), kind, 1e-6, h=0.5)
    Gb = orc.H2General(orc.Tree2(Q, P, 32), kind, 1e-6, h=0.5)
    assert np.array_equal(Gb.matvec(g), Ga.matvec(g, adjoint=True))
    assert np.array_equal(Gb.matvec(x, adjoint=True), Ga.matvec(x))
    y = Ga.matvec(x)
    assert abs(y @ g - x @ Ga.matvec(g, adjoint=True)) <= 1e-13 * np.abs(y).sum() * np.abs(g).max()


def test_degenerate_sets(orc):
    rng = np.random.default_rng(60)
    Q = rng.uniform(-1, 1, (3000, 3))
    x = rng.standard_normal(3000)
    # a single target; targets on top of sources (r = 0 pairs drop out);
    # targets far outside the sources' cloud
    for P in (rng.uniform(-1, 1, (1, 3)), Q[:500].copy(), rng.uniform(3, 4, (800, 3))):
        T = orc.Tree2(P, Q, 32)
        G = orc.H2General(T, "inv_r", 1e-9)
        assert rel(G.matvec(x), orc.direct2(P, Q, x, "inv_r")) <= 1e-7
    # a single source
    P = rng.uniform(-1, 1, (2000, 3))
    G = orc.H2General(orc.Tree2(P, Q[:1], 32), "inv_r", 1e-9)
    assert rel(G.matvec(x[:1]), orc.direct2(P, Q[:1], x[:1], "inv_r")) <= 1e-14


def test_multiple_columns_equal_single_columns(orc):
    rng = np.random.default_rng(61)
    P, Q = two_sets(rng, 2000, 1500, 3)
    X = rng.standard_normal((1500, 3))
    G = orc.H2General(orc.Tree2(P, Q, 32), "inv_r", 1e-6)
    Y = G.matvec(X)
    for c in range(3):
        assert np.array_equal(Y[:, c], G.matvec(X[:, c]))
