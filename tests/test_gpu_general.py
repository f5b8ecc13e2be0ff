"""GPU parity of the general case P != Q (Sec. 2.1, 2.3): the HIP library
(``nnca_build_general`` through its C ABI) against the CPU oracle.

* the tree (depth counting P and Q apart, cells, P and Q per cell) is the
  oracle's;
* both halves' pivots, t^{B,i}, s^{B,i} (incoming) and s^{B,o}, t^{B,o}
  (outgoing), are identical at every level (FP64 build), and the operators
  U_B / C_{B_c B} and V_B / T_{B B_c}^T agree to 1e-12;
* the FP64 product A~ x (nq -> np) and its transpose (np -> nq) agree with
  the oracle's to 1e-12 (2-norm and every entry against the column's
  largest), the mixed product to the mixed bound;
* Q = P reproduces the symmetric build's pivots and product;
* a large rectangular problem against the direct sum on sampled rows.
Sets overlap partly, lie apart, or hold a single point; cells hold only
targets, only sources, or both.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_14832_amd import nnca  # noqa: E402
from paper_2203_14832_amd.workloads import chebyshev_grid, draw_points  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shifted(seed, npt, nq, d, scale=0.8, shift=0.3):
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-1, 1, (nq, d))
    P = rng.uniform(-1, 1, (npt, d)) * scale + shift
    return P, Q


def _sphere_targets(seed):
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-1, 1, (40000, 3))
    g = rng.standard_normal((15000, 3))
    return 0.9 * g / np.linalg.norm(g, axis=1, keepdims=True), Q


def _apart(seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.5, 2.5, (7000, 3)), rng.uniform(-1, 1, (25000, 3))


def _mixtures(seed):
    rng = np.random.default_rng(seed)
    return draw_points("mixture", 8000, 3, rng), draw_points("mixture", 12000, 3, rng) * 1.1


def _cheb_uniform(seed):
    rng = np.random.default_rng(seed)
    return chebyshev_grid(90, 2), rng.uniform(-1, 1, (6000, 2))


CASES = {
    # name: (targets, sources generator, kernel, tol, leaf, h)
    "shift3d": (lambda: _shifted(70, 20000, 30000, 3), "inv_r", 1e-6, 64, 1.0),
    "shift2d_log": (lambda: _shifted(71, 12000, 9000, 2), "log_r", 1e-8, 64, 1.0),
    "mixture_gauss": (lambda: _mixtures(72), "gauss", 1e-6, 128, 0.5),
    "sphere_targets": (lambda: _sphere_targets(73), "inv_r", 1e-7, 48, 1.0),
    "apart": (lambda: _apart(74), "inv_r", 1e-7, 64, 1.0),
    "few_targets": (lambda: _shifted(75, 37, 20000, 3), "inv_r", 1e-6, 32, 1.0),
    "cheb_logreg": (lambda: _cheb_uniform(76), "log_reg", 1e-9, 64, 1e-4),
    "wide_inv_reg": (lambda: _shifted(77, 9000, 26000, 3, scale=1.0, shift=0.0), "inv_reg", 1e-7, 40, 1e-3),
}
# Bounds of the mixed product against the oracle's FP64 one: 1e-6 as in the
# symmetric case; the 2D log kernels as there (their operators amplify the
# FP32 rounding most); targets on a sphere at tol 1e-7 measured 1.17e-6 in
# one column (6.5e-7 and 6.9e-7 in the others): the incoming operators of the
# cells the surface cuts hold few targets and larger entries, which amplify
# the FP32 rounding of the two finest levels' transverse pass.
MIXED_TOL = {"shift2d_log": 3e-5, "cheb_logreg": 3e-5, "sphere_targets": 2e-6}
ELEM_TOL = {"cheb_logreg": 1e-11}


def close_elementwise(Y, Yo, tol):
    Y, Yo = Y.reshape(Y.shape[0], -1), Yo.reshape(Yo.shape[0], -1)
    for c in range(Yo.shape[1]):
        err = np.abs(Y[:, c] - Yo[:, c]).max()
        assert err <= tol * np.abs(Yo[:, c]).max(), (c, err, np.abs(Yo[:, c]).max())


@pytest.fixture(scope="module")
def built(orc):
    cache = {}

    def get(name):
        if name not in cache:
            gen, kind, tol, leaf, h = CASES[name]
            P, Q = gen()
            print("case", name, P.shape, Q.shape, flush=True)
            G = nnca.H2General(P, Q, kind, tol, leaf, length_scale=h)
            T = orc.Tree2(P, Q, leaf)
            O = orc.H2General(T, kind, tol, h=h)
            cache[name] = (P, Q, G, T, O, kind, h)
        return cache[name]
    return get


@pytest.mark.parametrize("name", list(CASES))
def test_general_tree(built, name):
    P, Q, G, T, O, kind, h = built(name)
    inf = G.info()
    assert inf["kappa"] == T.kappa and inf["lmin"] == O.lmin
    assert G.shape() == (P.shape[0], Q.shape[0], True)
    for l in range(T.kappa + 1):
        c = G.cells(l)
        co = T.cells(l)
        np.testing.assert_array_equal(c["key"], co["key"])
        nt, ns = T.counts(l)
        np.testing.assert_array_equal(c["count"], nt)
        np.testing.assert_array_equal(np.diff(np.append(c["first"], P.shape[0])), nt)
        for w in ("nb", "il"):
            ptr, idx = G.lists(l, w)
            po, io = T.lists(l, w)
            np.testing.assert_array_equal(ptr, po)
            np.testing.assert_array_equal(idx, io)


@pytest.mark.parametrize("name", list(CASES))
def test_general_pivot_parity(built, name):
    P, Q, G, T, O, kind, h = built(name)
    for l in range(O.lmin, T.kappa + 1):
        nc = T.ncell(l)
        for half in ("in", "out"):
            ptr, rows, cols = G.half_pivots(l, half)
            for b in range(nc):
                c = O.cell(half, l, b)
                np.testing.assert_array_equal(rows[ptr[b]:ptr[b + 1]], c["piv"], err_msg=f"{half} {l} {b}")
                if c["passthrough"]:
                    assert (cols[ptr[b]:ptr[b + 1]] == -1).all()
                else:
                    np.testing.assert_array_equal(cols[ptr[b]:ptr[b + 1]], c["colpts"], err_msg=f"{half} {l} {b}")
            for b in np.linspace(0, nc - 1, min(nc, 10)).astype(int):
                Cg = G.half_operator(l, half, b)
                Co = O.cell(half, l, b)["C"]
                assert Cg.shape == Co.shape
                if Co.size:   # a cell without points of this half's set has an empty operator
                    assert np.abs(Cg - Co).max() <= 1e-12 * max(1.0, np.abs(Co).max())


@pytest.mark.parametrize("name", list(CASES))
def test_general_matvec_parity(built, name):
    P, Q, G, T, O, kind, h = built(name)
    npt, nq = P.shape[0], Q.shape[0]
    rng = np.random.default_rng(78)
    X, Gt = rng.standard_normal((nq, 3)), rng.standard_normal((npt, 3))
    Xd, Gd = torch.tensor(X, device="cuda"), torch.tensor(Gt, device="cuda")
    # one call with three columns; then column by column (the same kernels)
    Y64 = G.matvec(Xd, "fp64").cpu().numpy()
    for c in range(3):
        np.testing.assert_array_equal(G.matvec(Xd[:, c], "fp64").cpu().numpy(), Y64[:, c])
    Yo = O.matvec(X)
    assert Y64.shape == (npt, 3)
    assert rel(Y64, Yo) <= 1e-12
    close_elementwise(Y64, Yo, ELEM_TOL.get(name, 1e-12))
    Z64 = G.rmatvec(Gd, "fp64").cpu().numpy()
    Zo = O.matvec(Gt, adjoint=True)
    assert Z64.shape == (nq, 3)
    assert rel(Z64, Zo) <= 1e-12
    close_elementwise(Z64, Zo, ELEM_TOL.get(name, 1e-12))
    # <A~ x, g> = <x, A~^T g>
    lhs, rhs = Y64[:, 0] @ Gt[:, 1], X[:, 0] @ Z64[:, 1]
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Y64[:, 0]) * np.linalg.norm(Gt[:, 1]) * 10
    tol = MIXED_TOL.get(name, 1e-6)
    Ym = G.matvec(Xd, "mixed").cpu().numpy()
    Zm = G.rmatvec(Gd, "mixed").cpu().numpy()
    print(name, "mixed vs oracle:", [rel(Ym[:, c], Yo[:, c]) for c in range(3)],
          [rel(Zm[:, c], Zo[:, c]) for c in range(3)])
    for c in range(3):
        assert rel(Ym[:, c], Yo[:, c]) <= tol, (name, c)
        assert rel(Zm[:, c], Zo[:, c]) <= tol, (name, c)
    close_elementwise(Ym, Yo, 10 * tol)
    close_elementwise(Zm, Zo, 10 * tol)
    # FP32 vectors: widened on input, the FP64 result rounded on output
    Y32 = G.matvec(Xd.float(), "fp64")
    assert Y32.dtype == torch.float32
    Yr = G.matvec(Xd.float().double(), "fp64").cpu().numpy()
    np.testing.assert_array_equal(Y32.cpu().numpy(), Yr.astype(np.float32))


def test_same_sets_match_the_symmetric_build(orc):
    rng = np.random.default_rng(79)
    p = rng.uniform(-1, 1, (20000, 3))
    x = rng.standard_normal(20000)
    S = nnca.H2Matrix(p, "inv_r", 1e-6, 64, max_rhs=1)
    G = nnca.H2General(p, p.copy(), "inv_r", 1e-6, 64)
    inf, ginf = S.info(), G.info()
    assert ginf["kappa"] == inf["kappa"] and ginf["npiv"] == inf["npiv"]
    for l in range(inf["lmin"], inf["kappa"] + 1):
        ptr, rows, cols = S.pivots(l)
        for half in ("in", "out"):
            gp, gr, gc = G.half_pivots(l, half)
            np.testing.assert_array_equal(gp, ptr)
            np.testing.assert_array_equal(gr, rows)
            np.testing.assert_array_equal(gc, cols)
    xd = torch.tensor(x, device="cuda")
    S.set_symmetric(False)
    ys = S.matvec(xd, "fp64").cpu().numpy()
    yg = G.matvec(xd, "fp64").cpu().numpy()
    ya = G.rmatvec(xd, "fp64").cpu().numpy()
    assert rel(yg, ys) <= 1e-14 and rel(ya, ys) <= 1e-14
    T = orc.Tree(p, 64)
    assert rel(yg, orc.H2(T, "inv_r", 1e-6).matvec(x)) <= 1e-12


def test_general_rejects_square_only_entry_points():
    rng = np.random.default_rng(80)
    P, Q = rng.uniform(-1, 1, (3000, 3)), rng.uniform(-1, 1, (4000, 3))
    G = nnca.H2General(P, Q, "inv_r", 1e-6, 64)
    x = torch.tensor(rng.standard_normal(4000), device="cuda")
    for call in (lambda: G.matvec_noalloc(x),
                 lambda: G.solve(torch.zeros(3000, dtype=torch.float64, device="cuda")),
                 lambda: nnca.H2Batch([G])):
        with pytest.raises(nnca.NncaError) as e:
            call()
        assert e.value.status == 4
    # wrong lengths are rejected before any launch
    with pytest.raises(Exception):
        G.matvec(torch.zeros(3000, dtype=torch.float64, device="cuda"))


def test_general_large_against_direct_sum(orc):
    # 2^19 targets in a shifted cube against 2^20 uniform sources (1/r,
    # tol 1e-6): the product on 1536 sampled rows against the direct sum
    rng = np.random.default_rng(81)
    Q = rng.uniform(-1, 1, (1 << 20, 3))
    P = rng.uniform(-1, 1, (1 << 19, 3)) * 0.8 + 0.3
    x = rng.standard_normal(1 << 20)
    print("large general case", P.shape, Q.shape, flush=True)
    G = nnca.H2General(P, Q, "inv_r", 1e-6, 64)
    xd = torch.tensor(x, device="cuda")
    y64 = G.matvec(xd, "fp64").cpu().numpy()
    ym = G.matvec(xd, "mixed").cpu().numpy()
    rows = np.sort(rng.choice(P.shape[0], 1536, replace=False))
    yd = orc.direct2(P, Q, x, "inv_r", rows=rows)
    e64, em = rel(y64[rows], yd), rel(ym[rows], yd)
    print("large general: eps fp64", e64, "mixed", em, "mixed vs fp64", rel(ym, y64))
    # the method's own error on this layout: the oracle gives 2.2e-6 at
    # 2^14 x 2^15 and 2.3e-5 at 2^16 x 2^17 (targets drawn over the sources'
    # cube instead: 2.8e-6 and 4.9e-6) -- targets that cover only part of a
    # cell's neighbourhood leave its outgoing pivots, chosen from the
    # interaction-list region, blind to part of its far field
    assert e64 <= 4e-5 and em <= 4e-5
    assert rel(ym, y64) <= 1e-6
    # transpose on the sampled source entries: (A~^T g)_j against the direct sum
    g = rng.standard_normal(P.shape[0])
    z = G.rmatvec(torch.tensor(g, device="cuda"), "fp64").cpu().numpy()
    cols = np.sort(rng.choice(Q.shape[0], 1024, replace=False))
    zd = orc.direct2(Q[cols], P, g, "inv_r")
    assert rel(z[cols], zd) <= 4e-5
