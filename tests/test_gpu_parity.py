"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

* the device evaluates the method's FP64 kernel bit for bit like the oracle;
* tree order, cells and lists are identical;
* pivot sets t^{B,i} and s^{B,i} are identical at every level (FP64 build);
* transfer operators agree to 1e-12 (in practice bit for bit);
* the FP64 matvec agrees with the oracle's to 1e-12 (relative 2-norm and
  every entry against the column's largest), the mixed one with the FP64 one
  and with the oracle's to 1e-6 (the tolerance the mixed form is specified
  to), also with the plain (every ordered pair) FP32 passes;
* the interaction counts per level equal the oracle's;
* the FP64 direct sum agrees with the oracle's compensated sum to 1e-13.
Sizes span several levels, partially filled tiles and ragged cells.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_14832_amd import nnca  # noqa: E402
from paper_2203_14832_amd.workloads import chebyshev_grid, draw_points, svm_dataset, workload  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# Bound on the mixed (FP32) matvec against the FP64 one.  1e-6 is the bound
# the mixed form is specified to for 1/r at tol >= 1e-7.  The 2D log case at
# tol 1e-8 (specified all-FP64) has interpolation operators with entries up
# to ~150, which amplify the FP32 unit roundoff (6e-8) to a few 1e-6; a CPU
# emulation with correctly rounded FP32 arithmetic gives 5e-6 on it.  The
# Gaussian case is bounded like the 1/r ones.
# exp(-r) on [-1.4,1.4]^2 (the SVM data) stays between e^-4 and 1, so each
# output sums n terms of like size with cancellation: sum_j |K_ij x_j| is
# ~100 times |y_i| for x ~ N(0,1), and FP32 rounding of those sums reaches
# ~1e-5 of the column's largest entry (2e-7 in the 2-norm).
MIXED_TOL = {"c1": 3e-5, "cheb2d_logreg": 3e-5, "svm2d_expr": 2e-6}
# Elementwise bound of the FP64 product against the oracle's, relative to the
# column's largest entry.  The regularised log kernel on the 2D Chebyshev grid
# sums ~10^4 terms of size ~0.5 per row into entries of ~20 (heavy
# cancellation) through interpolation operators with entries of ~10^2, so
# rounding-level differences of the two FP64 evaluations (summation order,
# libm log against the project-written one, a product with 1/log(a^2)
# against a quotient) reach ~2e-12 of the largest entry; the 2-norm bound
# stays 1e-12 for every case.
ELEM_TOL = {"cheb2d_logreg": 1e-11}

CASES = {
    # name: (points generator, kernel, tol, leaf, h, eta2)
    "c1": (lambda: workload("c1")[0], "log_r", 1e-8, 64, 1.0, None),
    "cube3d": (lambda: workload("c2", n=30000)[0], "inv_r", 1e-6, 64, 1.0, None),
    "sphere": (lambda: workload("c3", n=20000)[0], "inv_r", 1e-7, 64, 1.0, None),
    "mixture": (lambda: workload("c4", n=12000)[0], "gauss", 1e-6, 128, 0.5, None),
    "literal_sqrt2": (lambda: np.random.default_rng(7).uniform(-1, 1, (6000, 3)), "inv_r", 1e-6, 24, 1.0, (2, 1)),
    "cube2d_inv": (lambda: np.random.default_rng(8).uniform(-1, 1, (9000, 2)), "inv_r", 1e-9, 20, 1.0, None),
    # the headline distribution at N = 2^16 (kappa = 4): level kappa-1 has
    # ranks above 80, so the FP32 symmetric transverse pass runs its second
    # shape set there (ranks 81-224: 4-32 lane groups of up to seven
    # registers), as it does at level kappa-1 of the N = 2^20 problem
    "c2_64k": (lambda: workload("c2", n=65536)[0], "inv_r", 1e-6, 64, 1.0, None),
    # the regularised kernels (a = 1e-4) on the tensor-product Chebyshev
    # grids of Exp. 2 (2D, log) and Exp. 4 (3D, 1/r)
    "cheb2d_logreg": (lambda: chebyshev_grid(100, 2), "log_reg", 1e-9, 64, 1e-4, None),
    "cheb3d_invreg": (lambda: chebyshev_grid(22, 3), "inv_reg", 1e-7, 64, 1e-4, None),
    # the kernel SVM's training points of Exp. 6 (2D, [-1.4,1.4]^2) with the
    # paper's "Matern" kernel exp(-r)
    "svm2d_expr": (lambda: svm_dataset(24000, 2, "disk")[0], "exp_r", 1e-8, 64, 1.0, None),
    # a uniform cube with a dense Gaussian cluster: at levels 3-5 a few cells
    # (under a quarter) have ranks above 80, so the symmetric pass launches
    # them apart from the rest (rank classes) in all three arithmetic forms
    "cluster_split": (lambda: _cluster(), "inv_r", 1e-7, 64, 1.0, None),
}


def _cluster():
    rng = np.random.default_rng(31)
    return np.vstack([rng.uniform(-1, 1, (30000, 3)), 0.3 + 0.12 * rng.standard_normal((20000, 3))])


def close_elementwise(Y, Yo, tol):
    """max_i |Y_ic - Yo_ic| <= tol * max_i |Yo_ic| for every column c."""
    Y, Yo = Y.reshape(Y.shape[0], -1), Yo.reshape(Yo.shape[0], -1)
    for c in range(Yo.shape[1]):
        err = np.abs(Y[:, c] - Yo[:, c]).max()
        assert err <= tol * np.abs(Yo[:, c]).max(), (c, err, np.abs(Yo[:, c]).max())


def mixed_vs_oracle(name, Ym, Yo):
    """The mixed product against the oracle's FP64 product: the relative
    2-norm within the mixed bound per column, and every entry within ten
    times that bound of the column's largest entry."""
    tol = MIXED_TOL.get(name, 1e-6)
    for c in range(Yo.shape[1]):
        assert rel(Ym[:, c], Yo[:, c]) <= tol, (name, c, rel(Ym[:, c], Yo[:, c]))
    close_elementwise(Ym, Yo, 10 * tol)


@pytest.fixture(scope="module")
def built(orc):
    cache = {}

    def get(name):
        if name not in cache:
            gen, kind, tol, leaf, h, eta2 = CASES[name]
            p = gen()
            # the many-column workspace at its widest: blocks of 16-64 columns
            G = nnca.H2Matrix(p, kind, tol, leaf, length_scale=h, eta2=eta2, max_rhs=64)
            T = orc.Tree(p, leaf, eta2=eta2)
            O = orc.H2(T, kind, tol, h=h)
            cache[name] = (p, G, T, O, kind, h)
        return cache[name]
    return get


@pytest.mark.parametrize("kind,d", [("inv_r", 3), ("inv_r", 2), ("log_r", 2), ("gauss", 3), ("gauss", 2),
                                    ("log_reg", 2), ("inv_reg", 2), ("inv_reg", 3), ("exp_r", 2), ("exp_r", 3)])
def test_kernel_bits(orc, kind, d):
    rng = np.random.default_rng(11)
    a = rng.uniform(-1, 1, (4000, d))
    b = rng.uniform(-1, 1, (4000, d)) * 10.0 ** rng.uniform(-6, 1, (4000, 1))
    b[:7] = a[:7]   # r = 0
    g = nnca.debug_kernel_eval(kind, a, b, 0.37)
    o = np.array([orc.kernel_eval(kind, a[i], b[i], 0.37) for i in range(4000)])
    np.testing.assert_array_equal(g, o)


@pytest.mark.parametrize("name", list(CASES))
def test_tree_parity(built, name):
    p, G, T, O, kind, h = built(name)
    inf = G.info()
    assert inf["kappa"] == T.kappa and inf["lmin"] == O.lmin
    np.testing.assert_array_equal(G.order(), T.order())
    for l in range(T.kappa + 1):
        gc, oc = G.cells(l), T.cells(l)
        np.testing.assert_array_equal(gc["key"], oc["key"])
        np.testing.assert_array_equal(gc["first"], oc["first"])
        np.testing.assert_array_equal(gc["count"], oc["count"])
        for which in ("nb", "il"):
            gp, gi = G.lists(l, which)
            op, oi = T.lists(l, which)
            np.testing.assert_array_equal(gp, op)
            np.testing.assert_array_equal(gi, oi)


@pytest.mark.parametrize("name", list(CASES))
def test_interaction_counts(built, name):
    # the counts that the throughput figures divide by: transverse pairs per
    # level and near-field pairs, equal to the oracle's
    p, G, T, O, kind, h = built(name)
    inf = G.info()
    far, near = O.interactions()
    assert inf["m2l_level"] == O.interactions_by_level()
    assert inf["m2l_interactions"] == far
    assert inf["p2p_interactions"] == near


def test_headline_shape_sets(built):
    # c2_64k reaches the transverse-pass shape set for level ranks 81-224 at
    # level kappa-1, which runs in FP32 in the mixed form
    p, G, T, O, kind, h = built("c2_64k")
    inf = G.info()
    k = inf["kappa"]
    assert k == 4
    assert 80 < inf["max_rank"][k - 1] <= 224, inf["max_rank"]
    assert inf["mixed_fp32_levels"] == 2


@pytest.mark.parametrize("name", list(CASES))
def test_pivot_parity(built, name):
    p, G, T, O, kind, h = built(name)
    for l in range(O.lmin, T.kappa + 1):
        ptr, rows, cols = G.pivots(l)
        nc = T.ncell(l)
        for b in range(nc):
            c = O.cell(l, b)
            np.testing.assert_array_equal(rows[ptr[b]:ptr[b + 1]], c["piv"], err_msg=f"level {l} cell {b}")
            if c["passthrough"]:
                assert (cols[ptr[b]:ptr[b + 1]] == -1).all()
            else:
                np.testing.assert_array_equal(cols[ptr[b]:ptr[b + 1]], c["colpts"])
        for b in np.linspace(0, nc - 1, min(nc, 12)).astype(int):
            Cg = G.operator(l, b)
            Co = O.cell(l, b)["C"]
            assert Cg.shape == Co.shape
            assert np.abs(Cg - Co).max() <= 1e-12 * max(1.0, np.abs(Co).max())


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_parity(built, name):
    p, G, T, O, kind, h = built(name)
    n = p.shape[0]
    X = np.random.default_rng(12).standard_normal((n, 3))
    Xt = torch.tensor(X, device="cuda")
    # one column at a time (the single-column kernels)
    Y64 = np.stack([G.matvec(Xt[:, c], "fp64").cpu().numpy() for c in range(3)], 1)
    Yo = O.matvec(X)
    assert rel(Y64, Yo) <= 1e-12
    close_elementwise(Y64, Yo, ELEM_TOL.get(name, 1e-12))
    Ym = np.stack([G.matvec(Xt[:, c], "mixed").cpu().numpy() for c in range(3)], 1)
    print(name, "mixed vs fp64:", [rel(Ym[:, c], Y64[:, c]) for c in range(3)],
          "vs oracle:", [rel(Ym[:, c], Yo[:, c]) for c in range(3)])
    mixed_vs_oracle(name, Ym, Yo)
    # FP32 transverse pass at the two finest levels for 1/r, the leaf level
    # only for the kernels whose interpolation operators amplify more; the
    # symmetric near field where near pairs exceed 1/12 of the transverse
    # interactions (all of these small problems)
    inf = G.info()
    assert inf["mixed_fp32_levels"] == (2 if kind in ("inv_r", "inv_reg") else 1)
    assert inf["mixed_near_symmetric"] == (12 * inf["p2p_interactions"] > inf["m2l_interactions"])
    for c in range(3):
        assert rel(Ym[:, c], Y64[:, c]) <= MIXED_TOL.get(name, 1e-6), (name, c, rel(Ym[:, c], Y64[:, c]))
    # the plain (every ordered pair) FP32 transverse pass and near field give
    # the same product to the same bound; the symmetric ones are the default
    # FP64 too: the plain transverse pass, against the oracle like the
    # symmetric one (the default of both forms)
    G.set_symmetric(False)
    try:
        Yp = np.stack([G.matvec(Xt[:, c], "mixed").cpu().numpy() for c in range(3)], 1)
        Y64p = np.stack([G.matvec(Xt[:, c], "fp64").cpu().numpy() for c in range(3)], 1)
    finally:
        G.set_symmetric(True)
    assert rel(Y64p, Yo) <= 1e-12
    close_elementwise(Y64p, Yo, ELEM_TOL.get(name, 1e-12))
    for c in range(3):
        assert rel(Yp[:, c], Y64[:, c]) <= MIXED_TOL.get(name, 1e-6), (name, c)
        assert rel(Yp[:, c], Ym[:, c]) <= MIXED_TOL.get(name, 1e-6), (name, c)
    mixed_vs_oracle(name, Yp, Yo)
    # adjoint: <A x, y> = <x, A^T y>
    Ya = G.rmatvec(Xt, "fp64").cpu().numpy()
    lhs, rhs = X[:, 0] @ Ya[:, 1], Y64[:, 0] @ X[:, 1]
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(X[:, 0]) * np.linalg.norm(Y64[:, 1])


def test_rank_class_split_reached(built):
    # the library splits a level's symmetric launch when its largest rank is
    # above 80 and at most a quarter of its cells are: this case must have
    # such levels on both sides of the FP32 / FP64-refined boundary
    p, G, T, O, kind, h = built("cluster_split")
    kap = G.info()["kappa"]
    split = []
    for l in range(O.lmin, kap + 1):
        k = np.diff(np.asarray(G.pivots(l)[0]))
        if k.max() > 80 and 4 * (k > 80).sum() <= k.size:
            split.append(l)
    assert kap in (6,) and 5 in split and 4 in split, split


def test_symmetric_near_field(built):
    # at least one of the parity problems runs the symmetric near field; its
    # mixed product equals the plain one (every ordered near pair) to the
    # mixed bound and the FP64 product to the same bound
    used = [nm for nm in CASES if built(nm)[1].info()["mixed_near_symmetric"]]
    assert used, "no parity problem exercises the symmetric near field"
    for nm in used:
        p, G, T, O, kind, h = built(nm)
        x = torch.tensor(np.random.default_rng(21).standard_normal(p.shape[0]), device="cuda")
        y64 = G.matvec(x, "fp64").cpu().numpy()
        ys = G.matvec(x, "mixed").cpu().numpy()
        G.set_symmetric(False)
        try:
            yp = G.matvec(x, "mixed").cpu().numpy()
        finally:
            G.set_symmetric(True)
        tol = MIXED_TOL.get(nm, 1e-6)
        assert rel(ys, y64) <= tol and rel(yp, y64) <= tol and rel(ys, yp) <= tol, nm


@pytest.mark.parametrize("kind,d,h", [("inv_r", 3, 1.0), ("log_r", 2, 1.0), ("gauss", 3, 0.6), ("inv_reg", 3, 0.01),
                                      ("log_reg", 2, 0.01), ("exp_r", 2, 1.0), ("exp_r", 3, 0.3)])
def test_direct_parity(orc, kind, d, h):
    rng = np.random.default_rng(13)
    p = rng.uniform(-1, 1, (5000, d))
    p[10] = p[20]
    x = rng.standard_normal((5000, 2))
    yg = nnca.direct(p, torch.tensor(x, device="cuda"), kind, h).cpu().numpy()
    yo = orc.direct(p, x, kind, h)
    assert rel(yg, yo) <= 1e-13


def test_edge_cases(orc):
    rng = np.random.default_rng(14)
    cases = [
        (np.zeros((1, 3)), "inv_r", 1e-6, 1),                       # one point
        (rng.uniform(-1, 1, (50, 3)), "inv_r", 1e-6, 64),            # single leaf
        (np.ones((40, 3)), "gauss", 1e-6, 4),                        # all points identical
        (rng.uniform(-1, 1, (3000, 3)), "inv_r", 0.0, 16),            # tol = 0
        (np.vstack([rng.uniform(-1, 1, (1500, 3)), np.tile([[0.1, 0.2, 0.3]], (80, 1))]), "inv_r", 1e-7, 16),
    ]
    for p, kind, tol, leaf in cases:
        x = rng.standard_normal(p.shape[0])
        G = nnca.H2Matrix(p, kind, tol, leaf, length_scale=0.5)
        T = orc.Tree(p, leaf)
        O = orc.H2(T, kind, tol, h=0.5)
        y = G.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
        yo = O.matvec(x)
        if np.linalg.norm(yo) == 0:
            assert np.linalg.norm(y) == 0
        else:
            assert rel(y, yo) <= 1e-12
        ym = G.matvec(torch.tensor(x, device="cuda"), "mixed").cpu().numpy()
        if np.linalg.norm(yo) > 0:
            assert rel(ym, y) <= 1e-6


def test_policy_literal(orc):
    p = np.random.default_rng(15).uniform(-1, 1, (5000, 3))
    p[100:160] = p[7]
    G = nnca.H2Matrix(p, "inv_r", 1e-6, 16, policy=0)
    T = orc.Tree(p, 16)
    O = orc.H2(T, "inv_r", 1e-6, policy=0)
    for l in range(O.lmin, T.kappa + 1):
        ptr, rows, cols = G.pivots(l)
        for b in range(T.ncell(l)):
            np.testing.assert_array_equal(rows[ptr[b]:ptr[b + 1]], O.cell(l, b)["piv"])


def test_rank_cap_retry_and_chunking(orc):
    # A reserve of 8 panel rows per non-leaf cell is outgrown by most cells, so
    # they are re-run with full room; a small workspace cap splits every level
    # into many chunks.  Pivots must not change in either case.
    rng = np.random.default_rng(16)
    p = rng.uniform(-1, 1, (3000, 3))
    T = orc.Tree(p, 16)
    O = orc.H2(T, "inv_r", 1e-7)
    G1 = nnca.H2Matrix(p, "inv_r", 1e-7, 16, rank_reserve=8)
    G2 = nnca.H2Matrix(p, "inv_r", 1e-7, 16, workspace_bytes=1 << 20)
    assert max(G1.info()["max_rank"][:T.kappa]) > 8
    for l in range(O.lmin, T.kappa + 1):
        for G in (G1, G2):
            ptr, rows, cols = G.pivots(l)
            for b in range(T.ncell(l)):
                np.testing.assert_array_equal(rows[ptr[b]:ptr[b + 1]], O.cell(l, b)["piv"])
    x = torch.tensor(rng.standard_normal(3000), device="cuda")
    np.testing.assert_array_equal(G1.matvec(x).cpu().numpy(), G2.matvec(x).cpu().numpy())


@pytest.mark.parametrize("name,R", [("cube3d", 5), ("cube3d", 37), ("sphere", 64), ("mixture", 16), ("c1", 20),
                                    ("literal_sqrt2", 33), ("c2_64k", 16), ("svm2d_expr", 12),
                                    ("cluster_split", 8)])
def test_many_rhs_parity(built, name, R):
    # The block path (columns innermost, MFMA for the FP32 transverse pass)
    # against the oracle and against one column at a time.
    p, G, T, O, kind, h = built(name)
    n = p.shape[0]
    X = np.random.default_rng(17).standard_normal((n, R))
    Xt = torch.tensor(X, device="cuda")
    Y64 = G.matvec(Xt, "fp64").cpu().numpy()
    Yo = O.matvec(X[:, :3])
    assert rel(Y64[:, :3], Yo) <= 1e-12
    close_elementwise(Y64[:, :3], Yo, ELEM_TOL.get(name, 1e-12))
    one = np.stack([G.matvec(Xt[:, c], "fp64").cpu().numpy() for c in (0, R - 1)], 1)
    assert rel(Y64[:, [0, R - 1]], one) <= 1e-13
    Ym = G.matvec(Xt, "mixed").cpu().numpy()
    errs = [rel(Ym[:, c], Y64[:, c]) for c in range(R)]
    print(name, R, "block mixed vs fp64: max", max(errs))
    assert max(errs) <= MIXED_TOL.get(name, 1e-6)
    mixed_vs_oracle(name, Ym[:, :3], Yo)
