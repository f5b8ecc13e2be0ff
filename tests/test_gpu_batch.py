"""GPU parity of the uneven batch (many problems, one set of launches).

* every problem's rows of the batched product equal that problem's own
  matvec: FP64 to 1e-13 (only the order of partial sums of split transverse
  launches can differ), mixed within the mixed bound of 1e-6 of the FP64
  product; one problem is also checked against the oracle;
* graph replays equal the eager result bit for bit, with eager work and
  synchronisations between the replays; new arguments re-capture;
* one column (single-column path) and 8 columns (many-column path);
* mismatched handles and problems without a far field are rejected.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_14832_amd import nnca  # noqa: E402
from paper_2203_14832_amd.workloads import batch_problem, batch_sizes  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def problems():
    # the uneven-batch recipe scaled down 10x: 12 problems of 1e3 .. 2e4 points
    sizes = [max(1500, s // 10) for s in batch_sizes()[:12]]
    out = []
    for b, n in enumerate(sizes):
        p, x = batch_problem(b, n, 8)
        out.append((p, x, nnca.H2Matrix(p, "inv_r", 1e-6, 64)))
    return out


def _stack(problems, cols):
    return np.concatenate([x[:, :cols] for _, x, _ in problems], axis=0)


def _split(B, Y):
    return [Y[B.offsets[b]:B.offsets[b + 1]] for b in range(B.count)]


@pytest.mark.parametrize("cols", [1, 8])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_separate(problems, cols, graph):
    B = nnca.H2Batch([h for _, _, h in problems], graph=graph, autotune=graph)
    assert B.count == len(problems) and B.rows == sum(p.shape[0] for p, _, _ in problems)
    X = _stack(problems, cols)
    Xd = torch.tensor(X, device="cuda")
    sep64 = [h.matvec(torch.tensor(x[:, :cols]), "fp64").cpu().numpy() for _, x, h in problems]
    Y64 = B.matvec(Xd, "fp64").cpu().numpy()
    Ymx = B.matvec(Xd, "mixed").cpu().numpy()
    if cols == 1:
        Y64, Ymx = Y64.reshape(-1, 1), Ymx.reshape(-1, 1)
        sep64 = [s.reshape(-1, 1) for s in sep64]
    for b, (y64, ymx) in enumerate(zip(_split(B, Y64), _split(B, Ymx))):
        assert rel(y64, sep64[b]) <= 1e-13, b
        assert rel(ymx, sep64[b]) <= 1e-6, b
    B.close()


def test_batch_against_oracle(orc, problems):
    B = nnca.H2Batch([h for _, _, h in problems], graph=False, autotune=False)
    X = _stack(problems, 2)
    Y = B.matvec(torch.tensor(X, device="cuda"), "fp64").cpu().numpy()
    b = 3
    p, x, _ = problems[b]
    T = orc.Tree(p, 64)
    O = orc.H2(T, "inv_r", 1e-6)
    ref = O.matvec(x[:, :2])
    assert rel(_split(B, Y)[b], ref) <= 1e-12


def test_graph_replays_are_identical(problems):
    B = nnca.H2Batch([h for _, _, h in problems], graph=True, autotune=True)
    X = _stack(problems, 8)
    Xc = torch.tensor(X.T.copy(), device="cuda")            # column-major (8, rows)
    Y = torch.empty_like(Xc)
    for prec in ("mixed", "fp64"):
        B.matvec_raw(Xc, Y, 8, prec)                        # eager run + capture + first replay
        torch.cuda.synchronize()
        first = Y.clone()
        for rep in range(3):
            Y.fill_(float("nan"))
            junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
            torch.cuda.synchronize()
            B.matvec_raw(Xc, Y, 8, prec)
            torch.cuda.synchronize()
            assert torch.equal(Y, first), (prec, rep)
            assert torch.isfinite(junk)
    # new output buffer: a new capture with the same result
    Y2 = torch.empty_like(Xc)
    B.matvec_raw(Xc, Y2, 8, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(Y2, first)


def test_batch_errors(problems):
    _, _, h0 = problems[0]
    g = nnca.H2Matrix(problems[0][0], "gauss", 1e-6, 64, length_scale=0.5)
    with pytest.raises(nnca.NncaError) as e:
        nnca.H2Batch([h0, g])
    assert e.value.status == 1
    tiny = nnca.H2Matrix(np.random.default_rng(1).uniform(-1, 1, (40, 3)), "inv_r", 1e-6, 64)
    with pytest.raises(nnca.NncaError) as e:
        nnca.H2Batch([h0, tiny])
    assert e.value.status == 4


@pytest.mark.parametrize("kind,dim,h", [("log_r", 2, 1.0), ("gauss", 3, 0.5)])
def test_batch_other_kernels(orc, kind, dim, h):
    rng = np.random.default_rng(31)
    sizes = [2500, 6000, 1800, 9000]
    probs = []
    for n in sizes:
        p = rng.uniform(-1, 1, (n, dim)) if kind != "gauss" else 0.5 * rng.standard_normal((n, dim))
        x = rng.standard_normal((n, 5))
        probs.append((p, x, nnca.H2Matrix(p, kind, 1e-7, 64, length_scale=h)))
    B = nnca.H2Batch([hd for _, _, hd in probs], graph=True, autotune=True)
    X = np.concatenate([x for _, x, _ in probs], 0)
    Xc = torch.tensor(X.T.copy(), device="cuda")
    Y = torch.empty_like(Xc)
    # mixed: the 2D log kernel's interpolation operators (entries ~150)
    # amplify FP32 rounding to a few 1e-6 (the bound of the single-handle
    # parity tests for that kernel is 3e-5); the Gaussian stays within 3e-6
    mixed_tol = 3e-5 if kind == "log_r" else 3e-6
    for prec, tol in (("fp64", 1e-13), ("mixed", mixed_tol)):
        B.matvec_raw(Xc, Y, 5, prec)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy().T
        for b, (p, x, hd) in enumerate(probs):
            ref = hd.matvec(torch.tensor(x), "fp64").cpu().numpy()
            assert rel(Yh[B.offsets[b]:B.offsets[b + 1]], ref) <= tol, (kind, prec, b)
    # one problem also against the oracle
    p, x, _ = probs[1]
    O = orc.H2(orc.Tree(p, 64), kind, 1e-7, h=h)
    B.matvec_raw(Xc, Y, 5, "fp64")
    torch.cuda.synchronize()
    got = Y.cpu().numpy().T[B.offsets[1]:B.offsets[2]]
    assert rel(got, O.matvec(x)) <= 1e-12


def test_batch_wide_and_single(problems):
    # 20 columns: two column blocks of 16 on the matrix cores
    hs = [h for _, _, h in problems[:5]]
    B = nnca.H2Batch(hs, graph=True, autotune=True)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((B.rows, 20))
    Y = B.matvec(torch.tensor(X, device="cuda"), "mixed").cpu().numpy()
    for b, h in enumerate(hs):
        ref = h.matvec(torch.tensor(X[B.offsets[b]:B.offsets[b + 1]]), "fp64").cpu().numpy()
        assert rel(Y[B.offsets[b]:B.offsets[b + 1]], ref) <= 1e-6, b
    # a batch of one problem is that problem
    p, x, h = problems[2]
    B1 = nnca.H2Batch([h], graph=False, autotune=False)
    assert B1.count == 1 and B1.rows == p.shape[0]
    y1 = B1.matvec(torch.tensor(x[:, 0], device="cuda"), "fp64").cpu().numpy()
    ref = h.matvec(torch.tensor(x[:, 0]), "fp64").cpu().numpy()
    assert rel(y1, ref) <= 1e-13


def test_profile_pass_mask(problems):
    p, x, h = problems[0]
    X = torch.tensor(x[:, 0], device="cuda")
    h.profile(True, passes=[2])
    h.matvec(X, "mixed")
    torch.cuda.synchronize()
    ps, lv, ms = h.profile_read()
    h.profile(False)
    assert len(ps) > 0 and set(ps.tolist()) == {2} and (ms >= 0).all()
    h.profile(True)
    h.matvec(X, "mixed")
    torch.cuda.synchronize()
    ps, lv, ms = h.profile_read()
    h.profile(False)
    assert {0, 1, 2, 3, 4}.issubset(set(ps.tolist()))


def test_autotune_cache_file(problems, tmp_path, monkeypatch):
    # the first autotuned batch times every level's candidates (split factor,
    # and the tile shape on the FP32 levels) and appends one line per level
    # shape to NNCA_TUNE_CACHE; a second batch over the same problems finds
    # every shape there, appends nothing and gives the same product bit for bit
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("NNCA_TUNE_CACHE", str(path))
    X = torch.tensor(_stack(problems, 8), device="cuda")
    B1 = nnca.H2Batch([h for _, _, h in problems], graph=False, autotune=True)
    Y1 = {prec: B1.matvec(X, prec).cpu().numpy() for prec in ("mixed", "fp64")}
    B1.close()
    lines = path.read_text().splitlines()
    assert lines, "no tuning lines written"
    for ln in lines:
        f = ln.split()
        assert f[1] == "m2l" and f[2] in ("f32", "f64") and f[3].startswith("ncb=")
        code = int(f[-1])
        assert 2 <= code <= 129 and (code % 2 == 0 or f[2] == "f32")
    assert any(ln.split()[2] == "f32" for ln in lines) and any(ln.split()[2] == "f64" for ln in lines)
    before = path.read_text()
    B2 = nnca.H2Batch([h for _, _, h in problems], graph=False, autotune=True)
    Y2 = {prec: B2.matvec(X, prec).cpu().numpy() for prec in ("mixed", "fp64")}
    B2.close()
    assert path.read_text() == before
    for prec in Y1:
        np.testing.assert_array_equal(Y2[prec], Y1[prec])
    # against the separate products, as for the default choices
    sep64 = [h.matvec(torch.tensor(x[:, :8]), "fp64").cpu().numpy() for _, x, h in problems]
    B3 = nnca.H2Batch([h for _, _, h in problems], graph=False, autotune=False)
    for b, (y64, ymx) in enumerate(zip(_split(B3, Y1["fp64"]), _split(B3, Y1["mixed"]))):
        assert rel(y64, sep64[b]) <= 1e-13, b
        assert rel(ymx, sep64[b]) <= 1e-6, b
    B3.close()
