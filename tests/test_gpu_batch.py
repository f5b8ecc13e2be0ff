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
