"""The C ABI's memory and element-type contract, on the GPU:
* every device buffer of a handle comes from the caller's allocator (here the
  torch caching allocator through the hooks), and no matvec allocates or
  frees: the workspace is sized at build time;
* destroying the handle returns every buffer through the same hooks;
* FP32 X and Y: the input is widened exactly and the FP64 result rounded, so
  an FP32 call equals the FP64 call on the widened input, rounded, bit for bit
  (one column and the many-column path, both precisions);
* the many-column workspace width (max_rhs) changes only the blocking:
  without one the columns run one at a time, bit-equal to single calls;
* calls on one handle from two streams are ordered.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_14832_amd import nnca  # noqa: E402
from paper_2203_14832_amd.workloads import workload  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_no_allocation_in_matvec():
    p, x = workload("c2", n=20000, nrhs=40)
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64, max_rhs=32)
    rec = H.alloc_record
    assert rec is not None and rec.allocs > 0 and rec.bytes > 0
    a0, f0 = rec.allocs, rec.frees
    X = torch.tensor(x, device="cuda")
    for prec in ("fp64", "mixed"):
        H.matvec(X[:, 0], prec)
        H.matvec(X[:, :5], prec)
        H.matvec(X, prec)                     # two blocks of the 32-column workspace
        H.rmatvec(X[:, :3], prec)
        H.matvec(X[:, :2].float(), prec)
    torch.cuda.synchronize()
    assert (rec.allocs, rec.frees) == (a0, f0)
    H.close()
    assert rec.frees == rec.allocs


@pytest.mark.parametrize("nrhs", [1, 21])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fp32_vectors(nrhs, prec):
    p, x = workload("c2", n=15000, nrhs=nrhs)
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64)
    X32 = torch.tensor(x, device="cuda", dtype=torch.float32)
    Y32 = H.matvec(X32 if nrhs > 1 else X32[:, 0], prec)
    assert Y32.dtype == torch.float32
    Y64 = H.matvec(X32.double() if nrhs > 1 else X32[:, 0].double(), prec)
    assert torch.equal(Y32, Y64.float())


def test_workspace_width():
    p, x = workload("c2", n=12000, nrhs=5)
    X = torch.tensor(x, device="cuda")
    H1 = nnca.H2Matrix(p, "inv_r", 1e-6, 64, max_rhs=1)
    for prec in ("fp64", "mixed"):
        Y = H1.matvec(X, prec)
        one = torch.stack([H1.matvec(X[:, c], prec) for c in range(5)], 1)
        assert torch.equal(Y, one)
    H64 = nnca.H2Matrix(p, "inv_r", 1e-6, 64, max_rhs=64)
    Yb = H64.matvec(X, "fp64")
    Y1 = H1.matvec(X, "fp64")
    assert float(torch.linalg.norm(Yb - Y1)) <= 1e-13 * float(torch.linalg.norm(Y1))


def test_calls_on_two_streams_are_ordered():
    p, x = workload("c2", n=30000, nrhs=2)
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64)
    X = torch.tensor(x, device="cuda")
    ref0 = H.matvec(X[:, 0], "mixed").clone()
    ref1 = H.matvec(X[:, 1], "mixed").clone()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        y0 = H.matvec(X[:, 0], "mixed")
    with torch.cuda.stream(s2):
        y1 = H.matvec(X[:, 1], "mixed")
    torch.cuda.synchronize()
    assert torch.equal(y0, ref0) and torch.equal(y1, ref1)
