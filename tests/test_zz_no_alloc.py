"""nnca_matvec_noalloc, the allocation-free variant of nnca_matvec (per-call
buffers in the library's static device array), against nnca_matvec through
the C ABI: bit-equal results on two calls in a row, the second on a smaller
problem (the array keeps the first call's contents), FP64 and mixed, FP32
and FP64 vectors; a problem whose buffers exceed the array is refused."""
import ctypes as C

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


def _call(fn, H, X, Y, nrhs, prec):
    dt = nnca.DTYPE_F32 if X.dtype == torch.float32 else nnca.DTYPE_F64
    st = fn(H._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), nrhs, H.n, H.n, dt, nnca.PRECISION[prec],
            nnca._stream(torch))
    torch.cuda.synchronize()
    return st


def _reference(H, X, prec):
    """nnca_matvec one column at a time (the same one-column passes)."""
    nrhs = X.shape[0]
    Y = torch.empty_like(X)
    for c in range(nrhs):
        assert _call(nnca.lib().nnca_matvec, H, X[c:c + 1].contiguous(), Y[c:c + 1], 1, prec) == 0
    return Y


def test_noalloc_matches_matvec_twice():
    lib = nnca.lib()
    big = workload("c2", n=30000, nrhs=3)
    small = workload("c3", n=7000, nrhs=3)      # the second call: a smaller problem
    for (p, x), kind, tol in ((big, "inv_r", 1e-6), (small, "inv_r", 1e-7)):
        H = nnca.H2Matrix(p, kind, tol, 64)
        for prec in ("fp64", "mixed"):
            for dtype in (torch.float64, torch.float32):
                X = torch.tensor(x.T.copy(), device="cuda", dtype=dtype)    # (nrhs, n) column-major
                Y = torch.full_like(X, float("nan"))
                assert _call(lib.nnca_matvec_noalloc, H, X, Y, 3, prec) == 0, nnca.lib().nnca_last_error()
                ref = _reference(H, X, prec)
                assert torch.equal(Y, ref), (p.shape[0], prec, dtype)
        H.close()


def test_noalloc_refuses_what_does_not_fit():
    p, x = workload("c2", n=200000)
    H = nnca.H2Matrix(p, "inv_r", 1e-6, 64)
    X = torch.tensor(x[:, 0], device="cuda").reshape(1, -1)
    Y = torch.empty_like(X)
    st = _call(nnca.lib().nnca_matvec_noalloc, H, X, Y, 1, "fp64")
    assert st == 4, st                           # NNCA_ERR_NOT_SUPPORTED
    assert b"static scratch" in nnca.lib().nnca_last_error()
    # the handle still works through nnca_matvec
    assert _call(nnca.lib().nnca_matvec, H, X, Y, 1, "fp64") == 0
