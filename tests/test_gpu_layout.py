"""GPU: the C ABI's column-major layout with leading dimensions above N.

X and Y are caller-owned column-major device buffers with ldx, ldy >= N.  The
product must not depend on the padding of X, must leave the padding of Y
untouched, and must equal the product of densely packed buffers bit for bit
(the same launches read the same values).  Column counts cover one column
(the single-column path), a ragged block (20 columns: two 16-column blocks,
the second partly padding) and more than one 64-column block (70).  The
point count is not a multiple of the 64-point tiles of the input gather and
output scatter.
"""
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


@pytest.fixture(scope="module")
def op():
    p = workload("c2", n=9001)[0]
    return nnca.H2Matrix(p, "inv_r", 1e-6, 64)


def _raw(h, X, Y, nrhs, ldx, ldy, precision):
    dt = nnca.DTYPE_F32 if X.dtype == torch.float32 else nnca.DTYPE_F64
    st = nnca.lib().nnca_matvec(h._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), nrhs, ldx, ldy, dt,
                                nnca.PRECISION[precision], nnca._stream(torch))
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("nrhs", [1, 20, 70])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_leading_dimensions(op, nrhs, precision):
    n = op.n
    ldx, ldy = n + 37, n + 5
    rng = np.random.default_rng(nrhs)
    x = rng.standard_normal((nrhs, n))
    dense_x = torch.tensor(x, device="cuda")
    dense_y = torch.empty((nrhs, n), dtype=torch.float64, device="cuda")
    assert _raw(op, dense_x, dense_y, nrhs, n, n, precision) == 0
    # padded X: garbage in the padding; padded Y: a sentinel that must survive
    px = torch.full((nrhs, ldx), 1e300, dtype=torch.float64, device="cuda")
    px[:, :n] = dense_x
    py = torch.full((nrhs, ldy), -7.25, dtype=torch.float64, device="cuda")
    assert _raw(op, px, py, nrhs, ldx, ldy, precision) == 0
    assert torch.equal(py[:, :n], dense_y), (nrhs, precision)
    assert bool((py[:, n:] == -7.25).all())
    # and the dense product is the matvec of the high-level binding
    ref = op.matvec(torch.tensor(x.T.copy()), precision).cpu().numpy()
    ref = ref.reshape(n, -1)
    got = dense_y.cpu().numpy().T
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_leading_dimension_too_small(op):
    n = op.n
    buf = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    assert _raw(op, buf, buf.clone(), 2, n - 1, n, "fp64") == 1
