"""The C-ABI library loads, exports every entry point of include/nnca.h and
rejects bad arguments with the documented status before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nnca.h")).read()
    return sorted(set(re.findall(r"\b(nnca_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2203_14832_amd import nnca
    return nnca.lib()


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "nnca_build" in syms and "nnca_matvec" in syms and "nnca_matvec_adjoint" in syms
    for s in syms:
        assert hasattr(lib, s), s


def test_status_strings(lib):
    for s in range(7):
        assert lib.nnca_status_string(s)


def _build(lib, pts, n, dim, ld, kind=2, h=1.0, tol=1e-6, leaf=64, out=True):
    handle = C.c_void_p()
    return lib.nnca_build(pts, n, dim, ld, 0, kind, h, tol, leaf, None, None,
                          C.byref(handle) if out else None), handle


def test_invalid_arguments(lib):
    p = np.zeros((3, 10))
    P = p.ctypes.data_as(C.c_void_p)
    assert _build(lib, None, 10, 3, 10)[0] == 1
    assert _build(lib, P, 10, 3, 10, out=False)[0] == 1
    assert _build(lib, P, 0, 3, 10)[0] == 1
    assert _build(lib, P, 10, 4, 10)[0] == 1
    assert _build(lib, P, 10, 3, 5)[0] == 1
    assert _build(lib, P, 10, 3, 10, leaf=0)[0] == 1
    assert _build(lib, P, 10, 3, 10, tol=-1.0)[0] == 1
    assert _build(lib, P, 10, 3, 10, tol=float("nan"))[0] == 1
    assert _build(lib, P, 10, 3, 10, kind=7)[0] == 1
    assert _build(lib, P, 10, 3, 10, kind=3, h=0.0)[0] == 1
    assert _build(lib, P, 10, 3, 10, kind=6, h=-1.0)[0] == 1   # exp(-r/h) needs h > 0
    assert _build(lib, P, 10, 3, 10, kind=1)[0] == 4   # log only in 2D
    assert b"dim" in lib.nnca_last_error() or lib.nnca_last_error()
    assert lib.nnca_matvec(None, None, None, 1, 1, 1, 1, 0, None) == 1
    assert lib.nnca_matvec_noalloc(None, None, None, 1, 1, 1, 1, 0, None) == 1
    assert lib.nnca_matvec_adjoint(None, None, None, 1, 1, 1, 1, 0, None) == 1
    assert lib.nnca_query(None, None) == 1
    assert lib.nnca_probe_rates(None, 5, None) == 1
    assert lib.nnca_gmres(None, 1.0, 1.0, None, None, 1e-10, 10, 5, 0, None, None, None) == 1
    assert lib.nnca_destroy(None) == 0
    assert lib.nnca_direct(None, 10, 3, 10, 2, 1.0, None, None, 1, 10, 10, None) == 1
    assert lib.nnca_matvec_backward(None, None, None, 1, 1, 1, 0, None, 1, None, None) == 1
    assert lib.nnca_svm_train(None, None, None, 1.0, 1.0, 0.0, 1e-8, 10, 0, None, None, None, None) == 1
    assert lib.nnca_svm_decision(None, None, None, 0.0, None, 0, None) == 1


def test_general_build_invalid_arguments(lib):
    p = np.zeros((3, 10))
    q = np.zeros((3, 12))
    P, Q = p.ctypes.data_as(C.c_void_p), q.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()

    def bg(Pp, np_, ldp, Qp, nq, ldq, dim=3, kind=2, hh=1.0, tol=1e-6, leaf=64, out=True):
        return lib.nnca_build_general(Pp, np_, ldp, Qp, nq, ldq, dim, 0, kind, hh, tol, leaf, None, None,
                                      C.byref(h) if out else None)
    assert bg(None, 10, 10, Q, 12, 12) == 1
    assert bg(P, 10, 10, None, 12, 12) == 1
    assert bg(P, 10, 10, Q, 12, 12, out=False) == 1
    assert bg(P, 0, 10, Q, 12, 12) == 1
    assert bg(P, 10, 10, Q, 0, 12) == 1
    assert bg(P, 10, 5, Q, 12, 12) == 1
    assert bg(P, 10, 10, Q, 12, 11) == 1
    assert bg(P, 10, 10, Q, 12, 12, dim=4) == 1
    assert bg(P, 10, 10, Q, 12, 12, tol=-1.0) == 1
    assert bg(P, 10, 10, Q, 12, 12, kind=1) == 4   # log only in 2D
    assert bg(P, 10, 10, Q, 12, 12, kind=3, hh=0.0) == 1
    assert not h.value
    assert lib.nnca_query_shape(None, None, None, None) == 1
    assert lib.nnca_query_build(None, None, 3) == 1
    assert lib.nnca_export_half(None, 0, 0, None, None, None) == 1
    assert lib.nnca_export_half_operator(None, 0, 0, 0, None, 0, None, None) == 1


def test_build_options_layout(lib):
    # the struct grew at its end: the first version ends at `reserved` (32
    # bytes); the allocator fields follow the column-workspace size
    from paper_2203_14832_amd import nnca
    O = nnca.BuildOptions
    assert O.max_rhs.offset == 32 and O.alloc.offset == 40 and O.free.offset == 48 and O.alloc_ctx.offset == 56
    assert C.sizeof(O) == 64


def test_build_rejects_bad_options(lib):
    from paper_2203_14832_amd import nnca
    p = np.zeros((3, 10))
    P = p.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    o = nnca.BuildOptions(C.sizeof(nnca.BuildOptions))
    o.alloc = nnca._TORCH_ALLOC          # alloc without free
    assert lib.nnca_build(P, 10, 3, 10, 0, 2, 1.0, 1e-6, 64, C.byref(o), None, C.byref(h)) == 1
    o = nnca.BuildOptions(C.sizeof(nnca.BuildOptions))
    o.max_rhs = -1
    assert lib.nnca_build(P, 10, 3, 10, 0, 2, 1.0, 1e-6, 64, C.byref(o), None, C.byref(h)) == 1
    o = nnca.BuildOptions(20)             # neither version's size
    assert lib.nnca_build(P, 10, 3, 10, 0, 2, 1.0, 1e-6, 64, C.byref(o), None, C.byref(h)) == 1
    assert not h.value
