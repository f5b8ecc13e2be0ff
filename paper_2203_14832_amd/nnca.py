"""Thin ctypes binding of the C ABI in ``include/nnca.h``.

Argument marshalling only: every step of the build and of the matvec runs in
the HIP library.  Importing this module does not touch the GPU; the library is
loaded on first use and a missing library is an error (there is no CPU path).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnca.so")

KINDS = {"log_r": 1, "inv_r": 2, "gauss": 3, "log_reg": 4, "inv_reg": 5, "exp_r": 6}
PRECISION = {"fp64": 0, "mixed": 1}
DTYPE_F32, DTYPE_F64 = 0, 1
MAX_LEVELS = 64
NOALLOC_SCRATCH_BYTES = 64 << 20

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class NncaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nnca status {status}: {msg}")
        self.status = status


class BuildOptions(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("eta2_num", C.c_int32), ("eta2_den", C.c_int32),
                ("exhausted_policy", C.c_int32), ("workspace_bytes", C.c_int64), ("rank_reserve", C.c_int32),
                ("reserved", C.c_int32), ("max_rhs", C.c_int32), ("reserved2", C.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


# Device memory of the handles built with allocator="torch": the torch
# caching allocator, through the C ABI's allocator hooks.  Each handle gets a
# context number; its record counts the calls (a batch made from handles
# keeps using the first handle's record, so records are never dropped).
_alloc_records = {}


class AllocRecord:
    def __init__(self, device):
        self.device = device
        self.allocs = 0
        self.frees = 0
        self.bytes = 0


def _torch_alloc(nbytes, ctx):
    try:
        import torch
        rec = _alloc_records[ctx]
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device=rec.device)
        rec.allocs += 1
        rec.bytes += int(nbytes)
        return ptr
    except Exception:   # the library reports NULL as out of memory
        return None


def _torch_free(ptr, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(ptr)
        _alloc_records[ctx].frees += 1
    except Exception:
        pass


_TORCH_ALLOC = ALLOC_FN(_torch_alloc)
_TORCH_FREE = FREE_FN(_torch_free)


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("kappa", C.c_int32), ("lmin", C.c_int32),
                ("leaf_size", C.c_int32), ("kernel_kind", C.c_int32), ("length_scale", C.c_double),
                ("tol", C.c_double), ("lo", C.c_double * 3), ("side", C.c_double),
                ("ncell", C.c_int64 * MAX_LEVELS), ("npiv", C.c_int64 * MAX_LEVELS),
                ("nlist", (C.c_int64 * 2) * MAX_LEVELS), ("max_rank", C.c_int32 * MAX_LEVELS),
                ("m2l_level", C.c_int64 * MAX_LEVELS),
                ("transfer_entries", C.c_int64), ("m2l_interactions", C.c_int64),
                ("p2p_interactions", C.c_int64), ("build_seconds", C.c_double),
                ("mixed_fp32_levels", C.c_int32), ("mixed_near_symmetric", C.c_int32)]


_lib = None
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device memory while the HIP runtime is still up
    for m in list(_live):
        m.close()


def lib():
    """Load libnnca.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "nnca_build": [P, i64, i32, i64, i32, i32, f64, f64, i32, P, P, P],
            "nnca_matvec": [P, P, P, i64, i64, i64, i32, i32, P],
            "nnca_matvec_adjoint": [P, P, P, i64, i64, i64, i32, i32, P],
            "nnca_matvec_noalloc": [P, P, P, i64, i64, i64, i32, i32, P],
            "nnca_matvec_backward": [P, P, P, i64, i64, i64, i32, P, i64, P, P],
            "nnca_direct": [P, i64, i32, i64, i32, f64, P, P, i64, i64, i64, P],
            "nnca_query": [P, P],
            "nnca_export_order": [P, P],
            "nnca_export_cells": [P, i32, P, P, P],
            "nnca_export_lists": [P, i32, i32, P, P],
            "nnca_export_pivots": [P, i32, P, P, P],
            "nnca_export_operator": [P, i32, i64, P, i64, P, P],
            "nnca_debug_kernel_eval": [i32, f64, i32, P, P, i64, P],
            "nnca_destroy": [P],
            "nnca_profile_enable": [P, i32],
            "nnca_profile_read": [P, P, P, P, P, i64],
            "nnca_set_apply_flags": [P, i32],
            "nnca_batch_create": [P, i32, i32, P],
            "nnca_batch_query": [P, P, P, P],
            "nnca_batch_matvec": [P, P, P, i64, i64, i64, i32, P],
            "nnca_batch_destroy": [P],
            "nnca_probe_rates": [P, i32, P],
            "nnca_gmres": [P, f64, f64, P, P, f64, i32, i32, i32, P, P, P],
            "nnca_build_general": [P, i64, i64, P, i64, i64, i32, i32, i32, f64, f64, i32, P, P, P],
            "nnca_query_shape": [P, P, P, P],
            "nnca_query_build": [P, P, i32],
            "nnca_export_half": [P, i32, i32, P, P, P],
            "nnca_export_half_operator": [P, i32, i32, i64, P, i64, P, P],
            "nnca_svm_train": [P, P, P, f64, f64, f64, f64, i32, i32, P, P, P, P],
            "nnca_svm_decision": [P, P, P, f64, P, i32, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.nnca_last_error.restype = C.c_char_p
        L.nnca_status_string.restype = C.c_char_p
        L.nnca_status_string.argtypes = [C.c_int]
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise NncaError(status, lib().nnca_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _as_columns(torch, X, n, device, keep_f32=False):
    """(n,) or (n, r) -> column-major device buffer (r, n) and r: FP64, or
    FP32 when keep_f32 and X is FP32."""
    X = torch.as_tensor(X, device=device)
    dt = torch.float32 if (keep_f32 and X.dtype == torch.float32) else torch.float64
    X = X.to(dtype=dt)
    if X.dim() == 1:
        return X.contiguous().reshape(1, n), 1, True
    return X.t().contiguous(), X.shape[1], False


class H2Matrix:
    """H2 representation built by NNCA on the GPU (``nnca_build``)."""

    def __init__(self, points, kernel: str = "inv_r", tol: float = 1e-6, leaf_size: int = 64,
                 length_scale: float = 1.0, eta2=None, policy: int = 1, workspace_bytes: int = 0,
                 rank_reserve: int = 0, device="cuda:0", max_rhs: int = 0, allocator: str | None = "torch"):
        """``max_rhs``: columns of the many-column workspace (0: 16; 1: none);
        ``allocator``: "torch" (the caching allocator, through the C ABI's
        hooks) or None (the library's hipMalloc)."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        pts = torch.as_tensor(points, dtype=torch.float64)
        n, d = pts.shape
        self.n, self.dim, self.kernel = n, d, kernel
        self.length_scale = float(length_scale)
        soa = pts.t().contiguous().to(self.device)
        opts = BuildOptions(C.sizeof(BuildOptions), 0, 0, int(policy), int(workspace_bytes), int(rank_reserve), 0,
                            int(max_rhs), 0)
        if eta2 is not None:
            opts.eta2_num, opts.eta2_den = int(eta2[0]), int(eta2[1])
        self.alloc_record = None
        if allocator == "torch":
            ctx = len(_alloc_records) + 1
            self.alloc_record = _alloc_records[ctx] = AllocRecord(self.device)
            opts.alloc, opts.free, opts.alloc_ctx = _TORCH_ALLOC, _TORCH_FREE, ctx
        elif allocator is not None:
            raise ValueError("allocator must be 'torch' or None")
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().nnca_build(C.c_void_p(soa.data_ptr()), n, d, n, 1, KINDS[kernel], float(length_scale),
                                    float(tol), int(leaf_size), C.byref(opts), _stream(torch), C.byref(h)))
        self._h = h
        self._soa = soa
        self._destroy = lib().nnca_destroy
        _live.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._destroy(self._h)
        self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # module globals may already be gone at interpreter exit
        if not _finalizing():
            self.close()

    def _apply(self, X, precision: str, adjoint: bool, out=None, fn=None):
        torch = self.torch
        Xc, r, vec = _as_columns(torch, X, self.n, self.device, keep_f32=True)
        Y = torch.empty((r, self.n), dtype=Xc.dtype, device=self.device) if out is None else out
        dt = DTYPE_F32 if Xc.dtype == torch.float32 else DTYPE_F64
        if fn is None:
            fn = lib().nnca_matvec_adjoint if adjoint else lib().nnca_matvec
        with torch.cuda.device(self.device):
            _check(fn(self._h, C.c_void_p(Xc.data_ptr()), C.c_void_p(Y.data_ptr()), r, self.n, self.n, dt,
                      PRECISION[precision], _stream(torch)))
        return Y.reshape(self.n) if vec else Y.t()

    def matvec(self, X, precision: str = "fp64"):
        """Y = A~ X for a device tensor (n,) or (n, r), FP64 or FP32 (the
        result has X's type; the arithmetic is set by ``precision``)."""
        return self._apply(X, precision, False)

    def rmatvec(self, X, precision: str = "fp64"):
        """Y = A~^T X."""
        return self._apply(X, precision, True)

    def matvec_noalloc(self, X, precision: str = "fp64"):
        """Y = A~ X through ``nnca_matvec_noalloc`` (per-call buffers in the
        library's static device array; columns one at a time)."""
        return self._apply(X, precision, False, fn=lib().nnca_matvec_noalloc)

    def solve(self, F, alpha: float = 1.0, beta: float = 1.0, tol: float = 1e-10, max_iter: int = 500,
              restart: int = 50, precision: str = "fp64", x0=None):
        """Solve (alpha I + beta A~) X = F by GMRES (``nnca_gmres``); returns
        (X, matvecs, final relative residual)."""
        torch = self.torch
        Fd = torch.as_tensor(F, dtype=torch.float64, device=self.device).reshape(self.n).contiguous()
        X = (torch.zeros_like(Fd) if x0 is None
             else torch.as_tensor(x0, dtype=torch.float64, device=self.device).reshape(self.n).clone())
        it = C.c_int32()
        rr = C.c_double()
        with torch.cuda.device(self.device):
            _check(lib().nnca_gmres(self._h, float(alpha), float(beta), C.c_void_p(Fd.data_ptr()),
                                    C.c_void_p(X.data_ptr()), float(tol), int(max_iter), int(restart),
                                    PRECISION[precision], C.byref(it), C.byref(rr), _stream(torch)))
        return X, it.value, rr.value

    def shape(self):
        """(rows, columns, general) of the operator (``nnca_query_shape``)."""
        r, c, g = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().nnca_query_shape(self._h, C.byref(r), C.byref(c), C.byref(g)))
        return r.value, c.value, bool(g.value)

    def svm_train(self, y, lam: float = 1.0, beta: float = 1.0, eta: float = 0.0, tol: float = 1e-8,
                  max_iter: int = 1000, precision: str = "fp64", alpha0=None):
        """Kernel SVM dual by projected gradient ascent (``nnca_svm_train``):
        labels y (+1 / -1) in the original point order; eta <= 0 picks
        1 / (||K~|| + beta n).  Returns (alpha, bias, steps, eta)."""
        torch = self.torch
        yd = torch.as_tensor(y, dtype=torch.float64, device=self.device).reshape(self.n).contiguous()
        a = (torch.zeros_like(yd) if alpha0 is None
             else torch.as_tensor(alpha0, dtype=torch.float64, device=self.device).reshape(self.n).clone())
        it = C.c_int32()
        b = C.c_double()
        e = C.c_double()
        with torch.cuda.device(self.device):
            _check(lib().nnca_svm_train(self._h, C.c_void_p(yd.data_ptr()), C.c_void_p(a.data_ptr()), float(lam),
                                        float(beta), float(eta), float(tol), int(max_iter), PRECISION[precision],
                                        C.byref(it), C.byref(b), C.byref(e), _stream(torch)))
        return a, b.value, it.value, e.value

    def svm_decision(self, y, alpha, bias: float, precision: str = "fp64"):
        """f = K~ (y .* alpha) + bias at the rows of the operator
        (``nnca_svm_decision``); y and alpha have one entry per column."""
        torch = self.torch
        rows, cols, _ = self.shape()
        yd = torch.as_tensor(y, dtype=torch.float64, device=self.device).reshape(cols).contiguous()
        ad = torch.as_tensor(alpha, dtype=torch.float64, device=self.device).reshape(cols).contiguous()
        f = torch.empty(rows, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().nnca_svm_decision(self._h, C.c_void_p(yd.data_ptr()), C.c_void_p(ad.data_ptr()),
                                           float(bias), C.c_void_p(f.data_ptr()), PRECISION[precision],
                                           _stream(torch)))
        return f

    def set_symmetric(self, enable: bool = True):
        """Use (default) or not the symmetric evaluation (transverse pass and
        near field) of the mixed form."""
        _check(lib().nnca_set_apply_flags(self._h, 0 if enable else 1))

    def backward(self, X, G, precision: str = "fp64", need_x: bool = True, need_h: bool = True):
        """Backward of Y = A~ X with G = dL/dY: (A~^T G or None, dL/dh or
        None); dL/dh (Gaussian kernel, pivots frozen) is a 0-dim FP64 device
        tensor."""
        torch = self.torch
        Xc, r, vec = _as_columns(torch, X, self.n, self.device)
        Gc, rg, _ = _as_columns(torch, G, self.n, self.device)
        if rg != r:
            raise ValueError("X and G have different numbers of columns")
        DX = torch.empty((r, self.n), dtype=torch.float64, device=self.device) if need_x else None
        dh = torch.zeros((), dtype=torch.float64, device=self.device) if need_h else None
        with torch.cuda.device(self.device):
            _check(lib().nnca_matvec_backward(
                self._h, C.c_void_p(Xc.data_ptr()), C.c_void_p(Gc.data_ptr()), r, self.n, self.n,
                PRECISION[precision], None if DX is None else C.c_void_p(DX.data_ptr()), self.n,
                None if dh is None else C.c_void_p(dh.data_ptr()), _stream(torch)))
        if DX is not None:
            DX = DX.reshape(self.n) if vec else DX.t()
        return DX, dh

    def apply(self, X, length_scale=None, precision: str = "fp64"):
        """Differentiable Y = A~ X (torch.autograd): gradients flow to X and,
        for the Gaussian kernel, to ``length_scale`` -- a tensor holding the
        length scale the handle was built with (pivots frozen)."""
        fn = _autograd_function(self.torch)
        if length_scale is not None:
            if self.kernel != "gauss":
                raise ValueError("a length scale is differentiable for the Gaussian kernel only")
            hv = float(length_scale.detach())
            if abs(hv - self.length_scale) > 1e-14 * self.length_scale:
                raise ValueError(f"length_scale {hv} differs from the built {self.length_scale}; rebuild the handle")
        return fn.apply(X, length_scale, self, precision)

    def matvec_raw(self, Xc, Y, nrhs: int, precision: str = "fp64"):
        """Column-major device buffers (nrhs, n) in, (nrhs, n) out, both FP64
        or both FP32; no copies."""
        dt = DTYPE_F32 if Xc.dtype == self.torch.float32 else DTYPE_F64
        _check(lib().nnca_matvec(self._h, C.c_void_p(Xc.data_ptr()), C.c_void_p(Y.data_ptr()), nrhs, self.n,
                                 self.n, dt, PRECISION[precision], _stream(self.torch)))

    def profile(self, enable: bool = True, passes=None):
        """Start (and clear) or stop per-launch event timing of matvec passes
        (``passes``: iterable of pass numbers, default all)."""
        mask = 0
        if enable:
            mask = -1 if passes is None else sum(1 << int(p) for p in passes)
        _check(lib().nnca_profile_enable(self._h, mask))

    def profile_read(self, cap: int = 1 << 16):
        """Records (pass, level, ms) since profile(True); clears them."""
        cnt = C.c_int64()
        ps = np.zeros(cap, np.int32)
        lv = np.zeros(cap, np.int32)
        ms = np.zeros(cap)
        _check(lib().nnca_profile_read(self._h, C.byref(cnt), _np_ptr(ps), _np_ptr(lv), _np_ptr(ms), cap))
        k = min(cnt.value, cap)
        return ps[:k].copy(), lv[:k].copy(), ms[:k].copy()

    def build_stats(self) -> dict:
        """Build seconds, pivot-traversal seconds and its algorithmic panel
        bytes (``nnca_query_build``)."""
        out = np.zeros(3)
        _check(lib().nnca_query_build(self._h, _np_ptr(out), 3))
        return dict(build_seconds=float(out[0]), aca_seconds=float(out[1]), aca_panel_bytes=float(out[2]))

    def info(self) -> dict:
        inf = Info()
        _check(lib().nnca_query(self._h, C.byref(inf)))
        L = inf.kappa + 1
        return dict(n=inf.n, dim=inf.dim, kappa=inf.kappa, lmin=inf.lmin, leaf_size=inf.leaf_size,
                    tol=inf.tol, lo=list(inf.lo)[: inf.dim], side=inf.side,
                    ncell=[inf.ncell[l] for l in range(L)], npiv=[inf.npiv[l] for l in range(L)],
                    nlist=[(inf.nlist[l][0], inf.nlist[l][1]) for l in range(L)],
                    max_rank=[inf.max_rank[l] for l in range(L)], m2l_level=[inf.m2l_level[l] for l in range(L)],
                    transfer_entries=inf.transfer_entries,
                    m2l_interactions=inf.m2l_interactions, p2p_interactions=inf.p2p_interactions,
                    build_seconds=inf.build_seconds, mixed_fp32_levels=inf.mixed_fp32_levels,
                    mixed_near_symmetric=bool(inf.mixed_near_symmetric))

    # parity exports -----------------------------------------------------
    def order(self):
        o = np.zeros(self.n, np.int64)
        _check(lib().nnca_export_order(self._h, _np_ptr(o)))
        return o

    def cells(self, level: int):
        nc = self.info()["ncell"][level]
        key = np.zeros(nc, np.uint64)
        first = np.zeros(nc, np.int64)
        count = np.zeros(nc, np.int64)
        _check(lib().nnca_export_cells(self._h, level, _np_ptr(key), _np_ptr(first), _np_ptr(count)))
        return dict(key=key, first=first, count=count)

    def lists(self, level: int, which: str):
        inf = self.info()
        w = 1 if which == "il" else 0
        tot = inf["nlist"][level][w]
        ptr = np.zeros(inf["ncell"][level] + 1, np.int64)
        idx = np.zeros(max(tot, 1), np.int64)
        _check(lib().nnca_export_lists(self._h, level, w, _np_ptr(ptr), _np_ptr(idx)))
        return ptr, idx[:tot]

    def pivots(self, level: int):
        inf = self.info()
        npv = inf["npiv"][level]
        ptr = np.zeros(inf["ncell"][level] + 1, np.int64)
        rows = np.zeros(max(npv, 1), np.int64)
        cols = np.zeros(max(npv, 1), np.int64)
        _check(lib().nnca_export_pivots(self._h, level, _np_ptr(ptr), _np_ptr(rows), _np_ptr(cols)))
        return ptr, rows[:npv], cols[:npv]

    def operator(self, level: int, cell: int):
        m = C.c_int64()
        k = C.c_int64()
        _check(lib().nnca_export_operator(self._h, level, cell, None, 0, C.byref(m), C.byref(k)))
        Cm = np.zeros(max(m.value * k.value, 1))
        _check(lib().nnca_export_operator(self._h, level, cell, _np_ptr(Cm), Cm.size, C.byref(m), C.byref(k)))
        return Cm[: m.value * k.value].reshape(m.value, k.value)


class H2General(H2Matrix):
    """H2 representation of the general case A_ij = K(p_i, q_j), targets P
    and sources Q (``nnca_build_general``): ``matvec`` maps (nq,) or (nq, r)
    to (np,) or (np, r), ``rmatvec`` the other way."""

    def __init__(self, targets, sources, kernel: str = "inv_r", tol: float = 1e-6, leaf_size: int = 64,
                 length_scale: float = 1.0, eta2=None, policy: int = 1, workspace_bytes: int = 0,
                 rank_reserve: int = 0, device="cuda:0", allocator: str | None = "torch"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        P = torch.as_tensor(targets, dtype=torch.float64)
        Q = torch.as_tensor(sources, dtype=torch.float64)
        npt, d = P.shape
        nq = Q.shape[0]
        if Q.shape[1] != d:
            raise ValueError("targets and sources differ in dimension")
        self.n, self.nq, self.dim, self.kernel = npt, nq, d, kernel
        self.length_scale = float(length_scale)
        ps = P.t().contiguous().to(self.device)
        qs = Q.t().contiguous().to(self.device)
        opts = BuildOptions(C.sizeof(BuildOptions), 0, 0, int(policy), int(workspace_bytes), int(rank_reserve), 0,
                            1, 0)
        if eta2 is not None:
            opts.eta2_num, opts.eta2_den = int(eta2[0]), int(eta2[1])
        self.alloc_record = None
        if allocator == "torch":
            ctx = len(_alloc_records) + 1
            self.alloc_record = _alloc_records[ctx] = AllocRecord(self.device)
            opts.alloc, opts.free, opts.alloc_ctx = _TORCH_ALLOC, _TORCH_FREE, ctx
        elif allocator is not None:
            raise ValueError("allocator must be 'torch' or None")
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().nnca_build_general(C.c_void_p(ps.data_ptr()), npt, npt, C.c_void_p(qs.data_ptr()), nq, nq,
                                            d, 1, KINDS[kernel], float(length_scale), float(tol), int(leaf_size),
                                            C.byref(opts), _stream(torch), C.byref(h)))
        self._h = h
        self._soa = (ps, qs)
        self._destroy = lib().nnca_destroy
        _live.add(self)

    def _apply(self, X, precision: str, adjoint: bool, out=None, fn=None):
        torch = self.torch
        nin, nout = (self.n, self.nq) if adjoint else (self.nq, self.n)
        Xc, r, vec = _as_columns(torch, X, nin, self.device, keep_f32=True)
        Y = torch.empty((r, nout), dtype=Xc.dtype, device=self.device) if out is None else out
        dt = DTYPE_F32 if Xc.dtype == torch.float32 else DTYPE_F64
        if fn is None:
            fn = lib().nnca_matvec_adjoint if adjoint else lib().nnca_matvec
        with torch.cuda.device(self.device):
            _check(fn(self._h, C.c_void_p(Xc.data_ptr()), C.c_void_p(Y.data_ptr()), r, nin, nout, dt,
                      PRECISION[precision], _stream(torch)))
        return Y.reshape(nout) if vec else Y.t()

    def half_pivots(self, level: int, half: str):
        """(ptr, rows, cols): half "in" rows t^{B,i} (into P), cols s^{B,i}
        (into Q); half "out" rows s^{B,o} (into Q), cols t^{B,o} (into P)."""
        hf = 0 if half == "in" else 1
        ptr = np.zeros(self.info()["ncell"][level] + 1, np.int64)
        _check(lib().nnca_export_half(self._h, level, hf, _np_ptr(ptr), None, None))
        npv = int(ptr[-1])
        rows = np.zeros(max(npv, 1), np.int64)
        cols = np.zeros(max(npv, 1), np.int64)
        _check(lib().nnca_export_half(self._h, level, hf, _np_ptr(ptr), _np_ptr(rows), _np_ptr(cols)))
        return ptr, rows[:npv], cols[:npv]

    def half_operator(self, level: int, half: str, cell: int):
        hf = 0 if half == "in" else 1
        m = C.c_int64()
        k = C.c_int64()
        _check(lib().nnca_export_half_operator(self._h, level, hf, cell, None, 0, C.byref(m), C.byref(k)))
        Cm = np.zeros(max(m.value * k.value, 1))
        _check(lib().nnca_export_half_operator(self._h, level, hf, cell, _np_ptr(Cm), Cm.size, C.byref(m),
                                               C.byref(k)))
        return Cm[: m.value * k.value].reshape(m.value, k.value)


class H2Batch:
    """Uneven batch of built handles applied by one set of launches
    (``nnca_batch_create``): Y_b = A~_b X_b for every problem b, rows of the
    batched vectors stacked in handle order."""

    GRAPH, AUTOTUNE = 1, 2

    def __init__(self, handles, graph: bool = True, autotune: bool = True):
        import torch
        self.torch = torch
        self.device = handles[0].device
        arr = (C.c_void_p * len(handles))(*[h._h.value for h in handles])
        b = C.c_void_p()
        flags = (self.GRAPH if graph else 0) | (self.AUTOTUNE if autotune else 0)
        with torch.cuda.device(self.device):
            _check(lib().nnca_batch_create(arr, len(handles), flags, C.byref(b)))
        self._b = b
        self._destroy = lib().nnca_batch_destroy
        cnt, rows = C.c_int32(), C.c_int64()
        _check(lib().nnca_batch_query(b, C.byref(cnt), C.byref(rows), None))
        off = np.zeros(cnt.value + 1, np.int64)
        _check(lib().nnca_batch_query(b, None, None, _np_ptr(off)))
        self.count, self.rows, self.offsets = cnt.value, rows.value, off
        _live.add(self)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._destroy(self._b)
        self._b = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():
            self.close()

    def matvec_raw(self, Xc, Y, nrhs: int, precision: str = "fp64"):
        """Column-major device buffers (nrhs, rows) in and out; no copies."""
        _check(lib().nnca_batch_matvec(self._b, C.c_void_p(Xc.data_ptr()), C.c_void_p(Y.data_ptr()), nrhs,
                                       self.rows, self.rows, PRECISION[precision], _stream(self.torch)))

    def matvec(self, X, precision: str = "fp64"):
        """Y = diag(A~_b) X for a (rows,) or (rows, r) FP64 tensor."""
        torch = self.torch
        Xc, r, vec = _as_columns(torch, X, self.rows, self.device)
        Y = torch.empty((r, self.rows), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self.matvec_raw(Xc, Y, r, precision)
        return Y.reshape(self.rows) if vec else Y.t()


_fn_cache = {}


def _autograd_function(torch):
    """torch.autograd.Function over nnca_matvec / nnca_matvec_backward."""
    if "fn" not in _fn_cache:
        class H2Apply(torch.autograd.Function):
            @staticmethod
            def forward(ctx, x, h, op, precision):
                ctx.op, ctx.precision = op, precision
                ctx.h_meta = None if h is None else (h.device, h.dtype, h.shape)
                ctx.save_for_backward(x)
                return op._apply(x, precision, False)

            @staticmethod
            def backward(ctx, gy):
                (x,) = ctx.saved_tensors
                need_x, need_h = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
                if not (need_x or need_h):
                    return None, None, None, None
                dx, dh = ctx.op.backward(x, gy, ctx.precision, need_x, need_h)
                if dx is not None:
                    dx = dx.to(dtype=x.dtype)
                if dh is not None:
                    dev, dt, shp = ctx.h_meta
                    dh = dh.to(device=dev, dtype=dt).reshape(shp)
                return dx, dh, None, None

        _fn_cache["fn"] = H2Apply
    return _fn_cache["fn"]


def direct(points, X, kernel: str = "inv_r", length_scale: float = 1.0, device="cuda:0"):
    """Dense FP64 direct sum on the GPU (``nnca_direct``)."""
    import torch
    dev = torch.device(device)
    pts = torch.as_tensor(points, dtype=torch.float64)
    n, d = pts.shape
    soa = pts.t().contiguous().to(dev)
    Xc, r, vec = _as_columns(torch, X, n, dev)
    Y = torch.empty((r, n), dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        _check(lib().nnca_direct(C.c_void_p(soa.data_ptr()), n, d, n, KINDS[kernel], float(length_scale),
                                 C.c_void_p(Xc.data_ptr()), C.c_void_p(Y.data_ptr()), r, n, n, _stream(torch)))
    return Y.reshape(n) if vec else Y.t()


def probe_rates(device="cuda:0") -> dict:
    """Attainable rates of the device (``nnca_probe_rates``)."""
    import torch
    out = np.zeros(5)
    with torch.cuda.device(torch.device(device)):
        _check(lib().nnca_probe_rates(_np_ptr(out), 5, _stream(torch)))
    keys = ["copy_bytes_per_s", "fma_f32_lane_ops_per_s", "rsq_f32_lane_ops_per_s", "sym_pairs_per_s_valu",
            "sym_pairs_per_s_mfma_r2"]
    return dict(zip(keys, out.tolist()))


def debug_kernel_eval(kernel: str, a, b, length_scale: float = 1.0):
    """Evaluate the method's FP64 kernel on the device for pairs (a[i], b[i])."""
    a = np.ascontiguousarray(np.asarray(a, np.float64).T)
    b = np.ascontiguousarray(np.asarray(b, np.float64).T)
    d, cnt = a.shape
    out = np.zeros(cnt)
    _check(lib().nnca_debug_kernel_eval(KINDS[kernel], float(length_scale), d, _np_ptr(a), _np_ptr(b), cnt,
                                        _np_ptr(out)))
    return out
