"""Plain FP64 CPU oracle of the NNCA H2 matrix-vector product.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The GPU library and
its Python binding never import this package.

The arithmetic lives in ``nnca_oracle.c`` (plain C, FP64, compiled with
``-ffp-contract=off``); this module only builds it with gcc and marshals numpy
arrays through ctypes.  Each function of the C file cites the section of the
paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnca_oracle.c")
_LIB = os.path.join(_HERE, "libnnca_oracle.so")

KINDS = {"log_r": 1, "inv_r": 2, "gauss": 3, "log_reg": 4, "inv_reg": 5, "exp_r": 6, "poly2": 99}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int, C.c_double
        L.orc_log.restype = f64; L.orc_log.argtypes = [f64]
        L.orc_exp.restype = f64; L.orc_exp.argtypes = [f64]
        L.orc_kernel_eval.restype = f64
        L.orc_kernel_eval.argtypes = [i32, f64, P, P, i32]
        L.orc_direct.restype = None
        L.orc_direct.argtypes = [P, i64, i32, i32, f64, P, i64, P, i64, P]
        L.orc_tree_build.restype = P
        L.orc_tree_build.argtypes = [P, i64, i32, i32, i64, i64]
        L.orc_tree_free.argtypes = [P]
        L.orc_tree_kappa.restype = i32; L.orc_tree_kappa.argtypes = [P]
        L.orc_tree_ncell.restype = i64; L.orc_tree_ncell.argtypes = [P, i32]
        L.orc_tree_domain.argtypes = [P, P, P]
        L.orc_tree_order.argtypes = [P, P]
        L.orc_tree_cells.argtypes = [P, i32, P, P, P, P, P]
        L.orc_tree_lists.restype = i64; L.orc_tree_lists.argtypes = [P, i32, i32, P, P]
        L.orc_aca_block.restype = i64
        L.orc_aca_block.argtypes = [P, i64, P, i64, i32, i32, f64, f64, P, P, P, P, P]
        L.orc_h2_new.restype = P; L.orc_h2_new.argtypes = [P, i32, f64, f64, i32]
        L.orc_h2_lmin.restype = i32; L.orc_h2_lmin.argtypes = [P]
        L.orc_h2_build.restype = i32; L.orc_h2_build.argtypes = [P, i32, P, i64]
        L.orc_h2_free.argtypes = [P]
        L.orc_h2_cell.restype = i32; L.orc_h2_cell.argtypes = [P, i32, i64, P, P, P, P, P]
        L.orc_h2_matvec.argtypes = [P, P, P, i64, i32]
        L.orc_h2_interactions.argtypes = [P, P]
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_h2_frozen.restype = P; L.orc_h2_frozen.argtypes = [P, f64]
        L.orc_h2_grad_h.restype = f64; L.orc_h2_grad_h.argtypes = [P, P, P, i32]
        L.orc_dense_grad_h.restype = f64; L.orc_dense_grad_h.argtypes = [P, i64, i32, f64, P, P]
        L.orc_tree_build2.restype = P
        L.orc_tree_build2.argtypes = [P, i64, P, i64, i32, i32, i64, i64]
        L.orc_g2_new.restype = P; L.orc_g2_new.argtypes = [P, i32, f64, f64, i32]
        L.orc_g2_lmin.restype = i32; L.orc_g2_lmin.argtypes = [P]
        L.orc_g2_build.restype = i32; L.orc_g2_build.argtypes = [P]
        L.orc_g2_free.argtypes = [P]
        L.orc_g2_cell.restype = i32; L.orc_g2_cell.argtypes = [P, i32, i32, i64, P, P, P, P, P]
        L.orc_g2_matvec.argtypes = [P, P, P, i64, i32]
        L.orc_g2_interactions.argtypes = [P, P]
        L.orc_direct2.restype = None
        L.orc_direct2.argtypes = [P, i64, P, i64, i32, i32, f64, P, i64, P, i64, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops (timing runs)."""
    lib().orc_set_num_threads(int(k))


def log(x: float) -> float:
    return lib().orc_log(float(x))


def exp(x: float) -> float:
    return lib().orc_exp(float(x))


def kernel_eval(kind: str, a, b, h: float = 1.0) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib().orc_kernel_eval(KINDS[kind], float(h), _p(a), _p(b), a.shape[0])


def direct(points, x, kind: str, h: float = 1.0, rows=None) -> np.ndarray:
    """Dense sum y_i = sum_j K(p_i, p_j) x_j (compensated, FP64).

    ``points`` is (n, d); ``x`` is (n,) or (n, r).  ``rows`` restricts the
    output to the listed target indices."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = np.ascontiguousarray(x.reshape(n, -1).T)  # column-major columns
    nrhs = X.shape[0]
    if rows is None:
        r = None
        nr = n
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        nr = r.shape[0]
    Y = np.zeros((nrhs, nr))
    lib().orc_direct(_p(pts), n, d, KINDS[kind], float(h), _p(X), nrhs, _p(r), nr, _p(Y))
    return Y[0] if vec else Y.T.copy()


def direct2(P, Q, x, kind: str, h: float = 1.0, rows=None) -> np.ndarray:
    """Dense sum of the general case y_i = sum_j K(p_i, q_j) x_j
    (compensated, FP64); ``x`` is (nq,) or (nq, r)."""
    Pp = np.ascontiguousarray(P, dtype=np.float64)
    Qp = np.ascontiguousarray(Q, dtype=np.float64)
    np_, d = Pp.shape
    nq = Qp.shape[0]
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = np.ascontiguousarray(x.reshape(nq, -1).T)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = np_ if r is None else r.shape[0]
    Y = np.zeros((X.shape[0], nr))
    lib().orc_direct2(_p(Pp), np_, _p(Qp), nq, d, KINDS[kind], float(h), _p(X), X.shape[0], _p(r), nr, _p(Y))
    return Y[0] if vec else Y.T.copy()


def aca_block(prow, pcol, kind: str, tol: float, h: float = 1.0):
    """ACA of the block K(prow, pcol); returns (rowpos, colpos, U, V, C)."""
    pr = np.ascontiguousarray(prow, dtype=np.float64)
    pc = np.ascontiguousarray(pcol, dtype=np.float64)
    m, d = pr.shape
    n = pc.shape[0]
    kcap = min(m, n)
    rp = np.zeros(max(kcap, 1), np.int64)
    cp = np.zeros(max(kcap, 1), np.int64)
    U = np.zeros((max(kcap, 1), m))
    V = np.zeros((max(kcap, 1), n))
    Cm = np.zeros(max(m * kcap, 1))
    k = lib().orc_aca_block(_p(pr), m, _p(pc), n, d, KINDS[kind], float(h), float(tol),
                            _p(rp), _p(cp), _p(U), _p(V), _p(Cm))
    return rp[:k].copy(), cp[:k].copy(), U[:k].T.copy(), V[:k].copy(), Cm[: m * k].reshape(m, k).copy()


class Tree:
    """Uniform 2^d tree with neighbour and interaction lists (Sec. 2.1-2.2)."""

    def __init__(self, points, leaf_size: int, eta2=None):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        self.n, self.d = pts.shape
        if eta2 is None:
            eta2 = (self.d, 1)
        num, den = eta2
        self._free = lib().orc_tree_free
        self._h = lib().orc_tree_build(_p(pts), self.n, self.d, int(leaf_size), int(num), int(den))
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        self.kappa = lib().orc_tree_kappa(self._h)

    def __del__(self):
        # at interpreter exit the process frees everything; the order in which
        # objects die there is arbitrary, so nothing is released explicitly
        if getattr(self, "_h", None) and not sys.is_finalizing():
            self._free(self._h)
        self._h = None

    def domain(self):
        lo = np.zeros(3)
        L = np.zeros(1)
        lib().orc_tree_domain(self._h, _p(lo), _p(L))
        return lo[: self.d], float(L[0])

    def order(self):
        o = np.zeros(self.n, np.int64)
        lib().orc_tree_order(self._h, _p(o))
        return o

    def ncell(self, l: int) -> int:
        return int(lib().orc_tree_ncell(self._h, l))

    def cells(self, l: int):
        nc = self.ncell(l)
        key = np.zeros(nc, np.uint64)
        coord = np.zeros((nc, self.d), np.int64)
        first = np.zeros(nc, np.int64)
        count = np.zeros(nc, np.int64)
        parent = np.zeros(nc, np.int64)
        lib().orc_tree_cells(self._h, l, _p(key), _p(coord), _p(first), _p(count), _p(parent))
        return dict(key=key, coord=coord, first=first, count=count, parent=parent)

    def lists(self, l: int, which: str):
        w = 1 if which == "il" else 0
        tot = lib().orc_tree_lists(self._h, l, w, None, None)
        ptr = np.zeros(self.ncell(l) + 1, np.int64)
        idx = np.zeros(max(tot, 1), np.int64)
        lib().orc_tree_lists(self._h, l, w, _p(ptr), _p(idx))
        return ptr, idx[:tot]


class Tree2(Tree):
    """The tree of the general case over the union of targets P and sources
    Q (Sec. 2.1: a leaf holds at most ``leaf_size`` points of each set).
    Union index i < np is p_i, np + j is q_j."""

    def __init__(self, P, Q, leaf_size: int, eta2=None):
        Pp = np.ascontiguousarray(P, dtype=np.float64)
        Qp = np.ascontiguousarray(Q, dtype=np.float64)
        self.np, self.d = Pp.shape
        self.nq = Qp.shape[0]
        self.n = self.np + self.nq
        if eta2 is None:
            eta2 = (self.d, 1)
        num, den = eta2
        self._free = lib().orc_tree_free
        self._h = lib().orc_tree_build2(_p(Pp), self.np, _p(Qp), self.nq, self.d, int(leaf_size), int(num), int(den))
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        self.kappa = lib().orc_tree_kappa(self._h)

    def counts(self, l: int):
        """(targets, sources) per cell of level l."""
        c = self.cells(l)
        src = self.order() >= self.np
        ns = np.array([src[f:f + k].sum() for f, k in zip(c["first"], c["count"])], np.int64)
        return c["count"] - ns, ns


class H2General:
    """NNCA of the general case (Sec. 2.3): incoming and outgoing pivots and
    operators per cell and the matvec y = A~ x, A_ij = K(p_i, q_j)."""

    def __init__(self, tree: Tree2, kind: str, tol: float, h: float = 1.0, policy: int = 1):
        self.tree = tree
        self.kind = kind
        self.h = float(h)
        self._free = lib().orc_g2_free
        self._h = lib().orc_g2_new(tree._h, KINDS[kind], float(h), float(tol), int(policy))
        if not self._h:
            raise ValueError("not a tree of the general case")
        self.lmin = lib().orc_g2_lmin(self._h)
        lib().orc_g2_build(self._h)

    def __del__(self):
        if getattr(self, "_h", None) and not sys.is_finalizing():
            self._free(self._h)
        self._h = None

    def cell(self, half: str, l: int, b: int):
        """half "in": piv = t^{B,i} (P indices), colpts = s^{B,i} (Q), C (m x k)
        = U_B or the stacked C_{B_c B}; half "out": piv = s^{B,o} (Q),
        colpts = t^{B,o} (P), C = V_B or the stacked T_{B B_c}^T."""
        h = 0 if half == "in" else 1
        mnk = np.zeros(4, np.int64)
        if lib().orc_g2_cell(self._h, h, l, b, _p(mnk), None, None, None, None) != 0:
            raise KeyError((half, l, b))
        m, n, k, pt = (int(v) for v in mnk)
        piv = np.zeros(max(k, 1), np.int64)
        col = np.zeros(max(k, 1), np.int64)
        tt = np.zeros(max(m, 1), np.int64)
        Cm = np.zeros(max(m * k, 1))
        lib().orc_g2_cell(self._h, h, l, b, None, _p(piv), _p(col), _p(tt), _p(Cm))
        return dict(m=m, n=n, k=k, passthrough=bool(pt), piv=piv[:k].copy(),
                    colpts=None if pt else col[:k].copy(), tt=tt[:m].copy(),
                    C=Cm[: m * k].reshape(m, k).copy())

    def matvec(self, x, adjoint: bool = False) -> np.ndarray:
        """A~ x (x over Q) or, with adjoint, A~^T x (x over P)."""
        x = np.asarray(x, dtype=np.float64)
        nin, nout = (self.tree.np, self.tree.nq) if adjoint else (self.tree.nq, self.tree.np)
        vec = x.ndim == 1
        X = np.ascontiguousarray(x.reshape(nin, -1).T)
        Y = np.zeros((X.shape[0], nout))
        lib().orc_g2_matvec(self._h, _p(X), _p(Y), X.shape[0], int(adjoint))
        return Y[0] if vec else Y.T.copy()

    def interactions(self):
        out = np.zeros(2 + self.tree.kappa + 1, np.int64)
        lib().orc_g2_interactions(self._h, _p(out))
        return int(out[0]), int(out[1])

    def interactions_by_level(self):
        out = np.zeros(2 + self.tree.kappa + 1, np.int64)
        lib().orc_g2_interactions(self._h, _p(out))
        return [int(v) for v in out[2:]]


class H2:
    """NNCA pivots, transfer operators and the H2 matvec (Sec. 2.3-4)."""

    def __init__(self, tree: Tree, kind: str, tol: float, h: float = 1.0, policy: int = 1,
                 build: bool = True, _handle=None):
        self.tree = tree
        self.kind = kind
        self.h = float(h)
        self._free = lib().orc_h2_free
        if _handle is not None:
            self._h = _handle
            self.lmin = lib().orc_h2_lmin(self._h)
            return
        self._h = lib().orc_h2_new(tree._h, KINDS[kind], float(h), float(tol), int(policy))
        self.lmin = lib().orc_h2_lmin(self._h)
        if build:
            self.build()

    def __del__(self):
        if getattr(self, "_h", None) and not sys.is_finalizing():
            self._free(self._h)
        self._h = None

    def build(self, level: int | None = None, cells=None):
        if level is None:
            lib().orc_h2_build(self._h, 0, None, -1)
        else:
            c = np.ascontiguousarray(cells, dtype=np.int64)
            lib().orc_h2_build(self._h, int(level), _p(c), c.shape[0])

    def cell(self, l: int, b: int):
        mnk = np.zeros(4, np.int64)
        if lib().orc_h2_cell(self._h, l, b, _p(mnk), None, None, None, None) != 0:
            raise KeyError((l, b))
        m, n, k, pt = (int(v) for v in mnk)
        piv = np.zeros(max(k, 1), np.int64)
        col = np.zeros(max(k, 1), np.int64)
        tt = np.zeros(max(m, 1), np.int64)
        Cm = np.zeros(max(m * k, 1))
        lib().orc_h2_cell(self._h, l, b, None, _p(piv), _p(col), _p(tt), _p(Cm))
        return dict(m=m, n=n, k=k, passthrough=bool(pt), piv=piv[:k].copy(),
                    colpts=None if pt else col[:k].copy(), tt=tt[:m].copy(),
                    C=Cm[: m * k].reshape(m, k).copy())

    def matvec(self, x, adjoint: bool = False) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        n = self.tree.n
        vec = x.ndim == 1
        X = np.ascontiguousarray(x.reshape(n, -1).T)
        Y = np.zeros_like(X)
        lib().orc_h2_matvec(self._h, _p(X), _p(Y), X.shape[0], int(adjoint))
        return Y[0] if vec else Y.T.copy()

    def interactions(self):
        """(transverse, near-field) kernel interactions of one matvec column."""
        out = np.zeros(2 + self.tree.kappa + 1, np.int64)
        lib().orc_h2_interactions(self._h, _p(out))
        return int(out[0]), int(out[1])

    def interactions_by_level(self):
        """Transverse interactions of each level 0..kappa (one column)."""
        out = np.zeros(2 + self.tree.kappa + 1, np.int64)
        lib().orc_h2_interactions(self._h, _p(out))
        return [int(v) for v in out[2:]]

    def frozen(self, h: float) -> "H2":
        """The same pivots with every operator re-evaluated at length scale h
        (Gaussian only): C_B = K_h(t~, J) K_h(I, J)^{-1}, M2L and near field
        at h."""
        p = lib().orc_h2_frozen(self._h, float(h))
        if not p:
            raise ValueError("frozen re-evaluation failed (kernel or zero pivot)")
        return H2(self.tree, self.kind, 0.0, h=h, _handle=p)

    def grad_h(self, x, g, parts: int = 7) -> float:
        """g^T (dA~/dh) x with the pivots frozen (forward-mode derivative of
        every step of the matvec); x, g: (n,) in original order."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        return float(lib().orc_h2_grad_h(self._h, _p(x), _p(g), int(parts)))


def dense_grad_h(points, x, g, h: float) -> float:
    """The plain definition sum_ij g_i x_j dK/dh(r_ij) for the Gaussian."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n, d = pts.shape
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return float(lib().orc_dense_grad_h(_p(pts), n, d, float(h), _p(x), _p(g)))


def gmres(apply, f, tol: float = 1e-10, max_iter: int = 500, restart: int = 50, x0=None):
    """Restarted GMRES(restart) for M x = f, M given by ``apply`` (Saad,
    Iterative Methods for Sparse Linear Systems, Alg. 6.9 with Givens
    rotations, Sec. 6.5.3): Arnoldi by modified Gram-Schmidt, the
    least-squares problem of the Hessenberg matrix by plane rotations.
    Stops when the recurrence's relative residual is at most tol or after
    max_iter applications.  Returns (x, applications, relative residual of
    the final x recomputed as ||f - M x|| / ||f||)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    fn = np.linalg.norm(f)
    if fn == 0.0:
        return np.zeros(n), 0, 0.0
    it = 0
    while True:
        r = f - apply(x)
        beta = np.linalg.norm(r)
        if beta / fn <= tol or it >= max_iter:
            return x, it, beta / fn
        m = restart
        V = np.zeros((m + 1, n))
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j = 0
        done = False
        while j < m and it < max_iter:
            w = apply(V[j])
            it += 1
            for i in range(j + 1):
                Hm[i, j] = w @ V[i]
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] > 0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                a = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = a
            rr = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / rr if rr > 0 else 1.0
            sn[j] = Hm[j + 1, j] / rr if rr > 0 else 0.0
            Hm[j, j] = rr
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j += 1
            if abs(g[j]) / fn <= tol or Hm[j, j - 1] == 0 and rr == 0:
                done = True
                break
        y = np.linalg.solve(np.triu(Hm[:j, :j]), g[:j]) if j > 0 else np.zeros(0)
        x = x + V[:j].T @ y
        if done or it >= max_iter:
            return x, it, np.linalg.norm(f - apply(x)) / fn


def svm_objective(K, y, alpha, beta: float) -> float:
    """The penalised SVM dual L(alpha) of Exp. 6 (Sec. 5) from a dense kernel
    matrix: the sum of alpha, minus half the quadratic form of K with the
    signed weights y * alpha, minus half of beta times the squared constraint
    residual sum(alpha * y)."""
    v = np.asarray(y, dtype=np.float64) * np.asarray(alpha, dtype=np.float64)
    return float(np.sum(alpha) - 0.5 * (v @ (K @ v)) - 0.5 * beta * np.sum(v) ** 2)


def svm_step_size(apply, n: int, beta: float, steps: int = 30) -> float:
    """The gradient-ascent step 1 / (||K||_2 + beta n): ||K||_2 by `steps`
    power-method steps on the symmetric positive definite K, started at the
    normalised all-ones vector (beta n bounds the penalty's Hessian beta y
    y^T for labels of modulus 1)."""
    u = np.full(n, 1.0 / np.sqrt(n))
    lam = 0.0
    for _ in range(steps):
        w = apply(u)
        lam = float(np.linalg.norm(w))
        if not lam > 0.0:
            raise ValueError("the kernel matrix has no positive norm")
        u = w / lam
    return 1.0 / (lam + beta * n)


def svm_train(apply, y, lam: float = 1.0, beta: float = 1.0, eta: float = 0.0, tol: float = 1e-8,
              max_iter: int = 1000, alpha0=None):
    """Kernel SVM training of Exp. 6 (Sec. 5): gradient ascent on the
    penalised dual, alpha <- alpha + eta dL/dalpha with the gradient in the
    paper's vector form 1 - y .* (K v) - beta sum(v) y, v = y .* alpha, each
    step followed by the projection onto the box 0 <= alpha <= lam.  K v is
    `apply(v)`.  eta <= 0 takes svm_step_size.  Stops after max_iter steps or
    at the first step with ||alpha_new - alpha|| <= tol ||alpha_new|| (||.||
    read as 1 when alpha_new = 0).  Returns (alpha, bias, steps, eta); the
    bias is the mean of y_i - (K v)_i over the free support vectors 0 <
    alpha_i < lam of the final iterate (0 when there are none)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    if not eta > 0.0:
        eta = svm_step_size(apply, n, beta)
    a = np.zeros(n) if alpha0 is None else np.array(alpha0, dtype=np.float64)
    it = 0
    while it < max_iter:
        v = y * a
        g = 1.0 - y * apply(v) - beta * np.sum(v) * y
        an = np.clip(a + eta * g, 0.0, lam)
        dn = np.linalg.norm(an - a)
        nn = np.linalg.norm(an)
        a = an
        it += 1
        if dn <= tol * (nn if nn > 0.0 else 1.0):
            break
    kv = apply(y * a)
    free = (a > 0.0) & (a < lam)
    b = float(np.mean(y[free] - kv[free])) if free.any() else 0.0
    return a, b, it, eta


def svm_decision(apply, y, alpha, bias: float):
    """The SVM decision function of Exp. 6, f(x) = sum_i alpha_i y_i K(x_i, x)
    + b, at the points where `apply` evaluates the kernel sums over the
    training points; the label is sgn f."""
    return apply(np.asarray(y, dtype=np.float64) * np.asarray(alpha, dtype=np.float64)) + bias
