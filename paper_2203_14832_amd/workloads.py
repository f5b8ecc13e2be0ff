"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws points and
right-hand sides.  Every workload is generated on the host in FP64 with
``numpy.random.default_rng(1000 + config_index)`` and fed bit-identically to
the GPU library and to the CPU oracle.

Configurations (the point distributions of the paper's experiments, Sec. 5):
  c1  2D, N=4096 uniform in [-1,1]^2, log|x-y|, leaf 64, tol 1e-8, x ~ U(-1,1)
  c2  3D, N=2^20 uniform in [-1,1]^3, 1/|x-y|, leaf 64, tol 1e-6, x ~ N(0,1)
  c3  3D, N=262144 uniform on the unit sphere, 1/|x-y|, leaf 64, tol 1e-7,
      64 columns N(0,1)
  c4  3D, N=200000 two-component Gaussian mixture (means +-0.5 per axis,
      std 0.3), exp(-r^2/h^2) with h=0.5, leaf 128, tol 1e-6
  c5  32 independent problems, N_b = round(exp(U(ln 1e4, ln 2e5))) points
      uniform in [-1,1]^3, 1/r, leaf 64, tol 1e-6, 8 columns each
The experiments' other point sets: chebyshev_grid (Exp. 2 and 4) and
nystrom_grid (the integral equation of Exp. 5).
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    "c1": dict(index=0, dim=2, n=4096, kernel="log_r", leaf=64, tol=1e-8, dist="cube", rhs="uniform", nrhs=1, h=1.0),
    "c2": dict(index=1, dim=3, n=1 << 20, kernel="inv_r", leaf=64, tol=1e-6, dist="cube", rhs="normal", nrhs=1, h=1.0),
    "c3": dict(index=2, dim=3, n=262144, kernel="inv_r", leaf=64, tol=1e-7, dist="sphere", rhs="normal", nrhs=64, h=1.0),
    "c4": dict(index=3, dim=3, n=200000, kernel="gauss", leaf=128, tol=1e-6, dist="mixture", rhs="normal", nrhs=1, h=0.5),
}


def seed_of(config: str) -> int:
    return 1000 + CONFIGS[config]["index"]


def draw_points(dist: str, n: int, dim: int, rng: np.random.Generator) -> np.ndarray:
    """(n, dim) FP64 points of the named distribution."""
    if dist == "cube":
        return rng.uniform(-1.0, 1.0, size=(n, dim))
    if dist == "sphere":
        g = rng.standard_normal(size=(n, dim))
        return g / np.linalg.norm(g, axis=1, keepdims=True)
    if dist == "mixture":
        z = rng.integers(0, 2, size=n)
        mu = np.where(z[:, None] == 0, 0.5, -0.5)
        return mu + 0.3 * rng.standard_normal(size=(n, dim))
    raise ValueError(dist)


def draw_rhs(kind: str, n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """(n, nrhs) FP64 right-hand sides."""
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, size=(n, nrhs))
    return rng.standard_normal(size=(n, nrhs))


def workload(config: str, n: int | None = None, nrhs: int | None = None, seed_offset: int = 0):
    """Points (n, d) and right-hand sides (n, r) of a configuration.

    ``n``/``nrhs`` override the sizes (same distribution, same seed), which is
    how the tests build reduced cases of every configuration."""
    c = CONFIGS[config]
    n = c["n"] if n is None else int(n)
    r = c["nrhs"] if nrhs is None else int(nrhs)
    rng = np.random.default_rng(seed_of(config) + seed_offset)
    pts = draw_points(c["dist"], n, c["dim"], rng)
    x = draw_rhs(c["rhs"], n, r, rng)
    return pts, x


def cotangent(config: str, n: int | None = None) -> np.ndarray:
    """(n,) FP64 seeded output cotangent g = dL/dy ~ N(0,1) for the backward
    of a configuration (its own stream, seed + 100)."""
    c = CONFIGS[config]
    n = c["n"] if n is None else int(n)
    return np.random.default_rng(seed_of(config) + 100).standard_normal(n)


def chebyshev_grid(n_axis: int, dim: int) -> np.ndarray:
    """(n_axis^dim, dim) points of the tensor-product Chebyshev grid of
    [-1,1]^dim (Exp. 2 and 4): the first-kind nodes cos((2i + 1) pi / (2 n))
    on every axis."""
    c = np.cos((2.0 * np.arange(n_axis) + 1.0) * np.pi / (2.0 * n_axis))
    return np.stack(np.meshgrid(*([c] * dim), indexing="ij"), -1).reshape(-1, dim)


def nystrom_grid(n_axis: int, seed: int = 1005):
    """Points, quadrature weight and density of the integral-equation solve
    (Exp. 5): the n_axis^3 cell centres of a uniform grid on [-1,1]^3, the
    weight (2 / n_axis)^3 of each, and sigma ~ N(0,1) (seeded)."""
    c = -1.0 + (np.arange(n_axis) + 0.5) * (2.0 / n_axis)
    g = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    sigma = np.random.default_rng(seed).standard_normal(g.shape[0])
    return g, (2.0 / n_axis) ** 3, sigma


def batch_sizes(count: int = 32, lo: float = 1e4, hi: float = 2e5, seed: int = 1004):
    """Sizes of the uneven batch: N_b = round(exp(U(ln lo, ln hi)))."""
    ss = np.random.SeedSequence(seed).spawn(count)
    out = []
    for s in ss:
        rng = np.random.default_rng(s)
        out.append(int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi)))))))
    return out


def batch_problem(b: int, n: int, nrhs: int = 8, seed: int = 1004):
    """Points and right-hand sides of problem b of the uneven batch."""
    ss = np.random.SeedSequence(seed).spawn(b + 1)[b]
    rng = np.random.default_rng(ss)
    rng.uniform(size=1)  # the draw that fixed N_b
    pts = rng.uniform(-1.0, 1.0, size=(n, 3))
    x = rng.standard_normal(size=(n, nrhs))
    return pts, x


def svm_dataset(m: int, dim: int = 2, rule: str = "disk", seed: int = 1006, train_frac: float = 0.85):
    """The synthetic two-class data of the kernel SVM (Exp. 6): m points
    uniform in [-1.4,1.4]^2 (dim 2) or [-1,1]^dim (otherwise), labels +1 / -1
    in nearly equal numbers, split per class into train_frac training points
    and the rest for testing (so both parts stay balanced).  Label rules:
      disk  +1 where |x| is below the sample median of |x| (any dim);
      wave  +1 where x_2 > 0.6 sin(1.5 x_1) (2D; balanced by the point
            symmetry x -> -x of the box, which swaps the classes).
    Returns (train points, train labels, test points, test labels), FP64."""
    rng = np.random.default_rng(seed)
    half = 1.4 if dim == 2 else 1.0
    x = rng.uniform(-half, half, size=(m, dim))
    if rule == "disk":
        r = np.linalg.norm(x, axis=1)
        y = np.where(r < np.median(r), 1.0, -1.0)
    elif rule == "wave":
        if dim != 2:
            raise ValueError("the wave rule is 2D")
        y = np.where(x[:, 1] > 0.6 * np.sin(1.5 * x[:, 0]), 1.0, -1.0)
    else:
        raise ValueError(rule)
    tr = []
    te = []
    for c in (1.0, -1.0):
        idx = np.flatnonzero(y == c)
        idx = idx[rng.permutation(idx.size)]
        k = int(round(train_frac * idx.size))
        tr.append(idx[:k])
        te.append(idx[k:])
    tr = np.sort(np.concatenate(tr))
    te = np.sort(np.concatenate(te))
    return x[tr], y[tr], x[te], y[te]
