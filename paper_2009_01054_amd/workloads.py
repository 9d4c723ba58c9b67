"""Seeded synthetic inputs shaped like the paper's interaction data sets.

This module holds input preparation only — feature draws, base kernel
matrices built from them, pair sampling and labels — and none of the
pairwise-kernel or solver arithmetic.  Both the GPU path and the CPU oracle
consume what it produces; neither imports the other.

Every generator draws from ``numpy.random.default_rng([200901054, cfg, pid])``
in a fixed order, so a (config, problem) id always yields the same arrays.

Shapes follow the data sets of Table 5 (Section 5): a Merget-like
heterogeneous set (drugs x targets at ~20-25% density), a homogeneous
kernel-filling-scale set of unordered pairs, a complete (100% dense) grid, and
many uneven Metz/Merget-sized problems.  The real data sets are not used;
these draws stand in for them.

Base kernels: Gaussian ``exp(-||x - y||^2 / (2 sigma^2))`` with sigma = 4
(the squared norm follows the Gaussian definition given with the Metz data in
Section 5; the bandwidth is a reading, see the design notes) and the linear
kernel ``<x, y>``.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 200901054
SIGMA = 4.0
LAMBDA_GRID = tuple(10.0 ** k for k in range(-4, 4))  # 1e-4 .. 1e3, 8 values


def rng_for(cfg: int, pid: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, int(cfg), int(pid)])


# ----------------------------------------------------------------- base kernels
def gaussian_kernel(X: np.ndarray, Y: np.ndarray | None = None, sigma: float = SIGMA) -> np.ndarray:
    """Gaussian base kernel matrix, FP64, exactly symmetric when Y is None."""
    X = np.asarray(X, dtype=np.float64)
    Yv = X if Y is None else np.asarray(Y, dtype=np.float64)
    sq = (X * X).sum(1)[:, None] + (Yv * Yv).sum(1)[None, :] - 2.0 * (X @ Yv.T)
    np.maximum(sq, 0.0, out=sq)
    K = np.exp(-sq / (2.0 * sigma * sigma))
    if Y is None:
        K = 0.5 * (K + K.T)
        np.fill_diagonal(K, 1.0)
    return np.ascontiguousarray(K)


def linear_kernel(X: np.ndarray, Y: np.ndarray | None = None) -> np.ndarray:
    """Linear base kernel matrix <x, y>, FP64, exactly symmetric when Y is None."""
    X = np.asarray(X, dtype=np.float64)
    Yv = X if Y is None else np.asarray(Y, dtype=np.float64)
    K = X @ Yv.T
    if Y is None:
        K = 0.5 * (K + K.T)
    return np.ascontiguousarray(K)


# --------------------------------------------------------------------- sampling
def sample_grid_pairs(rng: np.random.Generator, m: int, q: int, n: int):
    """n distinct (drug, target) cells of the m x q grid, uniform, in draw order."""
    idx = rng.choice(m * q, size=n, replace=False)
    return (idx // q).astype(np.int32), (idx % q).astype(np.int32)


def sample_unordered_pairs(rng: np.random.Generator, m: int, n: int):
    """n distinct unordered pairs {p, p'} (p != p') of m objects, stored (min, max)."""
    total = m * (m - 1) // 2
    k = rng.choice(total, size=n, replace=False).astype(np.int64)
    # row-major enumeration of the strict upper triangle
    p = np.arange(m, dtype=np.int64)
    start = p * (m - 1) - p * (p - 1) // 2  # index of (p, p+1)
    row = np.searchsorted(start, k, side="right") - 1
    col = k - start[row] + row + 1
    return row.astype(np.int32), col.astype(np.int32)


def bilinear_labels(rng, Xd, Xt, d, t, rank: int = 10, noise_std: float = 0.1):
    """y_j = x_{d_j}^T A B^T x_{t_j}, normalised to unit variance, plus N(0, noise_std^2)."""
    A = rng.standard_normal((Xd.shape[1], rank))
    B = rng.standard_normal((Xt.shape[1], rank))
    Ld = Xd @ A  # (m, rank)
    Lt = Xt @ B  # (q, rank)
    y = np.einsum("ij,ij->i", Ld[d], Lt[t])
    y = (y - y.mean()) / max(y.std(), 1e-300)
    y = y + noise_std * rng.standard_normal(len(y))
    return y


# ---------------------------------------------------------------------- problems
def make_heterogeneous(cfg: int, pid: int, m: int, q: int, n: int, dim: int,
                       n_out: int | None = None, kernel: str = "gaussian",
                       labels: bool = False, nrhs: int = 1):
    """Heterogeneous drug x target problem.

    Output pairs are the training pairs unless ``n_out`` asks for a separate
    sample of output pairs (a prediction set drawn from the same grid).
    """
    rng = rng_for(cfg, pid)
    Xd = rng.standard_normal((m, dim))
    Xt = rng.standard_normal((q, dim))
    if kernel == "gaussian":
        D, T = gaussian_kernel(Xd), gaussian_kernel(Xt)
    else:
        D, T = linear_kernel(Xd), linear_kernel(Xt)
    c, e = sample_grid_pairs(rng, m, q, n)
    if n_out is None:
        a, b = c.copy(), e.copy()
    else:
        a, b = sample_grid_pairs(rng, m, q, n_out)
    v = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    out = dict(D=D, T=T, a=a, b=b, c=c, e=e, v=v, m=m, q=q, Xd=Xd, Xt=Xt)
    if labels:
        out["y"] = bilinear_labels(rng, Xd, Xt, c, e)
    return out


def make_homogeneous(cfg: int, pid: int, m: int, n: int, dim: int, n_out: int | None = None,
                     kernel: str = "linear", nrhs: int = 1):
    """Homogeneous problem: n distinct unordered pairs of m objects (stored (min, max))."""
    rng = rng_for(cfg, pid)
    X = rng.standard_normal((m, dim))
    D = linear_kernel(X) if kernel == "linear" else gaussian_kernel(X)
    c, e = sample_unordered_pairs(rng, m, n)
    if n_out is None:
        a, b = c.copy(), e.copy()
    else:
        a, b = sample_unordered_pairs(rng, m, n_out)
    v = rng.standard_normal((n, nrhs)) if nrhs > 1 else rng.standard_normal(n)
    return dict(D=D, T=D, a=a, b=b, c=c, e=e, v=v, m=m, q=m, X=X)


# ------------------------------------------------- the five benchmark workloads
def config1():
    """Kronecker GVT, FP64: m=q=64, Gaussian(sigma=4) on 16-dim N(0,1) features,
    n=2000 pairs of the 64x64 grid without replacement, outputs = training pairs."""
    return make_heterogeneous(1, 0, 64, 64, 2000, 16)


def config2():
    """KRR-CG: m=2000 drugs, q=500 targets, Gaussian on 64-dim features,
    n=200k pairs (20% density), rank-10 bilinear labels + N(0, 0.1^2), lambda=1e-2."""
    p = make_heterogeneous(2, 0, 2000, 500, 200_000, 64, labels=True)
    p["lam"] = 1e-2
    return p


def config3(nrhs: int = 1):
    """Fused homogeneous kinds: m=5000 proteins, linear kernel on 128-dim features,
    n=1M unordered pairs; outputs = training pairs."""
    return make_homogeneous(3, 0, 5000, 1_000_000, 128, kernel="linear", nrhs=nrhs)


def config4(m: int = 8192, q: int = 4096, dim: int = 32):
    """Complete data: every (d, t) pair of an m x q grid in natural order;
    Gaussian bases on 32-dim features; V ~ N(0,1) of shape (m, q)."""
    rng = rng_for(4, 0)
    Xd = rng.standard_normal((m, dim))
    Xt = rng.standard_normal((q, dim))
    D, T = gaussian_kernel(Xd), gaussian_kernel(Xt)
    V = rng.standard_normal((m, q))
    return dict(D=D, T=T, V=V, m=m, q=q)


def config5_shapes(nprob: int = 256):
    """(m, q, n) of the batched problems: m, q ~ U{50..1000},
    n ~ U{1000..min(200000, floor(m q / 2))}."""
    rng = rng_for(5, 10_000)
    shapes = []
    for _ in range(nprob):
        m = int(rng.integers(50, 1001))
        q = int(rng.integers(50, 1001))
        hi = min(200_000, (m * q) // 2)
        n = int(rng.integers(1000, hi + 1))
        shapes.append((m, q, n))
    return shapes


def config5_problem(pid: int, shape):
    m, q, n = shape
    return make_heterogeneous(5, pid, m, q, n, 32, labels=True)
