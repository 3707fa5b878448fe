"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds no arithmetic of the solver: it only draws grid jitter and
right-hand sides from a counter-based generator.  The generator is
SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the k-th draw for a seed is
the SplitMix64 finaliser applied to ``seed + (k + 1) * 0x9E3779B97F4A7C15``,
and a uniform double in [0, 1) is its top 53 bits times 2^-53.  The GPU
library implements the same published generator on its own side, so jitter
generated on the device equals the one generated here bit for bit.

Workload recipes (the paper's synthetic Poisson problems, Sec. 2.1 / 6.2):
  * grid: N = 2^L + 1 nodes per side, node (i, j) at (i h + dx, j h + dy),
    h = 1/(N-1); boundary nodes are not moved; interior nodes move by
    dx = (2u - 1) a h, dy likewise, with u drawn at k = 2p (x) and 2p + 1 (y);
  * uniform right-hand side: b_p = 2u - 1 (k = p) on nodes off the
    Dirichlet sides (all interior nodes when every side is Dirichlet), 0 on
    them -- the load vector itself, not f at the nodes;
  * Gaussian right-hand side: Box-Muller on (u at k = 2p, u at k = 2p + 1).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """SplitMix64 output for counters ``k`` (uint64 array) under ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k.astype(np.uint64) + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, k: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def grid_size(L: int) -> int:
    return (1 << L) + 1


def coords(L: int, jitter: float = 0.0, seed: int = 0) -> np.ndarray:
    """Finest-level node coordinates, shape (n, 2), p = j*N + i."""
    N = grid_size(L)
    h = 1.0 / (N - 1)
    i = np.tile(np.arange(N, dtype=np.float64), N)
    j = np.repeat(np.arange(N, dtype=np.float64), N)
    x = i * h
    y = j * h
    if jitter != 0.0:
        p = np.arange(N * N, dtype=np.uint64)
        ii = np.tile(np.arange(N), N)
        jj = np.repeat(np.arange(N), N)
        interior = (ii > 0) & (jj > 0) & (ii < N - 1) & (jj < N - 1)
        ux = uniform(seed, np.uint64(2) * p)
        uy = uniform(seed, np.uint64(2) * p + np.uint64(1))
        dx = (2.0 * ux - 1.0) * jitter * h
        dy = (2.0 * uy - 1.0) * jitter * h
        x = np.where(interior, x + dx, x)
        y = np.where(interior, y + dy, y)
    return np.ascontiguousarray(np.stack([x, y], axis=1))


def interior_mask(L: int) -> np.ndarray:
    N = grid_size(L)
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    return (ii > 0) & (jj > 0) & (ii < N - 1) & (jj < N - 1)


def free_mask(L: int, dirichlet_sides: int = 15) -> np.ndarray:
    """Nodes off the Dirichlet sides (bits 1: x = 0, 2: x = 1, 4: y = 0,
    8: y = 1); with every side Dirichlet, the interior nodes."""
    N = grid_size(L)
    ii = np.tile(np.arange(N), N)
    jj = np.repeat(np.arange(N), N)
    on = (((ii == 0) & bool(dirichlet_sides & 1)) | ((ii == N - 1) & bool(dirichlet_sides & 2)) |
          ((jj == 0) & bool(dirichlet_sides & 4)) | ((jj == N - 1) & bool(dirichlet_sides & 8)))
    return ~on


def rhs_uniform(L: int, seed: int, dirichlet_sides: int = 15) -> np.ndarray:
    """b_p = 2u - 1 off the Dirichlet sides, 0 on them."""
    N = grid_size(L)
    u = uniform(seed, np.arange(N * N, dtype=np.uint64))
    return np.where(free_mask(L, dirichlet_sides), 2.0 * u - 1.0, 0.0)


def rhs_gaussian(L: int, seed: int) -> np.ndarray:
    """Standard normal b_p (Box-Muller) on interior nodes, 0 on the boundary."""
    N = grid_size(L)
    p = np.arange(N * N, dtype=np.uint64)
    u1 = uniform(seed, np.uint64(2) * p)
    u2 = uniform(seed, np.uint64(2) * p + np.uint64(1))
    g = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return np.where(interior_mask(L), g, 0.0)


def batch_levels(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Levels drawn uniformly from {lo..hi} (one draw per problem)."""
    u = uniform(seed, np.arange(count, dtype=np.uint64))
    return lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)


def batch_jitter(count: int, amax: float, seed: int) -> np.ndarray:
    """Per-problem jitter amplitudes drawn uniformly from [0, amax)."""
    return uniform(seed, np.arange(count, dtype=np.uint64)) * amax


def serving_requests(count: int, rate: float, seed: int, lo: int = 6, hi: int = 11,
                     tols=(1e-6, 1e-8, 1e-10), amax: float = 0.25):
    """Open-loop request stream: exponential inter-arrival times at `rate`
    per second (draws 4r), levels with P(L) proportional to 1/L on lo..hi
    (draws 4r+1), tolerances uniform over `tols` (draws 4r+2), jitter
    amplitudes uniform in [0, amax) (draws 4r+3); request r uses grid seed
    5100 + r and right-hand-side seed 5200 + r."""
    r = np.arange(count, dtype=np.uint64)
    u = [uniform(seed, np.uint64(4) * r + np.uint64(c)) for c in range(4)]
    gaps = -np.log1p(-u[0]) / rate
    levels = np.arange(lo, hi + 1)
    w = 1.0 / levels
    cdf = np.cumsum(w) / w.sum()
    L = levels[np.minimum(np.searchsorted(cdf, u[1], side="right"), len(levels) - 1)]
    tol = np.asarray(tols)[np.minimum((u[2] * len(tols)).astype(np.int64), len(tols) - 1)]
    return {"t": np.cumsum(gaps), "L": L.astype(np.int64), "tol": tol, "jitter": u[3] * amax,
            "geom_seed": 5100 + r.astype(np.int64), "rhs_seed": 5200 + r.astype(np.int64)}
