"""Seeded synthetic path generators for the signature-kernel workloads.

This module holds no arithmetic of the numerical schemes: it only draws
piecewise-linear paths (arrays of points) with numpy's PCG64 generator.  Both
the FP64 oracle tests and the GPU path consume its output.

Every path is returned as points, shape ``(n_paths, n_points, d)``, starting at
the origin unless stated.  Conventions:

* "L steps" means L increments, i.e. L + 1 points.
* Draws happen in FP64 in the order written in each function, so a seed fixes
  the values exactly.
* FP32 workloads are rounded to FP32 here; the oracle then reads those FP32
  values promoted to FP64, so input quantisation is not counted as error.

The paper's experiments use Brownian paths and sin/cos-of-Gaussian paths
(Section 4 and Appendix B, eq. (sinpath)); the named workloads below follow the
same families at the sizes of the benchmark configurations.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "brownian",
    "sin_cos_paths",
    "oscillatory_pairs",
    "small_fp64_gram",
    "batched_interp_gram",
    "uneven_pairs",
    "mmd_sets",
    "large_gram",
    "long_pair",
    "WORKLOADS",
]


def _points_from_increments(dx: np.ndarray) -> np.ndarray:
    z = np.zeros(dx.shape[:-2] + (1, dx.shape[-1]), dtype=np.float64)
    return np.concatenate([z, np.cumsum(dx, axis=-2)], axis=-2)


def brownian(rng: np.random.Generator, n: int, steps: int, d: int, std: float,
             drift: float = 0.0) -> np.ndarray:
    """Brownian paths from 0: increments i.i.d. N(drift, std^2) per coordinate."""
    dx = rng.normal(drift, std, size=(n, steps, d))
    return _points_from_increments(dx)


def sin_cos_paths(rng: np.random.Generator, n: int, length: int, d: int = 2):
    """Appendix B, eq. (sinpath): x_i = sin(U_i), y_i = cos(V_i), U, V ~ N(0, I)."""
    u = rng.normal(size=(n, length, d))
    v = rng.normal(size=(n, length, d))
    return np.sin(u), np.cos(v)


def small_fp64_gram(seed: int = 0):
    """8x8 Gram, paths in R^3 with 64 Brownian steps of variance 1/64 per
    coordinate from 0, plus a time channel t_m = m/64 (so d = 4). FP64.

    Draw order: all X increments (8, 64, 3), then all Y increments.
    """
    rng = np.random.default_rng(seed)
    steps = 64
    x = brownian(rng, 8, steps, 3, np.sqrt(1.0 / steps))
    y = brownian(rng, 8, steps, 3, np.sqrt(1.0 / steps))
    t = (np.arange(steps + 1, dtype=np.float64) / steps)[None, :, None]
    x = np.concatenate([x, np.broadcast_to(t, (8, steps + 1, 1))], axis=-1)
    y = np.concatenate([y, np.broadcast_to(t, (8, steps + 1, 1))], axis=-1)
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def batched_interp_gram(seed: int = 0, n: int = 128, steps: int = 256, d: int = 8):
    """128x128 Gram, paths in R^8 with 256 Brownian steps of std 0.5/sqrt(256).
    FP32 (rounded here)."""
    rng = np.random.default_rng(seed)
    std = 0.5 / np.sqrt(steps)
    x = brownian(rng, n, steps, d, std)
    y = brownian(rng, n, steps, d, std)
    return x.astype(np.float32), y.astype(np.float32)


def oscillatory_pairs(rng: np.random.Generator, lengths, d: int = 16,
                      n_sines: int = 3):
    """Each coordinate = sum of n_sines terms (1/sqrt(d)) sin(w t + phi) plus
    N(0, 0.01) noise, with w ~ U[10, 200], phi ~ U[0, 2 pi), t_m = m/(len-1)."""
    out = []
    amp = 1.0 / np.sqrt(d)
    for ln in lengths:
        ln = int(ln)
        t = np.arange(ln, dtype=np.float64) / max(ln - 1, 1)
        w = rng.uniform(10.0, 200.0, size=(n_sines, d))
        phi = rng.uniform(0.0, 2 * np.pi, size=(n_sines, d))
        p = amp * np.sin(t[:, None, None] * w[None] + phi[None]).sum(axis=1)
        p = p + rng.normal(0.0, 0.1, size=(ln, d))
        out.append(p)
    return out


def uneven_pairs(seed: int = 0, npairs: int = 4096, lo: int = 32, hi: int = 2048,
                 d: int = 16):
    """4096 independent (x, y) pairs; point counts uniform on {lo..hi}, drawn
    independently for x and y; oscillatory paths in R^16. FP32.

    Returns (xs, ys): two lists of (len_i, d) float32 arrays."""
    rng = np.random.default_rng(seed)
    lx = rng.integers(lo, hi + 1, size=npairs)
    ly = rng.integers(lo, hi + 1, size=npairs)
    xs = [a.astype(np.float32) for a in oscillatory_pairs(rng, lx, d)]
    ys = [a.astype(np.float32) for a in oscillatory_pairs(rng, ly, d)]
    return xs, ys


def mmd_sets(seed: int = 0, n: int = 64, steps: int = 512, d: int = 5,
             drift: float = 0.3):
    """Two sets of 64 Brownian paths in R^5 with 512 steps of variance 1/512;
    Y has drift 0.3 per unit time (0.3/512 per step). FP32."""
    rng = np.random.default_rng(seed)
    std = np.sqrt(1.0 / steps)
    x = brownian(rng, n, steps, d, std)
    y = brownian(rng, n, steps, d, std, drift=drift / steps)
    return x.astype(np.float32), y.astype(np.float32)


def large_gram(seed: int = 0, n: int = 1024, steps: int = 1024, d: int = 32):
    """1024x1024 cross Gram, paths in R^32, 1024 Brownian steps with
    per-coordinate variance 1/sqrt(32) so that the cell constants have unit
    standard deviation. FP32."""
    rng = np.random.default_rng(seed)
    std = np.sqrt(1.0 / np.sqrt(d))
    x = brownian(rng, n, steps, d, std)
    y = brownian(rng, n, steps, d, std)
    return x.astype(np.float32), y.astype(np.float32)


def long_pair(seed: int = 0, steps: int = 16384, d: int = 8):
    """One pair of long paths (far more rows than one wave's 64 lanes): R^d
    Brownian paths with `steps` steps of std 0.5/sqrt(steps), x then y.
    FP32 (rounded here)."""
    rng = np.random.default_rng(seed)
    std = 0.5 / np.sqrt(steps)
    x = brownian(rng, 1, steps, d, std)
    y = brownian(rng, 1, steps, d, std)
    return x.astype(np.float32), y.astype(np.float32)


def long_paths_gram(seed: int = 0, n: int = 4, steps: int = 8192, d: int = 8):
    """A small Gram of long paths (few pairs, each spanning many 64-row
    strips): X then Y, n R^d Brownian paths each with `steps` steps of std
    0.5/sqrt(steps).  FP32 (rounded here)."""
    rng = np.random.default_rng(seed)
    std = 0.5 / np.sqrt(steps)
    X = brownian(rng, n, steps, d, std)
    Y = brownian(rng, n, steps, d, std)
    return X.astype(np.float32), Y.astype(np.float32)


WORKLOADS = {
    "small_fp64_gram": small_fp64_gram,
    "batched_interp_gram": batched_interp_gram,
    "uneven_pairs": uneven_pairs,
    "mmd_sets": mmd_sets,
    "large_gram": large_gram,
    "long_pair": long_pair,
    "long_paths_gram": long_paths_gram,
}
