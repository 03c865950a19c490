"""ctypes binding of the C FP64 oracle ``sko.c`` (test infrastructure only).

Results are (mantissa, exponent) pairs with value mantissa * 2**exponent.
Paths are points with unit partitions s_i = i, t_j = j.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

FD, APPROX, INTERP, FD2 = 0, 1, 2, 3
# the approximation scheme evaluated with FP32-rounded increments, constants
# and edge coefficients of degree >= 2 (FP64 arithmetic): a pair's
# conditioning floor for evaluation with that FP32 state, used to tell
# FP32-resolvable pairs apart (not a scheme)
APPROX_F32MODEL = 4
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i64, dp, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        L.sko_gram.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64, i64, dp, i64, i64, i64,
                               dp, i64p, ctypes.c_int]
        L.sko_gram.restype = ctypes.c_int
        L.sko_pairs.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, dp, i64p, i64, i64,
                                dp, i64p, ctypes.c_int]
        L.sko_pairs.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def default_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _refine(paths, lam: int):
    """Dyadic refinement of the points (hybrid method: the polynomial scheme
    on the refined grid); no scheme arithmetic."""
    from .schemes import refine_points
    return [refine_points(p, lam) for p in paths]


def gram(X, Y, scheme: int, order: int, threads: int | None = None, lam: int = 0):
    """Mantissa/exponent Gram K[a, b] of paths X (nx, lx_pts, d), Y (ny, ly_pts, d).
    lam > 0 with a polynomial scheme: the hybrid method (scheme on the
    lam-order dyadic refinement of the grid)."""
    if lam and scheme in (APPROX, INTERP):
        X = np.stack(_refine(np.asarray(X, dtype=np.float64), lam))
        Y = np.stack(_refine(np.asarray(Y, dtype=np.float64), lam))
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    nx, lxp, d = X.shape
    ny, lyp, d2 = Y.shape
    assert d == d2
    mant = np.zeros((nx, ny))
    expo = np.zeros((nx, ny), dtype=np.int64)
    rc = lib().sko_gram(scheme, order, _dp(X), nx, lxp, _dp(Y), ny, lyp, d, _dp(mant), _ip(expo),
                        threads or default_threads())
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return mant, expo


def pairs(xs, ys, scheme: int, order: int, threads: int | None = None, lam: int = 0):
    """Mantissa/exponent of k(xs[p], ys[p]) for lists of (len_p, d) point arrays
    (lam > 0 with a polynomial scheme: the hybrid method, as in gram)."""
    assert len(xs) == len(ys)
    if lam and scheme in (APPROX, INTERP):
        xs = _refine([np.asarray(a, dtype=np.float64) for a in xs], lam)
        ys = _refine([np.asarray(b, dtype=np.float64) for b in ys], lam)
    d = xs[0].shape[1]
    xoff = np.zeros(len(xs) + 1, dtype=np.int64)
    yoff = np.zeros(len(ys) + 1, dtype=np.int64)
    xoff[1:] = np.cumsum([len(a) for a in xs])
    yoff[1:] = np.cumsum([len(a) for a in ys])
    Xc = np.ascontiguousarray(np.concatenate(xs), dtype=np.float64)
    Yc = np.ascontiguousarray(np.concatenate(ys), dtype=np.float64)
    mant = np.zeros(len(xs))
    expo = np.zeros(len(xs), dtype=np.int64)
    rc = lib().sko_pairs(scheme, order, _dp(Xc), _ip(xoff), _dp(Yc), _ip(yoff), len(xs), d,
                         _dp(mant), _ip(expo), threads or default_threads())
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return mant, expo


def value(mant, expo):
    """mantissa * 2**exponent as float64 (may overflow to inf)."""
    return np.ldexp(np.asarray(mant, dtype=np.float64), np.asarray(expo, dtype=np.int64))
