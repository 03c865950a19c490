"""Gradients of the oracle's forward schemes (test infrastructure only).

* ``complex_step_grad`` -- derivative of a scheme's endpoint with respect to
  every coordinate of every point of x (and y), by the complex-step method:
  f'(v) = Im f(v + i h) / h with h = 1e-30.  Both polynomial schemes are
  analytic in the path points (the approximation scheme is a polynomial in the
  cell constants; the interpolation scheme composes 0F1 series and a linear
  solve), so the result is exact to rounding and independent of any adjoint
  derivation.  Small inputs only (one complex forward per coordinate).
* ``central_fd`` -- central finite differences of any real forward, the check
  used at realistic sizes (step h, error O(h^2)).
"""
from __future__ import annotations

import numpy as np

H_CS = 1e-30


def complex_step_grad(fn, x, y, wrt: str = "x", **kw) -> np.ndarray:
    """d fn(x, y) / d (x or y), same shape as that argument."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    target = x if wrt == "x" else y
    g = np.zeros_like(target)
    for idx in np.ndindex(target.shape):
        pert = target.astype(np.complex128)
        pert[idx] += 1j * H_CS
        val = fn(pert, y, **kw) if wrt == "x" else fn(x, pert, **kw)
        g[idx] = np.imag(val) / H_CS
    return g


def central_fd(f, v: np.ndarray, idx, h: float = 1e-4) -> float:
    """(f(v + h e_idx) - f(v - h e_idx)) / (2h) for a real function f of an array."""
    vp = np.array(v, dtype=np.float64, copy=True)
    vm = np.array(v, dtype=np.float64, copy=True)
    vp[idx] += h
    vm[idx] -= h
    return (f(vp) - f(vm)) / (2.0 * h)
