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
* ``continuous_adjoint_grad`` -- the gradient of the exact kernel by the
  continuous adjoint: the Goursat problem d^2k/dsdt = c(s,t) k is linear in the
  cell constants, and Riemann's method for it gives
      dk(S,T)/dc_ij = integral over cell (i,j) of k(s,t) R(s,t) ds dt,
  with R the solution of the same problem started from the far corner (value
  1 on s = S and on t = T), i.e. the signature kernel of the reversed remaining
  paths.  Both k and R are evaluated inside each cell from their edges by the
  double series of Proposition "prop:a1" (eq. appeq2); their edges come from
  the approximation scheme at a high order on the paths and on the reversed
  paths.  The paper does not treat gradients: this is a second, independent
  route to the gradient of the exact kernel (the GPU computes the discrete
  adjoint of its scheme instead).
"""
from __future__ import annotations

import math

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


def _cell_edges(dx: np.ndarray, dy: np.ndarray, N: int):
    """Bottom and left edges (coefficients in the unit-cell variables) of every
    cell of the approximation scheme at order N on unit partitions, visiting
    rows j, then cells i, as the scheme's definition does."""
    from .schemes import approx_cell
    lx, ly = len(dx), len(dy)
    C = dx @ dy.T
    e0 = np.zeros(N + 1)
    e0[0] = 1.0
    P = np.zeros((lx, ly, N + 1))
    Q = np.zeros((lx, ly, N + 1))
    p = [e0.copy() for _ in range(lx)]
    for j in range(ly):
        q = e0.copy()
        for i in range(lx):
            P[i, j], Q[i, j] = p[i], q
            p[i], q = approx_cell(p[i], q, C[i, j], 1.0, 1.0, N)
    return C, P, Q


def _interior(p: np.ndarray, q: np.ndarray, c: float, M: int) -> np.ndarray:
    """Coefficients a[alpha, beta] of u^alpha v^beta (alpha, beta <= M) of the
    solution inside a unit cell with constant c whose bottom edge is
    sum p_n u^n and left edge sum q_n v^n, from eq. appeq2 of Proposition
    "prop:a1": the p part (n >= 1) contributes to alpha = n + m, beta = m and
    the q part (n >= 0) to alpha = m, beta = n + m, each with weight
    c^m n! / (m! (n + m)!)."""
    fact = np.array([float(math.factorial(k)) for k in range(M + 1)])
    a = np.zeros((M + 1, M + 1))
    for n in range(1, min(len(p), M + 1)):
        m = np.arange(0, M + 1 - n)
        a[n + m, m] += p[n] * c ** m * fact[n] / (fact[m] * fact[n + m])
    for n in range(0, min(len(q), M + 1)):
        m = np.arange(0, M + 1 - n)
        a[m, n + m] += q[n] * c ** m * fact[n] / (fact[m] * fact[n + m])
    return a


def continuous_adjoint_grad(x, y, N: int = 24, M: int = 48):
    """(dk/dc, dk/dx, dk/dy) of the exact signature kernel of the paths x, y
    (points, unit partitions) by the continuous adjoint described above:
    per cell, the integral over [0,1]^2 of k(u, v) R(u, v), with
    R(u, v) = k_rev(1 - u, 1 - v) from the reversed paths' scheme, computed as
    sum_{alpha beta alpha' beta'} a[alpha,beta] a_rev[alpha',beta']
    B(alpha, alpha') B(beta, beta'), B(a, b) = a! b! / (a + b + 1)! the Beta
    integral of u^a (1-u)^b.  Then the chain rule through c_ij = <dx_i, dy_j>."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx, dy = np.diff(x, axis=0), np.diff(y, axis=0)
    lx, ly = len(dx), len(dy)
    C, P, Q = _cell_edges(dx, dy, N)
    _, Pr, Qr = _cell_edges(-dx[::-1], -dy[::-1], N)  # increments of the reversed paths
    f = math.factorial
    B = np.array([[f(a) * f(b) / f(a + b + 1) for b in range(M + 1)] for a in range(M + 1)])
    G = np.zeros((lx, ly))
    for i in range(lx):
        for j in range(ly):
            a = _interior(P[i, j], Q[i, j], C[i, j], M)
            ar = _interior(Pr[lx - 1 - i, ly - 1 - j], Qr[lx - 1 - i, ly - 1 - j], C[i, j], M)
            G[i, j] = float(np.sum(a * (B @ ar @ B.T)))
    gdx = G @ dy          # dk/d(dx_i) = sum_j g_ij dy_j
    gdy = G.T @ dx
    gx = np.zeros_like(x)
    gx[1:] += gdx
    gx[:-1] -= gdx
    gy = np.zeros_like(y)
    gy[1:] += gdy
    gy[:-1] -= gdy
    return G, gx, gy
