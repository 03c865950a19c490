"""FP64 reference implementation of the signature-kernel schemes (test
infrastructure only; never part of the GPU product path).

Everything here is written from "Numerical Schemes for Signature Kernels"
(Cass, Piatti, Pei) in the paper's own order and notation, with no blocking,
fusion or reformulation:

* ``fd_scheme``           -- Definition "Dyadic finite differences approximation
                             scheme" (Section 2), first-order explicit rule on
                             the lambda-refined grid.
* ``fd2_scheme``          -- the second-order explicit rule of Remark
                             "higherfd" (eq. secondexplicitscheme) on the same
                             refined grid.
* ``approx_cell``         -- Proposition "approxsolution" (eqs. powerseries1/2)
                             truncated at order N, i.e. the explicit map of the
                             remark after Definition "Polynomial approximation
                             numerical scheme" (Section 3.2).
* ``approx_scheme``       -- that definition: recursion over the grid of
                             Definition "lambda" and the averaged endpoint.
* ``hyp0f1``              -- the confluent hypergeometric limit function 0F1
                             defined with Proposition "propinterp".
* ``interp_cell``         -- Proposition "propinterp" (eq. interpformula)
                             evaluated at the Chebyshev extrema of
                             eq. (chebextr), followed by the interpolation
                             operator of Definition "interpooperator".
* ``interp_scheme``       -- Definition "Polynomial interpolation numerical
                             scheme" (Section 3.3).
* ``refine_points`` / ``hybrid_scheme`` -- the hybrid method of the remark
                             after Theorem "prop:globalte": a polynomial scheme
                             run on the lambda-order dyadic refinement of the
                             grid (every segment split into 2**lam equal
                             pieces, as in the finite-difference refinement).
* ``truncated_signature_kernel`` -- the benchmark method of Section 4: inner
                             product of signatures truncated at a level, with
                             signatures from the definition in Section 1 (Chen
                             products of tensor exponentials of increments).

Readings where the paper is ambiguous (kept identical in every implementation):

* Chebyshev extrema: N + 1 nodes, m = 0..N (the definition of the
  interpolation operator asks for N + 1 extrema; the node formula's range
  m = 0..N-1 cannot determine a degree-N interpolant).
* The finite-difference rule uses the kernel at (s_{i+1}, t_j) and
  (s_i, t_{j+1}) in its last term (the index letters printed in the
  definition are taken as a typo, following the trapezoid rule above it).
* Partition times: any increasing partitions may be passed; by default
  s_i = i and t_j = j.

Exponent tracking (optional): the state is kept as mantissa * 2**E with E an
integer, rescaled by exact powers of two after every row of cells, so that
kernels far beyond the FP64 range (long, high-variance paths) stay
representable.  Rescaling by powers of two is exact, so it does not change any
result that is representable.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "increments",
    "cell_constants",
    "fd_scheme",
    "fd2_scheme",
    "approx_cell",
    "approx_scheme",
    "hyp0f1",
    "chebyshev_extrema",
    "interp_cell",
    "interp_scheme",
    "truncated_signature",
    "truncated_signature_kernel",
    "gram",
    "mmd2_unbiased",
    "refine_points",
    "hybrid_scheme",
    "mmd_permutation_stats",
    "mmd_permutation_pvalue",
]


def increments(x: np.ndarray) -> np.ndarray:
    """Increments x_{i+1} - x_i of a piecewise-linear path given by points."""
    x = np.asarray(x)
    x = x.astype(np.result_type(x.dtype, np.float64))
    return x[1:] - x[:-1]


def _partition(n_points: int, times: Optional[Sequence[float]]) -> np.ndarray:
    if times is None:
        return np.arange(n_points, dtype=np.float64)
    t = np.asarray(times, dtype=np.float64)
    if t.shape != (n_points,) or np.any(np.diff(t) <= 0):
        raise ValueError("partition must be increasing with one time per point")
    return t


def cell_constants(x, y, s=None, t=None) -> np.ndarray:
    """C_ij = <x_{s_{i+1}} - x_{s_i}, y_{t_{j+1}} - y_{t_j}> / ((s_{i+1}-s_i)(t_{j+1}-t_j)),
    the constant of the PDE on rectangle (i, j) (Definition of the polynomial
    approximation scheme)."""
    dx, dy = increments(x), increments(y)
    s = _partition(len(dx) + 1, s)
    t = _partition(len(dy) + 1, t)
    return (dx @ dy.T) / np.outer(np.diff(s), np.diff(t))


# ---------------------------------------------------------------------------
# Finite differences (Section 2)
# ---------------------------------------------------------------------------

def fd_scheme(x, y, lam: int = 0) -> float:
    """First-order explicit finite-difference scheme on the lambda-order dyadic
    refinement of the grid (Definition "Dyadic finite differences approximation
    scheme").

    The refined partition splits every interval into 2**lam equal pieces; on a
    linear segment the path increment of each piece is the segment increment
    divided by 2**lam.  k(s_0, .) = k(., t_0) = 1, and

        k(s_{i+1}, t_{j+1}) = k(s_{i+1}, t_j) + k(s_i, t_{j+1}) - k(s_i, t_j)
                              + 1/2 <dx_i, dy_j> (k(s_{i+1}, t_j) + k(s_i, t_{j+1})).
    """
    dx, dy = increments(x), increments(y)
    r = 2 ** lam
    dxr = np.repeat(dx / r, r, axis=0)
    dyr = np.repeat(dy / r, r, axis=0)
    m, n = len(dxr), len(dyr)
    k = np.ones((m + 1, n + 1), dtype=np.result_type(dx, dy))
    for i in range(m):
        for j in range(n):
            inner = np.dot(dxr[i], dyr[j])
            k[i + 1, j + 1] = (k[i + 1, j] + k[i, j + 1] - k[i, j]
                               + 0.5 * inner * (k[i + 1, j] + k[i, j + 1]))
    return k[m, n]


def fd2_scheme(x, y, lam: int = 0) -> float:
    """Second-order explicit finite-difference scheme (Remark "higherfd",
    eq. secondexplicitscheme) on the lambda-order dyadic refinement: the
    first-order rule plus the c^2 term of the quadrature,

        k(s_{i+1}, t_{j+1}) = k(s_{i+1}, t_j) + k(s_i, t_{j+1}) - k(s_i, t_j)
                              + 1/2 c (k(s_{i+1}, t_j) + k(s_i, t_{j+1}))
                              + 1/12 c^2 (k(s_{i+1}, t_j) + k(s_i, t_{j+1}) + k(s_i, t_j)),

    with c = <dx_i, dy_j> of the refined pieces (the time steps cancel as in
    the first-order rule)."""
    dx, dy = increments(x), increments(y)
    r = 2 ** lam
    dxr = np.repeat(dx / r, r, axis=0)
    dyr = np.repeat(dy / r, r, axis=0)
    m, n = len(dxr), len(dyr)
    k = np.ones((m + 1, n + 1), dtype=np.result_type(dx, dy))
    for i in range(m):
        for j in range(n):
            c = np.dot(dxr[i], dyr[j])
            k[i + 1, j + 1] = (k[i + 1, j] + k[i, j + 1] - k[i, j]
                               + 0.5 * c * (k[i + 1, j] + k[i, j + 1])
                               + c * c / 12.0 * (k[i + 1, j] + k[i, j + 1] + k[i, j]))
    return k[m, n]


# ---------------------------------------------------------------------------
# Polynomial approximation scheme (Section 3.2)
# ---------------------------------------------------------------------------

def approx_cell(p: np.ndarray, q: np.ndarray, C: float, ds: float, dt: float,
                N: int) -> Tuple[np.ndarray, np.ndarray]:
    """Truncated one-step map Lambda^{<=N} on rectangle [a,b]x[c,d] with
    b - a = ds, d - c = dt (Proposition "approxsolution" followed by the
    truncation pi_N):

      p~_n = sum_{k=0}^{n} p_k (C dt)^{n-k} k! / ((n-k)! n!)
             + sum_{k=1}^{N} q_k C^n dt^{n+k} k! / ((n+k)! n!)
      q~_n = sum_{k=0}^{n} q_k (C ds)^{n-k} k! / ((n-k)! n!)
             + sum_{k=1}^{N} p_k C^n ds^{n+k} k! / ((n+k)! n!)

    for n = 0..N.  p are the coefficients of the bottom edge in powers of
    (s - a), q those of the left edge in powers of (t - c); the outputs are the
    top and right edges in the same variables.
    """
    dtype = np.result_type(p, q, C)
    pt = np.zeros(N + 1, dtype=dtype)
    qt = np.zeros(N + 1, dtype=dtype)
    f = math.factorial
    for n in range(N + 1):
        a = 0.0
        b = 0.0
        for k in range(n + 1):
            a += p[k] * (C * dt) ** (n - k) * f(k) / (f(n - k) * f(n))
            b += q[k] * (C * ds) ** (n - k) * f(k) / (f(n - k) * f(n))
        for k in range(1, N + 1):
            a += q[k] * C ** n * dt ** (n + k) * f(k) / (f(n + k) * f(n))
            b += p[k] * C ** n * ds ** (n + k) * f(k) / (f(n + k) * f(n))
        pt[n] = a
        qt[n] = b
    return pt, qt


def _rescale(vectors, E: int) -> int:
    """Rescale a list of arrays in place by a common power of two so the
    largest magnitude lies in [0.5, 1); return the updated exponent."""
    mx = max((float(np.max(np.abs(v.real))) for v in vectors), default=0.0)
    if mx == 0.0 or not math.isfinite(mx):
        return E
    e = math.frexp(mx)[1]
    for v in vectors:
        v *= 2.0 ** (-e)
    return E + e


def approx_scheme(x, y, N: int, s=None, t=None, track_exponent: bool = False):
    """Order-N polynomial approximation scheme (Definition "Polynomial
    approximation numerical scheme") for the paths given by points x, y on
    partitions s, t.

    Edges start as p^{i,0} = q^{0,j} = (1, 0, ..., 0); cells are visited row by
    row (j outer, i inner), which is a topological order of the recursion
    (p^{i,j+1}, q^{i+1,j}) = Lambda^{<=N}(p^{i,j}, q^{i,j}).  The endpoint is
    the average of the top edge of the last cell at s_{l_x} and its right edge
    at t_{l_y}.

    Returns the kernel value, or (mantissa, exponent) with value
    mantissa * 2**exponent if ``track_exponent``.
    """
    if N < 2:
        raise ValueError("the scheme is defined for N >= 2")
    dx, dy = increments(x), increments(y)
    lx, ly = len(dx), len(dy)
    if lx == 0 or ly == 0:
        return (1.0, 0) if track_exponent else 1.0
    s = _partition(lx + 1, s)
    t = _partition(ly + 1, t)
    ds_all, dt_all = np.diff(s), np.diff(t)
    C = (dx @ dy.T) / np.outer(ds_all, dt_all)
    e0 = np.zeros(N + 1, dtype=C.dtype)
    e0[0] = 1.0
    E = 0
    p = [e0.copy() for _ in range(lx)]  # p^{i,j} for the current row j
    q = e0.copy()
    for j in range(ly):
        q = e0 * 2.0 ** (-E)  # q^{0,j} = 1, in the current scale
        for i in range(lx):
            p[i], q = approx_cell(p[i], q, C[i, j], ds_all[i], dt_all[j], N)
        if track_exponent:
            E = _rescale(p + [q], E)
    ds, dt = ds_all[-1], dt_all[-1]
    top = sum(p[lx - 1][n] * ds ** n for n in range(N + 1))
    right = sum(q[n] * dt ** n for n in range(N + 1))
    m = 0.5 * (top + right)
    return (m, E) if track_exponent else m * 2.0 ** E


# ---------------------------------------------------------------------------
# Polynomial interpolation scheme (Section 3.3)
# ---------------------------------------------------------------------------

def hyp0f1(b: float, z, tol: float = 2.0 ** -60, max_terms: int = 10000):
    """0F1(b; z) = sum_{n>=0} z^n / ((b)_n n!), (b)_n the rising factorial.
    Summed term by term until the term is below tol times the running sum."""
    z = np.asarray(z, dtype=np.result_type(z, np.float64))
    term = np.ones_like(z)
    total = np.ones_like(z)
    for n in range(max_terms):
        term = term * z / ((b + n) * (n + 1))
        total = total + term
        if np.all(np.abs(term) <= tol * np.maximum(np.abs(total), 1e-300)):
            break
    return total


def chebyshev_extrema(N: int, u: float, v: float) -> np.ndarray:
    """Chebyshev extrema rescaled to [u, v] (eq. chebextr), m = 0..N."""
    m = np.arange(N + 1)
    return (v - u) / 2.0 * np.cos(np.pi * m / N) + (u + v) / 2.0


def interp_cell(g: np.ndarray, h: np.ndarray, C: float, a: float, b: float,
                c: float, d: float, N: int) -> Tuple[np.ndarray, np.ndarray]:
    """One step of the interpolation scheme on [a,b]x[c,d].

    g, h: coefficients of the bottom / left polynomials in powers of (s - a),
    (t - c).  The exact solution with polynomial data (Proposition
    "propinterp"),

      k(s,t) = g_0 0F1(1; C(s-a)(t-c))
               + sum_{n=1}^{N} (g_n (s-a)^n + h_n (t-c)^n) 0F1(n+1; C(s-a)(t-c)),

    is evaluated on the top edge t = d at the Chebyshev extrema of [a, b] and
    on the right edge s = b at those of [c, d]; each set of values is then
    interpolated by the unique polynomial of degree <= N (Definition
    "interpooperator"), returned as coefficients in powers of (s - a) and
    (t - c).
    """
    sn = chebyshev_extrema(N, a, b)
    tn = chebyshev_extrema(N, c, d)

    def k_at(s_, t_):
        z = C * (s_ - a) * (t_ - c)
        val = g[0] * hyp0f1(1.0, z)
        for n in range(1, N + 1):
            val = val + (g[n] * (s_ - a) ** n + h[n] * (t_ - c) ** n) * hyp0f1(n + 1.0, z)
        return val

    top_vals = k_at(sn, d)
    right_vals = k_at(b, tn)
    Vs = np.vander(sn - a, N + 1, increasing=True)
    Vt = np.vander(tn - c, N + 1, increasing=True)
    g_new = np.linalg.solve(Vs, top_vals)
    h_new = np.linalg.solve(Vt, right_vals)
    return g_new, h_new


def interp_scheme(x, y, N: int, s=None, t=None, track_exponent: bool = False):
    """Order-N polynomial interpolation scheme (Definition "Polynomial
    interpolation numerical scheme").

    Edges start as the constant 1.  On every rectangle the interpolants of the
    bottom and left edges are mapped by Phi^N to the top and right edges and
    re-interpolated at the Chebyshev extrema; coefficients are stored in the
    monomial basis.  The endpoint averages the top edge of the last cell at
    s_{l_x} and its right edge at t_{l_y}.
    """
    if N < 2:
        raise ValueError("the scheme is defined for N >= 2")
    dx, dy = increments(x), increments(y)
    lx, ly = len(dx), len(dy)
    if lx == 0 or ly == 0:
        return (1.0, 0) if track_exponent else 1.0
    s = _partition(lx + 1, s)
    t = _partition(ly + 1, t)
    C = (dx @ dy.T) / np.outer(np.diff(s), np.diff(t))
    e0 = np.zeros(N + 1, dtype=C.dtype)
    e0[0] = 1.0
    E = 0
    g = [e0.copy() for _ in range(lx)]
    h = e0.copy()
    for j in range(ly):
        h = e0 * 2.0 ** (-E)
        for i in range(lx):
            g[i], h = interp_cell(g[i], h, C[i, j], s[i], s[i + 1], t[j], t[j + 1], N)
        if track_exponent:
            E = _rescale(g + [h], E)
    ds, dt = s[lx] - s[lx - 1], t[ly] - t[ly - 1]
    top = sum(g[lx - 1][n] * ds ** n for n in range(N + 1))
    right = sum(h[n] * dt ** n for n in range(N + 1))
    m = 0.5 * (top + right)
    return (m, E) if track_exponent else m * 2.0 ** E


def refine_points(x, lam: int) -> np.ndarray:
    """Points of the piecewise-linear path x with every segment split into
    2**lam equal pieces (the dyadic refinement of Definition "Dyadic finite
    differences approximation scheme" applied to the path itself)."""
    x = np.asarray(x)
    r = 2 ** lam
    if len(x) < 2 or r == 1:
        return x.copy()
    frac = np.arange(r) / r
    pts = x[:-1, None, :] + frac[None, :, None] * (x[1:] - x[:-1])[:, None, :]
    return np.concatenate([pts.reshape(-1, x.shape[1]), x[-1:]], 0)


def hybrid_scheme(x, y, N: int, lam: int, scheme: str = "approx", track_exponent: bool = False):
    """Hybrid of the finite-difference refinement and a polynomial scheme
    (remark after Theorem "prop:globalte"): the approximation or
    interpolation scheme of order N on the lambda-refined grid."""
    fn = approx_scheme if scheme == "approx" else interp_scheme
    return fn(refine_points(x, lam), refine_points(y, lam), N, track_exponent=track_exponent)


# ---------------------------------------------------------------------------
# Truncated signatures (ground truth of Section 4)
# ---------------------------------------------------------------------------

def _tensor_exp(v: np.ndarray, level: int):
    """exp of a vector in the truncated tensor algebra: levels v^{(x)k} / k!."""
    out = [np.ones(())]
    cur = np.ones(())
    for k in range(1, level + 1):
        cur = np.multiply.outer(cur, v) / k
        out.append(cur)
    return out


def _chen(a, b, level: int):
    """Truncated tensor product (a (x) b)_k = sum_{i+j=k} a_i (x) b_j."""
    out = []
    for k in range(level + 1):
        acc = np.zeros(a[k].shape)
        for i in range(k + 1):
            acc = acc + np.multiply.outer(a[i], b[k - i])
        out.append(acc)
    return out


def truncated_signature(x, level: int):
    """Signature of a piecewise-linear path truncated at ``level``: the
    product, in path order, of the tensor exponentials of its increments (the
    solution of dS = S (x) dx on each linear piece)."""
    dx = increments(x)
    d = dx.shape[1]
    sig = [np.ones(())] + [np.zeros((d,) * k) for k in range(1, level + 1)]
    for inc in dx:
        sig = _chen(sig, _tensor_exp(inc, level), level)
    return sig


def truncated_signature_kernel(x, y, level: int) -> float:
    """<S^{<=level}(x), S^{<=level}(y)> with the Hilbert-Schmidt inner product
    on each tensor level (Section 1)."""
    sx = truncated_signature(x, level)
    sy = truncated_signature(y, level)
    return float(sum(np.sum(a * b) for a, b in zip(sx, sy)))


# ---------------------------------------------------------------------------
# Batch helpers
# ---------------------------------------------------------------------------

def gram(X, Y, fn, **kw) -> np.ndarray:
    """K[a, b] = fn(X[a], Y[b], **kw)."""
    return np.array([[fn(xa, yb, **kw) for yb in Y] for xa in X], dtype=np.float64)


def mmd2_unbiased(Kxx: np.ndarray, Kyy: np.ndarray, Kxy: np.ndarray) -> float:
    """Unbiased (U-statistic) estimate of the squared maximum mean discrepancy
    from the three Gram matrices: the within-sample diagonals are excluded."""
    n, m = Kxx.shape[0], Kyy.shape[0]
    sxx = (Kxx.sum() - np.trace(Kxx)) / (n * (n - 1))
    syy = (Kyy.sum() - np.trace(Kyy)) / (m * (m - 1))
    sxy = Kxy.mean()
    return float(sxx + syy - 2.0 * sxy)


def mmd_permutation_stats(Kzz: np.ndarray, m: int, perms: np.ndarray) -> np.ndarray:
    """Unbiased MMD^2 of every relabelling of a pooled sample (the permutation
    two-sample test the paper's library offers with its MMD tools; the test
    itself is the standard one, the paper gives no formula).

    Kzz: (m+n) x (m+n) Gram matrix of the pooled paths; perms: rows that are
    permutations of 0..m+n-1, whose first m entries form the first sample.
    Returns one statistic per row."""
    out = np.empty(len(perms))
    for p, pi in enumerate(np.asarray(perms)):
        a, b = pi[:m], pi[m:]
        out[p] = mmd2_unbiased(Kzz[np.ix_(a, a)], Kzz[np.ix_(b, b)], Kzz[np.ix_(a, b)])
    return out


def mmd_permutation_pvalue(stats: np.ndarray) -> float:
    """p-value of the statistic stats[0] (the observed split) against the
    permutation statistics stats[1:]: (1 + #{stats[1:] >= stats[0]}) / len(stats)."""
    stats = np.asarray(stats)
    return float((1 + np.count_nonzero(stats[1:] >= stats[0])) / len(stats))
