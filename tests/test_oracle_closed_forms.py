"""Pins of the FP64 oracle against closed forms that follow from the paper and
from classical special functions (no GPU).

Each test names the passage of the paper it relies on.  The closed forms are
computed here independently of the oracle's arithmetic (scipy special
functions, hand-derived sums), so a dropped term, wrong index or sign in the
oracle's cell maps fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import c_oracle as C
from oracle import schemes as S


def hyp0f1_one(z):
    """0F1(1; z) from the modified Bessel function I_0 (remark after
    Proposition "propinterp"), or J_0 for negative z."""
    if z >= 0:
        return float(sp.iv(0, 2.0 * math.sqrt(z)))
    return float(sp.jv(0, 2.0 * math.sqrt(-z)))


def one_cell(c, d=2):
    x = np.zeros((2, d))
    y = np.zeros((2, d))
    x[1, 0] = 1.0
    y[1, 0] = c
    return x, y


CS = [-3.0, -0.4, 0.0, 0.013, 0.7, 2.5]


@pytest.mark.parametrize("c", CS)
@pytest.mark.parametrize("N", [2, 3, 4, 6, 9])
def test_one_cell_approximation_is_truncated_bessel_series(c, N):
    # Proof of Proposition "multistepestimate": p^{01}_n = C^n t_1^n / (n!)^2, so
    # the averaged endpoint of a single cell is sum_{n<=N} c^n/(n!)^2.
    want = sum(c ** n / math.factorial(n) ** 2 for n in range(N + 1))
    x, y = one_cell(c)
    assert S.approx_scheme(x, y, N) == pytest.approx(want, rel=1e-15, abs=1e-15)
    m, e = C.gram(x[None], y[None], C.APPROX, N)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-15, abs=1e-15)


@pytest.mark.parametrize("c", CS)
@pytest.mark.parametrize("N", [2, 4, 7])
def test_one_cell_interpolation_is_bessel(c, N):
    # Proposition "propinterp" with constant unit boundary data: k = 0F1(1; C s t)
    # = I_0(2 sqrt(C s t)); the corner u = 1 is an interpolation node, so the
    # endpoint is exact for every N.
    x, y = one_cell(c)
    want = hyp0f1_one(c)
    assert S.interp_scheme(x, y, N) == pytest.approx(want, rel=1e-14)
    m, e = C.gram(x[None], y[None], C.INTERP, N)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("c", CS)
def test_one_cell_finite_difference(c):
    # Definition "Dyadic finite differences approximation scheme", lambda = 0:
    # k(1,1) = 1 + 1 - 1 + c/2 (1 + 1) = 1 + c.
    x, y = one_cell(c)
    assert S.fd_scheme(x, y, 0) == pytest.approx(1.0 + c, rel=1e-15, abs=1e-15)
    m, e = C.gram(x[None], y[None], C.FD, 0)
    assert C.value(m, e)[0, 0] == pytest.approx(1.0 + c, rel=1e-15, abs=1e-15)


@pytest.mark.parametrize("c", CS)
def test_one_cell_second_order_finite_difference(c):
    # Remark "higherfd", eq. secondexplicitscheme, lambda = 0: the c^2 term adds
    # c^2/12 (1 + 1 + 1), so k(1,1) = 1 + c + c^2/4.
    x, y = one_cell(c)
    want = 1.0 + c + c * c / 4.0
    assert S.fd2_scheme(x, y, 0) == pytest.approx(want, rel=1e-15, abs=1e-15)
    m, e = C.gram(x[None], y[None], C.FD2, 0)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-15, abs=1e-15)


def first_row_closed_form(cs, N):
    """One x-segment against a y-polyline whose cells have constants cs.

    Along the column the left edges stay (1, 0, ...), so the Hankel term of the
    top map vanishes and the bottom edge of cell j is p_n = S_j^n/(n!)^2 with
    S_j the sum of the previous constants.  The right edge of the last cell is
    q~_n = c^n/n! * sum_{k=0}^{N} S'^k / (k! (n+k)!) (the k = 0 term from the
    left edge, k >= 1 from the Hankel term), S' the sum of all but the last
    constant.  Endpoint: the average of top(1) and right(1)."""
    S_all = float(np.sum(cs))
    S_prev = float(np.sum(cs[:-1]))
    c = float(cs[-1])
    f = math.factorial
    top = sum(S_all ** n / f(n) ** 2 for n in range(N + 1))
    right = sum(c ** n / f(n) * sum(S_prev ** k / (f(k) * f(n + k)) for k in range(N + 1))
                for n in range(N + 1))
    return 0.5 * (top + right)


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_first_column_closed_form_pins_hankel_term(N):
    # Definition "Polynomial approximation numerical scheme" on a 1 x l grid:
    # exercises the Toeplitz recursion and, in the last cell, the Hankel sum
    # with a non-trivial bottom edge at finite N.
    rng = np.random.default_rng(N)
    dx = rng.normal(size=3)
    y = np.concatenate([np.zeros((1, 3)), np.cumsum(rng.normal(size=(5, 3)) * 0.4, axis=0)])
    x = np.stack([np.zeros(3), dx])
    cs = (np.diff(y, axis=0) @ dx)
    want = first_row_closed_form(cs, N)
    assert S.approx_scheme(x, y, N) == pytest.approx(want, rel=1e-14)
    m, e = C.gram(x[None], y[None], C.APPROX, N)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-14)


def collinear(rng, lx, ly, scale=0.5):
    """x = f(t) v, y = g(t) w with piecewise-linear f, g: the signature of a
    1-d path is the tensor exponential of its increment, so the kernel is
    0F1(1; (f_end - f_0)(g_end - g_0) <v, w>)."""
    d = 3
    v, w = rng.normal(size=d), rng.normal(size=d)
    f = np.concatenate([[0.0], np.cumsum(rng.normal(size=lx) * scale)])
    g = np.concatenate([[0.0], np.cumsum(rng.normal(size=ly) * scale)])
    x = f[:, None] * v[None]
    y = g[:, None] * w[None]
    z = (f[-1] - f[0]) * (g[-1] - g[0]) * float(v @ w)
    return x, y, z


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_collinear_paths_converge_to_exact_kernel(seed):
    rng = np.random.default_rng(seed)
    x, y, z = collinear(rng, 5, 4)
    want = hyp0f1_one(z)
    assert S.approx_scheme(x, y, 24) == pytest.approx(want, rel=1e-13)
    assert S.interp_scheme(x, y, 14) == pytest.approx(want, rel=1e-12)
    m, e = C.gram(x[None], y[None], C.APPROX, 24)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-13)
    m, e = C.gram(x[None], y[None], C.INTERP, 14)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-12)


def test_segment_against_polyline_exact_kernel():
    # <v^{(x)n}/n!, S^n(y)> = <v, y_end - y_0>^n/(n!)^2 for a straight x.
    rng = np.random.default_rng(7)
    x = np.stack([np.zeros(3), rng.normal(size=3)])
    y = np.concatenate([np.zeros((1, 3)), np.cumsum(rng.normal(size=(6, 3)) * 0.5, axis=0)])
    want = hyp0f1_one(float((x[1] - x[0]) @ (y[-1] - y[0])))
    assert S.approx_scheme(x, y, 24) == pytest.approx(want, rel=1e-13)
    assert S.approx_scheme(y, x, 24) == pytest.approx(want, rel=1e-13)
    assert S.interp_scheme(x, y, 14) == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("d,lx,ly", [(2, 3, 4), (3, 2, 3), (2, 5, 2)])
def test_schemes_match_bruteforce_truncated_signatures(d, lx, ly):
    # Section 4 uses the truncated signature kernel as ground truth; here it is
    # computed by Chen products of tensor exponentials (Section 1) and compared
    # with the converged schemes.
    rng = np.random.default_rng(100 + d * 10 + lx)
    x = np.concatenate([np.zeros((1, d)), np.cumsum(rng.normal(size=(lx, d)) * 0.4, axis=0)])
    y = np.concatenate([np.zeros((1, d)), np.cumsum(rng.normal(size=(ly, d)) * 0.4, axis=0)])
    want = S.truncated_signature_kernel(x, y, 14)
    assert S.approx_scheme(x, y, 20) == pytest.approx(want, rel=1e-13)
    assert S.interp_scheme(x, y, 12) == pytest.approx(want, rel=1e-12)
    m, e = C.gram(x[None], y[None], C.APPROX, 20)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-13)
    m, e = C.gram(x[None], y[None], C.INTERP, 12)
    assert C.value(m, e)[0, 0] == pytest.approx(want, rel=1e-12)
