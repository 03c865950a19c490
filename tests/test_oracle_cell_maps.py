"""Pins of the oracle's one-cell maps against the PDE they solve (no GPU).

* The interpolation formula (Proposition "propinterp") is checked against the
  Goursat problem itself: boundary data on the bottom/left edges and the
  residual of d^2k/dsdt = C k at interior points.
* The truncated map of the approximation scheme (remark after Definition
  "Polynomial approximation numerical scheme") must return the first N + 1
  Taylor coefficients of the exact top/right edges; those coefficients are
  extracted here from the interpolation formula by a discrete Cauchy integral
  (FFT on a circle), an independent route.
* The interpolation nodes are the Chebyshev points of the second kind
  (extrema), compared with numpy's own generator.
"""
import math

import numpy as np
import pytest

from oracle import schemes as S


def phi_formula(g, h, C, s, t):
    """k(s, t) on [0,1]^2 from eq. (interpformula) with polynomial data g, h."""
    z = C * s * t
    val = g[0] * S.hyp0f1(1.0, z)
    for n in range(1, len(g)):
        val = val + (g[n] * s ** n + h[n] * t ** n) * S.hyp0f1(n + 1.0, z)
    return val


def random_data(rng, N):
    g = rng.normal(size=N + 1) / np.array([math.factorial(n) for n in range(N + 1)])
    h = rng.normal(size=N + 1) / np.array([math.factorial(n) for n in range(N + 1)])
    h[0] = g[0]
    return g, h


@pytest.mark.parametrize("C", [-1.7, 0.3, 2.2])
def test_interp_formula_solves_goursat_problem(C):
    rng = np.random.default_rng(3)
    g, h = random_data(rng, 5)
    u = np.linspace(0, 1, 7)
    # boundary data
    np.testing.assert_allclose(phi_formula(g, h, C, u, 0.0), np.polyval(g[::-1], u), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(phi_formula(g, h, C, 0.0, u), np.polyval(h[::-1], u), rtol=1e-14, atol=1e-14)
    # PDE residual by a 4-point central mixed difference
    eps = 1e-4
    for s in (0.2, 0.55, 0.9):
        for t in (0.15, 0.5, 0.8):
            mixed = (phi_formula(g, h, C, s + eps, t + eps) - phi_formula(g, h, C, s + eps, t - eps)
                     - phi_formula(g, h, C, s - eps, t + eps) + phi_formula(g, h, C, s - eps, t - eps)) / (4 * eps * eps)
            assert mixed == pytest.approx(C * phi_formula(g, h, C, s, t), rel=1e-6, abs=1e-7)


def taylor_coeffs(f, n_coeffs, radius=0.5, n_pts=128):
    th = 2 * np.pi * np.arange(n_pts) / n_pts
    vals = f(radius * np.exp(1j * th))
    c = np.fft.fft(vals) / n_pts
    return (c[:n_coeffs] / radius ** np.arange(n_coeffs)).real


@pytest.mark.parametrize("C", [-2.5, -0.2, 0.05, 1.3, 4.0])
@pytest.mark.parametrize("N", [2, 4, 7])
def test_truncated_map_equals_taylor_coefficients_of_exact_edges(C, N):
    rng = np.random.default_rng(11 + N)
    g, h = random_data(rng, N)
    pt, qt = S.approx_cell(g, h, C, 1.0, 1.0, N)
    top = taylor_coeffs(lambda u: phi_formula(g, h, C, u, 1.0), N + 1)
    right = taylor_coeffs(lambda v: phi_formula(g, h, C, 1.0, v), N + 1)
    np.testing.assert_allclose(pt, top, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(qt, right, rtol=1e-11, atol=1e-13)


def test_approx_cell_general_rectangle_matches_normalised_cell():
    # On [a,b]x[c,d] the map depends on C (b-a)(d-c) once coefficients are
    # expressed in the normalised variables (s-a)/(b-a), (t-c)/(d-c).
    rng = np.random.default_rng(5)
    N, C, ds, dt = 5, 0.8, 0.37, 1.9
    g, h = random_data(rng, N)
    sc_s = ds ** np.arange(N + 1)
    sc_t = dt ** np.arange(N + 1)
    pt, qt = S.approx_cell(g / sc_s, h / sc_t, C, ds, dt, N)
    pn, qn = S.approx_cell(g, h, C * ds * dt, 1.0, 1.0, N)
    np.testing.assert_allclose(pt * sc_s, pn, rtol=1e-13)
    np.testing.assert_allclose(qt * sc_t, qn, rtol=1e-13)


@pytest.mark.parametrize("N", [2, 5, 8])
def test_chebyshev_extrema_are_second_kind_points(N):
    want = np.sort(np.polynomial.chebyshev.chebpts2(N + 1))
    got = np.sort(S.chebyshev_extrema(N, -1.0, 1.0))
    np.testing.assert_allclose(got, want, atol=1e-15)
    got01 = S.chebyshev_extrema(N, 0.0, 1.0)
    assert got01[0] == pytest.approx(1.0) and got01[-1] == pytest.approx(0.0, abs=1e-16)


@pytest.mark.parametrize("C", [-1.0, 0.6])
def test_interp_cell_reproduces_formula_at_nodes(C):
    # Omega^N returns the interpolant of the exact edges: at the nodes it must
    # equal eq. (interpformula).
    rng = np.random.default_rng(9)
    N = 6
    g, h = random_data(rng, N)
    gn, hn = S.interp_cell(g, h, C, 0.0, 1.0, 0.0, 1.0, N)
    u = S.chebyshev_extrema(N, 0.0, 1.0)
    np.testing.assert_allclose(np.polyval(gn[::-1], u), phi_formula(g, h, C, u, 1.0), rtol=1e-12)
    np.testing.assert_allclose(np.polyval(hn[::-1], u), phi_formula(g, h, C, 1.0, u), rtol=1e-12)


def test_hyp0f1_matches_scipy():
    import scipy.special as sp
    for b in (1.0, 2.0, 5.0, 9.0):
        for z in (-6.0, -0.3, 0.0, 0.01, 2.0, 7.5):
            assert S.hyp0f1(b, z) == pytest.approx(float(sp.hyp0f1(b, z)), rel=1e-13, abs=1e-15)
