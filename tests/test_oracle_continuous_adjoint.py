"""Pins of the oracle's continuous-adjoint gradient (no GPU): the derivative
of the exact kernel with respect to the cell constants from Riemann's method,
evaluated inside every cell with the double series of Proposition "prop:a1"
(eq. appeq2).  Checked against a closed form, against central differences of
the converged kernel and against the complex-step derivative of the converged
scheme, which are independent of it."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import derivatives as D
from oracle import schemes as S


@pytest.mark.parametrize("c", [0.3, -0.7, 1.5, 4.0])
def test_one_cell_gradient_is_derivative_of_bessel(c):
    # one cell of constant c: k = I0(2 sqrt c) = sum c^n/(n!)^2, so
    # dk/dc = sum n c^(n-1)/(n!)^2 = I1(2 sqrt c)/sqrt c (J1 for c < 0)
    x = np.array([[0.0, 0.0], [1.0, 0.0]])
    y = np.array([[0.0, 0.0], [c, 0.0]])
    G, gx, gy = D.continuous_adjoint_grad(x, y, N=24, M=60)
    r = math.sqrt(abs(c))
    want = sp.iv(1, 2 * r) / r if c > 0 else sp.jv(1, 2 * r) / r
    assert G[0, 0] == pytest.approx(want, rel=1e-13)
    # chain rule: c = <dx, dy> = dx_0 dy_0, x = (0,0) -> (1,0)
    assert gx[1, 0] == pytest.approx(want * c, rel=1e-13)
    assert gx[0, 0] == pytest.approx(-want * c, rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_differences_of_the_converged_kernel(seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([np.zeros((1, 2)), np.cumsum(rng.normal(0, 0.4, (4, 2)), 0)])
    y = np.concatenate([np.zeros((1, 2)), np.cumsum(rng.normal(0, 0.4, (3, 2)), 0)])
    G, gx, gy = D.continuous_adjoint_grad(x, y)
    fx = lambda xx: S.approx_scheme(xx, y, 24)
    fy = lambda yy: S.approx_scheme(x, yy, 24)
    for t in range(len(x)):
        for k in range(2):
            assert gx[t, k] == pytest.approx(D.central_fd(fx, x, (t, k), 1e-5), abs=1e-9)
    for t in range(len(y)):
        for k in range(2):
            assert gy[t, k] == pytest.approx(D.central_fd(fy, y, (t, k), 1e-5), abs=1e-9)


def test_gradient_matches_complex_step_of_the_converged_scheme():
    # the discrete gradient of the scheme at N = 24 is the exact gradient to
    # rounding, reached by a route (complex step) that shares nothing with
    # the adjoint's interior integrals
    rng = np.random.default_rng(2)
    x = np.concatenate([np.zeros((1, 3)), np.cumsum(rng.normal(0, 0.3, (5, 3)), 0)])
    y = np.concatenate([np.zeros((1, 3)), np.cumsum(rng.normal(0, 0.3, (4, 3)), 0)])
    G, gx, gy = D.continuous_adjoint_grad(x, y)
    cs = D.complex_step_grad(lambda a, b: S.approx_scheme(a, b, 24), x, y)
    np.testing.assert_allclose(gx, cs, rtol=0, atol=1e-14 * np.abs(cs).max())
    csy = D.complex_step_grad(lambda a, b: S.approx_scheme(a, b, 24), x, y, wrt="y")
    np.testing.assert_allclose(gy, csy, rtol=0, atol=1e-14 * np.abs(csy).max())


def test_reversal_symmetry():
    # reversing both paths maps cell (i, j) to (lx-1-i, ly-1-j) with the same
    # constant and leaves the kernel unchanged, so dk/dc is reversed too
    rng = np.random.default_rng(3)
    x = np.concatenate([np.zeros((1, 2)), np.cumsum(rng.normal(0, 0.5, (3, 2)), 0)])
    y = np.concatenate([np.zeros((1, 2)), np.cumsum(rng.normal(0, 0.5, (4, 2)), 0)])
    G, _, _ = D.continuous_adjoint_grad(x, y)
    Gr, _, _ = D.continuous_adjoint_grad(x[::-1], y[::-1])
    np.testing.assert_allclose(Gr, G[::-1, ::-1], rtol=1e-13, atol=0)
