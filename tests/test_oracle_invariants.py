"""Invariants, convergence and cross-checks of the oracle (no GPU)."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import c_oracle as C
from oracle import derivatives as D
from oracle import schemes as S


def bm(rng, n_steps, d, std=0.4):
    return np.concatenate([np.zeros((1, d)), np.cumsum(rng.normal(size=(n_steps, d)) * std, axis=0)])


@pytest.mark.parametrize("scheme", ["approx", "interp", "fd"])
def test_symmetry(scheme):
    # The kernel is symmetric; each scheme's map is symmetric under exchanging
    # the roles of the two paths (Remark "symmetry1" for the exact solution).
    rng = np.random.default_rng(1)
    x, y = bm(rng, 5, 3), bm(rng, 4, 3)
    f = {"approx": lambda a, b: S.approx_scheme(a, b, 5),
         "interp": lambda a, b: S.interp_scheme(a, b, 5),
         "fd": lambda a, b: S.fd_scheme(a, b, 1)}[scheme]
    assert f(x, y) == pytest.approx(f(y, x), rel=1e-13)


def test_translation_and_scaling():
    # Only increments enter; scaling one path scales every cell constant.
    rng = np.random.default_rng(2)
    x, y = bm(rng, 6, 2), bm(rng, 5, 2)
    base = S.approx_scheme(x, y, 6)
    assert S.approx_scheme(x + 3.7, y - 1.1, 6) == pytest.approx(base, rel=1e-13)
    lam = 1.7
    assert S.approx_scheme(lam * x, y, 6) == pytest.approx(S.approx_scheme(x, lam * y, 6), rel=1e-13)


def test_partition_invariance():
    # With C_ij = <dx, dy>/(ds dt) and coefficients in powers of (s - s_i),
    # the time partition drops out of both polynomial schemes.
    rng = np.random.default_rng(3)
    x, y = bm(rng, 5, 3), bm(rng, 4, 3)
    s = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 2.0, 5))])
    t = np.concatenate([[0.0], np.cumsum(rng.uniform(0.1, 2.0, 4))])
    assert S.approx_scheme(x, y, 6, s, t) == pytest.approx(S.approx_scheme(x, y, 6), rel=1e-13)
    assert S.interp_scheme(x, y, 6, s, t) == pytest.approx(S.interp_scheme(x, y, 6), rel=1e-12)


def test_zero_paths_and_empty():
    x = np.zeros((5, 2))
    y = np.random.default_rng(0).normal(size=(4, 2))
    assert S.approx_scheme(x, y, 4) == pytest.approx(1.0)
    assert S.approx_scheme(x[:1], y, 4) == 1.0
    m, e = C.gram(x[None, :1], y[None], C.APPROX, 4)
    assert C.value(m, e)[0, 0] == 1.0


def test_gram_is_symmetric_positive_semidefinite():
    rng = np.random.default_rng(4)
    X = np.stack([bm(rng, 6, 2, 0.3) for _ in range(7)])
    m, e = C.gram(X, X, C.APPROX, 16)
    K = C.value(m, e)
    np.testing.assert_allclose(K, K.T, rtol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.min() >= -1e-10 * ev.max()


def test_fd_converges_at_second_order_rate():
    # The dyadic scheme's error decreases like 2^{-2 lambda} (Section 2).
    rng = np.random.default_rng(5)
    x, y = bm(rng, 3, 2, 0.5), bm(rng, 3, 2, 0.5)
    exact = S.approx_scheme(x, y, 24)
    errs = [abs(C.value(*C.gram(x[None], y[None], C.FD, lam))[0, 0] - exact) for lam in range(2, 7)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.35), ratios


def test_second_order_fd_is_more_accurate_and_converges():
    # Remark "higherfd": the extra c^2 term of the quadrature shrinks the
    # error constant, and on the dyadic refinement the error still falls at
    # least like 4^-lambda (two refinement levels cut it by 8 or more; the
    # ratio of single levels approaches 4 but can jump where the error's
    # leading terms cancel).
    for seed in (0, 5):
        rng = np.random.default_rng(seed)
        x, y = bm(rng, 3, 2, 0.5), bm(rng, 3, 2, 0.5)
        exact = S.approx_scheme(x, y, 24)
        e1 = [abs(C.value(*C.gram(x[None], y[None], C.FD, lam))[0, 0] - exact) for lam in range(7)]
        e2 = [abs(C.value(*C.gram(x[None], y[None], C.FD2, lam))[0, 0] - exact) for lam in range(7)]
        assert all(b < a / 3 for a, b in zip(e1, e2)), (e1, e2)
        assert all(e2[lam + 2] <= e2[lam] / 8 for lam in range(2, 5)), e2


def test_second_order_fd_symmetric_and_c_matches_numpy():
    rng = np.random.default_rng(7)
    x, y = bm(rng, 4, 3, 0.5), bm(rng, 6, 3, 0.5)
    for lam in (0, 1, 2):
        a = S.fd2_scheme(x, y, lam)
        assert S.fd2_scheme(y, x, lam) == pytest.approx(a, rel=1e-14)
        assert C.value(*C.gram(x[None], y[None], C.FD2, lam))[0, 0] == pytest.approx(a, rel=1e-13)


def test_approx_error_decreases_with_order():
    rng = np.random.default_rng(6)
    x, y = bm(rng, 8, 2, 0.4), bm(rng, 8, 2, 0.4)
    exact = S.truncated_signature_kernel(x[:5], y[:5], 14)
    errs = [abs(S.approx_scheme(x[:5], y[:5], N) - exact) for N in (2, 4, 6, 8)]
    assert errs[0] > errs[1] > errs[2] > errs[3]
    errs_i = [abs(S.interp_scheme(x[:5], y[:5], N) - exact) for N in (2, 4, 6)]
    assert errs_i[0] > errs_i[1] > errs_i[2]


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_c_oracle_matches_numpy_oracle(N):
    rng = np.random.default_rng(10 + N)
    X = np.stack([bm(rng, 7, 3, 0.5) for _ in range(3)])
    Y = np.stack([bm(rng, 5, 3, 0.5) for _ in range(2)])
    for sch, fn in ((C.APPROX, S.approx_scheme), (C.INTERP, S.interp_scheme)):
        m, e = C.gram(X, Y, sch, N)
        got = C.value(m, e)
        want = S.gram(X, Y, fn, N=N)
        np.testing.assert_allclose(got, want, rtol=1e-12)
    m, e = C.gram(X, Y, C.FD, 2)
    np.testing.assert_allclose(C.value(m, e), S.gram(X, Y, S.fd_scheme, lam=2), rtol=1e-13)


def test_pairs_interface_matches_gram():
    rng = np.random.default_rng(12)
    xs = [bm(rng, n, 2, 0.5) for n in (3, 9, 1, 6)]
    ys = [bm(rng, n, 2, 0.5) for n in (4, 2, 5, 0)]
    m, e = C.pairs(xs, ys, C.APPROX, 5)
    want = [S.approx_scheme(a, b, 5) for a, b in zip(xs, ys)]
    np.testing.assert_allclose(C.value(m, e), want, rtol=1e-13)


def test_exponent_tracking_beyond_fp64_range():
    # Collinear paths with a huge total inner product z: k = I_0(2 sqrt z),
    # log k = log(ive(0, 2 sqrt z)) + 2 sqrt z, far beyond 1e308.
    rng = np.random.default_rng(13)
    n = 1200
    f = np.concatenate([[0.0], np.cumsum(np.abs(rng.normal(size=n)) * 0.6)])
    v = np.array([1.0, 0.5])
    x = f[:, None] * v[None]
    z = float((f[-1] - f[0]) ** 2 * (v @ v))
    m, e = C.gram(x[None], x[None], C.APPROX, 24)
    got_log = math.log(abs(m[0, 0])) + e[0, 0] * math.log(2.0)
    want_log = math.log(sp.ive(0, 2 * math.sqrt(z))) + 2 * math.sqrt(z)
    assert want_log > 800  # beyond FP64
    assert got_log == pytest.approx(want_log, rel=1e-12)
    # numpy oracle with tracking agrees on a smaller case
    xs = x[:40]
    mn, en = S.approx_scheme(xs, xs, 12, track_exponent=True)
    mc, ec = C.gram(xs[None], xs[None], C.APPROX, 12)
    assert math.ldexp(mn, en - int(ec[0, 0])) == pytest.approx(mc[0, 0], rel=1e-12)


def test_single_cell_gradient_closed_form():
    # d/dc sum_{n<=N} c^n/(n!)^2 = sum n c^{n-1}/(n!)^2; with x = (0, e1),
    # y = (0, c e1), dk/dy[1, 0] = dk/dc.
    for c in (-0.8, 0.3, 1.9):
        x = np.array([[0.0, 0.0], [1.0, 0.0]])
        y = np.array([[0.0, 0.0], [c, 0.0]])
        N = 6
        g = D.complex_step_grad(S.approx_scheme, x, y, wrt="y", N=N)
        want = sum(n * c ** (n - 1) / math.factorial(n) ** 2 for n in range(1, N + 1))
        assert g[1, 0] == pytest.approx(want, rel=1e-14)
        assert g[0, 0] == pytest.approx(-want, rel=1e-14)


@pytest.mark.parametrize("fn", [S.approx_scheme, S.interp_scheme])
def test_complex_step_gradient_matches_central_differences(fn):
    rng = np.random.default_rng(14)
    x, y = bm(rng, 4, 2, 0.5), bm(rng, 3, 2, 0.5)
    g = D.complex_step_grad(fn, x, y, wrt="x", N=5)
    for idx in [(0, 0), (1, 1), (2, 0), (4, 1)]:
        fd = D.central_fd(lambda v: fn(v, y, 5), x, idx, 1e-5)
        assert g[idx] == pytest.approx(fd, rel=1e-7, abs=1e-9)
    # translation invariance: the gradient sums to zero over points
    np.testing.assert_allclose(g.sum(axis=0), 0.0, atol=1e-13)


def test_mmd_unbiased_linear_kernel():
    # With the linear kernel k(a, b) = <a, b> the U-statistic expands to
    # sum_{i != j} <x_i, x_j>/(n(n-1)) + same for y - 2 <mean x, mean y>.
    rng = np.random.default_rng(15)
    X, Y = rng.normal(size=(6, 3)), rng.normal(size=(5, 3)) + 0.5
    Kxx, Kyy, Kxy = X @ X.T, Y @ Y.T, X @ Y.T
    sx = X.sum(0)
    sy = Y.sum(0)
    want = ((sx @ sx - (X * X).sum()) / 30 + (sy @ sy - (Y * Y).sum()) / 20
            - 2 * (X.mean(0) @ Y.mean(0)))
    assert S.mmd2_unbiased(Kxx, Kyy, Kxy) == pytest.approx(want, rel=1e-13)


def test_mmd_permutation_statistics_pins():
    # The unbiased MMD^2 of a relabelled pooled sample, checked against an
    # explicit double loop over its definition, and its invariances: any
    # reordering inside the two groups leaves it unchanged, and with equal
    # sizes exchanging the groups does too.
    rng = np.random.default_rng(21)
    m, n = 4, 5
    A = rng.normal(size=(m + n, 3))
    K = np.exp(-((A[:, None, :] - A[None, :, :]) ** 2).sum(-1))  # any symmetric Gram
    perms = np.stack([rng.permutation(m + n) for _ in range(6)] + [np.arange(m + n)])
    got = S.mmd_permutation_stats(K, m, perms)
    for p, pi in enumerate(perms):
        X, Y = pi[:m], pi[m:]
        sxx = sum(K[a, b] for a in X for b in X if a != b) / (m * (m - 1))
        syy = sum(K[a, b] for a in Y for b in Y if a != b) / (n * (n - 1))
        sxy = sum(K[a, b] for a in X for b in Y) / (m * n)
        assert got[p] == pytest.approx(sxx + syy - 2 * sxy, rel=1e-13, abs=1e-15)
    pi = perms[0]
    shuffled = np.concatenate([rng.permutation(pi[:m]), rng.permutation(pi[m:])])
    assert S.mmd_permutation_stats(K, m, shuffled[None])[0] == pytest.approx(got[0], rel=1e-13)
    K2 = K[:8, :8]
    pi = rng.permutation(8)
    swapped = np.concatenate([pi[4:], pi[:4]])
    a, b = S.mmd_permutation_stats(K2, 4, np.stack([pi, swapped]))
    assert a == pytest.approx(b, rel=1e-13)
    assert S.mmd_permutation_pvalue([0.5, 0.1, 0.7, 0.5, 0.2]) == pytest.approx(3 / 5)


def test_hybrid_refined_grid_scheme_pins():
    # Hybrid method (remark after Theorem "prop:globalte"): a polynomial scheme
    # on the dyadically refined grid.  The exact kernel does not change when
    # collinear points are inserted, so refinement must leave the converged
    # kernel unchanged; the hybrid converges to it as lambda grows (by more
    # than 3x per level here, the interpolation scheme faster); lambda = 0
    # is the plain scheme; the C oracle on refined points matches numpy.
    rng = np.random.default_rng(3)
    x, y = bm(rng, 4, 2, 0.5), bm(rng, 5, 2, 0.5)
    exact = S.approx_scheme(x, y, 24)
    assert S.approx_scheme(S.refine_points(x, 2), S.refine_points(y, 2), 24) == pytest.approx(exact, rel=1e-13)
    assert S.hybrid_scheme(x, y, 3, 0) == S.approx_scheme(x, y, 3)
    for sch in ("approx", "interp"):
        errs = [abs(S.hybrid_scheme(x, y, 2, lam, sch) - exact) for lam in range(4)]
        assert all(errs[i + 1] < errs[i] / 3 for i in range(3)), (sch, errs)
    r = S.refine_points(x, 2)
    assert len(r) == 4 * (len(x) - 1) + 1
    np.testing.assert_allclose(r[::4], x, rtol=0, atol=1e-15)
    kind = {"approx": C.APPROX, "interp": C.INTERP}
    for sch in ("approx", "interp"):
        m, e = C.gram(x[None], y[None], kind[sch], 4, lam=2)
        assert C.value(m, e)[0, 0] == pytest.approx(S.hybrid_scheme(x, y, 4, 2, sch), rel=1e-12)


def test_f32_model_is_the_scheme_to_fp32_resolution():
    """The FP32 model (a conditioning diagnostic) is the approximation scheme
    evaluated with FP32-rounded increments, constants and edge coefficients
    of degree >= 2: on a well-conditioned pair it departs from the FP64
    scheme by about the FP32 resolution -- not at all would mean nothing is
    rounded, much more would mean a different scheme."""
    from oracle import c_oracle as C
    rng = np.random.default_rng(12)
    X = np.concatenate([np.zeros((2, 1, 3)), np.cumsum(rng.normal(0, 0.15, (2, 60, 3)), 1)], 1)
    Y = np.concatenate([np.zeros((2, 1, 3)), np.cumsum(rng.normal(0, 0.15, (2, 45, 3)), 1)], 1)
    ref = np.ldexp(*C.gram(X, Y, C.APPROX, 6))
    f32 = np.ldexp(*C.gram(X, Y, C.APPROX_F32MODEL, 6))
    rel = np.abs(f32 / ref - 1)
    assert np.all(rel > 1e-12) and np.all(rel < 1e-5), rel
    # inputs whose increments, constants and state are exact in FP32 (one
    # cell, c = 1/4, N = 2: 1 + c + c^2/4 in dyadic rationals) give the FP64
    # value exactly
    x = np.array([[0.0], [0.5]])
    m0, e0 = C.gram(x[None], x[None], C.APPROX, 2)
    m1, e1 = C.gram(x[None], x[None], C.APPROX_F32MODEL, 2)
    assert np.ldexp(m0, e0)[0, 0] == np.ldexp(m1, e1)[0, 0] == 1 + 0.25 + 0.25 ** 2 / 4
