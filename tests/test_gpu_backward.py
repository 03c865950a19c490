"""GPU backward parity: the adjoint sweep against oracle gradients.

* Tiny FP64 inputs: complex-step derivatives of the numpy oracle (exact to
  rounding): 1e-10 relative in the max norm.
* Larger FP64 / FP32 inputs: central finite differences of the C oracle
  (h = 1e-4, FP64) on sampled coordinates; FP64 path within 1e-6 relative
  (the FD truncation error is O(h^2)), FP32 path within 1e-5 relative (the
  gradient target of the FP32 path).
"""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, oracle_gram

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("scheme,order", [("approx", 4), ("interp", 4), ("approx", 2)])
def test_tiny_gradient_matches_complex_step(sk, scheme, order):
    from oracle import derivatives as D
    from oracle import schemes as S
    log_banner(f"tiny gradient {scheme} {order}")
    rng = np.random.default_rng(3)
    X = bm_paths(rng, 2, 5, 2, 0.5)
    Y = bm_paths(rng, 3, 4, 2, 0.5)
    gK = rng.normal(size=(2, 3))
    fn = S.approx_scheme if scheme == "approx" else S.interp_scheme
    gXo = np.zeros_like(X)
    gYo = np.zeros_like(Y)
    for a in range(2):
        for b in range(3):
            gXo[a] += gK[a, b] * D.complex_step_grad(fn, X[a], Y[b], wrt="x", N=order)
            gYo[b] += gK[a, b] * D.complex_step_grad(fn, X[a], Y[b], wrt="y", N=order)
    gX, gY = sk.gram_backward(dev(X, torch.float64), dev(Y, torch.float64),
                              dev(gK, torch.float64), scheme, order)
    np.testing.assert_allclose(gX.cpu().numpy(), gXo, rtol=0, atol=1e-10 * np.abs(gXo).max())
    np.testing.assert_allclose(gY.cpu().numpy(), gYo, rtol=0, atol=1e-10 * np.abs(gYo).max())


def fd_gram_grad(X, Y, gK, scheme, order, idx, which, h=1e-4):
    """Central difference of sum(gK * K) in one coordinate of X or Y."""
    def loss(Xv, Yv):
        m, e = oracle_gram(Xv, Yv, scheme, order)
        return float(np.sum(gK * np.ldexp(m, e)))
    P = (X if which == "x" else Y).copy()
    P[idx] += h
    lp = loss(P, Y) if which == "x" else loss(X, P)
    P[idx] -= 2 * h
    lm = loss(P, Y) if which == "x" else loss(X, P)
    return (lp - lm) / (2 * h)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-5)])
@pytest.mark.parametrize("scheme,order", [("approx", 6), ("interp", 5)])
def test_multi_strip_gradient_matches_finite_differences(sk, dtype, tol, scheme, order):
    log_banner(f"multi-strip gradient {dtype} {scheme} {order}")
    rng = np.random.default_rng(21)
    X = bm_paths(rng, 2, 140, 3, 0.4 / np.sqrt(140))
    Y = bm_paths(rng, 2, 75, 3, 0.4 / np.sqrt(75))
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    gK = rng.normal(size=(2, 2))
    gX, gY = sk.gram_backward(dev(X, dtype), dev(Y, dtype), dev(gK, dtype), scheme, order)
    gX, gY = gX.cpu().double().numpy(), gY.cpu().double().numpy()
    picks = [("x", (0, 0, 0)), ("x", (1, 63, 1)), ("x", (0, 64, 2)), ("x", (1, 140, 0)),
             ("y", (0, 0, 1)), ("y", (1, 37, 2)), ("y", (0, 75, 0)), ("x", (1, 100, 1))]
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    for which, idx in picks:
        fd = fd_gram_grad(X, Y, gK, scheme, order, idx, which)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= tol * scale, (which, idx, got, fd)


def test_wide_dimension_gradient_matches_finite_differences(sk):
    # d = 37: the contraction runs three 16-dimension slices (the last of 5)
    log_banner("wide-dimension gradient")
    rng = np.random.default_rng(22)
    X = bm_paths(rng, 2, 100, 37, 0.2 / np.sqrt(100))
    Y = bm_paths(rng, 1, 80, 37, 0.2 / np.sqrt(80))
    gK = rng.normal(size=(2, 1))
    gX, gY = sk.gram_backward(dev(X, torch.float64), dev(Y, torch.float64),
                              dev(gK, torch.float64), "approx", 5)
    gX, gY = gX.cpu().numpy(), gY.cpu().numpy()
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    for which, idx in [("x", (0, 0, 0)), ("x", (1, 64, 15)), ("x", (0, 99, 16)), ("x", (1, 100, 36)),
                       ("y", (0, 0, 31)), ("y", (0, 40, 32)), ("y", (0, 80, 36))]:
        fd = fd_gram_grad(X, Y, gK, "approx", 5, idx, which)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= 1e-6 * scale, (which, idx, got, fd)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-5)])
def test_mfma_contraction_two_dimension_blocks(sk, dtype, tol):
    # d = 20: the MFMA contraction's two 16-dimension blocks (the second
    # partial), on ragged two-strip pairs whose columns end inside a tile
    log_banner(f"two-block MFMA contraction gradient {dtype}")
    rng = np.random.default_rng(23)
    X = bm_paths(rng, 2, 100, 20, 0.2 / np.sqrt(100))
    Y = bm_paths(rng, 2, 77, 20, 0.2 / np.sqrt(77))
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    gK = rng.normal(size=(2, 2))
    gX, gY = sk.gram_backward(dev(X, dtype), dev(Y, dtype), dev(gK, dtype), "approx", 5)
    gX, gY = gX.cpu().double().numpy(), gY.cpu().double().numpy()
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    for which, idx in [("x", (0, 0, 0)), ("x", (1, 63, 15)), ("x", (0, 64, 16)), ("x", (1, 100, 19)),
                       ("y", (0, 0, 3)), ("y", (1, 31, 17)), ("y", (0, 32, 16)), ("y", (1, 77, 19))]:
        fd = fd_gram_grad(X, Y, gK, "approx", 5, idx, which)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= tol * scale, (which, idx, got, fd)


def test_gradient_seed_exponent(sk):
    rng = np.random.default_rng(4)
    X = dev(bm_paths(rng, 2, 70, 3, 0.05), torch.float64)
    Y = dev(bm_paths(rng, 2, 80, 3, 0.05), torch.float64)
    gK = dev(rng.normal(size=(2, 2)), torch.float64)
    ge = torch.tensor([[3, -2], [0, 5]], dtype=torch.int32, device="cuda")
    gX1, gY1 = sk.gram_backward(X, Y, gK * torch.pow(2.0, ge.double()), "approx", 4)
    gX2, gY2 = sk.gram_backward(X, Y, gK, "approx", 4, gK_exp=ge)
    torch.testing.assert_close(gX1, gX2, rtol=1e-13, atol=0)
    torch.testing.assert_close(gY1, gY2, rtol=1e-13, atol=0)


def test_pairs_gradient_matches_finite_differences(sk):
    from oracle import c_oracle as C
    log_banner("pairs gradient")
    rng = np.random.default_rng(8)
    lens_x, lens_y = [70, 3, 130], [66, 90, 2]
    xs = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0] for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0] for n in lens_y]
    gk = rng.normal(size=3)
    gXc, gYc, xo, yo = sk.pairs_backward([dev(a, torch.float64) for a in xs],
                                         [dev(b, torch.float64) for b in ys],
                                         dev(gk, torch.float64), "approx", 5)
    gXc = gXc.cpu().numpy()
    for p, t, k in [(0, 0, 0), (0, 69, 2), (2, 64, 1), (1, 1, 0)]:
        def loss(v):
            xs2 = list(xs)
            xs2[p] = v
            m, e = C.pairs(xs2, ys, C.APPROX, 5)
            return float(np.sum(gk * np.ldexp(m, e)))
        h = 1e-4
        v = xs[p].copy()
        v[t, k] += h
        lp = loss(v)
        v[t, k] -= 2 * h
        lm = loss(v)
        fd = (lp - lm) / (2 * h)
        assert abs(gXc[xo[p] + t, k] - fd) <= 1e-6 * max(1.0, abs(fd)), (p, t, k)


def test_autograd_and_mmd_fp32(sk):
    log_banner("autograd mmd fp32")
    import workloads as W
    X, Y = W.mmd_sets(0, n=3, steps=256)
    Xt = dev(X, torch.float32).requires_grad_(True)
    Yt = dev(Y, torch.float32).requires_grad_(True)
    val = sk.mmd2(Xt, Yt, "approx", 8)
    val.backward()
    gX = Xt.grad.cpu().double().numpy()
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)

    def mmd(Xv, Yv):
        from oracle import schemes as S
        kxx = np.ldexp(*oracle_gram(Xv, Xv, "approx", 8))
        kyy = np.ldexp(*oracle_gram(Yv, Yv, "approx", 8))
        kxy = np.ldexp(*oracle_gram(Xv, Yv, "approx", 8))
        return S.mmd2_unbiased(kxx, kyy, kxy)
    assert float(val) == pytest.approx(mmd(Xd, Yd), rel=1e-4, abs=1e-6)
    scale = np.abs(gX).max()
    rng = np.random.default_rng(0)
    for _ in range(4):
        idx = (int(rng.integers(3)), int(rng.integers(257)), int(rng.integers(5)))
        h = 1e-4
        P = Xd.copy()
        P[idx] += h
        lp = mmd(P, Yd)
        P[idx] -= 2 * h
        lm = mmd(P, Yd)
        fd = (lp - lm) / (2 * h)
        assert abs(gX[idx] - fd) <= 1e-5 * scale, (idx, gX[idx], fd)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_saved_state_backward_matches_recompute(sk, dtype):
    log_banner(f"saved-state backward {dtype}")
    rng = np.random.default_rng(31)
    X = dev(bm_paths(rng, 3, 130, 4, 0.05), dtype)
    Y = dev(bm_paths(rng, 2, 70, 4, 0.05), dtype)
    gK = dev(rng.normal(size=(3, 2)), dtype)
    for scheme in ("approx", "interp"):
        K1, state = sk.gram_save(X, Y, scheme, 5)
        K0 = sk.gram(X, Y, scheme, 5)
        torch.testing.assert_close(K1, K0, rtol=1e-14 if dtype == torch.float64 else 1e-6, atol=0)
        gX1, gY1 = sk.gram_backward_saved(X, Y, gK, state, scheme, 5)
        gX0, gY0 = sk.gram_backward(X, Y, gK, scheme, 5)
        tol = 1e-12 if dtype == torch.float64 else 1e-6
        torch.testing.assert_close(gX1, gX0, rtol=tol, atol=tol * float(gX0.abs().max()))
        torch.testing.assert_close(gY1, gY0, rtol=tol, atol=tol * float(gY0.abs().max()))
    # batched autograd uses the saved path when the state fits; these six
    # pairs of 3-strip paths default to the strip pipeline, the same gradient
    gX0, gY0 = sk.gram_backward(X, Y, gK, "approx", 5)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    assert sk.api.gram_algo(X, Y) == "pipeline"
    for algo in ("batched", None):
        Xg = X.clone().requires_grad_(True)
        Yg = Y.clone().requires_grad_(True)
        (sk.sig_gram(Xg, Yg, "approx", 5, algo=algo) * gK).sum().backward()
        torch.testing.assert_close(Xg.grad, gX0, rtol=tol, atol=tol * float(gX0.abs().max()))
        torch.testing.assert_close(Yg.grad, gY0, rtol=tol, atol=tol * float(gY0.abs().max()))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_symmetric_gram_backward(sk, dtype, tol):
    # Y is X: one gradient holding both contributions, equal to gX + gY of
    # the general call; also through autograd and the saved-state path
    log_banner(f"symmetric backward {dtype}")
    rng = np.random.default_rng(41)
    X = dev(bm_paths(rng, 3, 90, 3, 0.05), dtype)
    gK = dev(rng.normal(size=(3, 3)), dtype)
    gX, gY = sk.gram_backward(X, X.clone(), gK, "approx", 5)
    ref = gX + gY
    gS, none = sk.gram_backward(X, X, gK, "approx", 5, symmetric=True)
    assert none is None
    scale = float(ref.abs().max())
    torch.testing.assert_close(gS, ref, rtol=tol, atol=tol * scale)
    for algo in ("batched", "pipeline"):
        Xg = X.clone().requires_grad_(True)
        (sk.sig_gram(Xg, Xg, "approx", 5, algo=algo) * gK).sum().backward()
        torch.testing.assert_close(Xg.grad, ref, rtol=tol, atol=tol * scale)


def test_bf16x3_backward_matches_native(sk):
    log_banner("bf16x3 backward")
    rng = np.random.default_rng(42)
    X = dev(bm_paths(rng, 2, 130, 16, 0.02), torch.float32)
    Y = dev(bm_paths(rng, 3, 70, 16, 0.02), torch.float32)
    gK = dev(rng.normal(size=(2, 3)), torch.float32)
    gX1, gY1 = sk.gram_backward(X, Y, gK, "approx", 6)
    gX3, gY3 = sk.gram_backward(X, Y, gK, "approx", 6, gram_mode="bf16x3")
    for a, b in ((gX1, gX3), (gY1, gY3)):
        torch.testing.assert_close(b, a, rtol=1e-4, atol=1e-4 * float(a.abs().max()))


@pytest.mark.parametrize("scheme,order,lam", [("approx", 4, 1), ("interp", 5, 1), ("approx", 3, 2)])
def test_hybrid_backward_matches_finite_differences(sk, scheme, order, lam):
    # the refined-grid (hybrid) scheme's gradient: sweeps on the lam-order
    # refinement (several refined strips), dL/dc folded onto the unrefined
    # cells, then the contraction; against central differences of the FP64
    # oracle of the same hybrid scheme, and the saved-state path against the
    # recomputing one
    from oracle import c_oracle as C
    log_banner(f"hybrid backward {scheme} {order} lam {lam}")
    rng = np.random.default_rng(51 + lam)
    X = bm_paths(rng, 2, 45, 3, 0.4 / np.sqrt(45))
    Y = bm_paths(rng, 2, 30, 3, 0.4 / np.sqrt(30))
    gK = rng.normal(size=(2, 2))
    Xt, Yt, gKt = dev(X, torch.float64), dev(Y, torch.float64), dev(gK, torch.float64)
    gX, gY = sk.gram_backward(Xt, Yt, gKt, scheme, order, dyadic=lam)
    gX, gY = gX.cpu().numpy(), gY.cpu().numpy()
    kind = C.APPROX if scheme == "approx" else C.INTERP

    def loss(Xv, Yv):
        m, e = C.gram(Xv, Yv, kind, order, lam=lam)
        return float(np.sum(gK * np.ldexp(m, e)))
    h = 1e-4
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    for which, idx in [("x", (0, 0, 0)), ("x", (1, 33, 1)), ("x", (0, 45, 2)), ("y", (1, 0, 2)),
                       ("y", (0, 17, 0)), ("y", (1, 30, 1))]:
        P = (X if which == "x" else Y).copy()
        P[idx] += h
        lp = loss(P, Y) if which == "x" else loss(X, P)
        P[idx] -= 2 * h
        lm = loss(P, Y) if which == "x" else loss(X, P)
        fd = (lp - lm) / (2 * h)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (which, idx, got, fd)
    K1, state = sk.gram_save(Xt, Yt, scheme, order, dyadic=lam)
    gX1, gY1 = sk.gram_backward_saved(Xt, Yt, gKt, state, scheme, order, dyadic=lam)
    assert np.array_equal(gX1.cpu().numpy(), gX) and np.array_equal(gY1.cpu().numpy(), gY)
    K0 = sk.gram(Xt, Yt, scheme, order, dyadic=lam)
    torch.testing.assert_close(K1, K0, rtol=1e-14, atol=0)
    # the strip pipeline on the refined grid: recomputing and saved-state
    gXp, gYp = sk.gram_backward(Xt, Yt, gKt, scheme, order, dyadic=lam, algo="pipeline")
    K2, state2 = sk.gram_save(Xt, Yt, scheme, order, dyadic=lam, algo="pipeline")
    gX2, gY2 = sk.gram_backward_saved(Xt, Yt, gKt, state2, scheme, order, dyadic=lam,
                                      algo="pipeline")
    torch.testing.assert_close(K2, K0, rtol=1e-14, atol=0)
    for a, b in ((gXp, gX), (gYp, gY), (gX2, gX), (gY2, gY)):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=0, atol=1e-11 * scale)


def test_hybrid_backward_pairs_and_long_columns(sk):
    # ragged pairs through a backward plan on the refined grid (the 1200
    # refined columns of the long pair exceed the adjoint's LDS ring, so its
    # global exchange runs too), against Gram backward calls of each pair
    log_banner("hybrid backward pairs")
    rng = np.random.default_rng(57)
    lens_x, lens_y = [40, 300, 2, 70], [301, 25, 9, 1]
    xs = [bm_paths(rng, 1, n - 1, 4, 0.4 / np.sqrt(n))[0] for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 4, 0.4 / np.sqrt(n))[0] for n in lens_y]
    gk = rng.normal(size=len(xs))
    xl = [dev(a, torch.float64) for a in xs]
    yl = [dev(b, torch.float64) for b in ys]
    gX, gY, xo, yo = sk.pairs_backward(xl, yl, dev(gk, torch.float64), "approx", 5, dyadic=2)
    gXp, gYp, _, _ = sk.pairs_backward(xl, yl, dev(gk, torch.float64), "approx", 5, dyadic=2,
                                       algo="pipeline")
    for a, b in ((gXp, gX), (gYp, gY)):
        torch.testing.assert_close(a, b, rtol=1e-11, atol=1e-11 * float(b.abs().max()))
    for i in range(len(xs)):
        gXi, gYi = sk.gram_backward(xl[i][None], yl[i][None], dev([[gk[i]]], torch.float64),
                                    "approx", 5, dyadic=2)
        s = max(float(gXi.abs().max()), float(gYi.abs().max()), 1e-300)
        torch.testing.assert_close(gX[xo[i]:xo[i + 1]], gXi[0], rtol=1e-11, atol=1e-11 * s)
        torch.testing.assert_close(gY[yo[i]:yo[i + 1]], gYi[0], rtol=1e-11, atol=1e-11 * s)


def test_hybrid_autograd(sk):
    # sig_gram and sig_pairs with the refined grid: autograd (saved state;
    # sig_gram takes the strip pipeline for these six pairs of 2-strip
    # paths) against the direct backward calls (batched Gram; pairs on a
    # plan with the pipeline on): different wave groupings, 1e-11
    log_banner("hybrid autograd")
    rng = np.random.default_rng(58)
    X = dev(bm_paths(rng, 2, 70, 3, 0.05), torch.float64)
    Y = dev(bm_paths(rng, 3, 40, 3, 0.05), torch.float64)
    gK = dev(rng.normal(size=(2, 3)), torch.float64)
    Xg, Yg = X.clone().requires_grad_(True), Y.clone().requires_grad_(True)
    (sk.sig_gram(Xg, Yg, "interp", 5, dyadic=1) * gK).sum().backward()
    gX, gY = sk.gram_backward(X, Y, gK, "interp", 5, dyadic=1)
    torch.testing.assert_close(Xg.grad, gX, rtol=1e-11, atol=1e-11 * float(gX.abs().max()))
    torch.testing.assert_close(Yg.grad, gY, rtol=1e-11, atol=1e-11 * float(gY.abs().max()))
    A = dev(bm_paths(rng, 4, 66, 3, 0.05), torch.float64)
    B = dev(bm_paths(rng, 4, 90, 3, 0.05), torch.float64)
    gk = dev(rng.normal(size=4), torch.float64)
    Ag, Bg = A.clone().requires_grad_(True), B.clone().requires_grad_(True)
    (sk.sig_pairs(Ag, Bg, "approx", 4, dyadic=2) * gk).sum().backward()
    gA, gB, _, _ = sk.pairs_backward([a for a in A], [b for b in B], gk, "approx", 4, dyadic=2)
    torch.testing.assert_close(Ag.grad.reshape(-1, 3), gA, rtol=1e-11,
                               atol=1e-11 * float(gA.abs().max()))
    torch.testing.assert_close(Bg.grad.reshape(-1, 3), gB, rtol=1e-11,
                               atol=1e-11 * float(gB.abs().max()))
