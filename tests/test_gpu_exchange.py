"""Long pairs whose strip-boundary edges go through the global exchange
(forward beyond ~270-410 columns, adjoint beyond ~650-1220 columns,
depending on dtype and N): forward against the FP64 oracle, gradients
against central differences, several strips each."""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, oracle_gram, rel_err

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


@pytest.mark.parametrize("scheme,order", [("approx", 6), ("interp", 5), ("approx", 3)])
def test_long_pairs_forward_fp64(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"global exchange fwd fp64 {scheme} {order}")
    rng = np.random.default_rng(61)
    lens_x, lens_y = [300, 130, 65, 201], [700, 1300, 900, 100]
    xs = [bm_paths(rng, 1, n - 1, 3, 0.5 / np.sqrt(n))[0] for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.5 / np.sqrt(n))[0] for n in lens_y]
    xl = [dev(a, torch.float64) for a in xs]
    yl = [dev(b, torch.float64) for b in ys]
    plan = sk.PairsPlan(xl, yl, scheme, order)
    plan.configure(1, 0, 1)  # not transposed: the long paths are the columns
    k = torch.empty(len(xs), dtype=torch.float64, device="cuda")
    plan.forward(torch.cat(xl), torch.cat(yl), k)
    kind = C.APPROX if scheme == "approx" else C.INTERP
    m, e = C.pairs(xs, ys, kind, order)
    err = rel_err(k.cpu().numpy(), np.ldexp(m, e))
    if scheme == "approx":
        assert err.max() < 1e-12, err
    else:
        # the literal FP64 oracle solves a monomial Vandermonde system per
        # cell (condition ~3e3 at N = 5); its rounding grows about linearly
        # with the number of cells (an extended-precision evaluation of the
        # same scheme agrees with the converged kernel to 1e-16 while the
        # FP64 oracle is 1e-13 off at 2e4 cells)
        cells = np.array([(a - 1) * (b - 1) for a, b in zip(lens_x, lens_y)], dtype=float)
        assert np.all(err < 1e-12 + 2e-17 * cells), err


def test_long_gram_fp32_interp(sk):
    log_banner("global exchange fwd fp32 interp")
    rng = np.random.default_rng(62)
    X = bm_paths(rng, 2, 130, 4, 0.5 / np.sqrt(1300)).astype(np.float32)
    Y = bm_paths(rng, 2, 1300, 4, 0.5 / np.sqrt(1300)).astype(np.float32)
    K = sk.gram(dev(X, torch.float32), dev(Y, torch.float32), "interp", 6).cpu().numpy()
    m, e = oracle_gram(X.astype(np.float64), Y.astype(np.float64), "interp", 6)
    err = rel_err(K, np.ldexp(m, e))
    assert err.mean() <= 1e-6, err


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-6), (torch.float32, 1e-5)])
def test_long_gram_gradients(sk, dtype, tol):
    from oracle import c_oracle as C
    log_banner(f"global exchange gradients {dtype}")
    rng = np.random.default_rng(63)
    # 1500 columns: beyond the adjoint's LDS ring in FP32 and FP64
    X = bm_paths(rng, 2, 150, 3, 0.4 / np.sqrt(150))
    Y = bm_paths(rng, 1, 1500, 3, 0.4 / np.sqrt(1500))
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    gK = rng.normal(size=(2, 1))
    Xt = dev(X, dtype).requires_grad_(True)
    Yt = dev(Y, dtype).requires_grad_(True)
    # the batched backward (its exchange variant) through autograd, against
    # the direct call and the pipelined backward
    (sk.sig_gram(Xt, Yt, "approx", 5, algo="batched") * dev(gK, dtype)).sum().backward()
    gX, gY = Xt.grad.cpu().double().numpy(), Yt.grad.cpu().double().numpy()
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    for algo in ("batched", "pipeline"):
        gX2, gY2 = sk.gram_backward(dev(X, dtype), dev(Y, dtype), dev(gK, dtype), "approx", 5,
                                    algo=algo)
        np.testing.assert_allclose(gX2.cpu().double().numpy(), gX, rtol=0, atol=tol * scale)
        np.testing.assert_allclose(gY2.cpu().double().numpy(), gY, rtol=0, atol=tol * scale)

    def loss(Xv, Yv):
        m, e = C.gram(Xv, Yv, C.APPROX, 5)
        return float(np.sum(gK * np.ldexp(m, e)))
    h = 1e-4
    for which, idx in [("x", (0, 64, 1)), ("x", (1, 150, 2)), ("y", (0, 0, 0)), ("y", (0, 700, 1)),
                       ("y", (0, 1500, 2))]:
        P = (X if which == "x" else Y).copy()
        P[idx] += h
        lp = loss(P, Y) if which == "x" else loss(X, P)
        P[idx] -= 2 * h
        lm = loss(P, Y) if which == "x" else loss(X, P)
        fd = (lp - lm) / (2 * h)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= tol * scale, (which, idx, got, fd)


def test_long_gram_interp_gradients_fp64(sk):
    # the interpolation scheme's backward on exchange pairs (1500 columns):
    # the checkpoint sweep's boundary-edge copy and the replayed tail lengths
    # against central differences of the oracle
    from oracle import c_oracle as C
    log_banner("global exchange interpolation gradients fp64")
    rng = np.random.default_rng(64)
    X = bm_paths(rng, 2, 130, 3, 0.5 / np.sqrt(130))
    Y = bm_paths(rng, 1, 1500, 3, 0.5 / np.sqrt(1500))
    gK = rng.normal(size=(2, 1))
    gX, gY = sk.gram_backward(dev(X, torch.float64), dev(Y, torch.float64), dev(gK, torch.float64),
                              "interp", 6, algo="batched")
    gX, gY = gX.cpu().numpy(), gY.cpu().numpy()
    scale = max(np.abs(gX).max(), np.abs(gY).max())

    def loss(Xv, Yv):
        m, e = C.gram(Xv, Yv, C.INTERP, 6)
        return float(np.sum(gK * np.ldexp(m, e)))
    h = 1e-4
    for which, idx in [("x", (0, 63, 0)), ("x", (1, 130, 2)), ("y", (0, 1, 1)), ("y", (0, 999, 0)),
                       ("y", (0, 1500, 2))]:
        P = (X if which == "x" else Y).copy()
        P[idx] += h
        lp = loss(P, Y) if which == "x" else loss(X, P)
        P[idx] -= 2 * h
        lm = loss(P, Y) if which == "x" else loss(X, P)
        fd = (lp - lm) / (2 * h)
        got = gX[idx] if which == "x" else gY[idx]
        assert abs(got - fd) <= 1e-6 * scale, (which, idx, got, fd)


def test_long_pairs_exponents_fp32(sk):
    # values far beyond FP32 range through the global exchange records
    log_banner("global exchange exponents")
    rng = np.random.default_rng(64)
    X = bm_paths(rng, 1, 200, 6, 0.6).astype(np.float32)
    Y = bm_paths(rng, 1, 800, 6, 0.3).astype(np.float32)
    K, Ke = sk.gram(dev(X, torch.float32), dev(Y, torch.float32), "approx", 8, return_exp=True)
    m, e = oracle_gram(X.astype(np.float64), Y.astype(np.float64), "approx", 8)
    assert (e + np.log2(np.abs(m))).max() > 150  # 2^203: beyond FP32
    got = np.ldexp(K.cpu().double().numpy(), Ke.cpu().numpy() - e)
    # at the pair's FP32 conditioning floor (oracle vs its FP32 model,
    # 6.9e-7 here): measured 10.7 times it
    from oracle import c_oracle as C
    mf, ef = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX_F32MODEL, 8)
    floor = np.maximum(np.abs(np.ldexp(mf, ef - e) / m - 1), 1e-7)
    assert (np.abs(got / m - 1) / floor).max() <= 30
