"""Strip pipeline (SK_ALGO_PIPELINE): the strips of one long pair run on
co-resident workgroups that hand their strip-boundary edges on through
global memory (the anti-diagonal wavefront of Section 3.2 over strips).
Parity with the FP64 oracle and with the batched algorithm, which runs the
same cell arithmetic on one wave per pair."""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, rel_err, rel_err_exp

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


# point counts: 16 strips, 3 strips with a 1-row last strip, 2 strips, 1 strip,
# one point; y shorter than a strip (padded strip period) and one segment
LENS_X = [1001, 130, 66, 40, 1, 700]
LENS_Y = [300, 37, 201, 2, 50, 650]


@pytest.mark.parametrize("scheme,order", [("approx", 4), ("interp", 5), ("approx", 8)])
def test_pipeline_fp64_matches_oracle(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"pipeline fp64 {scheme} {order}")
    rng = np.random.default_rng(81)
    xs = [bm_paths(rng, 1, n - 1, 3, 0.4 / np.sqrt(n))[0] for n in LENS_X]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.4 / np.sqrt(n))[0] for n in LENS_Y]
    k = sk.pairs([dev(a, torch.float64) for a in xs], [dev(b, torch.float64) for b in ys],
                 scheme, order, algo="pipeline").cpu().numpy()
    kind = C.APPROX if scheme == "approx" else C.INTERP
    m, e = C.pairs(xs, ys, kind, order)
    err = rel_err(k, np.ldexp(m, e))
    cells = np.array([(a - 1) * (b - 1) for a, b in zip(LENS_X, LENS_Y)], dtype=np.float64)
    # interpolation: the literal oracle's own Vandermonde rounding grows with the cells
    tol = 1e-12 if scheme == "approx" else 1e-12 + 2e-17 * cells
    assert np.all(err < tol), err
    assert k[4] == 1.0


@pytest.mark.parametrize("scheme,order", [("approx", 6), ("interp", 6)])
def test_pipeline_matches_batched_fp32(sk, scheme, order):
    # same cell arithmetic, different wave grouping: bit-identical for the
    # approximation scheme; the interpolation tail is decided per wave, so a
    # row below 2^-26 of the edge scale may be folded in one and not the other
    log_banner(f"pipeline vs batched fp32 {scheme} {order}")
    rng = np.random.default_rng(82)
    xs = [bm_paths(rng, 1, n - 1, 6, 0.5 / np.sqrt(n))[0].astype(np.float32) for n in LENS_X]
    ys = [bm_paths(rng, 1, n - 1, 6, 0.5 / np.sqrt(n))[0].astype(np.float32) for n in LENS_Y]
    # one-pair Grams: the batched algorithm then keeps the pair's orientation
    kp, kb = [], []
    for a, b in zip(xs, ys):
        at, bt = dev(a[None], torch.float32), dev(b[None], torch.float32)
        kp.append(sk.gram(at, bt, scheme, order, algo="pipeline").cpu().numpy()[0, 0])
        kb.append(sk.gram(at, bt, scheme, order).cpu().numpy()[0, 0])
    kp, kb = np.array(kp), np.array(kb)
    if scheme == "approx":
        assert np.array_equal(kp, kb), (kp, kb)
    else:
        assert rel_err(kp, kb).max() < 1e-6


def test_pipeline_exponent_tracking_fp32(sk):
    # kernel values far beyond the FP32 range (|c| large on long paths)
    from oracle import c_oracle as C
    log_banner("pipeline exponent tracking fp32")
    rng = np.random.default_rng(83)
    X = bm_paths(rng, 1, 600, 4, 0.35).astype(np.float32)
    Y = bm_paths(rng, 1, 500, 4, 0.35).astype(np.float32)
    Xt, Yt = dev(X, torch.float32), dev(Y, torch.float32)
    Kp, Ep = sk.gram(Xt, Yt, "approx", 8, algo="pipeline", return_exp=True)
    Kb, Eb = sk.gram(Xt, Yt, "approx", 8, return_exp=True)
    assert int(Ep.cpu().numpy()[0, 0]) > 128
    assert np.array_equal(Kp.cpu().numpy(), Kb.cpu().numpy())
    assert np.array_equal(Ep.cpu().numpy(), Eb.cpu().numpy())
    # the value (about -0.11 * 2^178) comes out of heavy cancellation: the
    # FP32 result is held to the pair's FP32 conditioning floor (the oracle
    # against its FP32 model, 1.6e-6 here; measured 0.5 times it)
    m, e = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX, 8)
    mf, ef = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX_F32MODEL, 8)
    floor = np.maximum(rel_err_exp(mf, ef, m, e), 1e-7)
    assert (rel_err_exp(Kp.cpu().numpy(), Ep.cpu().numpy(), m, e) / floor).max() <= 5


def test_pipeline_hybrid_fp64(sk):
    from oracle import c_oracle as C
    log_banner("pipeline hybrid fp64")
    rng = np.random.default_rng(84)
    X = bm_paths(rng, 2, 180, 3, 0.05)
    Y = bm_paths(rng, 1, 90, 3, 0.05)
    K = sk.gram(dev(X, torch.float64), dev(Y, torch.float64), "approx", 4, algo="pipeline",
                dyadic=1).cpu().numpy()
    m, e = C.gram(X, Y, C.APPROX, 4, lam=1)
    assert rel_err(K, np.ldexp(m, e)).max() < 1e-12


def test_pipeline_full_size_fp32(sk):
    # one pair of 2049-point paths in R^8 (32 strips of 2048 columns):
    # against the oracle; one pair of 8193-point paths (128 strips) against
    # the batched algorithm (bit-identical)
    from oracle import c_oracle as C
    log_banner("pipeline full size fp32")
    rng = np.random.default_rng(85)
    X = bm_paths(rng, 1, 2048, 8, 0.5 / np.sqrt(2048)).astype(np.float32)
    Y = bm_paths(rng, 1, 2048, 8, 0.5 / np.sqrt(2048)).astype(np.float32)
    K = sk.gram(dev(X, torch.float32), dev(Y, torch.float32), "approx", 8, algo="pipeline")
    m, e = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX, 8)
    assert rel_err(K.cpu().numpy(), np.ldexp(m, e)).max() < 2e-5
    X = bm_paths(rng, 1, 8192, 8, 0.5 / np.sqrt(8192)).astype(np.float32)
    Y = bm_paths(rng, 1, 8192, 8, 0.5 / np.sqrt(8192)).astype(np.float32)
    Xt, Yt = dev(X, torch.float32), dev(Y, torch.float32)
    log_banner("pipeline 8193 x 8193")
    Kp = sk.gram(Xt, Yt, "approx", 8, algo="pipeline").cpu().numpy()
    log_banner("batched 8193 x 8193")
    Kb = sk.gram(Xt, Yt, "approx", 8).cpu().numpy()
    assert np.isfinite(Kp).all() and np.array_equal(Kp, Kb), (Kp, Kb)


# ---------------------------------------------------------------------------
# backward: pipelined checkpoint sweep + pipelined adjoint
# ---------------------------------------------------------------------------
# point counts: 5 and 11 strips, 3 strips with a 1-row last strip, a pair
# transposed by the plan (y longer), one strip, a 1-segment y, one point
LENS_BX = [300, 129, 66, 40, 1, 700, 65]
LENS_BY = [200, 37, 201, 2, 50, 130, 700]


def _cat(paths, dtype):
    return torch.tensor(np.concatenate(paths, 0), dtype=dtype, device="cuda")


def _plan_grads(sk, plan, Xc, Yc, gk, pipeline):
    plan.configure(1, 1, 0, pipeline)
    assert plan.config()["pipeline"] == pipeline
    gX = torch.full_like(Xc, float("nan"))
    gY = torch.full_like(Yc, float("nan"))
    plan.backward(Xc, Yc, gk, gX, gY)
    return gX, gY


@pytest.mark.parametrize("scheme,order", [("approx", 5), ("interp", 4)])
def test_pipeline_backward_fp64_matches_batched_and_fd(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"pipeline backward fp64 {scheme} {order}")
    rng = np.random.default_rng(86)
    xs = [bm_paths(rng, 1, n - 1, 3, 0.4 / np.sqrt(n))[0] for n in LENS_BX]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.4 / np.sqrt(n))[0] for n in LENS_BY]
    gk = rng.normal(size=len(xs))
    xl = [dev(a, torch.float64) for a in xs]
    yl = [dev(b, torch.float64) for b in ys]
    Xc, Yc = _cat(xs, torch.float64), _cat(ys, torch.float64)
    gkt = dev(gk, torch.float64)
    plan = sk.PairsPlan(xl, yl, scheme, order, backward=True)
    gXb, gYb = _plan_grads(sk, plan, Xc, Yc, gkt, False)
    gXp, gYp = _plan_grads(sk, plan, Xc, Yc, gkt, True)
    assert torch.isfinite(gXp).all() and torch.isfinite(gYp).all()
    torch.testing.assert_close(gXp, gXb, rtol=1e-11, atol=1e-11 * float(gXb.abs().max()))
    torch.testing.assert_close(gYp, gYb, rtol=1e-11, atol=1e-11 * float(gYb.abs().max()))
    # the one-shot call with the pipeline algorithm runs the same launches
    gX1, gY1, xo, yo = sk.pairs_backward(xl, yl, gkt, scheme, order, algo="pipeline")
    assert torch.equal(gX1, gXp) and torch.equal(gY1, gYp)
    # central differences of the FP64 oracle: last point of a 5-strip x,
    # interior points of the 11-strip x and of the transposed pair's long y
    kind = C.APPROX if scheme == "approx" else C.INTERP
    gXn, gYn = gXp.cpu().numpy(), gYp.cpu().numpy()
    h = 1e-4
    for side, p, t, k in [("x", 0, 299, 2), ("x", 0, 0, 0), ("x", 5, 350, 1), ("y", 6, 640, 0),
                          ("x", 6, 64, 2), ("y", 2, 100, 1)]:
        base = xs[p] if side == "x" else ys[p]
        def loss(v):
            a, b = (v, ys[p]) if side == "x" else (xs[p], v)
            m, e = C.pairs([a], [b], kind, order)
            return gk[p] * float(np.ldexp(m, e)[0])
        v = base.copy()
        v[t, k] += h
        lp = loss(v)
        v[t, k] -= 2 * h
        lm = loss(v)
        fd = (lp - lm) / (2 * h)
        g = gXn[xo[p] + t, k] if side == "x" else gYn[yo[p] + t, k]
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (side, p, t, k, g, fd)


def test_pipeline_backward_fp32_interp_matches_batched(sk):
    # the bench's scheme (interpolation N = 6, FP32) on 96 uneven pairs of up
    # to 1500 points: same cell arithmetic, different rescaling schedule
    log_banner("pipeline backward fp32 interp")
    rng = np.random.default_rng(87)
    lx = rng.integers(32, 1501, size=96)
    ly = rng.integers(32, 1501, size=96)
    xs = [bm_paths(rng, 1, int(m) - 1, 8, 0.5 / np.sqrt(m))[0].astype(np.float32) for m in lx]
    ys = [bm_paths(rng, 1, int(m) - 1, 8, 0.5 / np.sqrt(m))[0].astype(np.float32) for m in ly]
    xl = [dev(a, torch.float32) for a in xs]
    yl = [dev(b, torch.float32) for b in ys]
    Xc, Yc = _cat(xs, torch.float32), _cat(ys, torch.float32)
    gk = dev(rng.normal(size=len(xs)), torch.float32)
    plan = sk.PairsPlan(xl, yl, "interp", 6, backward=True)
    gXb, gYb = _plan_grads(sk, plan, Xc, Yc, gk, False)
    gXp, gYp = _plan_grads(sk, plan, Xc, Yc, gk, True)
    assert torch.isfinite(gXp).all() and torch.isfinite(gYp).all()
    # per path: relative to the path's largest gradient entry
    xo = np.concatenate([[0], np.cumsum(lx)])
    yo = np.concatenate([[0], np.cumsum(ly)])
    for g1, g0, off in ((gXp, gXb, xo), (gYp, gYb, yo)):
        a, b = g1.cpu().numpy(), g0.cpu().numpy()
        for i in range(len(off) - 1):
            s = np.abs(b[off[i]:off[i + 1]]).max()
            assert np.abs(a[off[i]:off[i + 1]] - b[off[i]:off[i + 1]]).max() <= 2e-5 * s, i


@pytest.mark.parametrize("ckpt", [2, 4])
def test_pipeline_gram_backward_fp32_strides(sk, ckpt):
    # approximation N = 8, d = 16 (the uneven pairs' scheme) at both FP32
    # checkpoint strides: the pipelined adjoint's staged boundary edges and
    # per-block records against the batched backward at the same stride
    log_banner(f"pipeline gram backward fp32 stride {ckpt}")
    rng = np.random.default_rng(88)
    X = bm_paths(rng, 3, 300, 16, 0.5 / np.sqrt(300)).astype(np.float32)
    Y = bm_paths(rng, 2, 213, 16, 0.5 / np.sqrt(213)).astype(np.float32)
    gK = dev(rng.normal(size=(3, 2)), torch.float32)
    Xt, Yt = dev(X, torch.float32), dev(Y, torch.float32)
    gXb, gYb = sk.gram_backward(Xt, Yt, gK, "approx", 8, algo="batched", ckpt=ckpt)
    gXp, gYp = sk.gram_backward(Xt, Yt, gK, "approx", 8, algo="pipeline", ckpt=ckpt)
    assert torch.isfinite(gXp).all() and torch.isfinite(gYp).all()
    for g1, g0 in ((gXp, gXb), (gYp, gYb)):
        a, b = g1.cpu().double().numpy(), g0.cpu().double().numpy()
        for i in range(a.shape[0]):
            assert np.abs(a[i] - b[i]).max() <= 2e-5 * np.abs(b[i]).max(), i


def test_pipeline_backward_graph_replays_match_eager(sk):
    # the pipelined backward (Gram, two cooperative launches, counter fills,
    # contraction, reduction) captured into a HIP graph: every replay equals
    # the eager result
    log_banner("pipeline backward graph capture")
    rng = np.random.default_rng(88)
    lx = rng.integers(40, 700, size=32)
    ly = rng.integers(40, 700, size=32)
    xs = [bm_paths(rng, 1, int(m) - 1, 4, 0.4 / np.sqrt(m))[0].astype(np.float32) for m in lx]
    ys = [bm_paths(rng, 1, int(m) - 1, 4, 0.4 / np.sqrt(m))[0].astype(np.float32) for m in ly]
    xl = [dev(a, torch.float32) for a in xs]
    yl = [dev(b, torch.float32) for b in ys]
    Xc, Yc = _cat(xs, torch.float32), _cat(ys, torch.float32)
    gk = dev(rng.normal(size=len(xs)), torch.float32)
    plan = sk.PairsPlan(xl, yl, "approx", 6, backward=True)
    gX0, gY0 = _plan_grads(sk, plan, Xc, Yc, gk, True)
    torch.cuda.synchronize()
    gX, gY = torch.zeros_like(Xc), torch.zeros_like(Yc)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.backward(Xc, Yc, gk, gX, gY)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.backward(Xc, Yc, gk, gX, gY)
    for rep in range(3):
        gX.zero_()
        gY.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(gX, gX0) and torch.equal(gY, gY0), rep


# ---------------------------------------------------------------------------
# Gram backward on the pipeline
# ---------------------------------------------------------------------------
def _gram_backward_ws(sk, X, Y, gK, scheme, order, ws_bytes=None, symmetric=False):
    """sigkernel_backward(SK_OP_GRAM) with the pipeline and a chosen workspace."""
    import ctypes
    from paper_2502_08470_amd import _lib as L
    from paper_2502_08470_amd import api as A
    p = A._params(X.dtype, scheme, order, "pipeline", "native",
                  L.SK_SYMMETRIC if symmetric else 0)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    lib = L.lib()
    if ws_bytes is None:
        ws_bytes = lib.sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(p), 1)
    ws = torch.empty(int(ws_bytes), dtype=torch.uint8, device="cuda")
    gX = torch.full_like(X, float("nan"))
    gY = gX if symmetric else torch.full_like(Y, float("nan"))
    vp = ctypes.c_void_p
    L.check(lib.sigkernel_backward(L.SK_OP_GRAM, vp(X.data_ptr()), None, nx, lxp,
                                   vp(Y.data_ptr()), None, ny, lyp, d, ctypes.byref(p),
                                   vp(gK.data_ptr()), None, vp(gX.data_ptr()),
                                   vp(gY.data_ptr()), vp(ws.data_ptr()), int(ws_bytes),
                                   vp(torch.cuda.current_stream().cuda_stream)))
    return gX, gY


@pytest.mark.parametrize("scheme,order", [("approx", 5), ("interp", 6)])
def test_pipeline_gram_backward_fp64_matches_batched_and_fd(sk, scheme, order):
    # 3 x 2 Gram: x of 200 points (4 strips, a 7-row last strip), y of 90;
    # every chunk size: all six pairs, then chunks of 4 + 2 (a partial last
    # chunk with its own job list)
    from oracle import c_oracle as C
    log_banner(f"pipeline gram backward fp64 {scheme} {order}")
    rng = np.random.default_rng(89)
    X = bm_paths(rng, 3, 199, 3, 0.4 / np.sqrt(200))
    Y = bm_paths(rng, 2, 89, 3, 0.4 / np.sqrt(90))
    gK = rng.normal(size=(3, 2))
    Xt, Yt, gKt = dev(X, torch.float64), dev(Y, torch.float64), dev(gK, torch.float64)
    gXb, gYb = sk.gram_backward(Xt, Yt, gKt, scheme, order)
    gXp, gYp = sk.gram_backward(Xt, Yt, gKt, scheme, order, algo="pipeline")
    assert torch.isfinite(gXp).all() and torch.isfinite(gYp).all()
    torch.testing.assert_close(gXp, gXb, rtol=1e-11, atol=1e-11 * float(gXb.abs().max()))
    torch.testing.assert_close(gYp, gYb, rtol=1e-11, atol=1e-11 * float(gYb.abs().max()))
    import ctypes
    from paper_2502_08470_amd import _lib as L
    from paper_2502_08470_amd import api as A
    p = A._params(torch.float64, scheme, order, "pipeline")
    ws4 = L.lib().sigkernel_gram_workspace(2, 200, 2, 90, 3, ctypes.byref(p), 1) + (64 << 10)
    gXc, gYc = _gram_backward_ws(sk, Xt, Yt, gKt, scheme, order, ws_bytes=ws4)
    assert torch.equal(gXc, gXp) and torch.equal(gYc, gYp)
    # central differences of the FP64 oracle on the Gram loss
    kind = C.APPROX if scheme == "approx" else C.INTERP
    h = 1e-4
    gXn, gYn = gXp.cpu().numpy(), gYp.cpu().numpy()
    for side, a, t, k in [("x", 0, 199, 2), ("x", 2, 64, 0), ("x", 1, 130, 1), ("y", 1, 45, 2),
                          ("y", 0, 0, 0)]:
        def loss(Xv, Yv):
            m, e = C.gram(Xv, Yv, kind, order)
            return float(np.sum(gK * np.ldexp(m, e)))
        V = (X if side == "x" else Y).copy()
        V[a, t, k] += h
        lp = loss(V, Y) if side == "x" else loss(X, V)
        V[a, t, k] -= 2 * h
        lm = loss(V, Y) if side == "x" else loss(X, V)
        fd = (lp - lm) / (2 * h)
        g = gXn[a, t, k] if side == "x" else gYn[a, t, k]
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (side, a, t, k, g, fd)


def test_pipeline_gram_backward_fp32_symmetric_and_one_strip(sk):
    # FP32 interpolation N = 6 (the bench's scheme) on a symmetric 4 x 4 Gram
    # of 300-point paths: both contributions in gX, as the batched backward;
    # one-strip paths fall through to the batched backward unchanged
    log_banner("pipeline gram backward fp32 symmetric")
    rng = np.random.default_rng(90)
    X = bm_paths(rng, 4, 299, 8, 0.5 / np.sqrt(300)).astype(np.float32)
    gK = rng.normal(size=(4, 4)).astype(np.float32)
    Xt, gKt = dev(X, torch.float32), dev(gK, torch.float32)
    gXb, _ = sk.gram_backward(Xt, Xt, gKt, "interp", 6, symmetric=True)
    gXp, _ = sk.gram_backward(Xt, Xt, gKt, "interp", 6, symmetric=True, algo="pipeline")
    assert torch.isfinite(gXp).all()
    for a in range(4):
        s = float(gXb[a].abs().max())
        assert float((gXp[a] - gXb[a]).abs().max()) <= 2e-5 * s, a
    Xs = Xt[:, :60].contiguous()
    g1, _ = sk.gram_backward(Xs, Xs, gKt, "interp", 6, symmetric=True)
    g2, _ = sk.gram_backward(Xs, Xs, gKt, "interp", 6, symmetric=True, algo="pipeline")
    assert torch.equal(g1, g2)


@pytest.mark.parametrize("scheme,order", [("approx", 5), ("interp", 6)])
def test_pipeline_gram_saved_state(sk, scheme, order):
    # gram_save on the pipeline (the checkpoint sweep's values) against the
    # batched forward; gram_backward_saved against the recomputing
    # pipelined backward (the same kernels from the same state)
    log_banner(f"pipeline gram saved state {scheme} {order}")
    rng = np.random.default_rng(91)
    X = dev(bm_paths(rng, 3, 199, 3, 0.4 / np.sqrt(200)), torch.float64)
    Y = dev(bm_paths(rng, 2, 89, 3, 0.4 / np.sqrt(90)), torch.float64)
    gK = dev(rng.normal(size=(3, 2)), torch.float64)
    K1, state = sk.gram_save(X, Y, scheme, order, algo="pipeline")
    K0 = sk.gram(X, Y, scheme, order)
    torch.testing.assert_close(K1, K0, rtol=1e-14, atol=0)
    gX1, gY1 = sk.gram_backward_saved(X, Y, gK, state, scheme, order, algo="pipeline")
    gX0, gY0 = sk.gram_backward(X, Y, gK, scheme, order, algo="pipeline")
    assert torch.equal(gX1, gX0) and torch.equal(gY1, gY0)
    # the state's size query: the pipeline's own, larger than the batched one
    assert state.numel() == sk.gram_state_size(X, Y, scheme, order, algo="pipeline") > \
        sk.gram_state_size(X, Y, scheme, order)


def test_pipeline_gram_forward_chunks(sk):
    # the Gram forward on the pipeline with a workspace of 4 pairs' chunk for
    # a 3 x 2 Gram (chunks of 4 + 2, the last with its own job list): the
    # same values as the whole Gram in one chunk, and as the batched forward
    import ctypes
    from paper_2502_08470_amd import _lib as L
    from paper_2502_08470_amd import api as A
    log_banner("pipeline gram forward chunks")
    rng = np.random.default_rng(92)
    X = dev(bm_paths(rng, 3, 199, 3, 0.4 / np.sqrt(200)), torch.float64)
    Y = dev(bm_paths(rng, 2, 89, 3, 0.4 / np.sqrt(90)), torch.float64)
    K1 = sk.gram(X, Y, "approx", 6, algo="pipeline")
    K0 = sk.gram(X, Y, "approx", 6)
    assert torch.equal(K1, K0)
    p = A._params(torch.float64, "approx", 6, "pipeline")
    lib = L.lib()
    ws4 = lib.sigkernel_gram_workspace(2, 200, 2, 90, 3, ctypes.byref(p), 0) + (16 << 10)
    assert ws4 < lib.sigkernel_gram_workspace(3, 200, 2, 90, 3, ctypes.byref(p), 0)
    ws = torch.empty(int(ws4), dtype=torch.uint8, device="cuda")
    K = torch.full((3, 2), float("nan"), dtype=torch.float64, device="cuda")
    vp = ctypes.c_void_p
    L.check(lib.sigkernel_gram(vp(X.data_ptr()), 3, 200, vp(Y.data_ptr()), 2, 90, 3,
                               ctypes.byref(p), vp(K.data_ptr()), None, vp(ws.data_ptr()),
                               int(ws4), vp(torch.cuda.current_stream().cuda_stream)))
    assert torch.equal(K, K1)
