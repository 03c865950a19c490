"""Plans for uneven pairs: every launch configuration against the FP64
oracle, HIP-graph capture and replay against the eager result, the tuner,
and the plan backward against the one-shot backward."""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def uneven(rng, n, d, lo, hi):
    lx = rng.integers(lo, hi + 1, size=n)
    ly = rng.integers(lo, hi + 1, size=n)
    xs = [bm_paths(rng, 1, int(m) - 1, d, 0.3 / np.sqrt(m))[0] for m in lx]
    ys = [bm_paths(rng, 1, int(m) - 1, d, 0.3 / np.sqrt(m))[0] for m in ly]
    return xs, ys


def cat(paths, dtype):
    return torch.tensor(np.concatenate(paths, 0), dtype=dtype, device="cuda")


@pytest.mark.parametrize("scheme,order", [("approx", 6), ("interp", 5), ("fd", 1)])
def test_every_configuration_matches_oracle(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"plan configurations {scheme} {order}")
    rng = np.random.default_rng(51)
    xs, ys = uneven(rng, 40, 3, 1, 700)
    xs[3], ys[3] = xs[3][:1], ys[3]  # one single-point path
    Xc, Yc = cat(xs, torch.float64), cat(ys, torch.float64)
    plan = sk.PairsPlan([torch.empty(len(a), 3, dtype=torch.float64, device="cuda") for a in xs],
                        [torch.empty(len(b), 3, dtype=torch.float64, device="cuda") for b in ys],
                        scheme, order)
    kind = {"approx": C.APPROX, "interp": C.INTERP, "fd": C.FD}[scheme]
    m, e = C.pairs(xs, ys, kind, order)
    ref = np.ldexp(m, e)
    for o in (0, 1):
        for w in (0, 1):
            for b in (0, 1):
                for pp in (0, 1):  # strip pipeline for pairs of several strips
                    plan.configure(o, w, b, pp)
                    k = torch.full((len(xs),), float("nan"), dtype=torch.float64, device="cuda")
                    plan.forward(Xc, Yc, k)
                    err = rel_err(k.cpu().numpy(), ref)
                    assert err.max() < 1e-11, ((o, w, b, pp), err.max(), plan.config())


def test_graph_capture_replays_match_eager(sk):
    log_banner("plan graph capture")
    rng = np.random.default_rng(52)
    xs, ys = uneven(rng, 64, 4, 2, 400)
    Xc, Yc = cat(xs, torch.float32), cat(ys, torch.float32)
    lens_x = [torch.empty(len(a), 4, device="cuda") for a in xs]
    lens_y = [torch.empty(len(b), 4, device="cuda") for b in ys]
    plan = sk.PairsPlan(lens_x, lens_y, "interp", 6)
    plan.configure(1, 1, 1, False)
    k_eager = torch.empty(len(xs), device="cuda")
    plan.forward(Xc, Yc, k_eager)
    torch.cuda.synchronize()
    k = torch.zeros(len(xs), device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        plan.forward(Xc, Yc, k)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(Xc, Yc, k)
    for rep in range(3):
        k.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(k, k_eager), rep
        assert torch.isfinite(junk)


def test_tune_then_oneshot_calls_agree(sk):
    log_banner("plan tuning")
    rng = np.random.default_rng(53)
    xs, ys = uneven(rng, 96, 5, 2, 900)
    Xc, Yc = cat(xs, torch.float32), cat(ys, torch.float32)
    xl = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in xs]
    yl = [torch.tensor(b, dtype=torch.float32, device="cuda") for b in ys]
    plan = sk.PairsPlan(xl, yl, "approx", 8)
    ms = plan.tune(Xc, Yc)
    assert ms > 0
    cfg = plan.config()
    assert cfg["launches"] >= 1
    k = torch.empty(len(xs), device="cuda")
    plan.forward(Xc, Yc, k)
    k1 = sk.pairs(xl, yl, "approx", 8)  # one-shot call: uses the tuned configuration
    torch.testing.assert_close(k1, k, rtol=0, atol=0)


def test_plan_backward_matches_oneshot(sk):
    log_banner("plan backward")
    rng = np.random.default_rng(54)
    xs, ys = uneven(rng, 24, 3, 2, 300)
    xl = [torch.tensor(a, device="cuda") for a in xs]
    yl = [torch.tensor(b, device="cuda") for b in ys]
    Xc, Yc = cat(xs, torch.float64), cat(ys, torch.float64)
    gk = torch.tensor(rng.normal(size=len(xs)), device="cuda")
    gX0, gY0, _, _ = sk.pairs_backward(xl, yl, gk, "approx", 5)
    plan = sk.PairsPlan(xl, yl, "approx", 5, backward=True)
    for o, w, b in ((0, 0, 0), (1, 1, 1), (1, 0, 1), (0, 1, 0)):
        plan.configure(o, w, b)
        gX = torch.full_like(Xc, float("nan"))
        gY = torch.full_like(Yc, float("nan"))
        plan.backward(Xc, Yc, gk, gX, gY)
        torch.testing.assert_close(gX, gX0, rtol=1e-12, atol=1e-12 * float(gX0.abs().max()))
        torch.testing.assert_close(gY, gY0, rtol=1e-12, atol=1e-12 * float(gY0.abs().max()))


def test_pipeline_plan_matches_batched_plan(sk):
    # the forward of pairs with several strips on the strip pipeline against
    # the batched launch of the same plan: bit-identical for the
    # approximation scheme (same cell arithmetic, same orientation)
    log_banner("plan strip pipeline vs batched")
    rng = np.random.default_rng(55)
    xs, ys = uneven(rng, 200, 6, 2, 1500)
    Xc, Yc = cat(xs, torch.float32), cat(ys, torch.float32)
    xl = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in xs]
    yl = [torch.tensor(b, dtype=torch.float32, device="cuda") for b in ys]
    plan = sk.PairsPlan(xl, yl, "approx", 8)
    plan.configure(1, 1, 0, True)
    assert plan.config()["pipeline"]
    kp = torch.full((len(xs),), float("nan"), device="cuda")
    plan.forward(Xc, Yc, kp)
    plan.configure(1, 1, 0, False)
    kb = torch.full((len(xs),), float("nan"), device="cuda")
    plan.forward(Xc, Yc, kb)
    assert torch.equal(kp, kb)


def test_pipeline_plan_graph_replays_match_eager(sk):
    # the strip-pipeline forward (a cooperative launch and a counter fill)
    # captured into a HIP graph: every replay equals the eager result
    log_banner("plan strip pipeline graph capture")
    rng = np.random.default_rng(56)
    xs, ys = uneven(rng, 48, 4, 60, 900)
    Xc, Yc = cat(xs, torch.float32), cat(ys, torch.float32)
    plan = sk.PairsPlan([torch.empty(len(a), 4, device="cuda") for a in xs],
                        [torch.empty(len(b), 4, device="cuda") for b in ys], "approx", 6)
    plan.configure(1, 1, 0, True)
    k_eager = torch.empty(len(xs), device="cuda")
    plan.forward(Xc, Yc, k_eager)
    torch.cuda.synchronize()
    k = torch.zeros(len(xs), device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(Xc, Yc, k)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(Xc, Yc, k)
    for rep in range(3):
        k.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(k, k_eager), rep
        assert torch.isfinite(junk)


@pytest.mark.parametrize("pipeline", [False, True])
def test_saved_state_plan_matches_plan(sk, pipeline):
    # forward_save + backward_saved against forward + backward of the same
    # plan (same kernels on the same state: identical results)
    log_banner(f"plan saved state pipeline={pipeline}")
    rng = np.random.default_rng(57)
    xs, ys = uneven(rng, 40, 5, 70, 700)  # every pair has several strips
    Xc, Yc = cat(xs, torch.float32), cat(ys, torch.float32)
    xl = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in xs]
    yl = [torch.tensor(b, dtype=torch.float32, device="cuda") for b in ys]
    plan = sk.PairsPlan(xl, yl, "interp", 6, backward=True)
    plan.configure(1, 1, 1, pipeline)
    gk = torch.tensor(rng.normal(size=len(xs)), dtype=torch.float32, device="cuda")
    k0 = torch.empty(len(xs), device="cuda")
    plan.forward(Xc, Yc, k0)
    gX0, gY0 = torch.empty_like(Xc), torch.empty_like(Yc)
    plan.backward(Xc, Yc, gk, gX0, gY0)
    k1 = torch.full((len(xs),), float("nan"), device="cuda")
    plan.forward_save(Xc, Yc, k1)
    gX1, gY1 = torch.full_like(Xc, float("nan")), torch.full_like(Yc, float("nan"))
    plan.backward_saved(Xc, Yc, gk, gX1, gY1)
    if pipeline:
        assert torch.equal(k1, k0)
    else:  # the checkpoint sweep's interpolation tail is decided per wave as in the forward
        torch.testing.assert_close(k1, k0, rtol=1e-6, atol=0)
    assert torch.equal(gX1, gX0) and torch.equal(gY1, gY0)


def test_saved_state_needs_one_backward_chunk(sk):
    # pairs of one strip and of several strips: two backward chunks
    log_banner("plan saved state, two chunks")
    rng = np.random.default_rng(58)
    xs, ys = uneven(rng, 12, 3, 10, 300)
    xs[0], ys[0] = xs[0][:20], ys[0][:30]
    xl = [torch.tensor(a, device="cuda") for a in xs]
    yl = [torch.tensor(b, device="cuda") for b in ys]
    plan = sk.PairsPlan(xl, yl, "approx", 4, backward=True)
    plan.configure(1, 1, 1, True)
    k = torch.empty(len(xs), dtype=torch.float64, device="cuda")
    with pytest.raises(sk.SigKernelError) as ei:
        plan.forward_save(cat(xs, torch.float64), cat(ys, torch.float64), k)
    assert ei.value.status == -2  # SK_EWORKSPACE


def test_mmd_pair_list_matches_three_grams(sk):
    # the triangular pair-list MMD^2 against the three-Gram U-statistic
    log_banner("mmd pair list vs grams")
    import workloads as W
    X, Y = W.mmd_sets(0, n=6, steps=200)
    Xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
    val = float(sk.mmd2(Xt, Yt, "approx", 6))
    Kxx = sk.gram(Xt, Xt, "approx", 6)
    Kyy = sk.gram(Yt, Yt, "approx", 6)
    Kxy = sk.gram(Xt, Yt, "approx", 6)
    n = 6
    want = float((Kxx.sum() - Kxx.diagonal().sum()) / (n * (n - 1))
                 + (Kyy.sum() - Kyy.diagonal().sum()) / (n * (n - 1)) - 2.0 * Kxy.mean())
    assert abs(val - want) <= 1e-12 * max(1.0, float(Kxx.abs().max())), (val, want)
