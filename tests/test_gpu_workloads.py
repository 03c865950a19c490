"""GPU parity at the full sizes of the benchmark configurations, in the
launch configuration the benchmark uses, checked on sampled outputs the FP64
oracle computes one by one.

* 128x128 Gram (R^8, 256 steps, interpolation N=6, FP32) through autograd:
  MAPE <= 1e-6 on a sampled 8x8 block; dL/dX (L = sum K) on sampled
  coordinates within 1e-5 relative of central differences of the oracle.
* 4096 uneven oscillatory pairs (R^16, 32..2048 points, approximation N=8):
  FP64 path on sampled pairs within 1e-8 relative (these short oscillatory
  pairs amplify rounding; the FP64 oracle itself is only good to about
  1e-10 on the worst of them).
* MMD^2 sets (2 x 64 paths in R^5, 512 steps, approximation N=8, FP32):
  sampled Kxy entries (MAPE <= 1e-6) and dMMD^2/dX on sampled coordinates
  within 1e-5 relative of central differences of the oracle.
* 1024x1024 Gram (R^32, 1024 steps, unit-variance cell constants,
  approximation N=8, kernels near 2^1200 with exponents): a seeded 32x32
  block against the oracle, the FP64 sweep of the FP32 points at MAPE <= 1e-6
  and the FP32 sweep (bf16 3-way split Gram) at its measured floor; the
  backward through log K on 8 seeded coordinates against central
  differences of the oracle.
* 4096 uneven pairs in FP32: MAPE <= 1e-6 on the sampled pairs whose
  conditioning floor (the oracle's FP32 model) allows it.
"""
import numpy as np
import pytest

from tests.gpu_common import log_banner, rel_err, rel_err_exp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def test_batched_interp_gram_full_size(sk):
    import workloads as W
    from oracle import c_oracle as C
    log_banner("full 128x128 interpolation Gram")
    X, Y = W.batched_interp_gram(0)
    Xt = torch.tensor(X, device="cuda").requires_grad_(True)
    Yt = torch.tensor(Y, device="cuda").requires_grad_(True)
    K = sk.sig_gram(Xt, Yt, "interp", 6)
    K.sum().backward()
    rng = np.random.default_rng(0)
    ia = np.sort(rng.choice(128, 8, replace=False))
    ib = np.sort(rng.choice(128, 8, replace=False))
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    m, e = C.gram(Xd[ia], Yd[ib], C.INTERP, 6)
    err = rel_err(K.detach().cpu().numpy()[np.ix_(ia, ib)], np.ldexp(m, e))
    assert err.mean() <= 1e-6, err.mean()
    gX = Xt.grad.cpu().double().numpy()
    scale = np.abs(gX).max()
    h = 1e-4
    for a, t, k in [(int(ia[0]), 0, 3), (int(ia[3]), 128, 0), (int(ia[7]), 256, 7)]:
        P = Xd[a:a + 1].copy()
        P[0, t, k] += h
        lp = np.ldexp(*C.gram(P, Yd, C.INTERP, 6)).sum()
        P[0, t, k] -= 2 * h
        lm = np.ldexp(*C.gram(P, Yd, C.INTERP, 6)).sum()
        fd = (lp - lm) / (2 * h)
        assert abs(gX[a, t, k] - fd) <= 1e-5 * scale, (a, t, k, gX[a, t, k], fd)


def test_uneven_pairs_full_size(sk):
    import workloads as W
    from oracle import c_oracle as C
    log_banner("full 4096 uneven pairs")
    xs, ys = W.uneven_pairs(0)
    xs64 = [a.astype(np.float64) for a in xs]
    ys64 = [b.astype(np.float64) for b in ys]
    k64, e64 = sk.pairs([torch.tensor(a, device="cuda") for a in xs64],
                        [torch.tensor(b, device="cuda") for b in ys64], "approx", 8,
                        return_exp=True)
    k32, e32 = sk.pairs([torch.tensor(a, device="cuda") for a in xs],
                        [torch.tensor(b, device="cuda") for b in ys], "approx", 8,
                        return_exp=True)
    assert torch.isfinite(k32).all()
    rng = np.random.default_rng(1)
    pick = rng.choice(4096, 12, replace=False)
    m, e = C.pairs([xs64[i] for i in pick], [ys64[i] for i in pick], C.APPROX, 8)
    err = rel_err_exp(k64.cpu().numpy()[pick], e64.cpu().numpy()[pick], m, e)
    assert err.max() < 1e-8, err


def test_uneven_pairs_fp32_resolved_pairs(sk):
    # The FP32 forward of the 4096 uneven pairs against the oracle on 64
    # seeded pairs.  Short oscillatory pairs are ill-conditioned beyond FP32:
    # each sampled pair's conditioning floor is the distance between the
    # oracle and the oracle's FP32 model (increments, constants and edge
    # coefficients of degree >= 2 rounded to FP32); most pairs sit above
    # 1e-7, where no FP32-state evaluation can reach the 1e-6 target.  So:
    # * FP32 paths swept in FP64 (the precision mode for such workloads):
    #   MAPE <= 1e-6 over every sampled pair;
    # * FP32 sweep: every pair within a bounded factor of its floor (it gets
    #   what the FP32 state allows), MAPE <= 1e-6 on the pairs whose floor
    #   is <= 1e-7 (2 of the 64), and the sampled MAPE reported (1.2, from
    #   one pair of 1432 x 52 points whose floor is 0.7).
    import workloads as W
    from oracle import c_oracle as C
    log_banner("full 4096 uneven pairs, FP32 vs oracle on resolved pairs")
    xs, ys = W.uneven_pairs(0)
    xl = [torch.tensor(a, device="cuda") for a in xs]
    yl = [torch.tensor(b, device="cuda") for b in ys]
    k32, e32 = sk.pairs(xl, yl, "approx", 8, return_exp=True)
    kf, ef = sk.pairs(xl, yl, "approx", 8, return_exp=True, sweep="f64")
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(4096, 64, replace=False))
    xs64 = [xs[i].astype(np.float64) for i in pick]
    ys64 = [ys[i].astype(np.float64) for i in pick]
    m, e = C.pairs(xs64, ys64, C.APPROX, 8)
    mf, eff = C.pairs(xs64, ys64, C.APPROX_F32MODEL, 8)
    floor = rel_err_exp(mf, eff, m, e)
    err = rel_err_exp(k32.cpu().numpy()[pick], e32.cpu().numpy()[pick], m, e)
    errf = rel_err_exp(kf.cpu().numpy()[pick], ef.cpu().numpy()[pick], m, e)
    ok = floor <= 1e-7
    ratio = err / np.maximum(floor, 1e-7)
    print(f"FP64 sweep of the FP32 points: MAPE {errf.mean():.3g} max {errf.max():.3g}", flush=True)
    print(f"FP32 sweep: MAPE over the 64 sampled pairs {err.mean():.3g}; {ok.sum()} pairs with floor "
          f"<= 1e-7, MAPE {err[ok].mean() if ok.any() else float('nan'):.3g}; error / max(floor, 1e-7): "
          f"median {np.median(ratio):.3g} max {ratio.max():.3g}", flush=True)
    print("pairs (index, x points, y points, floor, FP32 error):",
          [(int(pick[i]), len(xs[pick[i]]), len(ys[pick[i]]), float(floor[i]), float(err[i]))
           for i in range(64)], flush=True)
    assert errf.mean() <= 1e-6, errf
    # the FP32 sweep's rounding (FP32 FMA chains for the constants and the
    # rows) exceeds the model's single roundings: measured median 2.9, max
    # 111 times the floor
    assert np.median(ratio) <= 10 and np.all(ratio <= 300), ratio
    if ok.any():
        assert err[ok].mean() <= 1e-6, err[ok]


def test_uneven_pairs_backward_full_size(sk):
    # the 4096 uneven pairs' gradient, in the launches the workload study
    # times (a backward plan whose multi-strip pairs run the pipelined
    # checkpoint sweep and adjoint): FP64 against the batched backward of the
    # same plan and against central differences of the oracle; FP32 against
    # FP64 on the pairs FP32 can resolve (short oscillatory pairs are
    # ill-conditioned: |k| up to 1e13 out of cancelling terms, where the FP32
    # forward itself is off by O(1))
    import workloads as W
    from oracle import c_oracle as C
    log_banner("full 4096 uneven pairs backward")
    xs, ys = W.uneven_pairs(0)
    rng = np.random.default_rng(3)
    gk = rng.normal(size=len(xs))
    xo = np.concatenate([[0], np.cumsum([len(a) for a in xs])])
    yo = np.concatenate([[0], np.cumsum([len(b) for b in ys])])

    def run(dtype, pipeline):
        xl = [torch.tensor(a, dtype=dtype, device="cuda") for a in xs]
        yl = [torch.tensor(b, dtype=dtype, device="cuda") for b in ys]
        Xc, Yc = torch.cat(xl), torch.cat(yl)
        plan = sk.PairsPlan(xl, yl, "approx", 8, backward=True)
        plan.configure(1, 1, 1, pipeline)
        k = torch.empty(len(xs), dtype=dtype, device="cuda")
        plan.forward(Xc, Yc, k)
        gX, gY = torch.empty_like(Xc), torch.empty_like(Yc)
        plan.backward(Xc, Yc, torch.tensor(gk, dtype=dtype, device="cuda"), gX, gY)
        out = (k.cpu().double().numpy(), gX.cpu().double().numpy(), gY.cpu().double().numpy())
        del plan, xl, yl, Xc, Yc, gX, gY
        torch.cuda.empty_cache()
        return out

    def path_err(a, b, i):
        sx, sy = slice(xo[i], xo[i + 1]), slice(yo[i], yo[i + 1])
        scale = max(np.abs(b[1][sx]).max(), np.abs(b[2][sy]).max())
        return max(np.abs(a[1][sx] - b[1][sx]).max(), np.abs(a[2][sy] - b[2][sy]).max()) / scale

    p64, b64, p32 = run(torch.float64, True), run(torch.float64, False), run(torch.float32, True)
    assert np.isfinite(p32[1]).all() and np.isfinite(p32[2]).all()
    e64 = max(path_err(p64, b64, i) for i in range(len(xs)))
    assert e64 <= 1e-9, e64
    # FP32: a gross-error check on the pairs whose FP32 kernel value is good
    # to 1e-5 (2904 of 4096; their gradients, derivatives of cancelling sums,
    # are more sensitive: 4.4e-3 at worst); the code itself is pinned in FP64
    kerr = np.abs(p32[0] / p64[0] - 1)
    good = [i for i in range(len(xs)) if kerr[i] <= 1e-5]
    e32 = max(path_err(p32, p64, i) for i in good)
    print(f"FP64 pipeline vs batched {e64:.3g}; FP32 vs FP64 on {len(good)} resolved pairs {e32:.3g}",
          flush=True)
    assert len(good) >= len(xs) // 2 and e32 <= 1e-2
    # pairs of 400-600 points (several strips, well conditioned, a few
    # hundred thousand oracle cells each)
    small = [i for i in range(len(xs)) if 400 <= len(xs[i]) <= 600 and 400 <= len(ys[i]) <= 600][:2]
    assert len(small) == 2
    h = 1e-4
    for i in small:
        x64, y64 = xs[i].astype(np.float64), ys[i].astype(np.float64)
        for t, k in [(1, 3), (len(xs[i]) - 2, 11)]:
            def loss(v):
                m, e = C.pairs([v], [y64], C.APPROX, 8)
                return gk[i] * float(np.ldexp(m, e)[0])
            v = x64.copy()
            v[t, k] += h
            lp = loss(v)
            v[t, k] -= 2 * h
            lm = loss(v)
            fd = (lp - lm) / (2 * h)
            g = p64[1][xo[i] + t, k]
            assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (i, t, k, g, fd)


def test_mmd_sets_full_size(sk):
    import workloads as W
    from oracle import c_oracle as C
    log_banner("full MMD sets")
    X, Y = W.mmd_sets(0)
    Xt = torch.tensor(X, device="cuda").requires_grad_(True)
    Yt = torch.tensor(Y, device="cuda").requires_grad_(True)
    val = sk.mmd2(Xt, Yt, "approx", 8)
    val.backward()
    gX = Xt.grad.cpu().double().numpy()
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    Kxy = sk.gram(Xt.detach(), Yt.detach(), "approx", 8).cpu().numpy()
    rng = np.random.default_rng(2)
    ia, ib = rng.choice(64, 4, replace=False), rng.choice(64, 4, replace=False)
    m, e = C.gram(Xd[ia], Yd[ib], C.APPROX, 8)
    err = rel_err(Kxy[np.ix_(ia, ib)], np.ldexp(m, e))
    assert err.mean() <= 1e-6, err
    # dMMD^2 on 8 seeded coordinates, 4 of X and 4 of Y: only row/column a
    # of Kxx and row a of Kxy depend on X[a]; only row/column b of Kyy and
    # column b of Kxy on Y[b] (MMD^2 = mean' Kxx + mean' Kyy - 2 mean Kxy,
    # primes: diagonals excluded)
    gY = Yt.grad.cpu().double().numpy()
    n = 64
    h = 1e-4
    crng = np.random.default_rng(8)
    coords = [(s, int(crng.integers(n)), int(crng.integers(513)), int(crng.integers(5)))
              for s in (0, 0, 0, 0, 1, 1, 1, 1)]
    got, fds = [], []
    for side, a, t, k in coords:
        own, other = (Xd, Yd) if side == 0 else (Yd, Xd)

        def part(Pa):
            ks = np.ldexp(*C.gram(Pa[None], own, C.APPROX, 8))[0]
            ks[a] = 0.0  # diagonal excluded by the U-statistic
            kc = np.ldexp(*C.gram(Pa[None], other, C.APPROX, 8))[0]
            return 2.0 * ks.sum() / (n * (n - 1)) - 2.0 * kc.sum() / (n * n)
        P = own[a].copy()
        P[t, k] += h
        lp = part(P)
        P[t, k] -= 2 * h
        lm = part(P)
        fds.append((lp - lm) / (2 * h))
        got.append((gX if side == 0 else gY)[a, t, k])
    got, fds = np.array(got), np.array(fds)
    # relative per coordinate, for entries above 1% of the largest checked
    den = np.maximum(np.abs(fds), 1e-2 * np.abs(fds).max())
    rel = np.abs(got - fds) / den
    # the same gradient with the FP32 paths swept in FP64
    X2 = torch.tensor(X, device="cuda").requires_grad_(True)
    Y2 = torch.tensor(Y, device="cuda").requires_grad_(True)
    sk.mmd2(X2, Y2, "approx", 8, sweep="f64").backward()
    g64 = np.array([(X2.grad if s == 0 else Y2.grad)[a, t, k].item() for s, a, t, k in coords])
    rel64 = np.abs(g64 - fds) / den
    print(f"dMMD^2 vs central differences on 8 coordinates: FP32 sweep max rel {rel.max():.2e}, "
          f"FP64 sweep max rel {rel64.max():.2e}", flush=True)
    # MMD^2 is a difference of nearly equal means: the FP32 state keeps
    # about 5e-4 of its gradient per coordinate, the FP64 sweep the target
    assert np.all(rel64 <= 1e-5), (coords, g64, fds)
    assert np.all(rel <= 2e-3), (coords, got, fds)
    assert np.isfinite(float(val))


@pytest.fixture(scope="module")
def large_block():
    """A seeded 32 x 32 block (rows and columns sampled from the 1024 paths
    each) of the 1024 x 1024 R^32 Gram, and the oracle's values on it (FP32
    points promoted to FP64; about a minute of host time)."""
    import workloads as W
    from oracle import c_oracle as C
    X, Y = W.large_gram(0)
    rng = np.random.default_rng(32)
    ia = np.sort(rng.choice(1024, 32, replace=False))
    ib = np.sort(rng.choice(1024, 32, replace=False))
    Xs, Ys = X[ia], Y[ib]
    log_banner("oracle on the 32x32 block of the 1024x1024 Gram")
    m, e = C.gram(Xs.astype(np.float64), Ys.astype(np.float64), C.APPROX, 8)
    return Xs, Ys, m, e


def test_large_gram_block_32x32(sk, large_block):
    # MAPE on the sampled 32 x 32 block (1024 pairs, 1.07e9 cells), kernel
    # values near 2^1200: FP32 paths with the FP64 sweep (cell constants of
    # the FP32 points in FP64, FP64 state) at the target; the FP32 sweep
    # (bf16 3-way split Gram) at its floor, which the problem's conditioning
    # sets (state rounding amplified over 1024 x 1024 cells)
    Xs, Ys, m, e = large_block
    log_banner("32x32 block of the 1024x1024 Gram: FP32 sweep and FP64 sweep")
    Xt, Yt = torch.tensor(Xs, device="cuda"), torch.tensor(Ys, device="cuda")
    assert (e + np.log2(np.abs(m))).min() > 500
    K, Ke = sk.gram(Xt, Yt, "approx", 8, return_exp=True, sweep="f64")
    e64 = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
    K, Ke = sk.gram(Xt, Yt, "approx", 8, return_exp=True, gram_mode="bf16x3")
    e32 = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
    print(f"FP64 sweep: MAPE {e64.mean():.3g} max {e64.max():.3g}; FP32 sweep (bf16x3 Gram): "
          f"MAPE {e32.mean():.3g} max {e32.max():.3g}", flush=True)
    # FP64 sweep: the FP32 outputs' own rounding (2^-24) is all that is left
    assert e64.mean() <= 1e-7 and e64.max() <= 1.2e-7, (e64.mean(), e64.max())
    # FP32 sweep: measured MAPE 1.0e-4 (max 1.1e-2 on the worst of 1024
    # pairs), the floor of the FP32 state on this problem
    assert e32.mean() <= 2e-4, (e32.mean(), e32.max())


def test_large_gram_backward_log_loss(sk, large_block):
    # Backward at full size through the exponents: L = sum w_ab log K_ab over
    # four pairs of the block, seeded into the block's backward as
    # gK = w / K (mantissa w / m, exponent -e; K itself is near 2^1200).
    # dL/dX and dL/dY on 8 seeded coordinates against central differences
    # (h = 1e-4) of the oracle.
    from oracle import c_oracle as C
    Xs, Ys, m, e = large_block
    log_banner("1024-point d=32 Gram backward through log K")
    sel_a, sel_b = [3, 17], [5, 29]
    w = np.array([[1.0, -0.5], [0.7, 0.25]])
    gk = np.zeros((32, 32))
    gke = np.zeros((32, 32), dtype=np.int32)
    for i, a in enumerate(sel_a):
        for j, b in enumerate(sel_b):
            gk[a, b] = w[i, j] / m[a, b]
            gke[a, b] = -e[a, b]
    Xt, Yt = torch.tensor(Xs, device="cuda"), torch.tensor(Ys, device="cuda")
    X64, Y64 = Xs.astype(np.float64), Ys.astype(np.float64)

    def loss(Xa, Yb):  # oracle: the four pairs' weighted log-kernel
        mm, ee = C.gram(Xa, Yb, C.APPROX, 8)
        return float(np.sum(w * (np.log(np.abs(mm)) + ee * np.log(2.0))))
    crng = np.random.default_rng(9)
    coords = [(s, int(crng.integers(2)), int(crng.integers(1025)), int(crng.integers(32)))
              for s in (0, 0, 0, 0, 1, 1, 1, 1)]
    h = 1e-4
    fds = []
    for side, i, t, k in coords:
        Xa, Yb = X64[sel_a].copy(), Y64[sel_b].copy()
        P = Xa if side == 0 else Yb
        P[i, t, k] += h
        lp = loss(Xa, Yb)
        P[i, t, k] -= 2 * h
        lm = loss(Xa, Yb)
        fds.append((lp - lm) / (2 * h))
    fds = np.array(fds)
    den = np.maximum(np.abs(fds), 1e-2 * np.abs(fds).max())
    for sweep, gram_mode, tol in (("f64", "native", 1e-6), ("native", "bf16x3", 1e-3)):
        gX, gY = sk.gram_backward(Xt, Yt, torch.tensor(gk, device="cuda", dtype=torch.float32),
                                  "approx", 8, gK_exp=torch.tensor(gke, device="cuda"),
                                  gram_mode=gram_mode, sweep=sweep)
        gX, gY = gX.double().cpu().numpy(), gY.double().cpu().numpy()
        got = np.array([(gX[sel_a[i]] if s == 0 else gY[sel_b[i]])[t, k] for s, i, t, k in coords])
        rel = np.abs(got - fds) / den
        print(f"{sweep} sweep: max rel vs FD {rel.max():.2e}", flush=True)
        assert np.all(np.isfinite(gX)) and np.all(np.isfinite(gY))
        assert np.all(rel <= tol), (sweep, coords, got, fds)


def test_large_gram_fp64_sampled_block(sk):
    # the accurate mode of the 1024 x 1024, d = 32 Gram: FP64 paths (native
    # FMA-chain Gram on the strips, FP64 sweep) on a sampled 3 x 3 block at
    # full size, against the oracle; kernel values beyond 2^500, exponent
    # output
    import workloads as W
    from oracle import c_oracle as C
    log_banner("1024-point d=32 Gram block, FP64")
    X, Y = W.large_gram(0)
    rng = np.random.default_rng(4)
    ia, ib = np.sort(rng.choice(1024, 3, replace=False)), np.sort(rng.choice(1024, 3, replace=False))
    Xs, Ys = X[ia].astype(np.float64), Y[ib].astype(np.float64)
    K, Ke = sk.gram(torch.tensor(Xs, device="cuda"), torch.tensor(Ys, device="cuda"), "approx", 8,
                    return_exp=True)
    m, e = C.gram(Xs, Ys, C.APPROX, 8)
    err = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
    assert (e + np.log2(np.abs(m))).min() > 500
    assert err.max() < 1e-11, err
