"""GPU forward parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances:
* FP64 path: 1e-12 relative per entry.  Both sides evaluate the same
  recursion in IEEE FP64; they differ only in summation order and FMA
  contraction, i.e. a few ulps per cell, accumulated over at most a few
  thousand cells of well-conditioned Brownian inputs.
* FP32 path: MAPE <= 1e-6 (the target of the FP32 sweep) and every entry
  within 2e-5 relative.  The oracle reads the FP32-rounded points.
"""
import numpy as np
import pytest

from oracle import c_oracle as C
from tests.gpu_common import bm_paths, log_banner, oracle_gram, rel_err, rel_err_exp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()  # must load: no fallback
    return P


def dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


# ---------------------------------------------------------------------------
# increment Gram (MFMA) -- exact up to FP rounding of a length-d dot product
# ---------------------------------------------------------------------------
# native, d <= 16: the FMA-chain kernel with a pair's increments in LDS (the
# first two shapes), or one wave per strip with the y increments in an LDS
# ring (the next two, whose increments exceed the LDS budget; the second has a
# strip period above ly), also for 16 < d <= 32 on pairs too long for the
# pair-resident MFMA kernel (the last shape); MFMA otherwise for d > 16.  mfma / bf16x3: the pair-resident
# MFMA kernel, and for the long shapes the strip-band MFMA kernel (FP32) or
# the 64-row block kernel (FP64, whose band tiles exceed the LDS budget)
@pytest.mark.parametrize("dtype,mode", [(torch.float64, "native"), (torch.float32, "native"),
                                        (torch.float64, "mfma"), (torch.float32, "mfma"),
                                        (torch.float32, "bf16x3")])
@pytest.mark.parametrize("shape", [(2, 65, 3, 130, 4), (3, 7, 2, 200, 9), (1, 150, 1, 64, 33),
                                   (1, 1500, 1, 1300, 16), (1, 3000, 2, 50, 13), (1, 900, 2, 800, 24)])
def test_cell_constants_match_increment_products(sk, dtype, mode, shape):
    nx, lxp, ny, lyp, d = shape
    log_banner(f"cell_constants {dtype} {mode} {shape}")
    rng = np.random.default_rng(1)
    X = rng.normal(size=(nx, lxp, d))
    Y = rng.normal(size=(ny, lyp, d))
    Xt, Yt = dev(X, dtype), dev(Y, dtype)
    Cg = sk.cell_constants(Xt, Yt, gram_mode=mode).cpu().numpy()
    Xr, Yr = Xt.cpu().double().numpy(), Yt.cpu().double().numpy()
    dX, dY = np.diff(Xr, axis=1), np.diff(Yr, axis=1)
    want = np.einsum("aik,bjk->abij", dX, dY)
    scale = np.einsum("aik,bjk->abij", np.abs(dX), np.abs(dY))
    # FP32: increments rounded once each (2 * 2^-24), products and a length-d
    # accumulation (d * 2^-24); the bf16 split adds the dropped products
    # mid*lo, lo*mid, lo*lo (< 3 * 2^-24) relative to sum |dx_k dy_k|
    tol = 1e-13 if dtype == torch.float64 else (d + 8) * 2.0 ** -24
    assert np.all(np.abs(Cg - want) <= tol * scale + 1e-300)


def test_bf16x3_gram_matches_oracle_and_fp32(sk):
    # paths in R^32 scaled so that std(c) = 1 (|c| up to about 5)
    import workloads as W
    log_banner("bf16x3 gram")
    X, Y = W.large_gram(0, n=4, steps=200)
    Xt, Yt = dev(X, torch.float32), dev(Y, torch.float32)
    K3, E3 = sk.gram(Xt, Yt, "approx", 8, return_exp=True, gram_mode="bf16x3")
    K1, E1 = sk.gram(Xt, Yt, "approx", 8, return_exp=True)
    m, e = oracle_gram(X.astype(np.float64), Y.astype(np.float64), "approx", 8)
    err3 = rel_err_exp(K3.cpu().numpy(), E3.cpu().numpy(), m, e)
    err1 = rel_err_exp(K1.cpu().numpy(), E1.cpu().numpy(), m, e)
    # each pair's FP32 conditioning floor: the oracle against its FP32 model
    # (increments, cell constants and edge rows >= 2 rounded to FP32)
    mf, ef = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX_F32MODEL, 8)
    floor = np.maximum(rel_err_exp(mf, ef, m, e), 1e-7)
    # both at the floor (measured: ratio median 2.1 / 1.0, max 72 / 61 for
    # the split / FP32 Gram; floors up to 5e-5), and of the same size
    for err in (err3, err1):
        ratio = err / floor
        assert np.median(ratio) <= 5 and ratio.max() <= 150, (np.median(ratio), ratio.max())
    assert err3.mean() < 4 * err1.mean() + 1e-6, (err3.mean(), err1.mean())


# ---------------------------------------------------------------------------
# small FP64 Gram: 8x8, R^3 + time, 64 steps; approximation N=4 and FD lambda=0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ["batched", "plain"])
@pytest.mark.parametrize("scheme,order", [("approx", 4), ("fd", 0), ("interp", 4), ("fd", 2),
                                          ("fd2", 0), ("fd2", 2)])
def test_small_fp64_gram(sk, algo, scheme, order):
    import workloads as W
    log_banner(f"small_fp64_gram {algo} {scheme} {order}")
    X, Y = W.small_fp64_gram(0)
    K = sk.gram(dev(X, torch.float64), dev(Y, torch.float64), scheme, order, algo=algo)
    m, e = oracle_gram(X, Y, scheme, order)
    want = np.ldexp(m, e)
    err = rel_err(K.cpu().numpy(), want)
    assert err.max() < 1e-12, err.max()


# ---------------------------------------------------------------------------
# ragged geometries: several strips, partial strips, short x or y, 1 segment
# ---------------------------------------------------------------------------
GEOMS = [(130, 70), (64, 64), (65, 200), (5, 300), (300, 5), (1, 40), (40, 1), (1, 1), (129, 129)]


@pytest.mark.parametrize("lxp,lyp", GEOMS)
@pytest.mark.parametrize("scheme,order", [("approx", 5), ("interp", 6), ("fd", 1)])
def test_geometries_fp64(sk, lxp, lyp, scheme, order):
    log_banner(f"geometry fp64 {lxp}x{lyp} {scheme} {order}")
    rng = np.random.default_rng(lxp * 1000 + lyp)
    X = bm_paths(rng, 2, lxp - 1, 3, 0.3 / np.sqrt(max(lxp, 2)))
    Y = bm_paths(rng, 3, lyp - 1, 3, 0.3 / np.sqrt(max(lyp, 2)))
    K, Ke = sk.gram(dev(X, torch.float64), dev(Y, torch.float64), scheme, order, return_exp=True)
    m, e = oracle_gram(X, Y, scheme, order)
    err = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
    assert err.max() < 1e-12, err.max()


def test_single_point_paths_give_one(sk):
    X = torch.zeros((2, 1, 3), dtype=torch.float64, device="cuda")
    Y = torch.randn((3, 9, 3), dtype=torch.float64, device="cuda")
    for scheme, order in (("approx", 4), ("interp", 4), ("fd", 0)):
        K = sk.gram(X, Y, scheme, order)
        assert torch.all(K == 1.0)
        K = sk.gram(Y, X, scheme, order)
        assert torch.all(K == 1.0)


# ---------------------------------------------------------------------------
# FP32 sweep
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,order", [("interp", 6), ("approx", 6), ("approx", 8)])
def test_fp32_brownian_mape(sk, scheme, order):
    import workloads as W
    log_banner(f"fp32 brownian {scheme} {order}")
    X, Y = W.batched_interp_gram(0, n=4)
    K = sk.gram(dev(X, torch.float32), dev(Y, torch.float32), scheme, order)
    m, e = oracle_gram(X.astype(np.float64), Y.astype(np.float64), scheme, order)
    err = rel_err(K.cpu().numpy(), np.ldexp(m, e))
    assert err.mean() <= 1e-6, err.mean()
    assert err.max() <= 2e-5, err.max()


def test_fp32_exponent_tracking(sk):
    # values far beyond the FP32 range: cross Gram of high-variance paths
    log_banner("fp32 exponent tracking")
    rng = np.random.default_rng(5)
    X = bm_paths(rng, 2, 150, 8, 1.0).astype(np.float32)
    Y = bm_paths(rng, 2, 90, 8, 1.0).astype(np.float32)
    K, Ke = sk.gram(dev(X, torch.float32), dev(Y, torch.float32), "approx", 8, return_exp=True)
    m, e = oracle_gram(X.astype(np.float64), Y.astype(np.float64), "approx", 8)
    assert (e + np.log2(np.abs(m))).max() > 200  # beyond FP32
    err = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
    # at the pairs' FP32 conditioning floor (oracle vs its FP32 model; here
    # up to 6e-4): measured ratio median 2.1, max 9.9
    mf, ef = C.gram(X.astype(np.float64), Y.astype(np.float64), C.APPROX_F32MODEL, 8)
    ratio = err / np.maximum(rel_err_exp(mf, ef, m, e), 1e-7)
    assert ratio.max() <= 30, ratio


# ---------------------------------------------------------------------------
# uneven pairs in one launch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_pairs_uneven_lengths(sk, dtype, tol):
    from oracle import c_oracle as C
    log_banner(f"pairs {dtype}")
    rng = np.random.default_rng(11)
    lens_x = [33, 1, 140, 70, 2, 65, 257, 12]
    lens_y = [90, 12, 3, 64, 1, 300, 129, 40]
    xs = [bm_paths(rng, 1, n - 1, 4, 0.2 / np.sqrt(n))[0] for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 4, 0.2 / np.sqrt(n))[0] for n in lens_y]
    if dtype == torch.float32:
        xs = [a.astype(np.float32).astype(np.float64) for a in xs]
        ys = [a.astype(np.float32).astype(np.float64) for a in ys]
    k = sk.pairs([dev(a, dtype) for a in xs], [dev(b, dtype) for b in ys], "approx", 6)
    m, e = C.pairs(xs, ys, C.APPROX, 6)
    err = rel_err(k.cpu().numpy(), np.ldexp(m, e))
    assert err.max() < tol, err
    k2 = sk.pairs([dev(a, dtype) for a in xs], [dev(b, dtype) for b in ys], "interp", 5)
    m, e = C.pairs(xs, ys, C.INTERP, 5)
    err = rel_err(k2.cpu().numpy(), np.ldexp(m, e))
    assert err.max() < tol, err


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-8)])
def test_second_order_fd_pairs_and_fp32(sk, dtype, tol):
    # ragged pairs (several strips, a one-point path) through the batched
    # second-order rule, against the oracle.  FP32: the recurrence carries
    # every node's rounding to all later nodes, so the error grows about
    # linearly with the refined cell count (a float32 emulation of the rule
    # itself is 4.3e-5 off on the 140 x 90 pair); the bound is tol per cell.
    from oracle import c_oracle as C
    log_banner(f"fd2 pairs {dtype}")
    rng = np.random.default_rng(71)
    lens_x, lens_y = [70, 1, 140, 9], [33, 20, 90, 200]
    xs = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0] for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0] for n in lens_y]
    if dtype == torch.float32:
        xs = [a.astype(np.float32).astype(np.float64) for a in xs]
        ys = [b.astype(np.float32).astype(np.float64) for b in ys]
    for lam in (0, 1):
        k = sk.pairs([dev(a, dtype) for a in xs], [dev(b, dtype) for b in ys], "fd2", lam)
        m, e = C.pairs(xs, ys, C.FD2, lam)
        err = rel_err(k.cpu().numpy(), np.ldexp(m, e))
        cells = np.array([(a - 1) * (b - 1) for a, b in zip(lens_x, lens_y)], float) * 4 ** lam
        bound = tol * (cells if dtype == torch.float32 else 1.0)
        assert np.all(err <= bound), (lam, err)


# ---------------------------------------------------------------------------
# hybrid: polynomial schemes on the dyadically refined grid
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ["batched", "plain"])
@pytest.mark.parametrize("scheme,order,lam", [("approx", 4, 1), ("interp", 3, 2), ("approx", 2, 3)])
def test_hybrid_refined_grid_fp64(sk, algo, scheme, order, lam):
    from oracle import c_oracle as C
    log_banner(f"hybrid {algo} {scheme} {order} lambda={lam}")
    rng = np.random.default_rng(91)
    X = bm_paths(rng, 3, 40, 3, 0.15)
    Y = bm_paths(rng, 2, 25, 3, 0.15)
    K = sk.gram(dev(X, torch.float64), dev(Y, torch.float64), scheme, order, algo=algo, dyadic=lam)
    kind = C.APPROX if scheme == "approx" else C.INTERP
    m, e = C.gram(X, Y, kind, order, lam=lam)
    err = rel_err(K.cpu().numpy(), np.ldexp(m, e))
    tol = 1e-12 if scheme == "approx" else 1e-12 + 2e-17 * (40 * 25 * 4 ** lam)
    assert err.max() < tol, err


def test_hybrid_pairs_fp32(sk):
    from oracle import c_oracle as C
    log_banner("hybrid pairs fp32")
    rng = np.random.default_rng(92)
    lens_x, lens_y = [70, 1, 140, 9], [33, 20, 90, 200]
    xs = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0].astype(np.float32) for n in lens_x]
    ys = [bm_paths(rng, 1, n - 1, 3, 0.3 / np.sqrt(n))[0].astype(np.float32) for n in lens_y]
    k = sk.pairs([dev(a, torch.float32) for a in xs], [dev(b, torch.float32) for b in ys],
                 "approx", 6, dyadic=1)
    m, e = C.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys],
                   C.APPROX, 6, lam=1)
    err = rel_err(k.cpu().numpy(), np.ldexp(m, e))
    assert err.max() < 2e-5, err
