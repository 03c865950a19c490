"""Parity over the parameter space: seeded random cases (scheme, order,
dtype, algorithm, Gram mode, batch sizes, ragged lengths from one point to
five strips, dimension 1..40) against the FP64 C oracle, and for the
polynomial schemes the backward of the batched algorithm against the strip
pipeline.

Inputs are Brownian paths with increments of standard deviation
0.3 / sqrt(points), so that every kernel value is O(1) and well conditioned.
Relative tolerances, loose enough for rounding and far below what a wrong
index or term gives (O(1e-3) and more):
* approximation scheme: FP64 1e-11;
* interpolation scheme: FP64 1e-9 + 1e-14 per cell (the literal oracle's
  Vandermonde solve, whose condition number grows to 5e5 at N = 8, adds its
  rounding at every cell);
* finite differences: FP64 1e-11 + 2e-16 per refined cell, FP32 1e-8 per
  refined cell (the recurrence carries every node's rounding to all later
  nodes, so the error grows about linearly with the cell count);
* FP32 polynomial schemes: 1e-4 (state rounding with FP64 corner
  coefficients; 1.5e-4 is the largest seen on the 48 x 64 bench block)."""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, rel_err_exp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NCASES = 96


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def draw_case(i):
    rng = np.random.default_rng(1000 + i)
    scheme = ["approx", "interp", "fd", "fd2"][int(rng.integers(0, 4))]
    dtype = [torch.float64, torch.float32][int(rng.integers(0, 2))]
    order = int(rng.integers(0, 3)) if scheme.startswith("fd") else int(rng.integers(2, 9))
    algo = "batched"
    if not scheme.startswith("fd") and rng.random() < 0.35:
        algo = "pipeline"
    modes = ["native", "mfma"] + (["bf16x3"] if dtype == torch.float32 else [])
    mode = modes[int(rng.integers(0, len(modes)))]
    lens = [1, 2, 3, 64, 65, 66, 129, 200, 321]
    lxp = int(rng.choice(lens)) if rng.random() < 0.5 else int(rng.integers(1, 322))
    lyp = int(rng.choice(lens)) if rng.random() < 0.5 else int(rng.integers(1, 322))
    nx, ny = int(rng.integers(1, 4)), int(rng.integers(1, 4))
    d = int(rng.integers(1, 41))
    X = bm_paths(rng, nx, lxp - 1, d, 0.3 / np.sqrt(lxp))
    Y = bm_paths(rng, ny, lyp - 1, d, 0.3 / np.sqrt(lyp))
    return dict(scheme=scheme, order=order, dtype=dtype, algo=algo, mode=mode, X=X, Y=Y)


@pytest.mark.parametrize("i", range(NCASES))
def test_random_gram_matches_oracle(sk, i):
    from tests.gpu_common import oracle_gram
    c = draw_case(i)
    X, Y, dtype = c["X"], c["Y"], c["dtype"]
    log_banner(f"random case {i}: {c['scheme']} {c['order']} {dtype} {c['algo']} {c['mode']} "
               f"X{X.shape} Y{Y.shape}")
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    Xt = torch.tensor(X, dtype=dtype, device="cuda")
    Yt = torch.tensor(Y, dtype=dtype, device="cuda")
    K, E = sk.gram(Xt, Yt, c["scheme"], c["order"], algo=c["algo"], return_exp=True,
                   gram_mode=c["mode"])
    m, e = oracle_gram(X, Y, c["scheme"], c["order"])
    err = rel_err_exp(K.cpu().double().numpy(), E.cpu().numpy(), m, e)
    fd = c["scheme"].startswith("fd")
    cells = float(max(X.shape[1] - 1, 0) * max(Y.shape[1] - 1, 0)) * (4.0 ** c["order"] if fd else 1.0)
    if dtype == torch.float64:
        tol = (1e-11 + 2e-16 * cells if fd else
               1e-9 + 1e-14 * cells if c["scheme"] == "interp" else 1e-11)
    else:
        tol = max(1e-4, 1e-8 * cells) if fd else 1e-4
    assert err.max() <= tol, (err.max(), tol, c["scheme"], c["order"])
    # one-point paths: k = 1 exactly
    if X.shape[1] == 1 or Y.shape[1] == 1:
        assert np.all(np.ldexp(K.cpu().double().numpy(), E.cpu().numpy()) == 1.0)


@pytest.mark.parametrize("i", range(0, NCASES, 3))
def test_random_backward_batched_matches_pipeline(sk, i):
    c = draw_case(i)
    if c["scheme"].startswith("fd"):
        pytest.skip("the finite-difference schemes are forward only")
    X, Y = c["X"], c["Y"]
    log_banner(f"random backward {i}: {c['scheme']} {c['order']} X{X.shape} Y{Y.shape}")
    Xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
    gK = torch.tensor(np.random.default_rng(i).normal(size=(X.shape[0], Y.shape[0])),
                      dtype=torch.float64, device="cuda")
    gXb, gYb = sk.gram_backward(Xt, Yt, gK, c["scheme"], c["order"])
    gXp, gYp = sk.gram_backward(Xt, Yt, gK, c["scheme"], c["order"], algo="pipeline")
    for a, b in ((gXp, gXb), (gYp, gYb)):
        scale = float(b.abs().max()) if b.numel() else 0.0
        torch.testing.assert_close(a, b, rtol=1e-10, atol=1e-10 * max(scale, 1e-300))


def draw_pairs_case(i):
    rng = np.random.default_rng(5000 + i)
    scheme = ["approx", "interp"][int(rng.integers(0, 2))]
    dtype = [torch.float64, torch.float32][int(rng.integers(0, 2))]
    order = int(rng.integers(2, 9))
    npairs = int(rng.integers(1, 13))
    d = int(rng.integers(1, 25))
    lx = rng.integers(1, 400, size=npairs)
    ly = rng.integers(1, 400, size=npairs)
    xs = [bm_paths(rng, 1, int(n) - 1, d, 0.3 / np.sqrt(n))[0] for n in lx]
    ys = [bm_paths(rng, 1, int(n) - 1, d, 0.3 / np.sqrt(n))[0] for n in ly]
    cfg = [bool(v) for v in rng.integers(0, 2, size=4)]
    return dict(scheme=scheme, order=order, dtype=dtype, xs=xs, ys=ys, cfg=cfg)


@pytest.mark.parametrize("i", range(32))
def test_random_pair_plans_match_oracle(sk, i):
    # ragged pair lists through a backward plan in a random configuration
    # (order, transposition, LDS classes, strip pipeline): forward against
    # the oracle, and the saved-state backward against the plan's
    # recomputing backward
    from oracle import c_oracle as C
    c = draw_pairs_case(i)
    dtype, xs, ys = c["dtype"], c["xs"], c["ys"]
    log_banner(f"random pairs {i}: {c['scheme']} {c['order']} {dtype} cfg {c['cfg']} "
               f"lengths {[len(a) for a in xs]} x {[len(b) for b in ys]}")
    if dtype == torch.float32:
        xs = [a.astype(np.float32).astype(np.float64) for a in xs]
        ys = [b.astype(np.float32).astype(np.float64) for b in ys]
    xl = [torch.tensor(a, dtype=dtype, device="cuda") for a in xs]
    yl = [torch.tensor(b, dtype=dtype, device="cuda") for b in ys]
    Xc, Yc = torch.cat(xl, 0), torch.cat(yl, 0)
    plan = sk.PairsPlan(xl, yl, c["scheme"], c["order"], backward=True)
    plan.configure(*c["cfg"])
    n = len(xs)
    k = torch.empty(n, dtype=dtype, device="cuda")
    ke = torch.empty(n, dtype=torch.int32, device="cuda")
    plan.forward(Xc, Yc, k, ke)
    m, e = C.pairs(xs, ys, C.APPROX if c["scheme"] == "approx" else C.INTERP, c["order"])
    err = rel_err_exp(k.cpu().double().numpy(), ke.cpu().numpy(), m, e)
    cells = np.array([(len(a) - 1) * (len(b) - 1) for a, b in zip(xs, ys)], dtype=np.float64)
    if dtype == torch.float64:
        tol = 1e-9 + 1e-14 * cells if c["scheme"] == "interp" else 1e-11
    else:
        tol = 1e-4
    assert np.all(err <= tol), (err, tol)
    gk = torch.tensor(np.random.default_rng(i).normal(size=n), dtype=dtype, device="cuda")
    gX0, gY0 = torch.empty_like(Xc), torch.empty_like(Yc)
    plan.backward(Xc, Yc, gk, gX0, gY0)
    try:
        k1 = torch.empty_like(k)
        plan.forward_save(Xc, Yc, k1)
    except sk.SigKernelError:
        return  # the saved state needs the backward in one chunk
    gX1, gY1 = torch.empty_like(Xc), torch.empty_like(Yc)
    plan.backward_saved(Xc, Yc, gk, gX1, gY1)
    assert torch.equal(gX1, gX0) and torch.equal(gY1, gY0)
