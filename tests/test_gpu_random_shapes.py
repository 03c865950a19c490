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
