"""GPU parity of the interpolation scheme at large cell constants.

Definition "Polynomial interpolation numerical scheme" (Section 3.3) maps
every cell with any constant c; the GPU applies Definition "interpooperator"
to the exact edge of Proposition "propinterp" as the untruncated rows of the
approximation map plus a fixed projection of the rows past N, folding as
many rows as the working precision needs.  The larger |c|, the longer that
tail: these tests draw increments like the 1024 x 1024 R^32 workload's
(unit-variance cell constants, scaled so that |c| reaches 5-6), where most
tails run past the rows the adjoints keep per replayed step and the adjoints
take their slow path.

* forward, orders 2, 4, 6, 8: batched, strip pipeline and plain kernels in
  FP64 against the FP64 oracle (literal 0F1 at the nodes + solve, itself
  consistent to about 5e-14 here) to 3e-11; FP32 at its measured floor
  (MAPE 4.9e-5 at N = 2, 8.8e-6, 4.3e-6 and 3.8e-6 at N = 4, 6, 8);
* backward: FP64 gradients against central differences of the oracle, the
  pipelined backward against the batched one, FP32 against FP64;
* a cell past the compiled tail (|c| = 60): its pair is NaN and the device
  status reports it; the other pairs of the call are unaffected.
"""
import numpy as np
import pytest

from tests.gpu_common import log_banner, rel_err_exp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


def large_c_paths(seed, n, pts, d, scale):
    """Brownian paths whose cross cell constants have standard deviation
    about scale (per-coordinate variance scale / sqrt(d))."""
    rng = np.random.default_rng(seed)
    z = np.zeros((n, 1, d))
    std = np.sqrt(scale / np.sqrt(d))
    return np.concatenate([z, np.cumsum(rng.normal(0.0, std, (n, pts - 1, d)), axis=1)], axis=1)


def max_c(X, Y):
    dX, dY = np.diff(X, axis=1), np.diff(Y, axis=1)
    return max(np.abs(a @ b.T).max() for a in dX for b in dY)


@pytest.fixture(scope="module")
def fwd_paths():
    X = large_c_paths(11, 3, 97, 32, 1.2)
    Y = large_c_paths(12, 2, 97, 32, 1.2)
    assert 4.5 < max_c(X, Y) < 8
    return X, Y


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_interp_forward_large_c_fp64(sk, fwd_paths, N):
    from oracle import c_oracle as C
    X, Y = fwd_paths
    log_banner(f"interp large |c| forward FP64 N={N}")
    m_o, e_o = C.gram(X, Y, C.INTERP, N)
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    sk.device_status(clear=True)
    for algo in ("batched", "pipeline", "plain"):
        m, e = sk.gram(Xt, Yt, "interp", N, algo=algo, return_exp=True) if algo != "plain" else \
            (sk.gram(Xt, Yt, "interp", N, algo="plain"), None)
        m = m.cpu().numpy()
        e = np.zeros_like(m, dtype=np.int64) if e is None else e.cpu().numpy()
        err = rel_err_exp(m, e, m_o, e_o)
        print(f"  {algo}: max rel err {err.max():.2e}", flush=True)
        # per-cell rounding at |c| ~ 5 over 9216 cells (measured 1e-11 at N = 2)
        assert err.max() <= 3e-11, (algo, err.max())
    assert sk.device_status() == 0


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_interp_forward_large_c_fp32(sk, fwd_paths, N):
    from oracle import c_oracle as C
    X, Y = fwd_paths
    X32, Y32 = X.astype(np.float32), Y.astype(np.float32)
    log_banner(f"interp large |c| forward FP32 N={N}")
    m_o, e_o = C.gram(X32.astype(np.float64), Y32.astype(np.float64), C.INTERP, N)
    m, e = sk.gram(torch.tensor(X32, device="cuda"), torch.tensor(Y32, device="cuda"), "interp", N,
                   return_exp=True)
    err = rel_err_exp(m.cpu().numpy(), e.cpu().numpy(), m_o, e_o)
    print(f"  FP32: mean {err.mean():.2e} max {err.max():.2e}", flush=True)
    # FP32 floor at |c| ~ 5: rounding of the rows n >= 2 (values up to
    # c^n/n! ~ 10) amplified over the grid; measured on one MI355X, N = 2:
    # mean 4.9e-5, max 2.5e-4 (the 1024-step workload of the same constants,
    # approximation N = 8: mean 2.8e-5)
    assert err.mean() <= 1e-4, err.mean()
    assert err.max() <= 5e-4, err.max()


def fd_grad(X, Y, gK, N, coords, h=1e-4):
    from oracle import c_oracle as C
    out = []
    for (side, a, t, k) in coords:
        P = (X if side == 0 else Y).copy()
        P[a, t, k] += h
        Kp = np.ldexp(*(C.gram(P, Y, C.INTERP, N) if side == 0 else C.gram(X, P, C.INTERP, N)))
        P[a, t, k] -= 2 * h
        Km = np.ldexp(*(C.gram(P, Y, C.INTERP, N) if side == 0 else C.gram(X, P, C.INTERP, N)))
        out.append(np.sum(gK * (Kp - Km)) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("N", [3, 6])
def test_interp_backward_large_c(sk, N):
    X = large_c_paths(21, 2, 41, 4, 1.5)
    Y = large_c_paths(22, 2, 41, 4, 1.5)
    assert max_c(X, Y) > 4
    log_banner(f"interp large |c| backward N={N}")
    from oracle import c_oracle as C
    K = np.ldexp(*C.gram(X, Y, C.INTERP, N))
    gK = np.random.default_rng(N).normal(size=K.shape) / np.abs(K)  # L = sum gK K ~ O(1)
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    gX, gY = sk.gram_backward(Xt, Yt, torch.tensor(gK, device="cuda"), "interp", N)
    gX, gY = gX.cpu().numpy(), gY.cpu().numpy()
    rng = np.random.default_rng(100 + N)
    coords = [(0, 0, 0, 1), (0, 1, 40, 3), (1, 1, 17, 0)] + [
        (int(rng.integers(2)), int(rng.integers(2)), int(rng.integers(41)), int(rng.integers(4)))
        for _ in range(5)]
    fd = fd_grad(X, Y, gK, N, coords)
    got = np.array([(gX if s == 0 else gY)[a, t, k] for (s, a, t, k) in coords])
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    print(f"  max |gpu - fd| / max|g| = {np.abs(got - fd).max() / scale:.2e}", flush=True)
    assert np.all(np.abs(got - fd) <= 1e-6 * scale), (got, fd)
    # FP32 gradients of the same problem (paths as given, rounded)
    gX32, gY32 = sk.gram_backward(Xt.float(), Yt.float(), torch.tensor(gK, device="cuda").float(),
                                  "interp", N)
    d32 = max(np.abs(gX32.cpu().numpy() - gX).max(), np.abs(gY32.cpu().numpy() - gY).max())
    print(f"  FP32 vs FP64 gradient: {d32 / scale:.2e} of max|g|", flush=True)
    assert d32 <= 1e-3 * scale


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_interp_backward_large_c_pipeline_matches_batched(sk, dtype):
    X = large_c_paths(31, 2, 150, 4, 1.5)   # 149 segments: three strips
    Y = large_c_paths(32, 2, 90, 4, 1.5)
    log_banner(f"interp large |c| pipelined backward {dtype}")
    Xt, Yt = torch.tensor(X, device="cuda", dtype=dtype), torch.tensor(Y, device="cuda", dtype=dtype)
    K, Ke = sk.gram(Xt, Yt, "interp", 5, return_exp=True)
    gK = (1.0 / K.double()).to(dtype)
    gKe = -Ke
    gb = sk.gram_backward(Xt, Yt, gK, "interp", 5, gK_exp=gKe)
    gp = sk.gram_backward(Xt, Yt, gK, "interp", 5, gK_exp=gKe, algo="pipeline")
    for a, b in zip(gb, gp):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        tol = (1e-10 if dtype == torch.float64 else 2e-5) * np.abs(a).max()
        assert np.isfinite(a).all() and np.abs(a - b).max() <= tol, np.abs(a - b).max() / np.abs(a).max()


def test_cells_past_the_tail_cap_give_nan_and_status(sk):
    from oracle import c_oracle as C
    log_banner("interp tail cap exceeded")
    rng = np.random.default_rng(7)
    X = np.concatenate([np.zeros((2, 1, 3)), np.cumsum(rng.normal(0, 0.1, (2, 20, 3)), 1)], 1)
    Y = np.concatenate([np.zeros((1, 1, 3)), np.cumsum(rng.normal(0, 0.1, (1, 20, 3)), 1)], 1)
    X[1, 10:] += np.array([8.0, 0.0, 0.0])   # one segment of x1 of length 8
    Y[0, 5:] += np.array([7.5, 0.0, 0.0])    # and one of y of length 7.5: |c| = 60
    for dtype in (torch.float64, torch.float32):
        Xt, Yt = torch.tensor(X, device="cuda", dtype=dtype), torch.tensor(Y, device="cuda", dtype=dtype)
        sk.device_status(clear=True)
        m, e = sk.gram(Xt, Yt, "interp", 4, return_exp=True)
        m = m.double().cpu().numpy()
        from paper_2502_08470_amd import _lib
        st = sk.device_status(clear=True)
        assert st & _lib.SK_STATUS_TAIL_CAP, st
        assert np.isnan(m[1, 0])
        mo, eo = C.gram(X[:1].astype(np.float32 if dtype == torch.float32 else np.float64)
                        .astype(np.float64), Y.astype(np.float32 if dtype == torch.float32 else
                                                      np.float64).astype(np.float64), C.INTERP, 4)
        err = rel_err_exp(m[:1], e.cpu().numpy()[:1], mo, eo)
        # the other pair has |c| up to about 1.3 (one long y segment)
        assert err.max() <= (1e-12 if dtype == torch.float64 else 5e-5), err
        # the backward of the call: the failed pair's gradient is NaN, the
        # other pair's is finite
        gX, gY = sk.gram_backward(Xt, Yt, torch.ones((2, 1), device="cuda", dtype=dtype) *
                                  torch.tensor([[1.0], [0.0]], device="cuda", dtype=dtype), "interp", 4)
        assert torch.isfinite(gX[0]).all()
        assert torch.isnan(gX[1]).any()
        sk.device_status(clear=True)
    assert sk.device_status() == 0
