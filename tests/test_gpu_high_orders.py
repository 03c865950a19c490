"""FP64 polynomial orders 9..12 (the orders the paper's accuracy tables run
to reach the FP64 floor; Appendix B): parity with the FP64 oracle.

* forward, approximation and interpolation schemes, batched, strip pipeline
  and plain kernels, ragged geometries (several strips, a partial strip,
  a one-segment path): 1e-12 relative (interpolation: plus the literal
  oracle's per-cell Vandermonde rounding, 2e-17 per cell);
* FP32 points swept in FP64 reach the same orders;
* backward: gradients against central differences of the oracle (1e-6 of
  the largest entry), batched against pipelined (1e-11);
* FP32 sweeps stop at order 8 (SK_EUNSUPPORTED above).
"""
import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, rel_err_exp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


@pytest.mark.parametrize("scheme,order", [("approx", 9), ("approx", 12), ("interp", 10),
                                          ("interp", 12)])
def test_high_order_forward_fp64(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"FP64 {scheme} N={order}")
    rng = np.random.default_rng(order)
    X = bm_paths(rng, 3, 150, 3, 0.3 / np.sqrt(150))   # three strips, the last partial
    Y = bm_paths(rng, 2, 70, 3, 0.3 / np.sqrt(70))
    kind = C.APPROX if scheme == "approx" else C.INTERP
    m, e = C.gram(X, Y, kind, order)
    cells = 150 * 70
    tol = 1e-12 if scheme == "approx" else 1e-12 + 2e-17 * cells
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    for algo in ("batched", "pipeline", "plain"):
        if algo == "plain":
            K = sk.gram(Xt, Yt, scheme, order, algo=algo).cpu().numpy()
            err = np.abs(K / np.ldexp(m, e) - 1)
        else:
            K, Ke = sk.gram(Xt, Yt, scheme, order, algo=algo, return_exp=True)
            err = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m, e)
        assert err.max() <= tol, (algo, err.max())
    # FP32 points swept in FP64
    X32, Y32 = X.astype(np.float32), Y.astype(np.float32)
    m2, e2 = C.gram(X32.astype(np.float64), Y32.astype(np.float64), kind, order)
    K, Ke = sk.gram(torch.tensor(X32, device="cuda"), torch.tensor(Y32, device="cuda"), scheme, order,
                    return_exp=True, sweep="f64")
    err = rel_err_exp(K.cpu().numpy(), Ke.cpu().numpy(), m2, e2)
    assert err.max() <= 1.2e-7, err.max()  # the FP32 outputs' rounding


def test_high_order_ragged_pairs(sk):
    from oracle import c_oracle as C
    log_banner("FP64 approx N=11 ragged pairs")
    rng = np.random.default_rng(11)
    lens = [(2, 40), (65, 1), (130, 37), (1, 1), (64, 200)]
    xs = [bm_paths(rng, 1, a - 1, 2, 0.05)[0] for a, _ in lens]
    ys = [bm_paths(rng, 1, b - 1, 2, 0.05)[0] for _, b in lens]
    k, ke = sk.pairs([torch.tensor(a, device="cuda") for a in xs],
                     [torch.tensor(b, device="cuda") for b in ys], "approx", 11, return_exp=True)
    m, e = C.pairs(xs, ys, C.APPROX, 11)
    err = rel_err_exp(k.cpu().numpy(), ke.cpu().numpy(), m, e)
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("scheme,order", [("approx", 10), ("interp", 12)])
def test_high_order_backward_fp64(sk, scheme, order):
    from oracle import c_oracle as C
    log_banner(f"FP64 backward {scheme} N={order}")
    rng = np.random.default_rng(100 + order)
    X = bm_paths(rng, 2, 90, 3, 0.5 / np.sqrt(90))   # two strips
    Y = bm_paths(rng, 2, 45, 3, 0.5 / np.sqrt(45))
    gK = rng.normal(size=(2, 2))
    Xt, Yt = torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda")
    gt = torch.tensor(gK, device="cuda")
    gX, gY = sk.gram_backward(Xt, Yt, gt, scheme, order)
    pX, pY = sk.gram_backward(Xt, Yt, gt, scheme, order, algo="pipeline")
    gX, gY, pX, pY = (t.cpu().numpy() for t in (gX, gY, pX, pY))
    scale = max(np.abs(gX).max(), np.abs(gY).max())
    assert max(np.abs(gX - pX).max(), np.abs(gY - pY).max()) <= 1e-11 * scale
    kind = C.APPROX if scheme == "approx" else C.INTERP
    h = 1e-4
    for side, a, t, k in [(0, 0, 3, 1), (0, 1, 90, 2), (1, 1, 20, 0), (1, 0, 44, 2)]:
        P = (X if side == 0 else Y).copy()
        P[a, t, k] += h
        lp = np.sum(gK * np.ldexp(*(C.gram(P, Y, kind, order) if side == 0 else C.gram(X, P, kind, order))))
        P[a, t, k] -= 2 * h
        lm = np.sum(gK * np.ldexp(*(C.gram(P, Y, kind, order) if side == 0 else C.gram(X, P, kind, order))))
        fd = (lp - lm) / (2 * h)
        g = (gX if side == 0 else gY)[a, t, k]
        assert abs(g - fd) <= 1e-6 * scale, (side, a, t, k, g, fd)


def test_fp32_sweeps_stop_at_order_8(sk):
    from paper_2502_08470_amd import _lib
    X = torch.zeros((1, 5, 2), device="cuda")
    with pytest.raises(_lib.SigKernelError) as ei:
        sk.gram(X, X, "approx", 9)
    assert "compiled for orders up to 8" in str(ei.value)
    # the library itself: SK_EUNSUPPORTED
    import ctypes
    p = _lib.SkParams(_lib.SK_POLY_APPROX, 9, _lib.SK_F32, 0, 0, 0, 0)
    assert _lib.lib().sigkernel_gram(ctypes.c_void_p(X.data_ptr()), 1, 5, ctypes.c_void_p(X.data_ptr()),
                                     1, 5, 2, ctypes.byref(p), ctypes.c_void_p(X.data_ptr()), None,
                                     ctypes.c_void_p(X.data_ptr()), 1 << 20, None) == _lib.SK_EUNSUPPORTED
    # FP32 points swept in FP64 reach order 12
    K = sk.gram(X, X, "approx", 12, sweep="f64")
    assert torch.all(K == 1.0)
