"""sigkernel_gram_static: the Gram forward with the library's static
per-device scratch as workspace (for callers that cannot allocate), called
through the C ABI and compared with sigkernel_gram on its own workspace.

Two calls in a row, the second on a smaller input (the scratch keeps the
first call's contents, which the second must not depend on), then a request
beyond the scratch, rejected before any device work.  The computation per
pair does not depend on the chunking, so the outputs are bit-identical.
"""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return _lib


def run(L, fn, X, Y, params, ws=None):
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    K = torch.full((nx, ny), float("nan"), dtype=X.dtype, device=X.device)
    Ke = torch.full((nx, ny), -7, dtype=torch.int32, device=X.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    args = [vp(X.data_ptr()), nx, lxp, vp(Y.data_ptr()), ny, lyp, d, ctypes.byref(params),
            vp(K.data_ptr()), vp(Ke.data_ptr())]
    if fn == "gram":
        nb = L.lib().sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(params), 0)
        w = torch.empty(nb, dtype=torch.uint8, device=X.device)
        rc = L.lib().sigkernel_gram(*args, vp(w.data_ptr()), nb, st)
    else:
        rc = L.lib().sigkernel_gram_static(*args, st)
    L.check(rc)
    torch.cuda.synchronize()
    return K.cpu().numpy(), Ke.cpu().numpy()


def test_static_scratch_gram_matches_workspace_gram(L):
    rng = np.random.default_rng(2024)
    # first call: 64 x 64 Gram of 257-point paths in R^8 (FP32, interpolation
    # N = 6): 4096 pairs of 1.1 GB of state, so the 256 MiB scratch runs them
    # in several chunks
    log_banner("static scratch: 64x64 Gram FP32 interp 6")
    X = torch.tensor(bm_paths(rng, 64, 256, 8, 0.5 / 16), dtype=torch.float32, device="cuda")
    Y = torch.tensor(bm_paths(rng, 64, 256, 8, 0.5 / 16), dtype=torch.float32, device="cuda")
    p = L.SkParams(L.SK_POLY_INTERP, 6, L.SK_F32, L.SK_ALGO_BATCHED, L.SK_GRAM_NATIVE, 0, 0)
    Ks, Es = run(L, "static", X, Y, p)
    Kw, Ew = run(L, "gram", X, Y, p)
    assert np.isfinite(Ks).all()
    assert np.array_equal(Ks, Kw) and np.array_equal(Es, Ew)
    # second call, smaller: 3 x 5 Gram of ragged FP64 paths (two strips by 37
    # columns), approximation N = 5
    log_banner("static scratch: 3x5 Gram FP64 approx 5")
    X2 = torch.tensor(bm_paths(rng, 3, 100, 3, 0.1), device="cuda")
    Y2 = torch.tensor(bm_paths(rng, 5, 37, 3, 0.1), device="cuda")
    p2 = L.SkParams(L.SK_POLY_APPROX, 5, L.SK_F64, L.SK_ALGO_BATCHED, L.SK_GRAM_NATIVE, 0, 0)
    Ks2, Es2 = run(L, "static", X2, Y2, p2)
    Kw2, Ew2 = run(L, "gram", X2, Y2, p2)
    assert np.array_equal(Ks2, Kw2) and np.array_equal(Es2, Ew2)
    from oracle import c_oracle as C
    m, e = C.gram(X2.cpu().numpy(), Y2.cpu().numpy(), C.APPROX, 5)
    assert np.max(np.abs(np.ldexp(Ks2, Es2 - e) / m - 1)) < 1e-12


def test_static_scratch_rejects_pairs_beyond_it(L):
    log_banner("static scratch: oversize request")
    X = torch.zeros((1, 8193, 8), dtype=torch.float32, device="cuda")
    p = L.SkParams(L.SK_POLY_APPROX, 8, L.SK_F32, L.SK_ALGO_BATCHED, L.SK_GRAM_NATIVE, 0, 0)
    K = torch.full((1, 1), -1.0, device="cuda")
    vp = ctypes.c_void_p
    rc = L.lib().sigkernel_gram_static(vp(X.data_ptr()), 1, 8193, vp(X.data_ptr()), 1, 8193, 8,
                                       ctypes.byref(p), vp(K.data_ptr()), None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.SK_EWORKSPACE and "static scratch" in L.last_error()
    torch.cuda.synchronize()
    assert K.item() == -1.0  # nothing was queued
