"""The strip pipeline's give-up path, driven from the host.

Every wait of the strip pipeline is bounded: a wave that has polled its
predecessor's count `spin_limit` times raises the launch's abort flag, every
waiting wave then leaves, the values (gradients) that could not be completed
are written as NaN and the device status reports SK_STATUS_WAIT_ABORT.  Here
the limit is set to one poll, so that waits give up at once; every kernel
still runs to its end (no wait is left pending and nothing faults).  With
the default limit restored the same calls are complete and correct.
"""
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
    yield P
    _lib.set_spin_limit(0)


def test_pipeline_waits_give_up_cleanly(sk):
    from oracle import c_oracle as C
    from paper_2502_08470_amd import _lib
    log_banner("pipeline give-up path (spin limit 1)")
    rng = np.random.default_rng(91)
    X = bm_paths(rng, 2, 640, 3, 0.03)   # 10 strips per pair
    Y = bm_paths(rng, 2, 300, 3, 0.03)
    Xt = torch.tensor(X, device="cuda")
    Yt = torch.tensor(Y, device="cuda")
    ref = np.ldexp(*C.gram(X, Y, C.APPROX, 4))
    sk.device_status(clear=True)
    try:
        _lib.set_spin_limit(1)
        K = sk.gram(Xt, Yt, "approx", 4, algo="pipeline").cpu().numpy()
        st_fwd = sk.device_status(clear=True)
        gX, gY = sk.gram_backward(Xt, Yt, torch.ones((2, 2), device="cuda", dtype=torch.float64),
                                  "approx", 4, algo="pipeline")
        torch.cuda.synchronize()
        st_bwd = sk.device_status(clear=True)
    finally:
        _lib.set_spin_limit(0)
    # the waits gave up: reported, and the incomplete values are NaN
    assert st_fwd & _lib.SK_STATUS_WAIT_ABORT, st_fwd
    assert np.isnan(K).any()
    ok = ~np.isnan(K)
    assert np.all(rel_err(K[ok], ref[ok]) < 1e-12)
    assert st_bwd & _lib.SK_STATUS_WAIT_ABORT, st_bwd
    assert torch.isnan(gX).any() or torch.isnan(gY).any()
    # default limit: complete and correct, nothing reported
    K2 = sk.gram(Xt, Yt, "approx", 4, algo="pipeline").cpu().numpy()
    gX2, gY2 = sk.gram_backward(Xt, Yt, torch.ones((2, 2), device="cuda", dtype=torch.float64),
                                "approx", 4, algo="pipeline")
    gXb, gYb = sk.gram_backward(Xt, Yt, torch.ones((2, 2), device="cuda", dtype=torch.float64),
                                "approx", 4)
    assert sk.device_status(clear=True) == 0
    assert np.all(rel_err(K2, ref) < 1e-12)
    assert torch.allclose(gX2, gXb, rtol=0, atol=1e-11 * gXb.abs().max().item())
    assert torch.allclose(gY2, gYb, rtol=0, atol=1e-11 * gYb.abs().max().item())
