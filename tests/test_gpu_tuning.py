"""Tuned schedules on the GPU: every checkpoint stride against the oracle's
finite-difference gradient and against the default stride, the Gram tuner's
choice used by autograd, the plan tuner's widened search, and the tune
cache's file across a clear.

Stride parity: the checkpoint stride changes which forward states are
stored and replayed, not the arithmetic of a cell, so the gradients of two
strides agree to rounding order (FP32: 1e-6 relative in the max norm); the
stride-2 gradient also meets the oracle's central differences (FP32 path:
1e-5 relative, as for the default stride)."""
import os

import numpy as np
import pytest

from tests.gpu_common import bm_paths, log_banner, oracle_gram

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_2502_08470_amd as P
    from paper_2502_08470_amd import _lib
    _lib.lib()
    return P


@pytest.fixture(autouse=True)
def empty_cache(monkeypatch):
    from paper_2502_08470_amd import _lib
    monkeypatch.delenv("SK_TUNE_CACHE", raising=False)
    _lib.tune_cache_clear()
    yield
    _lib.tune_cache_clear()


def dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def rel_max(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def fd_grad(X, Y, gK, scheme, order, which, idx, h=1e-4):
    def loss(Xv, Yv):
        m, e = oracle_gram(Xv, Yv, scheme, order)
        return float(np.sum(gK * np.ldexp(m, e)))
    P = (X if which == "x" else Y).copy()
    P[idx] += h
    lp = loss(P, Y) if which == "x" else loss(X, P)
    P[idx] -= 2 * h
    lm = loss(P, Y) if which == "x" else loss(X, P)
    return (lp - lm) / (2 * h)


@pytest.mark.parametrize("algo", ["batched", "pipeline"])
@pytest.mark.parametrize("scheme,order", [("interp", 6), ("approx", 8), ("interp", 3)])
def test_stride_two_matches_default_and_oracle(sk, algo, scheme, order):
    log_banner(f"checkpoint stride 2 {scheme} {order} {algo}")
    rng = np.random.default_rng(91)
    X = bm_paths(rng, 3, 140, 3, 0.4 / np.sqrt(140)).astype(np.float32).astype(np.float64)
    Y = bm_paths(rng, 2, 203, 3, 0.4 / np.sqrt(203)).astype(np.float32).astype(np.float64)
    gK = rng.normal(size=(3, 2))
    out = {}
    for ck in (0, 4, 2):
        gX, gY = sk.gram_backward(dev(X), dev(Y), dev(gK), scheme, order, algo=algo, ckpt=ck)
        out[ck] = (gX.cpu().double().numpy(), gY.cpu().double().numpy())
    # 0 is the FP32 default, 4
    np.testing.assert_array_equal(out[0][0], out[4][0])
    np.testing.assert_array_equal(out[0][1], out[4][1])
    assert rel_max(out[2][0], out[4][0]) < 1e-6
    assert rel_max(out[2][1], out[4][1]) < 1e-6
    # stride 2 against the oracle on sampled coordinates (strip edges, ends)
    scale = max(np.abs(out[2][0]).max(), np.abs(out[2][1]).max())
    for which, idx in [("x", (0, 0, 0)), ("x", (1, 63, 1)), ("x", (2, 64, 2)), ("x", (0, 140, 0)),
                       ("y", (0, 0, 1)), ("y", (1, 128, 2)), ("y", (0, 203, 0)), ("y", (1, 65, 1))]:
        ref = fd_grad(X, Y, gK, scheme, order, which, idx)
        got = (out[2][0] if which == "x" else out[2][1])[idx]
        assert abs(got - ref) <= 1e-5 * scale, (which, idx, got, ref)


def test_stride_two_saved_state_and_autograd(sk):
    # the saved-state forward/backward with stride 2 equals the one-shot backward
    log_banner("checkpoint stride 2 saved state")
    rng = np.random.default_rng(92)
    X = dev(bm_paths(rng, 4, 300, 4, 0.5 / np.sqrt(300)))
    Y = dev(bm_paths(rng, 5, 257, 4, 0.5 / np.sqrt(257)))
    gK = dev(rng.normal(size=(4, 5)))
    for algo in ("batched", "pipeline"):
        K, state = sk.gram_save(X, Y, "interp", 6, algo=algo, ckpt=2)
        gX, gY = sk.gram_backward_saved(X, Y, gK, state, "interp", 6, algo=algo, ckpt=2)
        gX1, gY1 = sk.gram_backward(X, Y, gK, "interp", 6, algo=algo, ckpt=2)
        np.testing.assert_array_equal(gX.cpu().numpy(), gX1.cpu().numpy())
        np.testing.assert_array_equal(gY.cpu().numpy(), gY1.cpu().numpy())
        K0 = sk.gram(X, Y, "interp", 6)
        assert rel_max(K.cpu().numpy(), K0.cpu().numpy()) < 1e-6
    # FP64 offers stride 2 only (its default)
    with pytest.raises(sk.SigKernelError):
        sk.gram_backward(X.double(), Y.double(), gK.double(), "interp", 6, ckpt=4)


def test_gram_tuner_choice_drives_autograd(sk, tmp_path, monkeypatch):
    from paper_2502_08470_amd import _lib
    log_banner("Gram tuner")
    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("SK_TUNE_CACHE", path)
    rng = np.random.default_rng(93)
    X = dev(bm_paths(rng, 24, 256, 8, 0.5 / 16))
    Y = dev(bm_paths(rng, 20, 256, 8, 0.5 / 16))
    assert sk.gram_tuned(X, Y, "interp", 6) is None
    t = sk.tune_gram(X, Y, "interp", 6, backward=True)
    assert t["algo"] in ("batched", "pipeline") and t["ckpt"] in (2, 4) and t["ms"] > 0
    assert sk.gram_tuned(X, Y, "interp", 6) == {"algo": t["algo"], "ckpt": t["ckpt"]}
    assert os.path.exists(path)
    # autograd with algo None takes the tuned choice; same values as that choice by hand
    Xg, Yg = X.clone().requires_grad_(), Y.clone().requires_grad_()
    gK = dev(rng.normal(size=(24, 20)))
    (sk.sig_gram(Xg, Yg, "interp", 6) * gK).sum().backward()
    gX, gY = sk.gram_backward(X, Y, gK, "interp", 6, algo=t["algo"], ckpt=t["ckpt"])
    np.testing.assert_array_equal(Xg.grad.cpu().numpy(), gX.cpu().numpy())
    np.testing.assert_array_equal(Yg.grad.cpu().numpy(), gY.cpu().numpy())
    # the file brings the choice back after a clear
    _lib.tune_cache_clear()
    assert sk.gram_tuned(X, Y, "interp", 6) is None
    assert _lib.tune_cache_load(path) == (1, 0)
    assert sk.gram_tuned(X, Y, "interp", 6)["ckpt"] == t["ckpt"]
    # sig_gram(tune=True) tunes a class with no entry (here: forward only)
    Z = dev(bm_paths(rng, 3, 900, 8, 0.5 / 30))
    assert sk.gram_tuned(Z, Z, "approx", 8, backward=False, symmetric=True) is None
    sk.sig_gram(Z, Z, "approx", 8, tune=True)
    assert sk.gram_tuned(Z, Z, "approx", 8, backward=False, symmetric=True) is not None


def test_plan_tuner_widened_search(sk):
    from oracle import c_oracle as C
    log_banner("plan tuner: thresholds and strides")
    rng = np.random.default_rng(94)
    n, d = 48, 4
    lx = rng.integers(16, 1100, size=n)
    ly = rng.integers(16, 1100, size=n)
    xs = [bm_paths(rng, 1, int(m) - 1, d, 0.4 / np.sqrt(m))[0] for m in lx]
    ys = [bm_paths(rng, 1, int(m) - 1, d, 0.4 / np.sqrt(m))[0] for m in ly]
    Xc = dev(np.concatenate(xs, 0))
    Yc = dev(np.concatenate(ys, 0))
    xl = [dev(a) for a in xs]
    yl = [dev(b) for b in ys]
    plan = sk.PairsPlan(xl, yl, "approx", 8, backward=True)
    k0 = torch.empty(n, device="cuda")
    plan.forward(Xc, Yc, k0)
    gk = dev(rng.normal(size=n))
    gX0, gY0 = torch.empty_like(Xc), torch.empty_like(Yc)
    plan.backward(Xc, Yc, gk, gX0, gY0)
    ms = plan.tune(Xc, Yc)
    cfg = plan.config()
    assert ms > 0 and cfg["ckpt"] in (2, 4) and cfg["pipeline_min_strips"] in (0, 2, 3, 4, 6, 8, 12, 16, 24, 32, 64)
    k1 = torch.empty(n, device="cuda")
    plan.forward(Xc, Yc, k1)
    gX1, gY1 = torch.empty_like(Xc), torch.empty_like(Yc)
    plan.backward(Xc, Yc, gk, gX1, gY1)
    m, e = C.pairs([a.astype(np.float32).astype(np.float64) for a in xs],
                   [b.astype(np.float32).astype(np.float64) for b in ys], C.APPROX, 8)
    ref = np.ldexp(m, e)
    assert np.abs(k1.cpu().double().numpy() / ref - 1).max() < 1e-5
    assert rel_max(k1.cpu().numpy(), k0.cpu().numpy()) < 1e-6
    assert rel_max(gX1.cpu().numpy(), gX0.cpu().numpy()) < 1e-5
    assert rel_max(gY1.cpu().numpy(), gY0.cpu().numpy()) < 1e-5
    # a new plan of the same shape class starts from the tuned configuration
    plan2 = sk.PairsPlan(xl, yl, "approx", 8, backward=True)
    c2 = plan2.config()
    for key in ("longest_first", "transpose", "lds_classes", "pipeline_min_strips", "ckpt"):
        assert c2[key] == cfg[key], key
    # every threshold and stride by hand: same gradients
    for k in (0, 2, 8):
        for ck in (2, 4):
            plan2.configure(True, True, True, k, ck)
            gX2, gY2 = torch.empty_like(Xc), torch.empty_like(Yc)
            plan2.backward(Xc, Yc, gk, gX2, gY2)
            assert rel_max(gX2.cpu().numpy(), gX0.cpu().numpy()) < 1e-5, (k, ck)
            assert rel_max(gY2.cpu().numpy(), gY0.cpu().numpy()) < 1e-5, (k, ck)
