"""Host side of the tuner (no GPU): checkpoint-stride validation, the plan
configuration space, and the tune cache's keys and file format.

Without a device the cache names the architecture "none"; the keys built
here follow the format sigkernel_tune_cache_save writes."""
import ctypes
import itertools
import os

import pytest

from paper_2502_08470_amd import _lib as L

vp = ctypes.c_void_p


def P(scheme=1, order=4, dtype=1, algo=0, gram=0, flags=0, dyadic=0, ckpt=0):
    return L.SkParams(scheme, order, dtype, algo, gram, flags, dyadic, ckpt)


def gram_ws(p, backward=1, nx=4, lxp=300, ny=4, lyp=300, d=3):
    return L.lib().sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(p), backward)


@pytest.fixture(autouse=True)
def empty_cache():
    L.tune_cache_clear()
    yield
    L.tune_cache_clear()


def test_checkpoint_stride_validation():
    # FP32 sweeps compile strides 2 and 4, FP64 sweeps 2; 0 is the default
    for ck in (0, 2, 4):
        assert gram_ws(P(ckpt=ck)) > 0, (ck, L.last_error())
    for ck in (0, 2):
        assert gram_ws(P(dtype=L.SK_F64, ckpt=ck)) > 0
        assert gram_ws(P(flags=L.SK_SWEEP_F64, ckpt=ck)) > 0
    for bad, st in ((3, L.SK_EUNSUPPORTED), (8, L.SK_EUNSUPPORTED), (-1, L.SK_EINVAL)):
        assert gram_ws(P(ckpt=bad)) == 0
        assert L.last_error(), bad
    assert gram_ws(P(dtype=L.SK_F64, ckpt=4)) == 0 and "FP64" in L.last_error()
    assert gram_ws(P(flags=L.SK_SWEEP_F64, ckpt=4)) == 0
    # the finite-difference schemes have no checkpoints
    assert gram_ws(P(scheme=L.SK_FD, order=1, ckpt=2), backward=0) == 0
    # statuses through a call that reports them
    lib = L.lib()
    st = lib.sigkernel_gram(vp(1), 2, 10, vp(1), 2, 10, 3, ctypes.byref(P(ckpt=3)), vp(1), None, vp(1),
                            1 << 30, None)
    assert st == L.SK_EUNSUPPORTED
    st = lib.sigkernel_gram(vp(1), 2, 10, vp(1), 2, 10, 3, ctypes.byref(P(ckpt=-2)), vp(1), None, vp(1),
                            1 << 30, None)
    assert st == L.SK_EINVAL


def test_shorter_stride_keeps_more_checkpoints():
    # stride 2 stores twice the checkpoints of stride 4; the forward's
    # workspace does not depend on the stride
    w4, w2 = gram_ws(P(order=6, ckpt=4)), gram_ws(P(order=6, ckpt=2))
    assert w2 > w4 > 0
    assert gram_ws(P(order=6, ckpt=0)) == w4
    assert gram_ws(P(order=6, ckpt=2), backward=0) == gram_ws(P(order=6, ckpt=4), backward=0)


def _plan(lens_x, lens_y, p, backward):
    lib = L.lib()
    n = len(lens_x)
    xo = (ctypes.c_int64 * (n + 1))(0, *itertools.accumulate(lens_x))
    yo = (ctypes.c_int64 * (n + 1))(0, *itertools.accumulate(lens_y))
    h = ctypes.c_void_p(0)
    assert lib.sigkernel_plan_create(xo, yo, n, 3, ctypes.byref(p), backward, 0, ctypes.byref(h)) == L.SK_OK
    return h


def test_plan_configuration_space():
    lib = L.lib()
    lens_x = [300, 40, 700, 65, 10, 1500]
    lens_y = [200, 30, 100, 500, 64, 900]
    h = _plan(lens_x, lens_y, P(order=6), 1)
    try:
        c = L.SkPlanCfg()
        assert lib.sigkernel_plan_get_cfg(h, ctypes.byref(c)) == L.SK_OK
        assert (c.longest_first, c.transpose, c.lds_classes, c.pipeline_min_strips, c.ckpt) == (1, 1, 1, 2, 4)
        base = lib.sigkernel_plan_workspace(h)
        # thresholds: pairs of >= k strips pipelined; fewer pipelined pairs, fewer launch groups or equal
        groups = {}
        for k in (0, 2, 8, 16, 64):
            c2 = L.SkPlanCfg(1, 1, 0, k, 0, 0)
            assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(c2), 0) == L.SK_OK, L.last_error()
            assert lib.sigkernel_plan_get_cfg(h, ctypes.byref(c)) == L.SK_OK
            assert c.pipeline_min_strips == k
            groups[k] = c.launches
        assert groups[0] == 1 and groups[2] == 2 and groups[64] == 1
        # a threshold of one strip is not a threshold
        assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(L.SkPlanCfg(1, 1, 0, 1, 0, 0)), 0) == L.SK_EINVAL
        # the checkpoint stride: 2 needs more workspace, 3 is not compiled
        assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(L.SkPlanCfg(1, 1, 1, 2, 2, 0)), 0) == L.SK_OK
        assert lib.sigkernel_plan_get_cfg(h, ctypes.byref(c)) == L.SK_OK and c.ckpt == 2
        assert lib.sigkernel_plan_workspace(h) > base
        assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(L.SkPlanCfg(1, 1, 1, 2, 3, 0)), 0) == L.SK_EUNSUPPORTED
        # the failed call left the plan as it was
        assert lib.sigkernel_plan_get_cfg(h, ctypes.byref(c)) == L.SK_OK and c.ckpt == 2
        # the tuner's workspace covers every configuration it visits
        need = lib.sigkernel_plan_tune_workspace(h)
        assert need >= lib.sigkernel_plan_workspace(h)
        for o, w, b, k, ck in itertools.product((0, 1), (0, 1), (0, 1), (0, 2, 8), (2, 4)):
            assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(L.SkPlanCfg(o, w, b, k, ck, 0)), 0) == L.SK_OK
            assert lib.sigkernel_plan_workspace(h) <= need, (o, w, b, k, ck)
    finally:
        lib.sigkernel_plan_destroy(h)


def test_fp64_plan_offers_one_stride():
    lib = L.lib()
    h = _plan([300, 700], [200, 500], P(order=6, dtype=L.SK_F64), 1)
    try:
        assert lib.sigkernel_plan_set_cfg(h, ctypes.byref(L.SkPlanCfg(1, 1, 1, 2, 4, 0)), 0) == L.SK_EUNSUPPORTED
        c = L.SkPlanCfg()
        assert lib.sigkernel_plan_get_cfg(h, ctypes.byref(c)) == L.SK_OK and c.ckpt == 2
    finally:
        lib.sigkernel_plan_destroy(h)


def _tuned(nx, lxp, ny, lyp, d, p, backward=1):
    out, found = L.SkParams(), ctypes.c_int32(7)
    assert L.lib().sigkernel_gram_tuned(nx, lxp, ny, lyp, d, ctypes.byref(p), backward, ctypes.byref(out),
                                        ctypes.byref(found)) == L.SK_OK
    return found.value, out


HEADER = "# sigkernel tune cache 1\n"


def test_tune_cache_round_trip_and_shape_classes(tmp_path):
    path = str(tmp_path / "tune.txt")
    # a 128 x 128 Gram of 257-point paths in R^8, interpolation N = 6, FP32, backward
    key = "gram|none|s2|n6|t1|g0|y0|f0|b1|d8|P7,7|x8|y8"
    with open(path, "w") as f:
        f.write(HEADER + f"{key} 1 1 1 2 2 2 12.5\n")
    assert L.tune_cache_load(path) == (1, 0)
    p = P(scheme=L.SK_POLY_INTERP, order=6)
    found, out = _tuned(128, 257, 128, 257, 8, p)
    assert found == 1 and out.algo == L.SK_ALGO_PIPELINE and out.ckpt == 2
    assert (out.scheme, out.order, out.dtype) == (p.scheme, p.order, p.dtype)
    # the same shape class: 65..128 paths, 129..256 segments
    assert _tuned(100, 200, 65, 150, 8, p)[0] == 1
    # other classes, other keys: more paths, longer paths, other d, order, dtype, direction
    for args in ((129, 257, 128, 257, 8, p), (128, 258, 128, 257, 8, p), (128, 257, 128, 257, 9, p),
                 (128, 257, 128, 257, 8, P(scheme=L.SK_POLY_INTERP, order=5)),
                 (128, 257, 128, 257, 8, P(scheme=L.SK_POLY_APPROX, order=6)),
                 (128, 257, 128, 257, 8, P(scheme=L.SK_POLY_INTERP, order=6, dtype=L.SK_F64))):
        found, out = _tuned(*args)
        assert found == 0 and out.algo == args[-1].algo and out.ckpt == args[-1].ckpt, args
    assert _tuned(128, 257, 128, 257, 8, p, backward=0)[0] == 0
    # save and load back: identical text
    path2 = str(tmp_path / "again.txt")
    L.tune_cache_save(path2)
    text = open(path2).read()
    assert text.startswith(HEADER) and key in text
    L.tune_cache_clear()
    assert _tuned(128, 257, 128, 257, 8, p)[0] == 0
    assert L.tune_cache_load(path2) == (1, 0)
    assert _tuned(128, 257, 128, 257, 8, p)[0] == 1
    assert not os.path.exists(path2 + ".tmp")


def test_tune_cache_rejects_what_it_cannot_use(tmp_path):
    # a missing file is no cache yet; another file's text loads nothing;
    # malformed entries are skipped one by one
    assert L.tune_cache_load(str(tmp_path / "missing.txt")) == (0, 0)
    other = tmp_path / "other.txt"
    other.write_text("not a cache\ngram|none|s2|n6|t1|g0|y0|f0|b1|d8|P7,7|x8|y8 1 1 1 2 2 2 1.0\n")
    assert L.tune_cache_load(str(other)) == (0, 1)
    good = "gram|none|s2|n6|t1|g0|y0|f0|b1|d8|P7,7|x8|y8 1 1 1 2 4 0 3.0"
    bad = ["gram|x 1 1 1 2 3 0 1.0",           # stride 3 is not compiled
           "gram|x 1 1 1 1 4 0 1.0",           # a one-strip threshold
           "gram|x 2 1 1 2 4 0 1.0",           # flags are 0 or 1
           "gram|x 1 1 1 2 4 1 1.0",           # the plain algorithm is not a tuned choice
           "gram|x 1 1 1 2 4 0",               # short
           "gram|x 1 1 1 2 4 0 1.0 extra",     # long
           "other|x 1 1 1 2 4 0 1.0",          # unknown kind
           "gram|x 1 1 1 2 4 0 nan",           # not a time
           "x" * 2000]                          # over-long line
    f = tmp_path / "mixed.txt"
    f.write_text(HEADER + "\n".join(bad[:4]) + "\n" + good + "\n" + "\n".join(bad[4:]) + "\n")
    assert L.tune_cache_load(str(f)) == (1, len(bad))
    found, out = _tuned(128, 257, 128, 257, 8, P(scheme=L.SK_POLY_INTERP, order=6))
    assert found == 1 and out.algo == L.SK_ALGO_BATCHED and out.ckpt == 4


def test_stale_entry_falls_back_to_the_callers_parameters(tmp_path):
    # an FP64 entry with stride 4 (hand-edited: FP64 sweeps compile stride 2
    # only) is not applied
    f = tmp_path / "stale.txt"
    f.write_text(HEADER + "gram|none|s2|n6|t0|g0|y0|f0|b1|d8|P7,7|x8|y8 1 1 1 2 4 0 1.0\n")
    assert L.tune_cache_load(str(f)) == (1, 0)
    p = P(scheme=L.SK_POLY_INTERP, order=6, dtype=L.SK_F64)
    found, out = _tuned(128, 257, 128, 257, 8, p)
    assert found == 0 and out.ckpt == 0 and out.algo == L.SK_ALGO_BATCHED
