"""The C-ABI library: exports and host-side argument checking (no GPU).

Every call here fails in host-side validation before any device work, so it
runs on a machine without a GPU."""
import ctypes
import itertools
import os
import re

import pytest

from paper_2502_08470_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "sigkernel.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sigkernel_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def P(scheme=1, order=4, dtype=1, algo=0, gram=0, flags=0, dyadic=0):
    return ctypes.byref(L.SkParams(scheme, order, dtype, algo, gram, flags, dyadic))


def gram(p, nx=2, lxp=10, ny=2, lyp=10, d=3, X=1, Y=1, K=1, ws=1, wsb=1 << 30):
    vp = ctypes.c_void_p
    return L.lib().sigkernel_gram(vp(X), nx, lxp, vp(Y), ny, lyp, d, p, vp(K), None, vp(ws), wsb,
                                  None)


@pytest.mark.parametrize("args,code", [
    (dict(p=P(order=1)), L.SK_EINVAL),
    (dict(p=P(order=9)), L.SK_EUNSUPPORTED),
    (dict(p=P(scheme=0, order=9)), L.SK_EUNSUPPORTED),
    (dict(p=P(scheme=0, order=-1)), L.SK_EINVAL),
    (dict(p=P(scheme=7)), L.SK_EINVAL),
    (dict(p=P(dtype=3)), L.SK_EINVAL),
    (dict(p=P(algo=5)), L.SK_EINVAL),
    (dict(p=P(algo=1, dtype=1)), L.SK_EUNSUPPORTED),
    (dict(p=P(algo=2, scheme=0, order=1)), L.SK_EUNSUPPORTED),  # pipeline: polynomial schemes
    (dict(p=P(algo=3)), L.SK_EINVAL),
    (dict(p=P(), d=0), L.SK_EINVAL),
    (dict(p=P(), lxp=0), L.SK_EINVAL),
    (dict(p=P(), nx=-1), L.SK_EINVAL),
    (dict(p=P(), X=0), L.SK_EINVAL),
    (dict(p=P(), K=0), L.SK_EINVAL),
    (dict(p=P(), ws=0), L.SK_EINVAL),
    (dict(p=P(), wsb=16), L.SK_EWORKSPACE),
    (dict(p=P(algo=2), wsb=16), L.SK_EWORKSPACE),
    (dict(p=None), L.SK_EINVAL),
    (dict(p=P(gram=3)), L.SK_EINVAL),
    (dict(p=P(gram=1, dtype=0)), L.SK_EUNSUPPORTED),
    (dict(p=P(flags=4)), L.SK_EINVAL),
    (dict(p=P(flags=L.SK_SWEEP_F64, dtype=0)), L.SK_EINVAL),       # FP32 paths only
    (dict(p=P(flags=L.SK_SWEEP_F64, gram=1)), L.SK_EUNSUPPORTED),  # FP64 constants, no bf16 split
    (dict(p=P(dyadic=-1)), L.SK_EINVAL),
    (dict(p=P(dyadic=9)), L.SK_EUNSUPPORTED),
    (dict(p=P(scheme=0, order=1, dyadic=1)), L.SK_EINVAL),
])
def test_gram_argument_errors(args, code):
    assert gram(**args) == code
    assert L.last_error() != ""


def test_empty_batch_is_ok_without_device_work():
    assert gram(P(), nx=0) == L.SK_OK


def test_saved_state_plan_calls_need_a_backward_plan():
    lib = L.lib()
    xo = (ctypes.c_int64 * 3)(0, 10, 30)
    yo = (ctypes.c_int64 * 3)(0, 20, 25)
    h = ctypes.c_void_p(0)
    assert lib.sigkernel_plan_create(xo, yo, 2, 3, P(), 0, 0, ctypes.byref(h)) == L.SK_OK
    vp = ctypes.c_void_p
    try:
        assert lib.sigkernel_plan_forward_save(h, vp(1), vp(1), vp(1), None, vp(1), 1 << 20,
                                               None) == L.SK_EINVAL
        assert lib.sigkernel_plan_backward_saved(h, vp(1), vp(1), vp(1), None, vp(1), vp(1), vp(1),
                                                 1 << 20, None) == L.SK_EINVAL
        assert "backward" in L.last_error()
    finally:
        lib.sigkernel_plan_destroy(h)


def test_backward_rejections():
    lib = L.lib()
    vp = ctypes.c_void_p
    def bwd(p, op=0, d=3):
        return lib.sigkernel_backward(op, vp(1), None, 2, 10, vp(1), None, 2, 10, d, p, vp(1),
                                      None, vp(1), vp(1), vp(1), 1 << 30, None)
    assert bwd(P(scheme=0, order=0)) == L.SK_EUNSUPPORTED
    assert bwd(P(scheme=3, order=1)) == L.SK_EUNSUPPORTED  # second-order FD: forward only
    assert bwd(P(algo=1, dtype=0)) == L.SK_EUNSUPPORTED
    assert bwd(P(algo=2, scheme=0, order=0)) == L.SK_EUNSUPPORTED  # pipeline: polynomial schemes
    assert bwd(P(), d=65) == L.SK_EUNSUPPORTED
    assert bwd(P(), op=4) == L.SK_EINVAL
    # SK_SYMMETRIC needs a Gram call whose Y is X (same pointer and shape)
    def bwd_sym(op=0, X=1, Y=1, ny=2):
        return lib.sigkernel_backward(op, vp(X), None, 2, 10, vp(Y), None, ny, 10, 3,
                                      P(flags=L.SK_SYMMETRIC), vp(1), None, vp(1), None, vp(1),
                                      1 << 30, None)
    assert bwd_sym(Y=2) == L.SK_EINVAL
    assert bwd_sym(ny=3) == L.SK_EINVAL
    assert bwd_sym(op=1) == L.SK_EINVAL


def test_pairs_offset_validation():
    lib = L.lib()
    vp = ctypes.c_void_p
    off = lambda v: (ctypes.c_int64 * len(v))(*v)
    ok = off([0, 5, 9])
    bad0 = off([1, 5, 9])
    empty = off([0, 0, 9])
    def pr(xo, yo):
        return lib.sigkernel_pairs(vp(1), xo, vp(1), yo, 2, 3, P(), vp(1), None, vp(1), 1 << 30, None)
    assert pr(bad0, ok) == L.SK_EINVAL
    assert pr(ok, empty) == L.SK_EINVAL
    assert lib.sigkernel_pairs_workspace(ok, ok, 2, 3, P(), 0) > 0
    assert lib.sigkernel_pairs_workspace(ok, bad0, 2, 3, P(), 0) == 0


def test_workspace_sizes():
    lib = L.lib()
    f = lambda nx, b: lib.sigkernel_gram_workspace(nx, 257, nx, 257, 8, P(order=6), b)
    assert 0 < f(1, 0) < f(4, 0) < f(16, 0)
    assert f(16, 1) > f(16, 0)
    assert lib.sigkernel_gram_workspace(4, 1, 4, 1, 8, P(), 0) >= 256
    assert lib.sigkernel_gram_workspace(4, 10, 4, 10, 8, P(order=1), 0) == 0


def test_error_strings():
    lib = L.lib()
    for code in (0, -1, -2, -3, -4):
        assert lib.sigkernel_error_string(code).decode()
    assert lib.sigkernel_error_string(17).decode() == "unknown status"


def test_product_path_has_no_oracle_dependency():
    # the package must not import the oracle
    import paper_2502_08470_amd
    pkg = os.path.dirname(paper_2502_08470_amd.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(root, f)).read()
                assert "from oracle" not in src and "import oracle" not in src, f


def test_plan_host_side_checks():
    lib = L.lib()
    vp = ctypes.c_void_p
    xo = (ctypes.c_int64 * 4)(0, 5, 6, 40)
    yo = (ctypes.c_int64 * 4)(0, 30, 32, 33)
    h = vp(0)
    assert lib.sigkernel_plan_create(xo, yo, 3, 3, P(), 0, 0, None) == L.SK_EINVAL
    assert lib.sigkernel_plan_create(xo, yo, 3, 3, P(order=1), 0, 0, ctypes.byref(h)) == L.SK_EINVAL
    assert lib.sigkernel_plan_create(xo, yo, 3, 3, P(algo=1, dtype=0), 0, 0,
                                     ctypes.byref(h)) == L.SK_EUNSUPPORTED
    assert lib.sigkernel_plan_create(xo, yo, -1, 3, P(), 0, 0, ctypes.byref(h)) == L.SK_EINVAL
    bad = (ctypes.c_int64 * 4)(1, 5, 6, 40)
    assert lib.sigkernel_plan_create(bad, yo, 3, 3, P(), 0, 0, ctypes.byref(h)) == L.SK_EINVAL
    assert lib.sigkernel_plan_create(xo, yo, 3, 3, P(), 0, 0, ctypes.byref(h)) == L.SK_OK
    assert h.value
    need = lib.sigkernel_plan_workspace(h)
    assert need > 0
    # not uploaded: refused before any device work
    assert lib.sigkernel_plan_forward(h, vp(1), vp(1), vp(1), None, vp(1), need, None) == L.SK_EINVAL
    # forward-only plan: no backward
    assert lib.sigkernel_plan_backward(h, vp(1), vp(1), vp(1), None, vp(1), vp(1), vp(1), need,
                                       None) == L.SK_EINVAL
    o, w, b, pp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    n = ctypes.c_int64()
    assert lib.sigkernel_plan_config(h, ctypes.byref(o), ctypes.byref(w), ctypes.byref(b),
                                     ctypes.byref(pp), ctypes.byref(n)) == L.SK_OK
    assert (o.value, w.value, b.value, pp.value) == (1, 1, 1, 1) and n.value >= 1
    assert lib.sigkernel_plan_configure(h, 0, 0, 0, 0, 0) == L.SK_OK
    assert lib.sigkernel_plan_config(h, ctypes.byref(o), ctypes.byref(w), ctypes.byref(b),
                                     ctypes.byref(pp), ctypes.byref(n)) == L.SK_OK
    assert (o.value, w.value, b.value, pp.value, n.value) == (0, 0, 0, 0, 1)
    assert lib.sigkernel_plan_configure(h, 2, 0, 0, 0, 0) == L.SK_EINVAL
    assert lib.sigkernel_plan_configure(h, 0, 0, 0, 2, 0) == L.SK_EINVAL
    # a workspace too small for the descriptors and one pair
    assert lib.sigkernel_plan_configure(h, 1, 1, 1, 1, 64) == L.SK_EWORKSPACE
    lib.sigkernel_plan_destroy(h)
    lib.sigkernel_plan_destroy(None)


def test_mmd_permutation_argument_errors():
    lib = L.lib()
    vp = ctypes.c_void_p
    def call(m=4, n=4, nperm=3, dtype=1, K=1, P=1, S=1):
        return lib.sigkernel_mmd_permutation(vp(K), m, n, vp(P), nperm, dtype, vp(S), None, None)
    assert call(m=1) == L.SK_EINVAL
    assert call(n=1) == L.SK_EINVAL
    assert call(nperm=0) == L.SK_EINVAL
    assert call(dtype=7) == L.SK_EINVAL
    assert call(K=0) == L.SK_EINVAL
    assert call(P=0) == L.SK_EINVAL
    assert call(m=1 << 20, n=8) == L.SK_EUNSUPPORTED


def test_mmd2_pairs_argument_errors():
    lib = L.lib()
    vp = ctypes.c_void_p
    for fn in (lib.sigkernel_mmd2_pairs, lib.sigkernel_mmd2_pairs_backward):
        def call(nx=4, ny=5, dtype=1, a=1, b=1):
            return fn(vp(a), nx, ny, dtype, vp(b), None)
        assert call(nx=1) == L.SK_EINVAL
        assert call(ny=1) == L.SK_EINVAL
        assert call(dtype=7) == L.SK_EINVAL
        assert call(a=0) == L.SK_EINVAL
        assert call(b=0) == L.SK_EINVAL
        assert call(nx=(1 << 24) + 1) == L.SK_EUNSUPPORTED


def test_pipeline_plan_grouping_and_workspace():
    # host-side plan build: pairs of several 64-row strips form one launch
    # group on the strip pipeline, the rest run batched; a backward plan keeps
    # per-strip checkpoints on each strip's local steps, so it needs more
    # workspace than the batched layout
    lib = L.lib()
    lens_x = [300, 40, 700, 65, 10]
    lens_y = [200, 30, 100, 500, 64]
    xo = (ctypes.c_int64 * 6)(0, *itertools.accumulate(lens_x))
    yo = (ctypes.c_int64 * 6)(0, *itertools.accumulate(lens_y))
    o, w, b, pp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    n = ctypes.c_int64()
    sizes = {}
    for backward in (0, 1):
        h = ctypes.c_void_p(0)
        assert lib.sigkernel_plan_create(xo, yo, 5, 3, P(order=6), backward, 0, ctypes.byref(h)) == L.SK_OK
        try:
            for pipe in (0, 1):
                assert lib.sigkernel_plan_configure(h, 1, 1, 0, pipe, 0) == L.SK_OK
                assert lib.sigkernel_plan_config(h, ctypes.byref(o), ctypes.byref(w), ctypes.byref(b),
                                                 ctypes.byref(pp), ctypes.byref(n)) == L.SK_OK
                assert pp.value == pipe
                # one launch group without the pipeline; with it the 3 pairs of
                # several strips (transposed: 300, 700, 500 points) form their own
                assert n.value == (2 if pipe else 1), (backward, pipe, n.value)
                sizes[(backward, pipe)] = lib.sigkernel_plan_workspace(h)
        finally:
            lib.sigkernel_plan_destroy(h)
    assert sizes[(1, 1)] > sizes[(0, 1)] and sizes[(1, 0)] > sizes[(0, 0)]


def test_pipeline_workspace_queries():
    lib = L.lib()
    xo = (ctypes.c_int64 * 3)(0, 300, 340)
    yo = (ctypes.c_int64 * 3)(0, 200, 230)
    # pair lists: the pipeline's backward is a plan
    assert lib.sigkernel_pairs_workspace(xo, yo, 2, 3, P(algo=2), 1) > 0
    assert lib.sigkernel_pairs_workspace(xo, yo, 2, 3, P(algo=2), 0) > 0
    # Gram backward on the pipeline: descriptors of all pairs and two job
    # lists ahead of the chunk scratch; a Gram of one-strip pairs runs batched
    assert lib.sigkernel_gram_workspace(2, 300, 2, 200, 3, P(algo=2), 1) > \
        lib.sigkernel_gram_workspace(2, 300, 2, 200, 3, P(), 1) > 0
    assert lib.sigkernel_gram_workspace(2, 60, 2, 200, 3, P(algo=2), 1) == \
        lib.sigkernel_gram_workspace(2, 60, 2, 200, 3, P(), 1)
    assert lib.sigkernel_gram_workspace(2, 300, 2, 200, 3, P(algo=2), 0) > 0
    # the saved state on the pipeline: one chunk plus descriptors and jobs;
    # one-strip paths keep the batched state
    assert lib.sigkernel_gram_state_size(2, 300, 2, 200, 3, P(algo=2)) > \
        lib.sigkernel_gram_state_size(2, 300, 2, 200, 3, P()) > 0
    assert lib.sigkernel_gram_state_size(2, 60, 2, 200, 3, P(algo=2)) == \
        lib.sigkernel_gram_state_size(2, 60, 2, 200, 3, P())


# ---------------------------------------------------------------------------
# pair geometry: wavefront step counts are checked in 64 bits on the host
# ---------------------------------------------------------------------------
def _steps_error():
    return "wavefront steps" in L.last_error() or "exceed 2^24" in L.last_error()


@pytest.mark.parametrize("lxp,lyp,p", [
    (524289, 524289, dict(scheme=1, order=4)),      # 2^19 segments each: ~4.3e9 steps
    (1500, 1500, dict(scheme=0, order=8)),          # FD, 1499 * 256 refined segments each
    (1500, 1500, dict(scheme=2, order=6, dyadic=8)),  # hybrid scheme, same refined grid
    ((1 << 17) + 1, (1 << 20) + 1, dict(scheme=1, order=4)),  # ~2^31 steps either way round
])
def test_workspace_queries_reject_pairs_beyond_the_step_limit(lxp, lyp, p):
    lib = L.lib()
    for bwd in (0, 1):
        if bwd and p["scheme"] == 0:
            continue
        assert lib.sigkernel_gram_workspace(1, lxp, 1, lyp, 2, P(**p), bwd) == 0
        assert _steps_error(), L.last_error()
        xo = (ctypes.c_int64 * 2)(0, lxp)
        yo = (ctypes.c_int64 * 2)(0, lyp)
        assert lib.sigkernel_pairs_workspace(xo, yo, 1, 2, P(**p), bwd) == 0
        assert _steps_error(), L.last_error()
    if p["scheme"] != 0:
        assert lib.sigkernel_gram_state_size(1, lxp, 1, lyp, 2, P(**p)) == 0
        assert _steps_error(), L.last_error()


def test_backward_checks_the_refined_length_of_the_hybrid_scheme():
    # 70000 points refined 2^8 times exceed 2^24 segments; the backward used
    # to check the unrefined length only
    lib = L.lib()
    vp = ctypes.c_void_p
    rc = lib.sigkernel_backward(L.SK_OP_GRAM, vp(1), None, 1, 70000, vp(1), None, 1, 70000, 2,
                                P(scheme=1, order=4, dyadic=8), vp(1), None, vp(1), vp(1), vp(1),
                                1 << 30, None)
    assert rc == L.SK_EUNSUPPORTED and "2^24" in L.last_error()
    assert lib.sigkernel_gram_state_size(1, 70000, 1, 70000, 2, P(scheme=1, order=4, dyadic=8)) == 0


def test_long_pairs_within_the_step_limit_are_sized():
    lib = L.lib()
    # one 16385-point pair: 256 strips, about 4.2e6 steps
    assert lib.sigkernel_gram_workspace(1, 16385, 1, 16385, 8, P(scheme=1, order=8), 1) > 0
    xo = (ctypes.c_int64 * 3)(0, 16385, 16387)
    yo = (ctypes.c_int64 * 3)(0, 16385, 16386)
    assert lib.sigkernel_pairs_workspace(xo, yo, 2, 8, P(scheme=2, order=6), 0) > 0


def test_status_and_spin_limit_argument_errors():
    lib = L.lib()
    assert lib.sigkernel_status(None, 0, None) == L.SK_EINVAL
    assert lib.sigkernel_set_spin_limit(-1) == L.SK_EINVAL
    assert lib.sigkernel_set_spin_limit(0) == L.SK_OK


def test_sweep_f64_is_refused_where_not_offered():
    lib = L.lib()
    vp = ctypes.c_void_p
    p = P(flags=L.SK_SWEEP_F64)
    assert lib.sigkernel_gram_static(vp(1), 1, 10, vp(1), 1, 10, 3, p, vp(1), None, None) == \
        L.SK_EUNSUPPORTED
    assert lib.sigkernel_gram_state_size(1, 10, 1, 10, 3, p) == 0
    xo = (ctypes.c_int64 * 2)(0, 10)
    plan = ctypes.c_void_p()
    assert lib.sigkernel_plan_create(xo, xo, 1, 3, p, 1, 0, ctypes.byref(plan)) == L.SK_EUNSUPPORTED


def test_sweep_f64_workspace_adds_the_fp64_copies():
    lib = L.lib()
    p32 = P(scheme=1, order=8, dtype=1)
    pf = P(scheme=1, order=8, dtype=1, flags=L.SK_SWEEP_F64)
    p64 = P(scheme=1, order=8, dtype=0)
    for bwd in (0, 1):
        w64 = lib.sigkernel_gram_workspace(3, 100, 5, 70, 4, p64, bwd)
        wf = lib.sigkernel_gram_workspace(3, 100, 5, 70, 4, pf, bwd)
        head = (3 * 100 * 4 * 8 + 255) // 256 * 256 + (5 * 70 * 4 * 8 + 255) // 256 * 256 + 256
        if bwd:
            head += (3 * 100 * 4 * 8 + 255) // 256 * 256 + (5 * 70 * 4 * 8 + 255) // 256 * 256
        assert wf == w64 + head, (bwd, wf, w64, head)
        assert lib.sigkernel_gram_workspace(3, 100, 5, 70, 4, p32, bwd) < wf


def test_order_limits_per_sweep_precision():
    lib = L.lib()
    # FP64 sweeps to 12, FP32 sweeps to 8; FP32 points swept in FP64 to 12
    assert lib.sigkernel_gram_workspace(2, 10, 2, 10, 3, P(order=12, dtype=0), 1) > 0
    assert lib.sigkernel_gram_workspace(2, 10, 2, 10, 3, P(order=13, dtype=0), 0) == 0
    assert lib.sigkernel_gram_workspace(2, 10, 2, 10, 3, P(order=9, dtype=1), 0) == 0
    assert "up to 8" in L.last_error()
    assert lib.sigkernel_gram_workspace(2, 10, 2, 10, 3, P(order=12, dtype=1, flags=L.SK_SWEEP_F64), 1) > 0
