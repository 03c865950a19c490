"""ctypes binding of ``libsigkernel.so`` (argument marshalling only).

The library is loaded from this package's directory; there is no fallback:
if it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsigkernel.so")

SK_OK, SK_EINVAL, SK_EWORKSPACE, SK_EUNSUPPORTED, SK_EHIP = 0, -1, -2, -3, -4
SK_FD, SK_POLY_APPROX, SK_POLY_INTERP, SK_FD2 = 0, 1, 2, 3
SK_F64, SK_F32 = 0, 1
SK_ALGO_BATCHED, SK_ALGO_PLAIN, SK_ALGO_PIPELINE = 0, 1, 2
SK_OP_GRAM, SK_OP_PAIRS = 0, 1
SK_GRAM_NATIVE, SK_GRAM_BF16X3, SK_GRAM_MFMA = 0, 1, 2
SK_SYMMETRIC = 1
SK_SWEEP_F64 = 2
SK_STATUS_TAIL_CAP, SK_STATUS_WAIT_ABORT = 1, 2
SK_TAIL_TABLE = 20
SK_STATIC_SCRATCH_BYTES = 256 << 20

EXPORTS = (
    "sigkernel_gram_workspace",
    "sigkernel_pairs_workspace",
    "sigkernel_gram",
    "sigkernel_pairs",
    "sigkernel_backward",
    "sigkernel_cell_constants",
    "sigkernel_gram_state_size",
    "sigkernel_gram_save",
    "sigkernel_gram_backward_saved",
    "sigkernel_error_string",
    "sigkernel_last_error",
    "sigkernel_profile_enable",
    "sigkernel_profile_read",
    "sigkernel_plan_create",
    "sigkernel_plan_workspace",
    "sigkernel_plan_upload",
    "sigkernel_plan_forward",
    "sigkernel_plan_backward",
    "sigkernel_plan_forward_save",
    "sigkernel_plan_backward_saved",
    "sigkernel_plan_tune",
    "sigkernel_plan_config",
    "sigkernel_plan_configure",
    "sigkernel_plan_destroy",
    "sigkernel_mmd_permutation",
    "sigkernel_mmd2_pairs",
    "sigkernel_mmd2_pairs_backward",
    "sigkernel_status",
    "sigkernel_set_spin_limit",
    "sigkernel_interp_table",
    "sigkernel_gram_static",
    "sigkernel_plan_get_cfg",
    "sigkernel_plan_set_cfg",
    "sigkernel_plan_tune_workspace",
    "sigkernel_gram_tune",
    "sigkernel_gram_tuned",
    "sigkernel_tune_cache_save",
    "sigkernel_tune_cache_load",
    "sigkernel_tune_cache_clear",
)


class SkParams(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("order", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("gram", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("dyadic", ctypes.c_int32), ("ckpt", ctypes.c_int32)]


class SkPlanCfg(ctypes.Structure):
    _fields_ = [("longest_first", ctypes.c_int32), ("transpose", ctypes.c_int32),
                ("lds_classes", ctypes.c_int32), ("pipeline_min_strips", ctypes.c_int32),
                ("ckpt", ctypes.c_int32), ("launches", ctypes.c_int64)]


class SigKernelError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"sigkernel status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """Load (once) and return the library with its prototypes set."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2502_08470_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    i64p = ctypes.POINTER(ctypes.c_int64)
    pp = ctypes.POINTER(SkParams)
    L.sigkernel_gram_workspace.argtypes = [i64, i64, i64, i64, i64, pp, i32]
    L.sigkernel_gram_workspace.restype = sz
    L.sigkernel_pairs_workspace.argtypes = [i64p, i64p, i64, i64, pp, i32]
    L.sigkernel_pairs_workspace.restype = sz
    L.sigkernel_gram.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, vp, vp, vp, sz, vp]
    L.sigkernel_gram.restype = ctypes.c_int
    L.sigkernel_gram_static.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, vp, vp, vp]
    L.sigkernel_gram_static.restype = ctypes.c_int
    L.sigkernel_pairs.argtypes = [vp, i64p, vp, i64p, i64, i64, pp, vp, vp, vp, sz, vp]
    L.sigkernel_pairs.restype = ctypes.c_int
    L.sigkernel_backward.argtypes = [i32, vp, i64p, i64, i64, vp, i64p, i64, i64, i64, pp,
                                     vp, vp, vp, vp, vp, sz, vp]
    L.sigkernel_backward.restype = ctypes.c_int
    L.sigkernel_cell_constants.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, vp, vp, sz, vp]
    L.sigkernel_cell_constants.restype = ctypes.c_int
    L.sigkernel_gram_state_size.argtypes = [i64, i64, i64, i64, i64, pp]
    L.sigkernel_gram_state_size.restype = sz
    L.sigkernel_gram_save.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, vp, vp, vp, sz, vp]
    L.sigkernel_gram_save.restype = ctypes.c_int
    L.sigkernel_gram_backward_saved.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, vp, vp, vp,
                                                vp, vp, sz, vp]
    L.sigkernel_gram_backward_saved.restype = ctypes.c_int
    L.sigkernel_plan_create.argtypes = [i64p, i64p, i64, i64, pp, i32, sz,
                                        ctypes.POINTER(ctypes.c_void_p)]
    L.sigkernel_plan_create.restype = ctypes.c_int
    L.sigkernel_plan_workspace.argtypes = [vp]
    L.sigkernel_plan_workspace.restype = sz
    L.sigkernel_plan_upload.argtypes = [vp, vp, sz, vp]
    L.sigkernel_plan_upload.restype = ctypes.c_int
    L.sigkernel_plan_forward.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.sigkernel_plan_forward.restype = ctypes.c_int
    L.sigkernel_plan_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sigkernel_plan_backward.restype = ctypes.c_int
    L.sigkernel_plan_forward_save.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.sigkernel_plan_forward_save.restype = ctypes.c_int
    L.sigkernel_plan_backward_saved.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.sigkernel_plan_backward_saved.restype = ctypes.c_int
    L.sigkernel_plan_tune.argtypes = [vp, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_double)]
    L.sigkernel_plan_tune.restype = ctypes.c_int
    L.sigkernel_plan_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i64)]
    L.sigkernel_plan_config.restype = ctypes.c_int
    L.sigkernel_plan_configure.argtypes = [vp, i32, i32, i32, i32, sz]
    L.sigkernel_plan_configure.restype = ctypes.c_int
    cp = ctypes.POINTER(SkPlanCfg)
    L.sigkernel_plan_get_cfg.argtypes = [vp, cp]
    L.sigkernel_plan_get_cfg.restype = ctypes.c_int
    L.sigkernel_plan_set_cfg.argtypes = [vp, cp, sz]
    L.sigkernel_plan_set_cfg.restype = ctypes.c_int
    L.sigkernel_plan_tune_workspace.argtypes = [vp]
    L.sigkernel_plan_tune_workspace.restype = sz
    L.sigkernel_gram_tune.argtypes = [vp, i64, i64, vp, i64, i64, i64, pp, i32, vp, pp,
                                      ctypes.POINTER(ctypes.c_double)]
    L.sigkernel_gram_tune.restype = ctypes.c_int
    L.sigkernel_gram_tuned.argtypes = [i64, i64, i64, i64, i64, pp, i32, pp, ctypes.POINTER(i32)]
    L.sigkernel_gram_tuned.restype = ctypes.c_int
    L.sigkernel_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.sigkernel_tune_cache_save.restype = ctypes.c_int
    L.sigkernel_tune_cache_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.sigkernel_tune_cache_load.restype = ctypes.c_int
    L.sigkernel_tune_cache_clear.argtypes = []
    L.sigkernel_tune_cache_clear.restype = None
    L.sigkernel_plan_destroy.argtypes = [vp]
    L.sigkernel_plan_destroy.restype = None
    L.sigkernel_mmd_permutation.argtypes = [vp, i64, i64, vp, i64, i32, vp, vp, vp]
    L.sigkernel_mmd_permutation.restype = ctypes.c_int
    for name in ("sigkernel_mmd2_pairs", "sigkernel_mmd2_pairs_backward"):
        getattr(L, name).argtypes = [vp, i64, i64, i32, vp, vp]
        getattr(L, name).restype = ctypes.c_int
    L.sigkernel_status.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint32)]
    L.sigkernel_status.restype = ctypes.c_int
    L.sigkernel_set_spin_limit.argtypes = [i32]
    L.sigkernel_set_spin_limit.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.sigkernel_interp_table.argtypes = [i32, i32, dp, dp, dp, ctypes.POINTER(i32)]
    L.sigkernel_interp_table.restype = ctypes.c_int
    L.sigkernel_error_string.argtypes = [ctypes.c_int]
    L.sigkernel_error_string.restype = ctypes.c_char_p
    L.sigkernel_last_error.argtypes = []
    L.sigkernel_last_error.restype = ctypes.c_char_p
    L.sigkernel_profile_enable.argtypes = [i32]
    L.sigkernel_profile_enable.restype = ctypes.c_int
    L.sigkernel_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]
    L.sigkernel_profile_read.restype = ctypes.c_int
    _lib = L
    return L


def check(status: int) -> None:
    if status != SK_OK:
        L = lib()
        detail = L.sigkernel_last_error().decode() or L.sigkernel_error_string(status).decode()
        raise SigKernelError(status, detail)


def last_error() -> str:
    return lib().sigkernel_last_error().decode()


def profile_enable(on: bool) -> None:
    check(lib().sigkernel_profile_enable(1 if on else 0))


def profile_read(name: str):
    """(total milliseconds, launches) of the kernel ``name`` since enable."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    check(lib().sigkernel_profile_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def status(stream: int, clear: bool = True) -> int:
    """Device status bits (SK_STATUS_*) raised since the last clear; waits for ``stream``."""
    f = ctypes.c_uint32(0)
    check(lib().sigkernel_status(ctypes.c_void_p(stream), 1 if clear else 0, ctypes.byref(f)))
    return f.value


def set_spin_limit(polls: int) -> None:
    """Polls of a strip-pipeline wait before it gives up (0: the default)."""
    check(lib().sigkernel_set_spin_limit(int(polls)))


def interp_table(order: int, dtype: int):
    """(rs [N+1][SK_TAIL_TABLE], rmax, cmax, tail cap) of the interpolation tail (host only)."""
    import numpy as np
    rs = np.zeros((order + 1) * SK_TAIL_TABLE)
    rmax = np.zeros(SK_TAIL_TABLE + 1)
    cmax = np.zeros(SK_TAIL_TABLE + 1)
    cap = ctypes.c_int32(0)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().sigkernel_interp_table(int(order), int(dtype), rs.ctypes.data_as(dp),
                                       rmax.ctypes.data_as(dp), cmax.ctypes.data_as(dp),
                                       ctypes.byref(cap)))
    return rs.reshape(order + 1, SK_TAIL_TABLE), rmax, cmax, cap.value


def tune_cache_save(path: str) -> None:
    """Write the process's tune cache to ``path`` (text, replaced atomically)."""
    check(lib().sigkernel_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str):
    """Merge a saved tune cache; returns (entries loaded, entries skipped)."""
    n, k = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().sigkernel_tune_cache_load(os.fsencode(path), ctypes.byref(n), ctypes.byref(k)))
    return n.value, k.value


def tune_cache_clear() -> None:
    lib().sigkernel_tune_cache_clear()
