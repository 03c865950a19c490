"""PyTorch binding of the signature-kernel library.

PyTorch provides device memory and the current HIP stream; every step of
the computation runs in the library's HIP kernels.  Tensors must live on a
GPU ("cuda" device in PyTorch-ROCm) and be float32 or float64.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple, Union

import torch

from . import _lib as L

_SCHEMES = {"fd": L.SK_FD, "fd2": L.SK_FD2, "approx": L.SK_POLY_APPROX,
            "interp": L.SK_POLY_INTERP}
_ALGOS = {"batched": L.SK_ALGO_BATCHED, "plain": L.SK_ALGO_PLAIN, "pipeline": L.SK_ALGO_PIPELINE}
_ALGO_NAMES = {v: k for k, v in _ALGOS.items()}
_GRAMS = {"native": L.SK_GRAM_NATIVE, "bf16x3": L.SK_GRAM_BF16X3, "mfma": L.SK_GRAM_MFMA}


def _params(dtype: torch.dtype, scheme: str, order: int, algo: str, gram_mode: str = "native",
            flags: int = 0, dyadic: int = 0, sweep: str = "native", ckpt: int = 0) -> L.SkParams:
    if dtype == torch.float32:
        dt = L.SK_F32
    elif dtype == torch.float64:
        dt = L.SK_F64
    else:
        raise TypeError(f"unsupported dtype {dtype}")
    if scheme not in _SCHEMES:
        raise ValueError(f"scheme must be one of {sorted(_SCHEMES)}")
    if algo not in _ALGOS:
        raise ValueError(f"algo must be one of {sorted(_ALGOS)}")
    if gram_mode not in _GRAMS:
        raise ValueError(f"gram_mode must be one of {sorted(_GRAMS)}")
    if sweep not in ("native", "f64"):
        raise ValueError('sweep must be "native" or "f64"')
    if sweep == "f64":
        flags |= L.SK_SWEEP_F64
    return L.SkParams(_SCHEMES[scheme], int(order), dt, _ALGOS[algo], _GRAMS[gram_mode], int(flags),
                      int(dyadic), int(ckpt))


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensors must be on a GPU device")
    return t.contiguous()


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.SK_F32
    if t.dtype == torch.float64:
        return L.SK_F64
    raise L.SigKernelError(L.SK_EINVAL, f"dtype {t.dtype}: float32 or float64 expected")


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _i64arr(seq) -> ctypes.Array:
    a = (ctypes.c_int64 * len(seq))(*[int(v) for v in seq])
    return a


def _workspace(nbytes: int, device) -> torch.Tensor:
    if nbytes == 0:
        raise L.SigKernelError(L.SK_EINVAL, L.last_error())
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def device_status(device=None, clear: bool = True) -> int:
    """Status bits (``_lib.SK_STATUS_*``) the kernels raised on ``device`` since
    the last clear: a cell past the interpolation scheme's compiled tail, a
    strip-pipeline wait that gave up.  Waits for the current stream."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    with torch.cuda.device(dev):
        return L.status(torch.cuda.current_stream(dev).cuda_stream, clear)


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------
def gram(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx", order: int = 4,
         algo: str = "batched", return_exp: bool = False, gram_mode: str = "native",
         dyadic: int = 0, sweep: str = "native"):
    """K[a, b] = k(X[a], Y[b]) for paths X (nx, lx_pts, d), Y (ny, ly_pts, d).

    With ``return_exp`` returns (mantissa, exponent) with value
    mantissa * 2**exponent (exponent int32).  ``gram_mode`` "bf16x3"
    computes the cell constants of float32 paths by bf16 split MFMAs, "mfma"
    always by MFMA in the path dtype; "native" (default) uses a d-term FMA
    chain per cell for d <= 16 and MFMA otherwise.
    ``dyadic`` > 0 runs a polynomial scheme on the dyadically refined grid
    (hybrid method).  ``sweep`` "f64" sweeps float32 paths in FP64 (cell
    constants and state; outputs rounded to float32)."""
    X, Y = _dev(X), _dev(Y)
    if X.dim() != 3 or Y.dim() != 3 or X.shape[2] != Y.shape[2] or X.dtype != Y.dtype:
        raise ValueError("X and Y must be (n, points, d) with the same d and dtype")
    p = _params(X.dtype, scheme, order, algo, gram_mode, dyadic=dyadic, sweep=sweep)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    lib = L.lib()
    K = torch.empty((nx, ny), dtype=X.dtype, device=X.device)
    Ke = torch.empty((nx, ny), dtype=torch.int32, device=X.device) if return_exp else None
    if nx * ny == 0:
        return (K, Ke) if return_exp else K
    nb = lib.sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(p), 0)
    ws = _workspace(nb, X.device)
    L.check(lib.sigkernel_gram(_ptr(X), nx, lxp, _ptr(Y), ny, lyp, d, ctypes.byref(p), _ptr(K),
                               _ptr(Ke), _ptr(ws), nb, _stream(X)))
    return (K, Ke) if return_exp else K


def _concat(paths: Union[Sequence[torch.Tensor], Tuple[torch.Tensor, Sequence[int]]]):
    if isinstance(paths, tuple) and len(paths) == 2 and torch.is_tensor(paths[0]):
        cat, off = paths
        off = [int(v) for v in off]
        return _dev(cat), off
    lens = [int(p.shape[0]) for p in paths]
    off = [0]
    for n in lens:
        off.append(off[-1] + n)
    return _dev(torch.cat(list(paths), dim=0)), off


def pairs(xs, ys, scheme: str = "approx", order: int = 4, algo: str = "batched",
          return_exp: bool = False, gram_mode: str = "native", dyadic: int = 0,
          sweep: str = "native"):
    """k[i] = k(xs[i], ys[i]) for lists of (points_i, d) tensors of uneven
    lengths, or (concatenated points, offsets) tuples (``sweep`` as in gram)."""
    Xc, xo = _concat(xs)
    Yc, yo = _concat(ys)
    if len(xo) != len(yo):
        raise ValueError("xs and ys must hold the same number of paths")
    npairs = len(xo) - 1
    d = Xc.shape[1]
    p = _params(Xc.dtype, scheme, order, algo, gram_mode, dyadic=dyadic, sweep=sweep)
    lib = L.lib()
    k = torch.empty(npairs, dtype=Xc.dtype, device=Xc.device)
    ke = torch.empty(npairs, dtype=torch.int32, device=Xc.device) if return_exp else None
    if npairs == 0:
        return (k, ke) if return_exp else k
    xa, ya = _i64arr(xo), _i64arr(yo)
    nb = lib.sigkernel_pairs_workspace(xa, ya, npairs, d, ctypes.byref(p), 0)
    ws = _workspace(nb, Xc.device)
    L.check(lib.sigkernel_pairs(_ptr(Xc), xa, _ptr(Yc), ya, npairs, d, ctypes.byref(p), _ptr(k),
                                _ptr(ke), _ptr(ws), nb, _stream(Xc)))
    return (k, ke) if return_exp else k


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------
def gram_backward(X: torch.Tensor, Y: torch.Tensor, gK: torch.Tensor, scheme: str = "approx",
                  order: int = 4, gK_exp: Optional[torch.Tensor] = None,
                  gram_mode: str = "native", symmetric: bool = False, algo: str = "batched",
                  dyadic: int = 0, sweep: str = "native", ckpt: int = 0):
    """(dL/dX, dL/dY) for L = sum(gK * K) with K = gram(X, Y, scheme, order,
    dyadic=dyadic, sweep=sweep).  ``ckpt`` is the checkpoint stride (0: the
    precision's default; see tune_gram).
    ``symmetric`` (Y is X): returns (dL/dX with both contributions, None).
    ``algo`` "pipeline" runs pairs of several strips on the pipelined
    checkpoint sweep and adjoint (for few, long paths; the call synchronises
    the stream once to upload its job lists)."""
    X, Y = _dev(X), _dev(Y)
    if symmetric:
        Y = X
    if algo not in ("batched", "pipeline"):
        raise ValueError("gram_backward runs the batched algorithm or the strip pipeline")
    gK = _dev(gK.to(X.dtype))
    p = _params(X.dtype, scheme, order, algo, gram_mode, L.SK_SYMMETRIC if symmetric else 0,
                dyadic=dyadic, sweep=sweep, ckpt=ckpt)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    if gK.shape != (nx, ny):
        raise ValueError("gK must have shape (nx, ny)")
    lib = L.lib()
    gX = torch.empty_like(X)
    gY = None if symmetric else torch.empty_like(Y)
    if nx * ny == 0:
        return gX.zero_(), (None if gY is None else gY.zero_())
    ge = _dev(gK_exp.to(torch.int32)) if gK_exp is not None else None
    nb = lib.sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(p), 1)
    ws = _workspace(nb, X.device)
    L.check(lib.sigkernel_backward(L.SK_OP_GRAM, _ptr(X), None, nx, lxp, _ptr(Y), None, ny, lyp,
                                   d, ctypes.byref(p), _ptr(gK), _ptr(ge), _ptr(gX), _ptr(gY),
                                   _ptr(ws), nb, _stream(X)))
    return gX, gY


def pairs_backward(xs, ys, gk: torch.Tensor, scheme: str = "approx", order: int = 4,
                   gk_exp: Optional[torch.Tensor] = None, algo: str = "batched",
                   dyadic: int = 0, sweep: str = "native"):
    """Gradients of sum(gk * pairs(xs, ys)) with respect to the concatenated
    points; returns (gXcat, gYcat, x_offsets, y_offsets).  ``algo`` "batched"
    uses the tuned (or default) plan configuration of this shape; "pipeline"
    runs every pair with several strips on the pipelined checkpoint sweep and
    adjoint."""
    Xc, xo = _concat(xs)
    Yc, yo = _concat(ys)
    npairs = len(xo) - 1
    d = Xc.shape[1]
    if algo not in ("batched", "pipeline"):
        raise ValueError("pairs_backward runs the batched algorithm or the strip pipeline")
    p = _params(Xc.dtype, scheme, order, algo, dyadic=dyadic, sweep=sweep)
    lib = L.lib()
    gk = _dev(gk.to(Xc.dtype))
    gX = torch.empty_like(Xc)
    gY = torch.empty_like(Yc)
    xa, ya = _i64arr(xo), _i64arr(yo)
    ge = _dev(gk_exp.to(torch.int32)) if gk_exp is not None else None
    nb = lib.sigkernel_pairs_workspace(xa, ya, npairs, d, ctypes.byref(p), 1)
    ws = _workspace(nb, Xc.device)
    L.check(lib.sigkernel_backward(L.SK_OP_PAIRS, _ptr(Xc), xa, npairs, 0, _ptr(Yc), ya, 0, 0, d,
                                   ctypes.byref(p), _ptr(gk), _ptr(ge), _ptr(gX), _ptr(gY),
                                   _ptr(ws), nb, _stream(Xc)))
    return gX, gY, xo, yo


def cell_constants(X: torch.Tensor, Y: torch.Tensor, gram_mode: str = "native") -> torch.Tensor:
    """C[a, b, i, j] = <X[a, i+1] - X[a, i], Y[b, j+1] - Y[b, j]> from the
    increment-Gram kernel the path uses for ``gram_mode``."""
    X, Y = _dev(X), _dev(Y)
    p = _params(X.dtype, "approx", 2, "batched", gram_mode)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    lib = L.lib()
    C = torch.empty((nx, ny, lxp - 1, lyp - 1), dtype=X.dtype, device=X.device)
    nb = lib.sigkernel_gram_workspace(nx, lxp, ny, lyp, d, ctypes.byref(p), 0)
    ws = _workspace(nb, X.device)
    L.check(lib.sigkernel_cell_constants(_ptr(X), nx, lxp, _ptr(Y), ny, lyp, d, ctypes.byref(p),
                                         _ptr(C), _ptr(ws), nb, _stream(X)))
    return C


def gram_state_size(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx",
                    order: int = 4, gram_mode: str = "native", algo: str = "batched",
                    dyadic: int = 0, ckpt: int = 0) -> int:
    """Bytes of the backward state kept by gram_save for these shapes."""
    p = _params(X.dtype, scheme, order, algo, gram_mode, dyadic=dyadic, ckpt=ckpt)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    nb = L.lib().sigkernel_gram_state_size(nx, lxp, ny, lyp, d, ctypes.byref(p))
    if nb == 0:
        raise L.SigKernelError(L.SK_EINVAL, L.last_error())
    return int(nb)


def gram_save(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx", order: int = 4,
              return_exp: bool = False, gram_mode: str = "native", algo: str = "batched",
              dyadic: int = 0, ckpt: int = 0):
    """Gram matrix plus the state its backward needs: returns (K, state) or
    (K, K_exp, state).  Pass the state to gram_backward_saved with the same
    ``algo`` ("pipeline": the strip pipeline's checkpoint sweep; the call
    synchronises the stream once to upload its job lists)."""
    X, Y = _dev(X), _dev(Y)
    p = _params(X.dtype, scheme, order, algo, gram_mode, dyadic=dyadic, ckpt=ckpt)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    K = torch.empty((nx, ny), dtype=X.dtype, device=X.device)
    Ke = torch.empty((nx, ny), dtype=torch.int32, device=X.device) if return_exp else None
    state = _workspace(gram_state_size(X, Y, scheme, order, gram_mode, algo, dyadic, ckpt), X.device)
    L.check(L.lib().sigkernel_gram_save(_ptr(X), nx, lxp, _ptr(Y), ny, lyp, d, ctypes.byref(p),
                                        _ptr(K), _ptr(Ke), _ptr(state), state.numel(),
                                        _stream(X)))
    return (K, Ke, state) if return_exp else (K, state)


def gram_backward_saved(X: torch.Tensor, Y: torch.Tensor, gK: torch.Tensor,
                        state: torch.Tensor, scheme: str = "approx", order: int = 4,
                        gK_exp: Optional[torch.Tensor] = None, gram_mode: str = "native",
                        symmetric: bool = False, algo: str = "batched", dyadic: int = 0,
                        ckpt: int = 0):
    """Same result as gram_backward, from the state left by gram_save(X, Y)
    with the same ``algo``, ``dyadic`` and ``ckpt``."""
    X, Y = _dev(X), _dev(Y)
    if symmetric:
        Y = X
    gK = _dev(gK.to(X.dtype))
    p = _params(X.dtype, scheme, order, algo, gram_mode, L.SK_SYMMETRIC if symmetric else 0,
                dyadic=dyadic, ckpt=ckpt)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    gX = torch.empty_like(X)
    gY = None if symmetric else torch.empty_like(Y)
    ge = _dev(gK_exp.to(torch.int32)) if gK_exp is not None else None
    L.check(L.lib().sigkernel_gram_backward_saved(_ptr(X), nx, lxp, _ptr(Y), ny, lyp, d,
                                                  ctypes.byref(p), _ptr(gK), _ptr(ge), _ptr(gX),
                                                  _ptr(gY), _ptr(state), state.numel(),
                                                  _stream(X)))
    return gX, gY


# ---------------------------------------------------------------------------
# plans: repeated pairs calls, capturable in a HIP graph
# ---------------------------------------------------------------------------
class PairsPlan:
    """A plan for pairs calls over fixed path lengths (sigkernel_plan_*).

    ``xs``/``ys`` as for :func:`pairs` (only the lengths, dtype and device are
    taken from them).  The plan owns its workspace; after construction,
    :meth:`forward` and :meth:`backward` only launch kernels on the current
    stream, so they can be captured with ``torch.cuda.graph`` and replayed
    (outputs are written into the tensors passed in)."""

    def __init__(self, xs, ys, scheme: str = "approx", order: int = 4, backward: bool = False,
                 gram_mode: str = "native", dyadic: int = 0):
        Xc, xo = _concat(xs)
        Yc, yo = _concat(ys)
        if len(xo) != len(yo):
            raise ValueError("xs and ys must hold the same number of paths")
        self.npairs, self.d = len(xo) - 1, int(Xc.shape[1])
        self.dtype, self.device = Xc.dtype, Xc.device
        self.x_off, self.y_off = xo, yo
        self._p = _params(Xc.dtype, scheme, order, "batched", gram_mode, dyadic=dyadic)
        self._lib = L.lib()
        h = ctypes.c_void_p(0)
        _load_tune_cache()
        L.check(self._lib.sigkernel_plan_create(_i64arr(xo), _i64arr(yo), self.npairs, self.d,
                                                ctypes.byref(self._p), 1 if backward else 0, 0,
                                                ctypes.byref(h)))
        self._h = h
        nb = self._lib.sigkernel_plan_workspace(self._h)
        self.ws = _workspace(nb, self.device)
        self._upload()

    def _upload(self):
        L.check(self._lib.sigkernel_plan_upload(self._h, _ptr(self.ws), self.ws.numel(),
                                                _stream(self.ws)))

    def tune(self, Xcat: torch.Tensor, Ycat: torch.Tensor) -> float:
        """Time the tuner's configurations on these inputs (forward, and for
        a backward plan forward + backward), keep the fastest, store it in the
        tune cache (and the SK_TUNE_CACHE file); returns its time in ms.  The
        workspace grows to what the largest configuration needs while tuning
        and is then fitted to the choice."""
        _load_tune_cache()
        need = self._lib.sigkernel_plan_tune_workspace(self._h)
        if need > self.ws.numel():
            self.ws = _workspace(need, self.device)
        ms = ctypes.c_double(0.0)
        L.check(self._lib.sigkernel_plan_tune(self._h, _ptr(_dev(Xcat)), _ptr(_dev(Ycat)),
                                              _ptr(self.ws), self.ws.numel(), _stream(self.ws),
                                              ctypes.byref(ms)))
        self._fit_workspace()
        _save_tune_cache()
        return ms.value

    def _fit_workspace(self):
        nb = self._lib.sigkernel_plan_workspace(self._h)
        if nb > self.ws.numel() or nb < 0.75 * self.ws.numel():
            self.ws = _workspace(nb, self.device)
        self._upload()

    def config(self) -> dict:
        c = L.SkPlanCfg()
        L.check(self._lib.sigkernel_plan_get_cfg(self._h, ctypes.byref(c)))
        return {"longest_first": bool(c.longest_first), "transpose": bool(c.transpose),
                "lds_classes": bool(c.lds_classes), "pipeline": c.pipeline_min_strips >= 2,
                "pipeline_min_strips": int(c.pipeline_min_strips), "ckpt": int(c.ckpt),
                "launches": int(c.launches)}

    def configure(self, longest_first: bool, transpose: bool, lds_classes: bool,
                  pipeline: Union[bool, int] = False, ckpt: int = 0):
        """Set the configuration by hand (rebuilds the plan, grows the
        workspace if this configuration needs more, and uploads).  ``pipeline``
        runs pairs with several strips (True or 1: two or more; an int k >= 2:
        k or more) on the strip pipeline: their forward, and for a backward plan
        their checkpoint sweep and adjoint.  ``ckpt``: checkpoint stride of
        the backward (0: the precision's default)."""
        k = int(pipeline)
        if k in (0, 1):  # False / True: no pipeline / pairs of two or more strips
            k = 2 * k
        c = L.SkPlanCfg(int(longest_first), int(transpose), int(lds_classes), k, int(ckpt), 0)
        L.check(self._lib.sigkernel_plan_set_cfg(self._h, ctypes.byref(c), 0))
        self._fit_workspace()

    def forward(self, Xcat: torch.Tensor, Ycat: torch.Tensor, k: torch.Tensor,
                k_exp: Optional[torch.Tensor] = None) -> torch.Tensor:
        L.check(self._lib.sigkernel_plan_forward(self._h, _ptr(Xcat), _ptr(Ycat), _ptr(k),
                                                 _ptr(k_exp), _ptr(self.ws), self.ws.numel(),
                                                 _stream(Xcat)))
        return k

    def backward(self, Xcat: torch.Tensor, Ycat: torch.Tensor, gk: torch.Tensor,
                 gX: torch.Tensor, gY: torch.Tensor, gk_exp: Optional[torch.Tensor] = None):
        L.check(self._lib.sigkernel_plan_backward(self._h, _ptr(Xcat), _ptr(Ycat), _ptr(gk),
                                                  _ptr(gk_exp), _ptr(gX), _ptr(gY),
                                                  _ptr(self.ws), self.ws.numel(),
                                                  _stream(Xcat)))
        return gX, gY

    def forward_save(self, Xcat: torch.Tensor, Ycat: torch.Tensor, k: torch.Tensor,
                     k_exp: Optional[torch.Tensor] = None):
        """Forward that keeps the backward's state in the plan's workspace
        (backward plans whose backward is one chunk); :meth:`backward_saved`
        then starts from it.  No other call of this plan may come between."""
        L.check(self._lib.sigkernel_plan_forward_save(self._h, _ptr(Xcat), _ptr(Ycat), _ptr(k),
                                                      _ptr(k_exp), _ptr(self.ws), self.ws.numel(),
                                                      _stream(Xcat)))
        return k

    def backward_saved(self, Xcat: torch.Tensor, Ycat: torch.Tensor, gk: torch.Tensor,
                       gX: torch.Tensor, gY: torch.Tensor, gk_exp: Optional[torch.Tensor] = None):
        L.check(self._lib.sigkernel_plan_backward_saved(self._h, _ptr(Xcat), _ptr(Ycat), _ptr(gk),
                                                        _ptr(gk_exp), _ptr(gX), _ptr(gY),
                                                        _ptr(self.ws), self.ws.numel(),
                                                        _stream(Xcat)))
        return gX, gY

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.sigkernel_plan_destroy(h)
            self._h = None


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
def _state_budget(device) -> int:
    """Largest backward state kept between forward and backward: half the
    free device memory, capped by SK_STATE_BUDGET_GB (default 96)."""
    import os
    free, _ = torch.cuda.mem_get_info(device)
    cap = float(os.environ.get("SK_STATE_BUDGET_GB", "96")) * (1 << 30)
    return int(min(0.5 * free, cap))


# Gram calls with fewer pairs than this run paths of several 64-row strips
# on the strip pipeline: the batched algorithm gives every pair one wave,
# which leaves most of the GPU's 256 CUs x 4 SIMDs idle (an 8 x 8 Gram of
# 2049-point paths in R^16: backward 173 ms batched, 17 ms pipelined).
PIPELINE_MAX_PAIRS = 2048


def gram_algo(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx") -> str:
    """"pipeline" for polynomial-scheme Gram calls of few pairs whose paths
    span several strips, else "batched"."""
    if scheme in ("fd", "fd2"):
        return "batched"
    strips = (X.shape[1] - 2) // 64 + 1 if X.shape[1] > 1 else 0
    few = X.shape[0] * Y.shape[0] < PIPELINE_MAX_PAIRS
    return "pipeline" if strips >= 2 and Y.shape[1] > 1 and few else "batched"


# ---------------------------------------------------------------------------
# tuning: the library's tune cache, persisted in the file SK_TUNE_CACHE names
# ---------------------------------------------------------------------------
_cache_loaded = False


def _tune_cache_path() -> Optional[str]:
    import os
    return os.environ.get("SK_TUNE_CACHE") or None


def _load_tune_cache() -> None:
    """Merge the SK_TUNE_CACHE file into the library's cache, once."""
    global _cache_loaded
    if _cache_loaded:
        return
    _cache_loaded = True
    path = _tune_cache_path()
    if path:
        L.tune_cache_load(path)


def _save_tune_cache() -> None:
    path = _tune_cache_path()
    if path:
        L.tune_cache_save(path)


def gram_tuned(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx", order: int = 4,
               gram_mode: str = "native", dyadic: int = 0, sweep: str = "native",
               backward: bool = True, symmetric: bool = False) -> Optional[dict]:
    """The tune cache's choice for a Gram call of this shape class:
    {"algo", "ckpt"}, or None when the class has not been tuned."""
    _load_tune_cache()
    p = _params(X.dtype, scheme, order, "batched", gram_mode,
                L.SK_SYMMETRIC if symmetric else 0, dyadic=dyadic, sweep=sweep)
    out, found = L.SkParams(), ctypes.c_int32(0)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    L.check(L.lib().sigkernel_gram_tuned(nx, lxp, ny, lyp, d, ctypes.byref(p), int(backward),
                                         ctypes.byref(out), ctypes.byref(found)))
    if not found.value:
        return None
    return {"algo": _ALGO_NAMES[out.algo], "ckpt": int(out.ckpt)}


def tune_gram(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx", order: int = 4,
              gram_mode: str = "native", dyadic: int = 0, sweep: str = "native",
              backward: bool = True, symmetric: bool = False) -> dict:
    """Time every algorithm (batched, strip pipeline) and checkpoint stride
    on these inputs (forward, or forward + backward through the saved state),
    store the fastest in the tune cache (and the SK_TUNE_CACHE file), and
    return {"algo", "ckpt", "ms"}.  Synchronises the current stream."""
    _load_tune_cache()
    X, Y = _dev(X), _dev(Y)
    if symmetric:
        Y = X
    p = _params(X.dtype, scheme, order, "batched", gram_mode,
                L.SK_SYMMETRIC if symmetric else 0, dyadic=dyadic, sweep=sweep)
    best, ms = L.SkParams(), ctypes.c_double(0.0)
    nx, lxp, d = X.shape
    ny, lyp, _ = Y.shape
    L.check(L.lib().sigkernel_gram_tune(_ptr(X), nx, lxp, _ptr(Y), ny, lyp, d, ctypes.byref(p),
                                        int(backward), _stream(X), ctypes.byref(best),
                                        ctypes.byref(ms)))
    _save_tune_cache()
    return {"algo": _ALGO_NAMES[best.algo], "ckpt": int(best.ckpt), "ms": ms.value}


class SigKernelGram(torch.autograd.Function):
    """Differentiable Gram matrix; the backward runs the library's adjoint
    sweep (exact gradient of the computed scheme).  Batched: when the
    backward state fits the memory budget the forward keeps it (gram_save)
    and the backward starts from it; otherwise the backward recomputes it in
    chunks.  ``algo`` selects the batched algorithm or the strip pipeline for
    both; None takes the tune cache's choice for this shape class (algorithm
    and checkpoint stride, see tune_gram) and else gram_algo's.  ``tune``
    tunes the shape class on these inputs first when the cache has no entry."""

    @staticmethod
    def forward(ctx, X, Y, scheme="approx", order=4, gram_mode="native", algo=None, dyadic=0,
                sweep="native", tune=False):
        ctx.save_for_backward(X, Y)
        ctx.scheme, ctx.order, ctx.gram_mode, ctx.dyadic = scheme, order, gram_mode, dyadic
        ctx.sweep = sweep
        ctx.ckpt = 0
        if algo is None:
            bwd = scheme not in ("fd", "fd2") and (X.requires_grad or Y.requires_grad)
            t = gram_tuned(X, Y, scheme, order, gram_mode, dyadic, sweep, backward=bwd,
                           symmetric=X is Y)
            if t is None and tune and X.shape[0] * Y.shape[0] > 0:
                t = tune_gram(X.detach(), Y.detach(), scheme, order, gram_mode, dyadic, sweep,
                              backward=bwd, symmetric=X is Y)
            if t is not None:
                algo, ctx.ckpt = t["algo"], t["ckpt"]
        ctx.algo = algo or gram_algo(X, Y, scheme)
        # the same tensor on both sides: one gradient with both contributions
        ctx.symmetric = X is Y
        ctx.state = None
        if sweep == "f64":  # no saved state in this mode: the backward recomputes
            return gram(X, Y, scheme, order, algo=ctx.algo, gram_mode=gram_mode, dyadic=dyadic,
                        sweep=sweep)
        if scheme not in ("fd", "fd2") and (X.requires_grad or Y.requires_grad):
            size = gram_state_size(X, Y, scheme, order, gram_mode, ctx.algo, dyadic, ctx.ckpt)
            if size <= _state_budget(X.device):
                K, ctx.state = gram_save(X, Y, scheme, order, gram_mode=gram_mode, algo=ctx.algo,
                                         dyadic=dyadic, ckpt=ctx.ckpt)
                return K
        return gram(X, Y, scheme, order, algo=ctx.algo, gram_mode=gram_mode, dyadic=dyadic)

    @staticmethod
    def backward(ctx, gK):
        X, Y = ctx.saved_tensors
        kw = dict(gram_mode=ctx.gram_mode, symmetric=ctx.symmetric, algo=ctx.algo,
                  dyadic=ctx.dyadic, ckpt=ctx.ckpt)
        if ctx.state is not None:
            gX, gY = gram_backward_saved(X, Y, gK, ctx.state, ctx.scheme, ctx.order, **kw)
            ctx.state = None
        else:
            gX, gY = gram_backward(X, Y, gK, ctx.scheme, ctx.order, sweep=ctx.sweep, **kw)
        return gX, gY, None, None, None, None, None, None, None


def sig_gram(X, Y, scheme: str = "approx", order: int = 4, gram_mode: str = "native",
             algo: Optional[str] = None, dyadic: int = 0, sweep: str = "native",
             tune: bool = False) -> torch.Tensor:
    """Differentiable Gram matrix (SigKernelGram); ``dyadic`` > 0 runs the
    hybrid scheme on the dyadically refined grid; ``sweep`` "f64" sweeps
    float32 paths in FP64; ``algo`` None and ``tune`` as for SigKernelGram."""
    return SigKernelGram.apply(X, Y, scheme, order, gram_mode, algo, dyadic, sweep, tune)


class SigKernelPairs(torch.autograd.Function):
    """Differentiable k[i] = k(A[i], B[i]) for equal-length path batches A, B
    of shape (P, L, d), through a backward plan: a saved-state forward when
    the plan's backward is one chunk (the backward then starts from the
    kept state), otherwise a plain forward and a recomputing backward."""

    @staticmethod
    def forward(ctx, A, B, scheme="approx", order=4, pipeline=False, dyadic=0, sweep="native"):
        P, La, d = A.shape
        Lb = B.shape[1]
        Ac = A.reshape(P * La, d).contiguous()
        Bc = B.reshape(P * Lb, d).contiguous()
        xo = (Ac, [i * La for i in range(P + 1)])
        yo = (Bc, [i * Lb for i in range(P + 1)])
        ctx.shapes, ctx.sweep = (A.shape, B.shape), sweep
        if sweep == "f64":  # one-shot calls (plans do not offer the FP64 sweep)
            ctx.plan, ctx.args = None, (xo[1], yo[1], scheme, order, dyadic,
                                        "pipeline" if pipeline else "batched")
            ctx.save_for_backward(Ac, Bc)
            return pairs(xo, yo, scheme, order, algo=ctx.args[5], dyadic=dyadic, sweep=sweep)
        plan = PairsPlan(xo, yo, scheme, order, backward=True, dyadic=dyadic)
        plan.configure(True, True, True, pipeline)
        k = torch.empty(P, dtype=A.dtype, device=A.device)
        try:
            plan.forward_save(Ac, Bc, k)
            ctx.saved = True
        except L.SigKernelError as e:
            if e.status != L.SK_EWORKSPACE:
                raise
            plan.forward(Ac, Bc, k)
            ctx.saved = False
        ctx.plan = plan
        ctx.save_for_backward(Ac, Bc)
        return k

    @staticmethod
    def backward(ctx, gk):
        Ac, Bc = ctx.saved_tensors
        gk = gk.contiguous().to(Ac.dtype)
        sa, sb = ctx.shapes
        if ctx.sweep == "f64":
            xo, yo, scheme, order, dyadic, algo = ctx.args
            gA, gB, _, _ = pairs_backward((Ac, xo), (Bc, yo), gk, scheme, order, algo=algo,
                                          dyadic=dyadic, sweep="f64")
            return gA.reshape(sa), gB.reshape(sb), None, None, None, None, None
        gA, gB = torch.empty_like(Ac), torch.empty_like(Bc)
        if ctx.saved:
            ctx.plan.backward_saved(Ac, Bc, gk, gA, gB)
        else:
            ctx.plan.backward(Ac, Bc, gk, gA, gB)
        ctx.plan = None
        return gA.reshape(sa), gB.reshape(sb), None, None, None, None, None


def sig_pairs(A, B, scheme: str = "approx", order: int = 4, pipeline: bool = False,
              dyadic: int = 0, sweep: str = "native"):
    """Differentiable k(A[i], B[i]) (SigKernelPairs); ``dyadic`` and ``sweep``
    as for sig_gram."""
    return SigKernelPairs.apply(A, B, scheme, order, pipeline, dyadic, sweep)


class MMD2Pairs(torch.autograd.Function):
    """Unbiased MMD^2 from the kernel values of a [XX pairs a < b | YY pairs
    a < b | XY pairs] list (sigkernel_mmd2_pairs; FP64 accumulation), and its
    derivative with respect to those values (sigkernel_mmd2_pairs_backward)."""

    @staticmethod
    def forward(ctx, k, nx, ny):
        k = k.contiguous()
        out = torch.empty(1, dtype=k.dtype, device=k.device)
        L.check(L.lib().sigkernel_mmd2_pairs(_ptr(k), nx, ny, _dt(k), _ptr(out), _stream(k)))
        ctx.nx, ctx.ny, ctx.shape = nx, ny, k.shape
        return out[0]

    @staticmethod
    def backward(ctx, g):
        g = g.reshape(1).contiguous()
        gk = torch.empty(ctx.shape, dtype=g.dtype, device=g.device)
        L.check(L.lib().sigkernel_mmd2_pairs_backward(_ptr(g), ctx.nx, ctx.ny, _dt(g), _ptr(gk),
                                                      _stream(g)))
        return gk, None, None


def mmd2(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx", order: int = 4,
         gram_mode: str = "native", sweep: str = "native") -> torch.Tensor:
    """Unbiased (U-statistic) squared MMD between path sets X and Y, with the
    within-sample diagonals excluded; differentiable in X and Y.  The kernel
    values of the pairs a < b of each set and of all cross pairs (k is
    symmetric, and the diagonal pairs do not enter) go to the library's
    MMD^2 kernel.  Native Gram arithmetic with equal path lengths computes
    them as one pair list, otherwise they are taken from three Gram
    matrices.  ``sweep`` "f64" sweeps float32 paths in FP64 (the statistic
    is a difference of nearly equal means, so its gradient loses digits the
    FP32 state cannot spare)."""
    n, m = X.shape[0], Y.shape[0]
    ia, ib = torch.triu_indices(n, n, 1, device=X.device)
    ja, jb = torch.triu_indices(m, m, 1, device=Y.device)
    if gram_mode == "native" and X.shape[1] == Y.shape[1] and scheme not in ("fd", "fd2"):
        A = torch.cat([X[ia], Y[ja], X.repeat_interleave(m, 0)], 0)
        B = torch.cat([X[ib], Y[jb], Y.repeat(n, 1, 1)], 0)
        k = sig_pairs(A, B, scheme, order, sweep=sweep)
    else:
        Kxx = sig_gram(X, X, scheme, order, gram_mode, sweep=sweep)
        Kyy = sig_gram(Y, Y, scheme, order, gram_mode, sweep=sweep)
        Kxy = sig_gram(X, Y, scheme, order, gram_mode, sweep=sweep)
        k = torch.cat([Kxx[ia, ib], Kyy[ja, jb], Kxy.reshape(-1)])
    return MMD2Pairs.apply(k, n, m)


def mmd_permutation_test(X: torch.Tensor, Y: torch.Tensor, scheme: str = "approx",
                         order: int = 4, n_perm: int = 1000, seed: int = 0,
                         gram_mode: str = "native"):
    """Two-sample permutation test on the unbiased MMD^2 of path sets X and Y.

    The pooled Gram matrix comes from one library pairs call over the pairs
    a < b (k is symmetric and the unbiased statistic leaves out the
    diagonal, which is set to zero); the statistics of the observed split and
    of n_perm random relabellings (drawn on the host with
    numpy.random.default_rng(seed)) and the p-value are computed by the
    library's kernels.  Returns (statistic, p_value, permutation statistics)."""
    import numpy as np
    X, Y = _dev(X), _dev(Y)
    m, n = X.shape[0], Y.shape[0]
    Z = torch.cat([X, Y], 0)
    T, Lz, d = Z.shape
    ia, ib = torch.triu_indices(T, T, 1, device=Z.device)
    off = [i * Lz for i in range(ia.numel() + 1)]
    kab = pairs((Z[ia].reshape(-1, d), off), (Z[ib].reshape(-1, d), off), scheme, order,
                gram_mode=gram_mode)
    Kzz = torch.zeros(T, T, dtype=Z.dtype, device=Z.device)
    Kzz[ia, ib] = kab
    Kzz[ib, ia] = kab
    rng = np.random.default_rng(seed)
    perms = np.empty((n_perm + 1, m + n), dtype=np.int32)
    perms[0] = np.arange(m + n)
    for q in range(1, n_perm + 1):
        perms[q] = rng.permutation(m + n)
    P = torch.tensor(perms, device=X.device)
    stats = torch.empty(n_perm + 1, dtype=X.dtype, device=X.device)
    pv = torch.empty(1, dtype=torch.float64, device=X.device)
    dt = L.SK_F32 if X.dtype == torch.float32 else L.SK_F64
    L.check(L.lib().sigkernel_mmd_permutation(_ptr(Kzz), m, n, _ptr(P), n_perm + 1, dt,
                                              _ptr(stats), _ptr(pv), _stream(X)))
    return float(stats[0]), float(pv[0]), stats[1:]
