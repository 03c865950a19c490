"""Throughput benchmark of the batched signature-kernel path on one GPU.

One step = forward Gram + backward (adjoint) of a 128 x 128 Gram matrix of
paths in R^8 with 256 Brownian steps (std 0.5/sqrt(256) per coordinate),
polynomial interpolation scheme of order 6, FP32 cell sweep and FP32 MFMA
increment Gram; loss L = sum(K), differentiated with torch.autograd through
the library's SigKernelGram (gradients with respect to both path sets).
Inputs are resident on the GPU before timing.  Reported:

* value: PDE cell updates per second of the whole fwd+bwd step (cells
  counted once per step: 128 * 128 * 256 * 256).
* gram_entries_per_s: Gram entries per second (fwd+bwd).
* mape: mean |K_gpu / K_oracle - 1| on the 16 x 16 block X[0:16] x Y[0:16]
  against the FP64 oracle.
* roofline: dominant kernel, algorithmic FLOPs / its HIP-event time.
* cpu_baseline: the FP64 C oracle on that 16 x 16 block, host cores.
* plain_fp64: the plain single-pair FP64 kernel (one launch per pair,
  forward only) on a sample of pairs of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PDE cell-updates/sec & Gram entries/sec fwd+bwd at MAPE≤1e-6 vs FP64, plain vs batched"
PEAK_FP32_VALU = 157.3e12  # MI355X published FP32 vector peak (FLOP/s)
PEAK_FP64_VALU = 78.6e12
SCHEME, ORDER = "interp", 6
N_PATHS, STEPS, DIM = 128, 256, 8


def fwd_cell_flops(N: int, T: int) -> float:
    """Algorithmic FLOPs of one forward cell (FMA = 2): the Toeplitz part
    (N+1)(N+2)/2, Hankel part N(N+1) and combine (N+1) per edge, two edges,
    i.e. (N+1)(3N+4) FMA, plus 3N multiplies for the powers of c; the
    interpolation tail adds 6T(N+1) FMA (T tail rows: Toeplitz N+1, Hankel N
    and combine 1 per edge, and projection N+1 per edge)."""
    return 2.0 * ((N + 1) * (3 * N + 4) + 6 * T * (N + 1)) + 3 * N


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy MIB MiB device to device once (a plain copy "
                         "kernel of known size, to scale HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    import paper_2502_08470_amd as sk
    from paper_2502_08470_amd import _lib

    _lib.lib()
    dev = torch.device("cuda:0")
    X, Y = W.batched_interp_gram(0, n=N_PATHS, steps=STEPS, d=DIM)
    Xt = torch.tensor(X, device=dev).requires_grad_(True)
    Yt = torch.tensor(Y, device=dev).requires_grad_(True)

    def step():
        Xt.grad = None
        Yt.grad = None
        K = sk.sig_gram(Xt, Yt, SCHEME, ORDER)
        K.sum().backward()
        return K.detach(), Xt.grad, Yt.grad

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        K, gX, gY = step()
    torch.cuda.synchronize()
    kernels = ["gram", "sweep", "sweep_ckpt", "adjoint", "contract", "reduce"]
    _lib.profile_enable(True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        K, gX, gY = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = {k: _lib.profile_read(k) for k in kernels}
    _lib.profile_enable(False)
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    cells = float(N_PATHS * N_PATHS * STEPS * STEPS)
    value = cells / (ms_per_step * 1e-3)
    entries = N_PATHS * N_PATHS / (ms_per_step * 1e-3)

    # roofline of the dominant kernel (largest total event time)
    T_tail = 1  # the interpolation kernels always fold at least one tail row
    fl_fwd = fwd_cell_flops(ORDER, T_tail)
    flops_per_cell = {"sweep": fl_fwd, "sweep_ckpt": fl_fwd,
                      "adjoint": 2.0 * fl_fwd,  # transpose map + dL/dc (recompute not counted)
                      "gram": 2.0 * DIM, "contract": 4.0 * DIM}
    dom = max((k for k in flops_per_cell if ktimes[k][1] > 0), key=lambda k: ktimes[k][0])
    dom_ms, dom_n = ktimes[dom]
    # every step runs each kernel over all cells once (possibly in several
    # launches of part of the pairs): FLOPs per launch = cells * steps / launches
    cells_per_launch = cells * args.steps / dom_n
    achieved = flops_per_cell[dom] * cells_per_launch / (dom_ms / dom_n * 1e-3)
    roofline = {"kernel": dom, "bound": "alu", "achieved": achieved / 1e12,
                "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VALU, "traffic": None,
                "flops_per_cell": flops_per_cell[dom], "launch_ms": dom_ms / dom_n,
                "launches_per_step": dom_n / args.steps,
                "kernel_ms_per_step": {k: ktimes[k][0] / args.steps for k in kernels}}

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "128x128 Gram, paths in R^8, 256 Brownian steps "
                                  "(std 0.5/16), polynomial interpolation N=6, FP32 sweep, "
                                  "FP32 MFMA increment Gram, fwd+bwd (loss sum K)",
                      "pairs": N_PATHS * N_PATHS, "cells_per_pair": STEPS * STEPS},
           "gram_entries_per_s": entries, "roofline": roofline}

    # accuracy and CPU oracle on the 16 x 16 block
    from oracle import c_oracle as C
    Xb = X[:16].astype(np.float64)
    Yb = Y[:16].astype(np.float64)
    threads = C.default_threads()
    print(f"[bench] oracle 16x16 block on {threads} threads", file=sys.stderr, flush=True)
    c0 = time.perf_counter()
    m, e = C.gram(Xb, Yb, C.INTERP, ORDER, threads=threads)
    c1 = time.perf_counter()
    ref = np.ldexp(m, e)
    Kb = K[:16, :16].double().cpu().numpy()
    ape = np.abs(Kb / ref - 1.0)
    out["mape"] = float(ape.mean())
    out["max_ape"] = float(ape.max())
    if not args.no_cpu_baseline:
        ocells = 16 * 16 * STEPS * STEPS
        out["cpu_baseline"] = {"value": ocells / (c1 - c0), "unit": "cell-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "16x16 block X[0:16] x Y[0:16] of the same workload, "
                                         "forward only, FP64 C oracle (literal 0F1 at the "
                                         "Chebyshev extrema + Vandermonde solve)",
                               "seconds": c1 - c0}
    if not args.no_plain:
        npl = 16
        Xd = Xt.detach()[:1].double()
        Yd = Yt.detach()[:npl].double()
        sk.gram(Xd, Yd, SCHEME, ORDER, algo="plain")
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        Kp = sk.gram(Xd, Yd, SCHEME, ORDER, algo="plain")
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        out["plain_fp64"] = {"value": npl * STEPS * STEPS / (p1 - p0), "unit": "cell-updates/s",
                             "sample": f"{npl} pairs X[0] x Y[0:{npl}], forward only, one launch "
                                       "per pair",
                             "max_rel_vs_oracle": float(np.max(np.abs(
                                 Kp.cpu().numpy()[0] / ref[0, :npl] - 1.0)))}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
