"""Throughput benchmark of the batched signature-kernel path on one GPU.

One step = forward Gram + backward (adjoint) of a 128 x 128 Gram matrix of
paths in R^8 with 256 Brownian steps (std 0.5/sqrt(256) per coordinate),
polynomial interpolation scheme of order 6, FP32 cell sweep and FP32
increment Gram (an 8-term FMA chain per cell, k_gram_direct: at d = 8 the
16x16x4 MFMA tiles are slower; `gram_mfma_ms` times them on the same
input); loss L = sum(K), differentiated with torch.autograd through
the library's SigKernelGram (gradients with respect to both path sets).
Inputs are resident on the GPU before timing.  Reported:

* value: PDE cell updates per second of the whole fwd+bwd step (cells
  counted once per step: 128 * 128 * 256 * 256).
* gram_entries_per_s: Gram entries per second (fwd+bwd).
* mape: mean |K_gpu / K_oracle - 1| on the 16 x 16 block X[0:16] x Y[0:16]
  against the FP64 oracle.
* roofline: dominant kernel, algorithmic FLOPs / its HIP-event time.
* cpu_baseline: the FP64 C oracle on the 48 x 64 block X[0:48] x Y[0:64]
  (about 10-20 s on 16 host cores), all host threads OMP_NUM_THREADS allows;
  its `single_core` entry times one thread on the 4 x 8 block, and `host`
  names the CPU.
* roofline.traffic: HBM bytes per launch of the dominant kernel from the
  committed counter summary (FETCH_SIZE and WRITE_SIZE runs, scaled by the
  same counters read for a plain 1 GiB device copy), reported only when the
  kernel sources hash to the value recorded with the counters, else null.
* plain_fp64: the 8 x 8 FP64 Gram of R^3 paths with a time channel (64
  steps, approximation N = 4, and the finite-difference baseline): the plain
  single-pair kernel (one launch per pair, forward only) next to the batched
  kernels (forward, and forward + backward), with the largest relative
  departure from the oracle.
* large_gram_block: 16 rows x 1024 columns of the 1024 x 1024 R^32 Gram
  (1024 steps, approximation N = 8, kernels near 2^1200), forward + backward
  through log K, with the FP32 sweep (bf16 3-way split Gram) and with the
  FP32 points swept in FP64; MAPE of each on 8 sampled pairs of the block.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --pmc-summary FETCH.csv WRITE.csv OUT.json   (no GPU)
       python bench.py --accuracy-study   (synthetic re-run of the paper's accuracy tables)
       python bench.py --long-pair 16384  (strip pipeline on one long pair)
       python bench.py --long-gram        (4x4 Gram of long paths, pipeline vs batched)
       python bench.py --workloads        (time of every named workload)
"""
from __future__ import annotations

import argparse
import glob
import hashlib
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
CPU_BLOCK = (48, 64)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_batched_interp_gram_128x128.json")
CALIBRATE_MIB = 1024
# bench kernel label -> names of the kernels behind it (the adjoint has an
# entry point that asks for two waves per SIMD, k_adjoint_w2)
KERNEL_SYMBOL = {"gram": ("k_gram_direct",), "sweep": ("k_sweep",), "sweep_ckpt": ("k_sweep",),
                 "adjoint": ("k_adjoint", "k_adjoint_w2"), "sweep_pipe": ("k_sweep_pipe",),
                 "sweep_ckpt_pipe": ("k_sweep_pipe",),
                 "adjoint_pipe": ("k_adjoint_pipe",),
                 "contract": ("k_contract",),
                 "reduce": ("k_reduce_gram_x", "k_reduce_gram_y", "k_reduce_pairs")}


def template_args(symbol: str):
    """Template arguments of a kernel symbol 'void k_x<a, b, ...>(...)'."""
    if "<" not in symbol:
        return []
    inner = symbol.split("<", 1)[1].split(">(", 1)[0]
    return [a.strip() for a in inner.split(",")]


def symbol_matches(label: str, symbol: str, stride: int) -> bool:
    """Whether `symbol` is the kernel behind the bench label `label` when the
    backward runs with checkpoint stride `stride` (k_sweep<R, N, TMAX, CKPT,
    S, GX>, k_sweep_pipe<R, N, TMAX, CKPT, S>, k_adjoint<R, N, TMAX, S, GX>,
    k_adjoint_pipe<R, N, TMAX, S>)."""
    if not symbol.startswith("void ") or symbol[5:].split("<", 1)[0] not in KERNEL_SYMBOL[label]:
        return False
    a = template_args(symbol)
    if label in ("sweep", "sweep_pipe"):
        return len(a) > 3 and a[3] == "false"
    if label in ("sweep_ckpt", "sweep_ckpt_pipe"):
        return len(a) > 4 and a[3] == "true" and a[4] == str(stride)
    if label in ("adjoint", "adjoint_pipe"):
        return len(a) > 3 and a[3] == str(stride)
    return True


def kernel_source_hash() -> str:
    """sha256 over the HIP/C++ sources of the library (sorted by name)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2502_08470_amd", "csrc", "*"))):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def pmc_summary(fetch_csv: str, write_csv: str, out_json: str) -> int:
    """Per-kernel HBM bytes per dispatch from two rocprofv3 --pmc runs of
    `bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-plain --no-tune --calibrate-copy 1024`.
    Each counter is scaled by bytes / counter-KiB of the largest device copy
    dispatch (the 1 GiB calibration copy: 1 GiB read, 1 GiB written)."""
    import csv
    from collections import defaultdict

    def load(path, ctr):
        d = defaultdict(list)
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == ctr:
                    d[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return d
    def rel(path):
        return os.path.relpath(os.path.abspath(path), ROOT)

    f, w = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    cal = float(CALIBRATE_MIB << 20)
    copy_f = max(v for k, vs in f.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in w.items() if "copyBuffer" in k for v in vs)
    fscale, wscale = cal / copy_f, cal / copy_w  # bytes per counter unit
    kernels = {}
    for k in sorted(set(f) & set(w)):
        if not k.startswith("void k_"):
            continue
        fb = sum(f[k]) / len(f[k]) * fscale
        wb = sum(w[k]) / len(w[k]) * wscale
        kernels[k] = {"dispatches": len(f[k]), "fetch_bytes": fb, "write_bytes": wb,
                      "bytes": fb + wb}
    out = {"source_hash": kernel_source_hash(),
           "calibration": {"copy_bytes": cal, "fetch_counter": copy_f, "write_counter": copy_w,
                           "fetch_bytes_per_unit": fscale, "write_bytes_per_unit": wscale},
           # the commands, with the output folders of the two runs as given
           "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {rel(os.path.dirname(fetch_csv))} -o fetch -f csv -- "
                        "python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-plain --no-tune "
                        f"--calibrate-copy {CALIBRATE_MIB}",
                        f"rocprofv3 --pmc WRITE_SIZE -d {rel(os.path.dirname(write_csv))} -o write -f csv -- "
                        "python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-plain --no-tune "
                        f"--calibrate-copy {CALIBRATE_MIB}",
                        f"python3 bench.py --pmc-summary {rel(fetch_csv)} {rel(write_csv)} {rel(out_json)}"],
           "kernels": kernels}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    return 0


def cpu_model() -> str | None:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def traffic_for(label: str, stride: int = 4):
    """HBM bytes per launch of the kernel `label` (backward with checkpoint
    stride `stride`) from the committed counter summary, or None when absent
    or taken from other kernel sources."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            summ = json.load(fh)
    except OSError:
        return None
    if summ.get("source_hash") != kernel_source_hash():
        return None
    hits = [v for k, v in summ["kernels"].items() if symbol_matches(label, k, stride)]
    if len(hits) != 1:
        return None
    return hits[0]


def fwd_cell_flops(N: int, T: int, deciding: bool = False) -> float:
    """Algorithmic FLOPs of one forward cell (FMA = 2): the Toeplitz part
    (N+1)(N+2)/2, Hankel part N(N+1) and combine (N+1) per edge, two edges,
    i.e. (N+1)(3N+4) FMA, plus 3N multiplies for the powers of c; the
    interpolation tail adds 6T(N+1) FMA (T folded tail rows: Toeplitz N+1,
    Hankel N and combine 1 per edge, and projection N+1 per edge), and the
    row that ends the tail, computed but not folded, 4(N+1) FMA."""
    fma = (N + 1) * (3 * N + 4) + 6 * T * (N + 1) + (4 * (N + 1) if deciding else 0)
    return 2.0 * fma + 3 * N


def accuracy_study() -> int:
    """MAPE (fraction) of every scheme against the converged kernel on 8 x 8
    Grams of 2-d Brownian motions on [0, 1] with 10, 50 and 200 steps, the
    setting of the paper's accuracy tables (Section 4, Appendix B; its paths
    and seeds are not given, so only the trends compare).  Every scheme runs
    on the GPU in FP64 (batched); the reference is the FP64 oracle's
    approximation scheme at N = 24 with exponent tracking (converged; it
    stands in for the level-21 truncated signature kernel)."""
    import torch
    import paper_2502_08470_amd as sk
    from paper_2502_08470_amd import _lib
    from oracle import c_oracle as C

    _lib.lib()
    dev = torch.device("cuda:0")
    rows = []
    for steps in (10, 50, 200):
        rng = np.random.default_rng(steps)
        X = np.concatenate([np.zeros((8, 1, 2)),
                            np.cumsum(rng.normal(0, np.sqrt(1.0 / steps), (8, steps, 2)), 1)], 1)
        Y = np.concatenate([np.zeros((8, 1, 2)),
                            np.cumsum(rng.normal(0, np.sqrt(1.0 / steps), (8, steps, 2)), 1)], 1)
        ref = C.value(*C.gram(X, Y, C.APPROX, 24))
        Xt, Yt = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)

        def mape(scheme, order):
            K = sk.gram(Xt, Yt, scheme, order).cpu().numpy()
            return float(np.mean(np.abs(K / ref - 1.0)))
        for N in range(2, 13):  # compiled FP64 orders
            rows.append({"steps": steps, "scheme": "approx", "order": N, "mape": mape("approx", N)})
            rows.append({"steps": steps, "scheme": "interp", "order": N, "mape": mape("interp", N)})
        for lam in range(0, 5):
            rows.append({"steps": steps, "scheme": "fd", "refinement": 2 ** lam, "mape": mape("fd", lam)})
            rows.append({"steps": steps, "scheme": "fd2", "refinement": 2 ** lam, "mape": mape("fd2", lam)})
        print(f"[bench] accuracy study: {steps} steps done", file=sys.stderr, flush=True)
    print(json.dumps({"study": "MAPE vs converged kernel, 8x8 Grams of 2-d Brownian motions",
                      "rows": rows}), flush=True)
    return 0


def long_pair_study(steps: int = 16384) -> int:
    """One pair of R^8 Brownian paths with `steps` steps (FP32): forward time
    of the strip pipeline (strips on co-resident workgroups) against the
    batched algorithm (one wave sweeps the strips in turn), approximation
    N = 8 and interpolation N = 6.  The pipeline's rate is bounded by the
    pair's parallelism (one wave per 64-row strip, a 64 + 16-step lag per
    strip), not by the chip: it is reported as cells/s and as the FLOP rate
    of the forward cell count against the FP32 VALU peak."""
    import torch
    import paper_2502_08470_amd as sk
    from paper_2502_08470_amd import _lib
    import workloads as W

    dev = torch.device("cuda:0")
    x, y = W.long_pair(0, steps, 8)
    X, Y = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    cells = float(steps) * steps
    rows = []
    for scheme, order in (("approx", 8), ("interp", 6)):
        for algo in ("pipeline", "batched"):
            reps = 5 if algo == "pipeline" else 2
            k = sk.gram(X, Y, scheme, order, algo=algo)  # warm-up (and the tables)
            torch.cuda.synchronize()
            _lib.profile_enable(True)
            t0 = time.perf_counter()
            for _ in range(reps):
                k = sk.gram(X, Y, scheme, order, algo=algo)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            # HIP-event kernel times on the launch stream (the cooperative
            # launch of the pipeline is not traced by the profiler tools here)
            kern = {name: _lib.profile_read(name)[0] / reps
                    for name in ("gram", "sweep", "sweep_pipe")}
            _lib.profile_enable(False)
            fl = fwd_cell_flops(order, 0, deciding=scheme == "interp")
            rows.append({"scheme": scheme, "order": order, "algo": algo, "ms": ms,
                         "kernel_ms": {n: v for n, v in kern.items() if v > 0},
                         "cells_per_s": cells / (ms * 1e-3),
                         "tflops": fl * cells / (ms * 1e-3) / 1e12,
                         "frac_of_fp32_peak": fl * cells / (ms * 1e-3) / PEAK_FP32_VALU,
                         "k": float(k.cpu()[0, 0])})
            print(f"[bench] long pair {scheme} {order} {algo}: {ms:.2f} ms", file=sys.stderr,
                  flush=True)
    print(json.dumps({"study": f"single pair of {steps + 1}-point paths in R^8, FP32 forward",
                      "cells": cells, "rows": rows}), flush=True)
    return 0


def long_gram_study() -> int:
    """A 4x4 Gram of 8193-point R^8 Brownian paths (approximation N = 8,
    FP32), forward + backward as autograd runs it: on the strip pipeline
    (gram_save, then gram_backward_saved: checkpoint sweep, adjoint,
    contraction, reduction) and batched (forward, then a recomputing
    backward).  Kernel times are HIP events on the launch stream (library
    profiler), mean of 5 (pipeline) or 1 (batched) steps after a warm-up."""
    import torch
    import paper_2502_08470_amd as sk
    from paper_2502_08470_amd import _lib
    import workloads as W

    dev = torch.device("cuda:0")
    X, Y = W.long_paths_gram(0)
    Xt, Yt = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)
    gK = torch.ones(X.shape[0], Y.shape[0], device=dev)
    cells = float(X.shape[0] * Y.shape[0] * (X.shape[1] - 1) * (Y.shape[1] - 1))
    names = ("gram", "sweep", "sweep_ckpt", "sweep_ckpt_pipe", "adjoint", "adjoint_pipe",
             "contract", "reduce")

    def step_pipeline():
        K, state = sk.gram_save(Xt, Yt, "approx", 8, algo="pipeline")
        sk.gram_backward_saved(Xt, Yt, gK, state, "approx", 8, algo="pipeline")

    def step_batched():
        sk.gram(Xt, Yt, "approx", 8)
        sk.gram_backward(Xt, Yt, gK, "approx", 8)

    rows = []
    for algo, fn, reps in (("pipeline", step_pipeline, 5), ("batched", step_batched, 1)):
        fn()
        torch.cuda.synchronize()
        _lib.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        kern = {n: _lib.profile_read(n)[0] / reps for n in names}
        _lib.profile_enable(False)
        rows.append({"algo": algo, "fwd_bwd_ms": ms, "cells_per_s": cells / (ms * 1e-3),
                     "kernel_ms": {n: v for n, v in kern.items() if v > 0}})
        print(f"[bench] long-paths Gram {algo}: {ms:.2f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"study": "4x4 Gram of 8193-point paths in R^8, approximation N=8, FP32, "
                               "forward + backward", "cells": cells, "rows": rows}), flush=True)
    return 0


def workload_study(large_rows: int = 256) -> int:
    """Time of each named workload on one GPU with its cell count (inputs
    resident on the GPU; best of a few calls after a warm-up):
    * the 8x8 FP64 Gram with a time channel: approximation N=4 and FD lambda=0,
      batched and plain (one launch per pair), forward;
    * 4096 uneven oscillatory pairs, approximation N=8, FP32: forward with the
      tuned plan, the same replayed from a HIP graph, and forward + backward;
    * the MMD sets: unbiased MMD^2 (approximation N=8, FP32) forward and
      backward through autograd (three Grams, XX and YY symmetric);
    * a 4x4 Gram of 8193-point paths in R^8 (approximation N=8, FP32):
      forward and backward on the strip pipeline and batched, and the
      autograd step (pipeline, saved state);
    * the first `large_rows` rows of the 1024x1024 d=32 Gram (approximation
      N=8, FP32 sweep, BF16 3-way split Gram, exponents), forward, and the
      first 16 rows forward + backward."""
    import torch
    import paper_2502_08470_amd as sk
    import workloads as W

    dev = torch.device("cuda:0")
    out = {}

    def best_ms(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best * 1e3

    def say(msg):
        print(f"[bench] workloads: {msg}", file=sys.stderr, flush=True)

    X, Y = W.small_fp64_gram(0)
    Xt, Yt = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)
    cells = float(X.shape[0] * Y.shape[0] * (X.shape[1] - 1) * (Y.shape[1] - 1))
    small = {}
    for scheme, order in (("approx", 4), ("fd", 0)):
        for algo in ("batched", "plain"):
            ms = best_ms(lambda: sk.gram(Xt, Yt, scheme, order, algo=algo), 5)
            small[f"{scheme}{order}_{algo}"] = {"ms": ms, "cells_per_s": cells / ms * 1e3}
    out["small_fp64_gram"] = {"cells": cells, "forward": small}
    say("small FP64 Gram done")

    xs, ys = W.uneven_pairs(0)
    xl = [torch.tensor(a, device=dev) for a in xs]
    yl = [torch.tensor(b, device=dev) for b in ys]
    Xc, Yc = torch.cat(xl), torch.cat(yl)
    cells = float(sum((len(a) - 1) * (len(b) - 1) for a, b in zip(xs, ys)))
    plan = sk.PairsPlan(xl, yl, "approx", 8, backward=True)
    k = torch.empty(len(xs), device=dev)
    gk = torch.ones(len(xs), device=dev)
    gX, gY = torch.empty_like(Xc), torch.empty_like(Yc)
    default_cfg = plan.config()
    fb_default = best_ms(lambda: (plan.forward(Xc, Yc, k), plan.backward(Xc, Yc, gk, gX, gY)), 2)
    tt0 = time.perf_counter()
    plan.tune(Xc, Yc)
    tune_s = time.perf_counter() - tt0
    fwd = best_ms(lambda: plan.forward(Xc, Yc, k))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.forward(Xc, Yc, k)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.forward(Xc, Yc, k)
    graph = best_ms(lambda: g.replay())
    fb = best_ms(lambda: (plan.forward(Xc, Yc, k), plan.backward(Xc, Yc, gk, gX, gY)), 2)
    out["uneven_pairs"] = {"cells": cells, "plan": plan.config(), "plan_default": default_cfg,
                           "fwd_bwd_ms_default_plan": fb_default, "tuning_s": tune_s,
                           "forward_ms": fwd, "forward_graph_ms": graph, "fwd_bwd_ms": fb,
                           "forward_cells_per_s": cells / fwd * 1e3,
                           "fwd_bwd_cells_per_s": cells / fb * 1e3}
    del plan, xl, yl, Xc, Yc, gX, gY, g
    say("uneven pairs done")

    X, Y = W.mmd_sets(0)
    Xt = torch.tensor(X, device=dev).requires_grad_(True)
    Yt = torch.tensor(Y, device=dev).requires_grad_(True)

    def mmd_step():
        Xt.grad = None
        Yt.grad = None
        sk.mmd2(Xt, Yt, "approx", 8).backward()

    ms = best_ms(mmd_step)
    # cells of the three Gram matrices the statistic is defined on, and of
    # the pairs computed (a < b within each set, all cross pairs)
    n, m, steps = X.shape[0], Y.shape[0], X.shape[1] - 1
    cells = 3.0 * n * m * steps ** 2
    computed = (n * (n - 1) / 2 + m * (m - 1) / 2 + n * m) * float(steps) ** 2
    out["mmd_sets"] = {"cells": cells, "cells_computed": computed, "fwd_bwd_ms": ms,
                       "fwd_bwd_cells_per_s": cells / ms * 1e3,
                       "fwd_bwd_computed_cells_per_s": computed / ms * 1e3}
    del Xt, Yt
    say("MMD sets done")

    # few pairs of long paths: the Gram calls' strip pipeline (autograd's
    # choice for them) against the batched algorithm
    X, Y = W.long_paths_gram(0)
    Xt, Yt = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)
    cells = float(X.shape[0] * Y.shape[0] * (X.shape[1] - 1) * (Y.shape[1] - 1))
    gK = torch.ones(X.shape[0], Y.shape[0], device=dev)
    lp = {"algo_autograd": sk.gram_algo(Xt, Yt, "approx"), "cells": cells}
    for algo, reps in (("pipeline", 3), ("batched", 1)):
        fms = best_ms(lambda: sk.gram(Xt, Yt, "approx", 8, algo=algo), reps)
        bms = best_ms(lambda: sk.gram_backward(Xt, Yt, gK, "approx", 8, algo=algo), reps)
        lp[algo] = {"forward_ms": fms, "backward_ms": bms,
                    "fwd_bwd_cells_per_s": cells / (fms + bms) * 1e3}
    Xg = Xt.clone().requires_grad_(True)
    lp["autograd_fwd_bwd_ms"] = best_ms(lambda: sk.sig_gram(Xg, Yt, "approx", 8).sum().backward(), 3)
    out["long_paths_gram"] = lp
    del Xt, Yt, Xg
    say("long paths Gram done")

    X, Y = W.large_gram(0)
    Xt = torch.tensor(X[:large_rows], device=dev)
    Yt = torch.tensor(Y, device=dev)
    del X, Y
    cells = float(Xt.shape[0] * Yt.shape[0] * (Xt.shape[1] - 1) * (Yt.shape[1] - 1))
    ms = best_ms(lambda: sk.gram(Xt, Yt, "approx", 8, return_exp=True, gram_mode="bf16x3"), 1)
    out["large_gram_block"] = {"rows": large_rows, "cells": cells, "forward_ms": ms,
                               "forward_cells_per_s": cells / ms * 1e3,
                               "full_gram_forward_s_at_this_rate": 1024 * 1024 * 1024.0 ** 2 / (cells / ms * 1e3)}
    say("large Gram block done")
    # forward + backward of a smaller block (the backward recomputes the
    # forward with checkpoints under the default 160 GiB chunk cap); the seed
    # 2^-E K makes the loss the sum of the kernel values' mantissas
    bw_rows = 16
    Xb = Xt[:bw_rows].contiguous()
    del Xt
    torch.cuda.empty_cache()
    cells = float(Xb.shape[0] * Yt.shape[0] * (Xb.shape[1] - 1) * (Yt.shape[1] - 1))

    def large_fb():
        K, E = sk.gram(Xb, Yt, "approx", 8, return_exp=True, gram_mode="bf16x3")
        sk.gram_backward(Xb, Yt, torch.ones_like(K), "approx", 8, gK_exp=-E, gram_mode="bf16x3")

    ms = best_ms(large_fb, 1)
    out["large_gram_block_fwd_bwd"] = {"rows": bw_rows, "cells": cells, "fwd_bwd_ms": ms,
                                       "fwd_bwd_cells_per_s": cells / ms * 1e3}
    say("large Gram block forward + backward done")
    print(json.dumps({"study": "named workloads, one MI355X", "workloads": out}), flush=True)
    return 0


def best_of(torch, fn, reps=3):
    """Smallest wall time (ms) of `reps` synchronised calls, after one warm call."""
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) * 1e3)
    return best


def plain_leg(sk, torch, dev) -> dict:
    """The small FP64 Gram (8 x 8, R^3 + time channel, 64 steps): the plain
    one-pair-per-launch kernel against the batched kernels, approximation
    N = 4 and finite differences (dyadic order 0)."""
    import workloads as W
    from oracle import c_oracle as C
    X, Y = W.small_fp64_gram(0)
    Xt, Yt = torch.tensor(X, device=dev), torch.tensor(Y, device=dev)
    cells = float(X.shape[0] * Y.shape[0] * (X.shape[1] - 1) * (Y.shape[1] - 1))
    out = {"workload": "8x8 Gram, R^3 Brownian (variance 1/64 per step) + time channel, "
                       "64 steps, FP64", "cells": cells, "unit": "cell-updates/s"}
    for scheme, order, cid in (("approx", 4, C.APPROX), ("fd", 0, C.FD)):
        ref = np.ldexp(*C.gram(X, Y, cid, order))
        row = {}
        for algo in ("plain", "batched"):
            ms = best_of(torch, lambda: sk.gram(Xt, Yt, scheme, order, algo=algo))
            K = sk.gram(Xt, Yt, scheme, order, algo=algo).cpu().numpy()
            row[algo] = {"forward": cells / (ms * 1e-3), "forward_ms": ms,
                         "max_rel_vs_oracle": float(np.max(np.abs(K / ref - 1.0)))}
        if scheme == "approx":
            Xg, Yg = Xt.clone().requires_grad_(True), Yt.clone().requires_grad_(True)

            def fb():
                Xg.grad = None
                Yg.grad = None
                sk.sig_gram(Xg, Yg, scheme, order, algo="batched").sum().backward()
            ms = best_of(torch, fb)
            row["batched"]["fwd_bwd"] = cells / (ms * 1e-3)
            row["batched"]["fwd_bwd_ms"] = ms
        row["plain_vs_batched_forward"] = row["batched"]["forward"] / row["plain"]["forward"]
        out[f"{scheme}_{order}"] = row
    out["value"] = out["approx_4"]["plain"]["forward"]
    return out


def large_block_leg(sk, torch, dev, rows: int = 16) -> dict:
    """`rows` x 1024 block of the 1024 x 1024 R^32 Gram (approximation N = 8),
    forward + backward through log K (seed gK = 1/K by the exponents), FP32
    sweep with the bf16 3-way split Gram and FP32 points swept in FP64."""
    import workloads as W
    from oracle import c_oracle as C
    X, Y = W.large_gram(0)
    Xt = torch.tensor(X[:rows], device=dev)
    Yt = torch.tensor(Y, device=dev)
    cells = float(rows * Y.shape[0] * (X.shape[1] - 1) * (Y.shape[1] - 1))
    rng = np.random.default_rng(16)
    ia = rng.choice(rows, 8)
    ib = rng.choice(Y.shape[0], 8)
    m, e = C.pairs([X[a].astype(np.float64) for a in ia], [Y[b].astype(np.float64) for b in ib],
                   C.APPROX, 8)
    out = {"workload": f"{rows} x 1024 block of the 1024x1024 Gram, R^32, 1024 steps, "
                       "unit-variance cell constants, approximation N=8, FP32 points, "
                       "fwd+bwd through log K", "cells": cells, "unit": "cell-updates/s"}
    for mode, kw in (("fp32_sweep_bf16x3_gram", dict(gram_mode="bf16x3")),
                     ("fp64_sweep", dict(sweep="f64"))):
        res = {}

        def fb():
            K, Ke = sk.gram(Xt, Yt, "approx", 8, return_exp=True, **kw)
            gK = 1.0 / K
            sk.gram_backward(Xt, Yt, gK, "approx", 8, gK_exp=-Ke, **kw)
            res["K"], res["Ke"] = K, Ke
        ms = best_of(torch, fb, reps=2)
        K, Ke = res["K"].cpu().numpy(), res["Ke"].cpu().numpy()
        sh = Ke[ia, ib].astype(np.int64) - e
        err = np.abs(np.ldexp(K[ia, ib].astype(np.float64), sh) - m) / np.abs(m)
        out[mode] = {"fwd_bwd_ms": ms, "fwd_bwd": cells / (ms * 1e-3),
                     "gram_entries_per_s": rows * Y.shape[0] / (ms * 1e-3),
                     "mape_8_pairs": float(err.mean()), "max_ape_8_pairs": float(err.max())}
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the Gram tuner (algorithm and checkpoint stride) before the warm-up")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after timing, copy MIB MiB device to device once (a plain copy "
                         "kernel of known size, to scale HBM byte counters)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT_JSON"),
                    help="summarise two rocprofv3 --pmc runs into HBM bytes per dispatch")
    ap.add_argument("--accuracy-study", action="store_true",
                    help="MAPE of every scheme vs the converged kernel (paper's accuracy tables)")
    ap.add_argument("--long-gram", action="store_true",
                    help="forward + backward of a 4x4 Gram of 8193-point paths, pipeline vs batched")
    ap.add_argument("--long-pair", type=int, default=0, metavar="STEPS",
                    help="strip pipeline vs batched on one pair of STEPS-step paths")
    ap.add_argument("--workloads", action="store_true",
                    help="time every named workload (small FP64 Gram, uneven pairs, MMD, large Gram block)")
    args = ap.parse_args(argv)
    if args.workloads:
        return workload_study()
    if args.accuracy_study:
        return accuracy_study()
    if args.long_pair:
        return long_pair_study(args.long_pair)
    if args.long_gram:
        return long_gram_study()
    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)
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

    tuned = None
    if not args.no_tune:
        # the tuner times each algorithm and checkpoint stride on this
        # workload (outside the timed region); autograd then takes its choice
        tt0 = time.perf_counter()
        tuned = sk.tune_gram(Xt.detach(), Yt.detach(), SCHEME, ORDER, backward=True)
        tuned["tuning_s"] = time.perf_counter() - tt0
        print(f"[bench] tuned {tuned}", file=sys.stderr, flush=True)
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        K, gX, gY = step()
    torch.cuda.synchronize()
    kernels = ["gram", "sweep", "sweep_ckpt", "adjoint", "sweep_pipe", "sweep_ckpt_pipe",
               "adjoint_pipe", "contract", "reduce"]
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
    # interpolation tail on this workload (|c| < 0.05): the first tail row is
    # computed, found below the working precision and not folded (T = 0); the
    # adjoint replays the forward with the recorded T (no deciding row) and
    # applies the transposed map: 2 forwards without the deciding row (the
    # dL/dc terms are not counted)
    fl_fwd = fwd_cell_flops(ORDER, 0, deciding=True)
    fl_adj = 2.0 * fwd_cell_flops(ORDER, 0)
    flops_per_cell = {"sweep": fl_fwd, "sweep_ckpt": fl_fwd, "adjoint": fl_adj,
                      "sweep_pipe": fl_fwd, "sweep_ckpt_pipe": fl_fwd, "adjoint_pipe": fl_adj,
                      "gram": 2.0 * DIM, "contract": 4.0 * DIM}
    dom = max((k for k in flops_per_cell if ktimes[k][1] > 0), key=lambda k: ktimes[k][0])
    dom_ms, dom_n = ktimes[dom]
    # every step runs each kernel over all cells once (possibly in several
    # launches of part of the pairs): FLOPs per launch = cells * steps / launches
    cells_per_launch = cells * args.steps / dom_n
    achieved = flops_per_cell[dom] * cells_per_launch / (dom_ms / dom_n * 1e-3)
    stride = tuned["ckpt"] if tuned is not None else 4
    tr = traffic_for(dom, stride)
    roofline = {"kernel": dom, "ckpt_stride": stride, "bound": "alu", "achieved": achieved / 1e12,
                "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VALU,
                "traffic": None if tr is None else tr["bytes"],
                "traffic_unit": "bytes per launch (HBM fetch + write)",
                "flops_per_cell": flops_per_cell[dom], "launch_ms": dom_ms / dom_n,
                "launches_per_step": dom_n / args.steps,
                "kernel_ms_per_step": {k: ktimes[k][0] / args.steps for k in kernels}}

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "128x128 Gram, paths in R^8, 256 Brownian steps "
                                  "(std 0.5/16), polynomial interpolation N=6, FP32 sweep, "
                                  "FP32 increment Gram by an 8-term FMA chain per cell "
                                  "(k_gram_direct), fwd+bwd (loss sum K)",
                      "pairs": N_PATHS * N_PATHS, "cells_per_pair": STEPS * STEPS,
                      "gram_kernel": "k_gram_direct",
                      "schedule": tuned if tuned is not None else
                      {"algo": sk.gram_algo(Xt, Yt, SCHEME), "ckpt": 4, "tuned": False}},
           "gram_entries_per_s": entries, "roofline": roofline}

    # accuracy on the 16 x 16 block (and the larger CPU sample), CPU oracle
    from oracle import c_oracle as C
    threads = C.default_threads()
    bx, by = (16, 16) if args.no_cpu_baseline else CPU_BLOCK
    Xb = X[:bx].astype(np.float64)
    Yb = Y[:by].astype(np.float64)
    print(f"[bench] oracle {bx}x{by} block on {threads} threads", file=sys.stderr, flush=True)
    c0 = time.perf_counter()
    m, e = C.gram(Xb, Yb, C.INTERP, ORDER, threads=threads)
    c1 = time.perf_counter()
    ref = np.ldexp(m, e)
    Kb = K[:bx, :by].double().cpu().numpy()
    ape = np.abs(Kb / ref - 1.0)
    out["mape"] = float(ape[:16, :16].mean())
    out["max_ape"] = float(ape[:16, :16].max())
    if not args.no_cpu_baseline:
        out["mape_cpu_sample"] = float(ape.mean())
        out["max_ape_cpu_sample"] = float(ape.max())
        ocells = bx * by * STEPS * STEPS
        out["cpu_baseline"] = {"value": ocells / (c1 - c0), "unit": "cell-updates/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{bx}x{by} block X[0:{bx}] x Y[0:{by}] of the same "
                                         "workload, forward only, FP64 C oracle (literal 0F1 "
                                         "at the Chebyshev extrema + Vandermonde solve)",
                               "seconds": c1 - c0}
        # one core on a smaller block, and what the host is
        sx, sy = 4, 8
        s0 = time.perf_counter()
        C.gram(Xb[:sx], Yb[:sy], C.INTERP, ORDER, threads=1)
        s1 = time.perf_counter()
        out["cpu_baseline"]["single_core"] = {
            "value": sx * sy * STEPS * STEPS / (s1 - s0), "unit": "cell-updates/s",
            "sample": f"{sx}x{sy} block X[0:{sx}] x Y[0:{sy}], one thread", "seconds": s1 - s0}
        out["cpu_baseline"]["host"] = {"cpu_count": os.cpu_count(), "model": cpu_model(),
                                       "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    # the same Gram's constants by MFMA tiles (the label above names the
    # kernel the step runs)
    _lib.profile_enable(True)
    sk.gram(Xt.detach(), Yt.detach(), SCHEME, ORDER, gram_mode="mfma")
    torch.cuda.synchronize()
    out["gram_mfma_ms"] = _lib.profile_read("gram")[0]
    _lib.profile_enable(False)
    if not args.no_plain:
        out["plain_fp64"] = plain_leg(sk, torch, dev)
        out["large_gram_block"] = large_block_leg(sk, torch, dev)
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
