// Definitions of SkLaunch<R> (included once per real type).
#pragma once
#include <algorithm>

#include "sk_launch.h"

#define SK_CHECK_LAUNCH() \
    do {                  \
        hipError_t e_ = hipGetLastError(); \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

template <typename R>
hipError_t SkLaunch<R>::fill(R* p, int64_t n, R v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill<R>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::to_f64(const R* src, double* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_convert<R, double>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::from_f64(const double* src, R* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_convert<double, R>), dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::fill_u32(unsigned* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill<unsigned>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, 0u);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::gram(const GramArgs<R>& a, int ntau_blocks, int64_t npairs,
                             hipStream_t st) {
    if (npairs <= 0 || ntau_blocks <= 0) return hipSuccess;
    if (a.split) {
        if constexpr (sizeof(R) == 4)
            hipLaunchKernelGGL((k_gram_skew<R, true>), dim3((unsigned)npairs, ntau_blocks),
                               dim3(256), gram_lds(a.dpad), st, a);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_gram_skew<R, false>), dim3((unsigned)npairs, ntau_blocks), dim3(256),
                           gram_lds(a.dpad), st, a);
    }
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::gram_pair(const GramArgs<R>& a, int max_lx, int max_ly, int64_t npairs,
                                  hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    const size_t lds = gram_pair_lds(a.dpad, max_lx, max_ly);
    if (a.split) {
        if constexpr (sizeof(R) == 4)
            hipLaunchKernelGGL((k_gram_pair<R, true>), dim3((unsigned)npairs), dim3(256), lds, st, a);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_gram_pair<R, false>), dim3((unsigned)npairs), dim3(256), lds, st, a);
    }
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::gram_direct(const GramArgs<R>& a, int max_lx, int max_ly, int64_t npairs,
                                    hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    if (a.split || a.dpad > SK_GRAM_DIRECT_DMAX) return hipErrorInvalidValue;
    const size_t lds = gram_direct_lds(a.dpad, max_lx, max_ly);
    hipLaunchKernelGGL((k_gram_direct<R>), dim3((unsigned)npairs), dim3(256), lds, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::gram_band(const GramArgs<R>& a0, int max_strips, int max_rows,
                                  int64_t npairs, hipStream_t st) {
    if (npairs <= 0 || max_strips <= 0 || max_rows <= 0) return hipSuccess;
    // split each strip's rows so that the launch has about 2048 workgroups,
    // segments of at least 256 rows (a multiple of 64)
    const int64_t wgs = npairs * (int64_t)max_strips;
    int64_t nseg = wgs >= 2048 ? 1 : (2048 + wgs - 1) / wgs;
    nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, max_rows / 256));
    GramArgs<R> a = a0;
    a.rseg = (int)(((max_rows + nseg - 1) / nseg + 63) / 64 * 64);
    nseg = (max_rows + a.rseg - 1) / a.rseg;
    const dim3 grid((unsigned)npairs, (unsigned)max_strips, (unsigned)nseg);
    const size_t lds = gram_band_lds(a.dpad);
    if (a.split) {
        if constexpr (sizeof(R) == 4)
            hipLaunchKernelGGL((k_gram_band<R, true>), grid, dim3(256), lds, st, a);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_gram_band<R, false>), grid, dim3(256), lds, st, a);
    }
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::gram_strip(const GramArgs<R>& a0, int max_strips, int max_rows,
                                   int64_t npairs, hipStream_t st) {
    if (npairs <= 0 || max_strips <= 0 || max_rows <= 0) return hipSuccess;
    if (a0.split || a0.dpad > SK_GRAM_STRIP_DMAX) return hipErrorInvalidValue;
    // split each strip's rows so that the launch has about 2048 workgroups
    // (a few long pairs have few strips), segments of at least 256 rows
    constexpr int SW = SK_GRAM_STRIP_WAVES;  // strips per workgroup
    const int64_t groups = (max_strips + SW - 1) / SW;
    const int64_t wgs = npairs * groups;
    const int64_t want = 2048;
    int64_t nseg = wgs >= want ? 1 : (want + wgs - 1) / wgs;
    nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, max_rows / 256));
    GramArgs<R> a = a0;
    a.rseg = (int)(((max_rows + nseg - 1) / nseg + 7) / 8 * 8);
    nseg = (max_rows + a.rseg - 1) / a.rseg;
    const dim3 grid((unsigned)npairs, (unsigned)groups, (unsigned)nseg), blk(64 * SW);
    if (a.dpad <= 4)
        hipLaunchKernelGGL((k_gram_strip<R, 4>), grid, blk, (128 * sk_ring_ys<R, 4>() * sizeof(R)), st, a);
    else if (a.dpad <= 8)
        hipLaunchKernelGGL((k_gram_strip<R, 8>), grid, blk, (128 * sk_ring_ys<R, 8>() * sizeof(R)), st, a);
    else if (a.dpad <= 16)
        hipLaunchKernelGGL((k_gram_strip<R, 16>), grid, blk, (128 * sk_ring_ys<R, 16>() * sizeof(R)), st, a);
    else
        hipLaunchKernelGGL((k_gram_strip<R, 32>), grid, blk, (128 * sk_ring_ys<R, 32>() * sizeof(R)), st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

// Checkpoint strides compiled per precision (the stride the host chose is
// a.S; FP32 2 or 4, FP64 2).  Only checkpointing kernels depend on it.
template <typename R> constexpr bool sk_alt_stride() { return sizeof(R) == 4; }

template <typename R, int N, int TMAX, int S>
static hipError_t sk_sweep_s(const SweepArgs<R>& a, bool ckpt, int64_t npairs, int ring, bool gx,
                             hipStream_t st) {
    // exchange launches that checkpoint stage lane 63's records of a block
    size_t lds = SkLaunch<R>::sweep_lds(N, ring) + (ckpt && gx ? sk_gx_stage_bytes(N, (int)sizeof(R)) : 0);
    dim3 grid((unsigned)npairs), blk(64);
    if (ckpt && gx)
        hipLaunchKernelGGL((k_sweep<R, N, TMAX, true, S, true>), grid, blk, lds, st, a);
    else if (ckpt)
        hipLaunchKernelGGL((k_sweep<R, N, TMAX, true, S, false>), grid, blk, lds, st, a);
    else if (gx)
        hipLaunchKernelGGL((k_sweep<R, N, TMAX, false, S, true>), grid, blk, lds, st, a);
    else
        hipLaunchKernelGGL((k_sweep<R, N, TMAX, false, S, false>), grid, blk, lds, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R, int N, int TMAX>
static hipError_t sk_sweep_n(const SweepArgs<R>& a, bool ckpt, int64_t npairs, int ring, bool gx,
                             hipStream_t st) {
    constexpr int S = SkCkptStride<R>::value;
    if constexpr (sk_alt_stride<R>())
        if (ckpt && a.S == 2) return sk_sweep_s<R, N, TMAX, 2>(a, ckpt, npairs, ring, gx, st);
    if (ckpt && a.S != S) return hipErrorInvalidValue;
    return sk_sweep_s<R, N, TMAX, S>(a, ckpt, npairs, ring, gx, st);
}

template <typename R, int N>
static hipError_t sk_sweep_t(const SweepArgs<R>& a, bool interp, bool ckpt, int64_t npairs,
                             int ring, bool gx, hipStream_t st) {
    return interp ? sk_sweep_n<R, N, SkTailMax<R>::value>(a, ckpt, npairs, ring, gx, st)
                  : sk_sweep_n<R, N, 0>(a, ckpt, npairs, ring, gx, st);
}

template <typename R>
hipError_t SkLaunch<R>::sweep(const SweepArgs<R>& a, int N, bool interp, bool ckpt,
                              int64_t npairs, int ring, bool gx, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    switch (N) {
        case 2: return sk_sweep_t<R, 2>(a, interp, ckpt, npairs, ring, gx, st);
        case 3: return sk_sweep_t<R, 3>(a, interp, ckpt, npairs, ring, gx, st);
        case 4: return sk_sweep_t<R, 4>(a, interp, ckpt, npairs, ring, gx, st);
        case 5: return sk_sweep_t<R, 5>(a, interp, ckpt, npairs, ring, gx, st);
        case 6: return sk_sweep_t<R, 6>(a, interp, ckpt, npairs, ring, gx, st);
        case 7: return sk_sweep_t<R, 7>(a, interp, ckpt, npairs, ring, gx, st);
        case 8: return sk_sweep_t<R, 8>(a, interp, ckpt, npairs, ring, gx, st);
        default:
            if constexpr (sizeof(R) == 8)
                if (N > SK_MAX_ORDER && N <= SK_MAX_ORDER_F64)
                    return sk_hi_sweep(a, N, interp, ckpt, npairs, ring, gx, st);
            return hipErrorInvalidValue;
    }
}

// Cooperative launch of a strip-pipeline kernel: as many one-wave
// workgroups as fit on the device at once (every wave that another waits for
// must be resident), at most one per job.
template <typename Args>
static hipError_t sk_coop_launch(const void* kern, const Args& a, int64_t njobs, size_t lds,
                                 hipStream_t st) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 64, lds);
    if (e != hipSuccess) return e;
    int64_t W = std::min<int64_t>(std::max<int64_t>(1, njobs), (int64_t)per * ncu);
    if (W < 1) return hipErrorInvalidConfiguration;
    Args arg = a;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)W), dim3(64), args, (unsigned)lds, st);
}

template <typename R, int N, int TMAX>
static hipError_t sk_pipe_n(const PipeArgs<R>& a, bool ckpt, hipStream_t st) {
    constexpr int S = SkCkptStride<R>::value;
    const void* kern = ckpt ? reinterpret_cast<const void*>(&k_sweep_pipe<R, N, TMAX, true, S>)
                            : reinterpret_cast<const void*>(&k_sweep_pipe<R, N, TMAX, false, S>);
    if constexpr (sk_alt_stride<R>())
        if (ckpt && a.S == 2) kern = reinterpret_cast<const void*>(&k_sweep_pipe<R, N, TMAX, true, 2>);
    if (ckpt && a.S != S && !(sk_alt_stride<R>() && a.S == 2)) return hipErrorInvalidValue;
    return sk_coop_launch(kern, a, a.njobs, (size_t)2 * sk_gx_stage_bytes(N, (int)sizeof(R)), st);
}

template <typename R>
hipError_t SkLaunch<R>::sweep_pipe(const PipeArgs<R>& a, int N, bool interp, bool ckpt, hipStream_t st) {
    if (!a.desc || !a.jobs || a.njobs <= 0) return hipErrorInvalidValue;
    constexpr int T = SkTailMax<R>::value;
    switch (N) {
        case 2: return interp ? sk_pipe_n<R, 2, T>(a, ckpt, st) : sk_pipe_n<R, 2, 0>(a, ckpt, st);
        case 3: return interp ? sk_pipe_n<R, 3, T>(a, ckpt, st) : sk_pipe_n<R, 3, 0>(a, ckpt, st);
        case 4: return interp ? sk_pipe_n<R, 4, T>(a, ckpt, st) : sk_pipe_n<R, 4, 0>(a, ckpt, st);
        case 5: return interp ? sk_pipe_n<R, 5, T>(a, ckpt, st) : sk_pipe_n<R, 5, 0>(a, ckpt, st);
        case 6: return interp ? sk_pipe_n<R, 6, T>(a, ckpt, st) : sk_pipe_n<R, 6, 0>(a, ckpt, st);
        case 7: return interp ? sk_pipe_n<R, 7, T>(a, ckpt, st) : sk_pipe_n<R, 7, 0>(a, ckpt, st);
        case 8: return interp ? sk_pipe_n<R, 8, T>(a, ckpt, st) : sk_pipe_n<R, 8, 0>(a, ckpt, st);
        default:
            if constexpr (sizeof(R) == 8)
                if (N > SK_MAX_ORDER && N <= SK_MAX_ORDER_F64) return sk_hi_sweep_pipe(a, N, interp, ckpt, st);
            return hipErrorInvalidValue;
    }
}

template <typename R, int N, int TMAX>
static hipError_t sk_adj_pipe_n(const AdjPipeArgs<R>& a, hipStream_t st) {
    constexpr int S = SkCkptStride<R>::value;
    if constexpr (sk_alt_stride<R>())
        if (a.S == 2)
            return sk_coop_launch(reinterpret_cast<const void*>(&k_adjoint_pipe<R, N, TMAX, 2>), a,
                                  a.njobs, (size_t)sk_adj_pipe_lds<R>(N, TMAX, 2), st);
    if (a.S != S) return hipErrorInvalidValue;
    const void* kern = reinterpret_cast<const void*>(&k_adjoint_pipe<R, N, TMAX, S>);
    return sk_coop_launch(kern, a, a.njobs, (size_t)sk_adj_pipe_lds<R>(N, TMAX, S), st);
}

template <typename R>
hipError_t SkLaunch<R>::adjoint_pipe(const AdjPipeArgs<R>& a, int N, bool interp, hipStream_t st) {
    if (a.njobs <= 0) return hipSuccess;
    constexpr int T = SkTailMax<R>::value;
    switch (N) {
        case 2: return interp ? sk_adj_pipe_n<R, 2, T>(a, st) : sk_adj_pipe_n<R, 2, 0>(a, st);
        case 3: return interp ? sk_adj_pipe_n<R, 3, T>(a, st) : sk_adj_pipe_n<R, 3, 0>(a, st);
        case 4: return interp ? sk_adj_pipe_n<R, 4, T>(a, st) : sk_adj_pipe_n<R, 4, 0>(a, st);
        case 5: return interp ? sk_adj_pipe_n<R, 5, T>(a, st) : sk_adj_pipe_n<R, 5, 0>(a, st);
        case 6: return interp ? sk_adj_pipe_n<R, 6, T>(a, st) : sk_adj_pipe_n<R, 6, 0>(a, st);
        case 7: return interp ? sk_adj_pipe_n<R, 7, T>(a, st) : sk_adj_pipe_n<R, 7, 0>(a, st);
        case 8: return interp ? sk_adj_pipe_n<R, 8, T>(a, st) : sk_adj_pipe_n<R, 8, 0>(a, st);
        default:
            if constexpr (sizeof(R) == 8)
                if (N > SK_MAX_ORDER && N <= SK_MAX_ORDER_F64) return sk_hi_adjoint_pipe(a, N, interp, st);
            return hipErrorInvalidValue;
    }
}

template <typename R, int N, int TMAX, bool GX, int S>
static hipError_t sk_adj_gs(const AdjArgs<R>& a, int64_t npairs, int ring, hipStream_t st) {
    size_t lds = SkLaunch<R>::adjoint_lds(N, ring);
    if constexpr (sk_adj_two_waves<R, N, TMAX, GX>())
        hipLaunchKernelGGL((k_adjoint_w2<R, N, TMAX, S, GX>), dim3((unsigned)npairs), dim3(64), lds,
                           st, a);
    else
        hipLaunchKernelGGL((k_adjoint<R, N, TMAX, S, GX>), dim3((unsigned)npairs), dim3(64), lds,
                           st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R, int N, int TMAX, bool GX>
static hipError_t sk_adj_g(const AdjArgs<R>& a, int64_t npairs, int ring, hipStream_t st) {
    constexpr int S = SkCkptStride<R>::value;
    if constexpr (sk_alt_stride<R>())
        if (a.S == 2) return sk_adj_gs<R, N, TMAX, GX, 2>(a, npairs, ring, st);
    if (a.S != S) return hipErrorInvalidValue;
    return sk_adj_gs<R, N, TMAX, GX, S>(a, npairs, ring, st);
}

template <typename R, int N, int TMAX>
static hipError_t sk_adj_n(const AdjArgs<R>& a, int64_t npairs, int ring, bool gx,
                           hipStream_t st) {
    return gx ? sk_adj_g<R, N, TMAX, true>(a, npairs, ring, st)
              : sk_adj_g<R, N, TMAX, false>(a, npairs, ring, st);
}

template <typename R, int N>
static hipError_t sk_adj_t(const AdjArgs<R>& a, bool interp, int64_t npairs, int ring, bool gx,
                           hipStream_t st) {
    return interp ? sk_adj_n<R, N, SkTailMax<R>::value>(a, npairs, ring, gx, st)
                  : sk_adj_n<R, N, 0>(a, npairs, ring, gx, st);
}

template <typename R>
hipError_t SkLaunch<R>::adjoint(const AdjArgs<R>& a, int N, bool interp, int64_t npairs,
                                int ring, bool gx, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    switch (N) {
        case 2: return sk_adj_t<R, 2>(a, interp, npairs, ring, gx, st);
        case 3: return sk_adj_t<R, 3>(a, interp, npairs, ring, gx, st);
        case 4: return sk_adj_t<R, 4>(a, interp, npairs, ring, gx, st);
        case 5: return sk_adj_t<R, 5>(a, interp, npairs, ring, gx, st);
        case 6: return sk_adj_t<R, 6>(a, interp, npairs, ring, gx, st);
        case 7: return sk_adj_t<R, 7>(a, interp, npairs, ring, gx, st);
        case 8: return sk_adj_t<R, 8>(a, interp, npairs, ring, gx, st);
        default:
            if constexpr (sizeof(R) == 8)
                if (N > SK_MAX_ORDER && N <= SK_MAX_ORDER_F64)
                    return sk_hi_adjoint(a, N, interp, npairs, ring, gx, st);
            return hipErrorInvalidValue;
    }
}

template <typename R, int DMAX>
static void sk_contract_d(const ContractArgs<R>& a, dim3 grid, hipStream_t st) {
    const size_t lds = (size_t)128 * sk_ring_ys<R, DMAX>() * sizeof(R);
    hipLaunchKernelGGL((k_contract<R, DMAX>), grid, dim3(64), lds, st, a);
}

template <typename R>
hipError_t SkLaunch<R>::fold_refined(const FoldArgs<R>& a, int max_nsteps_pad, int64_t npairs,
                                     hipStream_t st) {
    if (npairs <= 0 || max_nsteps_pad <= 0) return hipSuccess;
    const int64_t by = std::min<int64_t>(((int64_t)max_nsteps_pad * SK_LANES + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fold_refined<R>, dim3((unsigned)npairs, (unsigned)by), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::contract(const ContractArgs<R>& a, int max_strips, int64_t npairs,
                                 hipStream_t st) {
    if (npairs <= 0 || max_strips <= 0) return hipSuccess;
    // d <= 32: the MFMA tiles (FP32, d = 8: 2.05 -> 1.64 ms on the 128 x 128
    // Gram of 256-step paths; d = 32: 2.3x faster); d > 32: the VALU
    // wavefront kernel
    if constexpr (sizeof(R) == 8) {
        if (a.d <= 32) {
            dim3 g2((unsigned)npairs, max_strips);
            if (a.d <= 16)
                hipLaunchKernelGGL(k_contract_mfma_f64<1>, g2, dim3(256), sk_cmfma64_lds<1>(), st, a);
            else
                hipLaunchKernelGGL(k_contract_mfma_f64<2>, g2, dim3(256), sk_cmfma64_lds<2>(), st, a);
            SK_CHECK_LAUNCH();
            return hipSuccess;
        }
    }
    if constexpr (sizeof(R) == 4) {
        if (a.d <= 32) {
            dim3 g2((unsigned)npairs, max_strips);
            if (a.d <= 16)
                hipLaunchKernelGGL(k_contract_mfma<1>, g2, dim3(256), sk_cmfma_lds<1>(), st, a);
            else
                hipLaunchKernelGGL(k_contract_mfma<2>, g2, dim3(256), sk_cmfma_lds<2>(), st, a);
            SK_CHECK_LAUNCH();
            return hipSuccess;
        }
    }
    // d > 16: slices of 16 dimensions on separate waves
    dim3 grid((unsigned)npairs, max_strips, (unsigned)((a.d + 15) / 16));
    if (a.d <= 4) sk_contract_d<R, 4>(a, grid, st);
    else if (a.d <= 8) sk_contract_d<R, 8>(a, grid, st);
    else sk_contract_d<R, 16>(a, grid, st);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::reduce_gram(const ReduceGramArgs<R>& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    const int64_t a_lo = a.first / a.ny, a_hi = (a.first + a.count - 1) / a.ny;
    int64_t nx_e = (a_hi - a_lo + 1) * a.lx_pts * a.d;
    int64_t ny_e = a.ny * a.ly_pts * a.d;
    hipLaunchKernelGGL(k_reduce_gram_x<R>, dim3((unsigned)((nx_e + 63) / 64)), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_reduce_gram_y<R>, dim3((unsigned)((ny_e + 63) / 64)), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::reduce_pairs(const ReducePairsArgs<R>& a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    int64_t e = a.max_pts * a.d;
    int64_t bx = (e + 255) / 256;
    if (bx > 64) bx = 64;
    hipLaunchKernelGGL(k_reduce_pairs<R>, dim3((unsigned)a.count, (unsigned)bx), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::sweep_fd(const FdArgs<R>& a, int64_t npairs, int max_ly_refined,
                                 hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sweep_fd<R>, dim3((unsigned)npairs), dim3(64),
                       (size_t)max_ly_refined * sizeof(R), st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R, int N>
static hipError_t sk_plain_n(const PlainArgs<R>& a, bool interp, hipStream_t st) {
    if (interp)
        hipLaunchKernelGGL((k_plain_poly<R, N, SkTailMax<R>::value>), dim3(1), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_plain_poly<R, N, 0>), dim3(1), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::plain_poly(const PlainArgs<R>& a, int N, bool interp, hipStream_t st) {
    switch (N) {
        case 2: return sk_plain_n<R, 2>(a, interp, st);
        case 3: return sk_plain_n<R, 3>(a, interp, st);
        case 4: return sk_plain_n<R, 4>(a, interp, st);
        case 5: return sk_plain_n<R, 5>(a, interp, st);
        case 6: return sk_plain_n<R, 6>(a, interp, st);
        case 7: return sk_plain_n<R, 7>(a, interp, st);
        case 8: return sk_plain_n<R, 8>(a, interp, st);
        default:
            if constexpr (sizeof(R) == 8)
                if (N > SK_MAX_ORDER && N <= SK_MAX_ORDER_F64) return sk_hi_plain_poly(a, N, interp, st);
            return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t SkLaunch<R>::plain_fd(const PlainArgs<R>& a, hipStream_t st) {
    hipLaunchKernelGGL(k_plain_fd<R>, dim3(1), dim3(256), 0, st, a);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::mmd_perm(const R* K, int64_t m, int64_t n, const int32_t* perms,
                                 int64_t nperm, R* stats, double* pvalue, hipStream_t st) {
    if (nperm <= 0) return hipSuccess;
    const size_t lds = (size_t)((m + n + 15) / 16) * 16 + 256 * sizeof(double);
    hipLaunchKernelGGL(k_mmd_perm<R>, dim3((unsigned)nperm), dim3(256), lds, st, K, m, n, perms,
                       stats);
    SK_CHECK_LAUNCH();
    if (pvalue) {
        hipLaunchKernelGGL(k_mmd_pvalue<R>, dim3(1), dim3(256), 0, st, stats, nperm, pvalue);
        SK_CHECK_LAUNCH();
    }
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::mmd2_pairs(const R* k, int64_t nx, int64_t ny, R* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mmd2_pairs<R>, dim3(1), dim3(256), 0, st, k, nx, ny, out);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::mmd2_pairs_seed(const R* gout, int64_t nx, int64_t ny, R* gk,
                                        hipStream_t st) {
    const int64_t tot = nx * (nx - 1) / 2 + ny * (ny - 1) / 2 + nx * ny;
    const unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mmd2_pairs_seed<R>, dim3(blocks), dim3(256), 0, st, gout, nx, ny, gk);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::unskew(const SkPairSrc& src, const R* cskew, R* C, int64_t first,
                               int64_t npairs, int64_t cells, hipStream_t st) {
    if (npairs <= 0 || cells <= 0) return hipSuccess;
    int64_t bx = (cells + 255) / 256;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_unskew<R>, dim3((unsigned)npairs, (unsigned)bx), dim3(256), 0, st, src,
                       cskew, C, first);
    SK_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename R>
hipError_t SkLaunch<R>::status_word(unsigned** p) {
    return hipGetSymbolAddress(reinterpret_cast<void**>(p), HIP_SYMBOL(sk_status_word));
}
