// Host-side launchers of the batched kernels (defined per real type in
// sk_inst_f32.hip / sk_inst_f64.hip).  Argument structs live in sk_kernels.h.
#pragma once
#include <hip/hip_runtime.h>

#include "sk_kernels.h"

// orders with compiled polynomial kernels (FP64 also N = 9..12, compiled in
// their own translation unit, sk_inst_f64_hi.hip)
#define SK_MIN_ORDER 2
#define SK_MAX_ORDER 8
#define SK_MAX_ORDER_F64 12
#define SK_MAX_DYADIC 8
#define SK_MAX_DIM 64
// checkpoint stride of the adjoint's forward recompute
template <typename R> struct SkCkptStride;
template <> struct SkCkptStride<float> { static constexpr int value = 4; };
template <> struct SkCkptStride<double> { static constexpr int value = 2; };

template <typename R>
struct SkLaunch {
    static hipError_t fill(R* p, int64_t n, R v, hipStream_t st);
    static hipError_t fill_u32(unsigned* p, int64_t n, hipStream_t st);
    // dst = (double)src and dst = (R)src, n elements
    static hipError_t to_f64(const R* src, double* dst, int64_t n, hipStream_t st);
    static hipError_t from_f64(const double* src, R* dst, int64_t n, hipStream_t st);
    static hipError_t gram(const GramArgs<R>& a, int ntau_blocks, int64_t npairs, hipStream_t st);
    // pair-resident Gram (all row blocks of a pair in one workgroup); max_lx, max_ly
    // are unrefined segment counts
    static hipError_t gram_pair(const GramArgs<R>& a, int max_lx, int max_ly, int64_t npairs,
                                hipStream_t st);
    // direct (VALU) Gram for dpad <= SK_GRAM_DIRECT_DMAX, native precision
    static hipError_t gram_direct(const GramArgs<R>& a, int max_lx, int max_ly, int64_t npairs,
                                  hipStream_t st);
    // MFMA tiles of a strip's 64 x ly band, one workgroup per (pair, strip,
    // row segment); max_strips and max_rows as for gram_strip
    static hipError_t gram_band(const GramArgs<R>& a, int max_strips, int max_rows,
                                int64_t npairs, hipStream_t st);
    // the same arithmetic, one wave per (pair, strip, row segment), for pairs
    // whose increments exceed the LDS of one workgroup; max_strips and
    // max_rows (skewed rows of the longest strip) of the refined grids
    static hipError_t gram_strip(const GramArgs<R>& a, int max_strips, int max_rows,
                                 int64_t npairs, hipStream_t st);
    // ring: LDS ring columns of the launch (largest among its pairs that do
    // not use the global strip-boundary exchange)
    // gx: some pair of the launch uses the global strip-boundary exchange
    static hipError_t sweep(const SweepArgs<R>& a, int N, bool interp, bool ckpt, int64_t npairs,
                            int ring, bool gx, hipStream_t st);
    static hipError_t adjoint(const AdjArgs<R>& a, int N, bool interp, int64_t npairs, int ring,
                              bool gx, hipStream_t st);
    // strip pipeline: strips of one pair, or of a job list, on co-resident
    // workgroups (cooperative launch; at most one workgroup per job).
    // ckpt: also store the pipelined adjoint's checkpoints (job lists only)
    static hipError_t sweep_pipe(const PipeArgs<R>& a, int N, bool interp, bool ckpt, hipStream_t st);
    // adjoint of strip-pipeline pairs: the job list's strips, each pair's in
    // decreasing order, on co-resident workgroups
    static hipError_t adjoint_pipe(const AdjPipeArgs<R>& a, int N, bool interp, hipStream_t st);
    static hipError_t fold_refined(const FoldArgs<R>& a, int max_nsteps_pad, int64_t npairs,
                                   hipStream_t st);
    static hipError_t contract(const ContractArgs<R>& a, int max_strips, int64_t npairs,
                               hipStream_t st);
    static hipError_t reduce_gram(const ReduceGramArgs<R>& a, hipStream_t st);
    static hipError_t reduce_pairs(const ReducePairsArgs<R>& a, hipStream_t st);
    static hipError_t sweep_fd(const FdArgs<R>& a, int64_t npairs, int max_ly_refined,
                               hipStream_t st);
    static hipError_t plain_poly(const PlainArgs<R>& a, int N, bool interp, hipStream_t st);
    static hipError_t plain_fd(const PlainArgs<R>& a, hipStream_t st);
    static hipError_t mmd_perm(const R* K, int64_t m, int64_t n, const int32_t* perms,
                               int64_t nperm, R* stats, double* pvalue, hipStream_t st);
    // unbiased MMD^2 from a [xx | yy | xy] pair list, and its seeds
    static hipError_t mmd2_pairs(const R* k, int64_t nx, int64_t ny, R* out, hipStream_t st);
    static hipError_t mmd2_pairs_seed(const R* gout, int64_t nx, int64_t ny, R* gk, hipStream_t st);
    static hipError_t unskew(const SkPairSrc& src, const R* cskew, R* C, int64_t first,
                             int64_t npairs, int64_t cells, hipStream_t st);
    // device address of the status word the kernels of this instantiation
    // raise bits in (SK_STATUS_*), for the current device
    static hipError_t status_word(unsigned** p);
    // LDS bytes per workgroup: the global-exchange staging slot plus an LDS
    // ring of `ring` columns (forward: 2 FP64 coefficients + N-1
    // coefficients + tag per column; adjoint: N+1 coefficients + tag)
    static size_t sweep_lds(int N, int ring) {
        return (size_t)sk_gx_stage_bytes(N, (int)sizeof(R)) +
               (size_t)ring * sk_ring_col_bytes_fwd(N, (int)sizeof(R));
    }
    static size_t adjoint_lds(int N, int ring) {
        return (size_t)sk_gx_stage_bytes(N, (int)sizeof(R)) +
               (size_t)sk_adj_qst_bytes(N, (int)sizeof(R)) +
               (size_t)ring * sk_ring_col_bytes_adj(N, (int)sizeof(R));
    }
    static size_t gram_lds(int dpad) { return (size_t)(192 * (dpad + 1) + 64 * 66) * sizeof(R); }
    static size_t gram_band_lds(int dpad) { return (size_t)(128 * (dpad + 1) + 2 * 64 * 66) * sizeof(R); }
    static size_t gram_pair_lds(int dpad, int max_lx, int max_ly) {
        return ((size_t)64 * 66 + (size_t)(max_lx + max_ly) * (dpad + 1)) * sizeof(R);
    }
    static size_t gram_direct_lds(int dpad, int max_lx, int max_ly) {
        return ((size_t)max_lx * dpad + (size_t)max_ly * (dpad + SkGramDirectPad<R>::value)) *
               sizeof(R);
    }
};

extern template struct SkLaunch<float>;
extern template struct SkLaunch<double>;

// FP64 orders SK_MAX_ORDER < N <= SK_MAX_ORDER_F64 (sk_inst_f64_hi.hip)
hipError_t sk_hi_sweep(const SweepArgs<double>& a, int N, bool interp, bool ckpt, int64_t npairs,
                       int ring, bool gx, hipStream_t st);
hipError_t sk_hi_sweep_pipe(const PipeArgs<double>& a, int N, bool interp, bool ckpt, hipStream_t st);
hipError_t sk_hi_adjoint(const AdjArgs<double>& a, int N, bool interp, int64_t npairs, int ring,
                         bool gx, hipStream_t st);
hipError_t sk_hi_adjoint_pipe(const AdjPipeArgs<double>& a, int N, bool interp, hipStream_t st);
hipError_t sk_hi_plain_poly(const PlainArgs<double>& a, int N, bool interp, hipStream_t st);
hipError_t sk_hi_status_word(unsigned** p);
