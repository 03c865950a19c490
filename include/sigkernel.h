/*
 * sigkernel.h -- C ABI of the MI355X (gfx950) signature-kernel library.
 *
 * Computes signature kernels k(x, y) = <S(x), S(y)> of piecewise-linear paths
 * by solving the Goursat problem d^2k/dsdt = <x'(s), y'(t)> k, k(0,.) =
 * k(.,0) = 1 (Theorem "sigpdetheorem" of Cass, Piatti, Pei, "Numerical
 * Schemes for Signature Kernels") cell by cell on the grid of the two paths,
 * with one of the paper's three schemes:
 *
 *   SK_FD           first-order explicit finite differences on the
 *                   lambda-order dyadic refinement of the grid (Section 2,
 *                   Definition "Dyadic finite differences approximation
 *                   scheme"); `order` = lambda.
 *   SK_POLY_APPROX  polynomial approximation scheme of order N (Section 3.2,
 *                   Definition "Polynomial approximation numerical scheme");
 *                   `order` = N.
 *   SK_POLY_INTERP  polynomial interpolation scheme of order N at the N+1
 *                   Chebyshev extrema (Section 3.3, Definition "Polynomial
 *                   interpolation numerical scheme"); `order` = N.  Exact
 *                   (to the working precision) for cell constants |c| up to
 *                   about 10; a cell beyond the compiled tail makes its
 *                   pair's value and gradient NaN and raises
 *                   SK_STATUS_TAIL_CAP (sigkernel_status).
 *   SK_FD2          second-order explicit finite differences (Remark
 *                   "higherfd", eq. secondexplicitscheme: the first-order
 *                   rule plus c^2/12 times the three known corners) on the
 *                   lambda-order dyadic refinement; `order` = lambda.
 *
 * Paths are given by their points only: the time partition drops out of all
 * schemes once each cell is normalised to the unit square, so only the cell
 * constants c_ij = <x_{i+1} - x_i, y_{j+1} - y_j> enter.  A path with one
 * point (no segment) has kernel 1 with every other path.
 *
 * Conventions of every call:
 *   - Pointers are device pointers unless stated otherwise; all arrays are
 *     dense, row-major, in the element type given by `dtype` (SK_F32: float,
 *     SK_F64: double).
 *   - Calls are asynchronous and ordered on `stream`, except that
 *     sigkernel_pairs / sigkernel_backward(SK_OP_PAIRS) synchronise `stream`
 *     once to upload per-pair descriptors (plans avoid even that).
 *   - No call allocates device memory: the caller passes a workspace `ws` of
 *     `ws_bytes` bytes (size it with sigkernel_*_workspace).  A smaller
 *     workspace is accepted as long as it holds one pair: work is then done
 *     in chunks of pairs.  The workspace must not be used concurrently by
 *     another call.
 *   - The caller owns all buffers.  The library keeps only immutable,
 *     c-independent coefficient tables (host side, built on first use).
 *   - Return value: SK_OK (0) on success, a negative SK_E* code on error (see
 *     sigkernel_error_string and sigkernel_last_error for a description).
 *     Errors in argument checking are reported before any device work is
 *     queued; no C++ exception crosses this interface.
 *
 * Exponent output: kernels of long or large paths exceed the floating-point
 * range.  When K_exp (k_exp) is non-null the value is K * 2^K_exp with K a
 * mantissa in [0.5, 1) in magnitude (or 0); when it is null the value is
 * written directly (and may overflow to inf).
 */
#ifndef SIGKERNEL_H
#define SIGKERNEL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SK_OK 0
#define SK_EINVAL (-1)        /* bad shape, null pointer, order out of range   */
#define SK_EWORKSPACE (-2)    /* workspace smaller than one pair needs          */
#define SK_EUNSUPPORTED (-3)  /* valid request this build does not implement    */
#define SK_EHIP (-4)          /* HIP runtime error (detail in sigkernel_last_error) */

/* schemes */
#define SK_FD 0
#define SK_POLY_APPROX 1
#define SK_POLY_INTERP 2
#define SK_FD2 3

/* element / arithmetic type of paths, outputs and the cell sweep */
#define SK_F64 0
#define SK_F32 1

/* execution algorithm */
#define SK_ALGO_BATCHED 0 /* all pairs of a chunk in one wavefront launch   */
#define SK_ALGO_PLAIN 1   /* one launch per pair, one workgroup sweeping the
                             anti-diagonals (FP64, forward only)             */
#define SK_ALGO_PIPELINE 2 /* the 64-row strips of every pair with several
                             strips spread over co-resident workgroups that
                             hand strip-boundary edges on through global
                             memory (Section 3.2's wavefront over strips),
                             the pairs of a chunk as one job list of
                             strips; for few, long pairs.  Pairs of one
                             strip run batched.  Gram calls build the job
                             lists on the host and copy them into the head
                             of the workspace (synchronising `stream` once);
                             pairs calls run a one-shot plan with the
                             pipeline on.  Polynomial schemes.  Backward
                             (sigkernel_backward, both ops): every pair with
                             several strips runs a pipelined checkpoint
                             sweep and a pipelined adjoint (the strips in
                             reverse order), the pairs of a chunk as one
                             job list; pairs of one strip run batched; the
                             saved-state Gram calls likewise.  A value that
                             could not be completed (a bounded wait gave up)
                             is written as NaN, and so is a gradient        */

/* arithmetic of the increment Gram C_ij = <dx_i, dy_j> */
#define SK_GRAM_NATIVE 0 /* products in the path dtype: a d-term FMA chain per cell for
                            d <= 16 when a pair's increments fit in LDS, otherwise
                            FP32 or FP64 16x16x4 MFMA                                  */
#define SK_GRAM_BF16X3 1 /* SK_F32 only: each increment split into three bf16 parts,
                            the six leading cross products on bf16 MFMA with FP32
                            accumulation (error at the FP32 level, 2^-24 |dx||dy|) */
#define SK_GRAM_MFMA 2   /* products in the path dtype, always on 16x16x4 MFMA       */

/* flags */
#define SK_SYMMETRIC 1 /* backward of a Gram call whose Y is the same array as X:
                          dL/dX sums both contributions and is written to gX
                          (gY is not used and may be NULL)                       */
#define SK_SWEEP_F64 2 /* SK_F32 paths swept in FP64: the points (and a backward's
                          seeds) are promoted to FP64 in the head of the
                          workspace, the cell constants and the sweep run on
                          the FP64 path, and the outputs are rounded to FP32.
                          For conditioning-limited workloads whose FP32 state
                          cannot reach the target accuracy (large |c|, long
                          paths): on this GPU an FP64 FMA issues at the rate
                          of an FP32 one, so the FP64 state costs about 1.5x
                          the FP32 sweep (registers, bytes), less than any
                          compensated FP32 state.  sigkernel_gram,
                          sigkernel_pairs, sigkernel_backward and their
                          workspace queries (which include the FP64 copies);
                          not with SK_GRAM_BF16X3 (the constants are FP64),
                          plans, the saved-state calls or the static-scratch
                          Gram (SK_EUNSUPPORTED)                               */

/* backward operations */
#define SK_OP_GRAM 0
#define SK_OP_PAIRS 1

/* compiled limits */
#define SK_MIN_POLY_ORDER 2
#define SK_MAX_POLY_ORDER 12     /* FP64 sweeps (SK_F64, or SK_F32 with SK_SWEEP_F64) */
#define SK_MAX_POLY_ORDER_F32 8  /* FP32 sweeps                                       */
#define SK_MAX_DYADIC_ORDER 8
#define SK_MAX_BACKWARD_DIM 64

typedef struct sk_params {
    int32_t scheme; /* SK_FD, SK_POLY_APPROX, SK_POLY_INTERP or SK_FD2              */
    int32_t order;  /* N in [SK_MIN_POLY_ORDER, SK_MAX_POLY_ORDER] for the polynomial
                       schemes (SK_MAX_POLY_ORDER_F32 for FP32 sweeps); lambda in
                       [0, SK_MAX_DYADIC_ORDER] for SK_FD, SK_FD2                    */
    int32_t dtype;  /* SK_F32 or SK_F64                                              */
    int32_t algo;   /* SK_ALGO_BATCHED, SK_ALGO_PLAIN or SK_ALGO_PIPELINE            */
    int32_t gram;   /* SK_GRAM_NATIVE, SK_GRAM_BF16X3 or SK_GRAM_MFMA (batched algorithm) */
    int32_t flags;  /* 0, SK_SYMMETRIC and/or SK_SWEEP_F64                            */
    int32_t dyadic; /* polynomial schemes: lambda in [0, SK_MAX_DYADIC_ORDER] runs the
                       scheme on the lambda-order dyadic refinement of the grid (the
                       hybrid method of the remark after Theorem "prop:globalte");
                       its backward sweeps the refined grid and sums dL/dc over
                       each cell's 4^lambda sub-cells, times 4^-lambda, before the
                       contraction; must be 0 for SK_FD, SK_FD2                     */
    int32_t ckpt;   /* checkpoint stride S of the backward (steps per segment of the
                       checkpointing sweep and the adjoint's replay): 0 picks the
                       precision's default (4 for FP32 sweeps, 2 for FP64 sweeps);
                       FP32 sweeps accept 2 or 4, FP64 sweeps (SK_F64 or
                       SK_SWEEP_F64) 2; other values give SK_EUNSUPPORTED, and any
                       nonzero value for SK_FD, SK_FD2 SK_EINVAL.  Every stride
                       computes the same kernel values and gradients up to rounding
                       order; the choice trades adjoint register pressure against
                       checkpoint traffic (see sigkernel_gram_tune)              */
} sk_params;

/*
 * Workspace sizes (bytes) for processing all pairs in one chunk (capped at
 * 160 GiB of the 288 GB of HBM, beyond which work is chunked).  Host-only, no device access.
 * Returns 0 on invalid arguments (see sigkernel_last_error).
 * `backward` != 0 sizes the workspace of sigkernel_backward.
 */
size_t sigkernel_gram_workspace(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                                const sk_params* p, int32_t backward);
/* x_off, y_off: HOST arrays of npairs + 1 point offsets (see sigkernel_pairs). */
size_t sigkernel_pairs_workspace(const int64_t* x_off, const int64_t* y_off, int64_t npairs,
                                 int64_t d, const sk_params* p, int32_t backward);

/*
 * Gram matrix K[a * ny + b] = k(X[a], Y[b]) (paper: the kernel evaluations
 * of Section 1 computed by the chosen scheme; endpoint as in the scheme's
 * definition, the average of the top and right edges of the last cell for
 * the polynomial schemes).
 *   X: nx paths of lx_pts points in R^d, shape (nx, lx_pts, d).
 *   Y: ny paths of ly_pts points, shape (ny, ly_pts, d).
 *   K: nx * ny outputs; K_exp: nx * ny int32 exponents or NULL.
 */
int sigkernel_gram(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                   int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                   void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * sigkernel_gram for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and outputs, with no workspace argument.  The
 * library's own static per-device scratch of SK_STATIC_SCRATCH_BYTES serves
 * as workspace (allocated when the library's code is loaded on a device and
 * held by that device until the process ends); work is chunked to it.  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library call.
 * Batched and plain algorithms (SK_EUNSUPPORTED for SK_ALGO_PIPELINE).
 * SK_EWORKSPACE, before any device work, when one pair needs more than the
 * scratch (e.g. pairs of about 4000 x 4000 FP32 cells and more: use
 * sigkernel_gram with a workspace).  Every call on a device shares that
 * device's scratch, which keeps the last call's contents: calls that overlap
 * on one device (other streams, other host threads) race and must be
 * serialised by the caller.  `stream` must belong to the current device.
 */
#define SK_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int sigkernel_gram_static(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                          int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                          hipStream_t stream);

/*
 * Independent pairs of uneven lengths: k[i] = k(x_i, y_i).
 *   Xcat: all x paths concatenated, shape (x_off[npairs], d); path x_i is
 *   rows [x_off[i], x_off[i+1]).  Likewise Ycat, y_off.  x_off and y_off are
 *   HOST arrays (npairs + 1 entries, non-decreasing, first entry 0); every
 *   path must have at least one point.
 *   k: npairs outputs; k_exp: npairs int32 exponents or NULL.
 */
int sigkernel_pairs(const void* Xcat, const int64_t* x_off, const void* Ycat, const int64_t* y_off,
                    int64_t npairs, int64_t d, const sk_params* p, void* k, int32_t* k_exp,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Reverse-mode derivative of a forward call (polynomial schemes; batched
 * algorithm or strip pipeline): the exact gradient of the computed scheme
 * (discrete adjoint of the cell recursion), for the loss
 * L = sum_i gK[i] * K[i] with K[i] the forward outputs.  SK_OP_PAIRS runs a
 * one-shot plan (tuned configuration of the shape if there is one; with
 * SK_ALGO_PIPELINE every pair of several strips on the pipeline).
 * SK_OP_GRAM with SK_ALGO_PIPELINE (paths of several strips) builds the
 * pairs' descriptors and job lists on the host and copies them into the
 * head of the workspace, synchronising `stream` once; size the workspace
 * with sigkernel_gram_workspace(..., backward = 1) and the same params.
 *   op == SK_OP_GRAM : X, nx, lx_pts, Y, ny, ly_pts as in sigkernel_gram;
 *                      x_off, y_off ignored; gK has nx * ny entries;
 *                      gX (nx, lx_pts, d) and gY (ny, ly_pts, d) are
 *                      overwritten with dL/dX and dL/dY.
 *   op == SK_OP_PAIRS: X, Y are Xcat, Ycat; x_off, y_off HOST offsets; nx is
 *                      npairs (ny, lx_pts, ly_pts ignored); gK has npairs
 *                      entries; gX, gY have the shapes of Xcat, Ycat.
 *   gK_exp: optional int32 exponents, seed gK * 2^gK_exp (so that the loss
 *   can be taken through log K when K itself overflows); NULL means 0.
 *   When X and Y are the same array, SK_SYMMETRIC in p->flags (SK_OP_GRAM,
 *   nx == ny, lx_pts == ly_pts) sums both contributions into gX; without
 *   it the caller sums gX and gY.
 */
int sigkernel_backward(int32_t op, const void* X, const int64_t* x_off, int64_t nx, int64_t lx_pts,
                       const void* Y, const int64_t* y_off, int64_t ny, int64_t ly_pts, int64_t d,
                       const sk_params* p, const void* gK, const int32_t* gK_exp, void* gX,
                       void* gY, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Plans for repeated pairs calls over fixed offsets (the ragged batching of
 * many independent pairs).  A plan fixes on the host: the launch order of
 * the pairs (longest first by wavefront steps, or as given), whether each
 * pair is computed transposed (k(x, y) = k(y, x) holds for every scheme, so
 * the shorter path can take the role whose edges are held in LDS), the
 * grouping of pairs into launches by the LDS size their sweep needs, whether
 * pairs with several 64-row strips run on the strip pipeline (their strips
 * as jobs on co-resident workgroups, which balances the load strip by strip;
 * see SK_ALGO_PIPELINE; in a backward plan their checkpoint sweep and adjoint
 * too), the chunking for a given workspace size and the workspace layout.
 * sigkernel_plan_upload copies the per-pair descriptors into the workspace
 * once (it synchronises `stream`); afterwards sigkernel_plan_forward and
 * sigkernel_plan_backward only queue kernels, with no host synchronisation,
 * copy or allocation, so they may be captured into a HIP graph and replayed
 * (the workspace and every buffer must then stay where they were).
 *   x_off, y_off: HOST offsets as for sigkernel_pairs (copied into the plan).
 *   backward != 0: the plan also serves sigkernel_plan_backward.
 *   ws_bytes: size of the workspace the plan will run with (chunks are sized
 *   to it); 0 lets sigkernel_plan_workspace report the size for one chunk
 *   per LDS class (capped at 160 GiB).
 * sigkernel_plan_tune times configurations of the schedule on the given
 * inputs (a warm-up and two timed runs each, device time on `stream`): the
 * forward for forward plans, forward + backward (dL/dk = 1, buffers the tuner
 * allocates and frees) for backward plans.  It searches in three stages, each
 * from the best so far: pair order x transposition x LDS classes; the
 * strip-pipeline threshold (every threshold that moves a different set of
 * pairs to the pipeline); the checkpoint strides of the precision (backward
 * plans).  Configurations needing more than ws_bytes are skipped
 * (sigkernel_plan_tune_workspace gives the largest any of them needs).  The
 * fastest is kept in the plan, uploaded, and stored in the process's tune
 * cache for plans and one-shot sigkernel_pairs / sigkernel_backward calls of
 * the same shape class (see sigkernel_tune_cache_save).  best_ms (nullable)
 * receives its time.  Every configuration computes the same values up to
 * rounding order.
 * sigkernel_plan_config reports the configuration in use and the number of
 * launches (chunks) of one forward; sigkernel_plan_configure sets it by hand
 * (each flag 0 or 1; pipeline 1 = pairs of two or more strips; the plan must
 * be uploaded again).  sigkernel_plan_get_cfg / sigkernel_plan_set_cfg do
 * the same with the whole configuration (sk_plan_cfg).  The caller owns the plan and destroys
 * it with sigkernel_plan_destroy; a plan may be used from one thread at a
 * time.  Errors: as for sigkernel_pairs; SK_EINVAL for a plan that was not
 * uploaded to this workspace, or a backward on a forward-only plan.
 */
typedef struct sk_plan sk_plan;
int sigkernel_plan_create(const int64_t* x_off, const int64_t* y_off, int64_t npairs, int64_t d,
                          const sk_params* p, int32_t backward, size_t ws_bytes, sk_plan** plan);
size_t sigkernel_plan_workspace(const sk_plan* plan);
int sigkernel_plan_upload(sk_plan* plan, void* ws, size_t ws_bytes, hipStream_t stream);
int sigkernel_plan_forward(const sk_plan* plan, const void* Xcat, const void* Ycat, void* k,
                           int32_t* k_exp, void* ws, size_t ws_bytes, hipStream_t stream);
int sigkernel_plan_backward(const sk_plan* plan, const void* Xcat, const void* Ycat,
                            const void* gk, const int32_t* gk_exp, void* gX, void* gY, void* ws,
                            size_t ws_bytes, hipStream_t stream);
int sigkernel_plan_tune(sk_plan* plan, const void* Xcat, const void* Ycat, void* ws,
                        size_t ws_bytes, hipStream_t stream, double* best_ms);
/*
 * Saved-state forward and backward of a backward plan whose backward runs in
 * one chunk (SK_EWORKSPACE otherwise; sigkernel_plan_config's `launches`
 * counts forward chunks, the backward's chunking follows the same workspace).
 * sigkernel_plan_forward_save computes k (and k_exp) as
 * sigkernel_plan_forward does, through the backward's checkpoint sweep, and
 * leaves the backward's state (cell constants, checkpoints, strip-boundary
 * edges) in the plan's workspace; sigkernel_plan_backward_saved then computes
 * gX, gY exactly as sigkernel_plan_backward would, without recomputing that
 * state.  Between the two calls the workspace must not be used by any other
 * call of this plan (a forward, backward or tune overwrites the state, and
 * the backward then reads the newer state).  Both only queue kernels.
 */
int sigkernel_plan_forward_save(const sk_plan* plan, const void* Xcat, const void* Ycat, void* k,
                                int32_t* k_exp, void* ws, size_t ws_bytes, hipStream_t stream);
int sigkernel_plan_backward_saved(const sk_plan* plan, const void* Xcat, const void* Ycat,
                                  const void* gk, const int32_t* gk_exp, void* gX, void* gY,
                                  void* ws, size_t ws_bytes, hipStream_t stream);
int sigkernel_plan_config(const sk_plan* plan, int32_t* order, int32_t* swap, int32_t* buckets,
                          int32_t* pipeline, int64_t* launches);
int sigkernel_plan_configure(sk_plan* plan, int32_t order, int32_t swap, int32_t buckets,
                             int32_t pipeline, size_t ws_bytes);
typedef struct sk_plan_cfg {
    int32_t longest_first;       /* 1: pairs in decreasing wavefront steps          */
    int32_t transpose;           /* 1: pairs whose second path is longer transposed */
    int32_t lds_classes;         /* 1: a forward launch per LDS class               */
    int32_t pipeline_min_strips; /* k >= 2: pairs of k or more 64-row strips run on
                                    the strip pipeline; 0: none (1 is SK_EINVAL)    */
    int32_t ckpt;                /* checkpoint stride (0: the plan's sk_params.ckpt;
                                    get_cfg reports the stride in use)            */
    int64_t launches;            /* get_cfg only: forward chunks                   */
} sk_plan_cfg;
int sigkernel_plan_get_cfg(const sk_plan* plan, sk_plan_cfg* cfg);
int sigkernel_plan_set_cfg(sk_plan* plan, const sk_plan_cfg* cfg, size_t ws_bytes);
size_t sigkernel_plan_tune_workspace(const sk_plan* plan);
void sigkernel_plan_destroy(sk_plan* plan);

/*
 * Gram tuner (the autotuned batching of uneven and few-pair workloads).
 * sigkernel_gram_tune times, on the given inputs, the forward (backward != 0:
 * forward + backward through the saved state, dL/dK = 1) of every algorithm
 * (SK_ALGO_BATCHED, and SK_ALGO_PIPELINE for polynomial schemes on paths of
 * several strips) and checkpoint stride the precision offers, with the
 * caller's other parameters; writes the fastest parameters to *best and their
 * time to *best_ms (nullable), and stores the choice in the tune cache under
 * the call's key.  It allocates and frees its own device memory and
 * synchronises `stream`.  sigkernel_gram_tuned looks a call's key up without
 * touching the device beyond naming its architecture: *found = 1 and *out =
 * the caller's parameters with the tuned algo and ckpt, or *found = 0 and
 * *out = *p.  Every candidate computes the same values up to rounding order.
 * Errors: as for sigkernel_gram; SK_EUNSUPPORTED for SK_ALGO_PLAIN.
 *
 * Tune cache.  Keys: GPU architecture, call kind (Gram or pairs), scheme,
 * order, dtype, Gram mode, refinement, flags, direction, d, and the shape
 * class (ceil(log2) of the pair counts and of the mean and largest segment
 * counts of each side).  sigkernel_tune_cache_save writes the cache as text
 * (a header line, then one entry a line), through a temporary file renamed
 * over `path`.  sigkernel_tune_cache_load merges a saved cache into the
 * process's: a missing file loads nothing and is not an error; a file whose
 * first line is not the header loads nothing (*skipped = 1); malformed
 * entries are skipped and counted.  *loaded / *skipped (nullable) receive
 * the counts.  sigkernel_tune_cache_clear empties the process's cache.
 */
int sigkernel_gram_tune(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                        int64_t ly_pts, int64_t d, const sk_params* p, int32_t backward,
                        hipStream_t stream, sk_params* best, double* best_ms);
int sigkernel_gram_tuned(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                         const sk_params* p, int32_t backward, sk_params* out, int32_t* found);
int sigkernel_tune_cache_save(const char* path);
int sigkernel_tune_cache_load(const char* path, int32_t* loaded, int32_t* skipped);
void sigkernel_tune_cache_clear(void);

/*
 * Permutation two-sample test on the unbiased MMD^2 (the statistical testing
 * the paper's library offers with its MMD tools; the procedure is the
 * standard permutation test).
 *   Kzz: (m + n) x (m + n) Gram matrix of the pooled paths (first sample
 *   then second), row-major, dtype SK_F32 or SK_F64, device.
 *   perms: nperm rows of m + n int32, device; each row a permutation of
 *   0..m+n-1 whose first m entries form the first group.  Row 0 should be
 *   the identity (the observed split); the caller draws the others.
 *   stats: nperm outputs (dtype), stats[p] = unbiased MMD^2 of split p,
 *   within-group diagonals excluded, accumulated in FP64.
 *   p_value: nullable device double, (1 + #{p >= 1 : stats[p] >= stats[0]})
 *   / nperm.
 * Errors: SK_EINVAL for m < 2, n < 2, nperm < 1, a NULL pointer or a bad
 * dtype; SK_EUNSUPPORTED above 2^20 pooled paths.  The rows of perms are not
 * checked: the first group of a row is the set of its first m entries that
 * lie in 0..m+n-1, every other path is in the second group.
 */
int sigkernel_mmd_permutation(const void* Kzz, int64_t m, int64_t n, const int32_t* perms,
                              int64_t nperm, int32_t dtype, void* stats, double* p_value,
                              hipStream_t stream);

/*
 * Unbiased (U-statistic) MMD^2 between path sets X (nx paths) and Y (ny
 * paths) from the kernel values of one pair list, as sigkernel_pairs
 * computes it: k holds first the nx(nx-1)/2 pairs a < b of X, then the
 * ny(ny-1)/2 pairs a < b of Y, then the nx*ny pairs of X with Y (each group
 * in any order).  Since k is symmetric and the within-set diagonals are left
 * out, MMD^2 = 2/(nx(nx-1)) sum_XX k + 2/(ny(ny-1)) sum_YY k
 * - 2/(nx ny) sum_XY k; the sums are accumulated in FP64 (the statistic of
 * sigkernel_mmd_permutation, for the observed split, from a pair list).
 *   k: device, dtype SK_F32 or SK_F64; out: device, one element of dtype.
 * sigkernel_mmd2_pairs_backward writes gk[i] = dMMD^2/dk_i * gout[0] over the
 * same pair list (gout: device, one element of dtype; gk: device, as k).
 * Both only queue one kernel on `stream`; the caller owns every buffer.
 * Errors: SK_EINVAL for nx < 2, ny < 2, a NULL pointer or a bad dtype;
 * SK_EUNSUPPORTED above 2^24 paths in a set.
 */
int sigkernel_mmd2_pairs(const void* k, int64_t nx, int64_t ny, int32_t dtype, void* out,
                         hipStream_t stream);
int sigkernel_mmd2_pairs_backward(const void* gout, int64_t nx, int64_t ny, int32_t dtype, void* gk,
                                  hipStream_t stream);

/*
 * Forward and backward of a Gram call with the backward's state kept in
 * between (trading memory for the recomputation sigkernel_backward does).
 * sigkernel_gram_save computes K (and K_exp) like sigkernel_gram with the
 * polynomial scheme `p` and additionally leaves in `state` the skewed cell
 * constants, the wavefront checkpoints and the strip-boundary edges of every
 * pair; `state` must hold sigkernel_gram_state_size bytes (one region for
 * all pairs, no chunking; the caller owns it).
 * sigkernel_gram_backward_saved then computes gX, gY exactly as
 * sigkernel_backward(SK_OP_GRAM, ...) would, for the same X, Y and params,
 * from that state (which it also uses as scratch).  Calling it with a state
 * not produced by sigkernel_gram_save for the same arguments gives undefined
 * results.  Errors as for sigkernel_backward; SK_EWORKSPACE when the state
 * is too small.  With SK_ALGO_PIPELINE (paths of several strips) the state
 * also holds the pairs' descriptors and job lists, which sigkernel_gram_save
 * copies in (synchronising `stream` once); both calls take the same params.
 */
size_t sigkernel_gram_state_size(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                                 const sk_params* p);
int sigkernel_gram_save(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                        int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                        void* state, size_t state_bytes, hipStream_t stream);
int sigkernel_gram_backward_saved(const void* X, int64_t nx, int64_t lx_pts, const void* Y,
                                  int64_t ny, int64_t ly_pts, int64_t d, const sk_params* p,
                                  const void* gK, const int32_t* gK_exp, void* gX, void* gY,
                                  void* state, size_t state_bytes, hipStream_t stream);

/*
 * The increment Gram matrices of a Gram call: C[((a * ny + b) * lx + i) * ly + j]
 * = <X[a, i+1] - X[a, i], Y[b, j+1] - Y[b, j]> with lx = lx_pts - 1,
 * ly = ly_pts - 1 (the constants C_ij of the schemes with unit time steps),
 * computed by the 64-row-block MFMA kernel of the sweeps, in p->dtype with
 * p->gram arithmetic (p->scheme, p->order are not used).  Needs the forward
 * workspace of the same call with scheme SK_POLY_APPROX.
 */
int sigkernel_cell_constants(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                             int64_t ly_pts, int64_t d, const sk_params* p, void* C, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/*
 * Kernel timing for measurement (diagnostics).  While enabled, every kernel
 * launch of the library is bracketed by two HIP events recorded on its
 * stream.  sigkernel_profile_enable(on) clears the records and switches
 * collection on or off.  sigkernel_profile_read(name, &ms, &n) waits for the
 * recorded events of kernels called `name` ("gram", "sweep", "sweep_ckpt",
 * "adjoint", "contract", "reduce", "fd_sweep", "plain") and returns their
 * summed elapsed time in milliseconds and the launch count.  Host memory
 * for the records grows with the number of launches until the next enable.
 */
int sigkernel_profile_enable(int32_t on);
int sigkernel_profile_read(const char* name, double* total_ms, int64_t* launches);

/*
 * Device status (diagnostics).  Kernels raise bits in a per-device status
 * word, which keeps them until cleared:
 *   SK_STATUS_TAIL_CAP   an interpolation cell needed more tail rows than the
 *                        compiled cap (cells with |c| beyond about 10; see
 *                        SK_POLY_INTERP): its pair's value (and gradient) is
 *                        NaN.
 *   SK_STATUS_WAIT_ABORT a bounded wait of the strip pipeline gave up: the
 *                        values (gradients) it could not complete are NaN.
 * sigkernel_status synchronises `stream`, then writes the bits raised on the
 * current device since the last clear to *flags, and clears them when
 * `clear` != 0.  Bits are shared by every stream and call on the device.
 */
#define SK_STATUS_TAIL_CAP 1u
#define SK_STATUS_WAIT_ABORT 2u
int sigkernel_status(hipStream_t stream, int32_t clear, uint32_t* flags);
/*
 * Polls a strip-pipeline wait makes before it gives up (diagnostics, for
 * tests of that path; process-wide, read when a call queues its kernels).
 * 0 restores the default of 2^24 polls (about ten seconds).  SK_EINVAL for a
 * negative count.
 */
int sigkernel_set_spin_limit(int32_t polls);

/*
 * The interpolation scheme's tail tables (diagnostics; host only).  The
 * interpolation of u^r at the order-N Chebyshev extrema, in the factorial
 * basis: rs[n * SK_TAIL_TABLE + t] = R[n][r] n!/r! for tail row r = N+1+t,
 * t < SK_TAIL_TABLE (rs holds (N + 1) * SK_TAIL_TABLE doubles); rmax[t] =
 * max_n |rs[n][t]| and cmax[t], the |c| up to which the projected rows from
 * r on shrink at least by half per row (SK_TAIL_TABLE + 1 doubles each);
 * *tail_cap = the longest tail compiled for `dtype`.  A cell folds tail rows
 * while 2 rmax[t] (|A^P_r| + |A^Q_r|) exceeds the working precision times
 * its corner values or |c| > cmax[t], for at most *tail_cap rows.
 * SK_EINVAL for an order outside [SK_MIN_POLY_ORDER, 12] or a NULL pointer.
 */
#define SK_TAIL_TABLE 20
int sigkernel_interp_table(int32_t order, int32_t dtype, double* rs, double* rmax, double* cmax,
                           int32_t* tail_cap);

/* Static description of a status code. */
const char* sigkernel_error_string(int status);
/* Detail of the last error on the calling thread ("" if none). */
const char* sigkernel_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIGKERNEL_H */
