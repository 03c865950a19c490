// C ABI of the signature-kernel library: argument checking, coefficient
// tables, workspace planning and chunked dispatch of the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sigkernel.h"
#include "sk_launch.h"

// Static per-device scratch of sigkernel_gram_static (the workspace of
// callers that cannot allocate).  Host code never uses this name as an
// address: it reads the array's device address once per device with
// hipGetSymbolAddress (scratch_of_current_device) and passes that on.
static __device__ __align__(256) unsigned char scratch[SK_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(SK_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define SK_TRY_HIP(expr, where)               \
    do {                                      \
        hipError_t e__ = (expr);              \
        if (e__ != hipSuccess) return hip_fail(e__, where); \
    } while (0)

// ---------------------------------------------------------------------------
// optional per-kernel timing with HIP events recorded on the launch stream
// ---------------------------------------------------------------------------
struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
};
std::atomic<bool> g_prof{false};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;

struct ProfScope {
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
        if (!g_prof.load(std::memory_order_relaxed)) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);  // profiling only: a failed record times nothing
    }
    ~ProfScope() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof_recs.push_back({name, a, b});
    }
};

#define SK_LAUNCH(name, st, expr, where)      \
    do {                                      \
        ProfScope ps__(name, st);             \
        SK_TRY_HIP(expr, where);              \
    } while (0)

constexpr int64_t kAlign = 256;
constexpr size_t kDefaultCap = (size_t)160 << 30;  // bytes of one default chunk (of 288 GB HBM)
// polls of a strip-pipeline wait before it gives up (about ten seconds);
// sigkernel_set_spin_limit changes it (diagnostics)
constexpr int kPipeSpinLimit = 1 << 24;
std::atomic<int> g_spin_limit{kPipeSpinLimit};

inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// interpolation tables (c-independent, built in FP64 on the host)
// ---------------------------------------------------------------------------
// Interpolation of u^r at the Chebyshev extrema of [0, 1]: the degree-N
// interpolant's monomial coefficients R[n][r], from a partial-pivoting LU
// solve of the Vandermonde system.  Scaled to the factorial basis:
// Rs[n][r] = R[n][r] n! / r!.
static_assert(SK_TMAX == SK_TAIL_TABLE, "the exported tail table has SK_TMAX rows");
struct InterpTableF64 {
    double rs[SK_NMAX + 1][SK_TMAX];
    double rmax[SK_TMAX + 1];
    double cmax[SK_TMAX + 1];
};

double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

void lu_solve_inplace(std::vector<double> a, int M, std::vector<double>& b) {
    std::vector<int> piv(M);
    for (int k = 0; k < M; ++k) {
        int p = k;
        for (int i = k + 1; i < M; ++i)
            if (std::fabs(a[i * M + k]) > std::fabs(a[p * M + k])) p = i;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < M; ++j) std::swap(a[k * M + j], a[p * M + j]);
        for (int i = k + 1; i < M; ++i) {
            a[i * M + k] /= a[k * M + k];
            for (int j = k + 1; j < M; ++j) a[i * M + j] -= a[i * M + k] * a[k * M + j];
        }
    }
    for (int k = 0; k < M; ++k) std::swap(b[k], b[piv[k]]);
    for (int i = 1; i < M; ++i)
        for (int j = 0; j < i; ++j) b[i] -= a[i * M + j] * b[j];
    for (int i = M - 1; i >= 0; --i) {
        for (int j = i + 1; j < M; ++j) b[i] -= a[i * M + j] * b[j];
        b[i] /= a[i * M + i];
    }
}

// Rows of the tail looked at when bounding how fast the projected rows
// shrink: far enough that the ratio has settled (it tends to 1/(r+1)).
constexpr int kTailHorizon = 160;

InterpTableF64 build_interp_table(int N) {
    const int M = N + 1;
    std::vector<double> u(M), V(M * M);
    for (int m = 0; m <= N; ++m) u[m] = 0.5 * std::cos(M_PI * m / N) + 0.5;
    for (int m = 0; m <= N; ++m)
        for (int n = 0; n <= N; ++n) V[m * M + n] = std::pow(u[m], n);
    InterpTableF64 t;
    std::memset(&t, 0, sizeof(t));
    // q[k] = max_n |R[n][r]| n! for r = N+1+k (the projection weight without
    // its 1/r!, which would underflow this far out)
    std::vector<double> q(kTailHorizon + 1, 0.0);
    for (int k = 0; k <= kTailHorizon; ++k) {
        const int r = N + 1 + k;
        std::vector<double> b(M);
        for (int m = 0; m <= N; ++m) b[m] = std::pow(u[m], r);
        lu_solve_inplace(V, M, b);
        for (int n = 0; n <= N; ++n) {
            q[k] = std::max(q[k], std::fabs(b[n]) * fact(n));
            if (k < SK_TMAX) t.rs[n][k] = b[n] * fact(n) / fact(r);
        }
        if (k <= SK_TMAX) t.rmax[k] = q[k] / fact(r);
    }
    // rho_k: largest growth factor of the weight from one row to the next
    // over rows k, k+1, ... (5% margin for the rounding of the solves);
    // cmax[k] = (k + 2) / (2 rho_k), see the decision rule of the device map
    for (int k = 0; k <= SK_TMAX; ++k) {
        double rho = 0.0;
        for (int j = k; j < kTailHorizon; ++j)
            rho = std::max(rho, q[j + 1] / (q[j] * (double)(N + 2 + j)));
        t.cmax[k] = (k + 2) / (2.0 * 1.05 * rho);
    }
    return t;
}

template <typename R>
const SkTab<R>& interp_table(int N) {
    static std::once_flag once[SK_NMAX + 1];
    static SkTab<R> tabs[SK_NMAX + 1];
    std::call_once(once[N], [N]() {
        InterpTableF64 t = build_interp_table(N);
        SkTab<R>& o = tabs[N];
        std::memset(&o, 0, sizeof(o));
        for (int n = 0; n <= N; ++n)
            for (int k = 0; k < SK_TMAX; ++k) o.rs[n][k] = (R)t.rs[n][k];
        for (int k = 0; k <= SK_TMAX; ++k) {
            o.rmax[k] = (R)t.rmax[k];
            o.cmax[k] = (R)t.cmax[k];
        }
        for (int m = 0; m < SK_IFA; ++m) o.ifa[m] = (R)(1.0 / fact(m));
    });
    return tabs[N];
}

template <typename R>
SkTab<R> table_for(const sk_params& p) {
    if (p.scheme == SK_POLY_INTERP) return interp_table<R>(p.order);
    SkTab<R> t;
    std::memset(&t, 0, sizeof(t));
    return t;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
bool is_fd(const sk_params& p) { return p.scheme == SK_FD || p.scheme == SK_FD2; }

int check_params(const sk_params* p, bool backward) {
    if (!p) return fail(SK_EINVAL, "params is NULL");
    if (p->dtype != SK_F32 && p->dtype != SK_F64) return fail(SK_EINVAL, "dtype %d", p->dtype);
    if (p->algo != SK_ALGO_BATCHED && p->algo != SK_ALGO_PLAIN && p->algo != SK_ALGO_PIPELINE)
        return fail(SK_EINVAL, "algo %d", p->algo);
    if (is_fd(*p)) {
        if (p->order < 0) return fail(SK_EINVAL, "dyadic order %d < 0", p->order);
        if (p->order > SK_MAX_DYADIC_ORDER)
            return fail(SK_EUNSUPPORTED, "dyadic order %d > %d", p->order, SK_MAX_DYADIC_ORDER);
        if (backward) return fail(SK_EUNSUPPORTED, "backward of the finite-difference scheme");
        if (p->dyadic != 0)
            return fail(SK_EINVAL, "finite differences take their refinement from `order`");
    } else if (p->scheme == SK_POLY_APPROX || p->scheme == SK_POLY_INTERP) {
        if (p->dyadic < 0) return fail(SK_EINVAL, "dyadic refinement %d < 0", p->dyadic);
        if (p->dyadic > SK_MAX_DYADIC_ORDER)
            return fail(SK_EUNSUPPORTED, "dyadic refinement %d > %d", p->dyadic, SK_MAX_DYADIC_ORDER);
        if (p->order < SK_MIN_POLY_ORDER)
            return fail(SK_EINVAL, "polynomial order %d < %d", p->order, SK_MIN_POLY_ORDER);
        if (p->order > SK_MAX_POLY_ORDER)
            return fail(SK_EUNSUPPORTED, "polynomial order %d > %d", p->order, SK_MAX_POLY_ORDER);
        if (p->dtype == SK_F32 && !(p->flags & SK_SWEEP_F64) && p->order > SK_MAX_POLY_ORDER_F32)
            return fail(SK_EUNSUPPORTED, "FP32 sweeps are compiled for orders up to %d (FP64 sweeps to %d)",
                        SK_MAX_POLY_ORDER_F32, SK_MAX_POLY_ORDER);
    } else {
        return fail(SK_EINVAL, "scheme %d", p->scheme);
    }
    if (p->algo == SK_ALGO_PLAIN) {
        if (p->dtype != SK_F64) return fail(SK_EUNSUPPORTED, "the plain algorithm is FP64 only");
        if (backward) return fail(SK_EUNSUPPORTED, "the plain algorithm is forward only");
    }
    if (p->algo == SK_ALGO_PIPELINE && is_fd(*p))
        return fail(SK_EUNSUPPORTED, "the strip pipeline runs the polynomial schemes");
    if (p->gram != SK_GRAM_NATIVE && p->gram != SK_GRAM_BF16X3 && p->gram != SK_GRAM_MFMA)
        return fail(SK_EINVAL, "gram mode %d", p->gram);
    if (p->gram == SK_GRAM_BF16X3 && p->dtype != SK_F32)
        return fail(SK_EUNSUPPORTED, "the bf16 split Gram is for SK_F32 paths");
    if (p->gram == SK_GRAM_BF16X3 && p->algo == SK_ALGO_PLAIN)
        return fail(SK_EUNSUPPORTED, "the bf16 split Gram is not a plain-algorithm mode");
    if (p->flags & ~(SK_SYMMETRIC | SK_SWEEP_F64)) return fail(SK_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->ckpt != 0) {
        const bool f64sweep = p->dtype == SK_F64 || (p->flags & SK_SWEEP_F64);
        if (p->ckpt < 0) return fail(SK_EINVAL, "checkpoint stride %d < 0", p->ckpt);
        if (is_fd(*p)) return fail(SK_EINVAL, "the finite-difference schemes have no checkpoint stride");
        if (f64sweep ? p->ckpt != 2 : (p->ckpt != 2 && p->ckpt != 4))
            return fail(SK_EUNSUPPORTED, "checkpoint stride %d (compiled: %s)", p->ckpt,
                        f64sweep ? "2 for FP64 sweeps" : "2 or 4 for FP32 sweeps");
    }
    if (p->flags & SK_SWEEP_F64) {
        if (p->dtype != SK_F32) return fail(SK_EINVAL, "SK_SWEEP_F64 applies to SK_F32 paths");
        if (p->gram == SK_GRAM_BF16X3)
            return fail(SK_EUNSUPPORTED, "SK_SWEEP_F64 computes the cell constants in FP64 (no bf16 split)");
    }
    return SK_OK;
}

// SK_SYMMETRIC: Y is X, so both gradient contributions go to gX (the
// reductions accumulate, x part then y part, on the same stream).
int check_symmetric(const sk_params& p, int32_t op, const void* X, int64_t nx, int64_t lx_pts,
                    const void* Y, int64_t ny, int64_t ly_pts, void* gX, void** gY) {
    if (!(p.flags & SK_SYMMETRIC)) return SK_OK;
    if (op != SK_OP_GRAM) return fail(SK_EINVAL, "SK_SYMMETRIC applies to Gram calls");
    if (X != Y || nx != ny || lx_pts != ly_pts)
        return fail(SK_EINVAL, "SK_SYMMETRIC needs Y to be the same array as X");
    *gY = gX;
    return SK_OK;
}

// K padding of the increments for the Gram MFMAs: 4 (16x16x4), 16 (bf16 16x16x16)
int gram_dpad(const sk_params& p, int64_t d) {
    return p.gram == SK_GRAM_BF16X3 ? (int)((d + 15) / 16 * 16) : (int)((d + 3) / 4 * 4);
}

int check_dims(int64_t d, bool backward) {
    if (d < 1) return fail(SK_EINVAL, "d = %lld < 1", (long long)d);
    if (backward && d > SK_MAX_BACKWARD_DIM)
        return fail(SK_EUNSUPPORTED, "backward needs d <= %d", SK_MAX_BACKWARD_DIM);
    return SK_OK;
}

int check_len(int64_t pts, int lam, const char* what) {
    if (pts < 1) return fail(SK_EINVAL, "%s has %lld points (need >= 1)", what, (long long)pts);
    if (((pts - 1) << lam) > (int64_t)1 << 24)
        return fail(SK_EUNSUPPORTED, "%s: %lld segments (refined) exceed 2^24", what,
                    (long long)((pts - 1) << lam));
    return SK_OK;
}

int check_offsets(const int64_t* off, int64_t npairs, int lam, const char* what) {
    if (!off) return fail(SK_EINVAL, "%s offsets are NULL", what);
    if (off[0] != 0) return fail(SK_EINVAL, "%s offsets must start at 0", what);
    for (int64_t i = 0; i < npairs; ++i) {
        int64_t n = off[i + 1] - off[i];
        int rc = check_len(n, lam, what);
        if (rc) return rc;
    }
    return SK_OK;
}

// Wavefront steps of one pair, in 64 bits (the kernels index steps in 32
// bits): computed for both orientations, since plans may transpose a pair.
constexpr int64_t kMaxSteps = (int64_t)1 << 30;
int64_t steps64(int64_t lx, int64_t ly) {
    if (lx <= 0 || ly <= 0) return 0;
    const int64_t W = std::min<int64_t>(lx, SK_LANES), nstrips = (lx + SK_LANES - 1) / SK_LANES;
    const int64_t Tp = std::max(ly, W), rlast = (lx - 1) - (nstrips - 1) * SK_LANES;
    return (nstrips - 1) * Tp + (ly - 1) + rlast + 1;
}
int check_geom(int64_t lx_pts, int64_t ly_pts, int lam) {
    const int64_t lx = (lx_pts - 1) << lam, ly = (ly_pts - 1) << lam;
    const int64_t st = std::max(steps64(lx, ly), steps64(ly, lx));
    if (st > kMaxSteps)
        return fail(SK_EUNSUPPORTED,
                    "a pair of %lld x %lld (refined) segments takes %lld wavefront steps (limit 2^30)",
                    (long long)lx, (long long)ly, (long long)st);
    return SK_OK;
}
// Both paths of a Gram call: point counts, refined lengths, pair geometry.
int check_gram_geom(int64_t lx_pts, int64_t ly_pts, int lam) {
    int rc;
    if ((rc = check_len(lx_pts, lam, "x")) || (rc = check_len(ly_pts, lam, "y"))) return rc;
    return check_geom(lx_pts, ly_pts, lam);
}
// Every pair of a pair list (host offsets).
int check_pairs_geom(const int64_t* x_off, const int64_t* y_off, int64_t npairs, int lam) {
    int rc;
    if ((rc = check_offsets(x_off, npairs, lam, "x")) || (rc = check_offsets(y_off, npairs, lam, "y")))
        return rc;
    for (int64_t i = 0; i < npairs; ++i)
        if ((rc = check_geom(x_off[i + 1] - x_off[i], y_off[i + 1] - y_off[i], lam))) return rc;
    return SK_OK;
}

size_t esize(const sk_params& p) { return p.dtype == SK_F32 ? 4 : 8; }
// dyadic refinement of the grid: `order` for finite differences, `dyadic`
// for the polynomial schemes (the hybrid method)
int lam_of(const sk_params& p) { return is_fd(p) ? p.order : p.dyadic; }
// LDS budgets of the strip-boundary rings; pairs that would need more pass
// their edges through the global exchange.  The forward sweep (about five
// waves per SIMD by registers) loses occupancy to its ring beyond ~16 KiB;
// the adjoint (two waves per SIMD, one with the exchange code) only when the
// ring would leave fewer than four waves per CU.
constexpr int kGxFwdLds = 16 << 10;
constexpr int kGxAdjLds = 38 << 10;
int gx_cols_fwd(const sk_params& p) {
    return std::max(SK_GX_MIN_COLS, kGxFwdLds / sk_ring_col_bytes_fwd(p.order, (int)esize(p)));
}
int gx_cols_adj(const sk_params& p) {
    return std::max(SK_GX_MIN_COLS, kGxAdjLds / sk_ring_col_bytes_adj(p.order, (int)esize(p)));
}
// All column counts below are of the (possibly refined) grid: ly segments
// of y become ly << lam_of(p) columns.
int grid_cols(const sk_params& p, int ly) { return ly << lam_of(p); }
// words per column of a pair's global exchange records (0: none needed)
int xb_words_of(const sk_params& p, int ly) {
    if (is_fd(p)) return 0;
    return grid_cols(p, ly) > std::min(gx_cols_fwd(p), gx_cols_adj(p))
               ? sk_gx_words(p.order, (int)esize(p)) : 0;
}
// LDS ring columns a pair with ly segments of y needs (0: global exchange)
int ring_fwd_of(const sk_params& p, int ly) {
    const int c = grid_cols(p, ly);
    return (!is_fd(p) && c > gx_cols_fwd(p)) ? 0 : c;
}
int ring_adj_of(const sk_params& p, int ly) {
    const int c = grid_cols(p, ly);
    return c > gx_cols_adj(p) ? 0 : c;
}
// Checkpoint stride S of the backward: p.ckpt when set (validated), else the
// precision's default.  Shorter segments shorten the adjoint's replay state
// (fewer registers, more waves per SIMD) at the cost of more checkpoints.
int ckpt_stride(const sk_params& p) {
    if (p.ckpt > 0) return p.ckpt;
    return p.dtype == SK_F32 ? SkCkptStride<float>::value : SkCkptStride<double>::value;
}

// ---------------------------------------------------------------------------
// workspace layout of one chunk
// ---------------------------------------------------------------------------
struct Layout {
    int64_t cskew, gskew, gcu, ck, ce, qb, qe, dxp, dyp, kbuf, kexp, desc, xb, pg, total;
};

// Region sizes for P pairs with total per-array element counts `z` (sum over
// the chunk's pairs).
Layout layout_for(const SkPairSizes& z, int64_t P, size_t es, bool backward, bool list, int N) {
    Layout L;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off += align_up(bytes);
        return o;
    };
    L.cskew = take(z.c * (int64_t)es);
    L.gskew = backward ? take(z.c * (int64_t)es) : off;
    L.gcu = backward ? take(z.cu * (int64_t)es) : off;  // refined grids only
    L.ck = backward ? take(z.ck * (int64_t)es) : off;
    L.ce = backward ? take(z.ce * 4) : off;
    L.qb = backward ? take(z.qb * (int64_t)es) : off;
    L.qe = backward ? take(z.qe * 4) : off;
    L.dxp = backward ? take(z.dx * (int64_t)es) : off;
    L.dyp = backward ? take(z.dy * (int64_t)es) : off;
    L.kbuf = backward ? take(P * (int64_t)es) : off;
    L.kexp = backward ? take(P * 4) : off;
    L.desc = list ? take(P * (int64_t)sizeof(SkPairDesc)) : off;
    L.xb = take(z.xb * 4);
    L.pg = take((z.pg + 1) * 4);  // strip-pipeline progress counters, then the abort flag
    L.total = off;
    return L;
}

SkPairSizes scale(const SkPairSizes& z, int64_t P) {
    SkPairSizes o = {z.c * P, z.ck * P, z.ce * P, z.qb * P, z.qe * P,
                     z.dx * P, z.dy * P, z.xb * P, z.pg * P, z.cu * P};
    return o;
}

SkPairSizes add(const SkPairSizes& a, const SkPairSizes& b) {
    SkPairSizes o = {a.c + b.c, a.ck + b.ck, a.ce + b.ce, a.qb + b.qb, a.qe + b.qe,
                     a.dx + b.dx, a.dy + b.dy, a.xb + b.xb, a.pg + b.pg, a.cu + b.cu};
    return o;
}

// Gram: largest chunk of uniform pairs that fits in `bytes`.
int64_t gram_chunk(const SkPairSizes& per, int64_t npairs, size_t es, bool backward,
                   size_t bytes, int N) {
    if (npairs <= 0) return 0;
    int64_t one = layout_for(per, 1, es, backward, false, N).total;
    if ((size_t)one > bytes) return 0;
    int64_t P = std::min<int64_t>(npairs, (int64_t)(bytes / (size_t)std::max<int64_t>(1, one)) + 1);
    while (P > 1 && (size_t)layout_for(scale(per, P), P, es, backward, false, N).total > bytes) {
        int64_t per_b = layout_for(scale(per, P), P, es, backward, false, N).total / P + 1;
        int64_t guess = (int64_t)(bytes / (size_t)per_b);
        P = std::max<int64_t>(1, std::min(P - 1, guess));
    }
    return P;
}

hipError_t lds_limit(size_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    *out = (size_t)v;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// LDS budget of the increment Gram kernels: a whole pair's increments
// resident in one workgroup (direct FMA chain for d <= 16 in the path dtype,
// else MFMA), else one wave per strip (FMA chain) or one workgroup per strip
// band (MFMA), else 64-row blocks.
constexpr size_t kGramPairLds = 64 << 10;

template <typename R>
hipError_t launch_gram(const GramArgs<R>& ga, int64_t P, int max_nsteps_pad, int max_lx,
                       int max_ly, bool direct, hipStream_t st) {
    // a strip's skewed rows: Tp = max(ly, min(lx, 64)), the last strip up to 127 more
    const int rows = std::max(max_ly << ga.lam, SK_LANES) + 2 * SK_LANES;
    const int strips = ((max_lx << ga.lam) + SK_LANES - 1) / SK_LANES;
    if (direct && !ga.split && ga.dpad <= SK_GRAM_DIRECT_DMAX &&
        SkLaunch<R>::gram_direct_lds(ga.dpad, max_lx, max_ly) <= kGramPairLds)
        return SkLaunch<R>::gram_direct(ga, max_lx, max_ly, P, st);
    // pairs too long for one workgroup's LDS: the FMA chain per strip (the
    // skewed rows' HBM writes bound it) for d <= 32 in the path dtype (d = 32
    // block: 74 ms FP32, 139 ms FP64, against 106 ms for the FP32 MFMA strip
    // bands and 730 ms for the FP64 64-row MFMA blocks); otherwise MFMA strip
    // bands where their tiles fit in LDS (the BF16 split, FP32 d <= 60), else
    // 64-row blocks
    const bool pair_fits = SkLaunch<R>::gram_pair_lds(ga.dpad, max_lx, max_ly) <= kGramPairLds;
    if (direct && !ga.split &&
        (ga.dpad <= SK_GRAM_DIRECT_DMAX || (ga.dpad <= SK_GRAM_STRIP_DMAX && !pair_fits)))
        return SkLaunch<R>::gram_strip(ga, strips, rows, P, st);
    if (pair_fits) return SkLaunch<R>::gram_pair(ga, max_lx, max_ly, P, st);
    if (ga.dpad <= 60 && SkLaunch<R>::gram_band_lds(ga.dpad) <= kGramPairLds)
        return SkLaunch<R>::gram_band(ga, strips, rows, P, st);
    return SkLaunch<R>::gram(ga, max_nsteps_pad / 64, P, st);
}

template <typename R>
int run_chunk_forward(const sk_params& p, const R* X, const R* Y, int64_t d, const SkPairSrc& src,
                      int64_t P, int max_nsteps_pad, int max_lx, int max_ly, int ring, char* ws,
                      const Layout& L, R* K, int32_t* Kexp, hipStream_t st) {
    const bool interp = p.scheme == SK_POLY_INTERP;
    const int lam = lam_of(p);
    R* cskew = reinterpret_cast<R*>(ws + L.cskew);
    GramArgs<R> ga;
    ga.X = X; ga.Y = Y; ga.d = d; ga.dpad = gram_dpad(p, d); ga.lam = lam;
    ga.src = src; ga.cskew = cskew; ga.maxc = nullptr; ga.split = p.gram == SK_GRAM_BF16X3;
    SK_LAUNCH("gram", st, launch_gram(ga, P, max_nsteps_pad, max_lx, max_ly, p.gram == SK_GRAM_NATIVE, st), "increment Gram");
    if (is_fd(p)) {
        FdArgs<R> fa;
        fa.src = src; fa.lam = lam; fa.cskew = cskew; fa.K = K; fa.Kexp = Kexp;
        fa.second = p.scheme == SK_FD2;
        SK_LAUNCH("fd_sweep", st, SkLaunch<R>::sweep_fd(fa, P, max_ly << lam, st), "finite-difference sweep");
    } else {
        SweepArgs<R> sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.src = src; sa.cskew = cskew; sa.tab = table_for<R>(p);
        sa.K = K; sa.Kexp = Kexp;
        sa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
        sa.gx_cols = gx_cols_fwd(p);
        sa.lam = lam; sa.S = ckpt_stride(p);
        SK_LAUNCH("sweep", st, SkLaunch<R>::sweep(sa, p.order, interp, false, P, ring,
                                                  grid_cols(p, max_ly) > sa.gx_cols, st), "sweep");
    }
    return SK_OK;
}

// Forward of a chunk of strip-pipeline pairs: increment Gram, then the
// pipelined sweep over the chunk's job list (strips on co-resident waves).
template <typename R>
int run_chunk_forward_pipe(const sk_params& p, const R* X, const R* Y, int64_t d,
                           const SkPairSrc& src, int64_t P, int max_nsteps_pad, int max_lx,
                           int max_ly, const int2* jobs, int64_t njobs, char* ws, const Layout& L,
                           R* K, int32_t* Kexp, hipStream_t st) {
    R* cskew = reinterpret_cast<R*>(ws + L.cskew);
    GramArgs<R> ga;
    ga.X = X; ga.Y = Y; ga.d = d; ga.dpad = gram_dpad(p, d); ga.lam = lam_of(p);
    ga.src = src; ga.cskew = cskew; ga.maxc = nullptr; ga.split = p.gram == SK_GRAM_BF16X3;
    SK_LAUNCH("gram", st, launch_gram(ga, P, max_nsteps_pad, max_lx, max_ly, p.gram == SK_GRAM_NATIVE, st),
              "increment Gram");
    // progress counters of every pair, then the abort flag: zero
    const int64_t npg = (L.total - L.pg) / 4;
    SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(ws + L.pg), npg, st), "fill");
    PipeArgs<R> pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.cskew = cskew; pa.tab = table_for<R>(p);
    pa.K = K; pa.Kexp = Kexp;
    pa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
    pa.progress = reinterpret_cast<int*>(ws + L.pg);
    pa.abort = reinterpret_cast<int*>(ws + L.total) - 1;
    pa.spin_limit = g_spin_limit.load();
    pa.desc = src.desc; pa.jobs = jobs; pa.njobs = njobs; pa.lam = lam_of(p);
    pa.S = ckpt_stride(p);
    SK_LAUNCH("sweep_pipe", st, SkLaunch<R>::sweep_pipe(pa, p.order, p.scheme == SK_POLY_INTERP, false, st),
              "pipelined strip sweep");
    return SK_OK;
}

template <typename R>
int run_contract(const R* X, const R* Y, int64_t d, const SkPairSrc& src, int64_t P,
                 int max_strips, char* ws, const Layout& L, hipStream_t st, int64_t gsrc = -1);

// Backward of a chunk of strip-pipeline pairs, first half: increment Gram
// and the pipelined checkpoint sweep over the forward job list (kernel
// values to K).
template <typename R>
int run_chunk_prepare_pipe(const sk_params& p, const R* X, const R* Y, int64_t d,
                           const SkPairSrc& src, int64_t P, int max_nsteps_pad, int max_lx,
                           int max_ly, const int2* jobs_fwd, int64_t njobs, char* ws,
                           const Layout& L, R* K, int32_t* Kexp, hipStream_t st) {
    const bool interp = p.scheme == SK_POLY_INTERP;
    R* cskew = reinterpret_cast<R*>(ws + L.cskew);
    GramArgs<R> ga;
    ga.X = X; ga.Y = Y; ga.d = d; ga.dpad = gram_dpad(p, d); ga.lam = lam_of(p);
    ga.src = src; ga.cskew = cskew; ga.maxc = nullptr; ga.split = p.gram == SK_GRAM_BF16X3;
    SK_LAUNCH("gram", st, launch_gram(ga, P, max_nsteps_pad, max_lx, max_ly, p.gram == SK_GRAM_NATIVE, st),
              "increment Gram");
    const int64_t npg = (L.total - L.pg) / 4;  // progress counters, then the abort flag
    int* prog = reinterpret_cast<int*>(ws + L.pg);
    int* abrt = reinterpret_cast<int*>(ws + L.total) - 1;
    SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(prog), npg, st), "fill");
    PipeArgs<R> pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.cskew = cskew; pa.tab = table_for<R>(p);
    pa.K = K; pa.Kexp = Kexp;
    pa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
    pa.progress = prog; pa.abort = abrt; pa.spin_limit = g_spin_limit.load();
    pa.desc = src.desc; pa.jobs = jobs_fwd; pa.njobs = njobs; pa.lam = lam_of(p);
    pa.S = ckpt_stride(p);
    pa.ck = reinterpret_cast<R*>(ws + L.ck);
    pa.ce = reinterpret_cast<int32_t*>(ws + L.ce);
    pa.qb = reinterpret_cast<R*>(ws + L.qb);
    pa.qe = reinterpret_cast<int32_t*>(ws + L.qe);
    SK_LAUNCH("sweep_ckpt_pipe", st, SkLaunch<R>::sweep_pipe(pa, p.order, interp, true, st),
              "pipelined checkpoint sweep");
    return SK_OK;
}

// Second half: the pipelined adjoint over the reversed job list from the
// state left by run_chunk_prepare_pipe, and the contraction.
template <typename R>
int run_chunk_adjoint_pipe(const sk_params& p, const R* X, const R* Y, int64_t d,
                           const SkPairSrc& src, int64_t P, int max_strips, int max_nsteps_pad,
                           const int2* jobs_adj, int64_t njobs, char* ws, const Layout& L,
                           const R* gK, const int32_t* gKexp, hipStream_t st) {
    const bool interp = p.scheme == SK_POLY_INTERP;
    // progress counters only: the abort flag keeps the checkpoint sweep's
    // (a strip whose checkpoints were not completed must not be replayed)
    const int64_t npg = (L.total - L.pg) / 4 - 1;
    int* prog = reinterpret_cast<int*>(ws + L.pg);
    SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(prog), npg, st), "fill");
    AdjPipeArgs<R> aa;
    std::memset(&aa, 0, sizeof(aa));
    aa.cskew = reinterpret_cast<const R*>(ws + L.cskew); aa.tab = table_for<R>(p);
    aa.gK = gK; aa.gKexp = gKexp;
    aa.ck = reinterpret_cast<const R*>(ws + L.ck);
    aa.ce = reinterpret_cast<const int32_t*>(ws + L.ce);
    aa.qb = reinterpret_cast<const R*>(ws + L.qb);
    aa.qe = reinterpret_cast<const int32_t*>(ws + L.qe);
    aa.gskew = reinterpret_cast<R*>(ws + L.gskew);
    aa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
    aa.progress = prog; aa.abort = reinterpret_cast<int*>(ws + L.total) - 1;
    aa.spin_limit = g_spin_limit.load();
    aa.desc = src.desc; aa.jobs = jobs_adj; aa.njobs = njobs; aa.lam = lam_of(p);
    aa.S = ckpt_stride(p);
    SK_LAUNCH("adjoint_pipe", st, SkLaunch<R>::adjoint_pipe(aa, p.order, interp, st),
              "pipelined adjoint sweep");
    if (aa.lam == 0) return run_contract<R>(X, Y, d, src, P, max_strips, ws, L, st);
    FoldArgs<R> fa;  // refined grid: dL/dc' folded onto the unrefined cells
    fa.src = src; fa.lam = aa.lam;
    fa.gref = reinterpret_cast<const R*>(ws + L.gskew);
    fa.gout = reinterpret_cast<R*>(ws + L.gcu);
    SK_LAUNCH("fold", st, SkLaunch<R>::fold_refined(fa, max_nsteps_pad, P, st), "refined-grid fold");
    return run_contract<R>(X, Y, d, src, P, max_strips, ws, L, st, L.gcu);
}

template <typename R>
int check_lds(const sk_params& p, int64_t max_ly, int64_t d) {
    size_t lim = 0;
    SK_TRY_HIP(lds_limit(&lim), "device query");
    size_t need = is_fd(p)
                      ? (size_t)(max_ly << lam_of(p)) * sizeof(R)
                      : std::max(SkLaunch<R>::sweep_lds(p.order, std::min<int>(grid_cols(p, (int)max_ly), gx_cols_fwd(p))),
                                 SkLaunch<R>::adjoint_lds(p.order, std::min<int>(grid_cols(p, (int)max_ly), gx_cols_adj(p))));
    need = std::max(need, SkLaunch<R>::gram_lds(gram_dpad(p, d)));
    if (need > lim)
        return fail(SK_EUNSUPPORTED, "paths too long for one workgroup's LDS (%zu > %zu bytes)",
                    need, lim);
    return SK_OK;
}

template <typename R>
int gram_forward_pipe(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                      int64_t d, const sk_params& p, R* K, int32_t* Kexp, void* ws, size_t wsb,
                      hipStream_t st);

template <typename R>
int gram_forward(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                 int64_t d, const sk_params& p, R* K, int32_t* Kexp, void* ws, size_t wsb,
                 hipStream_t st) {
    const int64_t npairs = nx * ny;
    if (npairs == 0) return SK_OK;
    const int lam = lam_of(p);
    const int64_t lx = lxp - 1, ly = lyp - 1;
    if (p.algo == SK_ALGO_PIPELINE)
        return gram_forward_pipe<R>(X, nx, lxp, Y, ny, lyp, d, p, K, Kexp, ws, wsb, st);
    if (p.algo == SK_ALGO_PLAIN) {
        const int64_t need = std::max<int64_t>(((lx + ly) << lam) * (p.order + 1), 3 * ((lx << lam) + 1)) * 8;
        if (wsb < (size_t)need) return fail(SK_EWORKSPACE, "plain needs %lld bytes", (long long)need);
        PlainArgs<R> pa;
        std::memset(&pa, 0, sizeof(pa));
        pa.d = d; pa.lx = (int)lx; pa.ly = (int)ly; pa.lam = lam;
        pa.pst = reinterpret_cast<R*>(ws); pa.diag = reinterpret_cast<R*>(ws);
        pa.tab = table_for<R>(p); pa.K = K; pa.Kexp = Kexp;
        pa.second = p.scheme == SK_FD2;
        for (int64_t a = 0; a < nx; ++a)
            for (int64_t b = 0; b < ny; ++b) {
                pa.x = X + a * lxp * d; pa.y = Y + b * lyp * d; pa.k_idx = a * ny + b;
                if (lx == 0 || ly == 0) {
                    SK_TRY_HIP(SkLaunch<R>::fill(K + pa.k_idx, 1, (R)1, st), "fill");
                    if (Kexp) SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(Kexp + pa.k_idx), 1, st), "fill");
                    continue;
                }
                if (is_fd(p))
                    SK_LAUNCH("plain", st, SkLaunch<R>::plain_fd(pa, st), "plain finite differences");
                else
                    SK_LAUNCH("plain", st, SkLaunch<R>::plain_poly(pa, p.order, p.scheme == SK_POLY_INTERP, st),
                              "plain polynomial sweep");
            }
        return SK_OK;
    }
    const SkPairSizes per = sk_pair_sizes((int)lx, (int)ly, lam, p.order, ckpt_stride(p), d, false, xb_words_of(p, (int)ly));
    const int64_t P = gram_chunk(per, npairs, sizeof(R), false, wsb, p.order);
    if (P <= 0) return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", wsb);
    int rc = check_lds<R>(p, ly, d);
    if (rc) return rc;
    const Layout L = layout_for(scale(per, P), P, sizeof(R), false, false, p.order);
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    for (int64_t first = 0; first < npairs; first += P) {
        const int64_t cnt = std::min(P, npairs - first);
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.ny = ny; src.lx_pts = lxp; src.ly_pts = lyp; src.stride = per; src.first = first;
        src.desc = nullptr;
        rc = run_chunk_forward<R>(p, X, Y, d, src, cnt, g.nsteps_pad, (int)lx, (int)ly,
                                  ring_fwd_of(p, (int)ly), (char*)ws, L, K, Kexp, st);
        if (rc) return rc;
    }
    return SK_OK;
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// Backward, first half: increment Gram and the forward sweep that stores
// lane checkpoints and strip-boundary edges.  Kernel values go to K (indexed
// by k_idx - kbase).
template <typename R>
int run_chunk_prepare(const sk_params& p, const R* X, const R* Y, int64_t d,
                      const SkPairSrc& src, int64_t P, int max_nsteps_pad, int max_lx, int max_ly,
                      int ring, char* ws,
                      const Layout& L, R* K, int32_t* Kexp, hipStream_t st) {
    const bool interp = p.scheme == SK_POLY_INTERP;
    R* cskew = reinterpret_cast<R*>(ws + L.cskew);
    GramArgs<R> ga;
    ga.X = X; ga.Y = Y; ga.d = d; ga.dpad = gram_dpad(p, d); ga.lam = lam_of(p);
    ga.src = src; ga.cskew = cskew; ga.maxc = nullptr; ga.split = p.gram == SK_GRAM_BF16X3;
    SK_LAUNCH("gram", st, launch_gram(ga, P, max_nsteps_pad, max_lx, max_ly, p.gram == SK_GRAM_NATIVE, st), "increment Gram");
    SweepArgs<R> sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.src = src; sa.cskew = cskew; sa.tab = table_for<R>(p);
    sa.K = K;
    sa.Kexp = Kexp;
    sa.ck = reinterpret_cast<R*>(ws + L.ck);
    sa.ce = reinterpret_cast<int32_t*>(ws + L.ce);
    sa.qb = reinterpret_cast<R*>(ws + L.qb);
    sa.qe = reinterpret_cast<int32_t*>(ws + L.qe);
    sa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
    sa.gx_cols = gx_cols_fwd(p);
    sa.lam = lam_of(p); sa.S = ckpt_stride(p);
    SK_LAUNCH("sweep_ckpt", st, SkLaunch<R>::sweep(sa, p.order, interp, true, P, ring,
                                                       grid_cols(p, max_ly) > sa.gx_cols, st), "checkpoint sweep");
    return SK_OK;
}

// dL/dc (skewed; at byte offset gsrc, default the adjoint's output) ->
// per-pair partials dL/d(dx), dL/d(dy).
template <typename R>
int run_contract(const R* X, const R* Y, int64_t d, const SkPairSrc& src, int64_t P,
                 int max_strips, char* ws, const Layout& L, hipStream_t st, int64_t gsrc) {
    ContractArgs<R> ca;
    ca.X = X; ca.Y = Y; ca.d = d; ca.src = src;
    ca.gskew = reinterpret_cast<const R*>(ws + (gsrc >= 0 ? gsrc : L.gskew));
    ca.dxp = reinterpret_cast<R*>(ws + L.dxp);
    ca.dyp = reinterpret_cast<R*>(ws + L.dyp);
    SK_LAUNCH("contract", st, SkLaunch<R>::contract(ca, max_strips, P, st), "gradient contraction");
    return SK_OK;
}

// Backward, second half: adjoint sweep and gradient contraction from the
// state left by run_chunk_prepare.
template <typename R>
int run_chunk_adjoint(const sk_params& p, const R* X, const R* Y, int64_t d,
                      const SkPairSrc& src, int64_t P, int max_ly, int ring, int max_strips,
                      int max_nsteps_pad, char* ws, const Layout& L, const R* gK,
                      const int32_t* gKexp, hipStream_t st) {
    const bool interp = p.scheme == SK_POLY_INTERP;
    AdjArgs<R> aa;
    std::memset(&aa, 0, sizeof(aa));
    aa.src = src; aa.cskew = reinterpret_cast<const R*>(ws + L.cskew); aa.tab = table_for<R>(p);
    aa.gK = gK; aa.gKexp = gKexp;
    aa.ck = reinterpret_cast<const R*>(ws + L.ck);
    aa.ce = reinterpret_cast<const int32_t*>(ws + L.ce);
    aa.qb = reinterpret_cast<const R*>(ws + L.qb);
    aa.qe = reinterpret_cast<const int32_t*>(ws + L.qe);
    aa.gskew = reinterpret_cast<R*>(ws + L.gskew);
    aa.xb = reinterpret_cast<unsigned*>(ws + L.xb);
    aa.gx_cols = gx_cols_adj(p);
    aa.lam = lam_of(p); aa.S = ckpt_stride(p);
    SK_LAUNCH("adjoint", st, SkLaunch<R>::adjoint(aa, p.order, interp, P, ring,
                                                  grid_cols(p, max_ly) > aa.gx_cols, st), "adjoint sweep");
    if (aa.lam == 0) return run_contract<R>(X, Y, d, src, P, max_strips, ws, L, st);
    // refined grid: dL/dc' of the sub-cells folded onto the unrefined grid,
    // whose geometry the contraction and the reductions use
    FoldArgs<R> fa;
    fa.src = src; fa.lam = aa.lam;
    fa.gref = reinterpret_cast<const R*>(ws + L.gskew);
    fa.gout = reinterpret_cast<R*>(ws + L.gcu);
    SK_LAUNCH("fold", st, SkLaunch<R>::fold_refined(fa, max_nsteps_pad, P, st), "refined-grid fold");
    return run_contract<R>(X, Y, d, src, P, max_strips, ws, L, st, L.gcu);
}

template <typename R>
int run_chunk_backward(const sk_params& p, const R* X, const R* Y, int64_t d,
                       const SkPairSrc& src, int64_t P, int max_nsteps_pad, int max_lx,
                       int max_ly, int ring_f, int ring_a, int max_strips, char* ws, const Layout& L,
                       const R* gK,
                       const int32_t* gKexp, hipStream_t st) {
    // the checkpoint pass's kernel values go to the chunk's scratch slots
    // (Gram mode: k_idx - first; list mode: descriptors carry local k_idx)
    const int64_t kbase = src.desc ? 0 : src.first;
    R* kbuf = reinterpret_cast<R*>(ws + L.kbuf) - kbase;
    int32_t* kexp = reinterpret_cast<int32_t*>(ws + L.kexp) - kbase;
    int rc = run_chunk_prepare<R>(p, X, Y, d, src, P, max_nsteps_pad, max_lx, max_ly, ring_f, ws, L, kbuf,
                                  kexp, st);
    if (rc) return rc;
    return run_chunk_adjoint<R>(p, X, Y, d, src, P, max_ly, ring_a, max_strips, max_nsteps_pad, ws, L,
                                gK, gKexp, st);
}

// Forward that keeps the whole backward state of a Gram call in `state`
// (one chunk holding every pair), and the backward that starts from it.
template <typename R>
int gram_state_layout(int64_t nx, int64_t lxp, int64_t ny, int64_t lyp, int64_t d,
                      const sk_params& p, SkPairSizes* per, Layout* L) {
    const int64_t npairs = nx * ny;
    *per = sk_pair_sizes((int)(lxp - 1), (int)(lyp - 1), lam_of(p), p.order, ckpt_stride(p), d, true,
                         xb_words_of(p, (int)(lyp - 1)));
    *L = layout_for(scale(*per, npairs), npairs, sizeof(R), true, false, p.order);
    return SK_OK;
}

template <typename R>
int gram_save(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp, int64_t d,
              const sk_params& p, R* K, int32_t* Kexp, void* state, size_t bytes, hipStream_t st) {
    const int64_t npairs = nx * ny, lx = lxp - 1, ly = lyp - 1;
    if (npairs == 0) return SK_OK;
    SkPairSizes per;
    Layout L;
    gram_state_layout<R>(nx, lxp, ny, lyp, d, p, &per, &L);
    if ((size_t)L.total > bytes)
        return fail(SK_EWORKSPACE, "state needs %lld bytes, got %zu", (long long)L.total, bytes);
    if (lx == 0 || ly == 0) {
        SK_TRY_HIP(SkLaunch<R>::fill(K, npairs, (R)1, st), "fill");
        if (Kexp) SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(Kexp), npairs, st), "fill");
        return SK_OK;
    }
    int rc = check_lds<R>(p, ly, d);
    if (rc) return rc;
    const int lam = lam_of(p);
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.ny = ny; src.lx_pts = lxp; src.ly_pts = lyp; src.stride = per; src.first = 0;
    return run_chunk_prepare<R>(p, X, Y, d, src, npairs, g.nsteps_pad, (int)lx, (int)ly,
                                ring_fwd_of(p, (int)ly), (char*)state, L, K, Kexp, st);
}

template <typename R>
int gram_backward_saved(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                        int64_t d, const sk_params& p, const R* gK, const int32_t* gKexp, R* gX,
                        R* gY, void* state, size_t bytes, hipStream_t st) {
    const int64_t npairs = nx * ny, lx = lxp - 1, ly = lyp - 1;
    SkPairSizes per;
    Layout L;
    gram_state_layout<R>(nx, lxp, ny, lyp, d, p, &per, &L);
    if ((size_t)L.total > bytes)
        return fail(SK_EWORKSPACE, "state needs %lld bytes, got %zu", (long long)L.total, bytes);
    SK_TRY_HIP(SkLaunch<R>::fill(gX, nx * lxp * d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, ny * lyp * d, (R)0, st), "fill");
    if (npairs == 0 || lx == 0 || ly == 0) return SK_OK;
    int rc = check_lds<R>(p, ly, d);
    if (rc) return rc;
    // sweeps on the (refined) grid; contraction and reductions on the unrefined one
    const int lam = lam_of(p);
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    const int nstrips_u = sk_make_geom((int)lx, (int)ly).nstrips;
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.ny = ny; src.lx_pts = lxp; src.ly_pts = lyp; src.stride = per; src.first = 0;
    rc = run_chunk_adjoint<R>(p, X, Y, d, src, npairs, (int)ly, ring_adj_of(p, (int)ly), nstrips_u,
                              g.nsteps_pad, (char*)state, L, gK, gKexp, st);
    if (rc) return rc;
    ReduceGramArgs<R> ra;
    ra.nx = nx; ra.ny = ny; ra.lx_pts = lxp; ra.ly_pts = lyp; ra.d = d;
    ra.first = 0; ra.count = npairs; ra.dx_stride = per.dx; ra.dy_stride = per.dy;
    ra.nstrips = nstrips_u;
    ra.dxp = reinterpret_cast<const R*>((char*)state + L.dxp);
    ra.dyp = reinterpret_cast<const R*>((char*)state + L.dyp);
    ra.gX = gX; ra.gY = gY;
    SK_LAUNCH("reduce", st, SkLaunch<R>::reduce_gram(ra, st), "gradient reduction");
    return SK_OK;
}

template <typename R>
int gram_backward(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                  int64_t d, const sk_params& p, const R* gK, const int32_t* gKexp, R* gX, R* gY,
                  void* ws, size_t wsb, hipStream_t st) {
    const int64_t npairs = nx * ny;
    const int64_t lx = lxp - 1, ly = lyp - 1;
    if (npairs == 0 || lx == 0 || ly == 0) {
        SK_TRY_HIP(SkLaunch<R>::fill(gX, nx * lxp * d, (R)0, st), "fill");
        SK_TRY_HIP(SkLaunch<R>::fill(gY, ny * lyp * d, (R)0, st), "fill");
        return SK_OK;
    }
    const int lam = lam_of(p);
    const SkPairSizes per = sk_pair_sizes((int)lx, (int)ly, lam, p.order, ckpt_stride(p), d, true, xb_words_of(p, (int)ly));
    const int64_t P = gram_chunk(per, npairs, sizeof(R), true, wsb, p.order);
    if (P <= 0) return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", wsb);
    int rc = check_lds<R>(p, ly, d);
    if (rc) return rc;
    SK_TRY_HIP(SkLaunch<R>::fill(gX, nx * lxp * d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, ny * lyp * d, (R)0, st), "fill");
    const Layout L = layout_for(scale(per, P), P, sizeof(R), true, false, p.order);
    // sweeps on the (refined) grid; contraction and reductions on the unrefined one
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    const int nstrips_u = sk_make_geom((int)lx, (int)ly).nstrips;
    for (int64_t first = 0; first < npairs; first += P) {
        const int64_t cnt = std::min(P, npairs - first);
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.ny = ny; src.lx_pts = lxp; src.ly_pts = lyp; src.stride = per; src.first = first;
        rc = run_chunk_backward<R>(p, X, Y, d, src, cnt, g.nsteps_pad, (int)lx, (int)ly,
                                   ring_fwd_of(p, (int)ly), ring_adj_of(p, (int)ly), nstrips_u,
                                   (char*)ws, L, gK, gKexp, st);
        if (rc) return rc;
        ReduceGramArgs<R> ra;
        ra.nx = nx; ra.ny = ny; ra.lx_pts = lxp; ra.ly_pts = lyp; ra.d = d;
        ra.first = first; ra.count = cnt; ra.dx_stride = per.dx; ra.dy_stride = per.dy;
        ra.nstrips = nstrips_u;
        ra.dxp = reinterpret_cast<const R*>((char*)ws + L.dxp);
        ra.dyp = reinterpret_cast<const R*>((char*)ws + L.dyp);
        ra.gX = gX; ra.gY = gY;
        SK_LAUNCH("reduce", st, SkLaunch<R>::reduce_gram(ra, st), "gradient reduction");
    }
    return SK_OK;
}

// Gram calls on the strip pipeline (SK_ALGO_PIPELINE).  Every pair of a
// Gram call has the same geometry, so the chunk size, the per-pair
// descriptors (chunk-relative workspace offsets, the same arrangement the
// implicit Gram descriptors use, so the Gram reductions apply unchanged) and
// the job lists are fixed on the host and uploaded once, ahead of the chunk
// scratch: [descriptors of all pairs][jobs of a full chunk][jobs of the last
// chunk][chunk scratch].  A job list holds the (checkpoint) sweep's jobs,
// every pair's first strip, then every pair's second, ..., so that a strip's
// predecessor always comes earlier in the list; a backward list continues
// with the adjoint's, every pair's last strip first.
struct GramPipePlan {
    SkPairSizes per = {};
    int64_t P = 0, nstrips = 0, desc = 0, jobs_full = 0, jobs_last = 0, scratch = 0, total = 0;
};

int gram_pipe_plan(int64_t nx, int64_t lxp, int64_t ny, int64_t lyp, int64_t d,
                   const sk_params& p, bool backward, size_t wsb, GramPipePlan* G) {
    const int64_t npairs = nx * ny, lx = lxp - 1, ly = lyp - 1;
    const int es = (int)esize(p), lam = lam_of(p);
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    G->per = sk_pair_sizes((int)lx, (int)ly, lam, p.order, ckpt_stride(p), d, backward,
                           2 * sk_gx_words(p.order, es), true);
    G->nstrips = g.nstrips;
    const int64_t dbytes = align_up(npairs * (int64_t)sizeof(SkPairDesc));
    // job lists sized for chunks of every pair (an upper bound for any chunk)
    const int64_t jbound = align_up((backward ? 2 : 1) * npairs * G->nstrips * (int64_t)sizeof(int2));
    const int64_t head = dbytes + 2 * jbound;
    if (wsb <= (size_t)head) return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", wsb);
    G->P = gram_chunk(G->per, npairs, (size_t)es, backward, wsb - (size_t)head, p.order);
    if (G->P <= 0) return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", wsb);
    G->desc = 0;
    G->jobs_full = dbytes;
    G->jobs_last = dbytes + jbound;
    G->scratch = head;
    G->total = head + layout_for(scale(G->per, G->P), G->P, (size_t)es, backward, false, p.order).total;
    return SK_OK;
}

// Builds and uploads the descriptors and job lists (synchronises `st`).
int gram_pipe_upload(const GramPipePlan& G, int64_t nx, int64_t lxp, int64_t ny, int64_t lyp,
                     bool backward, char* base, hipStream_t st) {
    const int64_t npairs = nx * ny;
    const int ns = (int)G.nstrips;
    std::vector<SkPairDesc> desc((size_t)npairs);
    for (int64_t q = 0; q < npairs; ++q) {
        const int64_t local = q % G.P;
        SkPairDesc& e = desc[(size_t)q];
        e.x_off = (q / ny) * lxp;
        e.y_off = (q % ny) * lyp;
        e.lx = (int32_t)(lxp - 1);
        e.ly = (int32_t)(lyp - 1);
        e.swap = 0;
        // the forward writes K directly; the checkpoint pass's kernel values
        // go to the chunk scratch
        e.k_idx = backward ? local : q;
        e.g_idx = q;
        e.c_off = local * G.per.c; e.ck_off = local * G.per.ck; e.ce_off = local * G.per.ce;
        e.qb_off = local * G.per.qb; e.qe_off = local * G.per.qe; e.dx_off = local * G.per.dx;
        e.dy_off = local * G.per.dy; e.xb_off = local * G.per.xb; e.pg_off = local * G.per.pg;
    }
    auto job_list = [&](int64_t cnt) {
        std::vector<int2> jobs;
        jobs.reserve((size_t)((backward ? 2 : 1) * cnt * ns));
        for (int s = 0; s < ns; ++s)
            for (int64_t li = 0; li < cnt; ++li) jobs.push_back(make_int2((int)li, s));
        if (backward)
            for (int s = ns - 1; s >= 0; --s)
                for (int64_t li = 0; li < cnt; ++li) jobs.push_back(make_int2((int)li, s));
        return jobs;
    };
    const int64_t cnt_last = npairs - (npairs - 1) / G.P * G.P;
    const std::vector<int2> jf = job_list(G.P), jl = job_list(cnt_last);
    SK_TRY_HIP(hipMemcpyAsync(base + G.desc, desc.data(), desc.size() * sizeof(SkPairDesc),
                              hipMemcpyHostToDevice, st), "descriptor upload");
    SK_TRY_HIP(hipMemcpyAsync(base + G.jobs_full, jf.data(), jf.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st), "job list upload");
    SK_TRY_HIP(hipMemcpyAsync(base + G.jobs_last, jl.data(), jl.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st), "job list upload");
    SK_TRY_HIP(hipStreamSynchronize(st), "descriptor upload");
    return SK_OK;
}

// Forward: paths of several strips (of the refined grid) on the pipeline,
// the pairs of a chunk as one job list; others batched.
template <typename R>
int gram_forward_pipe(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                      int64_t d, const sk_params& p, R* K, int32_t* Kexp, void* ws, size_t wsb,
                      hipStream_t st) {
    const int64_t npairs = nx * ny, lx = lxp - 1, ly = lyp - 1;
    const int lam = lam_of(p);
    if (lx == 0 || ly == 0) {
        SK_TRY_HIP(SkLaunch<R>::fill(K, npairs, (R)1, st), "fill");
        if (Kexp) SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(Kexp), npairs, st), "fill");
        return SK_OK;
    }
    if (sk_make_geom((int)(lx << lam), (int)(ly << lam)).nstrips < 2) {
        sk_params q = p;
        q.algo = SK_ALGO_BATCHED;
        return gram_forward<R>(X, nx, lxp, Y, ny, lyp, d, q, K, Kexp, ws, wsb, st);
    }
    GramPipePlan G;
    int rc = gram_pipe_plan(nx, lxp, ny, lyp, d, p, false, wsb, &G);
    if (rc) return rc;
    char* base = static_cast<char*>(ws);
    if ((rc = gram_pipe_upload(G, nx, lxp, ny, lyp, false, base, st))) return rc;
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    const Layout L = layout_for(scale(G.per, G.P), G.P, sizeof(R), false, false, p.order);
    char* ws_c = base + G.scratch;
    for (int64_t first = 0; first < npairs; first += G.P) {
        const int64_t cnt = std::min(G.P, npairs - first);
        const int2* jobs = reinterpret_cast<const int2*>(base + (cnt == G.P ? G.jobs_full : G.jobs_last));
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.desc = reinterpret_cast<const SkPairDesc*>(base + G.desc) + first;
        rc = run_chunk_forward_pipe<R>(p, X, Y, d, src, cnt, g.nsteps_pad, (int)lx, (int)ly, jobs,
                                       cnt * G.nstrips, ws_c, L, K, Kexp, st);
        if (rc) return rc;
    }
    return SK_OK;
}

// Backward: the pipelined checkpoint sweep and adjoint per chunk, then the
// Gram reductions; paths of one strip run the batched backward.
template <typename R>
int gram_backward_pipe(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                       int64_t d, const sk_params& p, const R* gK, const int32_t* gKexp, R* gX,
                       R* gY, void* ws, size_t wsb, hipStream_t st) {
    const int64_t npairs = nx * ny, lx = lxp - 1, ly = lyp - 1;
    const int lam = lam_of(p);
    if (npairs == 0 || lx == 0 || ly == 0 || sk_make_geom((int)(lx << lam), (int)(ly << lam)).nstrips < 2)
        return gram_backward<R>(X, nx, lxp, Y, ny, lyp, d, p, gK, gKexp, gX, gY, ws, wsb, st);
    GramPipePlan G;
    int rc = gram_pipe_plan(nx, lxp, ny, lyp, d, p, true, wsb, &G);
    if (rc) return rc;
    if ((rc = check_lds<R>(p, ly, d))) return rc;
    char* base = static_cast<char*>(ws);
    if ((rc = gram_pipe_upload(G, nx, lxp, ny, lyp, true, base, st))) return rc;
    // strips of the (refined) grid on the pipeline; the contraction and the
    // reductions on the unrefined one
    const SkGeom g = sk_make_geom((int)(lx << lam), (int)(ly << lam));
    const int ns = g.nstrips, nstrips_u = sk_make_geom((int)lx, (int)ly).nstrips;
    SK_TRY_HIP(SkLaunch<R>::fill(gX, nx * lxp * d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, ny * lyp * d, (R)0, st), "fill");
    const Layout L = layout_for(scale(G.per, G.P), G.P, sizeof(R), true, false, p.order);
    char* ws_c = base + G.scratch;
    R* kbuf = reinterpret_cast<R*>(ws_c + L.kbuf);
    int32_t* kexp = reinterpret_cast<int32_t*>(ws_c + L.kexp);
    for (int64_t first = 0; first < npairs; first += G.P) {
        const int64_t cnt = std::min(G.P, npairs - first);
        const int2* jobs = reinterpret_cast<const int2*>(base + (cnt == G.P ? G.jobs_full : G.jobs_last));
        const int64_t njobs = cnt * ns;
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.desc = reinterpret_cast<const SkPairDesc*>(base + G.desc) + first;
        rc = run_chunk_prepare_pipe<R>(p, X, Y, d, src, cnt, g.nsteps_pad, (int)lx, (int)ly, jobs,
                                       njobs, ws_c, L, kbuf, kexp, st);
        if (!rc)
            rc = run_chunk_adjoint_pipe<R>(p, X, Y, d, src, cnt, nstrips_u, g.nsteps_pad, jobs + njobs,
                                           njobs, ws_c, L, gK, gKexp, st);
        if (rc) return rc;
        ReduceGramArgs<R> ra;
        ra.nx = nx; ra.ny = ny; ra.lx_pts = lxp; ra.ly_pts = lyp; ra.d = d;
        ra.first = first; ra.count = cnt; ra.dx_stride = G.per.dx; ra.dy_stride = G.per.dy;
        ra.nstrips = nstrips_u;
        ra.dxp = reinterpret_cast<const R*>(ws_c + L.dxp);
        ra.dyp = reinterpret_cast<const R*>(ws_c + L.dyp);
        ra.gX = gX; ra.gY = gY;
        SK_LAUNCH("reduce", st, SkLaunch<R>::reduce_gram(ra, st), "gradient reduction");
    }
    return SK_OK;
}

// Saved state on the pipeline: the backward's whole state in one chunk
// (descriptors and job lists at its head), kept between a forward that
// also stores the checkpoints and the backward that starts from them.
bool gram_pipe_applies(const sk_params& p, int64_t nx, int64_t lxp, int64_t ny, int64_t lyp) {
    const int lam = lam_of(p);
    return p.algo == SK_ALGO_PIPELINE && nx * ny > 0 && lxp > 1 && lyp > 1 &&
           sk_make_geom((int)((lxp - 1) << lam), (int)((lyp - 1) << lam)).nstrips >= 2;
}

int gram_pipe_state(int64_t nx, int64_t lxp, int64_t ny, int64_t lyp, int64_t d,
                    const sk_params& p, GramPipePlan* G) {
    int rc = gram_pipe_plan(nx, lxp, ny, lyp, d, p, true, SIZE_MAX, G);
    if (!rc && G->P != nx * ny) rc = fail(SK_EWORKSPACE, "the saved state needs one chunk");
    return rc;
}

template <typename R>
int gram_save_pipe(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny, int64_t lyp,
                   int64_t d, const sk_params& p, R* K, int32_t* Kexp, void* state, size_t bytes,
                   hipStream_t st) {
    GramPipePlan G;
    int rc = gram_pipe_state(nx, lxp, ny, lyp, d, p, &G);
    if (rc) return rc;
    if ((size_t)G.total > bytes)
        return fail(SK_EWORKSPACE, "state needs %lld bytes, got %zu", (long long)G.total, bytes);
    if ((rc = check_lds<R>(p, lyp - 1, d))) return rc;
    char* base = static_cast<char*>(state);
    if ((rc = gram_pipe_upload(G, nx, lxp, ny, lyp, true, base, st))) return rc;
    const int lam = lam_of(p);
    const SkGeom g = sk_make_geom((int)((lxp - 1) << lam), (int)((lyp - 1) << lam));
    const Layout L = layout_for(scale(G.per, G.P), G.P, sizeof(R), true, false, p.order);
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.desc = reinterpret_cast<const SkPairDesc*>(base + G.desc);
    // one chunk: the descriptors' chunk-local k_idx is the pair index
    return run_chunk_prepare_pipe<R>(p, X, Y, d, src, G.P, g.nsteps_pad, (int)(lxp - 1), (int)(lyp - 1),
                                     reinterpret_cast<const int2*>(base + G.jobs_full),
                                     G.P * G.nstrips, base + G.scratch, L, K, Kexp, st);
}

template <typename R>
int gram_backward_saved_pipe(const R* X, int64_t nx, int64_t lxp, const R* Y, int64_t ny,
                             int64_t lyp, int64_t d, const sk_params& p, const R* gK,
                             const int32_t* gKexp, R* gX, R* gY, void* state, size_t bytes,
                             hipStream_t st) {
    GramPipePlan G;
    int rc = gram_pipe_state(nx, lxp, ny, lyp, d, p, &G);
    if (rc) return rc;
    if ((size_t)G.total > bytes)
        return fail(SK_EWORKSPACE, "state needs %lld bytes, got %zu", (long long)G.total, bytes);
    char* base = static_cast<char*>(state);
    const int lam = lam_of(p);
    const int ns = (int)G.nstrips, nstrips_u = sk_make_geom((int)(lxp - 1), (int)(lyp - 1)).nstrips;
    const int nsteps_pad = sk_make_geom((int)((lxp - 1) << lam), (int)((lyp - 1) << lam)).nsteps_pad;
    const Layout L = layout_for(scale(G.per, G.P), G.P, sizeof(R), true, false, p.order);
    char* ws_c = base + G.scratch;
    SK_TRY_HIP(SkLaunch<R>::fill(gX, nx * lxp * d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, ny * lyp * d, (R)0, st), "fill");
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.desc = reinterpret_cast<const SkPairDesc*>(base + G.desc);
    const int64_t njobs = G.P * ns;
    rc = run_chunk_adjoint_pipe<R>(p, X, Y, d, src, G.P, nstrips_u, nsteps_pad,
                                   reinterpret_cast<const int2*>(base + G.jobs_full) + njobs, njobs,
                                   ws_c, L, gK, gKexp, st);
    if (rc) return rc;
    ReduceGramArgs<R> ra;
    ra.nx = nx; ra.ny = ny; ra.lx_pts = lxp; ra.ly_pts = lyp; ra.d = d;
    ra.first = 0; ra.count = G.P; ra.dx_stride = G.per.dx; ra.dy_stride = G.per.dy;
    ra.nstrips = nstrips_u;
    ra.dxp = reinterpret_cast<const R*>(ws_c + L.dxp);
    ra.dyp = reinterpret_cast<const R*>(ws_c + L.dyp);
    ra.gX = gX; ra.gY = gY;
    SK_LAUNCH("reduce", st, SkLaunch<R>::reduce_gram(ra, st), "gradient reduction");
    return SK_OK;
}

// ---------------------------------------------------------------------------
// pair plans (independent pairs of uneven lengths)
// ---------------------------------------------------------------------------
// A plan fixes, for one set of offsets: the order in which pairs are
// launched, whether each pair is transposed (k(x, y) = k(y, x), so the
// shorter path can be the one whose edges wait in LDS), how pairs are grouped
// into launches, and the workspace layout.  All descriptors are uploaded
// once, so running a plan only launches kernels.
struct PlanCfg {
    int32_t order;    // 1: longest pairs first (by wavefront steps); 0: given order
    int32_t swap;     // 1: transpose pairs whose second path is longer
    int32_t buckets;  // 1: separate launches per LDS class of the forward sweep
    int32_t pipe;     // k >= 2: pairs of k or more strips on the strip pipeline (forward and
                      // backward); 0: none
    int32_t ckpt;     // checkpoint stride of the backward (0: the caller's sk_params.ckpt)
};
constexpr PlanCfg kDefaultPlanCfg = {1, 1, 1, 2, 0};

struct PlanChunk {
    int64_t first = 0, count = 0;  // range of the plan's descriptor array
    SkPairSizes tot = {};
    int max_nsteps_pad = 0, max_lx = 0, max_ly = 0, max_strips = 0;
    int ring_fwd = 0, ring_adj = 0;  // LDS ring columns (largest among pairs not using the global exchange)
    int64_t max_pts = 0;
    bool pipe = false;               // strip pipeline: jobs of the plan's job list
    int64_t jobs_first = 0, njobs = 0;  // the sweep's jobs; a backward chunk's adjoint
                                        // jobs follow them (njobs more)
};

struct PlanImpl {
    sk_params p;       // the parameters in use (ckpt: the configuration's stride)
    sk_params p_user;  // as the caller gave them
    int64_t npairs = 0, d = 0;
    bool backward = false;
    std::vector<int64_t> xo, yo;
    PlanCfg cfg = kDefaultPlanCfg;
    // forward and backward chunkings (the backward keeps more state per pair,
    // so its chunks are smaller); descriptors hold chunk-relative offsets
    std::vector<SkPairDesc> fdesc, bdesc;
    std::vector<PlanChunk> fchunks, bchunks;
    // strip-pipeline jobs (chunk-local pair, strip) of the pipeline chunks
    std::vector<int2> jobs;
    int max_ly = 0;  // longest column count of any pair (LDS check)
    // workspace regions (bytes): descriptors, kernel-value scratch, jobs, chunk scratch
    int64_t fdesc_off = 0, bdesc_off = 0, kbuf_off = 0, kexp_off = 0, jobs_off = 0, scratch_off = 0,
            total = 0;
    const void* uploaded = nullptr;
};

size_t sweep_lds_bytes(const sk_params& p, int ly) {
    if (is_fd(p)) return (size_t)(ly << lam_of(p)) * esize(p);
    return p.dtype == SK_F32 ? SkLaunch<float>::sweep_lds(p.order, grid_cols(p, ly))
                             : SkLaunch<double>::sweep_lds(p.order, grid_cols(p, ly));
}

// Launch groups: pairs whose edges go through the global exchange in the
// adjoint (and the forward), in the forward only, then LDS rings up to 4, 8
// and 17 KiB (and longer FD rings).
int lds_class(const sk_params& p, int ly) {
    if (!is_fd(p) && ring_adj_of(p, ly) == 0) return 5;
    if (ring_fwd_of(p, ly) == 0) return 4;
    const size_t b = sweep_lds_bytes(p, ly);
    return b <= (4u << 10) ? 0 : b <= (8u << 10) ? 1 : b <= (17u << 10) ? 2 : 3;
}

// Build descriptors and chunks for `cfg`, with chunk scratch sized to fit a
// workspace of ws_bytes (SIZE_MAX: the default chunk cap).
int plan_build_into(PlanImpl& P, const PlanCfg& cfg, size_t ws_bytes);

// Transactional: the plan is left unchanged when the build fails.
int plan_build(PlanImpl& P0, const PlanCfg& cfg, size_t ws_bytes) {
    PlanImpl P = P0;
    const int rc = plan_build_into(P, cfg, ws_bytes);
    if (rc == SK_OK) P0 = std::move(P);
    return rc;
}

int plan_build_into(PlanImpl& P, const PlanCfg& cfg, size_t ws_bytes) {
    if (cfg.pipe < 0 || cfg.pipe == 1) return fail(SK_EINVAL, "pipeline threshold %d strips", cfg.pipe);
    P.p = P.p_user;
    if (cfg.ckpt != 0) {
        P.p.ckpt = cfg.ckpt;
        const int rc = check_params(&P.p, P.backward);
        if (rc) return rc;
    }
    const sk_params& p = P.p;
    const int lam = lam_of(p);
    const size_t es = esize(p);
    const int64_t n = P.npairs;
    P.cfg = cfg;
    P.uploaded = nullptr;
    std::vector<int32_t> ex(n), ey(n), sw(n), clsb(n), clsf(n), pipe(n), nstr(n);
    std::vector<int64_t> cost(n), seqb(n), seqf(n);
    int64_t njobs_all = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int lx = (int)(P.xo[i + 1] - P.xo[i] - 1), ly = (int)(P.yo[i + 1] - P.yo[i] - 1);
        sw[i] = (cfg.swap && ly > lx) ? 1 : 0;
        ex[i] = sw[i] ? ly : lx;
        ey[i] = sw[i] ? lx : ly;
        const SkGeom g = sk_make_geom(ex[i] << lam, ey[i] << lam);
        cost[i] = g.nsteps;
        nstr[i] = g.nstrips;
        const int32_t cls_fwd = cfg.buckets ? lds_class(p, ey[i]) : 0;
        // pairs of several strips go to the strip pipeline (class 6), which
        // balances the load strip by strip instead of pair by pair
        pipe[i] = (cfg.pipe >= 2 && !is_fd(p) && g.nstrips >= cfg.pipe) ? 1 : 0;
        clsf[i] = pipe[i] ? 6 : cls_fwd;
        // the backward runs its other pairs in one launch per chunk: a launch
        // per LDS class pays the longest pairs' sequential tail once per
        // class, more than lower occupancy costs (one class measured 1.45x
        // faster on 4096 uneven pairs); the classes shape the forward only
        clsb[i] = pipe[i] ? 6 : 0;
        // forward jobs; a backward adds the checkpoint sweep's and the adjoint's
        if (pipe[i]) njobs_all += (int64_t)g.nstrips * (P.backward ? 3 : 1);
        seqb[i] = seqf[i] = i;
    }
    std::stable_sort(seqb.begin(), seqb.end(), [&](int64_t u, int64_t v) {
        if (clsb[u] != clsb[v]) return clsb[u] > clsb[v];
        return cfg.order ? cost[u] > cost[v] : false;
    });
    std::stable_sort(seqf.begin(), seqf.end(), [&](int64_t u, int64_t v) {
        if (clsf[u] != clsf[v]) return clsf[u] > clsf[v];
        return cfg.order ? cost[u] > cost[v] : false;
    });
    const int64_t dbytes = align_up(n * (int64_t)sizeof(SkPairDesc));
    P.fdesc_off = 0;
    P.bdesc_off = dbytes;
    P.kbuf_off = P.bdesc_off + (P.backward ? dbytes : 0);
    P.kexp_off = P.kbuf_off + align_up(n * (int64_t)es);
    P.jobs_off = P.kexp_off + align_up(n * 4);
    P.scratch_off = P.jobs_off + align_up(njobs_all * (int64_t)sizeof(int2));
    P.jobs.clear();
    size_t cap = kDefaultCap;
    if (ws_bytes != SIZE_MAX) {
        if (ws_bytes <= (size_t)P.scratch_off)
            return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", ws_bytes);
        cap = ws_bytes - (size_t)P.scratch_off;
    }
    P.max_ly = 0;
    for (int64_t i = 0; i < n; ++i) P.max_ly = std::max(P.max_ly, ey[i]);
    // Chunks: within each LDS class (one class without buckets), as few
    // chunks as the workspace allows, filled longest pair first into the
    // chunk with the least work that still fits, so that every launch mixes
    // long and short pairs (a chunk of only the longest pairs would leave
    // most of the GPU idle).  Each chunk launches its pairs longest first.
    auto chunk = [&](bool bwd, std::vector<SkPairDesc>& desc, std::vector<PlanChunk>& chunks,
                     int64_t* scratch) -> int {
        const std::vector<int32_t>& cls = bwd ? clsb : clsf;
        const std::vector<int64_t>& seq = bwd ? seqb : seqf;
        desc.assign(n, SkPairDesc());
        chunks.clear();
        *scratch = 0;
        std::vector<SkPairSizes> zs(n);
        for (int64_t i = 0; i < n; ++i) {
            const bool pp = pipe[i] != 0;  // two record slots, a progress counter per strip
            zs[i] = sk_pair_sizes(ex[i], ey[i], lam, p.order, ckpt_stride(p), P.d, bwd,
                                  pp ? 2 * sk_gx_words(p.order, (int)es) : xb_words_of(p, ey[i]), pp);
        }
        int64_t pos = 0;
        for (int64_t g0 = 0; g0 < n;) {
            int64_t g1 = g0 + 1;
            // a group: one LDS class (any class without buckets); strip-pipeline
            // pairs always form their own group
            auto same = [&](int64_t u, int64_t v) {
                return (cls[u] == 6) == (cls[v] == 6) && (bwd || !cfg.buckets || cls[u] == cls[v]);
            };
            while (g1 < n && same(seq[g1], seq[g0])) ++g1;
            // bins of this group
            struct Bin { SkPairSizes tot; int64_t count, work; std::vector<int64_t> pairs; };
            std::vector<Bin> bins;
            SkPairSizes all = SkPairSizes{};
            for (int64_t k = g0; k < g1; ++k) all = add(all, zs[seq[k]]);
            const int64_t total = layout_for(all, g1 - g0, es, bwd, false, p.order).total;
            const int64_t nb = std::max<int64_t>(1, (int64_t)((double)total / (double)cap * 1.05) + 1);
            bins.resize(total <= (int64_t)cap ? 1 : nb);
            for (Bin& bn : bins) { bn.tot = SkPairSizes{}; bn.count = 0; bn.work = 0; }
            for (int64_t k = g0; k < g1; ++k) {
                const int64_t i = seq[k];
                if ((size_t)layout_for(zs[i], 1, es, bwd, false, p.order).total > cap)
                    return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", ws_bytes);
                int64_t best = -1;
                for (int64_t q = 0; q < (int64_t)bins.size(); ++q) {
                    const Bin& bn = bins[q];
                    if ((size_t)layout_for(add(bn.tot, zs[i]), bn.count + 1, es, bwd, false, p.order).total > cap)
                        continue;
                    if (best < 0 || bn.work < bins[best].work) best = q;
                }
                if (best < 0) {
                    bins.push_back(Bin());
                    best = (int64_t)bins.size() - 1;
                    bins[best].tot = SkPairSizes{};
                    bins[best].count = 0;
                    bins[best].work = 0;
                }
                Bin& bn = bins[best];
                bn.tot = add(bn.tot, zs[i]);
                bn.count += 1;
                bn.work += cost[i];
                bn.pairs.push_back(i);
            }
            for (const Bin& bn : bins) {
                if (bn.count == 0) continue;
                PlanChunk cur;
                cur.first = pos;
                cur.pipe = cls[bn.pairs[0]] == 6;
                SkPairSizes run = SkPairSizes{};
                for (const int64_t i : bn.pairs) {  // already longest first
                    const SkGeom g = sk_make_geom(ex[i] << lam, ey[i] << lam);
                    SkPairDesc& q = desc[pos++];
                    q.x_off = sw[i] ? P.yo[i] : P.xo[i];
                    q.y_off = sw[i] ? P.xo[i] : P.yo[i];
                    q.lx = ex[i];
                    q.ly = ey[i];
                    q.swap = sw[i];
                    q.k_idx = i;
                    q.g_idx = i;
                    q.c_off = run.c; q.ck_off = run.ck; q.ce_off = run.ce; q.qb_off = run.qb;
                    q.qe_off = run.qe; q.dx_off = run.dx; q.dy_off = run.dy; q.xb_off = run.xb;
                    q.pg_off = run.pg;
                    run = add(run, zs[i]);
                    cur.count += 1;
                    cur.tot = add(cur.tot, zs[i]);
                    cur.max_nsteps_pad = std::max(cur.max_nsteps_pad, g.nsteps_pad);
                    cur.max_lx = std::max(cur.max_lx, ex[i]);
                    cur.max_ly = std::max(cur.max_ly, ey[i]);
                    cur.max_strips = std::max(cur.max_strips, g.nstrips);
                    cur.ring_fwd = std::max(cur.ring_fwd, ring_fwd_of(p, ey[i]));
                    cur.ring_adj = std::max(cur.ring_adj, ring_adj_of(p, ey[i]));
                    cur.max_pts = std::max<int64_t>(cur.max_pts, std::max(ex[i], ey[i]) + 1);
                }
                *scratch = std::max(*scratch, layout_for(cur.tot, cur.count, es, bwd, false, p.order).total);
                if (cur.pipe) {
                    // jobs strip by strip across the chunk's pairs: every pair's
                    // strips in increasing order, all pairs' first strips first
                    cur.jobs_first = (int64_t)P.jobs.size();
                    for (int st = 0; st < cur.max_strips; ++st)
                        for (int64_t li = 0; li < cur.count; ++li)
                            if (nstr[bn.pairs[li]] > st) P.jobs.push_back(make_int2((int)li, st));
                    cur.njobs = (int64_t)P.jobs.size() - cur.jobs_first;
                    if (bwd)  // the adjoint's: every pair's strips in decreasing
                              // order, all pairs' last strips first
                        for (int k = 0; k < cur.max_strips; ++k)
                            for (int64_t li = 0; li < cur.count; ++li) {
                                const int ns = nstr[bn.pairs[li]];
                                if (ns > k) P.jobs.push_back(make_int2((int)li, ns - 1 - k));
                            }
                }
                chunks.push_back(cur);
            }
            g0 = g1;
        }
        return SK_OK;
    };
    int64_t fs = 0, bs = 0;
    int rc = chunk(false, P.fdesc, P.fchunks, &fs);
    if (rc) return rc;
    if (P.backward) {
        rc = chunk(true, P.bdesc, P.bchunks, &bs);
        if (rc) return rc;
    } else {
        P.bdesc.clear();
        P.bchunks.clear();
    }
    P.total = P.scratch_off + std::max<int64_t>(std::max(fs, bs), 256);
    return SK_OK;
}

int plan_init(PlanImpl& P, const int64_t* xo, const int64_t* yo, int64_t npairs, int64_t d,
              const sk_params& p, bool backward) {
    P.p = P.p_user = p;
    P.npairs = npairs;
    P.d = d;
    P.backward = backward;
    P.xo.assign(xo, xo + npairs + 1);
    P.yo.assign(yo, yo + npairs + 1);
    return SK_OK;
}

// ---------------------------------------------------------------------------
// tune cache: tuned configurations keyed by (GPU architecture, scheme, order,
// precision, Gram mode, refinement, direction, d, shape class), where the
// shape class is the ceil(log2) of the pair count and of the mean and
// largest segment counts of each side.  Kept per process; saved to and
// loaded from a text file by sigkernel_tune_cache_save / _load.
// ---------------------------------------------------------------------------
struct TuneVal {
    PlanCfg cfg;     // plans (and one-shot pairs calls)
    int32_t algo;    // Gram calls: SK_ALGO_BATCHED or SK_ALGO_PIPELINE
    double ms;       // timed forward (+ backward) of the winner
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, TuneVal>> g_tune_cache;

int clog2(int64_t v) {
    int r = 0;
    while (r < 62 && ((int64_t)1 << r) < v) ++r;
    return r;
}

// gfx name of the current device ("none" without one), looked up once per device.
std::string device_arch() {
    static std::mutex mu;
    static std::vector<std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return "none";
    std::lock_guard<std::mutex> g(mu);
    if ((size_t)dev >= names.size()) names.resize(dev + 1);
    if (names[dev].empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "none";
        std::string n = prop.gcnArchName;
        const size_t colon = n.find(':');
        names[dev] = n.substr(0, colon);
        if (names[dev].empty()) names[dev] = "unknown";
    }
    return names[dev];
}

std::string params_key(const char* kind, const sk_params& p, bool backward, int64_t d) {
    char b[160];
    std::snprintf(b, sizeof(b), "%s|%s|s%d|n%d|t%d|g%d|y%d|f%d|b%d|d%lld", kind,
                  device_arch().c_str(), p.scheme, p.order, p.dtype, p.gram, p.dyadic,
                  p.flags, backward ? 1 : 0, (long long)d);
    return b;
}

std::string plan_key(const PlanImpl& P) {
    int64_t sx = 0, sy = 0, mx = 0, my = 0;
    for (int64_t i = 0; i < P.npairs; ++i) {
        const int64_t lx = P.xo[i + 1] - P.xo[i] - 1, ly = P.yo[i + 1] - P.yo[i] - 1;
        sx += lx; sy += ly;
        mx = std::max(mx, lx); my = std::max(my, ly);
    }
    const int64_t n = std::max<int64_t>(P.npairs, 1);
    char b[96];
    std::snprintf(b, sizeof(b), "|P%d|x%d,%d|y%d,%d", clog2(P.npairs), clog2((sx + n - 1) / n),
                  clog2(mx), clog2((sy + n - 1) / n), clog2(my));
    return params_key("pairs", P.p_user, P.backward, P.d) + b;
}

std::string gram_key(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                     const sk_params& p, bool backward) {
    sk_params q = p;
    q.algo = SK_ALGO_BATCHED;  // tuned
    q.ckpt = 0;                // tuned
    char b[96];
    std::snprintf(b, sizeof(b), "|P%d,%d|x%d|y%d", clog2(nx), clog2(ny), clog2(lx_pts - 1),
                  clog2(ly_pts - 1));
    return params_key("gram", q, backward, d) + b;
}

bool tune_lookup(const std::string& k, TuneVal* v) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& e : g_tune_cache)
        if (e.first == k) {
            *v = e.second;
            return true;
        }
    return false;
}

void tune_store(const std::string& k, const TuneVal& v) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (auto& e : g_tune_cache)
        if (e.first == k) {
            e.second = v;
            return;
        }
    g_tune_cache.push_back({k, v});
}

bool tuned_cfg(const PlanImpl& P, PlanCfg* cfg) {
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (g_tune_cache.empty()) return false;  // no device query for an empty cache
    }
    TuneVal v;
    if (!tune_lookup(plan_key(P), &v)) return false;
    // the cached stride must still be valid for these parameters
    sk_params q = P.p_user;
    if (v.cfg.ckpt) q.ckpt = v.cfg.ckpt;
    const std::string saved = g_last_error;
    if (check_params(&q, P.backward)) {
        g_last_error = saved;
        return false;
    }
    *cfg = v.cfg;
    return true;
}

void remember_cfg(const PlanImpl& P, const PlanCfg& cfg, double ms) {
    TuneVal v;
    v.cfg = cfg;
    v.algo = SK_ALGO_BATCHED;
    v.ms = ms;
    tune_store(plan_key(P), v);
}

int plan_check_device(const PlanImpl& P) {
    if (P.npairs == 0) return SK_OK;
    return P.p.dtype == SK_F32 ? check_lds<float>(P.p, P.max_ly, P.d)
                               : check_lds<double>(P.p, P.max_ly, P.d);
}

int plan_upload(PlanImpl& P, void* ws, size_t wsb, hipStream_t st) {
    if ((size_t)P.total > wsb)
        return fail(SK_EWORKSPACE, "plan needs %lld bytes, got %zu", (long long)P.total, wsb);
    int rc = plan_check_device(P);
    if (rc) return rc;
    if (P.npairs > 0) {
        SK_TRY_HIP(hipMemcpyAsync((char*)ws + P.fdesc_off, P.fdesc.data(),
                                  P.fdesc.size() * sizeof(SkPairDesc), hipMemcpyHostToDevice, st),
                   "descriptor upload");
        if (P.backward)
            SK_TRY_HIP(hipMemcpyAsync((char*)ws + P.bdesc_off, P.bdesc.data(),
                                      P.bdesc.size() * sizeof(SkPairDesc), hipMemcpyHostToDevice,
                                      st),
                       "descriptor upload");
        if (!P.jobs.empty())
            SK_TRY_HIP(hipMemcpyAsync((char*)ws + P.jobs_off, P.jobs.data(),
                                      P.jobs.size() * sizeof(int2), hipMemcpyHostToDevice, st),
                       "job list upload");
        SK_TRY_HIP(hipStreamSynchronize(st), "descriptor upload");
    }
    P.uploaded = ws;
    return SK_OK;
}

int plan_ready(const PlanImpl& P, const void* ws, size_t wsb) {
    if (!ws) return fail(SK_EINVAL, "NULL workspace");
    if (P.uploaded != ws) return fail(SK_EINVAL, "plan descriptors were not uploaded to this workspace");
    if ((size_t)P.total > wsb)
        return fail(SK_EWORKSPACE, "plan needs %lld bytes, got %zu", (long long)P.total, wsb);
    return SK_OK;
}

template <typename R>
int plan_forward(const PlanImpl& P, const R* Xc, const R* Yc, R* K, int32_t* Kexp, void* ws,
                 hipStream_t st) {
    char* base = (char*)ws;
    for (const PlanChunk& c : P.fchunks) {
        const Layout L = layout_for(c.tot, c.count, sizeof(R), false, false, P.p.order);
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.desc = reinterpret_cast<const SkPairDesc*>(base + P.fdesc_off) + c.first;
        int rc = c.pipe ? run_chunk_forward_pipe<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_nsteps_pad,
                                                    c.max_lx, c.max_ly,
                                                    reinterpret_cast<const int2*>(base + P.jobs_off) + c.jobs_first,
                                                    c.njobs, base + P.scratch_off, L, K, Kexp, st)
                        : run_chunk_forward<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_nsteps_pad, c.max_lx,
                                               c.max_ly, c.ring_fwd, base + P.scratch_off, L, K, Kexp, st);
        if (rc) return rc;
    }
    return SK_OK;
}

// Backward state of one plan chunk: increment Gram and checkpoint sweep
// (kernel values to K, indexed by the descriptors' k_idx) ...
template <typename R>
int plan_chunk_prepare(const PlanImpl& P, const PlanChunk& c, const R* Xc, const R* Yc, R* K,
                       int32_t* Kexp, void* ws, hipStream_t st) {
    char* base = (char*)ws;
    const Layout L = layout_for(c.tot, c.count, sizeof(R), true, false, P.p.order);
    char* ws_c = base + P.scratch_off;
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.desc = reinterpret_cast<const SkPairDesc*>(base + P.bdesc_off) + c.first;
    if (c.pipe) {
        const int2* jobs = reinterpret_cast<const int2*>(base + P.jobs_off) + c.jobs_first;
        return run_chunk_prepare_pipe<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_nsteps_pad, c.max_lx,
                                         c.max_ly, jobs, c.njobs, ws_c, L, K, Kexp, st);
    }
    return run_chunk_prepare<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_nsteps_pad, c.max_lx,
                                c.max_ly, c.ring_fwd, ws_c, L, K, Kexp, st);
}

// ... then the adjoint, the contraction and the reduction into gX, gY.
template <typename R>
int plan_chunk_adjoint(const PlanImpl& P, const PlanChunk& c, const R* Xc, const R* Yc,
                       const R* gK, const int32_t* gKexp, R* gX, R* gY, void* ws, hipStream_t st) {
    char* base = (char*)ws;
    const Layout L = layout_for(c.tot, c.count, sizeof(R), true, false, P.p.order);
    char* ws_c = base + P.scratch_off;
    SkPairSrc src;
    std::memset(&src, 0, sizeof(src));
    src.desc = reinterpret_cast<const SkPairDesc*>(base + P.bdesc_off) + c.first;
    int rc;
    if (c.pipe) {
        const int2* jobs = reinterpret_cast<const int2*>(base + P.jobs_off) + c.jobs_first;
        rc = run_chunk_adjoint_pipe<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_strips, c.max_nsteps_pad,
                                       jobs + c.njobs, c.njobs, ws_c, L, gK, gKexp, st);
    } else {
        rc = run_chunk_adjoint<R>(P.p, Xc, Yc, P.d, src, c.count, c.max_ly, c.ring_adj, c.max_strips,
                                  c.max_nsteps_pad, ws_c, L, gK, gKexp, st);
    }
    if (rc) return rc;
    ReducePairsArgs<R> ra;
    ra.desc = src.desc; ra.count = c.count; ra.d = P.d; ra.max_pts = c.max_pts;
    ra.dxp = reinterpret_cast<const R*>(ws_c + L.dxp);
    ra.dyp = reinterpret_cast<const R*>(ws_c + L.dyp);
    ra.gX = gX; ra.gY = gY;
    SK_LAUNCH("reduce", st, SkLaunch<R>::reduce_pairs(ra, st), "gradient reduction");
    return SK_OK;
}

template <typename R>
int plan_backward(const PlanImpl& P, const R* Xc, const R* Yc, const R* gK, const int32_t* gKexp,
                  R* gX, R* gY, void* ws, hipStream_t st) {
    char* base = (char*)ws;
    SK_TRY_HIP(SkLaunch<R>::fill(gX, P.xo[P.npairs] * P.d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, P.yo[P.npairs] * P.d, (R)0, st), "fill");
    // kernel values of the checkpoint pass: scratch indexed by k_idx
    R* kbuf = reinterpret_cast<R*>(base + P.kbuf_off);
    int32_t* kexp = reinterpret_cast<int32_t*>(base + P.kexp_off);
    for (const PlanChunk& c : P.bchunks) {
        int rc = plan_chunk_prepare<R>(P, c, Xc, Yc, kbuf, kexp, ws, st);
        if (!rc) rc = plan_chunk_adjoint<R>(P, c, Xc, Yc, gK, gKexp, gX, gY, ws, st);
        if (rc) return rc;
    }
    return SK_OK;
}

// Forward that keeps the backward's state in the plan's workspace (plans
// whose backward is one chunk), and the backward that starts from it.
template <typename R>
int plan_forward_save(const PlanImpl& P, const R* Xc, const R* Yc, R* K, int32_t* Kexp, void* ws,
                      hipStream_t st) {
    if (P.bchunks.size() != 1)
        return fail(SK_EWORKSPACE, "the saved state needs the backward in one chunk (%zu chunks)",
                    P.bchunks.size());
    return plan_chunk_prepare<R>(P, P.bchunks[0], Xc, Yc, K, Kexp, ws, st);
}

template <typename R>
int plan_backward_saved(const PlanImpl& P, const R* Xc, const R* Yc, const R* gK,
                        const int32_t* gKexp, R* gX, R* gY, void* ws, hipStream_t st) {
    if (P.bchunks.size() != 1)
        return fail(SK_EWORKSPACE, "the saved state needs the backward in one chunk (%zu chunks)",
                    P.bchunks.size());
    SK_TRY_HIP(SkLaunch<R>::fill(gX, P.xo[P.npairs] * P.d, (R)0, st), "fill");
    SK_TRY_HIP(SkLaunch<R>::fill(gY, P.yo[P.npairs] * P.d, (R)0, st), "fill");
    return plan_chunk_adjoint<R>(P, P.bchunks[0], Xc, Yc, gK, gKexp, gX, gY, ws, st);
}

// Device buffers of a tuning run's backward: dL/dk = 1 and the gradients.
template <typename R>
struct TuneBufs {
    R* gk = nullptr;
    R* gx = nullptr;
    R* gy = nullptr;
    ~TuneBufs() {
        if (gk) (void)hipFree(gk);
        if (gx) (void)hipFree(gx);
        if (gy) (void)hipFree(gy);
    }
    int alloc(int64_t nk, int64_t nxv, int64_t nyv, hipStream_t st) {
        SK_TRY_HIP(hipMalloc((void**)&gk, std::max<int64_t>(nk, 1) * sizeof(R)), "tuning buffers");
        SK_TRY_HIP(hipMalloc((void**)&gx, std::max<int64_t>(nxv, 1) * sizeof(R)), "tuning buffers");
        SK_TRY_HIP(hipMalloc((void**)&gy, std::max<int64_t>(nyv, 1) * sizeof(R)), "tuning buffers");
        SK_TRY_HIP(SkLaunch<R>::fill(gk, std::max<int64_t>(nk, 1), (R)1, st), "fill");
        return SK_OK;
    }
};

// Device time (ms) of `run` on `st`: a warm-up, then the best of two runs.
template <typename F>
int time_best(F&& run, hipStream_t st, double* ms_out) {
    hipEvent_t e0, e1;
    SK_TRY_HIP(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SK_EHIP, "event");
    }
    int rc = SK_OK;
    double t = 1e30;
    for (int rep = 0; rep < 3 && !rc; ++rep) {
        hipError_t he = hipEventRecord(e0, st);
        if (he == hipSuccess) rc = run();
        if (!rc && he == hipSuccess) he = hipEventRecord(e1, st);
        if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (!rc && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (!rc && he != hipSuccess) rc = hip_fail(he, "tuning run");
        if (!rc && rep > 0) t = std::min(t, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) *ms_out = t;
    return rc;
}

// Configurations the plan tuner visits, in three stages, each starting from
// the best so far: (1) pair order, transposition and LDS classes, (2) the
// strip-pipeline threshold (every threshold that moves a different set of
// pairs to the pipeline), (3) for backward plans the checkpoint strides the
// precision offers.  Workspace need of a configuration: plan total.
std::vector<int32_t> pipe_thresholds(const PlanImpl& P, const PlanCfg& cfg) {
    std::vector<int32_t> out = {0};
    if (is_fd(P.p_user)) return out;
    const int lam = lam_of(P.p_user);
    std::vector<int32_t> ns(P.npairs);
    for (int64_t i = 0; i < P.npairs; ++i) {
        int lx = (int)(P.xo[i + 1] - P.xo[i] - 1), ly = (int)(P.yo[i + 1] - P.yo[i] - 1);
        if (cfg.swap && ly > lx) std::swap(lx, ly);
        ns[i] = sk_make_geom(lx << lam, ly << lam).nstrips;
    }
    int64_t prev = -1;
    for (int32_t k : {2, 3, 4, 6, 8, 12, 16, 24, 32, 64}) {
        int64_t cnt = 0;
        for (int32_t v : ns) cnt += v >= k;
        if (cnt == 0) break;
        if (cnt != prev) out.push_back(k);
        prev = cnt;
    }
    return out;
}
std::vector<int32_t> ckpt_choices(const sk_params& p, bool backward) {
    if (!backward || is_fd(p)) return {0};
    const bool f64 = p.dtype == SK_F64 || (p.flags & SK_SWEEP_F64);
    return f64 ? std::vector<int32_t>{2} : std::vector<int32_t>{4, 2};
}

// Largest workspace any configuration the tuner visits can need (host only).
int64_t plan_tune_workspace(const PlanImpl& P0) {
    PlanImpl P = P0;
    int64_t need = P0.total;
    for (int o = 0; o < 2; ++o)
        for (int w = 0; w < 2; ++w)
            for (int b = 0; b < 2; ++b)
                for (int32_t k : pipe_thresholds(P0, PlanCfg{o, w, b, 0, 0}))
                    for (int32_t s : ckpt_choices(P0.p_user, P0.backward)) {
                        const PlanCfg cfg = {o, w, b, k, s};
                        if (plan_build_into(P, cfg, SIZE_MAX) == SK_OK) need = std::max(need, P.total);
                    }
    g_last_error.clear();
    return need;
}

// Time the tuner's configurations on these inputs (forward, and for backward
// plans forward + backward with dL/dk = 1), keep the fastest in the plan,
// upload it and remember it for plans and one-shot calls of the same shape
// class.  Configurations whose workspace exceeds wsb are skipped.
template <typename R>
int plan_tune(PlanImpl& P, const R* Xc, const R* Yc, void* ws, size_t wsb, hipStream_t st,
              double* best_ms) {
    TuneBufs<R> tb;
    int rc = SK_OK;
    if (P.backward && (rc = tb.alloc(P.npairs, P.xo[P.npairs] * P.d, P.yo[P.npairs] * P.d, st)))
        return rc;
    PlanCfg best = P.cfg;
    double best_t = -1.0;
    auto visit = [&](const PlanCfg& cfg) -> int {
        int r = plan_build(P, cfg, wsb);
        if (r == SK_EWORKSPACE) {  // this configuration does not fit: skip it
            g_last_error.clear();
            return SK_OK;
        }
        if (r || (r = plan_upload(P, ws, wsb, st))) return r;
        R* K = reinterpret_cast<R*>((char*)ws + P.kbuf_off);
        double t = 0.0;
        r = time_best([&]() -> int {
            if (!P.backward) return plan_forward<R>(P, Xc, Yc, K, nullptr, ws, st);
            int q = plan_forward<R>(P, Xc, Yc, K, nullptr, ws, st);
            return q ? q : plan_backward<R>(P, Xc, Yc, tb.gk, nullptr, tb.gx, tb.gy, ws, st);
        }, st, &t);
        if (r) return r;
        if (best_t < 0 || t < best_t) {
            best_t = t;
            best = cfg;
        }
        return SK_OK;
    };
    const PlanCfg base = kDefaultPlanCfg;
    for (int o = 0; o < 2 && !rc; ++o)
        for (int w = 0; w < 2 && !rc; ++w)
            for (int b = 0; b < 2 && !rc; ++b) rc = visit(PlanCfg{o, w, b, base.pipe, base.ckpt});
    if (!rc) {
        const PlanCfg s1 = best;
        for (int32_t k : pipe_thresholds(P, s1))
            if (!rc && k != s1.pipe) rc = visit(PlanCfg{s1.order, s1.swap, s1.buckets, k, s1.ckpt});
    }
    if (!rc) {
        const PlanCfg s2 = best;
        for (int32_t c : ckpt_choices(P.p_user, P.backward))
            if (!rc && c != 0 && c != ckpt_stride(P.p_user))
                rc = visit(PlanCfg{s2.order, s2.swap, s2.buckets, s2.pipe, c});
    }
    if (rc) return rc;
    if (best_t < 0) return fail(SK_EWORKSPACE, "no configuration fits a workspace of %zu bytes", wsb);
    if ((rc = plan_build(P, best, wsb)) || (rc = plan_upload(P, ws, wsb, st))) return rc;
    remember_cfg(P, best, best_t);
    if (best_ms) *best_ms = best_t;
    return SK_OK;
}

// The plain algorithm on a list of pairs: one launch per pair, FP64.
template <typename R>
int pairs_plain(const R* Xc, const int64_t* xo, const R* Yc, const int64_t* yo, int64_t npairs,
                int64_t d, const sk_params& p, R* K, int32_t* Kexp, void* ws, size_t wsb,
                hipStream_t st) {
    const int lam = lam_of(p);
    PlainArgs<R> pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.d = d; pa.lam = lam; pa.tab = table_for<R>(p); pa.K = K; pa.Kexp = Kexp;
    pa.second = p.scheme == SK_FD2;
    pa.pst = reinterpret_cast<R*>(ws); pa.diag = reinterpret_cast<R*>(ws);
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t lx = xo[i + 1] - xo[i] - 1, ly = yo[i + 1] - yo[i] - 1;
        const int64_t need = std::max<int64_t>(((lx + ly) << lam) * (p.order + 1), 3 * ((lx << lam) + 1)) * 8;
        if (wsb < (size_t)need) return fail(SK_EWORKSPACE, "plain needs %lld bytes", (long long)need);
        pa.x = Xc + xo[i] * d; pa.y = Yc + yo[i] * d; pa.lx = (int)lx; pa.ly = (int)ly;
        pa.k_idx = i;
        if (lx == 0 || ly == 0) {
            SK_TRY_HIP(SkLaunch<R>::fill(K + i, 1, (R)1, st), "fill");
            if (Kexp) SK_TRY_HIP(SkLaunch<float>::fill_u32(reinterpret_cast<unsigned*>(Kexp + i), 1, st), "fill");
            continue;
        }
        if (is_fd(p))
            SK_LAUNCH("plain", st, SkLaunch<R>::plain_fd(pa, st), "plain finite differences");
        else
            SK_LAUNCH("plain", st, SkLaunch<R>::plain_poly(pa, p.order, p.scheme == SK_POLY_INTERP, st),
                      "plain polynomial sweep");
    }
    return SK_OK;
}

// One-shot pairs calls: a plan with the tuned configuration of this shape if
// there is one, else longest-first, transposed, bucketed and pipelined
// (SK_ALGO_PIPELINE: pipelined in any case, forward and backward).
int oneshot_plan(PlanImpl& P, const int64_t* xo, const int64_t* yo, int64_t npairs, int64_t d,
                 const sk_params& p, bool backward, size_t wsb) {
    plan_init(P, xo, yo, npairs, d, p, backward);
    PlanCfg cfg = kDefaultPlanCfg;
    tuned_cfg(P, &cfg);
    if (p.algo == SK_ALGO_PIPELINE) cfg.pipe = 2;  // the pipeline wherever a pair has several strips
    return plan_build(P, cfg, wsb);
}

// ---------------------------------------------------------------------------
// SK_SWEEP_F64: FP32 paths swept in FP64.  The points (and a backward's
// seeds) are promoted into the head of the workspace, the call runs on the
// FP64 path (cell constants of the promoted points in FP64, FP64 state),
// and its outputs are rounded back to FP32.
// ---------------------------------------------------------------------------
sk_params promoted(const sk_params& p) {
    sk_params q = p;
    q.dtype = SK_F64;
    q.flags &= ~SK_SWEEP_F64;
    return q;
}
// Head of the workspace: byte offsets of the FP64 copies.
struct PromoHead {
    int64_t x, y, k, gx, gy, total;
};
PromoHead promo_head(int64_t xn, int64_t yn, int64_t kn, bool backward, bool symmetric) {
    PromoHead h;
    int64_t o = 0;
    auto take = [&](int64_t n) { const int64_t at = o; o += align_up(n * 8); return at; };
    h.x = take(xn);
    h.y = symmetric ? h.x : take(yn);
    h.k = take(kn);  // K (forward) or gK (backward)
    h.gx = backward ? take(xn) : 0;
    h.gy = backward && !symmetric ? take(yn) : 0;
    h.total = o;
    return h;
}
int no_sweep_f64(const sk_params* p, const char* what) {
    if (p && (p->flags & SK_SWEEP_F64)) return fail(SK_EUNSUPPORTED, "SK_SWEEP_F64 is not offered by %s", what);
    return SK_OK;
}

// Device address of `scratch` on the current device, looked up on the first
// call on each device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
    int dev = 0;
    SK_TRY_HIP(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(SK_EUNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        SK_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static scratch address");
        if (!ptr) return fail(SK_EHIP, "static scratch address is NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SK_OK;
}

}  // namespace

struct sk_plan {
    PlanImpl impl;
};

// ===========================================================================
// exported C ABI
// ===========================================================================
extern "C" {

const char* sigkernel_error_string(int status) {
    switch (status) {
        case SK_OK: return "success";
        case SK_EINVAL: return "invalid argument";
        case SK_EWORKSPACE: return "workspace too small";
        case SK_EUNSUPPORTED: return "unsupported by this build";
        case SK_EHIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char* sigkernel_last_error(void) { return g_last_error.c_str(); }

int sigkernel_status(hipStream_t stream, int32_t clear, uint32_t* flags) {
    g_last_error.clear();
    if (!flags) return fail(SK_EINVAL, "flags is NULL");
    SK_TRY_HIP(hipStreamSynchronize(stream), "stream synchronize");
    unsigned* w[3] = {nullptr, nullptr, nullptr};
    SK_TRY_HIP(SkLaunch<float>::status_word(&w[0]), "status word (FP32 kernels)");
    SK_TRY_HIP(SkLaunch<double>::status_word(&w[1]), "status word (FP64 kernels)");
    SK_TRY_HIP(sk_hi_status_word(&w[2]), "status word (FP64 kernels, orders 9-12)");
    uint32_t f = 0;
    for (unsigned* p : w) {
        unsigned v = 0;
        SK_TRY_HIP(hipMemcpy(&v, p, sizeof(v), hipMemcpyDeviceToHost), "status read");
        f |= v;
        if (clear) {
            const unsigned z = 0;
            SK_TRY_HIP(hipMemcpy(p, &z, sizeof(z), hipMemcpyHostToDevice), "status clear");
        }
    }
    *flags = f;
    return SK_OK;
}

int sigkernel_interp_table(int32_t order, int32_t dtype, double* rs, double* rmax, double* cmax,
                           int32_t* tail_cap) {
    g_last_error.clear();
    if (order < SK_MIN_POLY_ORDER || order > SK_NMAX)
        return fail(SK_EINVAL, "order %d outside [%d, %d]", order, SK_MIN_POLY_ORDER, SK_NMAX);
    if (dtype != SK_F32 && dtype != SK_F64) return fail(SK_EINVAL, "dtype %d", dtype);
    if (!rs || !rmax || !cmax || !tail_cap) return fail(SK_EINVAL, "NULL pointer");
    const InterpTableF64 t = build_interp_table(order);
    for (int n = 0; n <= order; ++n)
        for (int k = 0; k < SK_TMAX; ++k) rs[n * SK_TMAX + k] = t.rs[n][k];
    for (int k = 0; k <= SK_TMAX; ++k) {
        rmax[k] = t.rmax[k];
        cmax[k] = t.cmax[k];
    }
    *tail_cap = dtype == SK_F32 ? SkTailMax<float>::value : SkTailMax<double>::value;
    return SK_OK;
}

int sigkernel_set_spin_limit(int32_t polls) {
    g_last_error.clear();
    if (polls < 0) return fail(SK_EINVAL, "spin limit %d < 0", polls);
    g_spin_limit.store(polls == 0 ? kPipeSpinLimit : polls);
    return SK_OK;
}

int sigkernel_profile_enable(int32_t on) {
    g_last_error.clear();
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (ProfRec& r : g_prof_recs) {
        (void)hipEventSynchronize(r.stop);
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_recs.clear();
    g_prof.store(on != 0);
    return SK_OK;
}

int sigkernel_profile_read(const char* name, double* total_ms, int64_t* launches) {
    g_last_error.clear();
    if (!name || !total_ms || !launches) return fail(SK_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> g(g_prof_mu);
    double tot = 0.0;
    int64_t n = 0;
    for (ProfRec& r : g_prof_recs) {
        if (std::strcmp(r.name, name) != 0) continue;
        SK_TRY_HIP(hipEventSynchronize(r.stop), "event synchronize");
        float ms = 0.f;
        SK_TRY_HIP(hipEventElapsedTime(&ms, r.start, r.stop), "event elapsed time");
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return SK_OK;
}

size_t sigkernel_gram_workspace(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                                const sk_params* p, int32_t backward) {
    g_last_error.clear();
    if (check_params(p, backward != 0) || check_dims(d, backward != 0) ||
        check_gram_geom(lx_pts, ly_pts, lam_of(*p)))
        return 0;
    if (nx < 0 || ny < 0) { fail(SK_EINVAL, "negative batch"); return 0; }
    if (p->flags & SK_SWEEP_F64) {
        const sk_params q = promoted(*p);
        const size_t inner = sigkernel_gram_workspace(nx, lx_pts, ny, ly_pts, d, &q, backward);
        if (!inner) return 0;
        const bool sym = (p->flags & SK_SYMMETRIC) != 0;
        return (size_t)promo_head(nx * lx_pts * d, ny * ly_pts * d, nx * ny, backward != 0, sym).total + inner;
    }
    const int lam = lam_of(*p);
    // the pipeline where the (refined) grid has several strips, else batched
    if (p->algo == SK_ALGO_PIPELINE && nx * ny > 0 &&
        sk_make_geom((int)((lx_pts - 1) << lam), (int)((ly_pts - 1) << lam)).nstrips >= 2) {
        GramPipePlan G;
        if (gram_pipe_plan(nx, lx_pts, ny, ly_pts, d, *p, backward != 0, kDefaultCap, &G)) return 0;
        return std::max<size_t>(256, (size_t)G.total);
    }
    if (p->algo == SK_ALGO_PLAIN) {
        int64_t lx = lx_pts - 1, ly = ly_pts - 1;
        return (size_t)std::max<int64_t>(256, std::max<int64_t>(((lx + ly) << lam) * (p->order + 1),
                                                               3 * ((lx << lam) + 1)) * 8);
    }
    const SkPairSizes per = sk_pair_sizes((int)(lx_pts - 1), (int)(ly_pts - 1), lam, p->order,
                                          ckpt_stride(*p), d, backward != 0,
                                          xb_words_of(*p, (int)(ly_pts - 1)));
    const int64_t npairs = std::max<int64_t>(1, nx * ny);
    int64_t P = gram_chunk(per, npairs, esize(*p), backward != 0, kDefaultCap, p->order);
    if (P <= 0) P = 1;
    return std::max<size_t>(256, (size_t)layout_for(scale(per, P), P, esize(*p), backward != 0, false, p->order).total);
}

size_t sigkernel_pairs_workspace(const int64_t* x_off, const int64_t* y_off, int64_t npairs,
                                 int64_t d, const sk_params* p, int32_t backward) {
    g_last_error.clear();
    if (check_params(p, backward != 0) || check_dims(d, backward != 0)) return 0;
    if (npairs < 0) { fail(SK_EINVAL, "negative npairs"); return 0; }
    if (check_pairs_geom(x_off, y_off, npairs, lam_of(*p)))
        return 0;
    if (p->flags & SK_SWEEP_F64) {
        const sk_params q = promoted(*p);
        const size_t inner = sigkernel_pairs_workspace(x_off, y_off, npairs, d, &q, backward);
        if (!inner) return 0;
        return (size_t)promo_head(x_off[npairs] * d, y_off[npairs] * d, npairs, backward != 0, false).total + inner;
    }
    const int lam = lam_of(*p);
    if (p->algo == SK_ALGO_PLAIN) {
        int64_t need = 256;
        for (int64_t i = 0; i < npairs; ++i) {
            int64_t lx = x_off[i + 1] - x_off[i] - 1, ly = y_off[i + 1] - y_off[i] - 1;
            need = std::max(need, std::max<int64_t>(((lx + ly) << lam) * (p->order + 1), 3 * ((lx << lam) + 1)) * 8);
        }
        return (size_t)need;
    }
    try {
        PlanImpl P;
        if (oneshot_plan(P, x_off, y_off, npairs, d, *p, backward != 0, SIZE_MAX)) return 0;
        return (size_t)P.total;
    } catch (...) {
        fail(SK_EINVAL, "internal exception");
        return 0;
    }
}

int sigkernel_gram(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                   int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                   void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc = check_params(p, false);
    if (!rc) rc = check_dims(d, false);
    if (rc) return rc;
    if (nx < 0 || ny < 0) return fail(SK_EINVAL, "negative batch");
    if ((rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p))))
        return rc;
    if (nx * ny == 0) return SK_OK;
    if (!X || !Y || !K || !ws) return fail(SK_EINVAL, "NULL pointer");
    if (p->flags & SK_SWEEP_F64) {
        const PromoHead h = promo_head(nx * lx_pts * d, ny * ly_pts * d, nx * ny, false, false);
        if (ws_bytes < (size_t)h.total) return fail(SK_EWORKSPACE, "workspace smaller than the FP64 copies");
        char* w = (char*)ws;
        double *X64 = (double*)(w + h.x), *Y64 = (double*)(w + h.y), *K64 = (double*)(w + h.k);
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)X, X64, nx * lx_pts * d, stream), "promote X");
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)Y, Y64, ny * ly_pts * d, stream), "promote Y");
        const sk_params q = promoted(*p);
        if ((rc = sigkernel_gram(X64, nx, lx_pts, Y64, ny, ly_pts, d, &q, K64, K_exp, w + h.total,
                                 ws_bytes - h.total, stream)))
            return rc;
        SK_TRY_HIP(SkLaunch<float>::from_f64(K64, (float*)K, nx * ny, stream), "round K");
        return SK_OK;
    }
    try {
        if (p->dtype == SK_F32)
            return gram_forward<float>((const float*)X, nx, lx_pts, (const float*)Y, ny, ly_pts, d,
                                       *p, (float*)K, K_exp, ws, ws_bytes, stream);
        return gram_forward<double>((const double*)X, nx, lx_pts, (const double*)Y, ny, ly_pts, d,
                                    *p, (double*)K, K_exp, ws, ws_bytes, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_gram_static(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                          int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                          hipStream_t stream) {
    g_last_error.clear();
    if (no_sweep_f64(p, "the static-scratch Gram")) return SK_EUNSUPPORTED;
    int rc = check_params(p, false);
    if (!rc) rc = check_dims(d, false);
    if (rc) return rc;
    if (p->algo == SK_ALGO_PIPELINE)
        return fail(SK_EUNSUPPORTED, "the static-scratch Gram runs the batched and plain algorithms");
    if (nx < 0 || ny < 0) return fail(SK_EINVAL, "negative batch");
    if ((rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p)))) return rc;
    if (nx * ny == 0) return SK_OK;
    if (!X || !Y || !K) return fail(SK_EINVAL, "NULL pointer");
    // one pair must fit in the scratch (work is chunked to it)
    const size_t one = sigkernel_gram_workspace(1, lx_pts, 1, ly_pts, d, p, 0);
    if (one == 0) return SK_EINVAL;
    if (one > SK_STATIC_SCRATCH_BYTES)
        return fail(SK_EWORKSPACE,
                    "one pair needs %zu bytes of workspace, more than the %zu-byte static scratch "
                    "(use sigkernel_gram with a workspace)", one, (size_t)SK_STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    try {
        if (p->dtype == SK_F32)
            return gram_forward<float>((const float*)X, nx, lx_pts, (const float*)Y, ny, ly_pts, d,
                                       *p, (float*)K, K_exp, ws, SK_STATIC_SCRATCH_BYTES, stream);
        return gram_forward<double>((const double*)X, nx, lx_pts, (const double*)Y, ny, ly_pts, d,
                                    *p, (double*)K, K_exp, ws, SK_STATIC_SCRATCH_BYTES, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_pairs(const void* Xcat, const int64_t* x_off, const void* Ycat, const int64_t* y_off,
                    int64_t npairs, int64_t d, const sk_params* p, void* k, int32_t* k_exp,
                    void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc = check_params(p, false);
    if (!rc) rc = check_dims(d, false);
    if (rc) return rc;
    if (npairs < 0) return fail(SK_EINVAL, "negative npairs");
    if (npairs == 0) return SK_OK;
    if ((rc = check_pairs_geom(x_off, y_off, npairs, lam_of(*p))))
        return rc;
    if (!Xcat || !Ycat || !k || !ws) return fail(SK_EINVAL, "NULL pointer");
    if (p->flags & SK_SWEEP_F64) {
        const int64_t xn = x_off[npairs] * d, yn = y_off[npairs] * d;
        const PromoHead h = promo_head(xn, yn, npairs, false, false);
        if (ws_bytes < (size_t)h.total) return fail(SK_EWORKSPACE, "workspace smaller than the FP64 copies");
        char* w = (char*)ws;
        double *X64 = (double*)(w + h.x), *Y64 = (double*)(w + h.y), *k64 = (double*)(w + h.k);
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)Xcat, X64, xn, stream), "promote X");
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)Ycat, Y64, yn, stream), "promote Y");
        const sk_params q = promoted(*p);
        if ((rc = sigkernel_pairs(X64, x_off, Y64, y_off, npairs, d, &q, k64, k_exp, w + h.total,
                                  ws_bytes - h.total, stream)))
            return rc;
        SK_TRY_HIP(SkLaunch<float>::from_f64(k64, (float*)k, npairs, stream), "round k");
        return SK_OK;
    }
    try {
        if (p->algo == SK_ALGO_PLAIN) {
            if (p->dtype == SK_F32)
                return pairs_plain<float>((const float*)Xcat, x_off, (const float*)Ycat, y_off,
                                          npairs, d, *p, (float*)k, k_exp, ws, ws_bytes, stream);
            return pairs_plain<double>((const double*)Xcat, x_off, (const double*)Ycat, y_off,
                                       npairs, d, *p, (double*)k, k_exp, ws, ws_bytes, stream);
        }
        PlanImpl P;
        if ((rc = oneshot_plan(P, x_off, y_off, npairs, d, *p, false, ws_bytes)) ||
            (rc = plan_upload(P, ws, ws_bytes, stream)))
            return rc;
        if (p->dtype == SK_F32)
            return plan_forward<float>(P, (const float*)Xcat, (const float*)Ycat, (float*)k, k_exp,
                                       ws, stream);
        return plan_forward<double>(P, (const double*)Xcat, (const double*)Ycat, (double*)k, k_exp,
                                    ws, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_backward(int32_t op, const void* X, const int64_t* x_off, int64_t nx, int64_t lx_pts,
                       const void* Y, const int64_t* y_off, int64_t ny, int64_t ly_pts, int64_t d,
                       const sk_params* p, const void* gK, const int32_t* gK_exp, void* gX,
                       void* gY, void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc = check_params(p, true);
    if (!rc) rc = check_dims(d, true);
    if (rc) return rc;
    if (is_fd(*p)) return fail(SK_EUNSUPPORTED, "backward of the finite-difference scheme");
    if (op != SK_OP_GRAM && op != SK_OP_PAIRS) return fail(SK_EINVAL, "op %d", op);
    if (nx < 0 || (op == SK_OP_GRAM && ny < 0)) return fail(SK_EINVAL, "negative batch");
    if (op == SK_OP_GRAM) {
        if ((rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p)))) return rc;
    } else {
        if ((rc = check_pairs_geom(x_off, y_off, nx, lam_of(*p))))
            return rc;
    }
    if ((rc = check_symmetric(*p, op, X, nx, lx_pts, Y, ny, ly_pts, gX, &gY))) return rc;
    if (!X || !Y || !gK || !gX || !gY || !ws) return fail(SK_EINVAL, "NULL pointer");
    if (p->flags & SK_SWEEP_F64) {
        const bool sym = (p->flags & SK_SYMMETRIC) != 0;
        const int64_t xn = (op == SK_OP_GRAM ? nx * lx_pts : x_off[nx]) * d;
        const int64_t yn = (op == SK_OP_GRAM ? ny * ly_pts : y_off[nx]) * d;
        const int64_t kn = op == SK_OP_GRAM ? nx * ny : nx;
        const PromoHead h = promo_head(xn, yn, kn, true, sym);
        if (ws_bytes < (size_t)h.total) return fail(SK_EWORKSPACE, "workspace smaller than the FP64 copies");
        char* w = (char*)ws;
        double *X64 = (double*)(w + h.x), *Y64 = (double*)(w + h.y), *gK64 = (double*)(w + h.k);
        double *gX64 = (double*)(w + h.gx), *gY64 = sym ? gX64 : (double*)(w + h.gy);
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)X, X64, xn, stream), "promote X");
        if (!sym) SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)Y, Y64, yn, stream), "promote Y");
        SK_TRY_HIP(SkLaunch<float>::to_f64((const float*)gK, gK64, kn, stream), "promote gK");
        const sk_params q = promoted(*p);
        if ((rc = sigkernel_backward(op, X64, x_off, nx, lx_pts, Y64, y_off, ny, ly_pts, d, &q, gK64,
                                     gK_exp, gX64, gY64, w + h.total, ws_bytes - h.total, stream)))
            return rc;
        SK_TRY_HIP(SkLaunch<float>::from_f64(gX64, (float*)gX, xn, stream), "round gX");
        if (!sym) SK_TRY_HIP(SkLaunch<float>::from_f64(gY64, (float*)gY, yn, stream), "round gY");
        return SK_OK;
    }
    try {
        if (op == SK_OP_GRAM && p->algo == SK_ALGO_PIPELINE) {
            if (p->dtype == SK_F32)
                return gram_backward_pipe<float>((const float*)X, nx, lx_pts, (const float*)Y, ny,
                                                 ly_pts, d, *p, (const float*)gK, gK_exp,
                                                 (float*)gX, (float*)gY, ws, ws_bytes, stream);
            return gram_backward_pipe<double>((const double*)X, nx, lx_pts, (const double*)Y, ny,
                                              ly_pts, d, *p, (const double*)gK, gK_exp,
                                              (double*)gX, (double*)gY, ws, ws_bytes, stream);
        }
        if (op == SK_OP_GRAM) {
            if (p->dtype == SK_F32)
                return gram_backward<float>((const float*)X, nx, lx_pts, (const float*)Y, ny,
                                            ly_pts, d, *p, (const float*)gK, gK_exp, (float*)gX,
                                            (float*)gY, ws, ws_bytes, stream);
            return gram_backward<double>((const double*)X, nx, lx_pts, (const double*)Y, ny,
                                         ly_pts, d, *p, (const double*)gK, gK_exp, (double*)gX,
                                         (double*)gY, ws, ws_bytes, stream);
        }
        PlanImpl P;
        if ((rc = oneshot_plan(P, x_off, y_off, nx, d, *p, true, ws_bytes)) ||
            (rc = plan_upload(P, ws, ws_bytes, stream)))
            return rc;
        if (p->dtype == SK_F32)
            return plan_backward<float>(P, (const float*)X, (const float*)Y, (const float*)gK,
                                        gK_exp, (float*)gX, (float*)gY, ws, stream);
        return plan_backward<double>(P, (const double*)X, (const double*)Y, (const double*)gK,
                                     gK_exp, (double*)gX, (double*)gY, ws, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_create(const int64_t* x_off, const int64_t* y_off, int64_t npairs, int64_t d,
                          const sk_params* p, int32_t backward, size_t ws_bytes, sk_plan** plan) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (no_sweep_f64(p, "plans")) return SK_EUNSUPPORTED;
    int rc = check_params(p, backward != 0);
    if (!rc) rc = check_dims(d, backward != 0);
    if (rc) return rc;
    if (p->algo != SK_ALGO_BATCHED) return fail(SK_EUNSUPPORTED, "plans run the batched algorithm");
    if (p->flags & SK_SYMMETRIC) return fail(SK_EINVAL, "SK_SYMMETRIC applies to Gram calls");
    if (npairs < 0) return fail(SK_EINVAL, "negative npairs");
    const int lam = lam_of(*p);
    if ((rc = check_pairs_geom(x_off, y_off, npairs, lam_of(*p))))
        return rc;
    try {
        sk_plan* P = new sk_plan();
        plan_init(P->impl, x_off, y_off, npairs, d, *p, backward != 0);
        PlanCfg cfg = kDefaultPlanCfg;
        tuned_cfg(P->impl, &cfg);
        rc = plan_build(P->impl, cfg, ws_bytes == 0 ? SIZE_MAX : ws_bytes);
        if (rc) {
            delete P;
            return rc;
        }
        *plan = P;
        return SK_OK;
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

size_t sigkernel_plan_workspace(const sk_plan* plan) {
    g_last_error.clear();
    if (!plan) {
        fail(SK_EINVAL, "plan is NULL");
        return 0;
    }
    return (size_t)plan->impl.total;
}

int sigkernel_plan_upload(sk_plan* plan, void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !ws) return fail(SK_EINVAL, "NULL pointer");
    try {
        return plan_upload(plan->impl, ws, ws_bytes, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_forward(const sk_plan* plan, const void* Xcat, const void* Ycat, void* k,
                           int32_t* k_exp, void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    const PlanImpl& P = plan->impl;
    int rc = plan_ready(P, ws, ws_bytes);
    if (rc) return rc;
    if (P.npairs == 0) return SK_OK;
    if (!Xcat || !Ycat || !k) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (P.p.dtype == SK_F32)
            return plan_forward<float>(P, (const float*)Xcat, (const float*)Ycat, (float*)k, k_exp,
                                       ws, stream);
        return plan_forward<double>(P, (const double*)Xcat, (const double*)Ycat, (double*)k, k_exp,
                                    ws, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_backward(const sk_plan* plan, const void* Xcat, const void* Ycat,
                            const void* gk, const int32_t* gk_exp, void* gX, void* gY, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    const PlanImpl& P = plan->impl;
    if (!P.backward) return fail(SK_EINVAL, "plan was created without backward");
    int rc = plan_ready(P, ws, ws_bytes);
    if (rc) return rc;
    if (P.npairs == 0) return SK_OK;
    if (!Xcat || !Ycat || !gk || !gX || !gY) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (P.p.dtype == SK_F32)
            return plan_backward<float>(P, (const float*)Xcat, (const float*)Ycat,
                                        (const float*)gk, gk_exp, (float*)gX, (float*)gY, ws,
                                        stream);
        return plan_backward<double>(P, (const double*)Xcat, (const double*)Ycat,
                                     (const double*)gk, gk_exp, (double*)gX, (double*)gY, ws,
                                     stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_forward_save(const sk_plan* plan, const void* Xcat, const void* Ycat, void* k,
                                int32_t* k_exp, void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    const PlanImpl& P = plan->impl;
    if (!P.backward) return fail(SK_EINVAL, "plan was created without backward");
    int rc = plan_ready(P, ws, ws_bytes);
    if (rc) return rc;
    if (P.npairs == 0) return SK_OK;
    if (!Xcat || !Ycat || !k) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (P.p.dtype == SK_F32)
            return plan_forward_save<float>(P, (const float*)Xcat, (const float*)Ycat, (float*)k,
                                            k_exp, ws, stream);
        return plan_forward_save<double>(P, (const double*)Xcat, (const double*)Ycat, (double*)k,
                                         k_exp, ws, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_backward_saved(const sk_plan* plan, const void* Xcat, const void* Ycat,
                                  const void* gk, const int32_t* gk_exp, void* gX, void* gY,
                                  void* ws, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    const PlanImpl& P = plan->impl;
    if (!P.backward) return fail(SK_EINVAL, "plan was created without backward");
    int rc = plan_ready(P, ws, ws_bytes);
    if (rc) return rc;
    if (P.npairs == 0) return SK_OK;
    if (!Xcat || !Ycat || !gk || !gX || !gY) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (P.p.dtype == SK_F32)
            return plan_backward_saved<float>(P, (const float*)Xcat, (const float*)Ycat,
                                              (const float*)gk, gk_exp, (float*)gX, (float*)gY, ws,
                                              stream);
        return plan_backward_saved<double>(P, (const double*)Xcat, (const double*)Ycat,
                                           (const double*)gk, gk_exp, (double*)gX, (double*)gY, ws,
                                           stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_tune(sk_plan* plan, const void* Xcat, const void* Ycat, void* ws,
                        size_t ws_bytes, hipStream_t stream, double* best_ms) {
    g_last_error.clear();
    if (!plan || !Xcat || !Ycat || !ws) return fail(SK_EINVAL, "NULL pointer");
    if (plan->impl.npairs == 0) return SK_OK;
    try {
        if (plan->impl.p.dtype == SK_F32)
            return plan_tune<float>(plan->impl, (const float*)Xcat, (const float*)Ycat, ws,
                                    ws_bytes, stream, best_ms);
        return plan_tune<double>(plan->impl, (const double*)Xcat, (const double*)Ycat, ws,
                                 ws_bytes, stream, best_ms);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_plan_config(const sk_plan* plan, int32_t* order, int32_t* swap, int32_t* buckets,
                          int32_t* pipeline, int64_t* launches) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    if (order) *order = plan->impl.cfg.order;
    if (swap) *swap = plan->impl.cfg.swap;
    if (buckets) *buckets = plan->impl.cfg.buckets;
    if (pipeline) *pipeline = plan->impl.cfg.pipe >= 2 ? 1 : 0;
    if (launches) *launches = (int64_t)plan->impl.fchunks.size();
    return SK_OK;
}

int sigkernel_plan_configure(sk_plan* plan, int32_t order, int32_t swap, int32_t buckets,
                             int32_t pipeline, size_t ws_bytes) {
    g_last_error.clear();
    if (!plan) return fail(SK_EINVAL, "plan is NULL");
    if ((order | swap | buckets | pipeline) & ~1) return fail(SK_EINVAL, "configuration flags are 0 or 1");
    try {
        PlanCfg cfg = plan->impl.cfg;
        cfg.order = order; cfg.swap = swap; cfg.buckets = buckets; cfg.pipe = pipeline ? 2 : 0;
        return plan_build(plan->impl, cfg, ws_bytes == 0 ? SIZE_MAX : ws_bytes);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

void sigkernel_plan_destroy(sk_plan* plan) { delete plan; }

int sigkernel_mmd_permutation(const void* Kzz, int64_t m, int64_t n, const int32_t* perms,
                              int64_t nperm, int32_t dtype, void* stats, double* p_value,
                              hipStream_t stream) {
    g_last_error.clear();
    if (dtype != SK_F32 && dtype != SK_F64) return fail(SK_EINVAL, "dtype %d", dtype);
    if (m < 2 || n < 2) return fail(SK_EINVAL, "each sample needs at least 2 paths (m=%lld, n=%lld)",
                                    (long long)m, (long long)n);
    if (m + n > (1 << 20)) return fail(SK_EUNSUPPORTED, "pooled sample above 2^20 paths");
    if (nperm < 1) return fail(SK_EINVAL, "nperm %lld < 1", (long long)nperm);
    if (!Kzz || !perms || !stats) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (dtype == SK_F32)
            SK_LAUNCH("mmd_perm", stream,
                      SkLaunch<float>::mmd_perm((const float*)Kzz, m, n, perms, nperm,
                                                (float*)stats, p_value, stream),
                      "MMD permutation statistics");
        else
            SK_LAUNCH("mmd_perm", stream,
                      SkLaunch<double>::mmd_perm((const double*)Kzz, m, n, perms, nperm,
                                                 (double*)stats, p_value, stream),
                      "MMD permutation statistics");
        return SK_OK;
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

static int check_mmd2(int64_t nx, int64_t ny, int32_t dtype, const void* a, const void* b) {
    if (dtype != SK_F32 && dtype != SK_F64) return fail(SK_EINVAL, "dtype %d", dtype);
    if (nx < 2 || ny < 2)
        return fail(SK_EINVAL, "each set needs at least 2 paths (nx=%lld, ny=%lld)", (long long)nx,
                    (long long)ny);
    if (nx > (1 << 24) || ny > (1 << 24)) return fail(SK_EUNSUPPORTED, "set above 2^24 paths");
    if (!a || !b) return fail(SK_EINVAL, "NULL pointer");
    return SK_OK;
}

int sigkernel_mmd2_pairs(const void* k, int64_t nx, int64_t ny, int32_t dtype, void* out,
                         hipStream_t stream) {
    g_last_error.clear();
    if (int rc = check_mmd2(nx, ny, dtype, k, out)) return rc;
    try {
        if (dtype == SK_F32)
            SK_LAUNCH("mmd2", stream,
                      SkLaunch<float>::mmd2_pairs((const float*)k, nx, ny, (float*)out, stream),
                      "MMD^2 of a pair list");
        else
            SK_LAUNCH("mmd2", stream,
                      SkLaunch<double>::mmd2_pairs((const double*)k, nx, ny, (double*)out, stream),
                      "MMD^2 of a pair list");
        return SK_OK;
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_mmd2_pairs_backward(const void* gout, int64_t nx, int64_t ny, int32_t dtype, void* gk,
                                  hipStream_t stream) {
    g_last_error.clear();
    if (int rc = check_mmd2(nx, ny, dtype, gout, gk)) return rc;
    try {
        if (dtype == SK_F32)
            SK_LAUNCH("mmd2", stream,
                      SkLaunch<float>::mmd2_pairs_seed((const float*)gout, nx, ny, (float*)gk,
                                                       stream),
                      "MMD^2 seeds");
        else
            SK_LAUNCH("mmd2", stream,
                      SkLaunch<double>::mmd2_pairs_seed((const double*)gout, nx, ny, (double*)gk,
                                                        stream),
                      "MMD^2 seeds");
        return SK_OK;
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

size_t sigkernel_gram_state_size(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                                 const sk_params* p) {
    g_last_error.clear();
    if (no_sweep_f64(p, "the saved-state calls")) return 0;
    if (check_params(p, true) || check_dims(d, true) || check_gram_geom(lx_pts, ly_pts, lam_of(*p)))
        return 0;
    if (nx < 0 || ny < 0) { fail(SK_EINVAL, "negative batch"); return 0; }
    if (gram_pipe_applies(*p, nx, lx_pts, ny, ly_pts)) {
        GramPipePlan G;
        if (gram_pipe_state(nx, lx_pts, ny, ly_pts, d, *p, &G)) return 0;
        return std::max<size_t>(256, (size_t)G.total);
    }
    SkPairSizes per;
    Layout L;
    if (p->dtype == SK_F32) gram_state_layout<float>(nx, lx_pts, ny, ly_pts, d, *p, &per, &L);
    else gram_state_layout<double>(nx, lx_pts, ny, ly_pts, d, *p, &per, &L);
    return std::max<size_t>(256, (size_t)L.total);
}

int sigkernel_gram_save(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                        int64_t ly_pts, int64_t d, const sk_params* p, void* K, int32_t* K_exp,
                        void* state, size_t state_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (no_sweep_f64(p, "the saved-state calls")) return SK_EUNSUPPORTED;
    int rc = check_params(p, true);
    if (!rc) rc = check_dims(d, true);
    if (rc) return rc;
    if (nx < 0 || ny < 0) return fail(SK_EINVAL, "negative batch");
    if ((rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p)))) return rc;
    if (nx * ny == 0) return SK_OK;
    if (!X || !Y || !K || !state) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (gram_pipe_applies(*p, nx, lx_pts, ny, ly_pts)) {
            if (p->dtype == SK_F32)
                return gram_save_pipe<float>((const float*)X, nx, lx_pts, (const float*)Y, ny, ly_pts,
                                             d, *p, (float*)K, K_exp, state, state_bytes, stream);
            return gram_save_pipe<double>((const double*)X, nx, lx_pts, (const double*)Y, ny, ly_pts,
                                          d, *p, (double*)K, K_exp, state, state_bytes, stream);
        }
        if (p->dtype == SK_F32)
            return gram_save<float>((const float*)X, nx, lx_pts, (const float*)Y, ny, ly_pts, d, *p,
                                    (float*)K, K_exp, state, state_bytes, stream);
        return gram_save<double>((const double*)X, nx, lx_pts, (const double*)Y, ny, ly_pts, d, *p,
                                 (double*)K, K_exp, state, state_bytes, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_gram_backward_saved(const void* X, int64_t nx, int64_t lx_pts, const void* Y,
                                  int64_t ny, int64_t ly_pts, int64_t d, const sk_params* p,
                                  const void* gK, const int32_t* gK_exp, void* gX, void* gY,
                                  void* state, size_t state_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (no_sweep_f64(p, "the saved-state calls")) return SK_EUNSUPPORTED;
    if (no_sweep_f64(p, "the saved-state calls")) return SK_EUNSUPPORTED;
    int rc = check_params(p, true);
    if (!rc) rc = check_dims(d, true);
    if (rc) return rc;
    if (nx < 0 || ny < 0) return fail(SK_EINVAL, "negative batch");
    if ((rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p)))) return rc;
    if ((rc = check_symmetric(*p, SK_OP_GRAM, X, nx, lx_pts, Y, ny, ly_pts, gX, &gY))) return rc;
    if (!X || !Y || !gK || !gX || !gY || !state) return fail(SK_EINVAL, "NULL pointer");
    try {
        if (gram_pipe_applies(*p, nx, lx_pts, ny, ly_pts)) {
            if (p->dtype == SK_F32)
                return gram_backward_saved_pipe<float>((const float*)X, nx, lx_pts, (const float*)Y,
                                                       ny, ly_pts, d, *p, (const float*)gK, gK_exp,
                                                       (float*)gX, (float*)gY, state, state_bytes,
                                                       stream);
            return gram_backward_saved_pipe<double>((const double*)X, nx, lx_pts, (const double*)Y,
                                                    ny, ly_pts, d, *p, (const double*)gK, gK_exp,
                                                    (double*)gX, (double*)gY, state, state_bytes,
                                                    stream);
        }
        if (p->dtype == SK_F32)
            return gram_backward_saved<float>((const float*)X, nx, lx_pts, (const float*)Y, ny,
                                              ly_pts, d, *p, (const float*)gK, gK_exp, (float*)gX,
                                              (float*)gY, state, state_bytes, stream);
        return gram_backward_saved<double>((const double*)X, nx, lx_pts, (const double*)Y, ny,
                                           ly_pts, d, *p, (const double*)gK, gK_exp, (double*)gX,
                                           (double*)gY, state, state_bytes, stream);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_cell_constants(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                             int64_t ly_pts, int64_t d, const sk_params* pp, void* C, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!pp) return fail(SK_EINVAL, "params is NULL");
    const int32_t dtype = pp->dtype;
    sk_params p = {SK_POLY_APPROX, SK_MIN_POLY_ORDER, dtype, SK_ALGO_BATCHED, pp->gram, 0};
    int rc = check_params(&p, false);
    if (!rc) rc = check_dims(d, false);
    if (rc) return rc;
    if (nx < 0 || ny < 0) return fail(SK_EINVAL, "negative batch");
    if ((rc = check_gram_geom(lx_pts, ly_pts, 0))) return rc;
    const int64_t npairs = nx * ny, lx = lx_pts - 1, ly = ly_pts - 1;
    if (npairs == 0 || lx == 0 || ly == 0) return SK_OK;
    if (!X || !Y || !C || !ws) return fail(SK_EINVAL, "NULL pointer");
    const size_t es = esize(p);
    const SkPairSizes per = sk_pair_sizes((int)lx, (int)ly, 0, p.order, ckpt_stride(p), d, false, xb_words_of(p, (int)ly));
    const int64_t P = gram_chunk(per, npairs, es, false, ws_bytes, p.order);
    if (P <= 0) return fail(SK_EWORKSPACE, "workspace of %zu bytes holds no pair", ws_bytes);
    const Layout L = layout_for(scale(per, P), P, es, false, false, p.order);
    const SkGeom g = sk_make_geom((int)lx, (int)ly);
    for (int64_t first = 0; first < npairs; first += P) {
        const int64_t cnt = std::min(P, npairs - first);
        SkPairSrc src;
        std::memset(&src, 0, sizeof(src));
        src.ny = ny; src.lx_pts = lx_pts; src.ly_pts = ly_pts; src.stride = per; src.first = first;
        if (dtype == SK_F32) {
            GramArgs<float> ga;
            ga.X = (const float*)X; ga.Y = (const float*)Y; ga.d = d; ga.dpad = gram_dpad(p, d);
            ga.lam = 0; ga.src = src; ga.cskew = (float*)((char*)ws + L.cskew); ga.maxc = nullptr;
            ga.split = p.gram == SK_GRAM_BF16X3;
            SK_TRY_HIP(launch_gram(ga, cnt, g.nsteps_pad, (int)lx, (int)ly, p.gram == SK_GRAM_NATIVE, stream),
                       "increment Gram");
            SK_TRY_HIP(SkLaunch<float>::unskew(src, ga.cskew, (float*)C, first, cnt, lx * ly, stream), "unskew");
        } else {
            GramArgs<double> ga;
            ga.X = (const double*)X; ga.Y = (const double*)Y; ga.d = d; ga.dpad = gram_dpad(p, d);
            ga.lam = 0; ga.src = src; ga.cskew = (double*)((char*)ws + L.cskew); ga.maxc = nullptr;
            ga.split = 0;
            SK_TRY_HIP(launch_gram(ga, cnt, g.nsteps_pad, (int)lx, (int)ly, p.gram == SK_GRAM_NATIVE, stream),
                       "increment Gram");
            SK_TRY_HIP(SkLaunch<double>::unskew(src, ga.cskew, (double*)C, first, cnt, lx * ly, stream), "unskew");
        }
    }
    return SK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Gram tuner and the tune cache's file
// ---------------------------------------------------------------------------
namespace {
// Device memory of one Gram tuning run, freed on every return path.
struct DevMem {
    void* p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t n) {
        SK_TRY_HIP(hipMalloc(&p, std::max<size_t>(n, 256)), "tuning buffers");
        return SK_OK;
    }
};

template <typename R>
int gram_tune_impl(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                   int64_t ly_pts, int64_t d, const sk_params& p, bool backward, hipStream_t st,
                   sk_params* best_p, double* best_ms) {
    const bool sym = (p.flags & SK_SYMMETRIC) != 0;
    const bool saved = backward && !(p.flags & SK_SWEEP_F64);
    std::vector<sk_params> cands;
    std::vector<int32_t> algos = {SK_ALGO_BATCHED};
    const int64_t segs = std::max(lx_pts, ly_pts) - 1;
    if (!is_fd(p) && (segs << lam_of(p)) > 64) algos.push_back(SK_ALGO_PIPELINE);
    for (int32_t a : algos)
        for (int32_t c : ckpt_choices(p, backward)) {
            sk_params q = p;
            q.algo = a;
            q.ckpt = c;
            cands.push_back(q);
        }
    // workspace: the largest any candidate needs
    size_t wsb = 0;
    for (const sk_params& q : cands) {
        const size_t w = saved ? sigkernel_gram_state_size(nx, lx_pts, ny, ly_pts, d, &q)
                               : std::max(sigkernel_gram_workspace(nx, lx_pts, ny, ly_pts, d, &q, 0),
                                          backward ? sigkernel_gram_workspace(nx, lx_pts, ny, ly_pts, d, &q, 1)
                                                   : (size_t)0);
        wsb = std::max(wsb, w);
    }
    g_last_error.clear();
    if (wsb == 0) return fail(SK_EINVAL, "no configuration applies to this Gram call");
    DevMem ws, K, gk, gx, gy;
    const int64_t nk = nx * ny, nxv = nx * lx_pts * d, nyv = ny * ly_pts * d;
    int rc = ws.alloc(wsb);
    if (!rc) rc = K.alloc(nk * sizeof(R));
    if (!rc && backward) {
        if (!(rc = gk.alloc(nk * sizeof(R))) && !(rc = gx.alloc(nxv * sizeof(R))) &&
            !(rc = gy.alloc(nyv * sizeof(R))))
            rc = SkLaunch<R>::fill((R*)gk.p, nk, (R)1, st) == hipSuccess ? SK_OK : fail(SK_EHIP, "fill");
    }
    if (rc) return rc;
    double bt = -1.0;
    for (const sk_params& q : cands) {
        double t = 0.0;
        int r = time_best([&]() -> int {
            int z;
            if (saved) {
                z = sigkernel_gram_save(X, nx, lx_pts, Y, ny, ly_pts, d, &q, K.p, nullptr, ws.p, wsb, st);
                if (!z)
                    z = sigkernel_gram_backward_saved(X, nx, lx_pts, Y, ny, ly_pts, d, &q, gk.p, nullptr,
                                                      gx.p, sym ? nullptr : gy.p, ws.p, wsb, st);
                return z;
            }
            z = sigkernel_gram(X, nx, lx_pts, Y, ny, ly_pts, d, &q, K.p, nullptr, ws.p, wsb, st);
            if (!z && backward)
                z = sigkernel_backward(SK_OP_GRAM, X, nullptr, nx, lx_pts, Y, nullptr, ny, ly_pts, d, &q,
                                       gk.p, nullptr, gx.p, sym ? nullptr : gy.p, ws.p, wsb, st);
            return z;
        }, st, &t);
        if (r == SK_EUNSUPPORTED || r == SK_EWORKSPACE) {  // not offered for this call: skip
            g_last_error.clear();
            continue;
        }
        if (r) return r;
        if (bt < 0 || t < bt) {
            bt = t;
            *best_p = q;
        }
    }
    if (bt < 0) return fail(SK_EUNSUPPORTED, "no configuration runs this Gram call");
    TuneVal v;
    v.cfg = kDefaultPlanCfg;
    v.cfg.ckpt = best_p->ckpt;
    v.algo = best_p->algo;
    v.ms = bt;
    tune_store(gram_key(nx, lx_pts, ny, ly_pts, d, p, backward), v);
    if (best_ms) *best_ms = bt;
    return SK_OK;
}

constexpr const char* kTuneHeader = "# sigkernel tune cache 1";
}  // namespace

extern "C" {

int sigkernel_gram_tune(const void* X, int64_t nx, int64_t lx_pts, const void* Y, int64_t ny,
                        int64_t ly_pts, int64_t d, const sk_params* p, int32_t backward,
                        hipStream_t stream, sk_params* best, double* best_ms) {
    g_last_error.clear();
    if (!X || !Y || !best) return fail(SK_EINVAL, "NULL pointer");
    int rc = check_params(p, backward != 0);
    if (!rc) rc = check_dims(d, backward != 0);
    if (!rc) rc = check_gram_geom(lx_pts, ly_pts, lam_of(*p));
    if (rc) return rc;
    if (p->algo == SK_ALGO_PLAIN) return fail(SK_EUNSUPPORTED, "the plain algorithm has nothing to tune");
    if (nx <= 0 || ny <= 0) return fail(SK_EINVAL, "empty Gram");
    try {
        if (p->dtype == SK_F32)
            return gram_tune_impl<float>(X, nx, lx_pts, Y, ny, ly_pts, d, *p, backward != 0, stream, best,
                                         best_ms);
        return gram_tune_impl<double>(X, nx, lx_pts, Y, ny, ly_pts, d, *p, backward != 0, stream, best,
                                      best_ms);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_gram_tuned(int64_t nx, int64_t lx_pts, int64_t ny, int64_t ly_pts, int64_t d,
                         const sk_params* p, int32_t backward, sk_params* out, int32_t* found) {
    g_last_error.clear();
    if (!p || !out || !found) return fail(SK_EINVAL, "NULL pointer");
    *found = 0;
    *out = *p;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (g_tune_cache.empty()) return SK_OK;
    }
    try {
        TuneVal v;
        if (!tune_lookup(gram_key(nx, lx_pts, ny, ly_pts, d, *p, backward != 0), &v)) return SK_OK;
        sk_params q = *p;
        q.algo = v.algo;
        q.ckpt = v.cfg.ckpt;
        if (check_params(&q, backward != 0)) {  // a stale entry: keep the caller's parameters
            g_last_error.clear();
            return SK_OK;
        }
        *out = q;
        *found = 1;
        return SK_OK;
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

int sigkernel_tune_cache_save(const char* path) {
    g_last_error.clear();
    if (!path) return fail(SK_EINVAL, "NULL path");
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(SK_EINVAL, "cannot write %s", tmp.c_str());
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        std::fprintf(f, "%s\n", kTuneHeader);
        for (const auto& e : g_tune_cache)
            std::fprintf(f, "%s %d %d %d %d %d %d %.6g\n", e.first.c_str(), e.second.cfg.order,
                         e.second.cfg.swap, e.second.cfg.buckets, e.second.cfg.pipe, e.second.cfg.ckpt,
                         e.second.algo, e.second.ms);
    }
    const bool ok = std::fflush(f) == 0 && !std::ferror(f);
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return fail(SK_EINVAL, "writing %s failed", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(SK_EINVAL, "cannot replace %s", path);
    }
    return SK_OK;
}

int sigkernel_tune_cache_load(const char* path, int32_t* loaded, int32_t* skipped) {
    g_last_error.clear();
    if (loaded) *loaded = 0;
    if (skipped) *skipped = 0;
    if (!path) return fail(SK_EINVAL, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return SK_OK;  // no cache yet: defaults
    char line[1024];
    bool header = false;
    int32_t nl = 0, ns = 0;
    while (std::fgets(line, sizeof(line), f)) {
        const size_t len = std::strlen(line);
        if (len == 0 || line[len - 1] != '\n') {  // over-long or unterminated line
            ++ns;
            if (len == sizeof(line) - 1) {
                int ch;
                while ((ch = std::fgetc(f)) != EOF && ch != '\n') {}
            }
            continue;
        }
        line[len - 1] = 0;
        if (!header) {
            header = std::strcmp(line, kTuneHeader) == 0;
            if (!header) break;  // not a tune cache: take nothing from it
            continue;
        }
        char key[512];
        int o, w, b, pp, ck, al, used = 0;
        double ms;
        const int got = std::sscanf(line, "%511s %d %d %d %d %d %d %lf%n", key, &o, &w, &b, &pp, &ck, &al,
                                    &ms, &used);
        const bool ok = got == 8 && line[used] == 0 && (o == 0 || o == 1) && (w == 0 || w == 1) &&
                        (b == 0 || b == 1) && (pp == 0 || (pp >= 2 && pp <= 1 << 20)) &&
                        (ck == 0 || ck == 2 || ck == 4) &&
                        (al == SK_ALGO_BATCHED || al == SK_ALGO_PIPELINE) && std::isfinite(ms) &&
                        (std::strncmp(key, "pairs|", 6) == 0 || std::strncmp(key, "gram|", 5) == 0);
        if (!ok) {
            ++ns;
            continue;
        }
        TuneVal v;
        v.cfg = PlanCfg{o, w, b, pp, ck};
        v.algo = al;
        v.ms = ms;
        tune_store(key, v);
        ++nl;
    }
    std::fclose(f);
    if (!header && (nl | ns) == 0) {
        if (skipped) *skipped = 1;
        return SK_OK;
    }
    if (loaded) *loaded = nl;
    if (skipped) *skipped = ns;
    return SK_OK;
}

void sigkernel_tune_cache_clear(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache.clear();
}

int sigkernel_plan_get_cfg(const sk_plan* plan, sk_plan_cfg* out) {
    g_last_error.clear();
    if (!plan || !out) return fail(SK_EINVAL, "NULL pointer");
    const PlanCfg& c = plan->impl.cfg;
    out->longest_first = c.order;
    out->transpose = c.swap;
    out->lds_classes = c.buckets;
    out->pipeline_min_strips = c.pipe;
    out->ckpt = ckpt_stride(plan->impl.p);
    out->launches = (int64_t)plan->impl.fchunks.size();
    return SK_OK;
}

int sigkernel_plan_set_cfg(sk_plan* plan, const sk_plan_cfg* cfg, size_t ws_bytes) {
    g_last_error.clear();
    if (!plan || !cfg) return fail(SK_EINVAL, "NULL pointer");
    if ((cfg->longest_first | cfg->transpose | cfg->lds_classes) & ~1)
        return fail(SK_EINVAL, "configuration flags are 0 or 1");
    try {
        const PlanCfg c = {cfg->longest_first, cfg->transpose, cfg->lds_classes, cfg->pipeline_min_strips,
                           cfg->ckpt};
        return plan_build(plan->impl, c, ws_bytes == 0 ? SIZE_MAX : ws_bytes);
    } catch (...) {
        return fail(SK_EINVAL, "internal exception");
    }
}

size_t sigkernel_plan_tune_workspace(const sk_plan* plan) {
    g_last_error.clear();
    if (!plan) {
        fail(SK_EINVAL, "plan is NULL");
        return 0;
    }
    try {
        return (size_t)plan_tune_workspace(plan->impl);
    } catch (...) {
        fail(SK_EINVAL, "internal exception");
        return 0;
    }
}

}  // extern "C"
