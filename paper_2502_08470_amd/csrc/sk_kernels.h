// Kernel templates of the batched signature-kernel path (instantiated per
// real type in sk_inst_*.hip).  See sk_common.h for the wavefront mapping
// and the skewed layout, sk_device.h for the cell maps.
#pragma once
#include <hip/hip_runtime.h>

#include "sk_common.h"
#include "sk_device.h"

typedef float sk_f4 __attribute__((ext_vector_type(4)));
typedef double sk_d4 __attribute__((ext_vector_type(4)));
typedef short sk_s4 __attribute__((ext_vector_type(4)));  // 4 bf16 bit patterns

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// element-wise type conversion (FP32 paths swept in FP64, SK_SWEEP_F64)
template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}

// ---------------------------------------------------------------------------
// (a) increment Gram: skewed cell constants by MFMA
// ---------------------------------------------------------------------------
template <typename R>
struct GramArgs {
    const R* X;
    const R* Y;
    int64_t d;
    int32_t dpad;       // d rounded up to a multiple of 4
    int32_t lam;        // dyadic refinement (finite differences), 0 otherwise
    SkPairSrc src;
    R* cskew;           // chunk buffer of skewed constants
    unsigned* maxc;     // per chunk-local pair: bits of max |c| (nullable)
    int32_t split;      // FP32 only: BF16 3-way split products instead of FP32 MFMA
    int32_t rseg;       // k_gram_strip: rows of a strip per workgroup (a multiple of 8)
};

template <typename R> struct SkMfma;

// Row stride of an LDS ring of y increments, one row per column (padded by
// 16 bytes so that 64 consecutive columns spread over the banks).
template <typename R, int DMAX>
constexpr int sk_ring_ys() { return DMAX + 16 / (int)sizeof(R); }
// 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element v of lane l holds D[row(l, v)][l % 16].  The FP32 and
// FP64 instructions place the four output rows of a lane differently.
template <> struct SkMfma<float> {
    typedef sk_f4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct SkMfma<double> {
    typedef sk_d4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// BF16 3-way split of an FP32 value: x = hi + mid + lo exactly (each part
// keeps 8 significant bits of what the previous ones left; the two
// subtractions are exact), as bf16 bit patterns rounded to nearest even.
__device__ __forceinline__ unsigned sk_bf16_rne(float v) {
    const unsigned u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
}
__device__ __forceinline__ void sk_bf16_split(float x, short& h, short& m, short& l) {
    const unsigned uh = sk_bf16_rne(x);
    const float r1 = x - __uint_as_float(uh);
    const unsigned um = sk_bf16_rne(r1);
    const float r2 = r1 - __uint_as_float(um);
    const unsigned ul = sk_bf16_rne(r2);
    h = (short)(uh >> 16);
    m = (short)(um >> 16);
    l = (short)(ul >> 16);
}

// One 16x16 tile of the increment Gram, D[m][n] = sum_k a_m[k] b_n[k] over
// k < dp, where this lane's row pointer `arow` is a_(lane%16) and `brow` is
// b_(lane%16) (rows flagged not ok read as zero).
//  SPLIT = false: 16x16x4 MFMA in R (lane supplies k = kk + lane/16).
//  SPLIT = true (FP32 only, dp a multiple of 16): each operand split into
//   three bf16 parts and the six products hi*hi, hi*mid, mid*hi, mid*mid,
//   hi*lo, lo*hi accumulated in FP32 by 16x16x16 bf16 MFMAs, smallest
//   first (lane supplies k = kk + 4 (lane/16) + j, j < 4).  The dropped
//   products are below 2^-24 of |a||b|, the FP32 level.
template <typename R, bool SPLIT>
__device__ __forceinline__ typename SkMfma<R>::acc_t sk_gram_tile(const R* arow, bool aok,
                                                                  const R* brow, bool bok, int dp,
                                                                  int lane) {
    typename SkMfma<R>::acc_t acc = {0, 0, 0, 0};
    if constexpr (!SPLIT) {
        for (int kk = 0; kk < dp; kk += 4) {
            const R av = aok ? arow[kk + (lane >> 4)] : (R)0;
            const R bv = bok ? brow[kk + (lane >> 4)] : (R)0;
            acc = SkMfma<R>::mma(av, bv, acc);
        }
    } else {
        static_assert(sizeof(R) == 4, "the split Gram is an FP32 mode");
        for (int kk = 0; kk < dp; kk += 16) {
            sk_s4 ah, am, al, bh, bm, bl;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kk + 4 * (lane >> 4) + j;
                short h, m, l;
                sk_bf16_split(aok ? (float)arow[k] : 0.0f, h, m, l);
                ah[j] = h; am[j] = m; al[j] = l;
                sk_bf16_split(bok ? (float)brow[k] : 0.0f, h, m, l);
                bh[j] = h; bm[j] = m; bl[j] = l;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
        }
    }
    return acc;
}

// One workgroup (4 waves) writes skewed rows [64 b, 64 b + 64) of one pair.
// For every strip s that owns one of those cells it stages the 64 x-rows of
// the strip and the 128 y-columns the rows can touch, multiplies them with
// 16x16x4 MFMAs (K = d) into an LDS tile, 64 columns at a time, and gathers
// each skewed element from the tile.  Rows are written once, whole,
// coalesced.
template <typename R, bool SPLIT>
__global__ __launch_bounds__(256) void k_gram_skew(const GramArgs<R> a) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    const int b = blockIdx.y;
    if (64 * b >= g.nsteps_pad) return;
    const int dp = a.dpad, ds = dp + 1;  // odd row stride: the 16 rows a tile reads hit distinct banks
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* Xs = reinterpret_cast<R*>(sk_smem);          // [64][ds]
    R* Ys = Xs + 64 * ds;                            // [128][ds]
    R* Tt = Ys + 128 * ds;                           // [64][66]: diagonal reads conflict-free
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * a.d;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * a.d;
    const R rscale = (R)1 / (R)(1 << a.lam);

    R val[16];
    int Le[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        val[q] = (R)0;
        int e = tid + 256 * q;
        Le[q] = 64 * b + (e >> 6) - (e & 63);
    }
    const int Lmin = 64 * b - 63, Lmax = 64 * b + 63;
    int s_lo = Lmin < 0 ? 0 : Lmin / g.Tp;
    int s_hi = Lmax / g.Tp;
    if (s_hi > g.nstrips - 1) s_hi = g.nstrips - 1;
    typedef typename SkMfma<R>::acc_t acc_t;
    for (int s = s_lo; s <= s_hi; ++s) {
        const int jb = Lmin - s * g.Tp;  // column of tile entry 0
        __syncthreads();
        // stage increments (refined: segment increment / 2^lam)
        for (int e = tid; e < 64 * dp; e += 256) {
            int rr = e / dp, k = e - rr * dp;
            int ir = s * 64 + rr;
            R v = (R)0;
            if (ir < g.lx && k < a.d) {
                int i = ir >> a.lam;
                v = (X[(int64_t)(i + 1) * a.d + k] - X[(int64_t)i * a.d + k]) * rscale;
            }
            Xs[rr * ds + k] = v;
        }
        for (int e = tid; e < 128 * dp; e += 256) {
            int cc = e / dp, k = e - cc * dp;
            int jr = jb + cc;
            R v = (R)0;
            if (jr >= 0 && jr < g.ly && k < a.d) {
                int j = jr >> a.lam;
                v = (Y[(int64_t)(j + 1) * a.d + k] - Y[(int64_t)j * a.d + k]) * rscale;
            }
            Ys[cc * ds + k] = v;
        }
        for (int h = 0; h < 2; ++h) {
            __syncthreads();
            // wave w: rows 16w..16w+15 against columns 64h..64h+63
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int col0 = 64 * h + 16 * ni;
                const acc_t acc = sk_gram_tile<R, SPLIT>(Xs + (16 * wave + (lane & 15)) * ds, true,
                                                         Ys + (col0 + (lane & 15)) * ds, true, dp,
                                                         lane);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Tt[(16 * wave + SkMfma<R>::row(lane, v)) * 66 + 16 * ni + (lane & 15)] = acc[v];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int L = Le[q];
                const int r = (tid + 256 * q) & 63;
                const int col = L - Lmin - 64 * h;
                if (L >= 0 && col >= 0 && col < 64) {
                    int ss = L / g.Tp, j = L - ss * g.Tp;
                    if (ss == s && j < g.ly && s * 64 + r < g.lx) val[q] = Tt[r * 66 + col];
                }
            }
        }
    }
    R* out = a.cskew + pd.c_off + (int64_t)64 * 64 * b;
    R mx = (R)0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        out[tid + 256 * q] = val[q];
        R av = sk_abs(val[q]);
        mx = av > mx ? av : mx;
    }
    if (a.maxc) {
        mx = wave_max(mx);
        if (lane == 0) atomicMax(a.maxc + local, __float_as_uint((float)mx));
    }
}

// Strip-band variant: one workgroup (4 waves) per (pair, strip s, segment z
// of rseg rows, a multiple of 64) computes the strip's 64 x ly band of C one
// 64-column tile at a time and writes the skewed rows s Tp + t of the
// segment.  At lane r, row t needs virtual column v = t - r (column v of
// strip s, or column Tp + v of strip s-1 when v < 0), which lies in the
// current tile or the previous one; both stay in LDS.  Every increment is
// loaded once per workgroup and every tile element computed once (the
// 64-row block kernel reloads 128 y columns and computes a 64 x 128 tile for
// every 64 rows).  Same tiles and MFMA order as k_gram_skew, so both give
// identical constants.
template <typename R, bool SPLIT>
__global__ __launch_bounds__(256) void k_gram_band(const GramArgs<R> a) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int s = blockIdx.y;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0 || s >= g.nstrips) return;
    const int Tstrip = (s == g.nstrips - 1) ? g.nsteps_pad - s * g.Tp : g.Tp;
    const int tbeg = (int)blockIdx.z * a.rseg;
    if (tbeg >= Tstrip) return;
    const int tend = tbeg + a.rseg < Tstrip ? tbeg + a.rseg : Tstrip;
    const int dp = a.dpad, ds = dp + 1;  // odd row stride: the 16 rows a tile reads hit distinct banks
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* Xs = reinterpret_cast<R*>(sk_smem);  // [64][ds]
    R* Ys = Xs + 64 * ds;                    // [64][ds]
    R* Tt = Ys + 64 * ds;                    // [2][64][66]: tiles by parity
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * a.d;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * a.d;
    const R rscale = (R)1 / (R)(1 << a.lam);
    auto stage_x = [&](int strip) {  // rows 64 strip .. + 63 (refined: segment i >> lam)
        for (int e = tid; e < 64 * dp; e += 256) {
            const int rr = e / dp, k = e - rr * dp, ir = strip * 64 + rr;
            R v = (R)0;
            if (ir >= 0 && ir < g.lx && k < a.d) {
                const int i = ir >> a.lam;
                v = (X[(int64_t)(i + 1) * a.d + k] - X[(int64_t)i * a.d + k]) * rscale;
            }
            Xs[rr * ds + k] = v;
        }
    };
    // y increments of virtual columns c0 .. c0 + 63, loaded into registers
    // one tile ahead (their latency overlaps the previous tile) and then
    // stored to LDS; 64 dp / 256 <= 16 values per thread (dp <= 60 here)
    constexpr int YV = 16;
    R yv[YV];
    auto load_y = [&](int c0) {
#pragma unroll
        for (int h = 0; h < YV; ++h) {
            const int e = tid + 256 * h, cc = e / dp, k = e - cc * dp, vv = c0 + cc;
            const int col = vv >= 0 ? vv : g.Tp + vv;
            yv[h] = (R)0;
            if (e < 64 * dp && k < a.d && (vv >= 0 || s > 0) && col >= 0 && col < g.ly) {
                const int j = col >> a.lam;
                yv[h] = (Y[(int64_t)(j + 1) * a.d + k] - Y[(int64_t)j * a.d + k]) * rscale;
            }
        }
    };
    auto store_y = [&]() {
#pragma unroll
        for (int h = 0; h < YV; ++h) {
            const int e = tid + 256 * h, cc = e / dp, k = e - cc * dp;
            if (e < 64 * dp) Ys[cc * ds + k] = yv[h];
        }
    };
    auto tile = [&](R* T) {  // T[r][c] = sum_k Xs[r][k] Ys[c][k]; wave w: rows 16w .. 16w+15
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const auto acc = sk_gram_tile<R, SPLIT>(Xs + (16 * wave + (lane & 15)) * ds, true,
                                                    Ys + (16 * ni + (lane & 15)) * ds, true, dp, lane);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                T[(16 * wave + SkMfma<R>::row(lane, v)) * 66 + 16 * ni + (lane & 15)] = acc[v];
        }
    };
    const int k0 = tbeg / 64;
    // the tile of virtual columns 64 (k0-1) .. 64 k0 - 1 (k0 = 0: strip s-1's
    // last 64 columns, rows of strip s-1)
    stage_x(k0 == 0 ? s - 1 : s);
    load_y(64 * (k0 - 1));
    store_y();
    __syncthreads();
    load_y(64 * k0);
    tile(Tt + ((k0 - 1) & 1) * 64 * 66);
    if (k0 == 0) {
        __syncthreads();
        stage_x(s);
    }
    R* out = a.cskew + pd.c_off + (int64_t)s * g.Tp * 64;
    for (int k = k0; 64 * k < tend; ++k) {
        __syncthreads();  // the previous rows are written: Ys and the older tile are free
        store_y();
        __syncthreads();
        if (64 * (k + 1) < tend) load_y(64 * (k + 1));
        R* Tc = Tt + (k & 1) * 64 * 66;
        const R* Tq = Tt + ((k - 1) & 1) * 64 * 66;
        tile(Tc);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, t = 64 * k + (e >> 6), r = e & 63;
            if (t < tend) {
                const int c = t - r - 64 * k;
                out[(int64_t)t * 64 + r] = c >= 0 ? Tc[r * 66 + c] : Tq[r * 66 + c + 64];
            }
        }
    }
}

// Direct variant for small d (native precision): one workgroup (4 waves) per
// pair stages the pair's increments in LDS once, then each wave writes a
// contiguous quarter of the skewed rows; lane r of row tau computes its own
// cell (64 s + r, L - s Tp), L = tau - r, as a d-term FMA chain.  Nothing is
// computed twice and there is no barrier after the staging.  The lane keeps
// the x increment of its row in registers (reloaded when its strip changes)
// and reads the y increment of its column from LDS, whose rows are padded so
// that the 8-byte reads of 16 consecutive lanes (consecutive columns) hit
// distinct banks.  Refined grids read cell (i >> lam, j >> lam) scaled by
// 4^-lam.
template <typename R> struct SkGramDirectPad;
template <> struct SkGramDirectPad<float> { static constexpr int value = 2; };
template <> struct SkGramDirectPad<double> { static constexpr int value = 1; };
#define SK_GRAM_DIRECT_DMAX 16
#define SK_GRAM_STRIP_DMAX 32

template <typename R>
__global__ __launch_bounds__(256) void k_gram_direct(const GramArgs<R> a) {
    constexpr int DMAX = SK_GRAM_DIRECT_DMAX;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, r = tid & 63;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) return;
    const int dp = a.dpad;  // multiple of 4, <= DMAX
    const int ys = dp + SkGramDirectPad<R>::value;  // padded LDS row of a y increment
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* Xs = reinterpret_cast<R*>(sk_smem);  // [lx][dp]
    R* Ys = Xs + (size_t)pd.lx * dp;        // [ly][ys]
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * a.d;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * a.d;
    for (int e = tid; e < pd.lx * dp; e += 256) {
        const int i = e / dp, k = e - i * dp;
        Xs[e] = k < a.d ? X[(int64_t)(i + 1) * a.d + k] - X[(int64_t)i * a.d + k] : (R)0;
    }
    for (int e = tid; e < pd.ly * dp; e += 256) {
        const int j = e / dp, k = e - j * dp;
        Ys[j * ys + k] = k < a.d ? Y[(int64_t)(j + 1) * a.d + k] - Y[(int64_t)j * a.d + k] : (R)0;
    }
    __syncthreads();
    const R scale = (R)1 / (R)(1 << (2 * a.lam));
    const int nr = g.nsteps_pad / 4;  // rows per wave (a multiple of 16)
    const int tau0 = wave * nr;
    // lane state at row tau0: linear index L, strip s, column j
    int L = tau0 - r, s = 0, j = 0;
    if (L >= 0) {
        s = L / g.Tp;
        j = L - s * g.Tp;
    }
    int xs_loaded = -1;  // strip whose x increment is in xr
    R xr[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) xr[k] = (R)0;
    R* out = a.cskew + pd.c_off;
    for (int t = 0; t < nr; ++t) {
        const int tau = tau0 + t;
        const int i = s * 64 + r;
        const bool live = L >= 0 && s < g.nstrips && j < g.ly && i < g.lx;
        R c = (R)0;
        if (live) {
            if (s != xs_loaded) {
                const R* xrow = Xs + (size_t)(i >> a.lam) * dp;
#pragma unroll
                for (int k = 0; k < DMAX; ++k) xr[k] = k < dp ? xrow[k] : (R)0;
                xs_loaded = s;
            }
            const R* yrow = Ys + (size_t)(j >> a.lam) * ys;
#pragma unroll
            for (int k = 0; k < DMAX; k += 2) {
                if (k < dp) {
                    c = fma(xr[k], yrow[k], c);
                    c = fma(xr[k + 1], yrow[k + 1], c);
                }
            }
            c *= scale;
        }
        out[(int64_t)tau * 64 + r] = c;
        ++L;
        if (L > 0 && ++j == g.Tp) {
            j = 0;
            ++s;
        }
    }
}

// Direct variant for pairs whose increments exceed one workgroup's LDS: one
// wave per (pair, strip s, segment z) writes the skewed rows s Tp + t,
// t in [z rseg, (z+1) rseg), of the strip's rows t < Tp (the last strip's
// up to nsteps_pad), whole.  Lane r's cell at row s Tp + t has linear index
// s Tp + v, v = t - r: row 64 s + r and column v when v >= 0, row
// 64 (s-1) + r and column Tp + v (strip s-1) when v < 0.  The lane keeps the
// x increments of both rows in registers; the y increments of the 64
// virtual columns t-63 .. t sit in an LDS ring of 128 (slot v mod 128),
// 8 columns added every 8 steps, loaded one block ahead.  The SW waves of a
// workgroup take SW consecutive strips in lockstep: their rows need the same
// virtual columns, so they share one ring (SW times less LDS per wave).
// Same FMA order and scaling as k_gram_direct, so both give identical
// constants.
#define SK_GRAM_STRIP_WAVES 4
template <typename R, int DMAX>
__global__ __launch_bounds__(64 * SK_GRAM_STRIP_WAVES) void k_gram_strip(const GramArgs<R> a) {
    constexpr int SW = SK_GRAM_STRIP_WAVES;
    const int tid = threadIdx.x, r = tid & 63;
    const int s0 = (int)blockIdx.y * SW, s = s0 + (tid >> 6);
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0 || s0 >= g.nstrips) return;  // workgroup-uniform
    auto rows_of = [&](int st) { return st == g.nstrips - 1 ? g.nsteps_pad - st * g.Tp : g.Tp; };
    const int slast = s0 + SW - 1 < g.nstrips - 1 ? s0 + SW - 1 : g.nstrips - 1;
    const int tbeg = (int)blockIdx.z * a.rseg;
    const int Tmax = rows_of(slast);  // the workgroup's longest strip (the pair's last if it holds it)
    if (tbeg >= Tmax) return;  // workgroup-uniform
    const int Tend = tbeg + a.rseg < Tmax ? tbeg + a.rseg : Tmax;
    const bool sok = s < g.nstrips;
    const int Tmine = sok ? (tbeg + a.rseg < rows_of(s) ? tbeg + a.rseg : rows_of(s)) : 0;
    constexpr int YS = sk_ring_ys<R, DMAX>();
    constexpr int NV = (8 * DMAX + 64 * SW - 1) / (64 * SW);  // ring values per thread per 8 columns
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* ring = reinterpret_cast<R*>(sk_smem);  // [128][YS]
    const int64_t d = a.d;
    const int lam = a.lam;
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * d;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * d;
    // x increments (segment i >> lam, unrefined) of the lane's rows in
    // strips s and s-1 (every row of a strip before the last exists)
    const int ia = s * 64 + r, ib = ia - 64;
    const bool oka = sok && ia < g.lx, okb = sok && s > 0;
    R xa[DMAX], xb[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        xa[k] = (R)0;
        xb[k] = (R)0;
        if (k < d && oka) xa[k] = X[(int64_t)((ia >> lam) + 1) * d + k] - X[(int64_t)(ia >> lam) * d + k];
        if (k < d && okb) xb[k] = X[(int64_t)((ib >> lam) + 1) * d + k] - X[(int64_t)(ib >> lam) * d + k];
    }
    // y increments of the 8 virtual columns from v0: value w is column
    // v0 + w / DMAX, dimension w % DMAX (negative v: column Tp + v, which
    // only the strips after the first read)
    R yv[NV];
    auto load_y = [&](int v0) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
            const int w = tid + 64 * SW * h, m = w / DMAX, k = w - m * DMAX, v = v0 + m;
            const int col = v >= 0 ? v : g.Tp + v;
            yv[h] = (R)0;
            if (w < 8 * DMAX && k < d && col >= 0 && col < g.ly) {
                const int j = col >> lam;
                yv[h] = Y[(int64_t)(j + 1) * d + k] - Y[(int64_t)j * d + k];
            }
        }
    };
    auto store_y = [&](int v0) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
            const int w = tid + 64 * SW * h, m = w / DMAX, k = w - m * DMAX;
            if (w < 8 * DMAX) ring[((v0 + m) & 127) * YS + k] = yv[h];
        }
    };
    for (int v0 = tbeg - 64; v0 <= tbeg; v0 += 8) {
        load_y(v0);
        store_y(v0);
    }
    load_y(tbeg + 8);
    __syncthreads();
    const R scale = (R)1 / (R)(1 << (2 * lam));
    R* out = a.cskew + pd.c_off + (int64_t)s * g.Tp * 64;
    for (int t0 = tbeg; t0 < Tend; t0 += 8) {
        if (t0 > tbeg) {  // columns t0 .. t0+7 replace t0-128 .. t0-121, which no lane reads again
            store_y(t0);
            __syncthreads();
            load_y(t0 + 8);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + u, v = t - r;
            if (t >= Tmine) break;  // wave-uniform
            const bool lo = v < 0;
            const int col = lo ? g.Tp + v : v;
            const bool live = (lo ? okb : oka) && col < g.ly;
            R c = (R)0;
            if (live) {
                const R* yr = ring + (v & 127) * YS;
#pragma unroll
                for (int k = 0; k < DMAX; k += 2) {
                    c = fma(lo ? xb[k] : xa[k], yr[k], c);
                    c = fma(lo ? xb[k + 1] : xa[k + 1], yr[k + 1], c);
                }
                c *= scale;
            }
            out[(int64_t)t * 64 + r] = c;
            // keep each step's ring reads in its step
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
    }
}

// Pair-resident variant: one workgroup (4 waves) per pair stages the pair's
// increments in LDS once ([lx][dp] and [ly][dp], unrefined; refined rows
// index i >> lam) and then produces all skewed row blocks of the pair in
// turn, so the global loads of the increments are paid once per pair instead
// of once per 64-row block.  Used when both increment arrays fit in LDS.
template <typename R, bool SPLIT>
__global__ __launch_bounds__(256) void k_gram_pair(const GramArgs<R> a) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) return;
    const int dp = a.dpad, ds = dp + 1;  // odd row stride: the 16 rows a tile reads hit distinct banks
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* Tt = reinterpret_cast<R*>(sk_smem);  // [64][66]
    R* Xs = Tt + 64 * 66;                    // [lx][ds]
    R* Ys = Xs + (size_t)pd.lx * ds;         // [ly][ds]
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * a.d;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * a.d;
    const R rscale = (R)1 / (R)(1 << a.lam);
    for (int e = tid; e < pd.lx * dp; e += 256) {
        const int i = e / dp, k = e - i * dp;
        Xs[i * ds + k] = k < a.d ? (X[(int64_t)(i + 1) * a.d + k] - X[(int64_t)i * a.d + k]) * rscale : (R)0;
    }
    for (int e = tid; e < pd.ly * dp; e += 256) {
        const int j = e / dp, k = e - j * dp;
        Ys[j * ds + k] = k < a.d ? (Y[(int64_t)(j + 1) * a.d + k] - Y[(int64_t)j * a.d + k]) * rscale : (R)0;
    }
    typedef typename SkMfma<R>::acc_t acc_t;
    const int nblk = g.nsteps_pad / 64;
    for (int b = 0; b < nblk; ++b) {
        R val[16];
        int Le[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            val[q] = (R)0;
            const int e = tid + 256 * q;
            Le[q] = 64 * b + (e >> 6) - (e & 63);
        }
        const int Lmin = 64 * b - 63, Lmax = 64 * b + 63;
        const int s_lo = Lmin < 0 ? 0 : Lmin / g.Tp;
        int s_hi = Lmax / g.Tp;
        if (s_hi > g.nstrips - 1) s_hi = g.nstrips - 1;
        for (int s = s_lo; s <= s_hi; ++s) {
            const int jb = Lmin - s * g.Tp;
            const int ir = s * 64 + 16 * wave + (lane & 15);
            const bool rok = ir < g.lx;
            const R* xrow = Xs + (size_t)(ir >> a.lam) * ds;
            for (int h = 0; h < 2; ++h) {
                __syncthreads();  // staging done / previous tile consumed
#pragma unroll
                for (int ni = 0; ni < 4; ++ni) {
                    const int jr = jb + 64 * h + 16 * ni + (lane & 15);
                    const bool cok = jr >= 0 && jr < g.ly;
                    const R* yrow = Ys + (size_t)(cok ? (jr >> a.lam) : 0) * ds;
                    const acc_t acc = sk_gram_tile<R, SPLIT>(xrow, rok, yrow, cok, dp, lane);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        Tt[(16 * wave + SkMfma<R>::row(lane, v)) * 66 + 16 * ni + (lane & 15)] = acc[v];
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int L = Le[q];
                    const int r = (tid + 256 * q) & 63;
                    const int col = L - Lmin - 64 * h;
                    if (L >= 0 && col >= 0 && col < 64) {
                        const int ss = L / g.Tp, j = L - ss * g.Tp;
                        if (ss == s && j < g.ly && s * 64 + r < g.lx) val[q] = Tt[r * 66 + col];
                    }
                }
            }
        }
        R* out = a.cskew + pd.c_off + (int64_t)64 * 64 * b;
#pragma unroll
        for (int q = 0; q < 16; ++q) out[tid + 256 * q] = val[q];
    }
}

// ---------------------------------------------------------------------------
// (b) forward wavefront sweep of the polynomial schemes
// ---------------------------------------------------------------------------
template <typename R>
struct SweepArgs {
    SkPairSrc src;
    const R* cskew;
    SkTab<R> tab;
    R* K;                  // kernel values (mantissas if Kexp)
    int32_t* Kexp;         // nullable
    // checkpoint outputs (backward recompute)
    R* ck;
    int32_t* ce;
    R* qb;
    int32_t* qe;
    unsigned* xb;          // global strip-boundary exchange records (long pairs)
    int32_t gx_cols;       // pairs with more columns use the global exchange
    int32_t lam;           // dyadic refinement of the grid (hybrid method), forward only
    int32_t S;             // checkpoint stride of the checkpointing sweep
};

// Global strip-boundary exchange, consumer side: at the start of every
// 8-step block the wave (1) fences, so that the records stored by the
// producing lane in earlier blocks are visible, (2) moves the records it
// loaded one block earlier into the LDS staging slot, and (3) loads the
// records the consuming lane will read in the next block.  `want(tau)`
// gives the record index (column) the consumer reads at step tau, or -1.
// A record is stored at least Tp - 63 - 15 steps before the block start
// that loads it, so Tp > 78 (exchange pairs have more than SK_GX_MIN_COLS
// columns) puts a fence between every store and its load.
// COHERENT: the records come from other workgroups (strip pipeline) and are
// read with device-coherent loads.
template <int W, bool COHERENT = false, typename F>
__device__ __forceinline__ void sk_gx_stage(unsigned (&xr)[(8 * W + 63) / 64], unsigned* stage,
                                            const unsigned* xg, int t_next, int r, F want) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
#pragma unroll
    for (int h = 0; h < (8 * W + 63) / 64; ++h)
        if (r + 64 * h < 8 * W) stage[r + 64 * h] = xr[h];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < (8 * W + 63) / 64; ++h) {
        const int w = r + 64 * h;
        xr[h] = 0u;
        if (w < 8 * W) {
            const int m = w / W, q = w - m * W;
            const int col = want(t_next + m);
            if (col >= 0)
                xr[h] = COHERENT ? __hip_atomic_load(xg + (int64_t)col * W + q, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : xg[(int64_t)col * W + q];
        }
    }
}

template <typename R>
__device__ __forceinline__ void sk_write_k(R* K, int32_t* Kexp, int64_t idx, double v, int E) {
    if (Kexp) {
        int e = (v == 0.0 || !isfinite(v)) ? 0 : sk_frexp_exp(v);
        K[idx] = (R)ldexp(v, -e);
        Kexp[idx] = E + e;
    } else {
        K[idx] = (R)ldexp(v, E);
    }
}

// A strip-boundary edge of the forward sweep in LDS (a ring entry or a
// staged exchange record, 8-byte aligned): FP64 coefficients 0 and 1 in
// words 0..3, coefficients 2..N from word 4, then the exponent.
template <typename R, int N>
__device__ __forceinline__ void sk_edge_read(SkLds<unsigned> rec, double& q0, double& q1,
                                             R (&q)[N + 1], int& e) {
    constexpr int ES = (int)sizeof(R), NW = 4 + (N - 1) * ES / 4 + 1, NW2 = (NW + 1) / 2;
    unsigned wv[2 * NW2];
#pragma unroll
    for (int k = 0; k < NW2; ++k) {
        const unsigned long long v = ((SkLds<unsigned long long>)rec)[k];
        wv[2 * k] = (unsigned)v;
        wv[2 * k + 1] = (unsigned)(v >> 32);
    }
    q0 = __hiloint2double((int)wv[1], (int)wv[0]);
    q1 = __hiloint2double((int)wv[3], (int)wv[2]);
#pragma unroll
    for (int n = 2; n <= N; ++n) {
        if constexpr (ES == 4)
            q[n] = __uint_as_float(wv[4 + n - 2]);
        else
            q[n] = __hiloint2double((int)wv[4 + 2 * (n - 2) + 1], (int)wv[4 + 2 * (n - 2)]);
    }
    e = (int)wv[NW - 1];
}
template <typename R, int N>
__device__ __forceinline__ void sk_edge_write(SkLds<unsigned> rec, double q0, double q1,
                                              const R (&q)[N + 1], int e) {
    constexpr int ES = (int)sizeof(R), NW = 4 + (N - 1) * ES / 4 + 1, NW2 = (NW + 1) / 2;
    unsigned wv[2 * NW2];
    wv[0] = (unsigned)__double2loint(q0);
    wv[1] = (unsigned)__double2hiint(q0);
    wv[2] = (unsigned)__double2loint(q1);
    wv[3] = (unsigned)__double2hiint(q1);
#pragma unroll
    for (int n = 2; n <= N; ++n) {
        if constexpr (ES == 4) {
            wv[4 + n - 2] = __float_as_uint(q[n]);
        } else {
            wv[4 + 2 * (n - 2)] = (unsigned)__double2loint(q[n]);
            wv[4 + 2 * (n - 2) + 1] = (unsigned)__double2hiint(q[n]);
        }
    }
    wv[NW - 1] = (unsigned)e;
    if (NW < 2 * NW2) wv[2 * NW2 - 1] = 0u;
#pragma unroll
    for (int k = 0; k < NW2; ++k)
        ((SkLds<unsigned long long>)rec)[k] = (unsigned long long)wv[2 * k] | ((unsigned long long)wv[2 * k + 1] << 32);
}

// Magnitude bookkeeping: every lane carries its own power-of-two exponent E
// (the edges it holds are mantissa * 2^E).  Lanes of one wave sit at very
// different places of the grid, whose kernel values can differ by far more
// than the floating-point range, so the exponent travels with the edge that
// moves to the next lane and the receiving lane aligns both inputs of its cell
// to the larger exponent (the smaller input loses only bits below the
// working precision of the larger one).  Every 8 steps each lane rescales its
// own state back into [2^-band, 2^band].
// GX: the launch may hold pairs whose strip-boundary edges go through the
// global exchange (compiled separately so launches without such pairs keep
// their register budget).
template <typename R, int N, int TMAX, bool CKPT, int S, bool GX>
__global__ __launch_bounds__(64) void k_sweep(const SweepArgs<R> a) {
    const int r = threadIdx.x;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) {
        if (r == 0) sk_write_k(a.K, a.Kexp, pd.k_idx, (R)1, 0);
        return;
    }
    // strip-boundary edges (FP64 coefficients 0, 1, coefficients 2..N,
    // exponent tags): an LDS ring of one entry per column, or for long pairs
    // global records staged through LDS one block ahead
    constexpr int ES = (int)sizeof(R), GXW = sk_gx_words(N, ES);
    const bool gx = GX && g.ly > a.gx_cols;  // wave-uniform
    extern __shared__ __align__(16) unsigned char sk_smem[];
    unsigned* stage = reinterpret_cast<unsigned*>(sk_smem);                // [8][GXW]
    // ring entry of a column: FP64 coefficients 0 and 1, coefficients 2..N,
    // exponent (the layout of a global exchange record), 8-byte aligned
    constexpr int RW = sk_ring_col_bytes_fwd(N, ES) / 4;
    // exchange launches that checkpoint also keep lane 63's records of the
    // current 8-step block in LDS ([8][GXW], before the ring), for the
    // adjoint's copy of the boundary edges
    constexpr int OST = (GX && CKPT) ? sk_gx_stage_bytes(N, ES) : 0;
    const SkLds<unsigned> ost = (SkLds<unsigned>)(sk_smem + sk_gx_stage_bytes(N, ES));
    const SkLds<unsigned> ring = (SkLds<unsigned>)(sk_smem + sk_gx_stage_bytes(N, ES) + OST);  // [ly][RW]
    unsigned* xg = a.xb + pd.xb_off;  // [ly][GXW] (exchange pairs only)
    unsigned xr[(8 * GXW + 63) / 64];
#pragma unroll
    for (int h = 0; h < (8 * GXW + 63) / 64; ++h) xr[h] = 0u;
    // column lane 0 reads at step tau (strips >= 1), or -1
    auto lane0_col = [&](int tau) -> int {
        const int s0 = tau / g.Tp, j0 = tau - s0 * g.Tp;
        return (tau < g.nsteps && s0 >= 1 && s0 < g.nstrips && j0 < g.ly) ? j0 : -1;
    };
    const R* cs = a.cskew + pd.c_off;

    R P[N + 1], Qs[N + 1];
    double P0 = 0.0, P1 = 0.0, Qs0 = 0.0, Qs1 = 0.0;
#pragma unroll
    for (int n = 0; n <= N; ++n) {
        P[n] = (R)0;
        Qs[n] = (R)0;
    }
    int E = 0, Es = 0;
    int L = -r, s = 0, j = 0;
    bool live = false;
    // The ring starts with the initial left edge (1, 0, ..., 0; exponent 0),
    // which lane 0 of strip 0 reads: the entry of column j is first written by
    // lane 63 of strip 0, 63 steps after that read.  (Exchange pairs take the
    // initial edge by a wave-uniform test instead.)
    if (!gx) {
        for (int col = r; col < g.ly; col += 64) {
            SkLds<unsigned> e = ring + __mul24(col, RW);
#pragma unroll
            for (int w = 0; w < RW; ++w) e[w] = (w == 1) ? 0x3ff00000u : 0u;  // words 0-1: 1.0
        }
    }
    const int nst8 = (g.nsteps + 7) & ~7;
    R cb[8], cn[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cb[u] = cs[u * 64 + r];
    unsigned tword = 0u;  // tail lengths of the current checkpoint segment
    for (int t0 = 0; t0 < nst8; t0 += 8) {
        if (gx) sk_gx_stage<GXW>(xr, stage, xg, t0 + 8, r, lane0_col);
        if (t0 + 8 < g.nsteps_pad) {
#pragma unroll
            for (int u = 0; u < 8; ++u) cn[u] = cs[(int64_t)(t0 + 8 + u) * 64 + r];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int tau = t0 + u;
            // lane 0's left edge: the strip-boundary entry of its column (the
            // ring, or the staged exchange record of this step), read alike by
            // every lane and merged into the lane move that feeds lanes 1..63
            const int j0 = __builtin_amdgcn_readfirstlane(j), s0 = __builtin_amdgcn_readfirstlane(s);
            double B0, B1;
            R Bq[N + 1];
            int Be;
            sk_edge_read<R, N>(gx ? (SkLds<unsigned>)stage + u * GXW
                                  : ring + __mul24(j0 < g.ly ? j0 : g.ly - 1, RW),
                               B0, B1, Bq, Be);
            if (gx && s0 == 0) {
                B0 = 1.0;
                B1 = 0.0;
#pragma unroll
                for (int n = 2; n <= N; ++n) Bq[n] = (R)0;
                Be = 0;
            }
            R Qin[N + 1];
#pragma unroll
            for (int n = 2; n <= N; ++n) Qin[n] = lane_from_prev_or(Qs[n], Bq[n]);
            double Qin0 = lane_from_prev_or(Qs0, B0), Qin1 = lane_from_prev_or(Qs1, B1);
            int Ein = lane_from_prev_or(Es, Be);
            const int i = s * 64 + r;
            live = (L >= 0) && (s < g.nstrips) && (j < g.ly) && (i < g.lx);
            if (live) {
                if (j == 0) {
                    P0 = 1.0;
                    P1 = 0.0;
#pragma unroll
                    for (int n = 2; n <= N; ++n) P[n] = (R)0;
                    E = 0;
                }
                const int Ec = E > Ein ? E : Ein;
                const int dp = E - Ec, dq = Ein - Ec;
                if (sk_wave_any(dp != 0 || dq != 0)) {  // rare: skip in the common case
                    P0 = ldexp(P0, dp);
                    P1 = ldexp(P1, dp);
                    Qin0 = ldexp(Qin0, dq);
                    Qin1 = ldexp(Qin1, dq);
#pragma unroll
                    for (int n = 2; n <= N; ++n) {
                        P[n] = sk_ldexp(P[n], dp);
                        Qin[n] = sk_ldexp(Qin[n], dq);
                    }
                }
                E = Ec;
            }
            P[0] = (R)P0;
            P[1] = (R)P1;
            Qin[0] = (R)Qin0;
            Qin[1] = (R)Qin1;
            if (CKPT && (tau % S) == 0 && tau < g.nsteps) {
                const int64_t kk = tau / S;
                R* ck = a.ck + pd.ck_off + kk * 2 * (N + 1) * 64;
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    sk_st_nt(ck + n * 64 + r, P[n]);
                    sk_st_nt(ck + (N + 1 + n) * 64 + r, Qin[n]);
                }
                sk_st_nt(a.ce + pd.ce_off + kk * (SK_LANES + 1) + r, E);
            }
            R Po[N + 1], Qo[N + 1];
            double Po0, Po1, Qo0, Qo1;
            int Tc = 0;
            sk_cell_fwd<R, N, TMAX>(P, Qin, P0, P1, Qin0, Qin1, cb[u], live, a.tab, Po, Qo, Po0,
                                    Po1, Qo0, Qo1, nullptr, nullptr,
                                    (CKPT && TMAX > 0) ? &Tc : nullptr);
            if (CKPT && TMAX > 0) {
                // the adjoint's replay folds the same tail rows
                tword |= (unsigned)Tc << (8 * (u % S));
                if (u % S == S - 1) {
                    if (r == 0 && tau - (S - 1) < g.nsteps)
                        a.ce[pd.ce_off + (int64_t)(tau / S) * (SK_LANES + 1) + SK_LANES] = (int)tword;
                    tword = 0u;
                }
            }
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                P[n] = Po[n];
                Qs[n] = Qo[n];
            }
            P0 = Po0;
            P1 = Po1;
            Qs0 = Qo0;
            Qs1 = Qo1;
            Es = E;
            if (live) {
                if (r == 63 && s + 1 < g.nstrips) {
                    if (gx) {
                        // the record in 16-byte stores (records are 16-byte
                        // aligned, GXW words each)
                        constexpr int NW = 4 + (N - 1) * (ES / 4) + 1, NQ = (NW + 3) / 4;
                        unsigned wd[4 * NQ];
                        wd[0] = (unsigned)__double2loint(Qo0);
                        wd[1] = (unsigned)__double2hiint(Qo0);
                        wd[2] = (unsigned)__double2loint(Qo1);
                        wd[3] = (unsigned)__double2hiint(Qo1);
#pragma unroll
                        for (int n = 2; n <= N; ++n) {
                            if constexpr (ES == 4) {
                                wd[4 + n - 2] = __float_as_uint(Qo[n]);
                            } else {
                                wd[4 + 2 * (n - 2)] = (unsigned)__double2loint(Qo[n]);
                                wd[4 + 2 * (n - 2) + 1] = (unsigned)__double2hiint(Qo[n]);
                            }
                        }
                        wd[NW - 1] = (unsigned)E;
#pragma unroll
                        for (int k = NW; k < 4 * NQ; ++k) wd[k] = 0u;
                        uint4* rec = reinterpret_cast<uint4*>(xg + (int64_t)j * GXW);
#pragma unroll
                        for (int k = 0; k < NQ; ++k)
                            rec[k] = make_uint4(wd[4 * k], wd[4 * k + 1], wd[4 * k + 2], wd[4 * k + 3]);
                        // (the checkpoint copy leaves once per block, from LDS)
                        if (CKPT) sk_edge_write<R, N>(ost + u * GXW, Qo0, Qo1, Qo, E);
                    } else {
                        // (the checkpoint copy of ring entries leaves once per block)
                        sk_edge_write<R, N>(ring + __mul24(j, RW), Qo0, Qo1, Qo, E);
                    }
                }
                if (i == g.lx - 1 && j == g.ly - 1) {
                    R kr = (R)0;
#pragma unroll
                    for (int n = N; n >= 2; --n) kr = fma(Po[n] + Qo[n], ifact<R>(n), kr);
                    const double kv = 0.5 * (Po0 + Qo0 + Po1 + Qo1 + (double)kr);
                    sk_write_k(a.K, a.Kexp, pd.k_idx, kv, E);
                }
            }
            if (L >= 0) {
                if (++j == g.Tp) {
                    j = 0;
                    ++s;
                }
            }
            ++L;
        }
        // the strip-boundary edges lane 63 handed over in this block, from
        // the ring (an entry is rewritten only Tp >= 64 steps after it was
        // written) or, for exchange pairs, the block's LDS staging, to the
        // adjoint's global copy in one coalesced pass
        if (CKPT) {
            // lane 63's place after the block: the place of step t0 + u is
            // 8 - u columns back (while L >= 0 it advanced every step)
            const int Le = __builtin_amdgcn_readlane(L, 63), se = __builtin_amdgcn_readlane(s, 63),
                      je = __builtin_amdgcn_readlane(j, 63);
            constexpr int QR = N + 2;  // N + 1 coefficients and the exponent
#pragma unroll
            for (int e0 = 0; e0 < 8 * QR; e0 += 64) {
                const int e = e0 + r, u = e / QR, w = e - u * QR;
                const int back = 8 - u;
                int jc = je - back, sc = se;
                if (jc < 0) {
                    jc += g.Tp;
                    --sc;
                }
                if (e < 8 * QR && Le - back >= 0 && sc + 1 < g.nstrips && jc < g.ly) {
                    const SkLds<unsigned> rec = gx ? ost + u * GXW : ring + __mul24(jc, RW);
                    const int64_t o = (int64_t)(sc + 1) * g.ly + jc;
                    if (w <= N) {
                        R v;
                        if (w < 2)
                            v = (R)(*(SkLds<double>)(rec + 2 * w));
                        else
                            v = *(SkLds<R>)(rec + 4 + (w - 2) * (ES / 4));
                        a.qb[pd.qb_off + o * (N + 1) + w] = v;
                    } else {
                        a.qe[pd.qe_off + o] = (int)rec[4 + (N - 1) * (ES / 4)];
                    }
                }
            }
        }
        // per-lane rescale of the live state
        if (live) {
            R m = (R)fmax(fmax(fabs(P0), fabs(Qs0)), fmax(fabs(P1), fabs(Qs1)));
#pragma unroll
            for (int n = 2; n <= N; ++n) {
                R ap = sk_abs(P[n]), aq = sk_abs(Qs[n]);
                m = ap > m ? ap : m;
                m = aq > m ? aq : m;
            }
            const int sh = sk_rescale_shift<R>(m);
            if (sh != 0) {
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = sk_ldexp(P[n], -sh);
                    Qs[n] = sk_ldexp(Qs[n], -sh);
                }
                P0 = ldexp(P0, -sh);
                P1 = ldexp(P1, -sh);
                Qs0 = ldexp(Qs0, -sh);
                Qs1 = ldexp(Qs1, -sh);
                E += sh;
                Es = E;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) cb[u] = cn[u];
    }
}

// ---------------------------------------------------------------------------
// (c') strip pipeline for single long pairs: the strips of one pair run on
// different co-resident workgroups (one wave each; workgroup w takes strips
// w, w + W, ...), in the anti-diagonal order of Section 3.2 applied to strips
// instead of cells.  Strip s hands the right edge of every column to strip
// s+1 through global records (two slots by strip parity) and publishes how
// many columns it has handed over; strip s+1 waits for that count before it
// loads the records of a block of columns, one 8-step block ahead of their
// use.  Strip s+2 rewrites a slot only after strip s+1 has loaded it (it
// depends on strip s+1's later columns), so two slots suffice.  Waits are
// bounded: a wave that waits too long raises the abort flag, and every
// waiting wave leaves on it, writing NaN for the pair.
// ---------------------------------------------------------------------------
// Jobs are strips.  One pair (desc == nullptr): the fields below describe
// it and job q is its strip q.  A job list (desc != nullptr): job q is strip
// jobs[q].y of the pair desc[jobs[q].x], whose arrays sit at the descriptor's
// offsets from the base pointers; every pair's strips appear in increasing
// order in the list (a wave only waits for jobs listed before its own).
// CKPT (job lists only): the sweep also stores what the pipelined adjoint
// replays: each strip's lane states every S local steps with their exponents
// and tail lengths, and the strip-boundary edges.
template <typename R>
struct PipeArgs {
    const R* cskew;        // skewed cell constants (rows s Tp + t of a pair)
    SkTab<R> tab;
    R* K;                  // indexed by the descriptors' k_idx
    int32_t* Kexp;         // nullable
    unsigned* xb;          // records [2][ly][sk_gx_words] per pair
    int* progress;         // [nstrips] per pair, zero at launch: columns handed over
    int* abort;            // zero at launch
    int32_t spin_limit;    // polls before a wait gives up
    const SkPairDesc* desc;  // pair descriptors
    const int2* jobs;        // (pair, strip), every pair's strips in increasing order
    int64_t njobs;
    int32_t lam;             // dyadic refinement of the pairs' grids
    R* ck;                   // CKPT: per strip, [sk_pipe_steps / S][2][N + 1][64]
    int32_t* ce;             // CKPT: per strip, [sk_pipe_steps / S][64 + 1]
    R* qb;                   // CKPT: strip-boundary edges [nstrips][ly][N + 1]
    int32_t* qe;             // CKPT: their exponents [nstrips][ly]
    int32_t S;               // CKPT: checkpoint stride
};

// Hand-over without cache-wide fences: the producer stores its records and
// counts with device-coherent stores and waits for its stores to complete
// before it raises a count; the consumer polls the count with
// device-coherent loads and only then issues its device-coherent record
// loads.  (An agent-scope release/acquire would write back or invalidate a
// whole L2 per block, which thousands of concurrent strips cannot afford.)
__device__ __forceinline__ void sk_store_coherent(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// a record of `nw` words (8-byte aligned; word nw is writable padding when
// nw is odd) in 8-byte device-coherent stores
template <int NW>
__device__ __forceinline__ void sk_store_record_coherent(unsigned* rec, const unsigned (&wd)[NW]) {
#pragma unroll
    for (int k = 0; k < NW; k += 2) {
        const unsigned long long v =
            (unsigned long long)wd[k] | ((unsigned long long)(k + 1 < NW ? wd[k + 1] : 0u) << 32);
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(rec + k), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}
__device__ __forceinline__ void sk_stores_complete() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // every counter of this wave at zero
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Wave-uniform bounded wait until *prog >= need.  Returns false on abort.
__device__ __forceinline__ bool sk_wait_count(const int* prog, int need, int* abort, int limit) {
    for (int it = 0;; ++it) {
        if (__hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);  // record loads stay after the poll
            return true;
        }
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (it >= limit) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__builtin_amdgcn_readfirstlane(__lane_id()) == __lane_id())
                sk_raise_status(SK_STATUS_WAIT_ABORT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

template <typename R, int N, int TMAX, bool CKPT, int S>
__global__ __launch_bounds__(64) void k_sweep_pipe(const PipeArgs<R> a) {
    const int r = threadIdx.x;
    constexpr int ES = (int)sizeof(R), GXW = sk_gx_words(N, ES);
    constexpr int XR = (8 * GXW + 63) / 64;
    extern __shared__ __align__(16) unsigned char sk_smem[];
    unsigned* stage = reinterpret_cast<unsigned*>(sk_smem);  // [8][GXW]
    // lane 63's records of the current 8-step block, stored to the global
    // slot by all lanes at the block's end (before it is published)
    const SkLds<unsigned> ost = (SkLds<unsigned>)(sk_smem + sk_gx_stage_bytes(N, ES));  // [8][GXW]
    constexpr int NW = 4 + (N - 1) * (ES / 4) + 1;  // words of a record
    for (int64_t q = blockIdx.x; q < a.njobs; q += gridDim.x) {
        // the job: strip s of a pair with geometry g and arrays at these bases
        const int2 jb = a.jobs[q];
        const SkPairDesc pd = a.desc[jb.x];
        const int s = jb.y;
        const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
        const R* cbase = a.cskew + pd.c_off;
        unsigned* xbase = a.xb + pd.xb_off;
        int* prog = a.progress + pd.pg_off;
        const int64_t k_idx = pd.k_idx;
        const int ly = g.ly;
        const int nloc = sk_pipe_steps(ly);
        // lane 0 reads column t at local step t
        auto col0 = [&](int t) -> int { return t < ly ? t : -1; };
        const int i = s * 64 + r;
        const bool rowok = i < g.lx;
        const bool has_next = s + 1 < g.nstrips;
        const unsigned* rin = xbase + (size_t)((s + 1) & 1) * ly * GXW;  // strip s-1's slot
        unsigned* rout = xbase + (size_t)(s & 1) * ly * GXW;
        const R* cs = cbase + (int64_t)s * g.Tp * 64;
        const int64_t rows_left = (int64_t)g.nsteps_pad - (int64_t)s * g.Tp;
        R* ckb = nullptr;
        int32_t* ceb = nullptr;
        if (CKPT) {
            const int64_t nckl = nloc / S;
            ckb = a.ck + pd.ck_off + (int64_t)s * nckl * 2 * (N + 1) * 64;
            ceb = a.ce + pd.ce_off + (int64_t)s * nckl * (SK_LANES + 1);
        }
        unsigned tword = 0u;  // tail lengths of the current checkpoint segment
        R P[N + 1], Qs[N + 1];
        double P0 = 0.0, P1 = 0.0, Qs0 = 0.0, Qs1 = 0.0;
#pragma unroll
        for (int n = 0; n <= N; ++n) {
            P[n] = (R)0;
            Qs[n] = (R)0;
        }
        int E = 0, Es = 0;
        unsigned xr[XR];
#pragma unroll
        for (int h = 0; h < XR; ++h) xr[h] = 0u;
        bool ok = true;
        if (s > 0) {  // records of columns 0..7
            ok = sk_wait_count(prog + s - 1, ly < 8 ? ly : 8, a.abort, a.spin_limit);
            if (ok) {
#pragma unroll
                for (int h = 0; h < XR; ++h) {
                    const int w = r + 64 * h;
                    if (w < 8 * GXW) {
                        const int m = w / GXW, qw = w - m * GXW;
                        const int col = col0(m);
                        if (col >= 0)
                            xr[h] = __hip_atomic_load(rin + (int64_t)col * GXW + qw, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
        }
        int published = 0;
        for (int t0 = 0; ok && t0 < nloc; t0 += 8) {
            if (s > 0) {
                const int need = t0 + 16 < ly ? t0 + 16 : ly;
                ok = sk_wait_count(prog + s - 1, need, a.abort, a.spin_limit);
                if (!ok) break;
                sk_gx_stage<GXW, true>(xr, stage, rin, t0 + 8, r, col0);
            }
            R cb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) cb[u] = (t0 + u < rows_left) ? cs[(int64_t)(t0 + u) * 64 + r] : (R)0;
            bool live = false;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u, j = t - r;
                R Qin[N + 1];
#pragma unroll
                for (int n = 2; n <= N; ++n) Qin[n] = lane_from_prev(Qs[n]);
                double Qin0 = lane_from_prev(Qs0), Qin1 = lane_from_prev(Qs1);
                int Ein = lane_from_prev(Es);
                live = rowok && j >= 0 && j < ly;
                if (live) {
                    if (j == 0) {
                        P0 = 1.0;
                        P1 = 0.0;
#pragma unroll
                        for (int n = 2; n <= N; ++n) P[n] = (R)0;
                        E = 0;
                    }
                    if (r == 0) {
                        if (s == 0) {
                            Qin0 = 1.0;
                            Qin1 = 0.0;
#pragma unroll
                            for (int n = 2; n <= N; ++n) Qin[n] = (R)0;
                            Ein = 0;
                        } else {
                            const unsigned* rec = stage + u * GXW;
                            Qin0 = *reinterpret_cast<const double*>(rec);
                            Qin1 = *reinterpret_cast<const double*>(rec + 2);
#pragma unroll
                            for (int n = 2; n <= N; ++n)
                                Qin[n] = *reinterpret_cast<const R*>(rec + 4 + (n - 2) * (ES / 4));
                            Ein = (int)rec[4 + (N - 1) * (ES / 4)];
                        }
                    }
                    const int Ec = E > Ein ? E : Ein;
                    const int dp = E - Ec, dq = Ein - Ec;
                    if (sk_wave_any(dp != 0 || dq != 0)) {
                        P0 = ldexp(P0, dp);
                        P1 = ldexp(P1, dp);
                        Qin0 = ldexp(Qin0, dq);
                        Qin1 = ldexp(Qin1, dq);
#pragma unroll
                        for (int n = 2; n <= N; ++n) {
                            P[n] = sk_ldexp(P[n], dp);
                            Qin[n] = sk_ldexp(Qin[n], dq);
                        }
                    }
                    E = Ec;
                }
                P[0] = (R)P0;
                P[1] = (R)P1;
                Qin[0] = (R)Qin0;
                Qin[1] = (R)Qin1;
                if (CKPT && (t % S) == 0) {
                    R* ck = ckb + (int64_t)(t / S) * 2 * (N + 1) * 64;
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        ck[n * 64 + r] = P[n];
                        ck[(N + 1 + n) * 64 + r] = Qin[n];
                    }
                    ceb[(int64_t)(t / S) * (SK_LANES + 1) + r] = E;
                }
                R Po[N + 1], Qo[N + 1];
                double Po0, Po1, Qo0, Qo1;
                int Tc = 0;
                sk_cell_fwd<R, N, TMAX>(P, Qin, P0, P1, Qin0, Qin1, cb[u], live, a.tab, Po, Qo, Po0,
                                        Po1, Qo0, Qo1, nullptr, nullptr,
                                        (CKPT && TMAX > 0) ? &Tc : nullptr);
                if (CKPT && TMAX > 0) {
                    // the adjoint's replay folds the same tail rows
                    tword |= (unsigned)Tc << (8 * (t % S));
                    if (t % S == S - 1) {
                        if (r == 0) ceb[(int64_t)(t / S) * (SK_LANES + 1) + SK_LANES] = (int)tword;
                        tword = 0u;
                    }
                }
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = Po[n];
                    Qs[n] = Qo[n];
                }
                P0 = Po0;
                P1 = Po1;
                Qs0 = Qo0;
                Qs1 = Qo1;
                Es = E;
                if (live) {
                    if (r == 63 && has_next) {
                        if (CKPT) {
                            sk_edge_write<R, N>(ost + u * GXW, Qo0, Qo1, Qo, E);
                        } else {
                            unsigned* rec = rout + (int64_t)j * GXW;
                            unsigned wd[NW];
                            *reinterpret_cast<double*>(wd) = Qo0;
                            *reinterpret_cast<double*>(wd + 2) = Qo1;
#pragma unroll
                            for (int n = 2; n <= N; ++n)
                                *reinterpret_cast<R*>(wd + 4 + (n - 2) * (ES / 4)) = Qo[n];
                            wd[NW - 1] = (unsigned)E;
                            sk_store_record_coherent<NW>(rec, wd);
                        }
                    }
                    if (i == g.lx - 1 && j == ly - 1) {
                        R kr = (R)0;
#pragma unroll
                        for (int n = N; n >= 2; --n) kr = fma(Po[n] + Qo[n], ifact<R>(n), kr);
                        const double kv = 0.5 * (Po0 + Qo0 + Po1 + Qo1 + (double)kr);
                        sk_write_k(a.K, a.Kexp, k_idx, kv, E);
                    }
                }
            }
            // CKPT: lane 63's records of this block (columns t0 + m - 63
            // that exist) to strip s+1's slot and to the adjoint's copy of
            // the boundary edges, in one pass of all lanes (without CKPT lane
            // 63 stores its records as it goes: the pass's registers would
            // cost that kernel a wave per SIMD)
            if (CKPT && has_next) {
#pragma unroll
                for (int h = 0; h < XR; ++h) {
                    const int w = r + 64 * h, m = w / GXW, qw = w - m * GXW, jc = t0 + m - 63;
                    if (w < 8 * GXW && qw < NW && jc >= 0 && jc < ly)
                        sk_store_coherent(rout + (int64_t)jc * GXW + qw, ost[w]);
                }
                {
                    constexpr int QR = N + 2;  // N + 1 coefficients and the exponent
#pragma unroll
                    for (int e0 = 0; e0 < 8 * QR; e0 += 64) {
                        const int e = e0 + r, m = e / QR, w = e - m * QR, jc = t0 + m - 63;
                        if (e < 8 * QR && jc >= 0 && jc < ly) {
                            const SkLds<unsigned> rec = ost + m * GXW;
                            const int64_t o = (int64_t)(s + 1) * ly + jc;
                            if (w <= N) {
                                R v;
                                if (w < 2)
                                    v = (R)(*(SkLds<double>)(rec + 2 * w));
                                else
                                    v = *(SkLds<R>)(rec + 4 + (w - 2) * (ES / 4));
                                a.qb[pd.qb_off + o * (N + 1) + w] = v;
                            } else {
                                a.qe[pd.qe_off + o] = (int)rec[NW - 1];
                            }
                        }
                    }
                }
            }
            // lane 63 has handed over the columns j <= t0 + 7 - 63: publish
            // them once its record stores have completed
            int done = t0 + 8 - 63;
            done = done < 0 ? 0 : (done > ly ? ly : done);
            if (has_next && done > published) {
                sk_stores_complete();
                if (r == 63) sk_store_coherent(reinterpret_cast<unsigned*>(prog + s), (unsigned)done);
                published = done;
            }
            // per-lane rescale of the live state (exact: powers of two)
            if (live) {
                R m = (R)fmax(fmax(fabs(P0), fabs(Qs0)), fmax(fabs(P1), fabs(Qs1)));
#pragma unroll
                for (int n = 2; n <= N; ++n) {
                    R ap = sk_abs(P[n]), aq = sk_abs(Qs[n]);
                    m = ap > m ? ap : m;
                    m = aq > m ? aq : m;
                }
                const int sh = sk_rescale_shift<R>(m);
                if (sh != 0) {
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        P[n] = sk_ldexp(P[n], -sh);
                        Qs[n] = sk_ldexp(Qs[n], -sh);
                    }
                    P0 = ldexp(P0, -sh);
                    P1 = ldexp(P1, -sh);
                    Qs0 = ldexp(Qs0, -sh);
                    Qs1 = ldexp(Qs1, -sh);
                    E += sh;
                    Es = E;
                }
            }
        }
        if (!ok) {  // a wait gave up: the pair's value is unknown (later
                    // jobs still run: their waits end at once on the flag)
            if (r == 0) sk_write_k(a.K, a.Kexp, k_idx, (double)NAN, 0);
        }
    }
}

// ---------------------------------------------------------------------------
// (d) adjoint sweep: reversed wavefront with segment recompute
// ---------------------------------------------------------------------------
template <typename R>
struct AdjArgs {
    SkPairSrc src;
    const R* cskew;
    SkTab<R> tab;
    const R* gK;           // dL/dK per output index
    const int32_t* gKexp;  // nullable: seed = gK * 2^gKexp
    const R* ck;
    const int32_t* ce;
    const R* qb;
    const int32_t* qe;
    R* gskew;              // out: skewed dL/dc
    unsigned* xb;          // global strip-boundary exchange records (long pairs)
    int32_t gx_cols;       // pairs with more columns use the global exchange
    int32_t lam;           // dyadic refinement of the pairs' grids (hybrid scheme)
    int32_t S;             // checkpoint stride (as the checkpointing sweep's)
};

// Exponent of an adjoint vector that is zero by construction: below any
// real exponent, so alignment to the larger exponent ignores it.
#define SK_ZERO_EXP (-(1 << 29))

template <typename R, int N, int TMAX, int S, bool GX>
__device__ __forceinline__ void sk_adjoint_body(const AdjArgs<R>& a) {
    const int r = threadIdx.x;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) return;
    // adjoint strip-boundary vectors handed from lane 0 of strip s to lane 63
    // of strip s-1: LDS ring, or global records staged one block ahead
    constexpr int ES = (int)sizeof(R), GXW = sk_gx_words(N, ES);
    const bool gx = GX && g.ly > a.gx_cols;  // wave-uniform
    extern __shared__ __align__(16) unsigned char sk_smem[];
    unsigned* stage = reinterpret_cast<unsigned*>(sk_smem);  // [8][GXW]
    // boundary edges lane 0 replays at steps 1..S-1 of the current segment
    // (LDS-typed pointers: 32-bit address arithmetic)
    SkLds<unsigned> qst = (SkLds<unsigned>)(sk_smem + sk_gx_stage_bytes(N, ES));
    SkLds<R> llds = (SkLds<R>)(sk_smem + sk_gx_stage_bytes(N, ES) + sk_adj_qst_bytes(N, ES));
    SkLds<int> ltag = (SkLds<int>)(llds + g.ly * (N + 1));
    unsigned* xg = a.xb + pd.xb_off;
    unsigned xr[(8 * GXW + 63) / 64];
#pragma unroll
    for (int h = 0; h < (8 * GXW + 63) / 64; ++h) xr[h] = 0u;
    // column lane 63 reads at step tau (rows that are not the last), or -1
    auto lane63_col = [&](int tau) -> int {
        const int L63 = tau - 63;
        if (tau < 0 || L63 < 0) return -1;
        const int s6 = L63 / g.Tp, j6 = L63 - s6 * g.Tp, i6 = s6 * 64 + 63;
        return (s6 < g.nstrips && j6 < g.ly && i6 < g.lx - 1) ? j6 : -1;
    };
    const R* cs = a.cskew + pd.c_off;
    R* gs = a.gskew + pd.c_off;
    const R gk = a.gK[pd.g_idx];
    const int gexp = a.gKexp ? a.gKexp[pd.g_idx] : 0;

    // adjoint state: lp (own, exponent El), lqs (sent to lane r-1, exponent Els)
    R lp[N + 1], lqs[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) {
        lp[n] = (R)0;
        lqs[n] = (R)0;
    }
    int El = SK_ZERO_EXP, Els = SK_ZERO_EXP;
    const int nck = (g.nsteps + S - 1) / S;
    // tail rows whose derivatives a replayed step keeps; segments with a
    // longer tail take the slow path below
    constexpr int TR = TMAX > 0 ? SkTailReg<R>::value : 0;
    // Inputs of a checkpoint segment are loaded one segment ahead (PF: the
    // stride-4 kernels, whose registers allow two waves per SIMD only, so
    // memory latency is not hidden by other waves): the segment's cell
    // constants at the top of the previous segment, the lane state, its
    // exponent and one word per lane of the boundary edges lane 0 reads at
    // steps 1..S-1 (plus, in lane TWL, the tail-length word) once the
    // previous segment's replay no longer needs its own.  The boundary edges
    // go through LDS, so no load is waited for inside a segment.
    constexpr bool PF = S >= 4;
    constexpr int QW = sk_adj_qst_words(N, ES), TWL = (S - 1) * QW;
    static_assert(!PF || (S <= 4 && TWL < 64), "staged boundary edges exceed one word per lane");
    R pfP[N + 1], pfQ[N + 1], pfc[S];
    int pfE = 0;
    unsigned pfq = 0u;
    auto prefetch_c = [&](int kk) {
#pragma unroll
        for (int u = 0; u < S; ++u) pfc[u] = cs[(int64_t)(kk * S + u) * 64 + r];
    };
    auto prefetch_state = [&](int kk) {
        const R* ck = a.ck + pd.ck_off + (int64_t)kk * 2 * (N + 1) * 64;
#pragma unroll
        for (int n = 0; n <= N; ++n) {
            pfP[n] = sk_ld_nt(ck + n * 64 + r);
            pfQ[n] = sk_ld_nt(ck + (N + 1 + n) * 64 + r);
        }
        pfE = sk_ld_nt(a.ce + pd.ce_off + (int64_t)kk * (SK_LANES + 1) + r);
        // word w of the edge lane 0 takes at step u (live, strips >= 1)
        pfq = 0u;
        if (r < TWL) {
            const int u = 1 + r / QW, w = r - (u - 1) * QW;
            const int L0 = kk * S + u, s0 = L0 / g.Tp, j0 = L0 - s0 * g.Tp;
            if (s0 >= 1 && s0 < g.nstrips && j0 < g.ly && s0 * 64 < g.lx) {
                const int64_t o = (int64_t)s0 * g.ly + j0;
                if (w < (N + 1) * (ES / 4))
                    pfq = reinterpret_cast<const unsigned*>(a.qb + pd.qb_off + o * (N + 1))[w];
                else if (w == QW - 1)
                    pfq = (unsigned)a.qe[pd.qe_off + o];
            }
        } else if (TMAX > 0 && r == TWL) {
            pfq = (unsigned)a.ce[pd.ce_off + (int64_t)kk * (SK_LANES + 1) + SK_LANES];
        }
    };
    // Inputs of replayed step u of a segment: the bottom edge P (this lane's
    // state) and the left edge Qin (from lane r-1, or the strip boundary /
    // the initial edge for lane 0), aligned to a common exponent E.  Step 0
    // takes the checkpoint as it is.  Returns whether the cell is live.
    auto replay_in = [&](int u, R (&P)[N + 1], const R (&Qs)[N + 1], R (&Qin)[N + 1], int& E,
                         int Es, int L, int s, int j) -> bool {
        const int i = s * 64 + r;
        const bool live = (L >= 0) && (s < g.nstrips) && (j < g.ly) && (i < g.lx);
        if (u == 0) {
#pragma unroll
            for (int n = 0; n <= N; ++n) Qin[n] = Qs[n];
            return live;
        }
#pragma unroll
        for (int n = 0; n <= N; ++n) Qin[n] = lane_from_prev(Qs[n]);
        int Ein = lane_from_prev(Es);
        if (live) {
            if (j == 0) {
#pragma unroll
                for (int n = 0; n <= N; ++n) P[n] = n == 0 ? (R)1 : (R)0;
                E = 0;
            }
            if (r == 0) {
                if (s == 0) {
#pragma unroll
                    for (int n = 0; n <= N; ++n) Qin[n] = n == 0 ? (R)1 : (R)0;
                    Ein = 0;
                } else if (PF) {
                    const SkLds<unsigned> q = qst + (u - 1) * QW;
#pragma unroll
                    for (int n = 0; n <= N; ++n) Qin[n] = ((SkLds<R>)q)[n];
                    Ein = (int)q[QW - 1];
                } else {
                    const int64_t o = (int64_t)s * g.ly + j;
#pragma unroll
                    for (int n = 0; n <= N; ++n) Qin[n] = a.qb[pd.qb_off + o * (N + 1) + n];
                    Ein = a.qe[pd.qe_off + o];
                }
            }
            const int Ec = E > Ein ? E : Ein;
            const int dp = E - Ec, dq = Ein - Ec;
            if (sk_wave_any(dp != 0 || dq != 0)) {
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = sk_ldexp(P[n], dp);
                    Qin[n] = sk_ldexp(Qin[n], dq);
                }
            }
            E = Ec;
        }
        return live;
    };
    // One adjoint step (replayed step u of the segment at tau0): the adjoint
    // of the cell's top edge comes from this lane's later cell, that of its
    // right edge from lane r+1 (lane 63: the next strip's lane 0, through the
    // ring or the staging slot); `cell(ap, aq, gv)` maps them to the inputs'
    // adjoints (lp, lqs) and dL/dc.
    auto adj_step = [&](int u, int tau0, bool live, int ss, int jj, int Eu, auto&& cell) {
        const int tau = tau0 + u;
        const int i = ss * 64 + r;
        const bool last_row = (i == g.lx - 1), last_col = (jj == g.ly - 1);
        R lq_recv[N + 1];
#pragma unroll
        for (int n = 0; n <= N; ++n) lq_recv[n] = lane_from_next(lqs[n]);
        int El_recv = lane_from_next(Els);
        if (r == 63 && live && !last_row) {
            if (gx) {
                const unsigned* rec = stage + (tau & 7) * GXW;
#pragma unroll
                for (int n = 0; n <= N; ++n)
                    lq_recv[n] = *reinterpret_cast<const R*>(rec + n * (ES / 4));
                El_recv = (int)rec[(N + 1) * (ES / 4)];
            } else {
#pragma unroll
                for (int n = 0; n <= N; ++n) lq_recv[n] = llds[__mul24(jj, N + 1) + n];
                El_recv = ltag[jj];
            }
        }
        // outputs nobody consumes have zero adjoint (a wave-uniform test
        // skips the selects on steps where every lane consumes both)
        const bool ta = live && !last_col, tb = live && !last_row;
        R ap[N + 1], aq[N + 1];
#pragma unroll
        for (int n = 0; n <= N; ++n) {
            ap[n] = lp[n];
            aq[n] = lq_recv[n];
        }
        int ea = El, eb = El_recv;
        if (sk_wave_any(!(ta && tb))) {
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                ap[n] = ta ? ap[n] : (R)0;
                aq[n] = tb ? aq[n] : (R)0;
            }
            ea = ta ? ea : SK_ZERO_EXP;
            eb = tb ? eb : SK_ZERO_EXP;
        }
        // endpoint seed (once per pair): L = gK * 1/2 sum_n (Po'_n + Qo'_n)/n!
        const bool seed = live && last_col && last_row;
        if (sk_wave_any(seed) && seed) {
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                ap[n] = (R)0.5 * gk * ifact<R>(n);
                aq[n] = ap[n];
            }
            ea = gexp;
            eb = gexp;
        }
        const int Ec = ea > eb ? ea : eb;
        // vectors tagged SK_ZERO_EXP are zero: only real exponents below
        // Ec need a shift, which is rare
        const bool sa = ea != Ec && ea != SK_ZERO_EXP, sb = eb != Ec && eb != SK_ZERO_EXP;
        if (sk_wave_any(sa || sb)) {
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                ap[n] = sk_ldexp(ap[n], ea - Ec);
                aq[n] = sk_ldexp(aq[n], eb - Ec);
            }
        }
        R gv;
        cell(ap, aq, gv);
        El = Ec;
        Els = Ec;
        if (live && r == 0 && ss > 0) {
            if (gx) {
                unsigned* rec = xg + (int64_t)jj * GXW;
#pragma unroll
                for (int n = 0; n <= N; ++n) *reinterpret_cast<R*>(rec + n * (ES / 4)) = lqs[n];
                rec[(N + 1) * (ES / 4)] = (unsigned)Ec;
            } else {
#pragma unroll
                for (int n = 0; n <= N; ++n) llds[__mul24(jj, N + 1) + n] = lqs[n];
                ltag[jj] = Ec;
            }
        }
        sk_st_nt(gs + (int64_t)tau * 64 + r, live ? sk_ldexp(gv, Ec + Eu) : (R)0);
        if ((tau & 7) == 0 && live) {
            R m = (R)0;
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                R x1 = sk_abs(lp[n]), x2 = sk_abs(lqs[n]);
                m = x1 > m ? x1 : m;
                m = x2 > m ? x2 : m;
            }
            const int sh = sk_rescale_shift<R>(m);
            if (sh != 0) {
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    lp[n] = sk_ldexp(lp[n], -sh);
                    lqs[n] = sk_ldexp(lqs[n], -sh);
                }
                El += sh;
                Els = El;
            }
        }
    };
    if (PF) {
        prefetch_c(nck - 1);
        prefetch_state(nck - 1);
    }
    for (int kk = nck - 1; kk >= 0; --kk) {
        const int tau0 = kk * S;
        // blocks of 8 steps, processed from the top; a segment never
        // straddles two blocks (S divides 8)
        if (gx && (kk == nck - 1 || ((tau0 + S) & 7) == 0))
            sk_gx_stage<GXW>(xr, stage, xg, (tau0 & ~7) - 8, r, lane63_col);
        const R* ck = a.ck + pd.ck_off + (int64_t)kk * 2 * (N + 1) * 64;
        R cseg[S];
        int E0;
        unsigned tword = 0u;  // tail lengths the forward folded at the segment's steps
        if (PF) {
#pragma unroll
            for (int u = 0; u < S; ++u) cseg[u] = pfc[u];
            E0 = pfE;
            if (TMAX > 0) tword = (unsigned)__builtin_amdgcn_readlane((int)pfq, TWL);
            // this segment's boundary edges into LDS (the wave's own earlier
            // LDS reads of the previous segment's are ordered before)
            if (r < TWL) qst[r] = pfq;
            if (kk > 0) prefetch_c(kk - 1);
        } else {
            E0 = sk_ld_nt(a.ce + pd.ce_off + (int64_t)kk * (SK_LANES + 1) + r);
            if (TMAX > 0)
                tword = (unsigned)__builtin_amdgcn_readfirstlane(
                    a.ce[pd.ce_off + (int64_t)kk * (SK_LANES + 1) + SK_LANES]);
        }
        unsigned tseg = 0u;  // longest tail of the segment (wave-uniform)
#pragma unroll
        for (int u = 0; u < S; ++u) {
            const unsigned tu = (tword >> (8 * u)) & 0xffu;
            tseg = tu > tseg ? tu : tseg;
        }
        if (TMAX == 0 || tseg <= (unsigned)TR) {
            // ---- replay the segment's forward from the checkpoint, recording
            // each cell's row derivatives, kept tail length and exponent
            constexpr int M = N + TR;
            R Dp[S][M], Dq[S][M];
            R Wst[S][N];  // c^m/m! of each step, kept for its adjoint (PF only)
            int Tst[S], Est[S];
            bool lv[S];
            int sst[S], jst[S];
            if (!PF) {
#pragma unroll
                for (int u = 0; u < S; ++u) cseg[u] = cs[(int64_t)(tau0 + u) * 64 + r];
            }
            int E = E0;
            R P[N + 1], Qs[N + 1];
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                P[n] = PF ? pfP[n] : sk_ld_nt(ck + n * 64 + r);
                Qs[n] = PF ? pfQ[n] : sk_ld_nt(ck + (N + 1 + n) * 64 + r);
            }
            int Es = E;
            int L = tau0 - r, s = 0, j = 0;
            if (L >= 0) {
                s = L / g.Tp;
                j = L - s * g.Tp;
            }
#pragma unroll
            for (int u = 0; u < S; ++u) {
                R Qin[N + 1];
                const bool live = replay_in(u, P, Qs, Qin, E, Es, L, s, j);
                lv[u] = live;
                sst[u] = s;
                jst[u] = j;
                Est[u] = E;
                R Po[N + 1], Qo[N + 1];
                double Po0, Po1, Qo0, Qo1;
                Tst[u] = (int)((tword >> (8 * u)) & 0xffu);
                sk_cell_fwd<R, N, TR, true, false, true>(P, Qin, 0.0, 0.0, 0.0, 0.0, cseg[u], live,
                                                         a.tab, Po, Qo, Po0, Po1, Qo0, Qo1, Dp[u],
                                                         Dq[u], nullptr, Tst[u],
                                                         PF ? Wst[u] : nullptr);
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = Po[n];
                    Qs[n] = Qo[n];
                }
                Es = E;
                if (L >= 0) {
                    if (++j == g.Tp) {
                        j = 0;
                        ++s;
                    }
                }
                ++L;
            }
            // the next segment's state loads while this one's adjoint runs
            if (PF && kk > 0) prefetch_state(kk - 1);
            // ---- adjoint steps in reverse
#pragma unroll
            for (int u = S - 1; u >= 0; --u)
                adj_step(u, tau0, lv[u], sst[u], jst[u], Est[u], [&](R (&ap)[N + 1], R (&aq)[N + 1], R& gv) {
                    sk_cell_adj<R, N, TR>(cseg[u], Tst[u], a.tab, ap, aq, Dp[u], Dq[u], lp, lqs, gv,
                                          PF ? Wst[u] : nullptr);
                });
        } else {
            // ---- slow path (a tail longer than TR rows in this segment):
            // for each step u, from the last, replay steps 0..u-1 from the
            // checkpoint to recover the cell's inputs, then take the adjoint
            // step with the row derivatives computed from those inputs
#pragma unroll 1
            for (int u = S - 1; u >= 0; --u) {
                int E = E0;
                R P[N + 1], Qs[N + 1], Qin[N + 1];
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = ck[n * 64 + r];
                    Qs[n] = ck[(N + 1 + n) * 64 + r];
                }
                int Es = E;
                int L = tau0 - r, s = 0, j = 0;
                if (L >= 0) {
                    s = L / g.Tp;
                    j = L - s * g.Tp;
                }
                bool live = false;
#pragma unroll 1
                for (int v = 0;; ++v) {
                    live = replay_in(v, P, Qs, Qin, E, Es, L, s, j);
                    if (v == u) break;
                    R Po[N + 1], Qo[N + 1];
                    double Po0, Po1, Qo0, Qo1;
                    const int Tv = (int)((tword >> (8 * v)) & 0xffu);
                    sk_cell_fwd<R, N, TMAX, false, false, true>(
                        P, Qin, 0.0, 0.0, 0.0, 0.0, cs[(int64_t)(tau0 + v) * 64 + r], live, a.tab,
                        Po, Qo, Po0, Po1, Qo0, Qo1, nullptr, nullptr, nullptr, Tv);
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        P[n] = Po[n];
                        Qs[n] = Qo[n];
                    }
                    Es = E;
                    if (L >= 0) {
                        if (++j == g.Tp) {
                            j = 0;
                            ++s;
                        }
                    }
                    ++L;
                }
                const int Tu = (int)((tword >> (8 * u)) & 0xffu);
                const R cu = cs[(int64_t)(tau0 + u) * 64 + r];
                adj_step(u, tau0, live, s, j, E, [&](R (&ap)[N + 1], R (&aq)[N + 1], R& gv) {
                    sk_cell_adj_in<R, N, TMAX>(cu, Tu, a.tab, ap, aq, P, Qin, lp, lqs, gv);
                });
            }
            if (PF && kk > 0) prefetch_state(kk - 1);
        }
    }
}

// Two entry points of the same body: where the register footprint allows it,
// the compiler is asked to fit two waves per SIMD (the adjoint is latency
// bound at one); elsewhere forcing it would spill to scratch.  The FP32
// exchange variant for N = 8 (approximation) spills 6 registers at two waves
// and is still faster (1024 x 1024 d = 32 Gram, 32 rows: 1021 -> 647 ms).
template <typename R, int N, int TMAX, bool GX>
constexpr bool sk_adj_two_waves() {
    return sizeof(R) == 4 ? (GX ? TMAX == 0 : (TMAX == 0 || N <= 6))
                          : (TMAX == 0 && N <= 6 && !GX);
}

template <typename R, int N, int TMAX, int S, bool GX>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_adjoint_w2(const AdjArgs<R> a) {
    sk_adjoint_body<R, N, TMAX, S, GX>(a);
}

template <typename R, int N, int TMAX, int S, bool GX>
__global__ __launch_bounds__(64) void k_adjoint(const AdjArgs<R> a) {
    sk_adjoint_body<R, N, TMAX, S, GX>(a);
}

// ---------------------------------------------------------------------------
// (d') strip pipeline of the adjoint: the reversed grid's strips on
// co-resident workgroups.  The adjoint flows from the last cell back to the
// first, so strip s needs, at lane 63, the adjoint of the left edge that
// lane 0 of strip s+1 produces: strip s+1 runs ahead.  Within a strip the
// local steps run backwards; lane r holds column t - r at local step t, so
// lane 0 hands over column j at step j and lane 63 consumes it at step
// j + 63.  The hand-over mirrors the forward pipeline's: records in two slots
// by strip parity (slot s & 1 written by strip s), device-coherent stores,
// a count of columns handed over from the top published by lane 0 once the
// block's stores have completed, bounded waits with the abort flag, and
// records loaded one 8-step block ahead through the LDS staging slot.  The
// lane states come from the checkpoints of the pipelined checkpoint sweep
// (per strip, on the same local steps), replayed S steps at a time as in
// the batched adjoint.  Only the strip's own cells of dL/dc are written: the
// skewed rows of neighbouring strips overlap it.
// ---------------------------------------------------------------------------
template <typename R>
struct AdjPipeArgs {
    const R* cskew;
    SkTab<R> tab;
    const R* gK;            // dL/dK per output index
    const int32_t* gKexp;   // nullable: seed = gK * 2^gKexp
    const R* ck;            // per strip, [sk_pipe_steps / S][2][N + 1][64]
    const int32_t* ce;      // per strip, [sk_pipe_steps / S][64 + 1]
    const R* qb;            // strip-boundary edges [nstrips][ly][N + 1]
    const int32_t* qe;
    R* gskew;               // out: skewed dL/dc (the strips' own cells)
    unsigned* xb;           // records [2][ly][sk_gx_words] per pair
    int* progress;          // [nstrips] per pair, zero at launch
    int* abort;             // zero at launch
    int32_t spin_limit;
    const SkPairDesc* desc;
    const int2* jobs;       // (pair, strip), every pair's strips in decreasing order
    int64_t njobs;
    int32_t lam;            // dyadic refinement of the pairs' grids (hybrid scheme)
    int32_t S;              // checkpoint stride (as the checkpointing sweep's)
};

// LDS of the pipelined adjoint: the exchange staging slot, then the
// segment's row derivatives [P/Q][S][N + TR][64 lanes] (in LDS rather than
// registers, which leaves room for two waves per SIMD without spilling), TR
// the tail rows kept per step (SkTailReg; 0 for the approximation scheme,
// TMAX = 0), the boundary edges lane 0 replays at steps 1..S-1 of a segment
// (staged one segment ahead, as in the batched adjoint), and lane 0's
// outgoing records of the current 8-step block.
template <typename R>
__host__ __device__ constexpr int sk_adj_pipe_lds(int N, int TMAX, int S) {
    return sk_gx_stage_bytes(N, (int)sizeof(R)) +
           2 * S * (N + (TMAX > 0 ? SkTailReg<R>::value : 0)) * 64 * (int)sizeof(R) +
           sk_adj_qst_bytes(N, (int)sizeof(R)) + sk_gx_stage_bytes(N, (int)sizeof(R));
}

template <typename R, int N, int TMAX, int S>
__device__ __forceinline__ void sk_adjoint_pipe_body(const AdjPipeArgs<R>& a) {
    const int r = threadIdx.x;
    constexpr int ES = (int)sizeof(R), GXW = sk_gx_words(N, ES);
    constexpr int TR = TMAX > 0 ? SkTailReg<R>::value : 0;
    constexpr int XR = (8 * GXW + 63) / 64, M = N + TR, RW = (N + 1) * (ES / 4) + 1;
    extern __shared__ __align__(16) unsigned char sk_smem[];
    unsigned* stage = reinterpret_cast<unsigned*>(sk_smem);  // [8][GXW]
    R* dlds = reinterpret_cast<R*>(sk_smem + sk_gx_stage_bytes(N, ES)) + r;  // [2][S][M][64], this lane's slot
    auto DPu = [&](int u) { return dlds + (0 * S + u) * M * 64; };
    auto DQu = [&](int u) { return dlds + (1 * S + u) * M * 64; };
    // FP32: lane 0's replayed boundary edges are loaded one segment ahead,
    // and lane 0's outgoing records leave once per block (FP64 has no
    // registers to spare for either).  (Loading the segment's lane state one
    // segment ahead as well costs this kernel a wave per SIMD: 85.8 -> 92.0 ms
    // on 4096 uneven pairs.)
    constexpr bool PF = ES == 4;
    constexpr int QW = sk_adj_qst_words(N, ES);
    static_assert(!PF || (S - 1) * QW <= 64, "staged boundary edges exceed one word per lane");
    const SkLds<unsigned> qst =
        (SkLds<unsigned>)(sk_smem + sk_gx_stage_bytes(N, ES) + 2 * S * M * 64 * ES);  // [S-1][QW]
    const SkLds<unsigned> ost = qst + sk_adj_qst_bytes(N, ES) / 4;                      // [8][GXW]
    for (int64_t q = blockIdx.x; q < a.njobs; q += gridDim.x) {
        const int2 jb = a.jobs[q];
        const SkPairDesc pd = a.desc[jb.x];
        const int s = jb.y;
        const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
        const int ly = g.ly;
        const int nloc = sk_pipe_steps(ly), nckl = nloc / S;
        const int i = s * 64 + r;
        const bool rowok = i < g.lx;
        const bool has_next = s + 1 < g.nstrips;  // lane 63 receives from strip s+1
        const unsigned* rin = a.xb + pd.xb_off + (size_t)((s + 1) & 1) * ly * GXW;
        unsigned* rout = a.xb + pd.xb_off + (size_t)(s & 1) * ly * GXW;
        int* prog = a.progress + pd.pg_off;
        const R* cs = a.cskew + pd.c_off + (int64_t)s * g.Tp * 64;
        R* gs = a.gskew + pd.c_off + (int64_t)s * g.Tp * 64;
        const int64_t rows_left = (int64_t)g.nsteps_pad - (int64_t)s * g.Tp;
        const R* ckb = a.ck + pd.ck_off + (int64_t)s * nckl * 2 * (N + 1) * 64;
        const int32_t* ceb = a.ce + pd.ce_off + (int64_t)s * nckl * (SK_LANES + 1);
        const R gk = a.gK[pd.g_idx];
        const int gexp = a.gKexp ? a.gKexp[pd.g_idx] : 0;
        // column lane 63 reads at local step t, or -1
        auto col63 = [&](int t) -> int {
            const int j = t - 63;
            return (has_next && j >= 0 && j < ly) ? j : -1;
        };
        // count of strip s+1 (columns handed over from the top) that covers
        // the columns of the block of steps b .. b+7
        auto need_of = [&](int b) -> int {
            const int lo = b - 63, hi = b + 7 - 63;
            if (!has_next || hi < 0 || lo >= ly) return 0;
            return ly - (lo < 0 ? 0 : lo);
        };
        R lp[N + 1], lqs[N + 1];
#pragma unroll
        for (int n = 0; n <= N; ++n) {
            lp[n] = (R)0;
            lqs[n] = (R)0;
        }
        int El = SK_ZERO_EXP, Els = SK_ZERO_EXP;
        unsigned xr[XR];
#pragma unroll
        for (int h = 0; h < XR; ++h) xr[h] = 0u;
        // a checkpoint sweep that gave up left incomplete checkpoints: no replay
        bool ok = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        if (ok) {  // records of the first (topmost) block
            const int nd = need_of(nloc - 8);
            if (nd > 0) {
                ok = sk_wait_count(prog + s + 1, nd, a.abort, a.spin_limit);
                if (ok) {
#pragma unroll
                    for (int h = 0; h < XR; ++h) {
                        const int w = r + 64 * h;
                        if (w < 8 * GXW) {
                            const int m = w / GXW, qw = w - m * GXW;
                            const int col = col63(nloc - 8 + m);
                            if (col >= 0)
                                xr[h] = __hip_atomic_load(rin + (int64_t)col * GXW + qw, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
            }
        }
        // inputs of replayed step u (column j of this lane): as in the
        // batched adjoint, with the strip's own first column and boundary
        auto replay_in = [&](int u, int j, R (&P)[N + 1], const R (&Qs)[N + 1], R (&Qin)[N + 1],
                             int& E, int Es) -> bool {
            const bool live = rowok && j >= 0 && j < ly;
            if (u == 0) {
#pragma unroll
                for (int n = 0; n <= N; ++n) Qin[n] = Qs[n];
                return live;
            }
#pragma unroll
            for (int n = 0; n <= N; ++n) Qin[n] = lane_from_prev(Qs[n]);
            int Ein = lane_from_prev(Es);
            if (live) {
                if (j == 0) {
#pragma unroll
                    for (int n = 0; n <= N; ++n) P[n] = n == 0 ? (R)1 : (R)0;
                    E = 0;
                }
                if (r == 0) {
                    if (s == 0) {
#pragma unroll
                        for (int n = 0; n <= N; ++n) Qin[n] = n == 0 ? (R)1 : (R)0;
                        Ein = 0;
                    } else if (PF) {
                        const SkLds<unsigned> qq = qst + (u - 1) * QW;
#pragma unroll
                        for (int n = 0; n <= N; ++n) Qin[n] = ((SkLds<R>)qq)[n];
                        Ein = (int)qq[QW - 1];
                    } else {
                        const int64_t o = (int64_t)s * ly + j;
#pragma unroll
                        for (int n = 0; n <= N; ++n) Qin[n] = a.qb[pd.qb_off + o * (N + 1) + n];
                        Ein = a.qe[pd.qe_off + o];
                    }
                }
                const int Ec = E > Ein ? E : Ein;
                const int dp = E - Ec, dq = Ein - Ec;
                if (sk_wave_any(dp != 0 || dq != 0)) {
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        P[n] = sk_ldexp(P[n], dp);
                        Qin[n] = sk_ldexp(Qin[n], dq);
                    }
                }
                E = Ec;
            }
            return live;
        };
        // one adjoint step at local step t (column jj of this lane)
        auto adj_step = [&](int t, bool live, int jj, int Eu, auto&& cell) {
            const bool last_row = (i == g.lx - 1), last_col = (jj == ly - 1);
            R lq_recv[N + 1];
#pragma unroll
            for (int n = 0; n <= N; ++n) lq_recv[n] = lane_from_next(lqs[n]);
            int El_recv = lane_from_next(Els);
            if (r == 63 && live && !last_row) {  // from strip s+1's lane 0
                const unsigned* rec = stage + (t & 7) * GXW;
#pragma unroll
                for (int n = 0; n <= N; ++n) lq_recv[n] = *reinterpret_cast<const R*>(rec + n * (ES / 4));
                El_recv = (int)rec[(N + 1) * (ES / 4)];
            }
            const bool ta = live && !last_col, tb = live && !last_row;
            R ap[N + 1], aq[N + 1];
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                ap[n] = lp[n];
                aq[n] = lq_recv[n];
            }
            int ea = El, eb = El_recv;
            if (sk_wave_any(!(ta && tb))) {  // selects only on steps that need them
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    ap[n] = ta ? ap[n] : (R)0;
                    aq[n] = tb ? aq[n] : (R)0;
                }
                ea = ta ? ea : SK_ZERO_EXP;
                eb = tb ? eb : SK_ZERO_EXP;
            }
            const bool seed = live && last_col && last_row;
            if (sk_wave_any(seed) && seed) {
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    ap[n] = (R)0.5 * gk * ifact<R>(n);
                    aq[n] = ap[n];
                }
                ea = gexp;
                eb = gexp;
            }
            const int Ec = ea > eb ? ea : eb;
            const bool sa = ea != Ec && ea != SK_ZERO_EXP, sb = eb != Ec && eb != SK_ZERO_EXP;
            if (sk_wave_any(sa || sb)) {
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    ap[n] = sk_ldexp(ap[n], ea - Ec);
                    aq[n] = sk_ldexp(aq[n], eb - Ec);
                }
            }
            R gv;
            cell(ap, aq, gv);
            El = Ec;
            Els = Ec;
            if (live && r == 0 && s > 0) {  // to strip s-1's lane 63
                if (PF) {  // (leaves with the block)
                    const SkLds<unsigned> rec = ost + (t & 7) * GXW;
#pragma unroll
                    for (int n = 0; n <= N; ++n) *(SkLds<R>)(rec + n * (ES / 4)) = lqs[n];
                    rec[RW - 1] = (unsigned)Ec;
                } else {
                    unsigned wd[RW];
#pragma unroll
                    for (int n = 0; n <= N; ++n) *reinterpret_cast<R*>(wd + n * (ES / 4)) = lqs[n];
                    wd[RW - 1] = (unsigned)Ec;
                    unsigned* rec = rout + (int64_t)jj * GXW;
#pragma unroll
                    for (int k = 0; k < RW; ++k) sk_store_coherent(rec + k, wd[k]);
                }
            }
            if (live) gs[(int64_t)t * 64 + r] = sk_ldexp(gv, Ec + Eu);
            if ((t & 7) == 0 && live) {
                R m = (R)0;
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    R x1 = sk_abs(lp[n]), x2 = sk_abs(lqs[n]);
                    m = x1 > m ? x1 : m;
                    m = x2 > m ? x2 : m;
                }
                const int sh = sk_rescale_shift<R>(m);
                if (sh != 0) {
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        lp[n] = sk_ldexp(lp[n], -sh);
                        lqs[n] = sk_ldexp(lqs[n], -sh);
                    }
                    El += sh;
                    Els = El;
                }
            }
        };
        // word r of the boundary edges lane 0 replays at steps 1..S-1 of
        // segment kk (strips >= 1), loaded one segment ahead of its use
        auto load_q = [&](int kk) -> unsigned {
            unsigned v = 0u;
            if (PF && s > 0 && r < (S - 1) * QW) {
                const int u = 1 + r / QW, w = r - (u - 1) * QW, j = kk * S + u;
                if (j < ly) {
                    const int64_t o = (int64_t)s * ly + j;
                    if (w < (N + 1) * (ES / 4))
                        v = reinterpret_cast<const unsigned*>(a.qb + pd.qb_off + o * (N + 1))[w];
                    else if (w == QW - 1)
                        v = (unsigned)a.qe[pd.qe_off + o];
                }
            }
            return v;
        };
        unsigned pq = load_q(nckl - 1);
        int published = 0;
        for (int kk = nckl - 1; ok && kk >= 0; --kk) {
            const int t0 = kk * S;
            if (has_next && ((t0 + S) & 7) == 0) {  // a block b = t0 + S - 8 starts
                const int b = t0 + S - 8;
                const int nd = need_of(b - 8);
                if (nd > 0) {
                    ok = sk_wait_count(prog + s + 1, nd, a.abort, a.spin_limit);
                    if (!ok) break;
                }
                sk_gx_stage<GXW, true>(xr, stage, rin, b - 8, r, col63);
            }
            // this segment's staged edges (the wave's own reads of the previous
            // segment's are ordered before), then the next segment's loads
            if (PF && r < (S - 1) * QW) qst[r] = pq;
            if (PF && kk > 0) pq = load_q(kk - 1);
            const R* ck = ckb + (int64_t)kk * 2 * (N + 1) * 64;
            const int E0 = ceb[(int64_t)kk * (SK_LANES + 1) + r];
            const unsigned tword =
                TMAX > 0 ? (unsigned)__builtin_amdgcn_readfirstlane(ceb[(int64_t)kk * (SK_LANES + 1) + SK_LANES])
                         : 0u;
            unsigned tseg = 0u;  // longest tail of the segment (wave-uniform)
#pragma unroll
            for (int u = 0; u < S; ++u) {
                const unsigned tu = (tword >> (8 * u)) & 0xffu;
                tseg = tu > tseg ? tu : tseg;
            }
            if (TMAX == 0 || tseg <= (unsigned)TR) {
                R cseg[S];
#pragma unroll
                for (int u = 0; u < S; ++u)
                    cseg[u] = (t0 + u < rows_left) ? cs[(int64_t)(t0 + u) * 64 + r] : (R)0;
                // ---- replay the segment's forward from the checkpoint
                int Tst[S], Est[S], jst[S];
                bool lv[S];
                int E = E0;
                R P[N + 1], Qs[N + 1];
#pragma unroll
                for (int n = 0; n <= N; ++n) {
                    P[n] = ck[n * 64 + r];
                    Qs[n] = ck[(N + 1 + n) * 64 + r];
                }
                int Es = E;
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    R Qin[N + 1];
                    const int j = t0 + u - r;
                    const bool live = replay_in(u, j, P, Qs, Qin, E, Es);
                    lv[u] = live;
                    jst[u] = j;
                    Est[u] = E;
                    R Po[N + 1], Qo[N + 1];
                    double Po0, Po1, Qo0, Qo1;
                    Tst[u] = (int)((tword >> (8 * u)) & 0xffu);
                    sk_cell_fwd<R, N, TR, true, false, true, 64>(P, Qin, 0.0, 0.0, 0.0, 0.0, cseg[u],
                                                                 live, a.tab, Po, Qo, Po0, Po1, Qo0, Qo1,
                                                                 DPu(u), DQu(u), nullptr, Tst[u]);
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        P[n] = Po[n];
                        Qs[n] = Qo[n];
                    }
                    Es = E;
                }
                // ---- adjoint steps in reverse
#pragma unroll
                for (int u = S - 1; u >= 0; --u)
                    adj_step(t0 + u, lv[u], jst[u], Est[u], [&](R (&ap)[N + 1], R (&aq)[N + 1], R& gv) {
                        sk_cell_adj<R, N, TR, 64>(cseg[u], Tst[u], a.tab, ap, aq, DPu(u), DQu(u), lp,
                                                  lqs, gv);
                    });
            } else {
                // ---- slow path (a tail longer than TR rows in this segment):
                // replay steps 0..u-1 for each step u, from the last, and take
                // the adjoint step with derivatives from the cell's inputs
#pragma unroll 1
                for (int u = S - 1; u >= 0; --u) {
                    int E = E0;
                    R P[N + 1], Qs[N + 1], Qin[N + 1];
#pragma unroll
                    for (int n = 0; n <= N; ++n) {
                        P[n] = ck[n * 64 + r];
                        Qs[n] = ck[(N + 1 + n) * 64 + r];
                    }
                    int Es = E;
                    bool live = false;
#pragma unroll 1
                    for (int v = 0;; ++v) {
                        live = replay_in(v, t0 + v - r, P, Qs, Qin, E, Es);
                        if (v == u) break;
                        R Po[N + 1], Qo[N + 1];
                        double Po0, Po1, Qo0, Qo1;
                        const int Tv = (int)((tword >> (8 * v)) & 0xffu);
                        const R cv = (t0 + v < rows_left) ? cs[(int64_t)(t0 + v) * 64 + r] : (R)0;
                        sk_cell_fwd<R, N, TMAX, false, false, true>(P, Qin, 0.0, 0.0, 0.0, 0.0, cv, live,
                                                                    a.tab, Po, Qo, Po0, Po1, Qo0, Qo1,
                                                                    nullptr, nullptr, nullptr, Tv);
#pragma unroll
                        for (int n = 0; n <= N; ++n) {
                            P[n] = Po[n];
                            Qs[n] = Qo[n];
                        }
                        Es = E;
                    }
                    const int Tu = (int)((tword >> (8 * u)) & 0xffu);
                    const R cu = (t0 + u < rows_left) ? cs[(int64_t)(t0 + u) * 64 + r] : (R)0;
                    adj_step(t0 + u, live, t0 + u - r, E, [&](R (&ap)[N + 1], R (&aq)[N + 1], R& gv) {
                        sk_cell_adj_in<R, N, TMAX>(cu, Tu, a.tab, ap, aq, P, Qin, lp, lqs, gv);
                    });
                }
            }
            // lane 0 has handed over the columns j >= t0: its records of the
            // block's steps t0..t0+7 (column t at step t) go to strip s-1's
            // slot in one pass of all lanes, then the count is published once
            // the stores have completed
            if (s > 0 && (t0 & 7) == 0) {
#pragma unroll
                for (int h = 0; h < (PF ? XR : 0); ++h) {
                    const int w = r + 64 * h, m = w / GXW, qw = w - m * GXW, jc = t0 + m;
                    if (w < 8 * GXW && qw < RW && jc < ly)
                        sk_store_coherent(rout + (int64_t)jc * GXW + qw, ost[w]);
                }
                int done = ly - t0;
                done = done < 0 ? 0 : (done > ly ? ly : done);
                if (done > published) {
                    sk_stores_complete();
                    if (r == 0) sk_store_coherent(reinterpret_cast<unsigned*>(prog + s), (unsigned)done);
                    published = done;
                }
            }
        }
        if (!ok) {  // a wait gave up: the pair's gradient is unknown
            if (rowok) gs[(int64_t)r * 64 + r] = (R)NAN;
        }
    }
}

// With the row derivatives in LDS every order fits two waves per SIMD (the
// derivatives' LDS allows no more); FP64 interpolation at N = 8 spills 120
// bytes per lane there.
template <typename R, int N, int TMAX, int S>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_adjoint_pipe(const AdjPipeArgs<R> a) {
    sk_adjoint_pipe_body<R, N, TMAX, S>(a);
}

// ---------------------------------------------------------------------------
// (e) gradient contraction: dL/dc -> dL/d(dx), dL/d(dy) per pair
// ---------------------------------------------------------------------------
template <typename R>
struct ContractArgs {
    const R* X;
    const R* Y;
    int64_t d;
    SkPairSrc src;
    const R* gskew;
    R* dxp;   // [pair][lx][d]
    R* dyp;   // [pair][strip][ly][d]
};

// One wave per (pair, strip, 16-dimension slice): lane r accumulates
// dL/d(dx_i) over the slice's dimensions for its row i = 64 s + r in
// registers (slices keep the register count at four waves per SIMD).  dL/d(dy_j) for the strip is a sum down the
// column j, whose cells lanes r = 0..63 visit at consecutive steps; the
// partial sum therefore travels with the wavefront (lane r-1 -> lane r, one
// DPP move per step) and the strip's last row writes it out.  The y
// increments sit in an LDS ring of 128 columns (column j in row j mod 128):
// at step t the lanes read columns t-63 .. t, and every 8 steps the next 8
// columns, loaded one block ahead, replace columns that no lane reads again.
// Rows of dL/dc are prefetched eight steps ahead.
template <typename R, int DMAX>
__global__ __launch_bounds__(64) void k_contract(const ContractArgs<R> a) {
    const int r = threadIdx.x;
    const int s = blockIdx.y;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    if (g.nsteps == 0 || s >= g.nstrips) return;
    constexpr int YS = sk_ring_ys<R, DMAX>();
    constexpr int NV = (8 * DMAX + 63) / 64;  // ring values per lane per 8 columns
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* ring = reinterpret_cast<R*>(sk_smem);  // [128][YS]
    const int64_t k0 = (int64_t)blockIdx.z * DMAX;  // first dimension of the slice
    const int64_t d = a.d - k0 < DMAX ? a.d - k0 : DMAX;  // dimensions of the slice
    const int64_t ld = a.d;
    const int ly = g.ly;
    const R* X = (pd.swap ? a.Y : a.X) + pd.x_off * ld + k0;
    const R* Y = (pd.swap ? a.X : a.Y) + pd.y_off * ld + k0;
    const R* gsk = a.gskew + pd.c_off + (int64_t)s * g.Tp * 64;
    const int i = s * 64 + r;
    const bool rowok = i < g.lx;
    const int last_r = (g.lx - 1 - s * 64) < 63 ? (g.lx - 1 - s * 64) : 63;
    const int nt = ly + last_r;  // local steps: the last row reaches column ly-1 at ly-1+last_r
    R xi[DMAX], accx[DMAX], accy[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        xi[k] = (R)0;
        accx[k] = (R)0;
        accy[k] = (R)0;
        if (k < d && rowok) xi[k] = X[(int64_t)(i + 1) * ld + k] - X[(int64_t)i * ld + k];
    }
    // y increments of the 8 columns from c0: value w is column c0 + w / DMAX, dimension w % DMAX
    R yv[NV];
    auto load_y = [&](int c0) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
            const int w = r + 64 * h, m = w / DMAX, k = w - m * DMAX, c = c0 + m;
            yv[h] = (R)0;
            if (w < 8 * DMAX && k < d && c < ly)
                yv[h] = Y[(int64_t)(c + 1) * ld + k] - Y[(int64_t)c * ld + k];
        }
    };
    auto store_y = [&](int c0) {
#pragma unroll
        for (int h = 0; h < NV; ++h) {
            const int w = r + 64 * h, m = w / DMAX, k = w - m * DMAX;
            if (w < 8 * DMAX) ring[((c0 + m) & 127) * YS + k] = yv[h];
        }
    };
    load_y(0);
    R gb[8], gn[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) gb[u] = u < nt ? gsk[(int64_t)u * 64 + r] : (R)0;
    for (int t0 = 0; t0 < nt; t0 += 8) {
        // columns t0 .. t0+7 into the ring (their rows held columns t0-128 ..
        // t0-121, which no lane reads again), then the next block's loads
        store_y(t0);
        __syncthreads();
        load_y(t0 + 8);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + 8 + u;
            gn[u] = t < nt ? gsk[(int64_t)t * 64 + r] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0 + u, j = t - r;
            // lane 0 receives zero (the DPP shift fills it), which starts the
            // column's sum
#pragma unroll
            for (int k = 0; k < DMAX; ++k) accy[k] = lane_from_prev(accy[k]);
            const bool ok = rowok && j >= 0 && j < ly && t < nt;
            // cells outside the strip contribute zero (no branch)
            const R gv = ok ? gb[u] : (R)0;
            const R* yj = ring + ((ok ? j : 0) & 127) * YS;
#pragma unroll
            for (int k = 0; k < DMAX; ++k) {
                accx[k] = fma(gv, yj[k], accx[k]);
                accy[k] = fma(gv, xi[k], accy[k]);
            }
            if (ok && r == last_r) {
                R* dyo = a.dyp + pd.dy_off + ((int64_t)s * ly + j) * ld + k0;
#pragma unroll
                for (int k = 0; k < DMAX; ++k)
                    if (k < d) dyo[k] = accy[k];
            }
            // keep each step's ring reads in its step (hoisting them holds
            // 8 * DMAX values in registers and halves the occupancy)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) gb[u] = gn[u];
    }
    if (rowok) {
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
            if (k < d) a.dxp[pd.dx_off + (int64_t)i * ld + k0 + k] = accx[k];
    }
}

// The same contraction on 16x16x4 MFMA tiles (FP32), for d up to 16 DB: it
// is two matrix products per (pair, strip), dL/d(dx) (64 x d) += G (64 x ly)
// dY (ly x d) and the strip's partial dL/d(dy) (ly x d) = G^T dX, with K = ly
// and 64 respectively.  One workgroup (4 waves) per (pair, strip) walks the
// columns in tiles of 64: the skewed rows of dL/dc are un-skewed into an LDS
// ring G[64][128] by column (each skewed row is read once, coalesced; a tile
// needs rows up to 63 past its last column, so the ring holds the tile and the
// next one's leading part), and the tile's y increments into LDS; the next
// tile's rows and increments load into registers during the current tile's
// MFMAs.  The x increments, the B operand of every tile's G^T dX, stay in
// registers, which keeps the LDS of a workgroup under 40 KiB: four
// workgroups per CU at d <= 16 (1.97 -> 1.64 ms on 128 x 128 Gram pairs of
// 256 steps in R^8; two chunks of rows in flight per wave, at two waves per
// SIMD, took 2.42 ms).  Wave w owns rows 16w..16w+15 of dL/d(dx)
// (accumulated in registers over the tiles) and columns 16w..16w+15 of each
// tile's dL/d(dy).
#define SK_CMFMA_GS 132  // LDS row stride of the ring (2-way conflicts at most)
template <int DB>
__host__ __device__ constexpr int sk_cmfma_ds() { return 16 * DB + 4; }  // stride of dY rows
template <int DB>
__host__ __device__ constexpr int sk_cmfma_lds() {
    return (64 * SK_CMFMA_GS + 64 * sk_cmfma_ds<DB>()) * 4;
}

template <int DB>
__global__ __launch_bounds__(256) void k_contract_mfma(const ContractArgs<float> a) {
    // (a scalar wave index, which makes the row loads' conditions scalar
    // branches, is slower: 2.05 against 1.64 ms on 128 x 128 Gram pairs)
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int s = blockIdx.y;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    if (g.nsteps == 0 || s >= g.nstrips) return;
    constexpr int DS = sk_cmfma_ds<DB>();
    extern __shared__ __align__(16) unsigned char sk_smem[];
    SkLds<float> G = (SkLds<float>)sk_smem;                 // [64][GS], column c at c & 127
    SkLds<float> Yt = G + 64 * SK_CMFMA_GS;                 // [64][DS]: y increments of the tile
    const int64_t ld = a.d;
    const int d = (int)a.d, ly = g.ly;
    const float* X = (pd.swap ? a.Y : a.X) + pd.x_off * ld;
    const float* Y = (pd.swap ? a.X : a.Y) + pd.y_off * ld;
    const int64_t tau0 = (int64_t)s * g.Tp;                  // skewed row of the strip's (0, 0)
    const float* gsk = a.gskew + pd.c_off + tau0 * 64;
    const int64_t rows_left = (int64_t)g.nsteps_pad - tau0;  // skewed rows of the pair from tau0
    const int nrow = g.lx - s * 64 < 64 ? g.lx - s * 64 : 64;
    const int ntiles = (ly + 63) / 64;
    // chunk c of skewed rows: rows 0..62 for c = -1 (the columns of tile 0
    // that rows below 63 hold), rows 64c + 63 .. 64c + 126 for c >= 0 (the
    // rest of tile c and the leading part of tile c + 1).  Lane `lane` of
    // wave w holds rows t0 + w + 4u, u < 16.
    auto load_rows = [&](float (&rows)[16], int c) {
        const int t0n = c < 0 ? 0 : 64 * c + 63, count = c < 0 ? 63 : (c < ntiles ? 64 : 0);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = t0n + w + 4 * u;
            rows[u] = (4 * u + w < count && t < rows_left) ? sk_ld_nt(gsk + (int64_t)t * 64 + lane) : 0.0f;
        }
    };
    auto store_rows = [&](const float (&rows)[16], int c) {
        const int t0n = c < 0 ? 0 : 64 * c + 63, count = c < 0 ? 63 : 64;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = t0n + w + 4 * u, j = t - lane;
            // only the strip's cells: past the strip's rows and the pair's
            // last step the skewed slots are not this strip's
            if (4 * u + w < count && lane < nrow && j >= 0 && j < ly)
                G[lane * SK_CMFMA_GS + (j & 127)] = rows[u];
        }
    };
    constexpr int YH = (64 * 16 * DB + 255) / 256;
    float yr[YH];
    auto load_y = [&](int j0) {
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int e = tid + 256 * h, jj = e / (16 * DB), k = e - jj * (16 * DB), j = j0 + jj;
            yr[h] = (e < 64 * 16 * DB && k < d && j < ly)
                        ? Y[(int64_t)(j + 1) * ld + k] - Y[(int64_t)j * ld + k] : 0.0f;
        }
    };
    auto store_y = [&]() {
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int e = tid + 256 * h, jj = e / (16 * DB), k = e - jj * (16 * DB);
            if (e < 64 * 16 * DB) Yt[jj * DS + k] = yr[h];
        }
    };
    // clear the ring once: rows past the strip's last row stay zero, and
    // columns j >= ly of the last tile keep earlier tiles' values, which meet
    // zero y increments.  The x increments of the strip's rows (zero past its
    // last row and past d) pass through the tile's y area into registers:
    // xb[b][q] is B[4q + lane / 16][lane % 16] of the q-th k-step of column
    // block b.
    for (int e = tid; e < 64 * SK_CMFMA_GS; e += 256) G[e] = 0.0f;
    for (int e = tid; e < 64 * 16 * DB; e += 256) {
        const int rr = e / (16 * DB), k = e - rr * (16 * DB);
        float v = 0.0f;
        if (rr < nrow && k < d) {
            const int64_t i = (int64_t)s * 64 + rr;
            v = X[(i + 1) * ld + k] - X[i * ld + k];
        }
        Yt[rr * DS + k] = v;
    }
    float gr[16];
    load_rows(gr, -1);
    __syncthreads();
    float xb[DB][16];
#pragma unroll
    for (int b = 0; b < DB; ++b)
#pragma unroll
        for (int q = 0; q < 16; ++q) xb[b][q] = Yt[(4 * q + (lane >> 4)) * DS + 16 * b + (lane & 15)];
    store_rows(gr, -1);
    load_rows(gr, 0);
    load_y(0);
    __syncthreads();  // the x increments are read before tile 0's y increments replace them
    sk_f4 accx[DB];
#pragma unroll
    for (int b = 0; b < DB; ++b) accx[b] = {0.0f, 0.0f, 0.0f, 0.0f};
    // tile jt: its chunk is in cur, which is then refilled with chunk jt + 1
    auto tile = [&](int jt, float (&cur)[16]) {
        // the tile's columns sit at cb .. cb + 63 of the ring, without wrapping
        const int j0 = 64 * jt, cb = j0 & 127;
        store_rows(cur, jt);
        store_y();
        __syncthreads();
        if (jt + 1 < ntiles) {
            load_y(j0 + 64);
            load_rows(cur, jt + 1);
        }
        // dL/d(dx)[16w + m][n] += sum_k G[16w + m][j0 + k] dY[k][n]
#pragma unroll
        for (int kk = 0; kk < 64; kk += 4) {
            const float av = G[(16 * w + (lane & 15)) * SK_CMFMA_GS + cb + kk + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < DB; ++b) {
                const float bv = Yt[(kk + (lane >> 4)) * DS + 16 * b + (lane & 15)];
                accx[b] = SkMfma<float>::mma(av, bv, accx[b]);
            }
        }
        // the strip's dL/d(dy)[j0 + 16w + m][n] = sum_k G[k][j0 + 16w + m] dX[k][n]
        sk_f4 accy[DB];
#pragma unroll
        for (int b = 0; b < DB; ++b) accy[b] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const float av = G[(4 * q + (lane >> 4)) * SK_CMFMA_GS + cb + 16 * w + (lane & 15)];
#pragma unroll
            for (int b = 0; b < DB; ++b) accy[b] = SkMfma<float>::mma(av, xb[b][q], accy[b]);
        }
#pragma unroll
        for (int b = 0; b < DB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + 16 * w + SkMfma<float>::row(lane, v), k = 16 * b + (lane & 15);
                if (j < ly && k < d) a.dyp[pd.dy_off + ((int64_t)s * ly + j) * ld + k] = accy[b][v];
            }
        __syncthreads();  // the ring's and the tile's next contents are stored after this
    };
    for (int jt = 0; jt < ntiles; ++jt) tile(jt, gr);
#pragma unroll
    for (int b = 0; b < DB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 16 * w + SkMfma<float>::row(lane, v), k = 16 * b + (lane & 15);
            if (rr < nrow && k < d) a.dxp[pd.dx_off + ((int64_t)s * 64 + rr) * ld + k] = accx[b][v];
        }
}

// FP64 version of the MFMA contraction (16x16x4 FP64 tiles), for d up to
// 16 DB.  FP64 doubles the bytes of every LDS operand, so the column tiles
// are 32 wide and the ring holds 96 columns (a tile and the 63 columns past
// it that its rows also hold), which keeps a workgroup under 64 KiB; the x
// increments, the B operand of G^T dX, stay in registers.  Wave w owns rows
// 16w..16w+15 of dL/d(dx) and, of each tile's 32 x 16 DB block of dL/d(dy),
// the 16 columns (w & 1) and the dimension block w >> 1 (waves whose block is
// past DB take no part in that product).
#define SK_CMFMA64_RC 96   // ring columns
#define SK_CMFMA64_GS 100  // LDS row stride of the ring, in doubles
template <int DB>
__host__ __device__ constexpr int sk_cmfma64_ds() { return 16 * DB + 2; }  // stride of dY rows
template <int DB>
__host__ __device__ constexpr int sk_cmfma64_lds() {
    return (64 * SK_CMFMA64_GS + 32 * sk_cmfma64_ds<DB>()) * 8;
}

template <int DB>
__global__ __launch_bounds__(256) void k_contract_mfma_f64(const ContractArgs<double> a) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int s = blockIdx.y;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    if (g.nsteps == 0 || s >= g.nstrips) return;
    constexpr int TW = 32, RC = SK_CMFMA64_RC, GS = SK_CMFMA64_GS, DS = sk_cmfma64_ds<DB>();
    extern __shared__ __align__(16) unsigned char sk_smem[];
    SkLds<double> G = (SkLds<double>)sk_smem;  // [64][GS], column c at c % RC
    SkLds<double> Yt = G + 64 * GS;            // [TW][DS]: y increments of the tile
    const int64_t ld = a.d;
    const int d = (int)a.d, ly = g.ly;
    const double* X = (pd.swap ? a.Y : a.X) + pd.x_off * ld;
    const double* Y = (pd.swap ? a.X : a.Y) + pd.y_off * ld;
    const int64_t tau0 = (int64_t)s * g.Tp;                  // skewed row of the strip's (0, 0)
    const double* gsk = a.gskew + pd.c_off + tau0 * 64;
    const int64_t rows_left = (int64_t)g.nsteps_pad - tau0;  // skewed rows of the pair from tau0
    const int nrow = g.lx - s * 64 < 64 ? g.lx - s * 64 : 64;
    const int ntiles = (ly + TW - 1) / TW;
    const int bb = w >> 1;  // this wave's dimension block of dL/d(dy)
    // x increments of the strip's rows (zero past the last row and past d),
    // staged through the ring's space: xb[q] = B[4q + lane / 16][lane % 16]
    // of the q-th k-step of dimension block bb
    for (int e = tid; e < 64 * 16 * DB; e += 256) {
        const int rr = e / (16 * DB), k = e - rr * (16 * DB);
        double v = 0.0;
        if (rr < nrow && k < d) {
            const int64_t i = (int64_t)s * 64 + rr;
            v = X[(i + 1) * ld + k] - X[i * ld + k];
        }
        G[rr * DS + k] = v;
    }
    __syncthreads();
    double xb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        xb[q] = bb < DB ? G[(4 * q + (lane >> 4)) * DS + 16 * bb + (lane & 15)] : 0.0;
    __syncthreads();
    // clear the ring once: rows past the strip's last row stay zero, and
    // columns j >= ly of the last tile keep earlier tiles' values, which meet
    // zero y increments
    for (int e = tid; e < 64 * GS; e += 256) G[e] = 0.0;
    // skewed rows t0n + w + 4u (u < 8) at this lane
    double gr[8];
    auto load_rows = [&](int t0n, int count) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0n + w + 4 * u;
            gr[u] = (4 * u + w < count && t < rows_left) ? sk_ld_nt(gsk + (int64_t)t * 64 + lane) : 0.0;
        }
    };
    auto store_rows = [&](int t0n, int count) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = t0n + w + 4 * u, j = t - lane;
            // only the strip's cells: past the strip's rows and the pair's
            // last step the skewed slots are not this strip's
            if (4 * u + w < count && lane < nrow && j >= 0 && j < ly) G[lane * GS + j % RC] = gr[u];
        }
    };
    constexpr int YH = (TW * 16 * DB + 255) / 256;
    double yr[YH];
    auto load_y = [&](int j0) {
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int e = tid + 256 * h, jj = e / (16 * DB), k = e - jj * (16 * DB), j = j0 + jj;
            yr[h] = (e < TW * 16 * DB && k < d && j < ly)
                        ? Y[(int64_t)(j + 1) * ld + k] - Y[(int64_t)j * ld + k] : 0.0;
        }
    };
    auto store_y = [&]() {
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int e = tid + 256 * h, jj = e / (16 * DB), k = e - jj * (16 * DB);
            if (e < TW * 16 * DB) Yt[jj * DS + k] = yr[h];
        }
    };
    __syncthreads();
    // prologue: skewed rows 0..62 (the columns of tile 0 that rows below 63 hold)
    load_rows(0, 32);
    store_rows(0, 32);
    load_rows(32, 31);
    store_rows(32, 31);
    // chunk of tile jt: skewed rows TW jt + 63 .. TW jt + 62 + TW (the rest of
    // tile jt and the leading part of the next tiles)
    load_rows(63, TW);
    load_y(0);
    sk_d4 accx[DB];
#pragma unroll
    for (int b = 0; b < DB; ++b) accx[b] = {0.0, 0.0, 0.0, 0.0};
    for (int jt = 0; jt < ntiles; ++jt) {
        // the tile's columns sit at cb .. cb + TW - 1 of the ring, without wrapping
        const int j0 = TW * jt, cb = j0 % RC;
        store_rows(j0 + 63, TW);
        store_y();
        __syncthreads();
        if (jt + 1 < ntiles) {  // the next tile's rows and increments load under the MFMAs
            load_y(j0 + TW);
            load_rows(j0 + TW + 63, TW);
        }
        // dL/d(dx)[16w + m][n] += sum_k G[16w + m][j0 + k] dY[k][n]
#pragma unroll
        for (int kk = 0; kk < TW; kk += 4) {
            const double av = G[(16 * w + (lane & 15)) * GS + cb + kk + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < DB; ++b) {
                const double bv = Yt[(kk + (lane >> 4)) * DS + 16 * b + (lane & 15)];
                accx[b] = SkMfma<double>::mma(av, bv, accx[b]);
            }
        }
        // the strip's dL/d(dy)[j0 + 16 (w & 1) + m][16 bb + n] = sum_k G[k][j0 + 16 (w & 1) + m] dX[k][16 bb + n]
        if (bb < DB) {
            sk_d4 accy = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const double av = G[(4 * q + (lane >> 4)) * GS + cb + 16 * (w & 1) + (lane & 15)];
                accy = SkMfma<double>::mma(av, xb[q], accy);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + 16 * (w & 1) + SkMfma<double>::row(lane, v), k = 16 * bb + (lane & 15);
                if (j < ly && k < d) a.dyp[pd.dy_off + ((int64_t)s * ly + j) * ld + k] = accy[v];
            }
        }
        __syncthreads();  // the ring's and the tile's next contents are stored after this
    }
#pragma unroll
    for (int b = 0; b < DB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 16 * w + SkMfma<double>::row(lane, v), k = 16 * b + (lane & 15);
            if (rr < nrow && k < d) a.dxp[pd.dx_off + ((int64_t)s * 64 + rr) * ld + k] = accx[b][v];
        }
}

// Hybrid scheme backward: every sub-cell of cell (i, j) on the lam-order
// refinement has the constant c_ij / 4^lam, so dL/dc_ij is 4^-lam times the
// sum of dL/dc' over its 4^lam sub-cells.  One thread per element (tau, r)
// of the unrefined grid's skewed layout (cell (64 s + r, j) with
// tau - r = s Tp + j, as the sweeps lay it out) gathers its sub-cells from
// the refined grid's skewed layout; idle slots get zero.  The contraction
// and the reductions then run on the unrefined grid.
template <typename R>
struct FoldArgs {
    SkPairSrc src;
    int32_t lam;
    const R* gref;  // refined skewed dL/dc', at each pair's c_off
    R* gout;        // unrefined skewed dL/dc, at each pair's c_off
};

template <typename R>
__global__ __launch_bounds__(256) void k_fold_refined(const FoldArgs<R> a) {
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    const SkGeom gr = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) return;
    const int64_t ne = (int64_t)g.nsteps_pad * SK_LANES;
    for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < ne; e += (int64_t)gridDim.y * 256) {
        const int tau = (int)(e >> 6), r = (int)(e & 63), L = tau - r;
        R sum = (R)0;
        if (L >= 0) {
            const int s = L / g.Tp, j = L - s * g.Tp, i = 64 * s + r;
            if (i < g.lx && j < g.ly) {
                const int n = 1 << a.lam;
                for (int u = 0; u < n; ++u) {
                    const int ir = i * n + u, sr = ir >> 6, rr = ir & 63;
                    const int64_t base = pd.c_off + ((int64_t)sr * gr.Tp + rr) * SK_LANES + rr;
                    for (int v = 0; v < n; ++v) sum += a.gref[base + (int64_t)(j * n + v) * SK_LANES];
                }
                sum *= (R)1 / (R)(1 << (2 * a.lam));
            }
        }
        a.gout[pd.c_off + e] = sum;
    }
}

// gX[a][t][k] += sum over chunk pairs (a, b) of (dx[t-1][k] - dx[t][k]);
// gY likewise over (a, b) and strips.  Gram mode.
template <typename R>
struct ReduceGramArgs {
    int64_t nx, ny, lx_pts, ly_pts, d;
    int64_t first, count;   // chunk pairs [first, first + count)
    int64_t dx_stride, dy_stride, nstrips;
    const R* dxp;
    const R* dyp;
    R* gX;
    R* gY;
};

// Both reductions: a workgroup of 256 threads owns 64 consecutive output
// elements; its four 64-thread groups sum interleaved quarters of the pairs
// (4x the memory-level parallelism of one thread per element) and combine
// through LDS.
template <typename R>
__device__ __forceinline__ R sk_group4_sum(R v, int tid) {
    __shared__ R part[256];
    part[tid] = v;
    __syncthreads();
    R s = (R)0;
    if (tid < 64) s = (part[tid] + part[tid + 64]) + (part[tid + 128] + part[tid + 192]);
    return s;
}

template <typename R>
__global__ __launch_bounds__(256) void k_reduce_gram_x(const ReduceGramArgs<R> a) {
    const int tid = threadIdx.x, grp = tid >> 6;
    const int64_t lx = a.lx_pts - 1, d = a.d;
    const int64_t a_lo = a.first / a.ny, a_hi = (a.first + a.count - 1) / a.ny;
    const int64_t per = a.lx_pts * d;
    const int64_t e = (int64_t)blockIdx.x * 64 + (tid & 63);
    const bool live = e < (a_hi - a_lo + 1) * per;
    int64_t ai = 0, t = 0, k = 0;
    R sum = (R)0;
    if (live) {
        ai = a_lo + e / per;
        const int64_t rem = e % per;
        t = rem / d;
        k = rem % d;
        int64_t p0 = ai * a.ny, p1 = p0 + a.ny;
        if (p0 < a.first) p0 = a.first;
        if (p1 > a.first + a.count) p1 = a.first + a.count;
#pragma unroll 4
        for (int64_t p = p0 + grp; p < p1; p += 4) {
            const R* dx = a.dxp + (p - a.first) * a.dx_stride;
            R v = (R)0;
            if (t > 0) v += dx[(t - 1) * d + k];
            if (t < lx) v -= dx[t * d + k];
            sum += v;
        }
    }
    sum = sk_group4_sum(sum, tid);
    if (live && tid < 64) a.gX[ai * per + t * d + k] += sum;
}

template <typename R>
__global__ __launch_bounds__(256) void k_reduce_gram_y(const ReduceGramArgs<R> a) {
    const int tid = threadIdx.x, grp = tid >> 6;
    const int64_t ly = a.ly_pts - 1, d = a.d;
    const int64_t per = a.ly_pts * d;
    const int64_t e = (int64_t)blockIdx.x * 64 + (tid & 63);
    const bool live = e < a.ny * per;
    int64_t bi = 0, t = 0, k = 0;
    R sum = (R)0;
    if (live) {
        bi = e / per;
        const int64_t rem = e % per;
        t = rem / d;
        k = rem % d;
        const int64_t a_lo = a.first / a.ny, a_hi = (a.first + a.count - 1) / a.ny;
        for (int64_t ai = a_lo + grp; ai <= a_hi; ai += 4) {
            const int64_t p = ai * a.ny + bi;
            if (p < a.first || p >= a.first + a.count) continue;
            const R* dy = a.dyp + (p - a.first) * a.dy_stride;
#pragma unroll 4
            for (int64_t s = 0; s < a.nstrips; ++s) {
                const R* dys = dy + s * ly * d;
                R v = (R)0;
                if (t > 0) v += dys[(t - 1) * d + k];
                if (t < ly) v -= dys[t * d + k];
                sum += v;
            }
        }
    }
    sum = sk_group4_sum(sum, tid);
    if (live && tid < 64) a.gY[bi * per + t * d + k] += sum;
}

// List mode: every pair owns its own x and y points.
template <typename R>
struct ReducePairsArgs {
    const SkPairDesc* desc;
    int64_t count, d, max_pts;
    const R* dxp;
    const R* dyp;
    R* gX;
    R* gY;
};

template <typename R>
__global__ void k_reduce_pairs(const ReducePairsArgs<R> a) {
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = a.desc[local];
    const int64_t d = a.d;
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
         e < a.max_pts * d; e += (int64_t)gridDim.y * blockDim.x) {
        const int64_t t = e / d, k = e % d;
        if (t <= pd.lx) {
            R v = (R)0;
            if (pd.lx > 0 && pd.ly > 0) {
                const R* dx = a.dxp + pd.dx_off;
                if (t > 0) v += dx[(t - 1) * d + k];
                if (t < pd.lx) v -= dx[t * d + k];
            }
            (pd.swap ? a.gY : a.gX)[(pd.x_off + t) * d + k] = v;
        }
        if (t <= pd.ly) {
            R v = (R)0;
            if (pd.lx > 0 && pd.ly > 0) {
                for (int s = 0; s < g.nstrips; ++s) {
                    const R* dy = a.dyp + pd.dy_off + (int64_t)s * pd.ly * d;
                    if (t > 0) v += dy[(t - 1) * d + k];
                    if (t < pd.ly) v -= dy[t * d + k];
                }
            }
            (pd.swap ? a.gX : a.gY)[(pd.y_off + t) * d + k] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// finite-difference baseline: batched wavefront over the refined grid
// ---------------------------------------------------------------------------
template <typename R>
struct FdArgs {
    SkPairSrc src;
    int32_t lam;
    int32_t second;   // second-order explicit rule (adds the c^2 term)
    const R* cskew;   // skewed refined constants c / 4^lam
    R* K;
    int32_t* Kexp;
};

// Lane r owns refined row i and keeps k(s_{i+1}, t_j); it receives
// k(s_i, t_{j+1}) from lane r-1 and remembers the value received one step
// earlier, k(s_i, t_j).
template <typename R>
__global__ __launch_bounds__(64) void k_sweep_fd(const FdArgs<R> a) {
    const int r = threadIdx.x;
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(a.src, local);
    const SkGeom g = sk_make_geom(pd.lx << a.lam, pd.ly << a.lam);
    if (g.nsteps == 0) {
        if (r == 0) sk_write_k(a.K, a.Kexp, pd.k_idx, (R)1, 0);
        return;
    }
    extern __shared__ __align__(16) unsigned char sk_smem[];
    R* blds = reinterpret_cast<R*>(sk_smem);  // k(s_{64 s}, t_{j+1}) from strip s-1
    const R* cs = a.cskew + pd.c_off;
    R kown = (R)1, bprev = (R)1, out = (R)1;
    int L = -r, s = 0, j = 0;
    for (int tau = 0; tau < g.nsteps; ++tau) {
        R b = lane_from_prev(out);
        const int i = s * 64 + r;
        const bool live = (L >= 0) && (s < g.nstrips) && (j < g.ly) && (i < g.lx);
        const R c = cs[(int64_t)tau * 64 + r];
        if (live) {
            R kij;
            if (j == 0) {
                kown = (R)1;
                kij = (R)1;
            } else {
                kij = bprev;
            }
            if (r == 0) {
                b = (s == 0) ? (R)1 : blds[j];
                kij = (s == 0 || j == 0) ? (R)1 : blds[j - 1];
            }
            out = kown + b - kij + (R)0.5 * c * (kown + b);
            if (a.second) out = fma(c * c * (R)(1.0 / 12.0), kown + b + kij, out);
            kown = out;
            bprev = b;
            if (r == 63 && s + 1 < g.nstrips) blds[j] = out;
            if (i == g.lx - 1 && j == g.ly - 1) sk_write_k(a.K, a.Kexp, pd.k_idx, out, 0);
        }
        if (L >= 0) {
            if (++j == g.Tp) {
                j = 0;
                ++s;
            }
        }
        ++L;
    }
}

// ---------------------------------------------------------------------------
// plain single-pair kernels (one pair per launch, anti-diagonal parallel,
// cell constants computed on the fly, state in workspace memory)
// ---------------------------------------------------------------------------
template <typename R>
struct PlainArgs {
    const R* x;        // points of x
    const R* y;
    int64_t d;
    int32_t lx, ly;    // segments
    int32_t lam;
    int32_t second;    // finite differences: second-order explicit rule
    R* pst;            // polynomial: [lx][N+1] bottom edges, [ly][N+1] left edges
    R* diag;           // finite differences: 3 rotating node diagonals of length lx*2^lam + 1
    SkTab<R> tab;
    R* K;
    int32_t* Kexp;
    int64_t k_idx;
};

template <typename R>
__device__ __forceinline__ R sk_dot_inc(const R* x, const R* y, int64_t d, int i, int j) {
    R acc = (R)0;
    for (int64_t k = 0; k < d; ++k)
        acc = fma(x[(int64_t)(i + 1) * d + k] - x[(int64_t)i * d + k],
                  y[(int64_t)(j + 1) * d + k] - y[(int64_t)j * d + k], acc);
    return acc;
}

template <typename R, int N, int TMAX>
__global__ __launch_bounds__(256) void k_plain_poly(const PlainArgs<R> a) {
    // grid of the lam-order dyadic refinement (lam = 0: the path grid)
    const int lx = a.lx << a.lam, ly = a.ly << a.lam;
    const R sc = (R)1 / (R)((int64_t)1 << (2 * a.lam));
    R* pe = a.pst;                         // p^{i, j}
    R* qe = a.pst + (int64_t)lx * (N + 1); // q^{i, j}
    for (int e = threadIdx.x; e < (lx + ly) * (N + 1); e += blockDim.x)
        a.pst[e] = (e % (N + 1)) == 0 ? (R)1 : (R)0;
    __syncthreads();
    for (int dg = 0; dg <= lx + ly - 2; ++dg) {
        int i_lo = dg - (ly - 1);
        if (i_lo < 0) i_lo = 0;
        const int i_hi = dg < lx - 1 ? dg : lx - 1;
        for (int i = i_lo + threadIdx.x; i <= i_hi; i += blockDim.x) {
            const int j = dg - i;
            const R c = sk_dot_inc(a.x, a.y, a.d, i >> a.lam, j >> a.lam) * sc;
            R P[N + 1], Q[N + 1], Po[N + 1], Qo[N + 1];
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                P[n] = pe[i * (N + 1) + n];
                Q[n] = qe[j * (N + 1) + n];
            }
            double Po0, Po1, Qo0, Qo1;
            sk_cell_fwd<R, N, TMAX>(P, Q, (double)P[0], (double)P[1], (double)Q[0], (double)Q[1], c,
                                    true, a.tab, Po, Qo, Po0, Po1, Qo0, Qo1);
#pragma unroll
            for (int n = 0; n <= N; ++n) {
                pe[i * (N + 1) + n] = Po[n];
                qe[j * (N + 1) + n] = Qo[n];
            }
            if (i == lx - 1 && j == ly - 1) {
                R kv = (R)0;
#pragma unroll
                for (int n = N; n >= 2; --n) kv = fma(Po[n] + Qo[n], ifact<R>(n), kv);
                sk_write_k(a.K, a.Kexp, a.k_idx, 0.5 * (Po0 + Qo0 + Po1 + Qo1 + (double)kv), 0);
            }
        }
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_plain_fd(const PlainArgs<R> a) {
    const int m = a.lx << a.lam, n = a.ly << a.lam;
    const R sc = (R)1 / (R)((int64_t)1 << (2 * a.lam));
    // node (x, y) lies on node diagonal x + y; three rotating diagonals indexed by x
    R* D[3] = {a.diag, a.diag + (m + 1), a.diag + 2 * (m + 1)};
    for (int e = threadIdx.x; e < 3 * (m + 1); e += blockDim.x) a.diag[e] = (R)1;
    __syncthreads();
    for (int dg = 0; dg <= m + n - 2; ++dg) {
        R* d0 = D[dg % 3];        // nodes on diagonal dg
        R* d1 = D[(dg + 1) % 3];  // dg + 1
        R* d2 = D[(dg + 2) % 3];  // dg + 2 (written)
        int i_lo = dg - (n - 1);
        if (i_lo < 0) i_lo = 0;
        const int i_hi = dg < m - 1 ? dg : m - 1;
        for (int i = i_lo + threadIdx.x; i <= i_hi; i += blockDim.x) {
            const int j = dg - i;
            const R c = sk_dot_inc(a.x, a.y, a.d, i >> a.lam, j >> a.lam) * sc;
            const R k00 = d0[i], k10 = d1[i + 1], k01 = d1[i];
            R k11 = k10 + k01 - k00 + (R)0.5 * c * (k10 + k01);
            if (a.second) k11 = fma(c * c * (R)(1.0 / 12.0), k10 + k01 + k00, k11);
            d2[i + 1] = k11;
            if (i == m - 1 && j == n - 1) sk_write_k(a.K, a.Kexp, a.k_idx, k11, 0);
        }
        // boundary nodes (0, dg + 2) and (dg + 2, 0) stay 1
        if (threadIdx.x == 0) d2[0] = (R)1;
        if (threadIdx.x == 0 && dg + 2 <= m) d2[dg + 2] = (R)1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// MMD permutation two-sample test
// ---------------------------------------------------------------------------
// One workgroup per permutation p of the pooled sample (m + n paths): the
// first m entries of perms[p] form the first group.  stats[p] is the
// unbiased MMD^2 of that split, sum over a != b of K[a][b] w(group a, group b)
// with w = 1/(m(m-1)), 1/(n(n-1)) within groups and -1/(mn) across, read
// row-major (coalesced) with the group labels in LDS, accumulated in FP64.
template <typename R>
__global__ __launch_bounds__(256) void k_mmd_perm(const R* K, int64_t m, int64_t n,
                                                  const int32_t* perms, R* stats) {
    const int64_t p = blockIdx.x, tot = m + n;
    extern __shared__ __align__(16) unsigned char sk_smem[];
    unsigned char* lab = sk_smem;                                  // [tot]
    double* red = reinterpret_cast<double*>(sk_smem + ((tot + 15) / 16) * 16);  // [256]
    const int32_t* pi = perms + p * tot;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) lab[t] = 1;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
        const int32_t v = pi[t];
        if (v >= 0 && v < tot) lab[v] = 0;  // rows are not validated: stay in bounds
    }
    __syncthreads();
    const double wxx = m > 1 ? 1.0 / ((double)m * (double)(m - 1)) : 0.0;
    const double wyy = n > 1 ? 1.0 / ((double)n * (double)(n - 1)) : 0.0;
    const double wxy = -1.0 / ((double)m * (double)n);
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < tot * tot; e += blockDim.x) {
        const int64_t a = e / tot, b = e - a * tot;
        if (a == b) continue;
        const int la = lab[a], lb = lab[b];
        const double w = la != lb ? wxy : (la == 0 ? wxx : wyy);
        acc += w * (double)K[e];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) stats[p] = (R)red[0];
}

// Unbiased MMD^2 of two path sets X (nx paths) and Y (ny paths) from the
// kernel values of one pair list: [pairs a < b of X][pairs a < b of Y][all
// X x Y pairs].  The within-set diagonals do not enter and k is symmetric, so
// each within-set pair stands for two entries of its Gram matrix:
//   MMD^2 = 2/(nx(nx-1)) sum_xx k + 2/(ny(ny-1)) sum_yy k - 2/(nx ny) sum_xy k.
// One workgroup, FP64 accumulation.
__host__ __device__ inline void sk_mmd2_weights(int64_t nx, int64_t ny, double* wxx, double* wyy,
                                                double* wxy) {
    *wxx = 2.0 / ((double)nx * (double)(nx - 1));
    *wyy = 2.0 / ((double)ny * (double)(ny - 1));
    *wxy = -2.0 / ((double)nx * (double)ny);
}

template <typename R>
__global__ __launch_bounds__(256) void k_mmd2_pairs(const R* k, int64_t nx, int64_t ny, R* out) {
    __shared__ double red[256];
    double wxx, wyy, wxy;
    sk_mmd2_weights(nx, ny, &wxx, &wyy, &wxy);
    const int64_t nxx = nx * (nx - 1) / 2, nyy = ny * (ny - 1) / 2, tot = nxx + nyy + nx * ny;
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int64_t i = threadIdx.x; i < tot; i += blockDim.x) {
        const double v = (double)k[i];
        if (i < nxx) sxx += v;
        else if (i < nxx + nyy) syy += v;
        else sxy += v;
    }
    red[threadIdx.x] = wxx * sxx + wyy * syy + wxy * sxy;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (R)red[0];
}

// Its derivative: gk[i] = dMMD^2/dk_i * gout[0] over the same pair list.
template <typename R>
__global__ __launch_bounds__(256) void k_mmd2_pairs_seed(const R* gout, int64_t nx, int64_t ny,
                                                         R* gk) {
    double wxx, wyy, wxy;
    sk_mmd2_weights(nx, ny, &wxx, &wyy, &wxy);
    const int64_t nxx = nx * (nx - 1) / 2, nyy = ny * (ny - 1) / 2, tot = nxx + nyy + nx * ny;
    const double g = (double)gout[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x)
        gk[i] = (R)(g * (i < nxx ? wxx : i < nxx + nyy ? wyy : wxy));
}

// p-value of stats[0] (the observed split) against stats[1..]:
// (1 + #{stats[q] >= stats[0], q >= 1}) / nperm, one workgroup.
template <typename R>
__global__ __launch_bounds__(256) void k_mmd_pvalue(const R* stats, int64_t nperm, double* pvalue) {
    __shared__ int64_t red[256];
    int64_t c = 0;
    for (int64_t q = 1 + threadIdx.x; q < nperm; q += blockDim.x) c += stats[q] >= stats[0] ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *pvalue = (double)(1 + red[0]) / (double)nperm;
}

// ---------------------------------------------------------------------------
// diagnostics: skewed constants back to row-major C[p][i][j]
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_unskew(SkPairSrc src, const R* cskew, R* C, int64_t first) {
    const int64_t local = blockIdx.x;
    const SkPairDesc pd = sk_pair(src, local);
    const SkGeom g = sk_make_geom(pd.lx, pd.ly);
    const int64_t n = (int64_t)pd.lx * pd.ly;
    for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.y * blockDim.x) {
        const int i = (int)(e / pd.ly), j = (int)(e % pd.ly);
        const int s = i / 64, r = i % 64;
        const int64_t tau = (int64_t)s * g.Tp + j + r;
        C[(first + local) * n + e] = cskew[pd.c_off + tau * 64 + r];
    }
}
