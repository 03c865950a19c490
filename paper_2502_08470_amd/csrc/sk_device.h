// Device-side building blocks: cross-lane moves, wave reductions and the
// one-cell maps of the polynomial schemes.
//
// Edge coefficients are kept in the factorial-scaled basis P'_n = n! P_n,
// in the working precision R, except coefficients 0 and 1 (the kernel value
// at the cell corner and the slope along the edge), which are carried and
// updated in FP64 as well: their updates add small corrections to large,
// long-lived values every cell, the dominant source of rounding error in an
// FP32 sweep.
// where P_n are the coefficients of an edge in its cell's local variable
// u in [0, 1].  In that basis the untruncated one-step map of Proposition
// "approxsolution" (eqs. powerseries1/2, normalised cell, constant c) reads
//
//   A^P_r = sum_{k<=min(r,N)} w_{r-k} P'_k + c^r sum_{k=1}^{N} Q'_k / (r+k)!,
//   A^Q_r = sum_{k<=min(r,N)} w_{r-k} Q'_k + c^r sum_{k=1}^{N} P'_k / (r+k)!,
//
// with w_m = c^m / m! (a Toeplitz part and a Hankel part).  The
// approximation scheme keeps rows r <= N (the truncation pi_N).  The
// interpolation scheme keeps rows up to N + T and folds rows N+1..N+T back
// with a fixed matrix: since the interpolation operator at the Chebyshev
// extrema reproduces polynomials of degree <= N, interpolating the exact edge
// sum_r A_r u^r equals A_{<=N} + sum_{r>N} A_r Omega^N(u^r), and in the scaled
// basis Omega^N(u^r) contributes Rs[n][r] = R[n][r] n!/r!.  Rs is independent
// of c and built once on the host in FP64.  The number of tail rows T is
// chosen adaptively per wavefront step (see below) so that the dropped rows
// are below the working precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SK_NMAX 12   // largest compiled polynomial order
#define SK_TMAX 20   // longest interpolation tail (table size)
#define SK_IFA (2 * SK_NMAX + SK_TMAX + 4)  // 1/m! entries the tail rows index

// Longest interpolation tail compiled per working precision.  The tail a
// cell needs grows with |c| and with the precision: FP64 needs 17 rows at
// |c| = 8 and FP32 12 (the decision rule below), so these caps hold every
// cell with |c| up to about 10.  A cell that still needs rows after the cap
// is not computed: its outputs are NaN (which reaches the pair's kernel value
// and gradient) and the device status word records SK_STATUS_TAIL_CAP.
template <typename R> struct SkTailMax;
template <> struct SkTailMax<float> { static constexpr int value = 14; };
template <> struct SkTailMax<double> { static constexpr int value = 20; };
// Tail rows whose row derivatives the adjoints keep per replayed step (in
// registers, or LDS for the strip pipeline).  A checkpoint segment with a
// longer tail takes the adjoints' slower path, which recomputes each step's
// inputs and derives the rows on the fly.
template <typename R> struct SkTailReg;
template <> struct SkTailReg<float> { static constexpr int value = 3; };
template <> struct SkTailReg<double> { static constexpr int value = 6; };

// Device status bits (a per-device word, read with sigkernel_status).
#define SK_STATUS_TAIL_CAP 1u   // an interpolation cell needed more tail rows than compiled
#define SK_STATUS_WAIT_ABORT 2u // a strip-pipeline wait gave up
// One word per translation unit that launches kernels; the host reads each
// through hipGetSymbolAddress.  Written only with vector atomics.
static __device__ unsigned sk_status_word;
__device__ __forceinline__ void sk_raise_status(unsigned bit) { atomicOr(&sk_status_word, bit); }

// Streaming accesses: data written once and read once by a later kernel
// (checkpoints, skewed dL/dc), far larger than the caches, bypass their
// retention with non-temporal loads and stores.
template <typename T>
__device__ __forceinline__ void sk_st_nt(T* p, T v) { __builtin_nontemporal_store(v, p); }
template <typename T>
__device__ __forceinline__ T sk_ld_nt(const T* p) { return __builtin_nontemporal_load(p); }

// A pointer into LDS (address space 3): its arithmetic is 32-bit, where a
// generic pointer's would be 64-bit with an unused high half.
template <typename T> using SkLds = __attribute__((address_space(3))) T*;

// Kernel-argument tables of the interpolation scheme.
template <typename R>
struct SkTab {
    R rs[SK_NMAX + 1][SK_TMAX];  // scaled projection of tail row N+1+t onto row n
    R rmax[SK_TMAX + 1];         // max_n |rs[n][t]|
    R cmax[SK_TMAX + 1];         // |c| up to which the projected rows from N+1+t on
                                 // shrink at least by half per row
    R ifa[SK_IFA];               // 1/m!, for rows indexed at run time
};

// ---------------------------------------------------------------------------
// compile-time constants
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double sk_inv_fact(int m) {
    double f = 1.0;
    for (int i = 2; i <= m; ++i) f *= (double)i;
    return 1.0 / f;
}

template <typename R>
__device__ __forceinline__ R ifact(int m) { return (R)sk_inv_fact(m); }

// ---------------------------------------------------------------------------
// cross-lane moves (DPP across the whole 64-lane wave) and reductions
// ---------------------------------------------------------------------------
// lane r receives the value of lane r-1 (lane 0 receives 0)
__device__ __forceinline__ float lane_from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_prev(double v) {
    int2 b = *reinterpret_cast<int2*>(&v);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(0, b.x, 0x138, 0xf, 0xf, true);
    o.y = __builtin_amdgcn_update_dpp(0, b.y, 0x138, 0xf, 0xf, true);
    return *reinterpret_cast<double*>(&o);
}
// lane r receives the value of lane r+1 (lane 63 receives 0)
__device__ __forceinline__ float lane_from_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_next(double v) {
    int2 b = *reinterpret_cast<int2*>(&v);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(0, b.x, 0x130, 0xf, 0xf, true);
    o.y = __builtin_amdgcn_update_dpp(0, b.y, 0x130, 0xf, 0xf, true);
    return *reinterpret_cast<double*>(&o);
}

__device__ __forceinline__ int lane_from_prev(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);
}
// lane r receives the value of lane r-1 and lane 0 receives `lane0` (its own
// value of that argument): the same lane move with the first lane's input
// merged in, for inputs every lane reads alike (a broadcast LDS read)
__device__ __forceinline__ float lane_from_prev_or(float v, float lane0) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(lane0), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_from_prev_or(double v, double lane0) {
    int2 b = *reinterpret_cast<int2*>(&v);
    int2 z = *reinterpret_cast<int2*>(&lane0);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(z.x, b.x, 0x138, 0xf, 0xf, false);
    o.y = __builtin_amdgcn_update_dpp(z.y, b.y, 0x138, 0xf, 0xf, false);
    return *reinterpret_cast<double*>(&o);
}
__device__ __forceinline__ int lane_from_prev_or(int v, int lane0) {
    return __builtin_amdgcn_update_dpp(lane0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int lane_from_next(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
}

template <typename R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        R u = __shfl_xor(v, o, 64);
        v = v > u ? v : u;
    }
    return v;
}

__device__ __forceinline__ float sk_ldexp(float v, int e) { return ldexpf(v, e); }
__device__ __forceinline__ double sk_ldexp(double v, int e) { return ldexp(v, e); }
__device__ __forceinline__ float sk_abs(float v) { return fabsf(v); }
__device__ __forceinline__ double sk_abs(double v) { return fabs(v); }
__device__ __forceinline__ int sk_frexp_exp(float v) { int e; frexpf(v, &e); return e; }
__device__ __forceinline__ int sk_frexp_exp(double v) { int e; frexp(v, &e); return e; }
__device__ __forceinline__ bool sk_finite(float v) { return isfinite(v); }
__device__ __forceinline__ bool sk_finite(double v) { return isfinite(v); }

// Rescale band: the wave exponent changes only when the largest live
// magnitude leaves [2^-band, 2^band].
template <typename R> struct SkBand;
template <> struct SkBand<float> { static constexpr int value = 32; };
template <> struct SkBand<double> { static constexpr int value = 256; };

// Exponent update from the largest magnitude `m` of a lane's state.
// Returns the shift to apply (0 = none).
template <typename R>
__device__ __forceinline__ int sk_rescale_shift(R m) {
    if (!(m > (R)0) || !sk_finite(m)) return 0;
    int e = sk_frexp_exp(m);
    constexpr int band = SkBand<R>::value;
    return (e > band || e < -band) ? e : 0;
}

// ---------------------------------------------------------------------------
// adaptive tail of the interpolation scheme
// ---------------------------------------------------------------------------
// Tail rows r = N+1, N+2, ... are computed one at a time, and folded while
// any active lane of the wave still needs them (a wave-uniform decision).  A
// lane no longer needs row r nor any later row when (i) the projection of
// row r, doubled, is below the working precision relative to the edge scale,
// 2 |A_r| max_n |Rs[n][r]| <= eps (|A_0^P| + |A_0^Q|), and (ii) the projected
// rows from r on shrink at least geometrically with ratio 1/2.  Each further
// row multiplies the terms of A by at most |c| / (r + 1 - N), and the
// projection weights max_n |Rs[n][r']| by at most rho_t from one row to the
// next (rho_t: the largest such ratio over all later rows, measured on the
// host), so (ii) holds once |c| <= cmax[t] = (t + 2) / (2 rho_t), t = r - N - 1.
// Under (i) and (ii) row r and everything after it together stay below eps
// relative, so row r is then dropped too: the row that decides is computed
// but not folded.  After TMAX folded rows one more row decides; a lane that
// still needs it is past the compiled cap (see SkTailMax).
template <typename R> struct SkEps;
template <> struct SkEps<float> { static constexpr double value = 1.0 / (1 << 26); };
template <> struct SkEps<double> { static constexpr double value = 1.0 / (double)(1ull << 55); };

__device__ __forceinline__ bool sk_wave_any(bool v) { return __any(v ? 1 : 0) != 0; }

// ---------------------------------------------------------------------------
// forward cell map
// ---------------------------------------------------------------------------
// (P, Q): bottom and left edges in the scaled basis; returns top (Po) and
// right (Qo).  TMAX = 0: approximation scheme.  TMAX > 0: interpolation
// scheme with the adaptive tail above; `active` lanes take part in the
// tail decision (idle lanes may hold stale values).
// Edge coefficients 0 and 1 (the value at the corner and the slope) are
// carried in FP64 by the caller (P0, P1, Q0, Q1) and updated here in FP64;
// P[0], P[1], Q[0], Q[1] must hold their rounded copies, used by the rows
// n >= 2, which are computed in R.  Outputs likewise: Po0, Po1, Qo0, Qo1 in
// FP64, Po[0..1], Qo[0..1] their rounded copies.
// WD: also return the c-derivatives of the untruncated rows,
//   D^P_r = dA^P_r/dc = (Toeplitz row r-1 of P) + r c^{r-1} (Hankel row r of Q),
// for r = 1..N+T in DP[r-1] (zero beyond the rows kept), and the number of
// tail rows kept T (wave-uniform).  These are all the adjoint needs from the
// forward: its transposed map does not depend on the edges.
// HI = false: every row in R (the FP64 arguments are ignored and the FP64
// outputs are the R results widened); used where FP32 accuracy of the state
// is enough, e.g. the adjoint's short replays.
// Tkept (nullable): receives the number of tail rows folded (wave-uniform).
// FIXT: fold exactly Tfix tail rows (wave-uniform) instead of deciding, so that
// a replay repeats the decisions of the forward it replays.
// DS: element stride of DP and DQ (1 for registers; 64 for an LDS array with
// one slot per lane).
// Wout (nullable): receives w_m = c^m/m!, m = 1..N (as the rows used them).
template <typename R, int N, int TMAX, bool WD = false, bool HI = true, bool FIXT = false,
          int DS = 1>
__device__ __forceinline__ void sk_cell_fwd(const R (&P)[N + 1], const R (&Q)[N + 1], double P0,
                                            double P1, double Q0, double Q1, R c, bool active,
                                            const SkTab<R>& tab, R (&Po)[N + 1], R (&Qo)[N + 1],
                                            double& Po0, double& Po1, double& Qo0, double& Qo1,
                                            R* DP = nullptr, R* DQ = nullptr,
                                            int* Tkept = nullptr, int Tfix = 0,
                                            R* Wout = nullptr) {
    // tail rows unrolled with constant indices (the rest in a loop)
    constexpr int TU = TMAX < SkTailReg<R>::value ? TMAX : SkTailReg<R>::value;
    // rows up to N + TU in the unrolled part (+1 that only decides, when
    // that part reaches the cap)
    constexpr int M = N + TU + ((TMAX > 0 && !FIXT && TMAX == TU) ? 1 : 0);
    // powers of c needed before the tail (the deciding row N+1 unless the
    // tail length is given); the tail computes its own as it goes
    constexpr int MU = (TMAX > 0 && !FIXT) ? N + 1 : N;
    R w[M + 1], cp[M + 1];
    w[0] = (R)1;
    cp[0] = (R)1;
    // the sweep's state takes c^m/m! by its own recurrence (independent
    // rounding of the Toeplitz and Hankel parts measured about twice as
    // accurate).  Where FP32 accuracy is enough (!HI) the rows up to N need no
    // c^m: their Hankel sums are taken against r!/(r+k)!, so that
    // c^r sum_k Q'_k/(r+k)! = w_r sum_k Q'_k r!/(r+k)!, and the tail rows
    // start c^m from w_N N!.
    auto power = [&](int m) {
        if (!HI && m <= N) {
            w[m] = m == 1 ? c : w[m - 1] * (c * (R)(1.0 / m));
            return;
        }
        if (!HI && m == N + 1) cp[N] = w[N] * (R)(1.0 / sk_inv_fact(N));
        cp[m] = cp[m - 1] * c;
        w[m] = HI ? w[m - 1] * (c * (R)(1.0 / m)) : cp[m] * ifact<R>(m);
    };
#pragma unroll
    for (int m = 1; m <= MU; ++m) power(m);
    if (Wout) {  // c^m/m!, m = 1..N, for the adjoint of the same cell
#pragma unroll
        for (int m = 1; m <= N; ++m) Wout[m - 1] = w[m];
    }
    if (WD && !FIXT) {
        // rows 0..N-1 are always written; tail rows only when kept (a replay
        // with the tail length given reads exactly the rows it folds)
#pragma unroll
        for (int r = N; r < N + TU; ++r) {
            DP[r * DS] = (R)0;
            DQ[r * DS] = (R)0;
        }
    }
    if (Tkept) *Tkept = 0;
    // rows 0 and 1 (in FP64 when HI):
    //   A_0 = P'_0 + sum_{k>=1} Q'_k/k!,  A_1 = P'_1 + c (P'_0 + sum_{k>=1} Q'_k/(k+1)!)
    double HQ1, HP1;
    if (HI) {
        R hq0 = (R)0, hp0 = (R)0, hq1 = (R)0, hp1 = (R)0;
#pragma unroll
        for (int k = N; k >= 2; --k) {
            hq0 = fma(Q[k], ifact<R>(k), hq0);
            hp0 = fma(P[k], ifact<R>(k), hp0);
            hq1 = fma(Q[k], ifact<R>(k + 1), hq1);
            hp1 = fma(P[k], ifact<R>(k + 1), hp1);
        }
        const double cd = (double)c;
        HQ1 = (double)hq1 + 0.5 * Q1;
        HP1 = (double)hp1 + 0.5 * P1;
        Po0 = P0 + ((double)hq0 + Q1);
        Qo0 = Q0 + ((double)hp0 + P1);
        Po1 = fma(cd, P0 + HQ1, P1);
        Qo1 = fma(cd, Q0 + HP1, Q1);
    } else {
        R hq0 = (R)0, hp0 = (R)0, hq1 = (R)0, hp1 = (R)0;
#pragma unroll
        for (int k = N; k >= 1; --k) {
            hq0 = fma(Q[k], ifact<R>(k), hq0);
            hp0 = fma(P[k], ifact<R>(k), hp0);
            hq1 = fma(Q[k], ifact<R>(k + 1), hq1);
            hp1 = fma(P[k], ifact<R>(k + 1), hp1);
        }
        HQ1 = (double)hq1;
        HP1 = (double)hp1;
        Po0 = (double)(P[0] + hq0);
        Qo0 = (double)(Q[0] + hp0);
        Po1 = (double)fma(c, P[0] + hq1, P[1]);
        Qo1 = (double)fma(c, Q[0] + hp1, Q[1]);
    }
    R tpp = P[0], tqp = Q[0];  // Toeplitz row r-1 (for D)
    if (WD) {
        // D_1 = (Toeplitz row 0) + 1 * c^0 * H_1
        DP[0] = P[0] + (R)HQ1;
        DQ[0] = Q[0] + (R)HP1;
        tpp = fma(c, P[0], P[1]);
        tqp = fma(c, Q[0], Q[1]);
    }
#pragma unroll
    for (int r = 2; r <= N; ++r) {
        // Toeplitz row r, from its k = r term (w_0 = 1)
        R tp = P[r], tq = Q[r];
#pragma unroll
        for (int k = r - 1; k >= 0; --k) {
            tp = fma(w[r - k], P[k], tp);
            tq = fma(w[r - k], Q[k], tq);
        }
        R hq = (R)0, hp = (R)0;
#pragma unroll
        for (int k = N; k >= 1; --k) {
            // HI: 1/(r+k)!;  !HI: r!/(r+k)! (see power)
            const R f = HI ? ifact<R>(r + k) : (R)(sk_inv_fact(r + k) / sk_inv_fact(r));
            hq = fma(Q[k], f, hq);
            hp = fma(P[k], f, hp);
        }
        // Hankel weight of row r, c^r (HI) or w_r; of its c-derivative,
        // r c^(r-1) (HI) or w_(r-1) (since r c^(r-1) / r! = w_(r-1))
        const R hw = HI ? cp[r] : w[r];
        Po[r] = fma(hw, hq, tp);
        Qo[r] = fma(hw, hp, tq);
        if (WD) {
            const R rc = HI ? (R)r * cp[r - 1] : w[r - 1];
            DP[(r - 1) * DS] = fma(rc, hq, tpp);
            DQ[(r - 1) * DS] = fma(rc, hp, tqp);
            tpp = tp;
            tqp = tq;
        }
    }
    if (TMAX > 0) {
        const R scale = (R)SkEps<R>::value * (R)(fabs(Po0) + fabs(Qo0));
        const R ac = sk_abs(c);
        R t0p = (R)0, t0q = (R)0, t1p = (R)0, t1q = (R)0;  // tail into rows 0, 1
        int folded = 0;        // wave-uniform
        bool capped = false;   // wave-uniform: some lane went past the cap
        bool poison = false;   // this lane's cell is past the cap
        // Tail row t (row r = N + 1 + t) with Toeplitz parts tp, tq and
        // Hankel parts hq, hp: decide whether it is needed and fold it.
        // Returns false once the tail has ended (wave-uniform).
        auto tail_row = [&](int t, int r, R cpr, R cpr1, R tp, R tq, R hq, R hp) -> bool {
            const R arp = fma(cpr, hq, tp), arq = fma(cpr, hp, tq);
            if (!FIXT) {
                const R tail = (R)2 * tab.rmax[t] * (sk_abs(arp) + sk_abs(arq));
                const bool need = active && (!(tail <= scale) || ac > tab.cmax[t]);
                if (!sk_wave_any(need)) return false;
                if (t == TMAX) {  // past the compiled cap: these lanes' cells are not computed
                    capped = true;
                    poison = need;
                    if (Tkept) *Tkept = TMAX + 1;
                    if (need && __builtin_amdgcn_readfirstlane(__lane_id()) == __lane_id())
                        sk_raise_status(SK_STATUS_TAIL_CAP);
                    return false;
                }
            }
            if (WD) {
                const R rc = (R)r * cpr1;
                DP[(r - 1) * DS] = fma(rc, hq, tpp);
                DQ[(r - 1) * DS] = fma(rc, hp, tqp);
                tpp = tp;
                tqp = tq;
            }
            if (Tkept) *Tkept = t + 1;
            folded = t + 1;
            t0p = fma(tab.rs[0][t], arp, t0p);
            t0q = fma(tab.rs[0][t], arq, t0q);
            t1p = fma(tab.rs[1][t], arp, t1p);
            t1q = fma(tab.rs[1][t], arq, t1q);
#pragma unroll
            for (int n = 2; n <= N; ++n) {
                Po[n] = fma(tab.rs[n][t], arp, Po[n]);
                Qo[n] = fma(tab.rs[n][t], arq, Qo[n]);
            }
            return true;
        };
        // The first TU rows are unrolled (constant indices; the common tails
        // end here).  A longer tail continues in a loop over a sliding window
        // of the powers, with the table entries indexed by the row.
        bool more = true;
#pragma unroll
        for (int t = 0; t < TU + ((!FIXT && TMAX == TU) ? 1 : 0); ++t) {
            if (FIXT && t >= Tfix) {
                more = false;
                break;
            }
            const int r = N + 1 + t;
            if (r > MU) power(r);
            R tp = (R)0, tq = (R)0;
#pragma unroll
            for (int k = N; k >= 0; --k) {
                tp = fma(w[r - k], P[k], tp);
                tq = fma(w[r - k], Q[k], tq);
            }
            R hq = (R)0, hp = (R)0;
#pragma unroll
            for (int k = N; k >= 1; --k) {
                hq = fma(Q[k], ifact<R>(r + k), hq);
                hp = fma(P[k], ifact<R>(r + k), hp);
            }
            if (!tail_row(t, r, cp[r], cp[r - 1], tp, tq, hq, hp)) {
                more = false;
                break;
            }
        }
        if constexpr (TMAX > TU) {
            static_assert(!WD || DS > 1, "row derivatives past the unrolled tail need an LDS array");
            if (__builtin_expect(more, false)) {  // wave-uniform; rare: laid out off the hot path
                R win[N + 1];  // win[k] = c^(r-k) / (r-k)! for the current row r
#pragma unroll
                for (int k = 0; k <= N; ++k) win[k] = w[N + TU - k];
                R cpr = cp[N + TU];
                const int tend = FIXT ? (Tfix < TMAX ? Tfix : TMAX) : TMAX + 1;
                // kept rolled: unrolled, the table entries would be hoisted
                // into scalar registers for the whole kernel
#pragma unroll 1
                for (int t = TU; t < tend; ++t) {
                    const int r = N + 1 + t;
                    const R cpr1 = cpr;
                    cpr = cpr * c;
#pragma unroll
                    for (int k = N; k >= 1; --k) win[k] = win[k - 1];
                    win[0] = cpr * tab.ifa[r];
                    R tp = (R)0, tq = (R)0;
#pragma unroll
                    for (int k = N; k >= 0; --k) {
                        tp = fma(win[k], P[k], tp);
                        tq = fma(win[k], Q[k], tq);
                    }
                    R hq = (R)0, hp = (R)0;
#pragma unroll
                    for (int k = N; k >= 1; --k) {
                        hq = fma(Q[k], tab.ifa[r + k], hq);
                        hp = fma(P[k], tab.ifa[r + k], hp);
                    }
                    if (!tail_row(t, r, cpr, cpr1, tp, tq, hq, hp)) break;
                }
            }
        }
        if (FIXT && Tfix > TMAX) {  // the forward went past its cap here
            capped = true;
            poison = active;
        }
        if (folded == 0) {
            // nothing folded (the common case for small |c|): rows 0, 1 stand
        } else if (HI) {
            Po0 += (double)t0p;
            Qo0 += (double)t0q;
            Po1 += (double)t1p;
            Qo1 += (double)t1q;
        } else {  // rows 0 and 1 are R values here: no FP64 arithmetic
            Po0 = (double)((R)Po0 + t0p);
            Qo0 = (double)((R)Qo0 + t0q);
            Po1 = (double)((R)Po1 + t1p);
            Qo1 = (double)((R)Qo1 + t1q);
        }
        // a scalar branch around the per-lane poisoning keeps the selects
        // off the common path
        if (__builtin_expect(capped, false) && poison) {
            Po0 = Qo0 = Po1 = Qo1 = (double)NAN;
#pragma unroll
            for (int n = 2; n <= N; ++n) Po[n] = Qo[n] = (R)NAN;
        }
    }
    Po[0] = (R)Po0;
    Qo[0] = (R)Qo0;
    Po[1] = (R)Po1;
    Qo[1] = (R)Qo1;
}

// ---------------------------------------------------------------------------
// adjoint cell map
// ---------------------------------------------------------------------------
// Given the adjoints a = dL/dPo, b = dL/dQo of a cell's outputs, returns the
// adjoints of its inputs (aP = dL/dP, aQ = dL/dQ) and g = dL/dc.  The map is
// linear in (P, Q), so its transpose needs only c and the number of tail rows
// T the forward kept; g needs the row derivatives D^P, D^Q recorded by the
// forward (sk_cell_fwd with WD).  Rows are visited once, in outer-product
// order, so no per-row arrays stay live:
//   aP_k += w_{r-k} ea_r (k <= min(r, N)),  aP_k += c^r eb_r / (r+k)! (k >= 1),
// with ea_r = a_r for r <= N and ea_r = sum_n Rs[n][r] a_n for tail rows.
// The rows up to N take their Hankel part as w_r eb_r against r!/(r+k)!
// (c^r/(r+k)! = w_r r!/(r+k)!), so they need only w_m = c^m/m!, which the
// forward replay of the same cell can hand over (Wpre, nullable: m = 1..N);
// tail rows continue c^m from w_N N!.
template <typename R, int N, int TMAX, int DS = 1>
__device__ __forceinline__ void sk_cell_adj(R c, int T, const SkTab<R>& tab, const R (&a)[N + 1],
                                            const R (&b)[N + 1], const R* DP, const R* DQ,
                                            R (&aP)[N + 1], R (&aQ)[N + 1], R& g,
                                            const R* Wpre = nullptr) {
    constexpr int M = N + TMAX;
    R w[M + 1], cp[M + 1];
    w[0] = (R)1;
    cp[0] = (R)1;
    auto power = [&](int m) {
        if (m == N + 1) cp[N] = w[N] * (R)(1.0 / sk_inv_fact(N));
        cp[m] = cp[m - 1] * c;
        w[m] = cp[m] * ifact<R>(m);  // gradients need FP32 accuracy only
    };
#pragma unroll
    for (int m = 1; m <= N; ++m)  // tail rows compute theirs as they go
        w[m] = Wpre ? Wpre[m - 1] : (m == 1 ? c : w[m - 1] * (c * (R)(1.0 / m)));
    // row 0 initialises the outputs (w_0 = c^0 = 1)
    aP[0] = a[0];
    aQ[0] = b[0];
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        aP[k] = b[0] * ifact<R>(k);
        aQ[k] = a[0] * ifact<R>(k);
    }
    R gacc = (R)0;
    // T is the same in every lane; reading it into a scalar register makes
    // the early exit a branch instead of masked execution of every tail row
    const int Tu = __builtin_amdgcn_readfirstlane(T);
#pragma unroll
    for (int r = 1; r <= M; ++r) {
        if (r > N && r - N > Tu) break;
        if (r > N) power(r);
        R ea, eb;
        if (r <= N) {
            ea = a[r];
            eb = b[r];
        } else {
            ea = tab.rs[0][r - N - 1] * a[0];
            eb = tab.rs[0][r - N - 1] * b[0];
#pragma unroll
            for (int n = 1; n <= N; ++n) {
                ea = fma(tab.rs[n][r - N - 1], a[n], ea);
                eb = fma(tab.rs[n][r - N - 1], b[n], eb);
            }
        }
        gacc = r == 1 ? ea * DP[0] : fma(ea, DP[(r - 1) * DS], gacc);
        gacc = fma(eb, DQ[(r - 1) * DS], gacc);
#pragma unroll
        for (int k = (r < N ? r : N); k >= 0; --k) {
            aP[k] = fma(w[r - k], ea, aP[k]);
            aQ[k] = fma(w[r - k], eb, aQ[k]);
        }
        const R hw = r <= N ? w[r] : cp[r];
        const R cb = hw * eb, ca = hw * ea;
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            const R f = r <= N ? (R)(sk_inv_fact(r + k) / sk_inv_fact(r)) : ifact<R>(r + k);
            aP[k] = fma(cb, f, aP[k]);
            aQ[k] = fma(ca, f, aQ[k]);
        }
    }
    g = gacc;
}

// The same transposed map, with the row derivatives D^P_r, D^Q_r computed
// here from the cell's inputs (P, Q) instead of read from a forward replay:
// D^P_r = sum_{k<=min(r-1,N)} w_{r-1-k} P'_k + r c^{r-1} sum_{k=1}^{N} Q'_k/(r+k)!.
// Used for the rare checkpoint segments whose tail is longer than the
// adjoints keep derivatives for (SkTailReg); T > TMAX (a cell past the
// compiled cap in the forward) gives g = NaN.
template <typename R, int N, int TMAX>
__device__ __forceinline__ void sk_cell_adj_in(R c, int T, const SkTab<R>& tab, const R (&a)[N + 1],
                                               const R (&b)[N + 1], const R (&P)[N + 1],
                                               const R (&Q)[N + 1], R (&aP)[N + 1],
                                               R (&aQ)[N + 1], R& g) {
    R w[N + 1], cp[N + 1];
    w[0] = (R)1;
    cp[0] = (R)1;
#pragma unroll
    for (int m = 1; m <= N; ++m) {
        cp[m] = cp[m - 1] * c;
        w[m] = cp[m] * ifact<R>(m);
    }
    aP[0] = a[0];
    aQ[0] = b[0];
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        aP[k] = b[0] * ifact<R>(k);
        aQ[k] = a[0] * ifact<R>(k);
    }
    R gacc = (R)0;
    // rows 1..N (constant indices)
#pragma unroll
    for (int r = 1; r <= N; ++r) {
        const R ea = a[r], eb = b[r];
        R tp = P[r - 1], tq = Q[r - 1];  // Toeplitz row r - 1, from its w_0 = 1 term
#pragma unroll
        for (int k = r - 2; k >= 0; --k) {
            tp = fma(w[r - 1 - k], P[k], tp);
            tq = fma(w[r - 1 - k], Q[k], tq);
        }
        R hq = (R)0, hp = (R)0;
#pragma unroll
        for (int k = N; k >= 1; --k) {
            hq = fma(Q[k], ifact<R>(r + k), hq);
            hp = fma(P[k], ifact<R>(r + k), hp);
        }
        const R rc = (R)r * cp[r - 1];
        gacc = fma(ea, fma(rc, hq, tp), gacc);
        gacc = fma(eb, fma(rc, hp, tq), gacc);
#pragma unroll
        for (int k = r; k >= 0; --k) {
            aP[k] = fma(w[r - k], ea, aP[k]);
            aQ[k] = fma(w[r - k], eb, aQ[k]);
        }
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            aP[k] = fma(cp[r] * eb, ifact<R>(r + k), aP[k]);
            aQ[k] = fma(cp[r] * ea, ifact<R>(r + k), aQ[k]);
        }
    }
    // tail rows r = N+1 .. N+T, in a loop: win[i] = c^(r-i) / (r-i)!
    const int Tu = __builtin_amdgcn_readfirstlane(T);
    const int tend = Tu < TMAX ? Tu : TMAX;
    R win[N + 2];
#pragma unroll
    for (int i = 0; i <= N; ++i) win[i] = w[N - i];
    win[N + 1] = (R)0;
    R cpr = cp[N];
#pragma unroll 1
    for (int t = 0; t < tend; ++t) {
        const int r = N + 1 + t;
        const R cpr1 = cpr;
        cpr = cpr * c;
#pragma unroll
        for (int i = N + 1; i >= 1; --i) win[i] = win[i - 1];
        win[0] = cpr * tab.ifa[r];
        R ea = tab.rs[0][t] * a[0], eb = tab.rs[0][t] * b[0];
#pragma unroll
        for (int n = 1; n <= N; ++n) {
            ea = fma(tab.rs[n][t], a[n], ea);
            eb = fma(tab.rs[n][t], b[n], eb);
        }
        R tp = (R)0, tq = (R)0;
#pragma unroll
        for (int k = N; k >= 0; --k) {
            tp = fma(win[k + 1], P[k], tp);
            tq = fma(win[k + 1], Q[k], tq);
        }
        R hq = (R)0, hp = (R)0;
#pragma unroll
        for (int k = N; k >= 1; --k) {
            hq = fma(Q[k], tab.ifa[r + k], hq);
            hp = fma(P[k], tab.ifa[r + k], hp);
        }
        const R rc = (R)r * cpr1;
        gacc = fma(ea, fma(rc, hq, tp), gacc);
        gacc = fma(eb, fma(rc, hp, tq), gacc);
#pragma unroll
        for (int k = N; k >= 0; --k) {
            aP[k] = fma(win[k], ea, aP[k]);
            aQ[k] = fma(win[k], eb, aQ[k]);
        }
        const R cb = cpr * eb, ca = cpr * ea;
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            aP[k] = fma(cb, tab.ifa[r + k], aP[k]);
            aQ[k] = fma(ca, tab.ifa[r + k], aQ[k]);
        }
    }
    g = T > TMAX ? (R)NAN : gacc;
}
