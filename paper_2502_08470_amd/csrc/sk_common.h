// Shared host/device definitions of the signature-kernel GPU library.
//
// Grid of one path pair: cells (i, j), 0 <= i < lx (segments of x),
// 0 <= j < ly (segments of y); cell constant c_ij = <dx_i, dy_j> (the PDE
// constant on the normalised unit cell; the time partition drops out once
// edge coefficients are expressed in the cell's local variables).
//
// Wavefront mapping (one 64-lane wave per pair): lane r owns the x-segments
// i = 64 s + r of strips s = 0, 1, ...; at step tau it processes the cell with
// linear index L = tau - r, strip s = L / Tp, column j = L % Tp.  Tp is the
// strip period max(ly, W), W = min(lx, 64), which guarantees that the last
// lane of strip s-1 has produced the left edge of (64 s, j) before lane 0 of
// strip s needs it.  Lanes run strips back to back, so all lanes stay busy
// except during the first and last 63 steps of the whole pair.
//
// The "skewed" layout stores any per-cell quantity (cell constants c, or
// dL/dc in the backward pass) as rows tau of 64 lane slots: element
// [tau][r] is the value of the cell that lane r processes at step tau, zero
// where that lane is idle.  The sweep then reads one contiguous 64-element row
// per step.
#pragma once
#include <stdint.h>

#ifndef __HIP__
#define __host__
#define __device__
#endif

#define SK_LANES 64

struct SkGeom {
    int32_t lx, ly;      // segments (after dyadic refinement for the FD scheme)
    int32_t nstrips;     // ceil(lx / 64)
    int32_t Tp;          // strip period max(ly, min(lx, 64))
    int32_t nsteps;      // steps until the last cell (lx-1, ly-1) is done
    int32_t nsteps_pad;  // nsteps rounded up to a multiple of 64
};

__host__ __device__ inline SkGeom sk_make_geom(int32_t lx, int32_t ly) {
    SkGeom g;
    g.lx = lx;
    g.ly = ly;
    if (lx <= 0 || ly <= 0) {
        g.nstrips = 0; g.Tp = 0; g.nsteps = 0; g.nsteps_pad = 0;
        return g;
    }
    int32_t W = lx < SK_LANES ? lx : SK_LANES;
    g.nstrips = (lx + SK_LANES - 1) / SK_LANES;
    g.Tp = ly > W ? ly : W;
    int32_t rlast = (lx - 1) - (g.nstrips - 1) * SK_LANES;
    g.nsteps = (g.nstrips - 1) * g.Tp + (ly - 1) + rlast + 1;
    g.nsteps_pad = (g.nsteps + 63) / 64 * 64;
    return g;
}

// Strip-boundary exchange.  Lane 63 of strip s hands the right edge of each
// column to lane 0 of strip s+1 (in the adjoint, lane 0 hands the adjoint of
// the left edge back to lane 63 of strip s-1), Tp - 63 steps before it is
// consumed.  Those edges wait in a ring of one entry per column: in LDS for
// pairs up to a column count the host chooses per kernel (gx_cols), longer
// pairs through a per-pair global buffer whose entries are staged through
// LDS one 8-step block ahead (so long pairs do not cap occupancy through
// their LDS).  The global protocol needs Tp > 78; the host never sets
// gx_cols below SK_GX_MIN_COLS.
#define SK_GX_BLOCK 8
#define SK_GX_MIN_COLS 96
__host__ __device__ constexpr int sk_ring_col_bytes_fwd(int N, int es) { return (16 + (N - 1) * es + 4 + 7) / 8 * 8; }
__host__ __device__ constexpr int sk_ring_col_bytes_adj(int N, int es) { return (N + 1) * es + 4; }
// 32-bit words of one global exchange record, rounded up to 16 bytes:
// forward: FP64 coefficients 0 and 1, coefficients 2..N, exponent;
// adjoint: coefficients 0..N, exponent
__host__ __device__ constexpr int sk_gx_words(int N, int es) {
    return ((4 + (N - 1) * es / 4 + 1 > (N + 1) * es / 4 + 1 ? 4 + (N - 1) * es / 4 + 1
                                                             : (N + 1) * es / 4 + 1) + 3) / 4 * 4;
}
__host__ __device__ constexpr int sk_gx_stage_bytes(int N, int es) { return SK_GX_BLOCK * sk_gx_words(N, es) * 4; }
// The batched adjoint stages, one checkpoint segment ahead, the strip-boundary
// edges its lane 0 replays at steps 1..S-1 of a segment, for strides S <= 4:
// per step the coefficients 0..N, then the exponent in the last word (N + 2
// words in FP32; 2N + 4 in FP64, an even count that keeps every step's
// coefficients 8-byte aligned); rounded up to 16 bytes.
__host__ __device__ constexpr int sk_adj_qst_words(int N, int es) { return (N + 1) * es / 4 + (es == 8 ? 2 : 1); }
__host__ __device__ constexpr int sk_adj_qst_bytes(int N, int es) {
    return (3 * sk_adj_qst_words(N, es) * 4 + 15) / 16 * 16;
}

// Local steps of one strip on the strip pipeline: lane r processes column
// t - r at local step t, so lane 63 finishes the last column at step
// ly + 62; rounded up to whole 8-step blocks.
__host__ __device__ inline int32_t sk_pipe_steps(int32_t ly) { return (ly + 63 + 7) & ~7; }

// Per-pair description.  Gram calls derive it from the pair index; list
// (ragged) calls read it from a device array.
struct SkPairDesc {
    int64_t x_off;    // offset of the first point of x, in points
    int64_t y_off;    // offset of the first point of y, in points
    int32_t lx, ly;   // segments of x and y (unrefined)
    int32_t swap;     // 1: x is read from the second path array and y from the
                      // first (k(x, y) = k(y, x); the kernels see the pair
                      // transposed so that the columns are the shorter path)
    int64_t k_idx;    // output index of the pair
    int64_t g_idx;    // index of the pair's gradient seed dL/dk
    // element offsets of the pair's blocks in the chunk's workspace arrays
    int64_t c_off;    // skewed cell constants / skewed dL/dc
    int64_t ck_off;   // lane checkpoints (backward only; strip-pipeline pairs keep
                      // them per strip, on the strip's local steps)
    int64_t ce_off;   // per checkpoint: 64 lane exponents, then one word with the
                      // interpolation tail length of each of the segment's steps
                      // (8 bits per step; int32 elements)
    int64_t qb_off;   // strip-boundary edge vectors (backward only)
    int64_t qe_off;   // strip-boundary exponents (int32 elements)
    int64_t dx_off;   // per-pair dL/d(dx) partials
    int64_t dy_off;   // per-pair, per-strip dL/d(dy) partials
    int64_t xb_off;   // global strip-boundary exchange records (32-bit words)
    int64_t pg_off;   // strip-pipeline progress counters (int32 elements)
};

// Per-pair workspace strides, all derived from the pair's geometry.
struct SkPairSizes {
    int64_t c, ck, ce, qb, qe, dx, dy, xb, pg;
    int64_t cu;  // backward on a refined grid: dL/dc folded onto the unrefined
                 // grid's skewed layout (at the pair's c_off, so sized as c)
};

// xb_words: 32-bit words per column of the pair's global exchange records
// (0 when it needs none; twice the record for a strip-pipeline pair, whose
// records alternate between two slots)
// pipe: the pair runs on the strip pipeline (one progress counter per strip;
// backward: checkpoints per strip, every S of its sk_pipe_steps local steps)
__host__ __device__ inline SkPairSizes sk_pair_sizes(int32_t lx, int32_t ly, int32_t lam,
                                                     int32_t N, int32_t S, int64_t d,
                                                     bool backward, int xb_words,
                                                     bool pipe = false) {
    SkPairSizes z = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    SkGeom g = sk_make_geom(lx << lam, ly << lam);
    z.c = (int64_t)g.nsteps_pad * SK_LANES;
    if (g.nsteps > 0) z.xb = (int64_t)g.ly * xb_words;
    if (pipe && g.nsteps > 0) z.pg = g.nstrips;
    if (backward && g.nsteps > 0) {
        const int64_t nck = pipe ? (int64_t)g.nstrips * (sk_pipe_steps(g.ly) / S)
                                 : (g.nsteps + S - 1) / S;
        z.ck = nck * 2 * (N + 1) * SK_LANES;
        z.ce = nck * (SK_LANES + 1);  // per-lane exponents + the segment's tail lengths
        z.qb = (int64_t)g.nstrips * g.ly * (N + 1);
        z.qe = (int64_t)g.nstrips * g.ly;
        z.dx = (int64_t)lx * d;
        z.dy = (int64_t)g.nstrips * ly * d;  // refined strips >= the unrefined grid's
        if (lam > 0) z.cu = z.c;
    }
    return z;
}

struct SkPairSrc {
    // Gram mode (desc == nullptr): pair p = a * ny + b, uniform strides.
    int64_t ny;
    int64_t lx_pts, ly_pts;
    SkPairSizes stride;
    int64_t first;          // global index of the chunk's first pair
    // List mode
    const SkPairDesc* desc; // device array indexed by chunk-local pair
};

__host__ __device__ inline SkPairDesc sk_pair(const SkPairSrc& s, int64_t local) {
    if (s.desc) return s.desc[local];
    SkPairDesc d;
    int64_t p = s.first + local;
    int64_t a = p / s.ny, b = p % s.ny;
    d.x_off = a * s.lx_pts;
    d.y_off = b * s.ly_pts;
    d.lx = (int32_t)(s.lx_pts - 1);
    d.ly = (int32_t)(s.ly_pts - 1);
    d.swap = 0;
    d.k_idx = p;
    d.g_idx = p;
    d.c_off = local * s.stride.c;
    d.ck_off = local * s.stride.ck;
    d.ce_off = local * s.stride.ce;
    d.qb_off = local * s.stride.qb;
    d.qe_off = local * s.stride.qe;
    d.dx_off = local * s.stride.dx;
    d.dy_off = local * s.stride.dy;
    d.xb_off = local * s.stride.xb;
    d.pg_off = local * s.stride.pg;
    return d;
}
