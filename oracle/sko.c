/*
 * FP64 CPU oracle for the signature-kernel schemes -- test infrastructure only.
 * It is never linked into, loaded by or called from the GPU library.
 *
 * Written from "Numerical Schemes for Signature Kernels" (Cass, Piatti, Pei):
 *   - sko_fd:      Definition "Dyadic finite differences approximation scheme"
 *   - sko_fd2:     the second-order explicit rule of Remark "higherfd"
 *                  (eq. secondexplicitscheme) on the same refined grid
 *                  (Section 2), first-order explicit rule, lambda-refined grid.
 *   - sko_approx:  Definition "Polynomial approximation numerical scheme"
 *                  (Section 3.2) with the explicit truncated map of the remark
 *                  after it (Proposition "approxsolution" truncated at N); the
 *                  factorial factors are precomputed as that section suggests.
 *   - sko_approx_f32model: the approximation scheme with increments, cell
 *                  constants and the edge coefficients of degree >= 2
 *                  rounded to FP32 (FP64 arithmetic), a diagnostic: its
 *                  distance from sko_approx is a pair's conditioning floor
 *                  for evaluation with that FP32 state.
 *   - sko_interp:  Definition "Polynomial interpolation numerical scheme"
 *                  (Section 3.3): Proposition "propinterp" (eq. interpformula)
 *                  evaluated at the N+1 Chebyshev extrema (eq. chebextr),
 *                  then the degree-N interpolant (Definition "interpooperator")
 *                  obtained by solving the Vandermonde system.
 *
 * Conventions: paths are given by points (row-major, n_pts x d); partitions
 * are s_i = i, t_j = j (unit spacing), so C_ij = <dx_i, dy_j>.  Results are
 * returned as mantissa * 2^exponent: after every row of cells the live edge
 * coefficients are rescaled by an exact power of two (exponent tracking), so
 * kernels beyond the FP64 range are representable.  No FMA contraction
 * (built with -ffp-contract=off), IEEE round-to-nearest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SKO_NMAX 32

static double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* largest |v| over the live state, then rescale by 2^-e so it is in [0.5,1) */
static void rescale(double* state, int64_t count, int64_t* E) {
    double mx = 0.0;
    for (int64_t k = 0; k < count; ++k) {
        double a = fabs(state[k]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0 || !isfinite(mx)) return;
    int e;
    frexp(mx, &e);
    for (int64_t k = 0; k < count; ++k) state[k] = ldexp(state[k], -e);
    *E += e;
}

static void increments(const double* x, int64_t n_pts, int64_t d, double* dx) {
    for (int64_t i = 0; i + 1 < n_pts; ++i)
        for (int64_t k = 0; k < d; ++k) dx[i * d + k] = x[(i + 1) * d + k] - x[i * d + k];
}

static double dot(const double* a, const double* b, int64_t d) {
    double s = 0.0;
    for (int64_t k = 0; k < d; ++k) s += a[k] * b[k];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Finite differences                                                        */
/* ------------------------------------------------------------------------ */
static int fd_rule(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts, int64_t d,
                   int lam, int second, double* mant, int64_t* expo) {
    if (nx_pts < 1 || ny_pts < 1 || d < 1 || lam < 0 || lam > 12) return -1;
    int64_t lx = nx_pts - 1, ly = ny_pts - 1;
    *expo = 0;
    if (lx == 0 || ly == 0) { *mant = 1.0; return 0; }
    int64_t r = (int64_t)1 << lam;
    int64_t m = lx * r, n = ly * r;
    double* dx = malloc(sizeof(double) * lx * d);
    double* dy = malloc(sizeof(double) * ly * d);
    double* prev = malloc(sizeof(double) * (n + 1)); /* k(s_i, .)   */
    double* cur = malloc(sizeof(double) * (n + 1));  /* k(s_{i+1}, .) */
    increments(x, nx_pts, d, dx);
    increments(y, ny_pts, d, dy);
    for (int64_t j = 0; j <= n; ++j) prev[j] = 1.0;
    for (int64_t i = 0; i < m; ++i) {
        cur[0] = 1.0;
        for (int64_t j = 0; j < n; ++j) {
            /* refined increments are the segment increments divided by 2^lam */
            double inner = dot(dx + (i / r) * d, dy + (j / r) * d, d) / (double)(r * r);
            cur[j + 1] = cur[j] + prev[j + 1] - prev[j] + 0.5 * inner * (cur[j] + prev[j + 1]);
            if (second) /* + c^2/12 (k(s_{i+1},t_j) + k(s_i,t_{j+1}) + k(s_i,t_j)) */
                cur[j + 1] += inner * inner / 12.0 * (cur[j] + prev[j + 1] + prev[j]);
        }
        double* t = prev; prev = cur; cur = t;
    }
    *mant = prev[n];
    free(dx); free(dy); free(prev); free(cur);
    return 0;
}

int sko_fd(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts, int64_t d,
           int lam, double* mant, int64_t* expo) {
    return fd_rule(x, nx_pts, y, ny_pts, d, lam, 0, mant, expo);
}

int sko_fd2(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts, int64_t d,
            int lam, double* mant, int64_t* expo) {
    return fd_rule(x, nx_pts, y, ny_pts, d, lam, 1, mant, expo);
}

/* ------------------------------------------------------------------------ */
/* Polynomial approximation scheme                                           */
/* ------------------------------------------------------------------------ */
/* f32model != 0: the same scheme with the increments, the cell constants
   and, after every cell, the edge coefficients of degree 2 and above rounded
   to FP32 (arithmetic in FP64; degrees 0 and 1, the corner value and the
   slope, stay FP64).  Its distance from the FP64 scheme estimates how far an
   evaluation with that FP32 state can be trusted on a pair: the pair's
   conditioning floor (a diagnostic for FP32 parity tests, not part of the
   scheme). */
static int approx_impl(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts,
                       int64_t d, int N, int f32model, double* mant, int64_t* expo) {
    if (nx_pts < 1 || ny_pts < 1 || d < 1 || N < 2 || N > SKO_NMAX) return -1;
    int64_t lx = nx_pts - 1, ly = ny_pts - 1;
    *expo = 0;
    if (lx == 0 || ly == 0) { *mant = 1.0; return 0; }
    const int M = N + 1;
    /* factorial factors of the truncated map: A[n][k] = k!/((n-k)! n!),
       B[n][k] = k!/((n+k)! n!) */
    double A[SKO_NMAX + 1][SKO_NMAX + 1], B[SKO_NMAX + 1][SKO_NMAX + 1];
    for (int n = 0; n <= N; ++n)
        for (int k = 0; k <= N; ++k) {
            A[n][k] = (k <= n) ? fact(k) / (fact(n - k) * fact(n)) : 0.0;
            B[n][k] = fact(k) / (fact(n + k) * fact(n));
        }
    double* dx = malloc(sizeof(double) * lx * d);
    double* dy = malloc(sizeof(double) * ly * d);
    /* state: p[i][0..N] (bottom edge of the current row) then q[0..N] */
    double* st = malloc(sizeof(double) * (lx + 1) * M);
    double* q = st + lx * M;
    increments(x, nx_pts, d, dx);
    increments(y, ny_pts, d, dy);
    if (f32model) {
        for (int64_t k = 0; k < lx * d; ++k) dx[k] = (double)(float)dx[k];
        for (int64_t k = 0; k < ly * d; ++k) dy[k] = (double)(float)dy[k];
    }
    for (int64_t i = 0; i < lx; ++i) {
        for (int n = 0; n < M; ++n) st[i * M + n] = 0.0;
        st[i * M] = 1.0;
    }
    int64_t E = 0;
    double pt[SKO_NMAX + 1], qt[SKO_NMAX + 1], cp[SKO_NMAX + 1];
    for (int64_t j = 0; j < ly; ++j) {
        for (int n = 0; n < M; ++n) q[n] = 0.0;
        q[0] = ldexp(1.0, (int)-E); /* q^{0,j} = 1 in the current scale */
        for (int64_t i = 0; i < lx; ++i) {
            double* p = st + i * M;
            double c = dot(dx + i * d, dy + j * d, d);
            if (f32model) c = (double)(float)c;
            cp[0] = 1.0;
            for (int n = 1; n <= N; ++n) cp[n] = cp[n - 1] * c;
            for (int n = 0; n <= N; ++n) {
                double a = 0.0, b = 0.0;
                for (int k = 0; k <= n; ++k) {
                    a += p[k] * cp[n - k] * A[n][k];
                    b += q[k] * cp[n - k] * A[n][k];
                }
                for (int k = 1; k <= N; ++k) {
                    a += q[k] * cp[n] * B[n][k];
                    b += p[k] * cp[n] * B[n][k];
                }
                pt[n] = (f32model && n >= 2) ? (double)(float)a : a;
                qt[n] = (f32model && n >= 2) ? (double)(float)b : b;
            }
            memcpy(p, pt, sizeof(double) * M);
            memcpy(q, qt, sizeof(double) * M);
        }
        rescale(st, (lx + 1) * M, &E);
    }
    double top = 0.0, right = 0.0;
    for (int n = 0; n <= N; ++n) { top += st[(lx - 1) * M + n]; right += q[n]; }
    *mant = 0.5 * (top + right);
    *expo = E;
    free(dx); free(dy); free(st);
    return 0;
}

int sko_approx(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts, int64_t d,
               int N, double* mant, int64_t* expo) {
    return approx_impl(x, nx_pts, y, ny_pts, d, N, 0, mant, expo);
}

int sko_approx_f32model(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts,
                        int64_t d, int N, double* mant, int64_t* expo) {
    return approx_impl(x, nx_pts, y, ny_pts, d, N, 1, mant, expo);
}

/* ------------------------------------------------------------------------ */
/* Polynomial interpolation scheme                                           */
/* ------------------------------------------------------------------------ */
/* 0F1(b; z) = sum_n z^n / ((b)_n n!), summed until the term is below 2^-60 of
   the running sum */
static double hyp0f1(double b, double z) {
    double term = 1.0, sum = 1.0;
    for (int n = 0; n < 100000; ++n) {
        term *= z / ((b + n) * (n + 1.0));
        sum += term;
        if (fabs(term) <= ldexp(fabs(sum), -60)) break;
    }
    return sum;
}

/* LU factorisation with partial pivoting of an M x M matrix (row-major) */
static int lu_factor(double* a, int* piv, int M) {
    for (int k = 0; k < M; ++k) {
        int p = k;
        for (int i = k + 1; i < M; ++i)
            if (fabs(a[i * M + k]) > fabs(a[p * M + k])) p = i;
        piv[k] = p;
        if (a[p * M + k] == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < M; ++j) {
                double t = a[k * M + j]; a[k * M + j] = a[p * M + j]; a[p * M + j] = t;
            }
        for (int i = k + 1; i < M; ++i) {
            a[i * M + k] /= a[k * M + k];
            for (int j = k + 1; j < M; ++j) a[i * M + j] -= a[i * M + k] * a[k * M + j];
        }
    }
    return 0;
}

static void lu_solve(const double* lu, const int* piv, int M, double* b) {
    for (int k = 0; k < M; ++k) {
        double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t;
    }
    for (int i = 1; i < M; ++i)
        for (int j = 0; j < i; ++j) b[i] -= lu[i * M + j] * b[j];
    for (int i = M - 1; i >= 0; --i) {
        for (int j = i + 1; j < M; ++j) b[i] -= lu[i * M + j] * b[j];
        b[i] /= lu[i * M + i];
    }
}

int sko_interp(const double* x, int64_t nx_pts, const double* y, int64_t ny_pts, int64_t d,
               int N, double* mant, int64_t* expo) {
    if (nx_pts < 1 || ny_pts < 1 || d < 1 || N < 2 || N > SKO_NMAX) return -1;
    int64_t lx = nx_pts - 1, ly = ny_pts - 1;
    *expo = 0;
    if (lx == 0 || ly == 0) { *mant = 1.0; return 0; }
    const int M = N + 1;
    /* Chebyshev extrema of [0,1] (unit partition), m = 0..N, and the
       Vandermonde matrix of the monomial basis at them */
    double u[SKO_NMAX + 1], upow[SKO_NMAX + 1][SKO_NMAX + 1];
    double V[(SKO_NMAX + 1) * (SKO_NMAX + 1)];
    int piv[SKO_NMAX + 1];
    for (int m = 0; m <= N; ++m) {
        u[m] = 0.5 * cos(M_PI * m / N) + 0.5;
        upow[m][0] = 1.0;
        for (int n = 1; n <= N; ++n) upow[m][n] = upow[m][n - 1] * u[m];
        for (int n = 0; n <= N; ++n) V[m * M + n] = upow[m][n];
    }
    if (lu_factor(V, piv, M) != 0) return -2;
    double* dx = malloc(sizeof(double) * lx * d);
    double* dy = malloc(sizeof(double) * ly * d);
    double* st = malloc(sizeof(double) * (lx + 1) * M);
    double* h = st + lx * M;
    increments(x, nx_pts, d, dx);
    increments(y, ny_pts, d, dy);
    for (int64_t i = 0; i < lx; ++i) {
        for (int n = 0; n < M; ++n) st[i * M + n] = 0.0;
        st[i * M] = 1.0;
    }
    int64_t E = 0;
    double top[SKO_NMAX + 1], right[SKO_NMAX + 1], F[SKO_NMAX + 2];
    for (int64_t j = 0; j < ly; ++j) {
        for (int n = 0; n < M; ++n) h[n] = 0.0;
        h[0] = ldexp(1.0, (int)-E);
        for (int64_t i = 0; i < lx; ++i) {
            double* g = st + i * M;
            double c = dot(dx + i * d, dy + j * d, d);
            for (int m = 0; m <= N; ++m) {
                /* top edge at s - a = u_m, t - c = 1; right edge at s - a = 1,
                   t - c = u_m; both have z = C u_m */
                double z = c * u[m];
                for (int n = 0; n <= N; ++n) F[n] = hyp0f1(n + 1.0, z);
                double tv = g[0] * F[0], rv = g[0] * F[0];
                for (int n = 1; n <= N; ++n) {
                    tv += (g[n] * upow[m][n] + h[n]) * F[n];
                    rv += (g[n] + h[n] * upow[m][n]) * F[n];
                }
                top[m] = tv;
                right[m] = rv;
            }
            lu_solve(V, piv, M, top);
            lu_solve(V, piv, M, right);
            memcpy(g, top, sizeof(double) * M);
            memcpy(h, right, sizeof(double) * M);
        }
        rescale(st, (lx + 1) * M, &E);
    }
    double tv = 0.0, rv = 0.0;
    for (int n = 0; n <= N; ++n) { tv += st[(lx - 1) * M + n]; rv += h[n]; }
    *mant = 0.5 * (tv + rv);
    *expo = E;
    free(dx); free(dy); free(st);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Batches (OpenMP over pairs)                                               */
/* ------------------------------------------------------------------------ */
enum { SKO_FD = 0, SKO_APPROX = 1, SKO_INTERP = 2, SKO_FD2 = 3, SKO_APPROX_F32MODEL = 4 };

static int run_one(int scheme, int order, const double* x, int64_t nx, const double* y,
                   int64_t ny, int64_t d, double* mant, int64_t* expo) {
    switch (scheme) {
        case SKO_FD: return sko_fd(x, nx, y, ny, d, order, mant, expo);
        case SKO_APPROX: return sko_approx(x, nx, y, ny, d, order, mant, expo);
        case SKO_INTERP: return sko_interp(x, nx, y, ny, d, order, mant, expo);
        case SKO_FD2: return sko_fd2(x, nx, y, ny, d, order, mant, expo);
        case SKO_APPROX_F32MODEL: return sko_approx_f32model(x, nx, y, ny, d, order, mant, expo);
        default: return -1;
    }
}

/* K[a*ny + b] for a < nx, b < ny; X: (nx, lx_pts, d), Y: (ny, ly_pts, d) */
int sko_gram(int scheme, int order, const double* X, int64_t nx, int64_t lx_pts,
             const double* Y, int64_t ny, int64_t ly_pts, int64_t d, double* mant,
             int64_t* expo, int nthreads) {
    int err = 0;
    int64_t total = nx * ny;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
    for (int64_t ab = 0; ab < total; ++ab) {
        int64_t a = ab / ny, b = ab % ny;
        err |= (run_one(scheme, order, X + a * lx_pts * d, lx_pts, Y + b * ly_pts * d, ly_pts,
                        d, mant + ab, expo + ab) != 0);
    }
    return err ? -1 : 0;
}

/* pairs: x of pair p is Xcat[xoff[p] .. xoff[p+1]) points, likewise y */
int sko_pairs(int scheme, int order, const double* Xcat, const int64_t* xoff,
              const double* Ycat, const int64_t* yoff, int64_t npairs, int64_t d,
              double* mant, int64_t* expo, int nthreads) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
    for (int64_t p = 0; p < npairs; ++p) {
        err |= (run_one(scheme, order, Xcat + xoff[p] * d, xoff[p + 1] - xoff[p],
                        Ycat + yoff[p] * d, yoff[p + 1] - yoff[p], d, mant + p,
                        expo + p) != 0);
    }
    return err ? -1 : 0;
}
