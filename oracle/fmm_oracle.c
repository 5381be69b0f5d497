/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference for the block-based restarted
 * narrow-band fast marching method of J. Yang, "An easily-implemented,
 * block-based fast marching method with superior sequential and parallel
 * performance" (2018).  It exists to check the HIP library; it shares no code,
 * header, table or helper with it, and the product path never loads it.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * use it.
 *
 * Contents (each function cites the passage it follows):
 *   orc_fmm_{f64,f32}        baseline single-heap FMM (Sec. 2.1 + Sec. 2.2)
 *   orc_block_fmm_{f64,f32}  multi-block restarted method, Alg. 6 verbatim
 *   orc_gauss_seidel         fixed point of the upwind scheme Eq. (2)-(3) by
 *                            ordered sweeps (no heap, no tags)
 *   orc_jacobi               the same fixed point by order-free iteration
 *   orc_mlp_*                FP64 reference of the stride network
 *
 * All routines return 0 or a negative ORC_E* code.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)

/* Point categories of Sec. 2.1 with KNOWN split as in Sec. 2.2. */
enum { ORC_FAR = 0, ORC_BAND = 1, ORC_KNOWN_FIX = 2, ORC_KNOWN_NEW = 3 };

#define REAL double
#define SFX f64
#define RSQRT sqrt
#include "fmm_oracle_impl.h"
#undef REAL
#undef SFX
#undef RSQRT

#define REAL float
#define SFX f32
#define RSQRT sqrtf
#include "fmm_oracle_impl.h"
#undef REAL
#undef SFX
#undef RSQRT

/* ------------------------------------------------------------------------ */
/* Fixed point of the Godunov upwind scheme, Eq. (2) with Eq. (3).           */
/*                                                                           */
/* The discrete solution is the function that equals psi0 on the sources    */
/* and, at every other point p with F_p > 0, satisfies                       */
/*     sum_d max((psi_p - a_d) / h, 0)^2 = 1 / F_p^2,                        */
/*     a_d = min(psi(p - e_d), psi(p + e_d)) over neighbours inside the grid. */
/* The local equation is solved here without the closed-form root: the left  */
/* side is increasing in psi_p above min a_d, so the root is bracketed by    */
/* [min a_d, min a_d + h/F_p] and found by bisection down to adjacent        */
/* doubles.  This keeps the check independent of Alg. 3's formula.           */
/* ------------------------------------------------------------------------ */
static double godunov_residual(double t, const double a[3], double rhs)
{
    double s = 0;
    for (int d = 0; d < 3; ++d) {
        double u = t - a[d];
        if (u > 0) s += u * u;
    }
    return s - rhs;
}

static double godunov_local(const double a[3], double h, double f)
{
    double lo = a[0];
    for (int d = 1; d < 3; ++d)
        if (a[d] < lo) lo = a[d];
    if (!isfinite(lo)) return INFINITY;
    const double rhs = (h / f) * (h / f);
    double hi = lo + h / f;
    /* make sure the bracket holds despite rounding in lo + h/f */
    while (godunov_residual(hi, a, rhs) < 0) hi = nextafter(hi, INFINITY);
    for (;;) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (godunov_residual(mid, a, rhs) < 0) lo = mid;
        else hi = mid;
    }
    return hi;
}

static void axis_minima(const double *psi, int64_t nx, int64_t ny, int64_t nz, int64_t i,
                        int64_t j, int64_t k, double a[3])
{
    const int64_t p = i + nx * (j + ny * k);
    a[0] = a[1] = a[2] = INFINITY;
    if (i > 0 && psi[p - 1] < a[0]) a[0] = psi[p - 1];
    if (i < nx - 1 && psi[p + 1] < a[0]) a[0] = psi[p + 1];
    if (j > 0 && psi[p - nx] < a[1]) a[1] = psi[p - nx];
    if (j < ny - 1 && psi[p + nx] < a[1]) a[1] = psi[p + nx];
    if (k > 0 && psi[p - nx * ny] < a[2]) a[2] = psi[p - nx * ny];
    if (k < nz - 1 && psi[p + nx * ny] < a[2]) a[2] = psi[p + nx * ny];
}

static int fixed_point_setup(int64_t nx, int64_t ny, int64_t nz, double h, int32_t nsrc,
                             const int64_t *src_idx, const double *src_val, double *psi,
                             uint8_t *is_src)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(h > 0) || nsrc <= 0) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    for (int64_t p = 0; p < N; ++p) {
        psi[p] = INFINITY;
        is_src[p] = 0;
    }
    for (int32_t s = 0; s < nsrc; ++s) {
        if (src_idx[s] < 0 || src_idx[s] >= N || !(src_val[s] >= 0)) return ORC_EINVAL;
        if (src_val[s] < psi[src_idx[s]]) psi[src_idx[s]] = src_val[s];
        is_src[src_idx[s]] = 1;
    }
    return 0;
}

/* Gauss-Seidel: sweep the grid in the 8 axis orderings in turn, replacing
   psi_p by min(psi_p, local root), until a full round of 8 sweeps changes
   nothing.  sweeps_out receives the number of sweeps done. */
int orc_gauss_seidel(int64_t nx, int64_t ny, int64_t nz, double h, const double *F, int32_t nsrc,
                     const int64_t *src_idx, const double *src_val, int64_t max_sweeps,
                     double *psi, int64_t *sweeps_out)
{
    const int64_t N = nx * ny * nz;
    uint8_t *is_src = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    if (!is_src) return ORC_ENOMEM;
    int rc = fixed_point_setup(nx, ny, nz, h, nsrc, src_idx, src_val, psi, is_src);
    int64_t sweeps = 0;
    int changed_in_round = 1;
    while (rc == 0 && changed_in_round) {
        changed_in_round = 0;
        for (int order = 0; order < 8; ++order) {
            if (max_sweeps > 0 && sweeps >= max_sweeps) {
                rc = ORC_ENOCONV;
                break;
            }
            ++sweeps;
            for (int64_t kk = 0; kk < nz; ++kk)
                for (int64_t jj = 0; jj < ny; ++jj)
                    for (int64_t ii = 0; ii < nx; ++ii) {
                        int64_t i = (order & 1) ? nx - 1 - ii : ii;
                        int64_t j = (order & 2) ? ny - 1 - jj : jj;
                        int64_t k = (order & 4) ? nz - 1 - kk : kk;
                        int64_t p = i + nx * (j + ny * k);
                        if (is_src[p] || F[p] == 0) continue;
                        double a[3];
                        axis_minima(psi, nx, ny, nz, i, j, k, a);
                        double t = godunov_local(a, h, F[p]);
                        if (t < psi[p]) {
                            psi[p] = t;
                            changed_in_round = 1;
                        }
                    }
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    free(is_src);
    return rc;
}

/* Jacobi: every point is updated from the previous iterate at once, with no
   ordering of any kind, until an iteration changes nothing. */
int orc_jacobi(int64_t nx, int64_t ny, int64_t nz, double h, const double *F, int32_t nsrc,
               const int64_t *src_idx, const double *src_val, int64_t max_iters, double *psi,
               int64_t *iters_out)
{
    const int64_t N = nx * ny * nz;
    uint8_t *is_src = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    double *next = (double *)malloc((size_t)(N > 0 ? N : 1) * sizeof(double));
    if (!is_src || !next) {
        free(is_src);
        free(next);
        return ORC_ENOMEM;
    }
    int rc = fixed_point_setup(nx, ny, nz, h, nsrc, src_idx, src_val, psi, is_src);
    int64_t it = 0;
    int changed = 1;
    while (rc == 0 && changed) {
        if (max_iters > 0 && it >= max_iters) {
            rc = ORC_ENOCONV;
            break;
        }
        ++it;
        changed = 0;
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t p = i + nx * (j + ny * k);
                    next[p] = psi[p];
                    if (is_src[p] || F[p] == 0) continue;
                    double a[3];
                    axis_minima(psi, nx, ny, nz, i, j, k, a);
                    double t = godunov_local(a, h, F[p]);
                    if (t < next[p]) {
                        next[p] = t;
                        changed = 1;
                    }
                }
        memcpy(psi, next, (size_t)N * sizeof(double));
    }
    if (iters_out) *iters_out = it;
    free(is_src);
    free(next);
    return rc;
}
