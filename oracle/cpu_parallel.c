/*
 * cpu_parallel.c -- TEST AND BENCHMARK INFRASTRUCTURE ONLY.
 *
 * The paper's parallel CPU solver (Sec. 2.7, measured in Sec. 3.5-3.6): the
 * block-based restarted method of Alg. 6 with the marching step and the
 * exchanging step of every restart spread over the blocks by OpenMP threads,
 * as a second CPU baseline beside the single-thread oracle.
 *
 * The per-block steps are the block reference's own (march_one, exchange_one
 * in fmm_oracle_impl.h).  Within one step the blocks are independent: a march
 * writes only its own block and raises flags on its neighbours, an exchange
 * writes only its own block and reads its neighbours' interior points and
 * Upsilon lists, which no exchange writes (Sec. 2.7).  So the result is bitwise
 * that of orc_block_fmm_f64, whatever the number of threads; a test checks it.
 * Nothing here is shared with the HIP library, and the product never loads it.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)

enum { ORC_FAR = 0, ORC_BAND = 1, ORC_KNOWN_FIX = 2, ORC_KNOWN_NEW = 3 };

#define REAL double
#define SFX par_f64
#define RSQRT sqrt
#include "fmm_oracle_impl.h"
#undef REAL
#undef SFX
#undef RSQRT

typedef blk_t_par_f64 pblk_t;

/* FP64 block method on `threads` OpenMP threads (0 = the runtime's default).
   Arguments as orc_block_fmm_f64 with a fixed stride; *threads_used reports the
   team size. */
int cpu_block_fmm_par_f64(int64_t nx, int64_t ny, int64_t nz, double h, const double *F,
                          int32_t nsrc, const int64_t *src_idx, const double *src_val,
                          int32_t B, double stride, double width, int32_t threads,
                          int64_t max_restarts, double *psi, int64_t *restarts_out,
                          int64_t *pops_out, int32_t *threads_used)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(h > 0) || nsrc <= 0 || B <= 0) return ORC_EINVAL;
    if (nx % B || ny % B || nz % B || !(stride > 0)) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    for (int32_t s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || src_idx[s] >= N || !(src_val[s] >= 0)) return ORC_EINVAL;
    const int64_t mx = nx / B, my = ny / B, mz = nz / B, nblk = mx * my * mz;
    const double hr = h;
    int rc = 0;
    if (threads > 0) omp_set_num_threads(threads);
    pblk_t *blk = (pblk_t *)calloc((size_t)nblk, sizeof(pblk_t));
    int64_t *list = (int64_t *)malloc((size_t)nblk * sizeof(int64_t));
    if (!blk || !list) {
        free(blk);
        free(list);
        return ORC_ENOMEM;
    }
    int64_t r = 0, pops = 0;
    int team = 1;
    if ((rc = blocks_init_par_f64(blk, nx, ny, B, mx, my, mz, nsrc, src_idx, src_val)) != 0)
        goto done;

    for (;;) {
        ++r;
        if (max_restarts > 0 && r > max_restarts) {
            rc = ORC_ENOCONV;
            break;
        }
        double bound = (double)r * stride;
        if (bound > width) bound = width;

        /* marching step over the blocks with A = TRUE */
        int64_t n = 0;
        for (int64_t ib = 0; ib < nblk; ++ib)
            if (blk[ib].A) list[n++] = ib;
        int err = 0;
#pragma omp parallel reduction(+ : pops) reduction(| : err)
        {
#pragma omp single
            team = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
            for (int64_t k = 0; k < n; ++k)
                err |= march_one_par_f64(blk, list[k], B, mx, my, mz, nx, ny, hr, F, bound, width,
                                         0, &pops) != 0;
        }
        if (err) {
            rc = ORC_ENOMEM;
            break;
        }

        /* exchanging step over the blocks with any C = TRUE */
        n = 0;
        for (int64_t ib = 0; ib < nblk; ++ib) {
            const pblk_t *b = &blk[ib];
            if (b->C[0] | b->C[1] | b->C[2] | b->C[3] | b->C[4] | b->C[5]) list[n++] = ib;
        }
#pragma omp parallel for schedule(dynamic, 4) reduction(| : err)
        for (int64_t k = 0; k < n; ++k) err |= exchange_one_par_f64(blk, list[k], B, mx, my, width) != 0;
        if (err) {
            rc = ORC_ENOMEM;
            break;
        }

        int any = 0;
        for (int64_t ib = 0; ib < nblk && !any; ++ib) any = blk[ib].A;
        if (!any) break;
    }
    if (rc == 0) blocks_gather_par_f64(blk, nx, ny, B, nblk, psi);
    if (restarts_out) *restarts_out = r;
    if (pops_out) *pops_out = pops;
    if (threads_used) *threads_used = team;
done:
    for (int64_t ib = 0; ib < nblk; ++ib) blk_free_par_f64(&blk[ib]);
    free(blk);
    free(list);
    return rc;
}
