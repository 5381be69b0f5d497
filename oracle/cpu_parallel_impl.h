/*
 * cpu_parallel_impl.h -- TEST AND BENCHMARK INFRASTRUCTURE ONLY (see cpu_parallel.c).
 *
 * Driver of the parallel block solver, instantiated by cpu_parallel.c for one
 * precision: REAL is the arithmetic type, SFX the suffix of the per-block steps
 * of fmm_oracle_impl.h it calls (par_f64 or par_f32).
 */

/* Block method on `threads` OpenMP threads (0 = the runtime's default).  Arguments
   as orc_block_fmm_{f64,f32} with a fixed stride; *threads_used reports the team
   size.  cpu_block_fmm_par_f64 / cpu_block_fmm_par_f32. */
int PAR_CAT(cpu_block_fmm, SFX)(int64_t nx, int64_t ny, int64_t nz, double h, const REAL *F,
                                int32_t nsrc, const int64_t *src_idx, const REAL *src_val,
                                int32_t B, double stride, double width, int32_t threads,
                                int64_t max_restarts, REAL *psi, int64_t *restarts_out,
                                int64_t *pops_out, int32_t *threads_used)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(h > 0) || nsrc <= 0 || B <= 0) return ORC_EINVAL;
    if (nx % B || ny % B || nz % B || !(stride > 0)) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    for (int32_t s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || src_idx[s] >= N || !(src_val[s] >= 0)) return ORC_EINVAL;
    const int64_t mx = nx / B, my = ny / B, mz = nz / B, nblk = mx * my * mz;
    const REAL hr = (REAL)h;
    int rc = 0;
    if (threads > 0) omp_set_num_threads(threads);
    PFN(blk_t) *blk = (PFN(blk_t) *)calloc((size_t)nblk, sizeof(PFN(blk_t)));
    int64_t *list = (int64_t *)malloc((size_t)nblk * sizeof(int64_t));
    if (!blk || !list) {
        free(blk);
        free(list);
        return ORC_ENOMEM;
    }
    int64_t r = 0, pops = 0;
    int team = 1;
    if ((rc = PFN(blocks_init)(blk, nx, ny, B, mx, my, mz, nsrc, src_idx, src_val)) != 0)
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
                err |= PFN(march_one)(blk, list[k], B, mx, my, mz, nx, ny, hr, F, bound, width, 0,
                                      &pops) != 0;
        }
        if (err) {
            rc = ORC_ENOMEM;
            break;
        }

        /* exchanging step over the blocks with any C = TRUE */
        n = 0;
        for (int64_t ib = 0; ib < nblk; ++ib) {
            const PFN(blk_t) *b = &blk[ib];
            if (b->C[0] | b->C[1] | b->C[2] | b->C[3] | b->C[4] | b->C[5]) list[n++] = ib;
        }
#pragma omp parallel for schedule(dynamic, 4) reduction(| : err)
        for (int64_t k = 0; k < n; ++k) err |= PFN(exchange_one)(blk, list[k], B, mx, my, width) != 0;
        if (err) {
            rc = ORC_ENOMEM;
            break;
        }

        int any = 0;
        for (int64_t ib = 0; ib < nblk && !any; ++ib) any = blk[ib].A;
        if (!any) break;
    }
    if (rc == 0) PFN(blocks_gather)(blk, nx, ny, B, nblk, psi);
    if (restarts_out) *restarts_out = r;
    if (pops_out) *pops_out = pops;
    if (threads_used) *threads_used = team;
done:
    for (int64_t ib = 0; ib < nblk; ++ib) PFN(blk_free)(&blk[ib]);
    free(blk);
    free(list);
    return rc;
}
