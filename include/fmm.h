/*
 * fmm.h -- C ABI of the MI355X (gfx950) block-based restarted narrow-band
 * fast marching library.
 *
 * The library solves the eikonal boundary-value problem |grad psi| F = 1 with
 * psi = psi0 on a set of source points (Yang 2018, Eq. (1)), discretised by
 * the first-order Godunov upwind scheme on a uniform grid (Eq. (2)-(3)), with
 * the block-based method of the paper: the grid is cut into B^3 blocks padded
 * by one ghost layer (Sec. 2.3), each block marches its own narrow band up to
 * a global bound that rises by a stride at every restart (Sec. 2.4, Alg. 4,
 * Alg. 6), blocks then exchange ghost faces (Alg. 5), and activation flags
 * skip idle blocks in both steps (Sec. 2.5, 2.6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Grid layout: linear index of point (i, j, k) is i + nx*(j + ny*k), i.e.
 *    a C-contiguous array of shape (nz, ny, nx).  Grid spacing h in all three
 *    directions.
 *  * Buffers named *_dev are device memory owned by the caller (for example
 *    torch tensors); the library never frees them.  Host arrays are read
 *    during the call only and may be freed when it returns.
 *  * Precision: FMM_F32 means F and psi are float, FMM_F64 means double.  The
 *    solver computes in that precision; the restart bound is kept in double.
 *  * Streams: work is queued on hip_stream (a hipStream_t; NULL = the null
 *    stream).  Every solve entry point returns after the result is complete,
 *    unless noted.
 *  * Errors: every int-returning function returns FMM_OK (0) or a negative
 *    FMM_E* code; fmm_strerror() gives text, fmm_last_error_detail() the
 *    message of the last failure on the calling thread.  No C++ exception
 *    crosses this boundary.
 *  * Library workspace (blocked tiles, bands, flags, lists) is allocated by the
 *    library from a per-device cache and reused across calls.
 *  * Calls are thread-compatible, not thread-safe: do not run two solves on the
 *    same device at once from different threads.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_OK 0
#define FMM_EINVAL (-1)   /* invalid argument                                   */
#define FMM_ENOMEM (-2)   /* device or host allocation failed                   */
#define FMM_EHIP (-3)     /* HIP runtime error; see fmm_last_error_detail()     */
#define FMM_ENOCONV (-4)  /* restart cap reached, or a device watchdog fired    */
#define FMM_ENOTSUP (-5)  /* unsupported combination (block size, launch mode)  */

typedef enum { FMM_F32 = 0, FMM_F64 = 1 } fmm_dtype;

/* Stride policy of the restart driver. */
typedef enum {
    FMM_STRIDE_FIXED = 0,   /* bound_r = min(r * stride, width)            (Alg. 6) */
    FMM_STRIDE_LEARNED = 1, /* bound_r = bound_{r-1} + m_r * stride, m_r from the
                               stride network evaluated on the device at the end
                               of restart r-1; falls back to m_r = 1 when the
                               weights are absent or the output is not finite */
    FMM_STRIDE_SCHEDULE = 2 /* a given bound sequence (fmm_options.bounds):
                               bound_r = min(bounds[r-1], width) for r <= nbounds, then
                               min(bounds[nbounds-1] + (r - nbounds) * stride, width);
                               any non-decreasing sequence gives the same psi, only the
                               restarts differ (used to replay and explore strides) */
} fmm_stride_mode;

/* Launch strategy of the restart loop. */
typedef enum {
    FMM_LAUNCH_PERSISTENT = 0, /* one cooperative persistent kernel runs every restart */
    FMM_LAUNCH_HOST = 1        /* one march and one exchange kernel per restart,
                                  driven from the host (diagnostic)                 */
} fmm_launch_mode;

/* A point of Gamma (Alg. 1): grid index and its value psi0 >= 0. */
typedef struct {
    int64_t i, j, k;
    double psi0;
} fmm_source;

/* Optional knobs; fmm_options_default() fills the defaults noted here. */
typedef struct {
    double width;             /* width_band of Alg. 4 / Alg. 5; +inf (default) = full solve */
    int32_t stride_mode;      /* fmm_stride_mode, default FIXED                               */
    const void *mlp_weights;  /* device pointer to FMM_MLP_BLOB_FLOATS floats (see below);
                                 NULL = fixed stride                                         */
    int32_t waves_per_block;  /* 64-lane waves cooperating on one block: 1, 2 or 4; 0 = 1     */
    int32_t launch_mode;      /* fmm_launch_mode, default PERSISTENT                          */
    int64_t max_restarts;     /* watchdog; 0 = default (1e7)                                  */
    int32_t grid_limit;       /* persistent workgroups cap; 0 = occupancy-derived              */
    void *trace_dev;          /* nullable device buffer of trace_cap fmm_trace_row             */
    int32_t trace_cap;        /* rows available in trace_dev                                   */
    int32_t band_lds_cap;     /* diagnostic: band slots kept in LDS while a block marches, a
                                 multiple of 512; 0 = the default (1024); slots beyond it are
                                 kept in device memory                                         */
    const double *bounds;     /* FMM_STRIDE_SCHEDULE: host array of nbounds finite, positive,
                                 non-decreasing bounds, copied during the call; else unused    */
    int32_t nbounds;          /* 1 .. 2^24 for FMM_STRIDE_SCHEDULE                            */
    int32_t per_problem_restarts; /* 1: the problems of a batch restart on their own (no
                                 barrier shared between problems; fixed stride, persistent
                                 launch, at most 2^20 - 2^17 blocks per problem); 0 (default):
                                 one restart sequence for the whole batch                     */
} fmm_options;

/* Solve statistics (host struct, filled after the call). */
typedef struct {
    int64_t restarts;          /* iterations of the loop of Alg. 6                          */
    int64_t pops;              /* Remove_Min events over all blocks (ghost points included) */
    int64_t march_calls;       /* March_Narrow_Band calls (blocks with A = TRUE)            */
    int64_t exchange_calls;    /* Integrate_Ghost_Cell_Data calls (blocks with any C)       */
    int64_t tile_loads;        /* march calls that had work below the bound                 */
    double final_bound;        /* bound of the last restart                                 */
    double elapsed_ms;         /* device time from the first to the last kernel             */
    double loop_ms;            /* device time of the restart loop alone (the persistent
                                  kernel, or all per-phase kernels in host mode)            */
    int32_t grid;              /* persistent workgroups used (0 in host mode)               */
    int32_t block;             /* block edge B used                                        */
    int32_t waves_per_block;   /* waves per block used                                     */
    int32_t reserved;
} fmm_stats;

/* One row per restart, written when fmm_options.trace_dev is given:
   the inputs of the stride network and what the restart cost. */
#define FMM_NFEAT 12
typedef struct {
    float feat[FMM_NFEAT];   /* raw features at the end of the restart (see fmm_mlp_*)   */
    double bound;            /* bound of this restart                                     */
    double stride_used;      /* bound - previous bound                                    */
    int64_t pops;            /* Remove_Min events in this restart                          */
    int64_t t_start;         /* device wall clock (100 MHz) at the start of the restart    */
    int64_t t_end;           /* and at its end                                             */
    int32_t active;          /* blocks in the march list of this restart                   */
    int32_t next_active;     /* blocks in the march list of the next restart               */
    double min_popped;       /* smallest value accepted (popped) in this restart; +inf when
                                none: a value below an earlier bound marks a late correction */
} fmm_trace_row;

void fmm_options_default(fmm_options *opt);

/*
 * Solve one problem (the main procedure of Alg. 6 with Alg. 1-5).
 *
 *   nx, ny, nz   grid points per axis (> 0, each divisible by block)
 *   h            grid spacing (> 0, finite)
 *   dtype        FMM_F32 or FMM_F64: element type of F_dev and psi_dev
 *   F_dev        speed F >= 0 at every point, nx*ny*nz elements; F = 0 marks an
 *                obstacle where the quadratic is never solved (paper Sec. 3.3)
 *   src, nsrc    host array of nsrc >= 1 points of Gamma, each inside the grid,
 *                psi0 >= 0 finite; a repeated point keeps the smallest psi0
 *   block        block edge B: 4, 8, 16 or 32 (the paper's dimBlock); 32^3 blocks take
 *                one wave per block and march their tile in device memory (a padded
 *                FP32 tile does not fit in LDS), FMM_ENOTSUP with more waves
 *   stride       restart stride (> 0, +inf allowed = the non-restarted block
 *                method of Sec. 2.3)
 *   psi_dev      output, nx*ny*nz elements; points never reached are +inf
 *   hip_stream   stream to queue on
 *   opt          nullable: defaults
 *   stats        nullable: filled on success
 */
int fmm_solve(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
              const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
              void *hip_stream, const fmm_options *opt, fmm_stats *stats);

/*
 * Stop and resume (for exploring stride schedules from a common state, as the stride
 * network's training labels do).  A solve given fmm_options.max_restarts stops after that
 * restart with FMM_ENOCONV, its state (tiles, bands, flags, lists) left in the library's
 * workspace on this device.  fmm_solve_resume continues it with restart from_restart + 1,
 * where from_restart is the restart it stopped after (stats->restarts of that call):
 *  * the arguments name the same problem as the stopped solve (grid, h, dtype, F, sources,
 *    block, waves per block), FMM_EINVAL otherwise; psi_dev receives the result (or, when
 *    it stops again, the values so far); stride_mode FIXED or SCHEDULE (at most 65536
 *    bounds), persistent launch only;
 *  * with a bound schedule, restart r takes bounds[r - 1]: a schedule that repeats the
 *    stopped solve's bounds up to from_restart continues it exactly as one solve with the
 *    whole schedule would; stats count the resumed restarts' pops and calls only.
 * fmm_workspace_save copies that state (*bytes_out bytes; dst_dev NULL = size query) into
 * a caller device buffer; fmm_workspace_restore copies it back, so several continuations
 * can start from one state.  Both are synchronous on hip_stream.  Another solve on the
 * device replaces the state.
 */
int fmm_solve_resume(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
                     const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
                     void *hip_stream, const fmm_options *opt, int64_t from_restart, fmm_stats *stats);
int fmm_workspace_save(void *dst_dev, size_t cap_bytes, size_t *bytes_out, void *hip_stream);
int fmm_workspace_restore(const void *src_dev, size_t bytes, void *hip_stream);

/*
 * fmm_solve without any device allocation, for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, semantics and errors as fmm_solve, with these differences:
 *  * the library's device workspace comes from one static device array of
 *    FMM_NOALLOC_SCRATCH_BYTES per GPU, which each GPU that loads the library holds
 *    until the process ends; no hipMalloc, hipFree, event or other allocating
 *    runtime call is made;
 *  * a grid whose workspace does not fit (about 4.2e6 points at block 16 and 3.1e6
 *    at block 8 in FP32, half that in FP64) fails with FMM_ENOMEM before any device
 *    work, and at most 256 sources are accepted (FMM_EINVAL beyond);
 *  * stats->elapsed_ms and stats->loop_ms are 0 (the call is not timed);
 *  * every call on a GPU uses that GPU's one array and leaves the last call's data in
 *    it; calls are serialised by the library's lock, but calls whose work overlaps on
 *    one GPU (another process excepted, which has its own array) would race.
 * The result is bitwise that of fmm_solve with the same arguments (same kernels).
 */
#define FMM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fmm_solve_noalloc(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
                      const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
                      void *hip_stream, const fmm_options *opt, fmm_stats *stats);

/* One problem of a batch (same meaning as the fmm_solve arguments).
   The stride of each problem is its own; dtype must be the same across a batch. */
typedef struct {
    int64_t nx, ny, nz;
    double h;
    const void *F_dev;
    void *psi_dev;
    const fmm_source *src;
    int32_t nsrc;
    double stride;
} fmm_problem;

/*
 * Solve nsolves independent problems in ONE launch.  By default the blocks of every
 * problem share the march and exchange lists of Alg. 6 and one restart index, and each
 * problem keeps its own bound (r * its stride).  With opt->per_problem_restarts every
 * problem runs its own restarts: work-groups take work items (blocks) of whichever
 * problem has some, and a problem moves to its next step when its own items are done,
 * with no barrier between problems.  Either way each problem's psi and counts are those
 * of its own fmm_solve.  block and waves_per_block apply to the whole batch
 * (fmm_autotune chooses them).  per_solve_stats is nullable or an array of nsolves;
 * restarts are per problem, elapsed_ms is the batch time.
 */
int fmm_solve_batched(int32_t nsolves, const fmm_problem *problems, int32_t dtype, int32_t block,
                      const fmm_options *opt, void *hip_stream, fmm_stats *per_solve_stats);

/* Autotuner result. */
typedef struct {
    int32_t block;
    int32_t waves_per_block;
    double ms;               /* measured time of the winning configuration */
} fmm_tuning;

/*
 * Choose block edge and waves per block for a batch by timing every supported
 * pair (block in {8, 16, 32} dividing all sides, waves in {1, 2, 4}, one wave for
 * 32) on the given
 * sample problems, once each after one warm-up.  Results are cached in memory
 * and, when cache_path is not NULL, in a small text file keyed by device name,
 * dtype and a size bin, so a later call with the same key does not time again.
 * psi_dev of the sample problems is overwritten.  The sample should carry about
 * as much work per restart as the batch it stands for: with too little, the grid
 * barrier dominates the timing and favours fewer, larger work-groups (8 of 512
 * uneven grids picked two waves per block, 32 pick one, which runs the whole
 * batch 2.2x faster).
 */
int fmm_autotune(int32_t nsamples, const fmm_problem *samples, int32_t dtype,
                 const char *cache_path, void *hip_stream, fmm_tuning *out);

/* ---------------------------------------------------------------- stride network
 * A 12-32-32-1 perceptron (ReLU hidden layers) maps standardised restart
 * features to log m = ln(1/4) + sigmoid(z) * ln(32), m in [1/4, 8]; the next
 * stride is m times the base stride.  Parameters (1505 floats), row-major
 * out x in: W1[32][12], b1[32], W2[32][32], b2[32], W3[1][32], b3[1].
 * The device blob given to fmm_options.mlp_weights holds the 1505 parameters
 * followed by the 12 feature means and the 12 feature standard deviations.
 *
 * Features (raw, in this order): bound / (n h), active-block fraction, the
 * fractions of active blocks whose band size falls in the bins {0}, [1,3],
 * [4,15], [16,63], [64,255], [256,1023], [1024,4095], [4096,inf), the restart
 * index / n, and the mean speed over active blocks; n is the largest grid side.
 */
#define FMM_MLP_NPARAMS 1505
#define FMM_MLP_BLOB_FLOATS (FMM_MLP_NPARAMS + 2 * FMM_NFEAT)

/* y_dev[s] = predicted log multiplier for standardised features x_dev[s][12].
   params_dev: 1505 floats.  Device buffers, FP32. */
int fmm_mlp_forward(const float *params_dev, const float *x_dev, int64_t n, float *y_dev,
                    void *hip_stream);

/* loss (device scalar) = mean_s (y_s - t_s)^2 and its gradient (1505 floats). */
int fmm_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n,
                      float *loss_dev, float *grad_dev, void *hip_stream);

/* One Adam step (Kingma & Ba 2015) at iteration t >= 1 on 1505 parameters;
   m_dev and v_dev are the moment buffers, updated in place. */
int fmm_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, float lr,
                 float beta1, float beta2, float eps, int64_t t, void *hip_stream);

/* Train for `steps` full-batch Adam steps from the parameters in params_dev
   (updated in place).  loss_hist_dev (nullable) receives one float per step. */
int fmm_mlp_train(float *params_dev, const float *x_dev, const float *t_dev, int64_t n,
                  int64_t steps, float lr, float *loss_hist_dev, void *hip_stream);

/* ---------------------------------------------------------------- diagnostics */
/* Each 64-lane wave w writes the minimum of in_dev[64w .. 64w+63] to out_dev[w],
   using the same cross-lane reduction as the march's argmin. */
int fmm_selftest_wave_min(const uint32_t *in_dev, uint32_t *out_dev, int32_t nwaves,
                          void *hip_stream);

/* Locate_Min (Alg. 4: the band point of least psi, ties to the lower tile index) of a
   march by one wave, on a given band: psi_dev holds the (B+2)^3 tile values of one block
   (dtype; entry 0, the tile corner, is never a band point and reads as +inf) and band_dev
   n distinct tile indices in [1, (B+2)^3), 1 <= n < (B+2)^3.  The tile is staged in LDS
   and the band held as a one-wave march holds it: the first `cap` slots (0 or a multiple
   of 512; 0 = as many as a march keeps there: 1024 for B = 16, 512 for 8, 256 for 4) in
   registers, the rest read from device memory.  Writes the picked value to val_out_dev[0] (dtype) and its tile
   index and band slot to idx_out_dev[0], idx_out_dev[1].  Synchronous on hip_stream;
   allocates a padded copy of the band.  FMM_EINVAL for null pointers, an unsupported
   dtype or block size (4, 8, 16), n out of range or a bad cap. */
int fmm_selftest_band_argmin(int dtype, int32_t block, const void *psi_dev,
                             const uint16_t *band_dev, int32_t n, int32_t cap,
                             void *val_out_dev, int32_t *idx_out_dev, void *hip_stream);

/* Frees the device memory and events the library holds on every device it has run on
   (workspace arenas, stride-network scratch, cached tunings); later calls allocate again.
   The static array of fmm_solve_noalloc stays with the loaded module.  The Python binding
   calls it when the interpreter exits, so that the HIP runtime's own teardown finds
   nothing of the library's left.  Must not overlap a call in flight. */
int fmm_release(void);

const char *fmm_strerror(int code);
const char *fmm_last_error_detail(void);
/* Library version string. */
const char *fmm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
