/*
 * cpu_parallel.c -- TEST AND BENCHMARK INFRASTRUCTURE ONLY.
 *
 * The paper's parallel CPU solver (Sec. 2.7, measured in Sec. 3.5-3.6): the
 * block-based restarted method of Alg. 6 with the marching step and the
 * exchanging step of every restart spread over the blocks by OpenMP threads,
 * as a second CPU baseline beside the single-thread oracle, and as the
 * reference that a whole 1024^3 grid can be checked against in a test's time.
 *
 * The per-block steps are the block reference's own (march_one, exchange_one
 * in fmm_oracle_impl.h).  Within one step the blocks are independent: a march
 * writes only its own block and raises flags on its neighbours, an exchange
 * writes only its own block and reads its neighbours' interior points and
 * Upsilon lists, which no exchange writes (Sec. 2.7).  So the result is bitwise
 * that of orc_block_fmm_{f64,f32}, whatever the number of threads; a test
 * checks it for both precisions.  Nothing here is shared with the HIP library,
 * and the product never loads it.
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

#define REAL float
#define SFX par_f32
#define RSQRT sqrtf
#include "fmm_oracle_impl.h"
#undef REAL
#undef SFX
#undef RSQRT

/* The restart loop of Alg. 6 with both steps spread over OpenMP threads, for one
   precision (REAL) and symbol suffix (SFX). */
#define PAR_CAT2(a, b) a##_##b
#define PAR_CAT(a, b) PAR_CAT2(a, b)
#define PFN(name) PAR_CAT(name, SFX)

#define REAL double
#define SFX par_f64
#include "cpu_parallel_impl.h"
#undef REAL
#undef SFX

#define REAL float
#define SFX par_f32
#include "cpu_parallel_impl.h"
#undef REAL
#undef SFX
