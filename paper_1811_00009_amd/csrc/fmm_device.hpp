// fmm_device.hpp -- device-side building blocks of the block-based restarted
// narrow-band fast marching method (Yang 2018) for gfx950.
//
// One block of the grid (B^3 interior points padded by one ghost layer on each
// face, Sec. 2.3) is held in LDS while it marches.  Its narrow band -- the heap
// of Sec. 2.1, unified with the KNOWN_FIX points as in Sec. 2.2 -- is an
// unordered array of tile indices in LDS; Locate_Min is a scan of that array
// by every lane followed by a cross-lane minimum (DPP row operations and the
// gfx950 permlane swaps), Remove_Min swaps the last entry into the hole and
// Up_Heap is free because the key is read from the psi tile itself.  The six
// neighbour updates of one accepted point run on six lanes at once: the six
// face neighbours of a point are pairwise not face-adjacent, so their solves
// read disjoint data and the parallel update equals the sequential loop of
// Alg. 2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmmdev {

// Pointers into the work-group's LDS carry the LDS address space, so every access
// through them is a ds_* instruction (never a flat access).
#define FMM_LDS __attribute__((address_space(3)))
typedef unsigned int v4u __attribute__((ext_vector_type(4)));  // 16-byte copy unit

// ---------------------------------------------------------------- tags
// bits 1-2: category (Sec. 2.1 with KNOWN split as in Sec. 2.2), ordered so that
// KNOWN_FIX and KNOWN_NEW are the two largest; bit 0: the point currently sits
// in the block's band array.
constexpr uint8_t kFar = 0, kBand = 2, kKnownFix = 4, kKnownNew = 6;
constexpr uint8_t kStatus = 6, kInBand = 1;
__device__ __forceinline__ bool is_known(uint32_t t) { return t >= kKnownFix; }  // one compare

// Faces: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z; the opposite face is f ^ 1.

// ---------------------------------------------------------------- cycle account
// Profiling build only (-DFMM_CYCLES, libfmm_hip_cycles.so): the march of every block
// takes a shader-clock timestamp at each segment boundary of a pop, after waiting for
// every memory and LDS operation in flight, and adds the segment's cycles to its
// work-group's row of fmm_cyc_rows.  The waits serialise what the normal build
// overlaps, so the segments add up to more than a pop costs without them; both totals
// are reported.  In the normal build every mark compiles to nothing.
#ifdef FMM_CYCLES
constexpr int kCycSegs = 18;
constexpr int kCycRows = 8192;
__device__ unsigned long long fmm_cyc_rows[kCycRows][kCycSegs];
struct Cyc {
    unsigned long long t = 0, tl = 0;
    unsigned long long acc[kCycSegs] = {};
    // waits for LDS and scalar loads only (vmcnt and expcnt left at their maximum)
    __device__ static __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }
    __device__ static __forceinline__ void wait_all() { __builtin_amdgcn_s_waitcnt(0); }
    __device__ __forceinline__ void start()
    {
        wait_all();
        t = __builtin_amdgcn_s_memtime();
    }
    // segment k ends here (wave-uniform code only); full = also wait for device memory
    __device__ __forceinline__ void mark(int k, bool full = false)
    {
        if (full) wait_all();
        else wait_lds();
        const unsigned long long n = __builtin_amdgcn_s_memtime();
        acc[k] += n - t;
        t = n;
    }
    // sub-segments inside a lane-divergent region: kept per lane (lane 0's are flushed)
    __device__ __forceinline__ void lstart()
    {
        wait_lds();
        tl = __builtin_amdgcn_s_memtime();
    }
    __device__ __forceinline__ void lmark(int k, bool full = false)
    {
        if (full) wait_all();
        else wait_lds();
        const unsigned long long n = __builtin_amdgcn_s_memtime();
        acc[k] += n - tl;
        tl = n;
    }
    __device__ __forceinline__ void count(int k, unsigned long long v) { acc[k] += v; }
    __device__ __forceinline__ void flush()
    {
        if (threadIdx.x == 0 && blockIdx.x < (unsigned)kCycRows)
            for (int k = 0; k < kCycSegs; ++k) fmm_cyc_rows[blockIdx.x][k] += acc[k];
    }
};
#define FMM_CYC_PARAM , Cyc &cyc
#define FMM_CYC_ARG , cyc
#define FMM_CYC_DECL Cyc cyc
#define FMM_CYC_START() cyc.start()
#define FMM_CYC(k) cyc.mark(k)
#define FMM_CYC_FULL(k) cyc.mark(k, true)
#define FMM_CYC_LSTART() cyc.lstart()
#define FMM_CYC_L(k) cyc.lmark(k)
#define FMM_CYC_LFULL(k) cyc.lmark(k, true)
#define FMM_CYC_COUNT(k, v) cyc.count(k, v)
#else
#define FMM_CYC_PARAM
#define FMM_CYC_ARG
#define FMM_CYC_DECL
#define FMM_CYC_START() ((void)0)
#define FMM_CYC(k) ((void)0)
#define FMM_CYC_FULL(k) ((void)0)
#define FMM_CYC_LSTART() ((void)0)
#define FMM_CYC_L(k) ((void)0)
#define FMM_CYC_LFULL(k) ((void)0)
#define FMM_CYC_COUNT(k, v) ((void)0)
#endif
// Segments of the account (wave-uniform, in order): 0 band read, 1 psi gather and
// per-lane minimum, 2 cross-lane minimum and key, 3 bound test, neighbour tag and psi
// reads and Remove_Min, 4 the six neighbour solves, 5 insert and loop back; per march:
// 6 tile load, 7 face test, tile store and flags.  Inside the solves, lane 0's own
// solves (the -x neighbour): 8 stencil reads, 9 wait for h^2/F^2, 10 quadratic root and
// write; 11 counts them.  Counters: 12 pops, 13 marches.

// ---------------------------------------------------------------- control block
constexpr int kBarGroups = 64;  // arrival groups of the grid barrier

struct Ctl {
    // Counters that every work-group touches in each restart sit on 128-byte lines of
    // their own, so the barrier's arrivals, its polled generation, the queue heads and
    // the list appends do not contend for one line.
    alignas(128) unsigned bar_count;  // grid barrier arrivals of the group leaders
    alignas(128) unsigned bar_gen;    // grid barrier generation (polled)
    int abort;                        // first error code raised on the device (0 = none)
    alignas(128) int q_head[2];       // march work-queue heads, by restart parity
    int x_head[2];                    // exchange work-queue heads, by restart parity
    alignas(128) int n_list[2];       // march-list sizes, by restart parity
    int bin_n[2][4];                  // march-list sizes per work bin, by restart parity
    int x_n[2];                       // exchange-list sizes, by restart parity
    alignas(128) unsigned long long pops, march_calls, exchange_calls, tile_loads;
    unsigned long long rpops[2];      // pops of the current restart, by parity
    unsigned long long rmin[2];       // bits of the smallest value popped in the restart (traces)
    alignas(128) unsigned long long feat[2][10]; // band-size bins (8), sum of block mean speed
                                      // (2^20 fixed point), unused; by parity of the list
    long long restarts;
    double final_bound;
    // batches with restarts of their own per problem (k_batched): the ready queue of
    // problem tokens, the count of problems still running and of phases started
    alignas(128) unsigned long long rq_head;
    alignas(128) unsigned long long rq_tail;
    alignas(128) int remaining;
    unsigned long long progress;
    struct alignas(128) BarGroup {
        unsigned count;
    } bar_grp[kBarGroups];            // grid barrier arrivals, work-group w in group w % 64
};

// One problem of a batch whose restarts are its own: the phase it is in and that phase's
// work items, claimed one at a time by the work-groups holding one of its tokens.  word =
// phase << 40 | items << 20 | claims; phase 2 (r - 1) is the marching step of restart r,
// phase 2 (r - 1) + 1 its exchanging step.  The list counters are the problem's own, by
// restart parity, as the launch-wide ones of Ctl.
constexpr int kItemsPerToken = 4;  // a phase of n items invites ceil(n / 4) work-groups

struct alignas(128) SolveState {
    unsigned long long word;
    int done;         // items of the current phase finished
    int r;            // restarts begun (the last one when finished)
    int n_list[2];
    int bin_n[2][4];
    int x_n[2];
    int finished;
    int queued;       // this problem's tokens in the ready queue (or about to be put there)
};

// Device-side error codes (stored in Ctl::abort; mapped to fmm.h codes by the host).
constexpr int kErrPopCap = 1, kErrTimeout = 2, kErrRestarts = 3, kErrBadSpeed = 4, kErrList = 5;

// Per-problem descriptor (a batch holds several).
struct ProbDesc {
    const void *F;      // caller's speed, linear layout
    void *psi;          // caller's output, linear layout
    int32_t nx, ny, nz, mx, my, mz;
    int64_t blk0, nblk; // range of this problem's blocks in the pooled arrays
    double h, stride, width;
    int32_t nmax, pad;
};

template <typename R>
struct KParams {
    R *psi_t;              // [nblk][T] psi tiles (interior + ghost faces)
    uint8_t *tag_t;        // [nblk][T] tags
    uint16_t *band_t;      // [nblk][T] band arrays (tile indices)
    int32_t *band_n;       // [nblk] band sizes
    R *rhs_t;              // [nblk][T] h^2 / F^2 of the interior points (tile layout)
    R *bmin;               // [nblk] exact minimum of the band (+inf when empty)
    uint8_t *A;            // [nblk] marching activation (Sec. 2.5)
    uint32_t *Cm;          // [nblk] exchange flags C, one bit per face (Sec. 2.6)
    int32_t *blk_prob;     // [nblk] problem of each block
    float *fmean;          // [nblk] mean speed of the block's interior
    int32_t *lastpops;     // [nblk] pops of the block's last march (work estimate)
    int32_t *list0, *list1;// march lists, by restart parity; 4 bins of nblk entries each
    int32_t *xlist;        // [nblk] blocks whose C flags went up in this restart
    Ctl *ctl;
    const ProbDesc *prob;
    int32_t nprob;
    int32_t stride_mode;   // 0 fixed, 1 learned, 2 given bound sequence
    const double *sched;   // stride_mode 2: bound of restart r is sched[r - 1] (r <= nsched)
    int32_t nsched;
    int64_t r0;            // restarts already done (a resumed solve continues with r0 + 1)
    SolveState *solves;    // [nprob] batches with restarts of their own, else nullptr
    unsigned long long *ring; // ready queue of problem tokens (seq << 32 | problem)
    uint32_t ring_mask;    // ring size - 1 (a power of two)
    int32_t tokens;        // tokens handed out per phase (work-groups that may share it)
    int64_t nblk;
    int64_t max_restarts;
    int64_t pop_cap;       // watchdog on pops of one march call
    int64_t timeout_ticks; // watchdog on one grid-barrier wait (100 MHz ticks)
    const float *mlp;      // learned-stride blob (params, mean, std) or nullptr
    void *trace;           // fmm_trace_row[trace_cap] or nullptr
    int32_t trace_cap;
    int32_t want_features; // accumulate restart features (trace or learned)
    int32_t band_cap;      // diagnostic cap on band slots kept in LDS (0 = all that fit)
    int32_t *prob_lastr;   // [nprob] last restart in which the problem had work queued
    unsigned long long *prob_pops; // [nprob]
};

// ---------------------------------------------------------------- tile geometry
// The band is a plain array of tile indices; Locate_Min reads it in chunks of
// 512 slots, lane l taking slots [8l, 8l + 8) of a chunk with one 16-byte LDS
// read, so the 64 lanes touch consecutive 16-byte pieces (no bank conflicts).
// BAND slots (a multiple of 512) hold every point of the padded tile.  Tags are
// padded to a multiple of 16 bytes.  For B <= 8 the block's h^2/F^2 values are
// staged in LDS as well.
// The first BANDC slots of the band stay in LDS while the block marches; the
// rare slots beyond (a band larger than BANDC) are read and written in place in
// the block's band array in device memory.
template <int B>
struct Geo {
    static constexpr int P = B + 2;
    static constexpr int T = P * P * P;
    static constexpr int B3 = B * B * B;
    static constexpr int BAND = (T + 511) / 512 * 512;
    static constexpr int BANDC = BAND < 1024 ? BAND : 1024;
    static constexpr int TAGB = (T + 15) / 16 * 16;
    static constexpr bool RHS_LDS = B <= 8;
    // 32^3 blocks: a padded FP32 tile alone is 157 KB, so the march works on the tile in
    // device memory (one wave per block); the band's first slots stay in LDS
    static constexpr bool TILE_LDS = B <= 16;
};

// Pointer to tile data: LDS for blocks up to 16^3, device memory beyond.
template <typename T, bool IN_LDS>
struct TilePtr {
    typedef T *type;
};
template <typename T>
struct TilePtr<T, true> {
    typedef FMM_LDS T *type;
};

// Tile index of the e-th point of the six boundary layers of the interior, e in [0, 6 B^2):
// face f = e / B^2 in the order -x, +x, -y, +y, -z, +z, then the two in-face coordinates.
template <int B>
__device__ __forceinline__ int face_point(int e)
{
    constexpr int P = B + 2;
    const int f = e / (B * B), r = e % (B * B);
    const int a = r % B + 1, b = r / B + 1, l = (f & 1) ? B : 1;
    return (f >> 1) == 0 ? l + P * (a + P * b) : ((f >> 1) == 1 ? a + P * (l + P * b) : a + P * (b + P * l));
}

template <typename R, int B, int W>
struct Lds {
    static constexpr int T = Geo<B>::T;
    static constexpr size_t TILEB = Geo<B>::TILE_LDS ? sizeof(R) * T : 0;  // psi tile
    static constexpr size_t TAGL = Geo<B>::TILE_LDS ? Geo<B>::TAGB : 0;     // tag tile
    static constexpr size_t psi_off = 0;
    static constexpr size_t band_off = (psi_off + TILEB + 15) / 16 * 16;
    static constexpr size_t tag_off = band_off + 2 * Geo<B>::BANDC;
    static constexpr size_t rhs_off = (tag_off + TAGL + 15) / 16 * 16;
    static constexpr size_t scr_off = rhs_off + (Geo<B>::RHS_LDS ? sizeof(R) * T : 0);
    static constexpr size_t bytes = scr_off + 16 * 8 + 64;
    // Waves per SIMD that the LDS footprint allows (160 KB per CU, 4 SIMDs).  The
    // register budget of the march kernels is capped to match, up to 4 waves (128
    // registers) for one FP32 wave per block and 3 waves (168 registers) otherwise.
    // At 128 registers the one-wave FP32 kernels of 4^3 and 8^3 blocks spill, almost
    // all of it outside the loop of march steps; 168 registers at 8^3 blocks (12
    // instead of 14 resident per CU) measured slower.
    static constexpr int wgs_per_cu = (int)(163840 / (bytes + 128));
    static constexpr int lds_waves_per_simd = (wgs_per_cu * W + 3) / 4;
    // a march in device memory (32^3 blocks) is not bound by LDS: three waves per SIMD
    static constexpr int max_waves = (W == 1 && sizeof(R) == 4 && Geo<B>::TILE_LDS) ? 4 : 3;
    static constexpr int waves_per_simd =
        lds_waves_per_simd > max_waves ? max_waves
                                       : (lds_waves_per_simd < 1 ? 1 : lds_waves_per_simd);
};

// Copy NVEC 16-byte vectors global -> LDS (or back), eight per thread in flight
// before the first wait.
template <int NT, int NVEC, typename D, typename S>
__device__ __forceinline__ void copy_vec16(D *__restrict__ dst, const S *__restrict__ src, int tid)
{
    constexpr int PER = (NVEC + NT - 1) / NT;
    constexpr int BATCH = 8;
#pragma unroll
    for (int b0 = 0; b0 < PER; b0 += BATCH) {
        v4u r[BATCH];
#pragma unroll
        for (int j = 0; j < BATCH; ++j) {
            const int i = tid + (b0 + j) * NT;
            if (b0 + j < PER) r[j] = src[i < NVEC ? i : NVEC - 1];  // clamped: always in bounds
        }
#pragma unroll
        for (int j = 0; j < BATCH; ++j) {
            const int i = tid + (b0 + j) * NT;
            if (b0 + j < PER && i < NVEC) dst[i] = r[j];
        }
    }
}

// Copy the first n entries (rounded up to 8) of a band array.
template <int NT, typename D, typename S>
__device__ __forceinline__ void copy_band(D *dst, const S *src, int n, int tid)
{
    const int nvec = (n + 7) >> 3;
    for (int v0 = 0; v0 < nvec; v0 += 4 * NT) {
        v4u r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int v = v0 + tid + j * NT;
            v = v < nvec ? v : nvec - 1;  // clamped: always in bounds
            r[j] = reinterpret_cast<const S *>(src)[v];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = v0 + tid + j * NT;
            if (v < nvec) reinterpret_cast<D *>(dst)[v] = r[j];
        }
    }
}

// Load the first m entries of a block's band array into the LDS band of SLOTS entries and
// set the LDS slots [m, SLOTS) to 0: tile point 0 (a corner ghost, psi +inf, never in a
// band), so that a scan of whole 8-slot groups needs no bounds test.  The march keeps
// this while it runs: each slot that Remove_Min vacates is set to 0 again.
template <int NT, int SLOTS>
__device__ __forceinline__ void load_band_lds(FMM_LDS v4u *dst, const v4u *src, int m, int tid)
{
    static_assert(SLOTS % 8 == 0, "whole 16-byte groups");
    constexpr int NV = SLOTS / 8;
    const int nvec = (m + 7) >> 3;
    for (int v0 = 0; v0 < NV; v0 += 4 * NT) {
        v4u r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = v0 + tid + j * NT;
            r[j] = src[v < nvec ? v : 0];  // index 0 is always in bounds; masked below
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = v0 + tid + j * NT;
            const int c = m - 8 * v;  // band entries in this group (<= 0: none)
            uint32_t w[4] = {r[j].x, r[j].y, r[j].z, r[j].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = c >= 2 * i + 2 ? w[i] : (c == 2 * i + 1 ? (w[i] & 0xffffu) : 0u);
            if (v < NV) dst[v] = v4u{w[0], w[1], w[2], w[3]};
        }
    }
}

// ---------------------------------------------------------------- cross-lane min
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false));
    auto s16 = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = min((uint32_t)s16[0], (uint32_t)s16[1]);
    auto s32 = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    x = min((uint32_t)s32[0], (uint32_t)s32[1]);
    return x;
}

__device__ __forceinline__ unsigned lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ unsigned lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <typename R>
struct KeyBits;
template <>
struct KeyBits<float> {
    __device__ static uint32_t hi(float v) { return __float_as_uint(v); }
    __device__ static uint32_t lo(float) { return 0u; }
    __device__ static float from(uint32_t h, uint32_t) { return __uint_as_float(h); }
};
template <>
struct KeyBits<double> {
    __device__ static uint32_t hi(double v) { return (uint32_t)(__double_as_longlong(v) >> 32); }
    __device__ static uint32_t lo(double v) { return (uint32_t)__double_as_longlong(v); }
    __device__ static double from(uint32_t h, uint32_t l)
    {
        return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
    }
};

// Result of Locate_Min over the band: value, tile index, band slot.
template <typename R>
struct MinPick {
    R v;
    int idx;
    int slot;
};

// Minimum of two band values.  FP32: on the bit patterns (one integer min; psi >= +0
// and +inf order like their bits).  FP64: a compare and select.
__device__ __forceinline__ float val_min(float a, float b)
{
    return __uint_as_float(min(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ double val_min(double a, double b) { return b < a ? b : a; }
__device__ __forceinline__ bool val_eq(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }
__device__ __forceinline__ bool val_eq(double a, double b) { return a == b; }

// Minimum (value, key) over the 8 slots [c0 + 8 lane, c0 + 8 lane + 8) of one 512-slot chunk
// of the band: two depth-3 trees, the minimum value first, then the smallest key
// index << 16 | slot among the slots holding it.
template <typename R, typename PsiP>
__device__ __forceinline__ void band_chunk_min(const FMM_LDS uint16_t *s_band, const uint16_t *g_band,
                                               int cap, PsiP s_psi, int n, int c0,
                                               int lane, R &m_out, uint32_t &k_out FMM_CYC_PARAM)
{
    const int base = c0 + lane * 8;
    v4u raw;
    if (c0 < cap) {
        raw = *reinterpret_cast<const FMM_LDS v4u *>(s_band + base);
    } else {
        // the band's memory part (nontemporal loads: never merged with the LDS
        // path into one flat access)
        const uint32_t *g = reinterpret_cast<const uint32_t *>(g_band + base);
        raw.x = __builtin_nontemporal_load(g);
        raw.y = __builtin_nontemporal_load(g + 1);
        raw.z = __builtin_nontemporal_load(g + 2);
        raw.w = __builtin_nontemporal_load(g + 3);
    }
    const uint32_t w4[4] = {raw.x, raw.y, raw.z, raw.w};
    FMM_CYC(0);
    uint32_t ids[8];
    R vs[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t sl = (uint32_t)(base + j);
        const uint32_t id = (w4[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
        ids[j] = sl < (uint32_t)n ? id : 0u;  // tile point 0 (a corner) is never used: +inf
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) vs[j] = s_psi[ids[j]];
    // minimum value of the 8 slots (tree of depth 3)
    const R m = val_min(val_min(val_min(vs[0], vs[1]), val_min(vs[2], vs[3])),
                        val_min(val_min(vs[4], vs[5]), val_min(vs[6], vs[7])));
    // smallest key among the slots holding it
    uint32_t ks[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        ks[j] = val_eq(vs[j], m) ? ((ids[j] << 16) | (uint32_t)(base + j)) : ~0u;
    const uint32_t k0 = min(min(ks[0], ks[1]), min(ks[2], ks[3]));
    const uint32_t k1 = min(min(ks[4], ks[5]), min(ks[6], ks[7]));
    const uint32_t km = min(k0, k1);
    m_out = m;
    k_out = km;
}

// Minimum (value, key) over the S slots [S lane, S lane + S) of a band of n <= 64 S slots
// held in LDS (S = 1, 2 or 4): the narrow form of band_chunk_min for small bands.
template <typename R, int S, typename PsiP>
__device__ __forceinline__ void band_small_min(const FMM_LDS uint16_t *s_band, PsiP s_psi,
                                               int n, int lane, R &m_out, uint32_t &k_out FMM_CYC_PARAM)
{
    const int base = lane * S;
    uint32_t w[S > 1 ? S / 2 : 1];
    if constexpr (S == 4) {
        typedef unsigned int v2u __attribute__((ext_vector_type(2)));
        const v2u r = *reinterpret_cast<const FMM_LDS v2u *>(s_band + base);
        w[0] = r.x;
        w[1] = r.y;
    } else if constexpr (S == 2) {
        w[0] = *reinterpret_cast<const FMM_LDS uint32_t *>(s_band + base);
    } else {
        w[0] = s_band[base];
    }
    FMM_CYC(0);
    uint32_t ids[S];
    R vs[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const uint32_t id = (w[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
        ids[j] = (uint32_t)(base + j) < (uint32_t)n ? id : 0u;  // tile point 0: +inf
    }
#pragma unroll
    for (int j = 0; j < S; ++j) vs[j] = s_psi[ids[j]];
    R m = vs[0];
#pragma unroll
    for (int j = 1; j < S; ++j) m = val_min(m, vs[j]);
    uint32_t km = ~0u;
#pragma unroll
    for (int j = 0; j < S; ++j)
        km = min(km, val_eq(vs[j], m) ? ((ids[j] << 16) | (uint32_t)(base + j)) : ~0u);
    m_out = m;
    k_out = km;
}

// The two smallest values (with multiplicity) over the lanes' sorted pairs (a1 <= a2),
// left in every lane.  Each stage merges the lane's pair with that of a lane holding a
// disjoint set of lanes (quad swaps, half-row and row mirrors, then the row and half-wave
// swaps), which a top-2 merge needs: first = min(a1, b1), second = min(max(a1, b1),
// min(a2, b2)).  The swaps return the two lanes' values in an order that depends on the
// lane, the same for both words of the pair.
__device__ __forceinline__ void top2_merge_u32(uint32_t &a1, uint32_t &a2, uint32_t b1, uint32_t b2)
{
    const uint32_t f = min(a1, b1), s = min(max(a1, b1), min(a2, b2));
    a1 = f;
    a2 = s;
}
template <int CTRL>
__device__ __forceinline__ void wave_top2_stage(uint32_t &a1, uint32_t &a2)
{
    const uint32_t b1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a1, CTRL, 0xF, 0xF, false);
    const uint32_t b2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a2, CTRL, 0xF, 0xF, false);
    top2_merge_u32(a1, a2, b1, b2);
}
__device__ __forceinline__ void wave_top2_u32(uint32_t &a1, uint32_t &a2)
{
    wave_top2_stage<0xB1>(a1, a2);   // quad_perm [1,0,3,2]
    wave_top2_stage<0x4E>(a1, a2);   // quad_perm [2,3,0,1]
    wave_top2_stage<0x141>(a1, a2);  // row_half_mirror
    wave_top2_stage<0x140>(a1, a2);  // row_mirror
    {
        auto x = __builtin_amdgcn_permlane16_swap(a1, a1, false, false);
        auto y = __builtin_amdgcn_permlane16_swap(a2, a2, false, false);
        a1 = x[0];
        a2 = y[0];
        top2_merge_u32(a1, a2, x[1], y[1]);
    }
    {
        auto x = __builtin_amdgcn_permlane32_swap(a1, a1, false, false);
        auto y = __builtin_amdgcn_permlane32_swap(a2, a2, false, false);
        a1 = x[0];
        a2 = y[0];
        top2_merge_u32(a1, a2, x[1], y[1]);
    }
}

// Cross-lane step of Locate_Min within one wave: the minimum value over the lanes (high
// then low word for FP64), then the smallest key among the lanes holding it -- usually one
// lane does, and its key is read directly; equal values in several lanes take the
// cross-lane minimum.  Returns (value bits high, low, key), wave-uniform.
template <typename R>
__device__ __forceinline__ void wave_pick(R bv, uint32_t bk, uint32_t &mh, uint32_t &ml, uint32_t &mk)
{
    const uint32_t vh = KeyBits<R>::hi(bv);
    mh = wave_min_u32(vh);
    bool tie = (vh == mh);
    ml = 0;
    if constexpr (sizeof(R) == 8) {
        const uint32_t vl = KeyBits<R>::lo(bv);
        ml = wave_min_u32(tie ? vl : ~0u);
        tie = tie && (vl == ml);
    }
    const uint64_t tm = ballot(tie);
    if (__builtin_popcountll(tm) == 1)
        mk = (uint32_t)__builtin_amdgcn_readlane((int)bk, (int)__builtin_ctzll(tm));
    else
        mk = wave_min_u32(tie ? bk : ~0u);
}

// Locate_Min over the band: the lexicographic (psi, tile index) minimum.
// Each lane reads 8 consecutive slots per 16-byte read (1, 2 or 4 for a small band
// marched by one wave) and reduces them with
// two shallow trees: the minimum value first, then the smallest key among its
// slots holding that value, key = index << 16 | slot.  psi >= 0 (+0 only), so
// IEEE bit patterns order like the values; the cross-lane step takes the
// minimum value first (high then low word for FP64), then the minimum key
// among the lanes holding it.  Returns the same result in every lane.
template <typename R, int W, typename PsiP>
__device__ __forceinline__ MinPick<R> band_argmin(const FMM_LDS uint16_t *s_band,
                                                  const uint16_t *g_band, int cap,
                                                  PsiP s_psi, int n FMM_CYC_PARAM)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const R inf = (R)INFINITY;
    R bv = inf;
    uint32_t bk = ~0u;
    if (W == 1 && n <= 256 && n <= cap) {
        // a small band in LDS: 1, 2 or 4 slots per lane (n is wave-uniform)
        if (n <= 64) band_small_min<R, 1, PsiP>(s_band, s_psi, n, lane, bv, bk FMM_CYC_ARG);
        else if (n <= 128) band_small_min<R, 2, PsiP>(s_band, s_psi, n, lane, bv, bk FMM_CYC_ARG);
        else band_small_min<R, 4, PsiP>(s_band, s_psi, n, lane, bv, bk FMM_CYC_ARG);
    } else {
        // the first chunk of each wave sets (bv, bk) directly; later chunks (bands of
        // more than 512 * W slots) are merged in
        int c0 = wid * 512;
        if (c0 < n) band_chunk_min<R, PsiP>(s_band, g_band, cap, s_psi, n, c0, lane, bv, bk FMM_CYC_ARG);
        for (c0 += 512 * W; c0 < n; c0 += 512 * W) {
            R m;
            uint32_t km;
            band_chunk_min<R, PsiP>(s_band, g_band, cap, s_psi, n, c0, lane, m, km FMM_CYC_ARG);
            const bool better = (m < bv) | (val_eq(m, bv) & (km < bk));
            bv = better ? m : bv;
            bk = better ? km : bk;
        }
    }
    FMM_CYC(1);
    uint32_t mh, ml, mk;
    wave_pick<R>(bv, bk, mh, ml, mk);
    uint32_t h = mh, l = ml;
    if constexpr (W > 1) {
        __shared__ uint32_t s[16];
        if (lane == 0) {
            s[4 * wid + 0] = mh;
            s[4 * wid + 1] = ml;
            s[4 * wid + 2] = mk;
        }
        __syncthreads();
        h = s[0];
        l = s[1];
        mk = s[2];
#pragma unroll
        for (int k = 1; k < W; ++k) {
            const uint32_t h2 = s[4 * k], l2 = s[4 * k + 1], k2 = s[4 * k + 2];
            const bool less = (h2 < h) || (h2 == h && (l2 < l || (l2 == l && k2 < mk)));
            if (less) {
                h = h2;
                l = l2;
                mk = k2;
            }
        }
    }
    h = __builtin_amdgcn_readfirstlane(h);
    l = __builtin_amdgcn_readfirstlane(l);
    mk = __builtin_amdgcn_readfirstlane(mk);
    FMM_CYC(2);
    return MinPick<R>{KeyBits<R>::from(h, l), (int)(mk >> 16), (int)(mk & 0xffffu)};
}

// The two smallest (psi, key) entries of a band of at most 1024 slots, all in LDS, marched
// by one wave (the two-point step of march_block), whose LDS slots beyond n hold tile
// point 0 (load_band_lds).  Each lane takes the minimum of its
// slots and, with that slot left out, the next one (two shallow trees each, as in
// band_chunk_min); the cross-lane step runs once on the lanes' minima and once more with
// the winning lane offering its second.  Slots per lane as in band_argmin: 1, 2 or 4 for
// bands of at most 256 slots, else 8 per 512-slot chunk.
template <typename R, int S>
__device__ __forceinline__ void lane_top2(const R (&vs)[S], const uint32_t (&ks)[S], R &v1, uint32_t &k1,
                                          R &v2, uint32_t &k2)
{
    const R inf = (R)INFINITY;
    R m = vs[0];
#pragma unroll
    for (int j = 1; j < S; ++j) m = val_min(m, vs[j]);
    uint32_t km = ~0u;
#pragma unroll
    for (int j = 0; j < S; ++j) km = min(km, val_eq(vs[j], m) ? ks[j] : ~0u);
    R w[S];
#pragma unroll
    for (int j = 0; j < S; ++j) w[j] = ks[j] == km ? inf : vs[j];
    R m2 = w[0];
#pragma unroll
    for (int j = 1; j < S; ++j) m2 = val_min(m2, w[j]);
    uint32_t k2m = ~0u;
#pragma unroll
    for (int j = 0; j < S; ++j) k2m = min(k2m, (val_eq(w[j], m2) && ks[j] != km) ? ks[j] : ~0u);
    v1 = m;
    k1 = km;
    v2 = m2;
    k2 = k2m;
}

// The index offsets di + P dj + P^2 dk of the 62 displacements of Manhattan length 1 to 3,
// one per lane (the last two lanes hold 0, which no pair of distinct points has).  Two
// tile points at Manhattan distance below 4 differ by one of them, whatever P, so a pair
// whose index difference matches no lane lies at distance >= 4, the condition for taking
// two points in one march step.  A distant pair whose difference equals a short
// displacement's offset is declined as well (at P = 18, 0.09 % of the distant pairs),
// which costs one one-point step and no correctness.
struct CloseOffsets {
    int off[64];
};
template <int P>
constexpr CloseOffsets make_close_offsets()
{
    CloseOffsets c{};
    int n = 0;
    for (int dk = -3; dk <= 3; ++dk)
        for (int dj = -3; dj <= 3; ++dj)
            for (int di = -3; di <= 3; ++di) {
                const int m = (di < 0 ? -di : di) + (dj < 0 ? -dj : dj) + (dk < 0 ? -dk : dk);
                if (m >= 1 && m <= 3) c.off[n++] = di + P * dj + P * P * dk;
            }
    for (; n < 64; ++n) c.off[n] = 0;
    return c;
}
template <int P>
__device__ const CloseOffsets kCloseOffsets = make_close_offsets<P>();

// The same condition for tile points a and b (indices i + P j + P^2 k) without the table,
// for march kernels whose register budget has no room for the lane's offset.  For P >= 8 it is decided from the
// index difference d = b - a alone: a pair closer than 4 has d = di + P dj + P^2 dk with
// |di| + |dj| + |dk| <= 3, and the decomposition below (offsets that keep every step
// non-negative for such d) recovers exactly those (di, dj, dk), so every close pair is
// found.  A distant pair whose difference decomposes to a short one is declined as well
// (0.09 % of the distant pairs at P = 18), which costs one one-point step and no
// correctness.  Smaller tiles use the coordinates themselves.
template <int P>
__device__ __forceinline__ bool far_apart(int a, int b)
{
    if constexpr (P >= 8) {
        const int d = b - a;
        const uint32_t e = (uint32_t)(d + 3 * P * P + P * P / 2);
        const uint32_t qk = e / (uint32_t)(P * P);
        const uint32_t g = e - qk * (uint32_t)(P * P) - (uint32_t)(P * P / 2) + (uint32_t)(P / 2 + 3 * P);
        const uint32_t qj = g / (uint32_t)P;
        const int di = (int)(g - qj * (uint32_t)P) - P / 2, dj = (int)qj - 3, dk = (int)qk - 3;
        const int m = (di < 0 ? -di : di) + (dj < 0 ? -dj : dj) + (dk < 0 ? -dk : dk);
        return (d > 3 * P * P) | (d < -3 * P * P) | (m > 3);
    } else {
        const int di = a % P - b % P, dj = (a / P) % P - (b / P) % P, dk = a / (P * P) - b / (P * P);
        return (di < 0 ? -di : di) + (dj < 0 ? -dj : dj) + (dk < 0 ? -dk : dk) >= 4;
    }
}


// FP32: the same two smallest entries from 64-bit keys value bits << 32 | (index << 16 |
// slot).  psi >= +0, so the bit patterns order like the values, and the low words are
// unique: the unsigned order of the keys is the (psi, key) order.  A top-2 network: pairs
// sorted, then sorted pairs merged (first = the smaller first; second = the smaller of the
// other first and the winner's second), one compare and two 32-bit selects per choice.
__device__ __forceinline__ void sort2_u64(uint64_t &a, uint64_t &b)
{
    const bool c = b < a;
    const uint64_t lo = c ? b : a, hi = c ? a : b;
    a = lo;
    b = hi;
}
__device__ __forceinline__ void merge_top2_u64(uint64_t &a1, uint64_t &a2, uint64_t b1, uint64_t b2)
{
    const bool c = b1 < a1;
    const uint64_t f = c ? b1 : a1, o = c ? a1 : b1, w2 = c ? b2 : a2;
    a1 = f;
    a2 = o < w2 ? o : w2;
}
template <int S>
__device__ __forceinline__ void lane_top2_f32(const float (&vs)[S], const uint32_t (&ks)[S], uint64_t &x1,
                                              uint64_t &x2)
{
    uint64_t x[S];
#pragma unroll
    for (int j = 0; j < S; ++j) x[j] = ((uint64_t)__float_as_uint(vs[j]) << 32) | ks[j];
    if constexpr (S == 1) {
        x1 = x[0];
        x2 = ~0ull;
    } else {
#pragma unroll
        for (int j = 0; j < S; j += 2) sort2_u64(x[j], x[j + 1]);
#pragma unroll
        for (int w = 2; w < S; w *= 2) {
#pragma unroll
            for (int j = 0; j < S; j += 2 * w) merge_top2_u64(x[j], x[j + 1], x[j + w], x[j + w + 1]);
        }
        x1 = x[0];
        x2 = x[1];
    }
}

template <typename R>
__device__ __forceinline__ bool key_less(R va, uint32_t ka, R vb, uint32_t kb)
{
    return (va < vb) | (val_eq(va, vb) & (ka < kb));
}

// Merge the top-2 (b1 <= b2) of one group of slots into the running top-2 (a1 <= a2).
template <typename R>
__device__ __forceinline__ void top2_merge(R &av1, uint32_t &ak1, R &av2, uint32_t &ak2, R bv1, uint32_t bk1,
                                           R bv2, uint32_t bk2)
{
    const bool bfirst = key_less(bv1, bk1, av1, ak1);
    // the overall first, and the best of the remaining three candidates for second
    const R fv = bfirst ? bv1 : av1;
    const uint32_t fk = bfirst ? bk1 : ak1;
    const R cv = bfirst ? av1 : bv1;  // the other list's first
    const uint32_t ck = bfirst ? ak1 : bk1;
    const R dv = bfirst ? bv2 : av2;  // the winning list's second
    const uint32_t dk = bfirst ? bk2 : ak2;
    const bool csec = key_less(cv, ck, dv, dk);
    av1 = fv;
    ak1 = fk;
    av2 = csec ? cv : dv;
    ak2 = csec ? ck : dk;
}

template <typename R, int S, typename PsiP>
__device__ __forceinline__ void lane_slots_top2(const FMM_LDS uint16_t *s_band, PsiP s_psi, int n, int base,
                                                R &v1, uint32_t &k1, R &v2, uint32_t &k2)
{
    uint32_t w[(S + 1) / 2];
    if constexpr (S == 8) {
        const v4u r = *reinterpret_cast<const FMM_LDS v4u *>(s_band + base);
        w[0] = r.x;
        w[1] = r.y;
        w[2] = r.z;
        w[3] = r.w;
    } else if constexpr (S == 4) {
        typedef unsigned int v2u __attribute__((ext_vector_type(2)));
        const v2u r = *reinterpret_cast<const FMM_LDS v2u *>(s_band + base);
        w[0] = r.x;
        w[1] = r.y;
    } else if constexpr (S == 2) {
        w[0] = *reinterpret_cast<const FMM_LDS uint32_t *>(s_band + base);
    } else {
        w[0] = s_band[base];
    }
    // slots at n and beyond hold tile point 0 (psi +inf): no bounds test
    uint32_t ids[S], ks[S];
    R vs[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        ids[j] = (w[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
        ks[j] = (ids[j] << 16) | (uint32_t)(base + j);
    }
#pragma unroll
    for (int j = 0; j < S; ++j) vs[j] = s_psi[ids[j]];
    if constexpr (sizeof(R) == 4) {
        uint64_t x1, x2;
        lane_top2_f32<S>(vs, ks, x1, x2);
        v1 = __uint_as_float((uint32_t)(x1 >> 32));
        k1 = (uint32_t)x1;
        v2 = __uint_as_float((uint32_t)(x2 >> 32));
        k2 = (uint32_t)x2;
    } else {
        lane_top2<R, S>(vs, ks, v1, k1, v2, k2);
    }
}

template <typename R, typename PsiP>
__device__ __forceinline__ void band_top2(const FMM_LDS uint16_t *s_band, PsiP s_psi, int n,
                                          MinPick<R> &a, MinPick<R> &b FMM_CYC_PARAM)
{
    const int lane = threadIdx.x & 63;
    R v1, v2;
    uint32_t k1, k2;
    if (n <= 64) lane_slots_top2<R, 1, PsiP>(s_band, s_psi, n, lane, v1, k1, v2, k2);
    else if (n <= 128) lane_slots_top2<R, 2, PsiP>(s_band, s_psi, n, 2 * lane, v1, k1, v2, k2);
    else if (n <= 256) lane_slots_top2<R, 4, PsiP>(s_band, s_psi, n, 4 * lane, v1, k1, v2, k2);
    else {
        lane_slots_top2<R, 8, PsiP>(s_band, s_psi, n, 8 * lane, v1, k1, v2, k2);
        if (n > 512) {
            R u1, u2;
            uint32_t l1, l2;
            lane_slots_top2<R, 8, PsiP>(s_band, s_psi, n, 512 + 8 * lane, u1, l1, u2, l2);
            if constexpr (sizeof(R) == 4) {
                uint64_t a1 = ((uint64_t)__float_as_uint(v1) << 32) | k1, a2 = ((uint64_t)__float_as_uint(v2) << 32) | k2;
                merge_top2_u64(a1, a2, ((uint64_t)__float_as_uint(u1) << 32) | l1,
                               ((uint64_t)__float_as_uint(u2) << 32) | l2);
                v1 = __uint_as_float((uint32_t)(a1 >> 32));
                k1 = (uint32_t)a1;
                v2 = __uint_as_float((uint32_t)(a2 >> 32));
                k2 = (uint32_t)a2;
            } else {
                top2_merge<R>(v1, k1, v2, k2, u1, l1, u2, l2);
            }
        }
    }
    FMM_CYC(1);
    if constexpr (sizeof(R) == 4) {
        // FP32: the two smallest values over the lanes at once.  When they differ, the first
        // occurs once in the band (a second copy would be some lane's first or second), so
        // one lane holds it as its first; the second is the smallest offer, the winning
        // lane offering its second and every other lane its first, and ties among the
        // offers take the smallest key.  Equal values take the general path below.
        uint32_t f = __float_as_uint(v1), s2 = __float_as_uint(v2);
        wave_top2_u32(f, s2);
        f = __builtin_amdgcn_readfirstlane(f);
        s2 = __builtin_amdgcn_readfirstlane(s2);
        if (f != s2) {
            const uint64_t m1 = ballot(__float_as_uint(v1) == f);
            const int L = (int)__builtin_ctzll(m1);
            const uint32_t mk = (uint32_t)__builtin_amdgcn_readlane((int)k1, L);
            const bool own = lane == L;
            const uint32_t ov = own ? __float_as_uint(v2) : __float_as_uint(v1), ok = own ? k2 : k1;
            const uint64_t m2 = ballot(ov == s2);
            uint32_t nk;
            if (__builtin_popcountll(m2) == 1) nk = (uint32_t)__builtin_amdgcn_readlane((int)ok, (int)__builtin_ctzll(m2));
            else nk = wave_min_u32(ov == s2 ? ok : ~0u);
            nk = __builtin_amdgcn_readfirstlane(nk);
            a = MinPick<R>{__uint_as_float(f), (int)(mk >> 16), (int)(mk & 0xffffu)};
            b = MinPick<R>{__uint_as_float(s2), (int)(nk >> 16), (int)(nk & 0xffffu)};
            FMM_CYC(2);
            return;
        }
    }
    uint32_t mh, ml, mk;
    wave_pick<R>(v1, k1, mh, ml, mk);
    mh = __builtin_amdgcn_readfirstlane(mh);
    ml = __builtin_amdgcn_readfirstlane(ml);
    mk = __builtin_amdgcn_readfirstlane(mk);
    a = MinPick<R>{KeyBits<R>::from(mh, ml), (int)(mk >> 16), (int)(mk & 0xffffu)};
    // the second: the winning lane offers its next entry, every other lane its first
    const bool own = k1 == mk;
    uint32_t nh, nl, nk;
    wave_pick<R>(own ? v2 : v1, own ? k2 : k1, nh, nl, nk);
    nh = __builtin_amdgcn_readfirstlane(nh);
    nl = __builtin_amdgcn_readfirstlane(nl);
    nk = __builtin_amdgcn_readfirstlane(nk);
    b = MinPick<R>{KeyBits<R>::from(nh, nl), (int)(nk >> 16), (int)(nk & 0xffffu)};
    FMM_CYC(2);
}

// ---------------------------------------------------------------- Solve_Quadratic (Alg. 3)
// Upwind candidates per axis: a KNOWN neighbour (FIX or NEW) whose value is
// below the current psi_q; of two, the upper one only when strictly smaller.
// Candidates are sorted (absent axes are +inf and sort last) and the quadratic
// of Eq. (2) is solved with the first k of them while its root exceeds the next
// candidate.  The root is computed in the variable shifted by the smallest
// candidate v0 -- the same quadratic, without the cancellation of b^2 - a c --
// and a negative discriminant is clamped to 0.
template <typename R>
__device__ __forceinline__ R axis_candidate(R psq, R lo, bool klo, R hi, bool khi)
{
    const R inf = (R)INFINITY;
    const R a = klo ? lo : inf, b = khi ? hi : inf;
    const R c = val_min(a, b);  // equal values: either side gives the same candidate
    return c < psq ? c : inf;
}

// The largest value of type R that is <= the double bound: "v > bound" in double equals
// "v > below_or_equal<R>(bound)" in R for every v of type R (bound >= 0).
__device__ __forceinline__ float below_or_equal_f(double bound)
{
    float f = (float)bound;
    if ((double)f > bound) f = __uint_as_float(__float_as_uint(f) - 1u);  // f > 0 here
    return f;
}
template <typename R>
__device__ __forceinline__ R bound_in(double bound);
template <>
__device__ __forceinline__ float bound_in<float>(double bound) { return below_or_equal_f(bound); }
template <>
__device__ __forceinline__ double bound_in<double>(double bound) { return bound; }

__device__ __forceinline__ float root2(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double root2(double x) { return __builtin_sqrt(x); }

// x / 3, rounded as the IEEE division.  FP32: the product with RN(1/3), corrected by
// one fused multiply-add on the exact residual x - 3 q0; for every finite binary32 x
// this is the correctly rounded quotient (checked over all non-negative values,
// denormals included; the rounding is odd-symmetric), and x = inf stays inf.
// FP64: the division itself.
__device__ __forceinline__ float div3(float x)
{
    const float c = 0x1.555556p-2f;  // RN(1/3)
    const float q0 = x * c;
    const float r = __builtin_fmaf(-3.0f, q0, x);
    const float q1 = __builtin_fmaf(r, c, q0);
    return q0 == INFINITY ? q0 : q1;
}
__device__ __forceinline__ double div3(double x) { return x / 3.0; }

template <typename R>
__device__ __forceinline__ R quad_root(R c0, R c1, R c2, R rhs)
{
    // sort three values ascending (+inf = absent)
    R a = c0 < c1 ? c0 : c1;
    R b = c0 < c1 ? c1 : c0;
    R v0 = a < c2 ? a : c2;
    R m = a < c2 ? c2 : a;
    R v1 = b < m ? b : m;
    R v2 = b < m ? m : b;
    const R inf = (R)INFINITY;
    if (!(v0 < inf)) return inf;
    R t = v0 + root2(rhs);  // k = 1
    if (v1 < inf && t > v1) {
        R u = v1 - v0;
        R s1 = u, s2 = u * u;
        R disc = s1 * s1 - (R)2 * (s2 - rhs);
        if (disc < 0) disc = 0;
        t = v0 + (s1 + root2(disc)) / (R)2;
        if (v2 < inf && t > v2) {
            R u1 = v1 - v0, u2 = v2 - v0;
            R s1b = u1 + u2;
            R s2b = u1 * u1 + u2 * u2;
            R disc3 = s1b * s1b - (R)3 * (s2b - rhs);
            if (disc3 < 0) disc3 = 0;
            t = v0 + div3(s1b + root2(disc3));
        }
    }
    return t;
}

// x / k for k = kk + 1 in {1, 2, 3}, rounded as the IEEE division.  FP32: the product
// with c_k = 1, 1/2, RN(1/3), corrected by one fused multiply-add on the exact residual
// x - k q0 (for k = 1 and 2 the product is already the quotient and the correction keeps
// it; the sequence is checked against x / k over all non-negative binary32 values for
// each k); x = inf stays inf.  FP64: the division itself.
__device__ __forceinline__ float div_k(float x, int kk)
{
    const float c = kk == 0 ? 1.0f : (kk == 1 ? 0.5f : 0x1.555556p-2f);
    const float kf = (float)(kk + 1);
    const float q0 = x * c;
    const float r = __builtin_fmaf(-kf, q0, x);
    const float q1 = __builtin_fmaf(r, c, q0);
    return q0 == INFINITY ? q0 : q1;
}
__device__ __forceinline__ double div_k(double x, int kk) { return x / (double)(kk + 1); }

// Alg. 3 with a given number of candidates: the root of the quadratic of Eq. (2) over the
// kk + 1 smallest of the three candidates (sorted here; +inf = absent), in the variable
// shifted by the smallest, with the same operations as quad_root takes for that count.
// Returns +inf when there is no candidate and leaves the sorted second and third
// candidates in v1o, v2o.  With more candidates asked for than there are, the result is
// not used (it may be NaN).
template <typename R>
__device__ __forceinline__ R quad_root_k(R c0, R c1, R c2, R rhs, int kk, R &v1o, R &v2o)
{
    R a = c0 < c1 ? c0 : c1;
    R b = c0 < c1 ? c1 : c0;
    R v0 = a < c2 ? a : c2;
    R m = a < c2 ? c2 : a;
    R v1 = b < m ? b : m;
    R v2 = b < m ? m : b;
    v1o = v1;
    v2o = v2;
    const R inf = (R)INFINITY;
    if (!(v0 < inf)) return inf;
    const R z = (R)0;
    const R u1 = kk >= 1 ? v1 - v0 : z;
    const R u2 = kk >= 2 ? v2 - v0 : z;
    const R s1 = u1 + u2;
    const R s2 = u1 * u1 + u2 * u2;
    R disc = s1 * s1 - (R)(kk + 1) * (s2 - rhs);
    if (disc < 0) disc = 0;
    return v0 + div_k(s1 + root2(disc), kk);
}

// The value of lane 4 (lane / 4) + J in every lane of each quad (DPP quad permute).
template <int J>
__device__ __forceinline__ float quad_bcast(float x)
{
    constexpr int ctrl = J | (J << 2) | (J << 4) | (J << 6);
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xF, 0xF, false));
}
template <int J>
__device__ __forceinline__ double quad_bcast(double x)
{
    constexpr int ctrl = J | (J << 2) | (J << 4) | (J << 6);
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, ctrl, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

} // namespace fmmdev
