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

// ---------------------------------------------------------------- tags
// bits 0-1: category (Sec. 2.1 with KNOWN split as in Sec. 2.2); bit 2: the
// point currently sits in the block's band array.
constexpr uint8_t kFar = 0, kBand = 1, kKnownFix = 2, kKnownNew = 3;
constexpr uint8_t kStatus = 3, kInBand = 4;
__device__ __forceinline__ bool is_known(uint8_t t) { return (t & 2) != 0; }

// Faces: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z; the opposite face is f ^ 1.

// ---------------------------------------------------------------- control block
struct Ctl {
    unsigned bar_count;            // grid barrier arrivals
    unsigned bar_gen;              // grid barrier generation
    int abort;                     // first error code raised on the device (0 = none)
    int pad0;
    int n_list[2];                 // march-list sizes, by restart parity
    int q_head[2];                 // march work-queue heads, by restart parity
    unsigned long long pops, march_calls, exchange_calls, tile_loads;
    unsigned long long rpops[2];   // pops of the current restart, by parity
    unsigned long long feat[2][10];// band-size bins (8), sum of block mean speed (2^20 fixed
                                   // point), unused; by parity of the list being built
    long long restarts;
    double final_bound;
};

// Device-side error codes (stored in Ctl::abort; mapped to fmm.h codes by the host).
constexpr int kErrPopCap = 1, kErrTimeout = 2, kErrRestarts = 3, kErrBadSpeed = 4;

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
    R *rhs_t;              // [nblk][B^3] h^2 / F^2 of the interior points
    R *bmin;               // [nblk] exact minimum of the band (+inf when empty)
    uint8_t *A;            // [nblk] marching activation (Sec. 2.5)
    uint32_t *Cm;          // [nblk] exchange flags C, one bit per face (Sec. 2.6)
    int32_t *blk_prob;     // [nblk] problem of each block
    float *fmean;          // [nblk] mean speed of the block's interior
    int32_t *list0, *list1;// march lists, by restart parity
    Ctl *ctl;
    const ProbDesc *prob;
    int32_t nprob;
    int32_t stride_mode;   // 0 fixed, 1 learned
    int64_t nblk;
    int64_t max_restarts;
    int64_t pop_cap;       // watchdog on pops of one march call
    int64_t timeout_ticks; // watchdog on one grid-barrier wait (100 MHz ticks)
    const float *mlp;      // learned-stride blob (params, mean, std) or nullptr
    void *trace;           // fmm_trace_row[trace_cap] or nullptr
    int32_t trace_cap;
    int32_t want_features; // accumulate restart features (trace or learned)
    int32_t *prob_lastr;   // [nprob] last restart in which the problem had work queued
    unsigned long long *prob_pops; // [nprob]
};

// ---------------------------------------------------------------- tile geometry
template <int B>
struct Geo {
    static constexpr int P = B + 2;
    static constexpr int T = P * P * P;
    static constexpr int B3 = B * B * B;
};

template <typename R, int B, int W>
struct Lds {
    static constexpr int T = Geo<B>::T;
    static constexpr size_t psi_off = 0;
    static constexpr size_t band_off = psi_off + sizeof(R) * T;
    static constexpr size_t tag_off = band_off + 2 * T;
    static constexpr size_t scr_off = (tag_off + T + 15) / 16 * 16;
    static constexpr size_t bytes = scr_off + 16 * 8 + 64;
};

// ---------------------------------------------------------------- cross-lane min
// Minimum of x over the 64 lanes of the wave, returned in every lane.  Within a
// row of 16 lanes: DPP quad permutations (xor 1, xor 2), then the half-row and
// row mirrors; across rows: v_permlane16_swap and v_permlane32_swap, which
// exchange whole rows between the two operands.  Must be called with all 64
// lanes active.
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

// Lexicographic (psi, tile index) minimum over all lanes of the work-group.
// psi >= 0 so IEEE bit patterns order like the values.  Each lane brings its
// own best candidate (v, idx, slot); lanes without one bring (+inf, 0xffff).
template <typename R, int W>
__device__ __forceinline__ MinPick<R> group_argmin(R v, int idx, int slot, char *scr)
{
    const uint32_t vh = KeyBits<R>::hi(v), vl = KeyBits<R>::lo(v);
    const uint32_t mh = wave_min_u32(vh);
    uint32_t ml = 0;
    bool tie = (vh == mh);
    if (sizeof(R) == 8) {
        ml = wave_min_u32(tie ? vl : 0xffffffffu);
        tie = tie && (vl == ml);
    }
    uint64_t tm = ballot(tie);
    int win;
    uint32_t widx;
    if (__popcll(tm) == 1) {
        win = __ffsll((long long)tm) - 1;
        widx = (uint32_t)__builtin_amdgcn_readlane(idx, win);
    } else {
        widx = wave_min_u32(tie ? (uint32_t)idx : 0xffffffffu);
        win = __ffsll((long long)ballot(tie && (uint32_t)idx == widx)) - 1;
    }
    int wslot = __builtin_amdgcn_readlane(slot, win);
    MinPick<R> out{KeyBits<R>::from(mh, ml), (int)widx, wslot};
    if constexpr (W > 1) {
        // combine the W wave results through LDS
        uint32_t *s = reinterpret_cast<uint32_t *>(scr);
        const int wid = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            s[4 * wid + 0] = mh;
            s[4 * wid + 1] = ml;
            s[4 * wid + 2] = widx;
            s[4 * wid + 3] = (uint32_t)wslot;
        }
        __syncthreads();
        uint32_t bh = s[0], bl = s[1], bi = s[2], bs = s[3];
#pragma unroll
        for (int k = 1; k < W; ++k) {
            uint32_t h2 = s[4 * k], l2 = s[4 * k + 1], i2 = s[4 * k + 2];
            bool less = (h2 < bh) || (h2 == bh && (l2 < bl || (l2 == bl && i2 < bi)));
            if (less) {
                bh = h2;
                bl = l2;
                bi = i2;
                bs = s[4 * k + 3];
            }
        }
        out.v = KeyBits<R>::from(bh, bl);
        out.idx = (int)bi;
        out.slot = (int)bs;
    }
    return out;
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
    int d = 0;
    if (klo && psq > lo) d = -1;
    if (khi && psq > hi) {
        if (d == 0 || hi < lo) d = 1;
    }
    return d < 0 ? lo : (d > 0 ? hi : inf);
}

__device__ __forceinline__ float root2(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double root2(double x) { return __builtin_sqrt(x); }

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
            t = v0 + (s1b + root2(disc3)) / (R)3;
        }
    }
    return t;
}

} // namespace fmmdev
