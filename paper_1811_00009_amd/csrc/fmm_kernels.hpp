// fmm_kernels.hpp -- the phases of one restart of the block-based restarted
// narrow-band FMM (Alg. 6) as device functions, and the kernels built from
// them: block set-up (Alg. 1), the persistent restart loop, the per-phase
// kernels of the host-driven loop, and the copy of the result back to the
// caller's linear layout.
#pragma once
#include "fmm_device.hpp"

namespace fmmdev {

// Row of the per-restart trace; same layout as fmm_trace_row in fmm.h.
struct TraceRow {
    float feat[12];
    double bound;
    double stride_used;
    int64_t pops;
    int64_t t_start;
    int64_t t_end;
    int32_t active;
    int32_t next_active;
    double min_popped;
};

constexpr double kLogMinMult = -1.3862943611198906;  // ln(1/4)
constexpr double kLogSpanMult = 3.4657359027997265;  // ln(8) - ln(1/4)
constexpr double kFixScale = 1048576.0;              // 2^20, fixed point of speed sums

__device__ __forceinline__ int64_t wall_ticks() { return (int64_t)wall_clock64(); }

__device__ __forceinline__ void raise_error(Ctl *ctl, int code)
{
    int expected = 0;
    __hip_atomic_compare_exchange_strong(&ctl->abort, &expected, code, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int read_abort(Ctl *ctl)
{
    return __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// bound_r = min(r * stride, width) evaluated in double (fixed stride, Alg. 6).
__device__ __forceinline__ double fixed_bound(int64_t r, double stride, double width)
{
    double b = (double)r * stride;
    return b > width ? width : b;
}

// Grid-wide barrier for the persistent kernel.  Every work-group's first
// thread arrives with an agent-scope release and waits for the generation to
// move with an acquire, so everything written before the barrier by any
// work-group is visible after it.  The wait is bounded: on timeout, or when
// another work-group has raised an error, it gives up and the caller leaves
// the restart loop.
//
// Arrivals go in two levels, so that no counter takes more than ~G/64 + 64
// of them: work-group w arrives at the counter of group w % 64, the last of
// each group (after an acquire, so it carries the group's stores on) arrives
// at the top counter, and the last of those releases the generation.  Each
// last arriver resets its counter before passing on; nobody arrives again
// before the generation moves, which happens after every reset.
//
// The wait polls with relaxed agent-scope loads (they read the coherent value
// without touching the caches) and acquires once after the generation moved:
// an acquire on every poll would invalidate the XCD's L2 under the work-groups
// that are still working.
__device__ void grid_barrier(Ctl *ctl, unsigned G, int64_t timeout_ticks)
{
    // every wave publishes its own stores before the work-group arrives
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        const unsigned w = blockIdx.x, grp = w % kBarGroups;
        const unsigned ngroups = G < (unsigned)kBarGroups ? G : (unsigned)kBarGroups;
        const unsigned gsize = (G - 1 - grp) / kBarGroups + 1;  // work-groups of group grp
        bool released = false;
        const unsigned pg = __hip_atomic_fetch_add(&ctl->bar_grp[grp].count, 1u, __ATOMIC_RELEASE,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (pg == gsize - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&ctl->bar_grp[grp].count, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            const unsigned prev = __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_RELEASE,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            if (prev == ngroups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->bar_gen, gen + 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            const int64_t t0 = wall_ticks();
            int polls = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                   gen) {
                __builtin_amdgcn_s_sleep(2);
                if ((++polls & 63) == 0) {
                    if (read_abort(ctl)) break;
                    if (wall_ticks() - t0 > timeout_ticks) {
                        raise_error(ctl, kErrTimeout);
                        break;
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Where a block's list entries go: the next march list (4 work bins of `stride` entries
// from `next`, counted in bins[] and *nlist) and the exchange list (xl, counted in *xn),
// each holding at most `cap` entries.  Either the whole launch's lists (restarts shared by
// every problem) or one problem's segment of them (restarts of its own).
struct ListSink {
    int32_t *next;
    int *bins;
    int *nlist;
    int32_t *xl;
    int *xn;
    int64_t stride, cap;
};

// The lists of the whole launch in restart r (list parity c = r & 1).
template <typename R>
__device__ __forceinline__ ListSink launch_sink(const KParams<R> &kp, int c)
{
    return ListSink{c ? kp.list0 : kp.list1, kp.ctl->bin_n[c ^ 1], &kp.ctl->n_list[c ^ 1],
                    kp.xlist, &kp.ctl->x_n[c], kp.nblk, kp.nblk};
}

// ---------------------------------------------------------------- Alg. 4 on one block
// March_Narrow_Band(ib): load the block's tile, band and tags into LDS, accept
// band points in increasing (psi, index) order while psi <= bound, relaxing the
// interior neighbours of each accepted point (Alg. 2 with Alg. 3), then store
// the tile back, record the new band minimum and raise the exchange flag of
// every neighbour whose ghost layer meets the updated boundary points.
//
// One step costs two LDS round trips for Locate_Min (a 16-byte read of 8 band
// slots per lane, then the 8 psi values) and one or two for Update_Neighbors
// (the quads read their neighbour's tag and psi while single lanes read the
// accepted points' tags and the band's last slots; the stencils in the same
// round trip, except in the one-point step with h^2/F^2 in device memory, where
// a second one covers that load, issued first).
// LANE_PAIR: the two-point step's pair test by the lanes' table of short displacements (one
// compare and a ballot), else by the index difference (scalar arithmetic); the batch kernel
// takes the latter, since the table's register spills there at 8^3 blocks.
template <typename R, int B, int W, bool LANE_PAIR = true>
__device__ void march_block(const KParams<R> &kp, int64_t ib, const ProbDesc &pd, double bound,
                            const ListSink &sink, char *smem, unsigned long long &pops_acc, bool &a_out,
                            int &n_out, int &pops_out FMM_CYC_PARAM)
{
    using L = Lds<R, B, W>;
    using Gm = Geo<B>;
    constexpr int P = Gm::P, T = Gm::T, NT = 64 * W, BAND = Gm::BAND, TAGB = Gm::TAGB;
    constexpr bool TL = Gm::TILE_LDS;  // tile staged in LDS (else marched in device memory)
    static_assert(TL || W == 1, "a tile in device memory is marched by one wave");
    // band slots [0, cap) live in LDS, [cap, n) in the block's band array in memory
    const int cap = kp.band_cap > 0 && kp.band_cap < Gm::BANDC ? kp.band_cap : Gm::BANDC;
    FMM_LDS char *lds = (FMM_LDS char *)smem;
    FMM_LDS uint16_t *s_band = reinterpret_cast<FMM_LDS uint16_t *>(lds + L::band_off);
    __shared__ int s_bc[1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const R inf = (R)INFINITY;

    R *g_psi = kp.psi_t + ib * (int64_t)T;
    uint8_t *g_tag = kp.tag_t + ib * (int64_t)TAGB;
    uint16_t *g_band = kp.band_t + ib * (int64_t)BAND;
    const R *g_rhs = kp.rhs_t + ib * (int64_t)T;
    typename TilePtr<R, TL>::type s_psi;
    typename TilePtr<uint8_t, TL>::type s_tag;
    if constexpr (TL) {
        s_psi = reinterpret_cast<FMM_LDS R *>(lds + L::psi_off);
        s_tag = reinterpret_cast<FMM_LDS uint8_t *>(lds + L::tag_off);
    } else {
        s_psi = g_psi;
        s_tag = g_tag;
    }

    FMM_CYC_START();
    int n = kp.band_n[ib];
    if constexpr (TL) {
        copy_vec16<NT, (int)(sizeof(R) * T / 16)>(reinterpret_cast<FMM_LDS v4u *>(s_psi),
                                                   reinterpret_cast<const v4u *>(g_psi), tid);
        copy_vec16<NT, TAGB / 16>(reinterpret_cast<FMM_LDS v4u *>(s_tag),
                                  reinterpret_cast<const v4u *>(g_tag), tid);
    }
    load_band_lds<NT, Gm::BANDC>(reinterpret_cast<FMM_LDS v4u *>(s_band), reinterpret_cast<const v4u *>(g_band),
                                 n < cap ? n : cap, tid);
    FMM_LDS R *s_rhs = reinterpret_cast<FMM_LDS R *>(lds + L::rhs_off);
    if constexpr (!TL) {
        // the tile is marched where it is; h^2/F^2 is read from memory as needed
    } else if constexpr (Gm::RHS_LDS) {
        copy_vec16<NT, (int)(sizeof(R) * T / 16)>(reinterpret_cast<FMM_LDS v4u *>(s_rhs),
                                                   reinterpret_cast<const v4u *>(g_rhs), tid);
    } else {
        // h^2/F^2 stays in device memory: touch each of its cache lines once now, so the
        // solves of the march hit in cache instead of each paying a memory round trip
        constexpr int LINE = 128 / (int)sizeof(R);
        R acc = (R)0;
#pragma unroll
        for (int k = 0; k < (T + LINE * NT - 1) / (LINE * NT); ++k) {
            const int l = tid + k * NT;
            acc += g_rhs[l * LINE < T ? l * LINE : T - 1];
        }
        asm volatile("" ::"v"(acc));  // keeps the loads (the ghost slots of the tile are unset)
    }
    __syncthreads();
    FMM_CYC_FULL(6);
    FMM_CYC_COUNT(13, 1);

    // Update_Neighbors by quads of wave 0: quad g (lanes 4g .. 4g+3, g < 6) takes face
    // neighbour g of the accepted point (-x, +x, -y, +y, -z, +z); its lanes kk = 0, 1, 2
    // solve the quadratic of Alg. 3 with kk + 1 candidates at once, and lane 4g takes the
    // root the sequential rule of Alg. 3 arrives at.  Lane 24 retags the accepted point,
    // lane 25 moves the band's last slot (Remove_Min).
    const int g = lane >> 2, kk = lane & 3;
    const int dI = (g == 1) - (g == 0), dJ = (g == 3) - (g == 2), dK = (g == 5) - (g == 4);
    const int dOff = dI + P * (dJ + P * dK);
    // Two accepted points per step (one wave, tile and band in LDS): quads 6-11 take the
    // face neighbours of the second point the way quads 0-5 take the first's
    constexpr bool PAIR = TL && W == 1;
    const int gdir = g < 6 ? g : (g < 12 ? g - 6 : 0);
    const int gpt = g < 6 ? 0 : (g < 12 ? 1 : 2);
    const int eI = (gdir == 1) - (gdir == 0), eJ = (gdir == 3) - (gdir == 2), eK = (gdir == 5) - (gdir == 4);
    const int eOff = eI + P * (eJ + P * eK);
    // The accepted point is q's low neighbour for the + directions and its high neighbour
    // for the - directions, on the quad's own axis; its tag is written after the step's
    // check, so it is taken as known: these tag bits (a KNOWN status) are or-ed into the
    // tag read on that side.  Kept as register data, not lane masks.
    uint32_t flo[3], fhi[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const bool own = ax == (gdir >> 1);
        flo[ax] = (own && (gdir & 1)) ? kKnownFix : 0u;
        fhi[ax] = (own && !(gdir & 1)) ? kKnownFix : 0u;
    }
    // the pair test of the two-point step: the lane's offset of a short displacement
    const int close_off = LANE_PAIR ? kCloseOffsets<P>.off[lane] : 0;
    uint32_t mine = 0;  // faces of Upsilon, recorded as points are lowered (tile in memory)
    constexpr int kMid = (B / 2) * (1 + P + P * P);  // an interior point of the tile
    bool active = true;
    R exit_min = inf;
    int npops = 0;
    const int pop_cap = __builtin_amdgcn_readfirstlane((int)kp.pop_cap);
    const R rbound = bound_in<R>(bound);  // psi > rbound  <=>  (double)psi > bound
    for (;;) {
        n = __builtin_amdgcn_readfirstlane(n);  // wave-uniform: scalar branches below
        if (n == 0) {  // empty heap: deactivate
            active = false;
            exit_min = inf;
            break;
        }
        if constexpr (PAIR) {
            if (n <= cap) {
                // Two steps of Alg. 4 at once.  p1 is the band's minimum; p2, the next entry,
                // is taken with it only when it lies at Manhattan distance >= 4 from p1
                // (kCloseOffsets or far_apart, which may decline a few such pairs as well): then p1's
                // step (p1 and its face neighbours written, their neighbours read) and p2's
                // touch disjoint points.  p2 is the point the sequential march accepts next
                // unless p1's step lowers a point below it, which is checked once the roots
                // are in: only then are p2's values, tag and slot written.  Every step is
                // the one of the sequential order, so psi and the counts are unchanged.
                MinPick<R> m1, m2;
                band_top2<R>(s_band, s_psi, n, m1, m2 FMM_CYC_ARG);
                if (m1.v > rbound) {  // beyond the restart bound: stop (deactivate past width)
                    if ((double)m1.v > pd.width) active = false;
                    exit_min = m1.v;
                    break;
                }
                const int p1 = m1.idx;
                FMM_CYC_COUNT(14, n <= 64 ? 1 : 0);
                FMM_CYC_COUNT(15, n <= 256 ? 1 : 0);
                if (++npops > pop_cap) {
                    raise_error(kp.ctl, kErrPopCap);
                    exit_min = m1.v;
                    break;
                }
                int p2 = p1;
                bool pair = false;
                if (n >= 2 && !(m2.v > rbound) && npops < pop_cap) {
                    if constexpr (LANE_PAIR) pair = ballot(close_off == m2.idx - p1) == 0ull;
                    else pair = far_apart<P>(p1, m2.idx);
                    if (pair) p2 = m2.idx;
                }
                // the lane's quad group, kk and lane id, re-read in each step: the lane
                // tests below are then computed where they are used instead of being held
                // across the loop as 64-bit lane masks (which the scalar registers cannot
                // hold alongside the loop's state)
                int gpt_s = gpt, kk_s = kk, ln_s = lane;
                asm volatile("" : "+v"(gpt_s), "+v"(kk_s), "+v"(ln_s));
                const int pp = gpt_s == 1 ? p2 : p1;
                const R vpp = gpt_s == 1 ? m2.v : m1.v;
                R rhs_mem = (R)0;
                if constexpr (!Gm::RHS_LDS) {
                    const int ql = pp + eOff;
                    rhs_mem = g_rhs[ql < 0 ? 0 : (ql > T - 1 ? T - 1 : ql)];
                }
                const uint32_t up = (uint32_t)pp;
                const int pi = (int)(up % P), pj = (int)((up / P) % P), pk = (int)(up / (P * P));
                const int qi = pi + eI, qj = pj + eJ, qk = pk + eK;
                const bool inb = (gpt_s == 0 || (gpt_s == 1 && pair)) && kk_s < 3 &&
                                 (unsigned)(qi - 1) < (unsigned)B && (unsigned)(qj - 1) < (unsigned)B &&
                                 (unsigned)(qk - 1) < (unsigned)B;
                // lane 48 reads p1's own tag, lane 49 p2's
                const int q = inb ? pp + eOff : (ln_s == 49 ? p2 : p1);
                R rhs = (R)0;
                if (inb) {
                    if constexpr (Gm::RHS_LDS) rhs = s_rhs[q];
                    else rhs = rhs_mem;
                }
                const uint8_t tq = s_tag[q];
                const R psq = s_psi[q];
                // the stencil is read in the same LDS round trip as q's own tag and value,
                // for every block size: one wait before the solves instead of two
                R lo[3], hi[3];
                uint32_t tlo[3], thi[3];
                {
                    const int qs = inb ? q : kMid;
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const int off = ax == 0 ? 1 : (ax == 1 ? P : P * P);
                        lo[ax] = s_psi[qs - off];
                        hi[ax] = s_psi[qs + off];
                        tlo[ax] = s_tag[qs - off];
                        thi[ax] = s_tag[qs + off];
                    }
                }
                // the band's last two slots, for Remove_Min of one or both points (read by
                // every lane, used by the writing lanes at the end of the step, so that no
                // wait for them falls before the solves)
                const uint16_t last1 = s_band[n - 1];
                const uint16_t last2 = s_band[n >= 2 ? n - 2 : n - 1];
                FMM_CYC(3);
                const bool solve = inb && (tq & kStatus) != kKnownFix && psq > vpp;
                R t = inf, r1 = inf, r2 = inf;
                if (solve) {
                    FMM_CYC_LSTART();
                    R c[3];
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        // the accepted point reads as known (flo, fhi)
                        const bool klo = is_known(tlo[ax] | flo[ax]);
                        const bool khi = is_known(thi[ax] | fhi[ax]);
                        c[ax] = axis_candidate<R>(psq, lo[ax], klo, hi[ax], khi);
                    }
                    FMM_CYC_L(8);
                    FMM_CYC_LFULL(9);
                    t = quad_root_k<R>(c[0], c[1], c[2], rhs, kk_s, r1, r2);
                    FMM_CYC_L(10);
                    FMM_CYC_COUNT(11, 1);
                }
                const R t2 = quad_bcast<1>(t), t3 = quad_bcast<2>(t);
                bool low = false, ins = false;
                R tf = inf;
                if (solve && kk_s == 0) {
                    tf = t;
                    if (r1 < inf && tf > r1) {
                        tf = t2;
                        if (r2 < inf && tf > r2) tf = t3;
                    }
                    if (tf < psq) {
                        low = true;
                        ins = !(tq & kInBand);
                    }
                }
                // p2 is the next point unless p1's step lowered a point below it
                const uint64_t beat = ballot(low && gpt_s == 0 && key_less<R>(tf, (uint32_t)q, m2.v, (uint32_t)p2));
                const uint64_t ins1 = ballot(ins && gpt_s == 0), ins2 = ballot(ins && gpt_s == 1);
                const bool acc2 = pair && beat == 0;
                const bool wr = low && (gpt_s == 0 || acc2);
                if (wr) {
                    s_psi[q] = tf;
                    s_tag[q] = kBand | kInBand;
                }
                // KNOWN_NEW unless KNOWN_FIX; the points leave the band
                if (ln_s == 48 || (ln_s == 49 && acc2))
                    s_tag[q] = ((tq & kStatus) == kKnownFix) ? kKnownFix : kKnownNew;
                FMM_CYC(4);
                FMM_CYC_COUNT(12, acc2 ? 2 : 1);
                FMM_CYC_COUNT(16, 1);  // two-point steps taken, and how many accepted p2
                FMM_CYC_COUNT(17, acc2 ? 1 : 0);
                // the slots that Remove_Min vacates (the last one or two) go back to tile
                // point 0; an insert below may take them again (its store comes later)
                if (ln_s == 52 || (ln_s == 53 && acc2)) s_band[n - 1 - (ln_s - 52)] = 0;
                if (!acc2) {  // Remove_Min of p1: the last slot moves into its hole
                    if (ln_s == 50 && m1.slot != n - 1) s_band[m1.slot] = (uint16_t)last1;
                    n -= 1;
                } else {
                    // Remove_Min of both: the holes below n - 2 take the entries of the last
                    // two slots that are not holes themselves (as many of each)
                    const int s1 = m1.slot, s2 = m2.slot, e1 = n - 1, e2 = n - 2;
                    int h0 = -1, h1 = -1;
                    if (s1 < e2) h0 = s1;
                    if (s2 < e2) {
                        if (h0 < 0) h0 = s2;
                        else h1 = s2;
                    }
                    // the fillers in order: slot e2's entry if it is not a hole, then e1's
                    const bool e2_stays = e2 != s1 && e2 != s2;
                    if (ln_s == 50 && h0 >= 0) s_band[h0] = e2_stays ? last2 : last1;
                    if (ln_s == 51 && h1 >= 0) s_band[h1] = last1;  // both fillers: e2's, e1's
                    n -= 2;
                    ++npops;
                }
                const uint64_t bal = ins1 | (acc2 ? ins2 : 0ull);
                if (ins && wr) {
                    const int at = n + (int)lanes_below(bal);
                    if (at < cap) s_band[at] = (uint16_t)q;
                    else __builtin_nontemporal_store((uint16_t)q, g_band + at);
                }
                n += (int)__popcll(bal);
                if (n + 8 > cap) {
                    // the band reaches its memory part: make this wave's stores there visible
                    // to its own later loads
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                FMM_CYC(5);
                continue;
            }
        }
        const MinPick<R> mp = band_argmin<R, W>(s_band, g_band, cap, s_psi, n FMM_CYC_ARG);
        if (mp.v > rbound) {  // beyond the restart bound: stop (deactivate past width)
            if ((double)mp.v > pd.width) active = false;
            exit_min = mp.v;
            break;
        }
        const int p = mp.idx;
        FMM_CYC_COUNT(14, n <= 64 ? 1 : 0);  // band sizes at the pick (profiling build)
        FMM_CYC_COUNT(15, n <= 256 ? 1 : 0);
        if (++npops > pop_cap) {
            raise_error(kp.ctl, kErrPopCap);
            exit_min = mp.v;
            break;
        }
        n -= 1;  // Remove_Min: the last slot moves into the hole (lanes 25-26 below)
        // Update_Neighbors(p): quads 0-5 take the six face neighbours (interior only)
        if (wid == 0) {
            // h^2/F^2 of the lane's neighbour from device memory, issued before anything
            // else of the step (the index is clamped to the tile; unused when the
            // neighbour is not interior)
            R rhs_mem = (R)0;
            if constexpr (!Gm::RHS_LDS) {
                const int ql = p + dOff;
                rhs_mem = g_rhs[ql < 0 ? 0 : (ql > T - 1 ? T - 1 : ql)];
            }
            const uint32_t up = (uint32_t)p;
            const int pi = (int)(up % P), pj = (int)((up / P) % P), pk = (int)(up / (P * P));
            const int qi = pi + dI, qj = pj + dJ, qk = pk + dK;
            const bool inb = lane < 24 && kk < 3 && (unsigned)(qi - 1) < (unsigned)B &&
                             (unsigned)(qj - 1) < (unsigned)B && (unsigned)(qk - 1) < (unsigned)B;
            const int q = inb ? p + dOff : p;
            R rhs = (R)0;
            if (inb) {
                if constexpr (Gm::RHS_LDS) rhs = s_rhs[q];
                else rhs = rhs_mem;
            }
            const uint8_t tq = s_tag[q];  // lane 24 reads the accepted point's own tag
            const R psq = s_psi[q];
            // With h^2/F^2 in LDS (small blocks) the stencil of q is read in the same
            // round trip: its points are not written in this step (the six neighbours are
            // pairwise not face-adjacent), except p's tag, which lane 24 turns KNOWN below;
            // p is taken as known instead.  Lanes without a neighbour read around an
            // interior point of the tile (unused).  With h^2/F^2 in device memory the
            // stencil is read after the check below, while that load is in flight.
            R lo[3], hi[3];
            uint32_t tlo[3], thi[3];
            if constexpr (Gm::RHS_LDS) {
                const int qs = inb ? q : kMid;
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    const int off = ax == 0 ? 1 : (ax == 1 ? P : P * P);
                    lo[ax] = s_psi[qs - off];
                    hi[ax] = s_psi[qs + off];
                    tlo[ax] = s_tag[qs - off];
                    thi[ax] = s_tag[qs + off];
                }
            }
            // Remove_Min: lane 25 moves the band's last slot into the hole, and lane 26 sets
            // the vacated LDS slot to tile point 0 (the band beyond n holds it).  The branch
            // on the wave-uniform n < cap keeps the usual all-LDS case free of any wait on
            // device memory (the h^2/F^2 load above stays in flight until the solve).
            if (n < cap) {
                const uint16_t last = (uint16_t)__builtin_amdgcn_readfirstlane(s_band[n]);
                if (lane == 25) s_band[mp.slot] = mp.slot == n ? (uint16_t)0 : last;  // mp.slot <= n < cap
                if (lane == 26 && mp.slot != n) s_band[n] = 0;
            } else {
                // every lane reads the same slot; taking it as a wave-uniform value also
                // completes the load inside this branch
                const uint16_t last =
                    (uint16_t)__builtin_amdgcn_readfirstlane(__builtin_nontemporal_load(g_band + n));
                if (lane == 25) {
                    if (mp.slot < cap) s_band[mp.slot] = last;
                    else __builtin_nontemporal_store(last, g_band + mp.slot);
                }
            }
            if (lane == 24)  // KNOWN_NEW unless KNOWN_FIX; leaves the band
                s_tag[p] = ((tq & kStatus) == kKnownFix) ? kKnownFix : kKnownNew;
            FMM_CYC(3);
            FMM_CYC_COUNT(12, 1);
            // the same in the three lanes of a quad (same neighbour, same reads)
            const bool solve = inb && (tq & kStatus) != kKnownFix && psq > mp.v;
            R t = inf, v1 = inf, v2 = inf;
            if (solve) {
                FMM_CYC_LSTART();
                R c[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    bool klo, khi;
                    if constexpr (Gm::RHS_LDS) {
                        // p is q's low neighbour for the + directions (odd quads) and its
                        // high neighbour for the - directions, on the quad's own axis
                        const bool own = ax == (g >> 1);
                        klo = is_known(tlo[ax]) || (own && (g & 1));
                        khi = is_known(thi[ax]) || (own && !(g & 1));
                    } else {
                        const int off = ax == 0 ? 1 : (ax == 1 ? P : P * P);
                        lo[ax] = s_psi[q - off];
                        hi[ax] = s_psi[q + off];
                        // p itself reads as known: lane 24 wrote its tag above, and one
                        // wave's accesses to one address complete in program order
                        klo = is_known(s_tag[q - off]);
                        khi = is_known(s_tag[q + off]);
                    }
                    c[ax] = axis_candidate<R>(psq, lo[ax], klo, hi[ax], khi);
                }
                FMM_CYC_L(8);
                FMM_CYC_LFULL(9);
                t = quad_root_k<R>(c[0], c[1], c[2], rhs, kk, v1, v2);
                FMM_CYC_L(10);
                FMM_CYC_COUNT(11, 1);
            }
            // lane 4g: the root with one candidate, then while it exceeds the next candidate
            // the root with one more (Alg. 3), from the quad's other lanes
            const R t2 = quad_bcast<1>(t), t3 = quad_bcast<2>(t);
            bool ins = false;
            if (solve && kk == 0) {
                R tf = t;
                if (v1 < inf && tf > v1) {
                    tf = t2;
                    if (v2 < inf && tf > v2) tf = t3;
                }
                if (tf < psq) {
                    s_psi[q] = tf;
                    s_tag[q] = kBand | kInBand;
                    ins = !(tq & kInBand);
                    if constexpr (!TL) {  // q on a boundary layer: its faces join Upsilon
                        mine |= (qi == 1 ? 1u : 0u) | (qi == B ? 2u : 0u) | (qj == 1 ? 4u : 0u) |
                                (qj == B ? 8u : 0u) | (qk == 1 ? 16u : 0u) | (qk == B ? 32u : 0u);
                    }
                }
            }
            FMM_CYC(4);
            const uint64_t bal = ballot(ins);
            if (ins) {
                const int at = n + (int)lanes_below(bal);
                if (at < cap) s_band[at] = (uint16_t)q;
                else __builtin_nontemporal_store((uint16_t)q, g_band + at);
            }
            n += (int)__popcll(bal);
            if (!TL || n + 8 > cap) {
                // the band reaches its memory part, or the tile is in memory: make this
                // wave's stores there visible to its own later loads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            if constexpr (W > 1) {
                if (lane == 0) s_bc[0] = n;
            }
        }
        if constexpr (W > 1) {
            __syncthreads();
            n = s_bc[0];
        } else {
            // one wave: its LDS operations complete in program order; keep the
            // compiler from moving them across iterations
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        FMM_CYC(5);
    }

    // Upsilon on the faces: a face is touched exactly when one of its boundary points got a
    // smaller value (every update of Update_Neighbors is a strict decrease, and nothing else
    // writes psi in the march); the block's tile in memory still holds the values the march
    // started from
    if constexpr (TL) {
        constexpr int NF = 6 * B * B, FPER = (NF + NT - 1) / NT;
#pragma unroll 4
        for (int k = 0; k < FPER; ++k) {
            const int e = tid + k * NT;
            if (e < NF) {
                const int t = face_point<B>(e);
                if (s_psi[t] < g_psi[t]) mine |= 1u << (e / (B * B));
            }
        }
    }
    uint32_t dirty = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) dirty |= ballot((mine >> f) & 1u) ? 1u << f : 0u;
    if constexpr (W > 1) {
        __shared__ uint32_t s_dirty[1];
        if (tid == 0) s_dirty[0] = 0u;
        __syncthreads();
        if (lane == 0 && dirty) atomicOr(s_dirty, dirty);
        __syncthreads();
        dirty = s_dirty[0];
    }
    // LDS -> tile
    if constexpr (TL) {
        copy_vec16<NT, (int)(sizeof(R) * T / 16)>(reinterpret_cast<v4u *>(g_psi),
                                                   reinterpret_cast<const FMM_LDS v4u *>(s_psi), tid);
        copy_vec16<NT, TAGB / 16>(reinterpret_cast<v4u *>(g_tag),
                                  reinterpret_cast<const FMM_LDS v4u *>(s_tag), tid);
    }
    copy_band<NT>(reinterpret_cast<v4u *>(g_band), reinterpret_cast<const FMM_LDS v4u *>(s_band),
                  n < cap ? n : cap, tid);
    if (tid == 0) {
        kp.band_n[ib] = n;
        kp.A[ib] = active ? 1 : 0;
        kp.bmin[ib] = exit_min;
        kp.lastpops[ib] = (int32_t)npops;
    }
    // C^nb(ib) <- TRUE for the neighbours whose ghosts meet Upsilon^ib
    if (tid < 6 && ((dirty >> tid) & 1u)) {
        const int64_t loc = ib - pd.blk0;
        int bx = (int)(loc % pd.mx), by = (int)((loc / pd.mx) % pd.my),
            bz = (int)(loc / ((int64_t)pd.mx * pd.my));
        const int f = tid;
        bx += (f == 1) - (f == 0);
        by += (f == 3) - (f == 2);
        bz += (f == 5) - (f == 4);
        if (bx >= 0 && by >= 0 && bz >= 0 && bx < pd.mx && by < pd.my && bz < pd.mz) {
            const int64_t nb = pd.blk0 + bx + (int64_t)pd.mx * (by + (int64_t)pd.my * bz);
            // the first flag raised on nb in this restart puts nb on the exchange list
            if (atomicOr(&kp.Cm[nb], 1u << (f ^ 1)) == 0u) {
                const int pos = atomicAdd(sink.xn, 1);
                if (pos < sink.cap) sink.xl[pos] = (int32_t)nb;
                else raise_error(kp.ctl, kErrList);  // cannot happen: one entry per block
            }
        }
    }
    a_out = active;
    n_out = n;
    pops_out = npops;
    pops_acc += (unsigned long long)npops;
    if (kp.nprob > 1 && tid == 0) atomicAdd(&kp.prob_pops[kp.blk_prob[ib]], (unsigned long long)npops);
    __syncthreads();  // LDS is reused by the next block
    FMM_CYC_FULL(7);
}

// ---------------------------------------------------------------- Alg. 5 on one block
// Integrate_Ghost_Cell_Data(ib) for the faces flagged in cm.  Every ghost point
// of a flagged face is compared with the point it copies in the neighbour
// (the whole face, which fires exactly on the points the neighbour updated in
// this restart: a ghost copy only ever holds an earlier, larger-or-equal value
// of the monotonically decreasing neighbour value).  A smaller neighbour value
// is copied with its category and enters (or moves up in) ib's band.  Then C is
// cleared and the block is activated when its band minimum is within width.
// Works directly on the tiles in device memory; returns the new activation and
// band size to every thread.
template <typename R, int B, int W>
__device__ void exchange_block(const KParams<R> &kp, int64_t ib, uint32_t cm, const ProbDesc &pd,
                               char *smem, bool &a_out, int &n_out)
{
    constexpr int P = Geo<B>::P, T = Geo<B>::T, NT = 64 * W, FB = B * B, BAND = Geo<B>::BAND,
                  TAGB = Geo<B>::TAGB;
    const int tid = threadIdx.x;
    __shared__ int s_cnt[1];
    using U = typename std::conditional<sizeof(R) == 4, uint32_t, unsigned long long>::type;
    __shared__ U s_min[1];
    if (tid == 0) {
        s_cnt[0] = 0;
        const R inf = (R)INFINITY;
        U ib_bits;
        __builtin_memcpy(&ib_bits, &inf, sizeof(R));
        s_min[0] = ib_bits;
    }
    __syncthreads();
    const int64_t loc = ib - pd.blk0;
    const int bx = (int)(loc % pd.mx), by = (int)((loc / pd.mx) % pd.my),
              bz = (int)(loc / ((int64_t)pd.mx * pd.my));
    R *g_psi = kp.psi_t + ib * (int64_t)T;
    uint8_t *g_tag = kp.tag_t + ib * (int64_t)TAGB;
    uint16_t *g_band = kp.band_t + ib * (int64_t)BAND;
    const int n0 = kp.band_n[ib];
    U my_min = ~(U)0;
    for (int e = tid; e < 6 * FB; e += NT) {
        const int f = e / FB;
        if (!((cm >> f) & 1u)) continue;
        const int a = e % FB % B + 1, b = e % FB / B + 1;
        const int axis = f >> 1, side = f & 1;
        const int nbx = bx + (f == 1) - (f == 0), nby = by + (f == 3) - (f == 2),
                  nbz = bz + (f == 5) - (f == 4);
        const int64_t nb = pd.blk0 + nbx + (int64_t)pd.mx * (nby + (int64_t)pd.my * nbz);
        const int gl = side ? B + 1 : 0;  // ghost layer of ib on face f
        const int nl = side ? 1 : B;      // boundary layer of nb facing ib
        int gt, st;
        if (axis == 0) {
            gt = gl + P * (a + P * b);
            st = nl + P * (a + P * b);
        } else if (axis == 1) {
            gt = a + P * (gl + P * b);
            st = a + P * (nl + P * b);
        } else {
            gt = a + P * (b + P * gl);
            st = a + P * (b + P * nl);
        }
        const R vn = kp.psi_t[nb * (int64_t)T + st];
        const R vi = g_psi[gt];
        if (vi > vn) {
            const uint8_t tn = kp.tag_t[nb * (int64_t)TAGB + st];
            const uint8_t ti = g_tag[gt];
            g_psi[gt] = vn;
            g_tag[gt] = (uint8_t)((tn & kStatus) | kInBand);
            if (!(ti & kInBand)) {
                const int pos = atomicAdd(s_cnt, 1);
                g_band[n0 + pos] = (uint16_t)gt;
            }
            U vb;
            __builtin_memcpy(&vb, &vn, sizeof(R));
            if (vb < my_min) my_min = vb;
        }
    }
    if (my_min != ~(U)0) atomicMin(s_min, my_min);
    __syncthreads();
    __shared__ int s_res[2];
    if (tid == 0) {
        const int nn = n0 + s_cnt[0];
        R cmin;
        U mb = s_min[0];
        __builtin_memcpy(&cmin, &mb, sizeof(R));
        R bm = kp.bmin[ib];
        if (cmin < bm) bm = cmin;
        kp.bmin[ib] = bm;
        kp.band_n[ib] = nn;
        kp.Cm[ib] = 0u;
        bool a = kp.A[ib] != 0;
        if (nn > 0 && (double)bm <= pd.width) a = true;
        kp.A[ib] = a ? 1 : 0;
        s_res[0] = nn;
        s_res[1] = a ? 1 : 0;
    }
    __syncthreads();
    n_out = s_res[0];
    a_out = s_res[1] != 0;
    __syncthreads();
}

// ---------------------------------------------------------------- phase drivers
// Band-size bin of the restart features (see fmm.h).
__device__ __forceinline__ int band_bin(int nb)
{
    return nb >= 4096 ? 7 : nb >= 1024 ? 6 : nb >= 256 ? 5 : nb >= 64 ? 4 : nb >= 16 ? 3
           : nb >= 4 ? 2 : nb >= 1 ? 1 : 0;
}

// Put active block ib on the march list of the next restart, list[(r + 1) & 1], in
// one of 4 bins by its expected work est (longest first), and add it to the restart
// features.  One thread per block.
template <typename R>
__device__ void append_next(const KParams<R> &kp, const ListSink &sink, int64_t r, int64_t ib, int est,
                            int nb, unsigned long long *lfeat)
{
    Ctl *ctl = kp.ctl;
    const int k = est >= 768 ? 0 : (est >= 256 ? 1 : (est >= 64 ? 2 : 3));
    const int pos = atomicAdd(&sink.bins[k], 1);
    if (pos < sink.cap) sink.next[(int64_t)k * sink.stride + pos] = (int32_t)ib;
    else raise_error(ctl, kErrList);  // cannot happen: one entry per block
    atomicAdd(sink.nlist, 1);
    if (kp.want_features) {  // the work-group's sums, added to ctl->feat by flush_features
        lfeat[band_bin(nb)] += 1ull;
        lfeat[8] += (unsigned long long)((double)kp.fmean[ib] * kFixScale + 0.5);
    }
    if (kp.nprob > 1) atomicMax(&kp.prob_lastr[kp.blk_prob[ib]], (int)r);
}

// Counts a work-group gathers over its phases (thread 0's copy), added to the control
// block once, when the kernel ends.
struct Totals {
    unsigned long long pops = 0, march_calls = 0, tile_loads = 0, exchange_calls = 0;
};

__device__ __forceinline__ void flush_totals(Ctl *ctl, const Totals &t)
{
    if (t.march_calls) {
        atomicAdd(&ctl->pops, t.pops);
        atomicAdd(&ctl->march_calls, t.march_calls);
        atomicAdd(&ctl->tile_loads, t.tile_loads);
    }
    if (t.exchange_calls) atomicAdd(&ctl->exchange_calls, t.exchange_calls);
}

// The restart features a work-group gathered in one phase (integer sums, so the order in
// which work-groups add them does not matter), one atomic per nonzero entry.
__device__ __forceinline__ void flush_features(Ctl *ctl, int cn, const unsigned long long *lfeat)
{
    for (int k = 0; k < 9; ++k)
        if (lfeat[k]) atomicAdd(&ctl->feat[cn][k], lfeat[k]);
}

// Marching step of restart r: blocks of the march list list[r & 1] are taken
// from a work queue, longest expected march first: the list is binned when it
// is built by each block's expected work (the pops of its previous march or its
// band size, whichever is larger), a cheap longest-job-first order that shortens
// the wait for the slowest block at the barrier.  A block whose exact band
// minimum is above its bound is not loaded: Alg. 4 would stop at once without
// changing anything (only the width test can flip its activation).  A block
// that stays active goes on the next march list right away (an exchange can
// only activate a block, never deactivate it).
template <typename R, int B, int W>
__device__ void march_phase(const KParams<R> &kp, int64_t r, double lbound, char *smem, int G, int w,
                            Totals &tot FMM_CYC_PARAM)
{
    const int c = (int)(r & 1);
    const int tid = threadIdx.x;
    Ctl *ctl = kp.ctl;
    const int32_t *cur = c ? kp.list1 : kp.list0;
    const int ncur = __hip_atomic_load(&ctl->n_list[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __shared__ int s_bins[3];
    __shared__ unsigned long long s_feat[9];
    if (tid < 3) s_bins[tid] = __hip_atomic_load(&ctl->bin_n[c][tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid < 9) s_feat[tid] = 0ull;
    __syncthreads();
    const int bn0 = s_bins[0], bn1 = s_bins[1], bn2 = s_bins[2];
    __shared__ int s_item[1];
    unsigned long long pops = 0, mcalls = 0, loads = 0;
    // item w goes to work-group w without touching the queue; items from G on come from
    // the queue, which a list no longer than the grid never reaches
    for (int it = 0;; ++it) {
        int item = w;
        if (it > 0) {
            if (G >= ncur) break;
            if (tid == 0) s_item[0] = G + atomicAdd(&ctl->q_head[c], 1);
            __syncthreads();
            item = s_item[0];
            __syncthreads();
        }
        if (item >= ncur) break;
        // bins in order: the blocks with the most expected work first
        int k = 0, off = item;
        if (off >= bn0) {
            off -= bn0;
            k = 1;
            if (off >= bn1) {
                off -= bn1;
                k = 2;
                if (off >= bn2) {
                    off -= bn2;
                    k = 3;
                }
            }
        }
        if (off >= kp.nblk) {  // counts out of step with the list: stop, never read past it
            if (tid == 0) raise_error(ctl, kErrList);
            break;
        }
        const int64_t ib = cur[(int64_t)k * kp.nblk + off];
        if ((uint64_t)ib >= (uint64_t)kp.nblk) {
            if (tid == 0) raise_error(ctl, kErrList);
            break;
        }
        const ProbDesc pd = kp.nprob == 1 ? kp.prob[0] : kp.prob[kp.blk_prob[ib]];
        const double bound = kp.stride_mode ? lbound : fixed_bound(r, pd.stride, pd.width);
        ++mcalls;
        const R bm = kp.bmin[ib];
        if ((double)bm > bound) {
            if (tid == 0) {
                if ((double)bm > pd.width) kp.A[ib] = 0;
                else {
                    const int nb = kp.band_n[ib];
                    append_next<R>(kp, launch_sink(kp, c), r, ib, max(kp.lastpops[ib], nb), nb, s_feat);
                }
            }
            continue;
        }
        ++loads;
        if (kp.trace && tid == 0) {  // the block accepts its band minimum first
            const double v = (double)bm;
            unsigned long long vb;
            __builtin_memcpy(&vb, &v, sizeof(v));
            atomicMin(&ctl->rmin[c], vb);
        }
        bool a;
        int nb, np;
        const ListSink sink = launch_sink(kp, c);
        march_block<R, B, W>(kp, ib, pd, bound, sink, smem, pops, a, nb, np FMM_CYC_ARG);
        if (tid == 0 && a) append_next<R>(kp, sink, r, ib, max(np, nb), nb, s_feat);
    }
    if (tid == 0 && kp.want_features) flush_features(ctl, c ^ 1, s_feat);
    tot.pops += pops;
    tot.march_calls += mcalls;
    tot.tile_loads += loads;
    if (kp.trace && tid == 0 && pops) atomicAdd(&ctl->rpops[c], pops);  // the restart's pops
}

// Exchanging step of restart r: the blocks whose C flags were raised in this
// restart's marching step (the exchange list, built as the flags went up) are
// taken from a work queue and run Alg. 5.  A block that the exchange activates
// joins the next march list; for a block that was already on it the band-size
// feature moves to the bin of its new band size.
template <typename R, int B, int W>
__device__ void exchange_phase(const KParams<R> &kp, int64_t r, char *smem, int G, int w, Totals &tot)
{
    const int c = (int)(r & 1);
    const int tid = threadIdx.x;
    Ctl *ctl = kp.ctl;
    const int nx = __hip_atomic_load(&ctl->x_n[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __shared__ int s_item[1];
    __shared__ unsigned long long s_feat[9];
    if (tid < 9) s_feat[tid] = 0ull;  // by wave 0, the only wave that adds to it and reads it
    unsigned long long xcalls = 0;
    // item w to work-group w, then the queue from G on (as in the marching step)
    for (int it = 0;; ++it) {
        int item = w;
        if (it > 0) {
            if (G >= nx) break;
            if (tid == 0) s_item[0] = G + atomicAdd(&ctl->x_head[c], 1);
            __syncthreads();
            item = s_item[0];
            __syncthreads();
        }
        if (item >= nx) break;
        const int64_t ib = item < kp.nblk ? kp.xlist[item] : -1;
        if ((uint64_t)ib >= (uint64_t)kp.nblk) {
            if (tid == 0) raise_error(ctl, kErrList);
            break;
        }
        const uint32_t cm = kp.Cm[ib];
        const bool a0 = kp.A[ib] != 0;
        const int n0 = kp.band_n[ib];
        const ProbDesc pd = kp.nprob == 1 ? kp.prob[0] : kp.prob[kp.blk_prob[ib]];
        bool an;
        int nn;
        exchange_block<R, B, W>(kp, ib, cm, pd, smem, an, nn);
        ++xcalls;
        if (tid == 0) {
            if (an && !a0) {
                append_next<R>(kp, launch_sink(kp, c), r, ib, max(kp.lastpops[ib], nn), nn, s_feat);
            } else if (a0 && kp.want_features && band_bin(nn) != band_bin(n0)) {
                s_feat[band_bin(n0)] += ~0ull;  // -1 (modulo 2^64, like the totals)
                s_feat[band_bin(nn)] += 1ull;
            }
        }
    }
    if (tid == 0 && kp.want_features) flush_features(ctl, c ^ 1, s_feat);
    tot.exchange_calls += xcalls;
}

// ---------------------------------------------------------------- stride network
// m = exp(ln(1/4) + sigmoid(z) ln 32) for the standardised features, FP32, evaluated by
// each wave on its lanes: lane o (o < 32) computes hidden unit o of each layer from its
// own row of weights, and reads the other units from their lanes.  Every sum runs in the
// same order as the layers' definition, so every work-group gets the same m.
__device__ float mlp_multiplier(const float *blob, const float *raw)
{
    const float *W1 = blob, *b1 = W1 + 32 * 12, *W2 = b1 + 32, *b2 = W2 + 32 * 32, *W3 = b2 + 32,
                *b3 = W3 + 32, *mu = b3 + 1, *sd = mu + 12;
    const int o = (int)(threadIdx.x & 31);
    float x[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) x[i] = (raw[i] - mu[i]) / sd[i];
    float s1 = b1[o];
#pragma unroll
    for (int i = 0; i < 12; ++i) s1 += W1[o * 12 + i] * x[i];
    const float h1 = s1 > 0.f ? s1 : 0.f;
    float s2 = b2[o];
#pragma unroll
    for (int i = 0; i < 32; ++i)
        s2 += W2[o * 32 + i] * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h1), i));
    const float t = W3[o] * (s2 > 0.f ? s2 : 0.f);
    float z = b3[0];
#pragma unroll
    for (int k = 0; k < 32; ++k) z += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), k));
    const float sig = 1.0f / (1.0f + expf(-z));
    const float m = expf((float)kLogMinMult + sig * (float)kLogSpanMult);
    return m;
}

// Raw features at the end of restart r (see fmm.h); n_next > 0.
__device__ void restart_features(const Ctl *ctl, int cn, int n_next, int64_t nblk, double bound,
                                 int64_t r, const ProbDesc &pd, float *f)
{
    const double inv = 1.0 / (double)n_next;
    f[0] = (float)(bound / ((double)pd.nmax * pd.h));
    f[1] = (float)((double)n_next / (double)nblk);
    for (int k = 0; k < 8; ++k) f[2 + k] = (float)((double)ctl->feat[cn][k] * inv);
    f[10] = (float)((double)r / (double)pd.nmax);
    f[11] = (float)((double)ctl->feat[cn][8] / kFixScale * inv);
}

// ---------------------------------------------------------------- persistent restart loop
// The whole main loop of Alg. 6 in one cooperative launch; two grid barriers
// per restart (after the marching step, after the exchanging step).  The bound
// lives in registers, identical in every work-group.
template <typename R, int B, int W>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(Lds<R, B, W>::waves_per_simd))) k_persistent(KParams<R> kp)
{
    extern __shared__ __align__(16) char smem[];
    const int G = (int)gridDim.x, w = (int)blockIdx.x, tid = threadIdx.x;
    Ctl *ctl = kp.ctl;
    if (read_abort(ctl)) return;
    const ProbDesc &p0 = kp.prob[0];
    double prev_bound = 0.0, lstride = p0.stride, lbound = 0.0;
    if (kp.r0 > 0) {  // resumed after restart r0 (fixed stride or a bound schedule)
        prev_bound = kp.stride_mode == 2
                         ? (kp.r0 <= kp.nsched ? kp.sched[kp.r0 - 1]
                                               : kp.sched[kp.nsched - 1] + (double)(kp.r0 - kp.nsched) * p0.stride)
                         : fixed_bound(kp.r0, p0.stride, p0.width);
        if (prev_bound > p0.width) prev_bound = p0.width;
    }
    Totals tot;
    FMM_CYC_DECL;
    for (int64_t r = kp.r0 + 1;; ++r) {
        const int c = (int)(r & 1);
        if (kp.stride_mode == 1) {
            lbound = prev_bound + lstride;
            if (lbound > p0.width) lbound = p0.width;
        } else if (kp.stride_mode == 2) {
            // a given bound sequence, then the last bound plus the stride per restart
            lbound = r <= kp.nsched ? kp.sched[r - 1]
                                    : kp.sched[kp.nsched - 1] + (double)(r - kp.nsched) * p0.stride;
            if (lbound > p0.width) lbound = p0.width;
        }
        int64_t t0 = 0;
        // Counters of the next restart's queues.  The next march list, list[c ^ 1], is
        // appended to from this restart's marching step on, so its size, bins and
        // features were cleared after the marching step of the previous restart (below).
        if (w == 0 && tid == 0) {
            ctl->q_head[c ^ 1] = 0;
            ctl->rpops[c ^ 1] = 0;
            ctl->rmin[c ^ 1] = ~0ull;
            ctl->x_n[c ^ 1] = 0;
            ctl->x_head[c ^ 1] = 0;
            t0 = wall_ticks();
        }
        const int ncur = __hip_atomic_load(&ctl->n_list[c], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        march_phase<R, B, W>(kp, r, lbound, smem, G, w, tot FMM_CYC_ARG);
        grid_barrier(ctl, (unsigned)G, kp.timeout_ticks);
        if (read_abort(ctl)) break;
        // list[c] has been consumed: clear its counters for restart r + 1, which appends
        // to it (nothing reads or appends to them again before the next barrier)
        if (w == 0 && tid == 0) {
            ctl->n_list[c] = 0;
            for (int k = 0; k < 4; ++k) ctl->bin_n[c][k] = 0;
            for (int k = 0; k < 10; ++k) ctl->feat[c][k] = 0;
        }
        exchange_phase<R, B, W>(kp, r, smem, G, w, tot);
        grid_barrier(ctl, (unsigned)G, kp.timeout_ticks);
        if (read_abort(ctl)) break;
        const int nnext = __hip_atomic_load(&ctl->n_list[c ^ 1], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        const double bound_r = kp.stride_mode ? lbound : fixed_bound(r, p0.stride, p0.width);
        float feat[12];
        if (kp.want_features && nnext > 0)
            restart_features(ctl, c ^ 1, nnext, kp.nblk, bound_r, r, p0, feat);
        if (w == 0 && tid == 0 && kp.trace && r <= kp.trace_cap) {
            TraceRow *row = reinterpret_cast<TraceRow *>(kp.trace) + (r - 1);
            for (int k = 0; k < 12; ++k) row->feat[k] = nnext > 0 ? feat[k] : 0.f;
            row->bound = bound_r;
            row->stride_used = bound_r - prev_bound;
            row->pops = (int64_t)ctl->rpops[c];
            row->t_start = t0;
            row->t_end = wall_ticks();
            row->active = ncur;
            row->next_active = nnext;
            const unsigned long long mb = ctl->rmin[c];
            double mv = INFINITY;
            if (mb != ~0ull) __builtin_memcpy(&mv, &mb, sizeof(mv));
            row->min_popped = mv;
        }
        if (nnext == 0) {
            if (w == 0 && tid == 0) {
                ctl->restarts = r;
                ctl->final_bound = bound_r;
            }
            break;
        }
        if (r >= kp.max_restarts) {
            if (w == 0 && tid == 0) {
                raise_error(ctl, kErrRestarts);
                ctl->restarts = r;
                ctl->final_bound = bound_r;
            }
            break;
        }
        if (kp.stride_mode == 1) {
            float m = 1.0f;
            if (kp.mlp) {
                m = mlp_multiplier(kp.mlp, feat);
                if (!(m >= 0.25f && m <= 8.0f)) m = 1.0f;  // not finite or out of range
            }
            prev_bound = lbound;
            lstride = (double)m * p0.stride;
        } else {
            prev_bound = bound_r;
        }
    }
    if (tid == 0) flush_totals(ctl, tot);
#ifdef FMM_CYCLES
    cyc.flush();
#endif
}

// ---------------------------------------------------------------- batches: restarts per problem
// A batch whose problems restart on their own: no barrier is shared between problems.
// Each problem runs Alg. 6 as a sequence of phases (the marching step of restart r, then
// its exchanging step), each a list of work items (blocks).  A work-group takes a token
// of some problem from the ready queue and claims that problem's items one at a time
// (one atomic on the problem's phase word); the work-group that finishes a phase's last
// item starts the problem's next phase and puts its tokens in the queue.  Within a problem
// the phases follow each other as in the launch-wide loop, with the same lists, so every
// problem's psi and counts are those of its own solve.

// The ready queue: a bounded ring of 64-bit slots (sequence << 32 | problem) in which every
// producer and consumer takes a position by compare-and-swap and waits on the slot's
// sequence (the classic bounded multi-producer multi-consumer queue).  A problem keeps at
// most kp.tokens tokens in it (SolveState::queued) and the capacity is at least that many
// per problem, so a push never finds it full.
// Every wait in the queue ends: each pass that does not take a slot counts a poll, and every
// 64 polls the work-group reads the abort flag and the watchdog.  The watchdog measures time
// in which no phase of any problem started (Ctl::progress); phases are finite, so once they
// stop the waits run out.
template <typename R>
__device__ __forceinline__ bool ring_wait_over(const KParams<R> &kp, int &polls, unsigned long long &seen,
                                               int64_t &t0)
{
    if ((++polls & 63) != 0) return false;
    Ctl *ctl = kp.ctl;
    if (read_abort(ctl)) return true;
    const unsigned long long pr = __hip_atomic_load(&ctl->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (pr != seen) {  // phases are still starting: progress
        seen = pr;
        t0 = wall_ticks();
        return false;
    }
    if (wall_ticks() - t0 > kp.timeout_ticks) {
        raise_error(ctl, kErrTimeout);
        return true;
    }
    return false;
}

template <typename R>
__device__ void ring_push(const KParams<R> &kp, int q)
{
    Ctl *ctl = kp.ctl;
    unsigned long long pos = __hip_atomic_load(&ctl->rq_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long seen = __hip_atomic_load(&ctl->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t t0 = wall_ticks();
    int polls = 0;
    for (;;) {
        unsigned long long *slot = kp.ring + (pos & kp.ring_mask);
        const unsigned long long v = __hip_atomic_load(slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const int dif = (int)((uint32_t)(v >> 32) - (uint32_t)pos);
        if (dif == 0) {
            if (__hip_atomic_compare_exchange_strong(&ctl->rq_tail, &pos, pos + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(slot, ((unsigned long long)(uint32_t)(pos + 1) << 32) | (uint32_t)q,
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            // pos now holds the current tail
        } else {
            if (dif < 0) __builtin_amdgcn_s_sleep(2);  // full: cannot happen with the capacity chosen
            pos = __hip_atomic_load(&ctl->rq_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ring_wait_over<R>(kp, polls, seen, t0)) return;  // aborting: the token is not needed
    }
}

// A token, or -1 when every problem has finished, the launch is aborting, or no token was
// put in anywhere for the watchdog's time.
template <typename R>
__device__ int ring_pop(const KParams<R> &kp)
{
    Ctl *ctl = kp.ctl;
    if (read_abort(ctl)) return -1;
    unsigned long long pos = __hip_atomic_load(&ctl->rq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long seen = __hip_atomic_load(&ctl->progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int64_t t0 = wall_ticks();
    int polls = 0, nap = 1;
    for (;;) {
        unsigned long long *slot = kp.ring + (pos & kp.ring_mask);
        const unsigned long long v = __hip_atomic_load(slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const int dif = (int)((uint32_t)(v >> 32) - (uint32_t)(pos + 1));
        if (dif == 0) {
            if (__hip_atomic_compare_exchange_strong(&ctl->rq_head, &pos, pos + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(slot, (unsigned long long)(uint32_t)(pos + kp.ring_mask + 1) << 32,
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                const int q = (int)(uint32_t)v;
                if (q >= kp.nprob) return q;  // the caller reports it
                // acquire: a phase start that counted this token stored its phase word first
                __hip_atomic_fetch_add(&kp.solves[q].queued, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                return q;
            }
            // pos now holds the current head
        } else {
            if (dif < 0) {  // empty: poll less often the longer it stays empty (up to ~4k cycles)
                if (__hip_atomic_load(&ctl->remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0)
                    return -1;
                for (int k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(4);
                nap = nap < 16 ? 2 * nap : 16;
            }
            pos = __hip_atomic_load(&ctl->rq_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ring_wait_over<R>(kp, polls, seen, t0)) return -1;
    }
}

// Problem q enters `phase` with n items: its claims and finished items start from zero.
// The work-group calling this (the one that finished the previous phase) goes on claiming
// q's items itself, so the phase always has a worker; the queue is topped up with tokens
// for ceil(n / kItemsPerToken) - 1 more work-groups (at most kp.tokens - 1), with at most
// that many pushes (other work-groups may pop them as fast as they come, so the count
// alone would not end the loop).  A token still queued from an earlier phase counts:
// whoever pops it claims from the new phase word, which is stored before the count is
// read.  A problem never holds more than kp.tokens queue slots, and its tokens, hence the
// claims beyond n in one phase, stay bounded.  One thread.
template <typename R>
__device__ void batch_start(const KParams<R> &kp, int q, int64_t phase, int n)
{
    SolveState &st = kp.solves[q];
    st.done = 0;  // ordered before the phase word by the release below
    __hip_atomic_store(&st.word, ((unsigned long long)phase << 40) | ((unsigned long long)n << 20),
                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&kp.ctl->progress, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int helpers = (n + kItemsPerToken - 1) / kItemsPerToken - 1;
    const int want = helpers < kp.tokens - 1 ? helpers : kp.tokens - 1;
    for (int k = 0; k < want; ++k) {
        const int had = __hip_atomic_fetch_add(&st.queued, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (had >= want) {
            __hip_atomic_fetch_add(&st.queued, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        ring_push<R>(kp, q);
    }
}

// The last item of problem q's `phase` is done (one thread, after an acquire): the next
// phase, the next restart, or the end of the problem's solve.
template <typename R>
__device__ void batch_advance(const KParams<R> &kp, int q, int64_t phase)
{
    SolveState &st = kp.solves[q];
    const int64_t r = phase / 2 + 1;
    const int c = (int)(r & 1);
    if ((phase & 1) == 0) {
        // restart r's marching step is over; its march list is consumed
        st.n_list[c] = 0;
        for (int k = 0; k < 4; ++k) st.bin_n[c][k] = 0;
        const int nx = st.x_n[c];
        if (nx > 0) {
            batch_start<R>(kp, q, phase + 1, nx);
            return;
        }
    }
    // restart r is over; its exchange list is consumed
    st.x_n[c] = 0;
    const int nn = st.n_list[c ^ 1];
    if (nn == 0 || r >= kp.max_restarts) {
        if (nn > 0) raise_error(kp.ctl, kErrRestarts);
        st.r = (int)r;
        st.finished = 1;
        kp.prob_lastr[q] = (int)r - 1;  // restarts = this + 1, as in the shared loop
        __hip_atomic_store(&st.word, (unsigned long long)(phase + 1) << 40, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&kp.ctl->remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    st.r = (int)r + 1;
    batch_start<R>(kp, q, 2 * r, nn);  // the marching step of restart r + 1
}

template <typename R, int B, int W>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(Lds<R, B, W>::waves_per_simd))) k_batched(KParams<R> kp)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x;
    Ctl *ctl = kp.ctl;
    SolveState *S = kp.solves;
    __shared__ int s_q, s_keep, s_stop;
    __shared__ unsigned long long s_w;
    __shared__ unsigned long long s_feat[9];  // no restart features in batches
    if (tid < 9) s_feat[tid] = 0ull;
    Totals tot;
    FMM_CYC_DECL;
    int q = -1;  // (ring_pop, thread 0's first step, reads the abort flag)
    // Memory ordering once per phase, not per item (thread 0's state): the acquire when this
    // work-group first claims an item of a phase (what it reads was written in earlier
    // phases, by any work-group on any XCD), and the release when the phase has no item
    // left for it, before its finished items are counted (pend of them, of a phase of
    // pend_n items).  The phase cannot end before that count, and this work-group makes it
    // at its very next claim, so nothing waits on the delay.
    int cur_q = -1, pend = 0, pend_n = 0;
    int64_t cur_phase = -1, pend_phase = -1;
    for (;;) {
        if (q < 0) {
            if (tid == 0) s_q = ring_pop<R>(kp);
            __syncthreads();
            q = s_q;
            __syncthreads();
            if (q < 0) break;
            if (q >= kp.nprob) {  // a token that names no problem: stop, never index with it
                if (tid == 0) raise_error(ctl, kErrList);
                break;
            }
        }
        // thread 0 decides for the work-group (the abort flag read once, so every wave
        // takes the same branch)
        if (tid == 0) s_stop = read_abort(ctl);
        __syncthreads();
        if (s_stop) break;
        if (tid == 0) {
            const unsigned long long w0 =
                __hip_atomic_fetch_add(&S[q].word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t ph = (int64_t)(w0 >> 40);
            const int nn = (int)((w0 >> 20) & 0xFFFFFu), ii = (int)(w0 & 0xFFFFFu);
            int keep = 1;
            if (ii >= nn) {
                // no item left for this work-group: count the ones it finished; the
                // work-group that completes the phase moves q on and keeps working on it
                keep = 0;
                if (pend > 0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    const int d = __hip_atomic_fetch_add(&S[q].done, pend, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if (d + pend == pend_n) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        batch_advance<R>(kp, q, pend_phase);
                        keep = 1;
                    }
                    pend = 0;
                }
            } else if (q != cur_q || ph != cur_phase) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the phase's lists and tiles
                cur_q = q;
                cur_phase = ph;
            }
            s_w = w0;
            s_keep = keep;
        }
        __syncthreads();
        const unsigned long long wv = s_w;
        const int keep = s_keep;
        __syncthreads();
        const int64_t phase = (int64_t)(wv >> 40);
        const int n = (int)((wv >> 20) & 0xFFFFFu), i = (int)(wv & 0xFFFFFu);
        if (i >= n) {  // drained: drop the token unless this work-group moved q on
            if (!keep) q = -1;
            continue;
        }
        const ProbDesc pd = kp.prob[q];
        const int64_t r = phase / 2 + 1;
        const int c = (int)(r & 1);
        const ListSink sink{(c ? kp.list0 : kp.list1) + pd.blk0, S[q].bin_n[c ^ 1], &S[q].n_list[c ^ 1],
                            kp.xlist + pd.blk0, &S[q].x_n[c], kp.nblk, pd.nblk};
        bool bad = false;
        if ((phase & 1) == 0) {
            // marching step of restart r, item i: the bins in order, the most expected work first
            const int32_t *cur = (c ? kp.list1 : kp.list0) + pd.blk0;
            int k = 0, off = i;
            while (k < 3 && off >= S[q].bin_n[c][k]) {
                off -= S[q].bin_n[c][k];
                ++k;
            }
            const int64_t ib = off < pd.nblk ? (int64_t)cur[(int64_t)k * kp.nblk + off] : -1;
            if (ib < pd.blk0 || ib >= pd.blk0 + pd.nblk) {
                bad = true;
            } else {
                const double bound = fixed_bound(r, pd.stride, pd.width);
                ++tot.march_calls;
                const R bm = kp.bmin[ib];
                if ((double)bm > bound) {
                    if (tid == 0) {
                        if ((double)bm > pd.width) kp.A[ib] = 0;
                        else {
                            const int nbb = kp.band_n[ib];
                            append_next<R>(kp, sink, r, ib, max(kp.lastpops[ib], nbb), nbb, s_feat);
                        }
                    }
                } else {
                    ++tot.tile_loads;
                    bool a;
                    int nbb, np;
                    march_block<R, B, W, false>(kp, ib, pd, bound, sink, smem, tot.pops, a, nbb, np FMM_CYC_ARG);
                    if (tid == 0 && a) append_next<R>(kp, sink, r, ib, max(np, nbb), nbb, s_feat);
                }
            }
        } else {
            // exchanging step of restart r, item i
            const int64_t ib = kp.xlist[pd.blk0 + i];
            if (ib < pd.blk0 || ib >= pd.blk0 + pd.nblk) {
                bad = true;
            } else {
                const uint32_t cm = kp.Cm[ib];
                const bool a0 = kp.A[ib] != 0;
                bool an;
                int nn;
                exchange_block<R, B, W>(kp, ib, cm, pd, smem, an, nn);
                ++tot.exchange_calls;
                if (tid == 0 && an && !a0) append_next<R>(kp, sink, r, ib, max(kp.lastpops[ib], nn), nn, s_feat);
            }
        }
        if (bad) {  // lists out of step with their counts: stop, never read past them
            if (tid == 0) raise_error(ctl, kErrList);
            break;
        }
        // the item is done (every lane's writes are complete: both steps end with a
        // barrier); it is counted, with the release, when the phase runs dry for this
        // work-group
        if (tid == 0) {
            ++pend;
            pend_n = n;
            pend_phase = phase;
        }
    }
    if (tid == 0) flush_totals(ctl, tot);
}

// ---------------------------------------------------------------- host-driven loop
template <typename R>
__global__ void k_restart_prologue(KParams<R> kp, int64_t r)
{
    const int c = (int)(r & 1);
    Ctl *ctl = kp.ctl;
    ctl->n_list[c ^ 1] = 0;
    ctl->q_head[c ^ 1] = 0;
    ctl->rpops[c ^ 1] = 0;
    ctl->rmin[c ^ 1] = ~0ull;
    ctl->x_n[c ^ 1] = 0;
    ctl->x_head[c ^ 1] = 0;
    for (int k = 0; k < 4; ++k) ctl->bin_n[c ^ 1][k] = 0;
    for (int k = 0; k < 10; ++k) ctl->feat[c ^ 1][k] = 0;
}

template <typename R, int B, int W>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(Lds<R, B, W>::waves_per_simd))) k_march(KParams<R> kp, int64_t r)
{
    extern __shared__ __align__(16) char smem[];
    if (read_abort(kp.ctl)) return;
    Totals tot;
    FMM_CYC_DECL;
    march_phase<R, B, W>(kp, r, 0.0, smem, (int)gridDim.x, (int)blockIdx.x, tot FMM_CYC_ARG);
    if (threadIdx.x == 0) flush_totals(kp.ctl, tot);
}

template <typename R, int B, int W>
__global__ void __launch_bounds__(64 * W) k_exchange(KParams<R> kp, int64_t r)
{
    extern __shared__ __align__(16) char smem[];
    if (read_abort(kp.ctl)) return;
    Totals tot;
    exchange_phase<R, B, W>(kp, r, smem, (int)gridDim.x, (int)blockIdx.x, tot);
    if (threadIdx.x == 0) flush_totals(kp.ctl, tot);
}

// ---------------------------------------------------------------- Alg. 1 and layout
// Per block: psi <- +inf and G <- FAR on the padded tile, empty band, A <- F,
// C <- F; h^2/F^2 of the interior from the caller's linear F; mean speed.
template <typename R, int B>
__global__ void __launch_bounds__(256) k_init(KParams<R> kp)
{
    constexpr int T = Geo<B>::T, B3 = Geo<B>::B3, TAGB = Geo<B>::TAGB;
    __shared__ float s_sum[256];
    const int tid = threadIdx.x;
    for (int64_t ib = blockIdx.x; ib < kp.nblk; ib += gridDim.x) {
        const ProbDesc &pd = kp.prob[kp.blk_prob[ib]];
        const int64_t loc = ib - pd.blk0;
        const int64_t bx = loc % pd.mx, by = (loc / pd.mx) % pd.my, bz = loc / ((int64_t)pd.mx * pd.my);
        R *gp = kp.psi_t + ib * (int64_t)T;
        uint8_t *gt = kp.tag_t + ib * (int64_t)TAGB;
        for (int t = tid; t < T; t += 256) gp[t] = (R)INFINITY;
        for (int t = tid; t < TAGB; t += 256) gt[t] = kFar;
        R *gr = kp.rhs_t + ib * (int64_t)T;
        const R *F = reinterpret_cast<const R *>(pd.F);
        const R hh = (R)pd.h;
        float fsum = 0.f;
        bool bad = false;
        for (int e = tid; e < B3; e += 256) {
            const int li = e % B, lj = (e / B) % B, lk = e / (B * B);
            const int64_t g = (bx * B + li) + (int64_t)pd.nx * ((by * B + lj) + (int64_t)pd.ny * (bz * B + lk));
            const R f = F[g];
            if (!(f >= (R)0) || !(f < (R)INFINITY)) bad = true;
            gr[(li + 1) + Geo<B>::P * ((lj + 1) + Geo<B>::P * (lk + 1))] = (hh * hh) / (f * f);
            fsum += (float)f;
        }
        if (bad) raise_error(kp.ctl, kErrBadSpeed);
        s_sum[tid] = fsum;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) s_sum[tid] += s_sum[tid + s];
            __syncthreads();
        }
        if (tid == 0) {
            kp.fmean[ib] = s_sum[0] / (float)B3;
            kp.band_n[ib] = 0;
            kp.A[ib] = 0;
            kp.Cm[ib] = 0u;
            kp.bmin[ib] = (R)INFINITY;
            kp.lastpops[ib] = 1 << 20;  // no history yet: schedule early
        }
        __syncthreads();
    }
}

// Points of Gamma: psi0, KNOWN_FIX, into the band, activate the block (Alg. 1).
// One entry per (block, tile point), duplicates already merged on the host.
struct SrcEntry {
    int64_t ib;
    int32_t t;
    int32_t pad;
    double v;
};

template <typename R, int B>
__global__ void k_sources(KParams<R> kp, const SrcEntry *e, int32_t n)
{
    constexpr int T = Geo<B>::T, BAND = Geo<B>::BAND, TAGB = Geo<B>::TAGB;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t ib = e[k].ib;
    const int t = e[k].t;
    const R v = (R)e[k].v;
    kp.psi_t[ib * (int64_t)T + t] = v;
    kp.tag_t[ib * (int64_t)TAGB + t] = kKnownFix | kInBand;
    const int pos = atomicAdd(&kp.band_n[ib], 1);
    kp.band_t[ib * (int64_t)BAND + pos] = (uint16_t)t;
    kp.A[ib] = 1;
    using U = typename std::conditional<sizeof(R) == 4, unsigned int, unsigned long long>::type;
    U vb;
    __builtin_memcpy(&vb, &v, sizeof(R));
    atomicMin(reinterpret_cast<U *>(&kp.bmin[ib]), vb);
}

// Interior of every block -> caller's linear psi.
template <typename R, int B>
__global__ void __launch_bounds__(256) k_unlayout(KParams<R> kp)
{
    constexpr int P = Geo<B>::P, T = Geo<B>::T, B3 = Geo<B>::B3;
    const int tid = threadIdx.x;
    for (int64_t ib = blockIdx.x; ib < kp.nblk; ib += gridDim.x) {
        const ProbDesc &pd = kp.prob[kp.blk_prob[ib]];
        const int64_t loc = ib - pd.blk0;
        const int64_t bx = loc % pd.mx, by = (loc / pd.mx) % pd.my, bz = loc / ((int64_t)pd.mx * pd.my);
        const R *gp = kp.psi_t + ib * (int64_t)T;
        R *out = reinterpret_cast<R *>(pd.psi);
        for (int e = tid; e < B3; e += 256) {
            const int li = e % B, lj = (e / B) % B, lk = e / (B * B);
            const int64_t g = (bx * B + li) + (int64_t)pd.nx * ((by * B + lj) + (int64_t)pd.ny * (bz * B + lk));
            out[g] = gp[(li + 1) + P * ((lj + 1) + P * (lk + 1))];
        }
    }
}

// Diagnostic: per-wave minimum through the same reduction as Locate_Min.
__global__ void k_wave_min(const uint32_t *in, uint32_t *out, int nwaves)
{
    const int wv = blockIdx.x;
    if (wv >= nwaves) return;
    const uint32_t m = wave_min_u32(in[(int64_t)wv * 64 + threadIdx.x]);
    if (threadIdx.x == 0) out[wv] = m;
}

// Locate_Min of a march by one wave on a given band (a test probe): the tile values and
// the band are staged as march_block stages them -- the first cap slots in LDS, the rest
// read from the padded band array in memory -- and the pick is written out.  The tile's
// corner 0 is never a band point and reads as +inf, as in every tile.
template <typename R, int B>
__global__ void __launch_bounds__(64) k_argmin_probe(const R *psi, const uint16_t *band, int n,
                                                     int cap, R *vout, int32_t *iout)
{
    using L = Lds<R, B, 1>;
    using Gm = Geo<B>;
    extern __shared__ __align__(16) char smem[];
    FMM_LDS char *lds = (FMM_LDS char *)smem;
    FMM_LDS R *s_psi = reinterpret_cast<FMM_LDS R *>(lds + L::psi_off);
    FMM_LDS uint16_t *s_band = reinterpret_cast<FMM_LDS uint16_t *>(lds + L::band_off);
    for (int t = threadIdx.x; t < Gm::T; t += 64) s_psi[t] = t == 0 ? (R)INFINITY : psi[t];
    for (int k = threadIdx.x; k < Gm::BANDC; k += 64) s_band[k] = k < n ? band[k] : (uint16_t)0;
    __syncthreads();
    FMM_CYC_DECL;
    const MinPick<R> mp = band_argmin<R, 1>(s_band, band, cap, s_psi, n FMM_CYC_ARG);
    if (threadIdx.x == 0) {
        vout[0] = mp.v;
        iout[0] = mp.idx;
        iout[1] = mp.slot;
    }
}

} // namespace fmmdev
