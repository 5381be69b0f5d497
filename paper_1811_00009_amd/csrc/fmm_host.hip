// fmm_host.hip -- host side of the C ABI declared in include/fmm.h: argument
// validation, the per-device workspace cache, source set-up (Alg. 1), kernel
// dispatch over (precision, block edge, waves per block), the persistent and
// host-driven restart loops (Alg. 6), statistics, the autotuner and the
// diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "fmm.h"
#include "fmm_kernels.hpp"

using namespace fmmdev;

static_assert(sizeof(TraceRow) == sizeof(fmm_trace_row), "trace row layout");

namespace {

thread_local std::string g_detail;

int fail(int code, const std::string &msg)
{
    g_detail = msg;
    return code;
}

} // namespace

// Used by the stride-network kernels to report through fmm_last_error_detail().
void fmm_internal_set_detail(const std::string &msg) { g_detail = msg; }
void fmm_internal_mlp_release();  // fmm_mlp.hip

namespace {

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            return fail(e_ == hipErrorOutOfMemory ? FMM_ENOMEM : FMM_EHIP,                     \
                        std::string(#x) + ": " + hipGetErrorString(e_));                      \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

int ensure(DevBuf &b, size_t bytes, const char *what)
{
    if (bytes == 0) bytes = 16;
    if (b.p && b.cap >= bytes) return 0;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(FMM_ENOMEM, std::string("allocating ") + what + " (" +
                                    std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    }
    b.cap = bytes;
    return 0;
}

// Library-owned device memory of one GPU: one arena, grown on demand and kept for
// reuse, that every launch carves its buffers from (ws_layout).
struct Workspace {
    DevBuf arena;
    hipEvent_t e0 = nullptr, e1 = nullptr, l0 = nullptr, l1 = nullptr;
    // the last launch on this arena: its problem (grid, block, waves, dtype, sources) and
    // the bytes of the arena it used, which fmm_solve_resume and the workspace copies check
    std::string last_sig;
    size_t last_total = 0;
};

// Buffers of one launch, each at a 256-byte aligned offset from one base address.
enum WsBuf {
    kWsPsi, kWsTag, kWsBand, kWsBandN, kWsRhs, kWsBmin, kWsA, kWsCm, kWsBprob, kWsFmean,
    kWsLastpops, kWsList0, kWsList1, kWsXlist, kWsCtl, kWsProb, kWsSrc, kWsPlastr, kWsPpops,
    kWsSched, kWsSolves, kWsRing, kWsCount
};

struct WsLayout {
    size_t off[kWsCount];
    size_t total;
};

template <typename R, int B>
WsLayout ws_layout(int64_t nblk, int32_t nprob, size_t nents, size_t nsched = 0, size_t nring = 0)
{
    constexpr size_t T = Geo<B>::T, BAND = Geo<B>::BAND, TAGB = Geo<B>::TAGB;
    const size_t nb = (size_t)nblk, np = (size_t)nprob;
    size_t bytes[kWsCount];
    bytes[kWsPsi] = nb * T * sizeof(R);
    bytes[kWsTag] = nb * TAGB;
    bytes[kWsBand] = nb * BAND * 2;
    bytes[kWsBandN] = nb * 4;
    bytes[kWsRhs] = nb * T * sizeof(R);
    bytes[kWsBmin] = nb * sizeof(R);
    bytes[kWsA] = nb;
    bytes[kWsCm] = nb * 4;
    bytes[kWsBprob] = nb * 4;
    bytes[kWsFmean] = nb * 4;
    bytes[kWsLastpops] = nb * 4;
    bytes[kWsList0] = nb * 4 * 4;  // 4 work bins
    bytes[kWsList1] = nb * 4 * 4;
    bytes[kWsXlist] = nb * 4;
    bytes[kWsCtl] = sizeof(Ctl);
    bytes[kWsProb] = sizeof(ProbDesc) * np;
    bytes[kWsSrc] = sizeof(SrcEntry) * std::max<size_t>(1, nents);
    bytes[kWsPlastr] = sizeof(int32_t) * np;
    bytes[kWsPpops] = sizeof(unsigned long long) * np;
    bytes[kWsSched] = sizeof(double) * nsched;
    bytes[kWsSolves] = nring ? sizeof(SolveState) * np : 0;  // per-problem restarts only
    bytes[kWsRing] = sizeof(unsigned long long) * nring;
    WsLayout L;
    size_t at = 0;
    for (int k = 0; k < kWsCount; ++k) {
        L.off[k] = at;
        at += (bytes[k] + 255) / 256 * 256;
    }
    L.total = at;
    return L;
}

template <typename R>
void ws_bind(KParams<R> &kp, char *base, const WsLayout &L)
{
    kp.psi_t = (R *)(base + L.off[kWsPsi]);
    kp.tag_t = (uint8_t *)(base + L.off[kWsTag]);
    kp.band_t = (uint16_t *)(base + L.off[kWsBand]);
    kp.band_n = (int32_t *)(base + L.off[kWsBandN]);
    kp.rhs_t = (R *)(base + L.off[kWsRhs]);
    kp.bmin = (R *)(base + L.off[kWsBmin]);
    kp.A = (uint8_t *)(base + L.off[kWsA]);
    kp.Cm = (uint32_t *)(base + L.off[kWsCm]);
    kp.blk_prob = (int32_t *)(base + L.off[kWsBprob]);
    kp.fmean = (float *)(base + L.off[kWsFmean]);
    kp.lastpops = (int32_t *)(base + L.off[kWsLastpops]);
    kp.list0 = (int32_t *)(base + L.off[kWsList0]);
    kp.list1 = (int32_t *)(base + L.off[kWsList1]);
    kp.xlist = (int32_t *)(base + L.off[kWsXlist]);
    kp.ctl = (Ctl *)(base + L.off[kWsCtl]);
    kp.prob = (const ProbDesc *)(base + L.off[kWsProb]);
    kp.prob_lastr = (int32_t *)(base + L.off[kWsPlastr]);
    kp.prob_pops = (unsigned long long *)(base + L.off[kWsPpops]);
    kp.sched = (const double *)(base + L.off[kWsSched]);
    kp.solves = (SolveState *)(base + L.off[kWsSolves]);
    kp.ring = (unsigned long long *)(base + L.off[kWsRing]);
}

std::mutex g_mu;
std::map<int, Workspace> g_ws;

struct Device {
    int id = 0;
    int cus = 0;
    int64_t ticks_per_s = 100000000;
    int coop = 0;
    std::string name;
};

int device_info(Device &d)
{
    HIPCHK(hipGetDevice(&d.id));
    HIPCHK(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, d.id));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d.id) == hipSuccess && khz > 0)
        d.ticks_per_s = (int64_t)khz * 1000;
    HIPCHK(hipDeviceGetAttribute(&d.coop, hipDeviceAttributeCooperativeLaunch, d.id));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, d.id));
    d.name = prop.gcnArchName;
    return 0;
}

// A problem after validation, with its sources in library form.
struct Prob {
    ProbDesc d;
    std::vector<fmm_source> src;
};

int validate_problem(int64_t nx, int64_t ny, int64_t nz, double h, const void *F, void *psi,
                     const fmm_source *src, int32_t nsrc, int32_t block, double stride,
                     const std::string &who)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(FMM_EINVAL, who + ": grid dimensions must be > 0");
    if (!(h > 0) || !std::isfinite(h)) return fail(FMM_EINVAL, who + ": h must be finite and > 0");
    if (!(stride > 0)) return fail(FMM_EINVAL, who + ": stride must be > 0 (inf allowed)");
    if (block != 4 && block != 8 && block != 16 && block != 32)
        return fail(FMM_ENOTSUP, who + ": block must be 4, 8, 16 or 32");
    if (nx % block || ny % block || nz % block)
        return fail(FMM_EINVAL, who + ": every grid dimension must be divisible by block");
    if (nx * ny * nz > ((int64_t)1 << 34)) return fail(FMM_EINVAL, who + ": grid too large");
    if (!F || !psi) return fail(FMM_EINVAL, who + ": NULL F or psi buffer");
    if (!src || nsrc <= 0) return fail(FMM_EINVAL, who + ": at least one source is required");
    for (int32_t s = 0; s < nsrc; ++s) {
        const fmm_source &p = src[s];
        if (p.i < 0 || p.j < 0 || p.k < 0 || p.i >= nx || p.j >= ny || p.k >= nz)
            return fail(FMM_EINVAL, who + ": source " + std::to_string(s) + " outside the grid");
        if (!(p.psi0 >= 0) || !std::isfinite(p.psi0))
            return fail(FMM_EINVAL, who + ": source value must be finite and >= 0");
    }
    return 0;
}

// Alg. 1, points of Gamma: every padded block (interior or ghost face, not
// ghost edges/corners) holding a source point gets an entry; repeated points
// keep the smallest value.
void build_sources(const std::vector<Prob> &probs, int B, std::vector<SrcEntry> &out,
                   std::vector<int32_t> &first_list)
{
    std::map<std::pair<int64_t, int32_t>, double> ent;
    const int P = B + 2;
    for (const Prob &pb : probs) {
        const ProbDesc &d = pb.d;
        for (const fmm_source &s : pb.src) {
            for (int64_t bz = s.k / B - 1; bz <= s.k / B + 1; ++bz)
                for (int64_t by = s.j / B - 1; by <= s.j / B + 1; ++by)
                    for (int64_t bx = s.i / B - 1; bx <= s.i / B + 1; ++bx) {
                        if (bx < 0 || by < 0 || bz < 0 || bx >= d.mx || by >= d.my || bz >= d.mz)
                            continue;
                        const int64_t li = s.i - bx * B + 1, lj = s.j - by * B + 1,
                                      lk = s.k - bz * B + 1;
                        if (li < 0 || lj < 0 || lk < 0 || li > B + 1 || lj > B + 1 || lk > B + 1)
                            continue;
                        const int ng = (li == 0 || li == B + 1) + (lj == 0 || lj == B + 1) +
                                       (lk == 0 || lk == B + 1);
                        if (ng > 1) continue;
                        const int64_t ib = d.blk0 + bx + (int64_t)d.mx * (by + (int64_t)d.my * bz);
                        const int32_t t = (int32_t)(li + P * (lj + P * lk));
                        const double v = s.psi0 + 0.0;  // -0 -> +0
                        auto key = std::make_pair(ib, t);
                        auto it = ent.find(key);
                        if (it == ent.end() || v < it->second) ent[key] = v;
                    }
        }
    }
    out.clear();
    first_list.clear();
    for (auto &kv : ent) {
        SrcEntry e{};
        e.ib = kv.first.first;
        e.t = kv.first.second;
        e.v = kv.second;
        out.push_back(e);
        if (first_list.empty() || first_list.back() != (int32_t)e.ib) first_list.push_back((int32_t)e.ib);
    }
}

template <typename R>
__global__ void k_fill_blkprob(int32_t *bp, const ProbDesc *prob, int32_t nprob, int64_t nblk)
{
    for (int64_t ib = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ib < nblk;
         ib += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {  // last problem with blk0 <= ib
            int mid = (lo + hi + 1) / 2;
            if (prob[mid].blk0 <= ib) lo = mid;
            else hi = mid - 1;
        }
        bp[ib] = lo;
    }
}

int map_device_error(int code)
{
    switch (code) {
    case 0: return 0;
    case kErrBadSpeed: return fail(FMM_EINVAL, "speed F has a negative, NaN or infinite value");
    case kErrPopCap: return fail(FMM_ENOCONV, "device watchdog: a march call exceeded the pop cap");
    case kErrTimeout: return fail(FMM_ENOCONV, "device watchdog: a wait timed out (grid barrier or ready queue)");
    case kErrRestarts: return fail(FMM_ENOCONV, "restart cap reached");
    case kErrList: return fail(FMM_EHIP, "internal error: a work list overflowed or held a bad block index");
    default: return fail(FMM_EHIP, "unknown device error " + std::to_string(code));
    }
}

struct RunOut {
    Ctl ctl;
    float ms;
    float loop_ms;
    int grid;
    std::vector<int32_t> lastr;
    std::vector<unsigned long long> ppops;
};

// Block ranges of the problems in the pooled arrays; returns the block count.
int64_t assign_blocks(ProbDesc *d, int32_t nprob, int B)
{
    int64_t nblk = 0;
    for (int32_t q = 0; q < nprob; ++q) {
        d[q].mx = d[q].nx / B;
        d[q].my = d[q].ny / B;
        d[q].mz = d[q].nz / B;
        d[q].blk0 = nblk;
        d[q].nblk = (int64_t)d[q].mx * d[q].my * d[q].mz;
        d[q].nmax = std::max(d[q].nx, std::max(d[q].ny, d[q].nz));
        nblk += d[q].nblk;
    }
    return nblk;
}

// Fills n 32-bit words with zero (used instead of a memset node, which callers that
// capture the stream into a graph cannot rely on).
__global__ void k_clear_words(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Host data of one launch.
struct LaunchIn {
    const ProbDesc *descs;
    int32_t nprob;
    int64_t nblk;
    const SrcEntry *ents;
    int32_t nents;
    SrcEntry *ents_dev;    // device copy of ents (a carved buffer)
    const int32_t *first;  // blocks of the first march list
    int32_t nfirst;
    const fmm_options *o;
    int64_t resume_from = 0;  // > 0: the workspace holds the state after this restart
    uint32_t nring = 0;       // > 0: a batch whose problems restart on their own (ring size)
};

// Tokens per phase of a problem with restarts of its own: enough for every work-group of
// the launch to find work when few problems run, few enough to spread them over many.
int batch_tokens(int64_t grid, int32_t nprob)
{
    const int64_t t = (2 * grid + nprob - 1) / nprob;
    return (int)std::max<int64_t>(8, std::min<int64_t>(1024, t));
}

// Events around the launch (all null: no timing).
struct LaunchEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr, l0 = nullptr, l1 = nullptr;
};

// The launch itself, on buffers already carved (kp bound by ws_bind): copy the problem
// table, the source entries, the first march list and the control block to the device,
// set up every block (Alg. 1), run the restart loop (Alg. 6) and copy psi back to the
// callers' linear layout.  Allocates no device memory.  Returns with the stream drained
// and ctl_out filled; the device error code, if any, is in ctl_out.abort.
template <typename R, int B, int W>
int launch_solve(KParams<R> &kp, const LaunchIn &in, const Device &dev, hipStream_t st,
                 const LaunchEvents &ev, Ctl &ctl_out, int &grid_out)
{
    using L = Lds<R, B, W>;
    const fmm_options &o = *in.o;
    const int64_t nblk = in.nblk;
    Ctl hc;
    std::memset(&hc, 0, sizeof(hc));
    hc.n_list[1] = in.nfirst;  // restart 1 marches list[1] (all in bin 0)
    hc.bin_n[1][0] = in.nfirst;
    hc.rmin[0] = hc.rmin[1] = ~0ull;

    const bool resume = in.resume_from > 0;
    HIPCHK(hipMemcpyAsync((void *)kp.prob, in.descs, sizeof(ProbDesc) * in.nprob, hipMemcpyHostToDevice, st));
    if (!resume) {
        if (in.nents > 0)
            HIPCHK(hipMemcpyAsync(in.ents_dev, in.ents, sizeof(SrcEntry) * in.nents, hipMemcpyHostToDevice, st));
        if (in.nfirst > 0 && in.nring == 0)  // (per-problem restarts: segments, below)
            HIPCHK(hipMemcpyAsync(kp.list1, in.first, sizeof(int32_t) * in.nfirst, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(kp.ctl, &hc, sizeof(Ctl), hipMemcpyHostToDevice, st));
    } else {
        // the control block, lists and tiles are those the stopped solve left; its stop
        // (the restart cap) and its pop and call counts are cleared
        k_clear_words<<<1, 64, 0, st>>>((uint32_t *)&kp.ctl->abort, 1);
        k_clear_words<<<1, 64, 0, st>>>((uint32_t *)&kp.ctl->pops, 8);
    }
    if (o.stride_mode == FMM_STRIDE_SCHEDULE)
        HIPCHK(hipMemcpyAsync((void *)kp.sched, o.bounds, sizeof(double) * o.nbounds, hipMemcpyHostToDevice, st));
    k_clear_words<<<1, 256, 0, st>>>((uint32_t *)kp.prob_lastr, in.nprob);
    k_clear_words<<<1, 256, 0, st>>>((uint32_t *)kp.prob_pops, 2 * (int64_t)in.nprob);

    kp.nprob = in.nprob;
    kp.stride_mode = o.stride_mode == FMM_STRIDE_LEARNED ? 1 : (o.stride_mode == FMM_STRIDE_SCHEDULE ? 2 : 0);
    kp.nsched = kp.stride_mode == 2 ? o.nbounds : 0;
    kp.nblk = nblk;
    kp.max_restarts = o.max_restarts > 0 ? o.max_restarts : 10000000;
    kp.pop_cap = (int64_t)64 * Geo<B>::T;
    kp.timeout_ticks = dev.ticks_per_s * 10;
    kp.mlp = (const float *)o.mlp_weights;
    kp.trace = o.trace_dev;
    kp.trace_cap = o.trace_dev ? o.trace_cap : 0;
    kp.want_features = (kp.trace_cap > 0 || kp.stride_mode == 1) ? 1 : 0;
    kp.band_cap = o.band_lds_cap;
    kp.r0 = in.resume_from;

    const size_t lds = L::bytes;
    if (ev.e0) HIPCHK(hipEventRecord(ev.e0, st));
    if (!resume) {
        k_fill_blkprob<R><<<(unsigned)std::min<int64_t>((nblk + 255) / 256, 4096), 256, 0, st>>>(
            kp.blk_prob, kp.prob, in.nprob, nblk);
        k_init<R, B><<<(unsigned)std::min<int64_t>(nblk, 65536), 256, 0, st>>>(kp);
        if (in.nents > 0)
            k_sources<R, B><<<(unsigned)((in.nents + 127) / 128), 128, 0, st>>>(kp, in.ents_dev, in.nents);
    }
    HIPCHK(hipGetLastError());

    int per_cu = 0;
    int grid = 0;
    if (ev.l0 && in.nring == 0) HIPCHK(hipEventRecord(ev.l0, st));
    if (in.nring > 0) {
        // a batch whose problems restart on their own: states, first lists and tokens
        auto kern = k_batched<R, B, W>;
        HIPCHK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * W, lds));
        if (per_cu <= 0) return fail(FMM_ENOTSUP, "batch kernel does not fit on a compute unit");
        int64_t g = (int64_t)per_cu * dev.cus;
        g = std::min<int64_t>(g, nblk);
        if (o.grid_limit > 0) g = std::min<int64_t>(g, o.grid_limit);
        grid = (int)std::max<int64_t>(g, 1);
        kp.tokens = batch_tokens(grid, in.nprob);
        kp.ring_mask = in.nring - 1;
        if ((uint64_t)in.nprob * (uint64_t)kp.tokens > in.nring)
            return fail(FMM_EHIP, "internal error: token ring too small");
        std::vector<SolveState> sst(in.nprob);
        std::vector<unsigned long long> ring(in.nring);
        for (uint32_t k = 0; k < in.nring; ++k) ring[k] = (unsigned long long)k << 32;  // empty slots
        uint32_t ntok = 0;
        int32_t f = 0;
        for (int32_t q = 0; q < in.nprob; ++q) {
            SolveState &ss = sst[q];
            std::memset(&ss, 0, sizeof(ss));
            const int64_t b0 = in.descs[q].blk0, b1 = b0 + in.descs[q].nblk;
            const int32_t f0 = f;
            while (f < in.nfirst && in.first[f] < b1) ++f;
            const int32_t cnt = f - f0;
            if (cnt <= 0 || in.first[f0] < b0)
                return fail(FMM_EHIP, "internal error: a batch problem without source blocks");
            ss.word = (unsigned long long)cnt << 20;  // phase 0: restart 1's marching step
            ss.r = 1;
            ss.n_list[1] = cnt;
            ss.bin_n[1][0] = cnt;
            HIPCHK(hipMemcpyAsync(kp.list1 + b0, in.first + f0, sizeof(int32_t) * cnt,
                                  hipMemcpyHostToDevice, st));
            const int t = std::min<int32_t>(cnt, kp.tokens);
            ss.queued = t;
            for (int k = 0; k < t; ++k, ++ntok)
                ring[ntok] = ((unsigned long long)(ntok + 1) << 32) | (uint32_t)q;
        }
        const unsigned long long head = 0, tail = ntok;
        const int remaining = in.nprob;
        HIPCHK(hipMemcpyAsync(&kp.ctl->rq_head, &head, sizeof(head), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(&kp.ctl->rq_tail, &tail, sizeof(tail), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(&kp.ctl->remaining, &remaining, sizeof(remaining), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(kp.solves, sst.data(), sizeof(SolveState) * in.nprob, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(kp.ring, ring.data(), sizeof(unsigned long long) * in.nring, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // the host arrays above are read before they go
        if (ev.l0) HIPCHK(hipEventRecord(ev.l0, st));
        kern<<<grid, 64 * W, lds, st>>>(kp);
        HIPCHK(hipGetLastError());
    } else if (o.launch_mode == FMM_LAUNCH_PERSISTENT) {
        auto kern = k_persistent<R, B, W>;
        HIPCHK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * W, lds));
        if (per_cu <= 0) return fail(FMM_ENOTSUP, "persistent kernel does not fit on a compute unit");
        if (!dev.coop) return fail(FMM_ENOTSUP, "device lacks cooperative launch");
        int64_t g = (int64_t)per_cu * dev.cus;
        g = std::min<int64_t>(g, nblk);
        if (o.grid_limit > 0) g = std::min<int64_t>(g, o.grid_limit);
        grid = (int)std::max<int64_t>(g, 1);
        void *args[] = {&kp};
        HIPCHK(hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(64 * W), args, lds, st));
    } else {
        if (kp.stride_mode) return fail(FMM_ENOTSUP, "learned or scheduled strides need the persistent launch");
        if (resume) return fail(FMM_ENOTSUP, "a resumed solve needs the persistent launch");
        auto km = k_march<R, B, W>;
        auto kx = k_exchange<R, B, W>;
        HIPCHK(hipFuncSetAttribute((const void *)km, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        HIPCHK(hipFuncSetAttribute((const void *)kx, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, km, 64 * W, lds));
        const int64_t cap = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * dev.cus);
        int ncur = in.nfirst;
        Ctl *dctl = kp.ctl;
        int64_t r = 1;
        for (;; ++r) {
            const int c = (int)(r & 1);
            k_restart_prologue<R><<<1, 1, 0, st>>>(kp, r);
            const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(ncur, cap));
            km<<<gm, 64 * W, lds, st>>>(kp, r);
            const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(nblk, cap));
            kx<<<gx, 64 * W, lds, st>>>(kp, r);
            HIPCHK(hipGetLastError());
            int nn = 0, ab = 0;
            HIPCHK(hipMemcpyAsync(&nn, &dctl->n_list[c ^ 1], sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&ab, &dctl->abort, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (ab) break;
            ncur = nn;
            if (nn == 0) break;
            if (r >= kp.max_restarts) {
                int code = kErrRestarts;
                HIPCHK(hipMemcpyAsync(&dctl->abort, &code, sizeof(int), hipMemcpyHostToDevice, st));
                break;
            }
        }
        const double fb = std::min((double)r * in.descs[0].stride, in.descs[0].width);
        long long rr = r;
        HIPCHK(hipMemcpyAsync(&dctl->restarts, &rr, sizeof(rr), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(&dctl->final_bound, &fb, sizeof(fb), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // rr and fb live on this stack frame
    }
    if (ev.l1) HIPCHK(hipEventRecord(ev.l1, st));
    k_unlayout<R, B><<<(unsigned)std::min<int64_t>(nblk, 65536), 256, 0, st>>>(kp);
    HIPCHK(hipGetLastError());
    if (ev.e1) HIPCHK(hipEventRecord(ev.e1, st));
    HIPCHK(hipMemcpyAsync(&ctl_out, kp.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    grid_out = grid;
    return 0;
}

constexpr int32_t kSchedReserve = 1 << 16;  // bounds a resumed solve may be given

// Identity of a launch's problem: what a resumed solve must share with the stopped one.
std::string launch_signature(const std::vector<Prob> &probs, int B, int W, size_t rsize)
{
    std::string sig = "B" + std::to_string(B) + "W" + std::to_string(W) + "R" + std::to_string(rsize);
    for (const Prob &pb : probs) {
        sig += ":" + std::to_string(pb.d.nx) + "x" + std::to_string(pb.d.ny) + "x" + std::to_string(pb.d.nz);
        for (const fmm_source &q : pb.src) {
            char b[96];
            std::snprintf(b, sizeof(b), "/%lld,%lld,%lld,%.17g", (long long)q.i, (long long)q.j,
                          (long long)q.k, q.psi0);
            sig += b;
        }
    }
    return sig;
}

// A solve on the library's cached arena (allocated and grown on demand); resume_from > 0
// continues the last solve on this device after that restart instead of starting one.
template <typename R, int B, int W>
int run_solve(std::vector<Prob> &probs, const fmm_options &o, hipStream_t st, RunOut &out,
              int64_t resume_from)
{
    Device dev;
    if (int rc = device_info(dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace &ws = g_ws[dev.id];

    const int32_t nprob = (int32_t)probs.size();
    std::vector<ProbDesc> descs(nprob);
    for (int32_t q = 0; q < nprob; ++q) descs[q] = probs[q].d;
    const int64_t nblk = assign_blocks(descs.data(), nprob, B);
    if (nblk >= ((int64_t)1 << 31)) return fail(FMM_EINVAL, "too many blocks");
    for (int32_t q = 0; q < nprob; ++q) probs[q].d = descs[q];

    std::vector<SrcEntry> ents;
    std::vector<int32_t> first;
    build_sources(probs, B, ents, first);
    // per-problem restarts: the token ring holds every token that can be out at once
    uint32_t nring = 0;
    if (o.per_problem_restarts) {
        if (resume_from > 0) return fail(FMM_ENOTSUP, "a batch with per-problem restarts cannot be resumed");
        for (const ProbDesc &d : descs)
            if (d.nblk >= (1 << 20) - (1 << 17))
                return fail(FMM_EINVAL, "per-problem restarts: a problem has too many blocks");
        // at most 32 one-wave work-groups fit on a compute unit, so the grid is below 32 * cus
        const uint64_t need = (uint64_t)nprob * (uint64_t)batch_tokens((int64_t)32 * dev.cus, nprob);
        if (need > (1u << 30)) return fail(FMM_EINVAL, "per-problem restarts: too many problems");
        nring = 1;
        while (nring < need) nring <<= 1;
    }
    // the layout is fixed by the problem; a schedule's bounds take the arena's last buffer
    const WsLayout L0 = ws_layout<R, B>(nblk, nprob, ents.size(), 0);
    const WsLayout Lw = ws_layout<R, B>(nblk, nprob, ents.size(),
                                       o.stride_mode == FMM_STRIDE_SCHEDULE ? (size_t)o.nbounds : 0,
                                       nring);
    const std::string sig = launch_signature(probs, B, W, sizeof(R));
    if (resume_from > 0) {
        if (ws.last_sig != sig || !ws.arena.p)
            return fail(FMM_EINVAL, "fmm_solve_resume: the last solve on this device was a different problem");
        if (Lw.total > ws.arena.cap)
            return fail(FMM_EINVAL, "fmm_solve_resume: the bound schedule does not fit the stopped solve's workspace");
    } else {
        // room for a later resume with a bound schedule of up to kSchedReserve bounds
        if (int rc = ensure(ws.arena, std::max(Lw.total, L0.total + 8 * (size_t)kSchedReserve),
                            "workspace"))
            return rc;
        ws.last_sig = sig;
        ws.last_total = L0.total;
    }
    if (!ws.e0) {
        HIPCHK(hipEventCreate(&ws.e0));
        HIPCHK(hipEventCreate(&ws.e1));
        HIPCHK(hipEventCreate(&ws.l0));
        HIPCHK(hipEventCreate(&ws.l1));
    }
    KParams<R> kp{};
    char *base = (char *)ws.arena.p;
    ws_bind<R>(kp, base, Lw);
    LaunchIn in{descs.data(), nprob, nblk, ents.data(), (int32_t)ents.size(),
                (SrcEntry *)(base + Lw.off[kWsSrc]), first.data(), (int32_t)first.size(), &o,
                resume_from, nring};
    LaunchEvents ev{ws.e0, ws.e1, ws.l0, ws.l1};
    if (int rc = launch_solve<R, B, W>(kp, in, dev, st, ev, out.ctl, out.grid)) return rc;
    out.lastr.resize(nprob);
    out.ppops.resize(nprob);
    HIPCHK(hipMemcpy(out.lastr.data(), kp.prob_lastr, sizeof(int32_t) * nprob, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(out.ppops.data(), kp.prob_pops, sizeof(unsigned long long) * nprob, hipMemcpyDeviceToHost));
    HIPCHK(hipEventElapsedTime(&out.ms, ws.e0, ws.e1));
    HIPCHK(hipEventElapsedTime(&out.loop_ms, ws.l0, ws.l1));
    return map_device_error(out.ctl.abort);
}

// ---------------------------------------------------------------- no-allocation solve
// Device memory of fmm_solve_noalloc: one fixed array per GPU, held from the library's
// first kernel launch on that GPU until the process ends.  Host code never uses the
// name `scratch` as an address (it is a host-side stand-in): the device address comes
// from hipGetSymbolAddress, once per device, and is kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device; under g_mu

// Device address of this device's scratch array (dev is the current device).
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(FMM_ENOTSUP, "fmm_solve_noalloc: device index too large");
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FMM_EHIP, std::string("fmm_solve_noalloc: hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

constexpr int kNoallocMaxSources = 256;
constexpr int kNoallocMaxEntries = 4 * kNoallocMaxSources;  // own block + up to 3 ghost faces

// build_sources for one problem into fixed arrays: the same entries, sorted by
// (block, tile point), repeated points keeping the smallest value.
int build_sources_fixed(const ProbDesc &d, const fmm_source *src, int32_t nsrc, int B,
                        SrcEntry *out, int32_t &nout, int32_t *first, int32_t &nfirst)
{
    const int P = B + 2;
    nout = 0;
    for (int32_t q = 0; q < nsrc; ++q) {
        const fmm_source &s = src[q];
        for (int64_t bz = s.k / B - 1; bz <= s.k / B + 1; ++bz)
            for (int64_t by = s.j / B - 1; by <= s.j / B + 1; ++by)
                for (int64_t bx = s.i / B - 1; bx <= s.i / B + 1; ++bx) {
                    if (bx < 0 || by < 0 || bz < 0 || bx >= d.mx || by >= d.my || bz >= d.mz) continue;
                    const int64_t li = s.i - bx * B + 1, lj = s.j - by * B + 1, lk = s.k - bz * B + 1;
                    if (li < 0 || lj < 0 || lk < 0 || li > B + 1 || lj > B + 1 || lk > B + 1) continue;
                    const int ng = (li == 0 || li == B + 1) + (lj == 0 || lj == B + 1) +
                                   (lk == 0 || lk == B + 1);
                    if (ng > 1) continue;
                    if (nout >= kNoallocMaxEntries)
                        return fail(FMM_EINVAL, "fmm_solve_noalloc: too many source entries");
                    SrcEntry &e = out[nout++];
                    e.ib = d.blk0 + bx + (int64_t)d.mx * (by + (int64_t)d.my * bz);
                    e.t = (int32_t)(li + P * (lj + P * lk));
                    e.pad = 0;
                    e.v = s.psi0 + 0.0;  // -0 -> +0
                }
    }
    std::sort(out, out + nout, [](const SrcEntry &a, const SrcEntry &b) {
        return a.ib != b.ib ? a.ib < b.ib : (a.t != b.t ? a.t < b.t : a.v < b.v);
    });
    int32_t m = 0;
    for (int32_t k = 0; k < nout; ++k)  // the first of equal (block, point) keeps the least value
        if (m == 0 || out[m - 1].ib != out[k].ib || out[m - 1].t != out[k].t) out[m++] = out[k];
    nout = m;
    nfirst = 0;
    for (int32_t k = 0; k < nout; ++k)
        if (nfirst == 0 || first[nfirst - 1] != (int32_t)out[k].ib) first[nfirst++] = (int32_t)out[k].ib;
    return 0;
}

template <typename R, int B, int W>
int run_solve_noalloc(const ProbDesc &d0, const fmm_source *src, int32_t nsrc, const fmm_options &o,
                      hipStream_t st, Ctl &ctl_out, int &grid_out)
{
    ProbDesc d = d0;
    const int64_t nblk = assign_blocks(&d, 1, B);
    SrcEntry ents[kNoallocMaxEntries];
    int32_t first[kNoallocMaxEntries];
    int32_t nents = 0, nfirst = 0;
    if (int rc = build_sources_fixed(d, src, nsrc, B, ents, nents, first, nfirst)) return rc;
    const WsLayout Lw = ws_layout<R, B>(nblk, 1, (size_t)nents,
                                       o.stride_mode == FMM_STRIDE_SCHEDULE ? (size_t)o.nbounds : 0);
    if (Lw.total > FMM_NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        std::snprintf(msg, sizeof(msg),
                      "fmm_solve_noalloc: the grid needs %zu bytes of device workspace, the static "
                      "scratch holds %zu",
                      Lw.total, (size_t)FMM_NOALLOC_SCRATCH_BYTES);
        return fail(FMM_ENOMEM, msg);
    }
    Device dev;
    if (int rc = device_info(dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    void *base = nullptr;
    if (int rc = scratch_address(dev.id, &base)) return rc;
    KParams<R> kp{};
    ws_bind<R>(kp, (char *)base, Lw);
    LaunchIn in{&d, 1, nblk, ents, nents, (SrcEntry *)((char *)base + Lw.off[kWsSrc]), first, nfirst, &o};
    LaunchEvents ev;  // no events: creating them is not part of this path
    if (int rc = launch_solve<R, B, W>(kp, in, dev, st, ev, ctl_out, grid_out)) return rc;
    return map_device_error(ctl_out.abort);
}

using NoallocFn = int (*)(const ProbDesc &, const fmm_source *, int32_t, const fmm_options &,
                          hipStream_t, Ctl &, int &);

template <typename R>
NoallocFn pick_noalloc(int B, int W)
{
#define FMM_CASE(b, w) \
    if (B == b && W == w) return &run_solve_noalloc<R, b, w>;
    FMM_CASE(4, 1)
    FMM_CASE(4, 2)
    FMM_CASE(4, 4)
    FMM_CASE(8, 1)
    FMM_CASE(8, 2)
    FMM_CASE(8, 4)
    FMM_CASE(16, 1)
    FMM_CASE(16, 2)
    FMM_CASE(16, 4)
    FMM_CASE(32, 1)
#undef FMM_CASE
    return nullptr;
}

using RunFn = int (*)(std::vector<Prob> &, const fmm_options &, hipStream_t, RunOut &, int64_t);

template <typename R>
RunFn pick(int B, int W)
{
#define FMM_CASE(b, w) \
    if (B == b && W == w) return &run_solve<R, b, w>;
    FMM_CASE(4, 1)
    FMM_CASE(4, 2)
    FMM_CASE(4, 4)
    FMM_CASE(8, 1)
    FMM_CASE(8, 2)
    FMM_CASE(8, 4)
    FMM_CASE(16, 1)
    FMM_CASE(16, 2)
    FMM_CASE(16, 4)
    FMM_CASE(32, 1)
#undef FMM_CASE
    return nullptr;
}

int dispatch(int dtype, int B, const fmm_options &o, std::vector<Prob> &probs, hipStream_t st, RunOut &out,
             int64_t resume_from = 0)
{
    const int W = o.waves_per_block <= 0 ? 1 : o.waves_per_block;
    if (W != 1 && W != 2 && W != 4) return fail(FMM_EINVAL, "waves_per_block must be 1, 2 or 4");
    RunFn fn = nullptr;
    if (dtype == FMM_F32) fn = pick<float>(B, W);
    else if (dtype == FMM_F64) fn = pick<double>(B, W);
    else return fail(FMM_EINVAL, "dtype must be FMM_F32 or FMM_F64");
    if (!fn)
        return fail(FMM_ENOTSUP, B == 32 ? "32^3 blocks march with one wave per block"
                                         : "unsupported block / waves combination");
    return fn(probs, o, st, out, resume_from);
}

int check_options(const fmm_options &o)
{
    if (!(o.width > 0)) return fail(FMM_EINVAL, "width must be > 0");
    if (o.stride_mode != FMM_STRIDE_FIXED && o.stride_mode != FMM_STRIDE_LEARNED &&
        o.stride_mode != FMM_STRIDE_SCHEDULE)
        return fail(FMM_EINVAL, "unknown stride_mode");
    if (o.stride_mode == FMM_STRIDE_SCHEDULE) {
        if (!o.bounds || o.nbounds < 1 || o.nbounds > (1 << 24))
            return fail(FMM_EINVAL, "a bound schedule needs 1 to 2^24 bounds");
        for (int32_t k = 0; k < o.nbounds; ++k)
            if (!(o.bounds[k] > 0) || !std::isfinite(o.bounds[k]) || (k > 0 && o.bounds[k] < o.bounds[k - 1]))
                return fail(FMM_EINVAL, "bound schedule: values must be finite, > 0 and non-decreasing");
    }
    if (o.launch_mode != FMM_LAUNCH_PERSISTENT && o.launch_mode != FMM_LAUNCH_HOST)
        return fail(FMM_EINVAL, "unknown launch_mode");
    if (o.trace_dev && o.trace_cap < 0) return fail(FMM_EINVAL, "trace_cap must be >= 0");
    if (o.max_restarts < 0) return fail(FMM_EINVAL, "max_restarts must be >= 0");
    if (o.band_lds_cap < 0 || o.band_lds_cap % 512)
        return fail(FMM_EINVAL, "band_lds_cap must be a non-negative multiple of 512");
    if (o.per_problem_restarts != 0 && o.per_problem_restarts != 1)
        return fail(FMM_EINVAL, "per_problem_restarts must be 0 or 1");
    if (o.per_problem_restarts &&
        (o.stride_mode != FMM_STRIDE_FIXED || o.launch_mode != FMM_LAUNCH_PERSISTENT))
        return fail(FMM_ENOTSUP, "per-problem restarts need a fixed stride and the persistent launch");
    return 0;
}

void fill_stats(fmm_stats *s, const RunOut &r, int B, int W, int64_t restarts, int64_t pops)
{
    std::memset(s, 0, sizeof(*s));
    s->restarts = restarts;
    s->pops = pops;
    s->march_calls = (int64_t)r.ctl.march_calls;
    s->exchange_calls = (int64_t)r.ctl.exchange_calls;
    s->tile_loads = (int64_t)r.ctl.tile_loads;
    s->final_bound = r.ctl.final_bound;
    s->elapsed_ms = r.ms;
    s->loop_ms = r.loop_ms;
    s->grid = r.grid;
    s->block = B;
    s->waves_per_block = W;
}

int build_batch(int32_t nsolves, const fmm_problem *problems, int32_t block, double width,
                const char *who, std::vector<Prob> &probs)
{
    probs.assign(nsolves, Prob{});
    for (int32_t q = 0; q < nsolves; ++q) {
        const fmm_problem &p = problems[q];
        if (int rc = validate_problem(p.nx, p.ny, p.nz, p.h, p.F_dev, p.psi_dev, p.src, p.nsrc, block,
                                      p.stride, std::string(who) + "[" + std::to_string(q) + "]"))
            return rc;
        ProbDesc &d = probs[q].d;
        std::memset(&d, 0, sizeof(d));
        d.F = p.F_dev;
        d.psi = p.psi_dev;
        d.nx = (int32_t)p.nx;
        d.ny = (int32_t)p.ny;
        d.nz = (int32_t)p.nz;
        d.h = p.h;
        d.stride = p.stride;
        d.width = width;
        probs[q].src.assign(p.src, p.src + p.nsrc);
    }
    return 0;
}

// Autotuner cache: key -> (block, waves, ms), in memory and optionally in a text file.
std::map<std::string, fmm_tuning> g_tune_cache;

// The key holds the gcd of every side of every sample, so that a cached block size
// divides the sides of any sample set that maps to the same key.
std::string tune_key(const std::string &arch, int32_t dtype, int32_t nsamples, const fmm_problem *s)
{
    double pts = 0;
    int64_t smin = INT64_MAX, smax = 0, g = 0;
    for (int32_t q = 0; q < nsamples; ++q) {
        pts += (double)s[q].nx * s[q].ny * s[q].nz;
        smin = std::min<int64_t>(smin, std::min(s[q].nx, std::min(s[q].ny, s[q].nz)));
        smax = std::max<int64_t>(smax, std::max(s[q].nx, std::max(s[q].ny, s[q].nz)));
        g = std::gcd(g, std::gcd(s[q].nx, std::gcd(s[q].ny, s[q].nz)));
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s:%s:n%d:pts2^%d:side%lld-%lld:gcd%lld", arch.c_str(),
                  dtype == FMM_F32 ? "f32" : "f64", (int)nsamples, (int)std::floor(std::log2(std::max(pts, 1.0))),
                  (long long)smin, (long long)smax, (long long)g);
    return buf;
}

// A cached (block, waves) is used only if the block divides every side of the samples.
bool tuning_fits(const fmm_tuning &t, int32_t nsamples, const fmm_problem *s)
{
    if (t.block <= 0) return false;
    if (t.waves_per_block != 1 && t.waves_per_block != 2 && t.waves_per_block != 4) return false;
    for (int32_t q = 0; q < nsamples; ++q)
        if (s[q].nx % t.block || s[q].ny % t.block || s[q].nz % t.block) return false;
    return true;
}

bool tune_file_lookup(const char *path, const std::string &key, fmm_tuning &t)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char k[256];
    int b, w;
    double ms;
    bool found = false;
    while (std::fscanf(f, "%255s %d %d %lf", k, &b, &w, &ms) == 4) {
        if (key == k) {
            t.block = b;
            t.waves_per_block = w;
            t.ms = ms;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_file_store(const char *path, const std::string &key, const fmm_tuning &t)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), t.block, t.waves_per_block, t.ms);
    std::fclose(f);
}

#ifdef FMM_CYCLES
// s_memtime and the 100 MHz constant clock over the same ~20 ms spin.
__global__ void k_clock_rate(unsigned long long *o)
{
    if (threadIdx.x != 0) return;
    const unsigned long long m0 = __builtin_amdgcn_s_memtime(), w0 = wall_clock64();
    while (wall_clock64() - w0 < 2000000ull) __builtin_amdgcn_s_sleep(10);
    const unsigned long long m1 = __builtin_amdgcn_s_memtime(), w1 = wall_clock64();
    o[0] = m0;
    o[1] = m1;
    o[2] = w0;
    o[3] = w1;
}
#endif

} // namespace

// ============================================================================ C ABI
namespace {
template <typename R, int B>
int argmin_probe(const void *psi_dev, const uint16_t *band_dev, int32_t n, int32_t cap,
                 void *val_out_dev, int32_t *idx_out_dev, hipStream_t st)
{
    using Gm = fmmdev::Geo<B>;
    if (n < 1 || n > Gm::T - 1) return fail(FMM_EINVAL, "fmm_selftest_band_argmin: n out of range");
    const int c = cap > 0 && cap < Gm::BANDC ? cap : Gm::BANDC;
    std::vector<uint16_t> hb((size_t)n);
    HIPCHK(hipMemcpyAsync(hb.data(), band_dev, sizeof(uint16_t) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (uint16_t t : hb)
        if (t < 1 || t >= Gm::T) return fail(FMM_EINVAL, "fmm_selftest_band_argmin: band index out of the tile");
    // the band array padded to whole 512-slot chunks, as in the workspace
    uint16_t *pad = nullptr;
    HIPCHK(hipMalloc(&pad, sizeof(uint16_t) * Gm::BAND));
    hipError_t e = hipMemsetAsync(pad, 0, sizeof(uint16_t) * Gm::BAND, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pad, band_dev, sizeof(uint16_t) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        fmmdev::k_argmin_probe<R, B><<<1, 64, fmmdev::Lds<R, B, 1>::bytes, st>>>(
            (const R *)psi_dev, pad, n, c, (R *)val_out_dev, idx_out_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(pad);
    HIPCHK(e);
    return 0;
}
} // namespace

extern "C" {

void fmm_options_default(fmm_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->width = INFINITY;
    opt->stride_mode = FMM_STRIDE_FIXED;
    opt->waves_per_block = 1;
    opt->launch_mode = FMM_LAUNCH_PERSISTENT;
}

int fmm_solve(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
              const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
              void *hip_stream, const fmm_options *opt, fmm_stats *stats)
{
    try {
        fmm_options o;
        fmm_options_default(&o);
        if (opt) o = *opt;
        if (int rc = check_options(o)) return rc;
        if (int rc = validate_problem(nx, ny, nz, h, F_dev, psi_dev, src, nsrc, block, stride, "fmm_solve"))
            return rc;
        if (o.stride_mode != FMM_STRIDE_FIXED && !std::isfinite(stride))
            return fail(FMM_EINVAL, "learned or scheduled strides need a finite base stride");
        std::vector<Prob> probs(1);
        ProbDesc &d = probs[0].d;
        std::memset(&d, 0, sizeof(d));
        d.F = F_dev;
        d.psi = psi_dev;
        d.nx = (int32_t)nx;
        d.ny = (int32_t)ny;
        d.nz = (int32_t)nz;
        d.h = h;
        d.stride = stride;
        d.width = o.width;
        probs[0].src.assign(src, src + nsrc);
        RunOut out{};
        int rc = dispatch(dtype, block, o, probs, (hipStream_t)hip_stream, out);
        if (stats && (rc == 0 || rc == FMM_ENOCONV))
            fill_stats(stats, out, block, o.waves_per_block <= 0 ? 1 : o.waves_per_block,
                       out.ctl.restarts, (int64_t)out.ctl.pops);
        return rc;
    } catch (const std::exception &e) {
        return fail(FMM_EHIP, std::string("fmm_solve: ") + e.what());
    } catch (...) {
        return fail(FMM_EHIP, "fmm_solve: unknown exception");
    }
}

int fmm_solve_resume(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
                     const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
                     void *hip_stream, const fmm_options *opt, int64_t from_restart, fmm_stats *stats)
{
    try {
        fmm_options o;
        fmm_options_default(&o);
        if (opt) o = *opt;
        if (int rc = check_options(o)) return rc;
        if (int rc = validate_problem(nx, ny, nz, h, F_dev, psi_dev, src, nsrc, block, stride, "resume"))
            return rc;
        if (from_restart < 1) return fail(FMM_EINVAL, "fmm_solve_resume: from_restart must be >= 1");
        if (o.stride_mode == FMM_STRIDE_LEARNED)
            return fail(FMM_ENOTSUP, "fmm_solve_resume: fixed strides and bound schedules only");
        if (o.stride_mode == FMM_STRIDE_SCHEDULE && o.nbounds > kSchedReserve)
            return fail(FMM_EINVAL, "fmm_solve_resume: at most 65536 bounds");
        if (o.launch_mode != FMM_LAUNCH_PERSISTENT)
            return fail(FMM_ENOTSUP, "fmm_solve_resume: persistent launch only");
        if (o.stride_mode == FMM_STRIDE_SCHEDULE && !std::isfinite(stride))
            return fail(FMM_EINVAL, "fmm_solve_resume: a bound schedule needs a finite stride");
        std::vector<Prob> probs(1);
        ProbDesc &d = probs[0].d;
        std::memset(&d, 0, sizeof(d));
        d.F = F_dev;
        d.psi = psi_dev;
        d.nx = (int32_t)nx;
        d.ny = (int32_t)ny;
        d.nz = (int32_t)nz;
        d.h = h;
        d.stride = stride;
        d.width = o.width;
        probs[0].src.assign(src, src + nsrc);
        RunOut out{};
        int rc = dispatch(dtype, block, o, probs, (hipStream_t)hip_stream, out, from_restart);
        if (stats && (rc == 0 || rc == FMM_ENOCONV))
            fill_stats(stats, out, block, o.waves_per_block <= 0 ? 1 : o.waves_per_block,
                       out.ctl.restarts, (int64_t)out.ctl.pops);
        return rc;
    } catch (const std::exception &e) {
        return fail(FMM_EHIP, std::string("fmm_solve_resume: ") + e.what());
    } catch (...) {
        return fail(FMM_EHIP, "fmm_solve_resume: unknown exception");
    }
}

int fmm_workspace_save(void *dst_dev, size_t cap_bytes, size_t *bytes_out, void *hip_stream)
{
    Device dev;
    if (int rc = device_info(dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace &ws = g_ws[dev.id];
    if (bytes_out) *bytes_out = ws.last_total;
    if (!ws.arena.p || ws.last_total == 0) return fail(FMM_EINVAL, "fmm_workspace_save: no solve on this device yet");
    if (!dst_dev) return 0;  // size query
    if (cap_bytes < ws.last_total) return fail(FMM_EINVAL, "fmm_workspace_save: destination too small");
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipMemcpyAsync(dst_dev, ws.arena.p, ws.last_total, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

int fmm_workspace_restore(const void *src_dev, size_t bytes, void *hip_stream)
{
    Device dev;
    if (int rc = device_info(dev)) return rc;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace &ws = g_ws[dev.id];
    if (!src_dev || !ws.arena.p || ws.last_total == 0 || bytes != ws.last_total)
        return fail(FMM_EINVAL, "fmm_workspace_restore: not a saved state of the last solve on this device");
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipMemcpyAsync(ws.arena.p, src_dev, bytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}

int fmm_solve_noalloc(int64_t nx, int64_t ny, int64_t nz, double h, int32_t dtype, const void *F_dev,
                      const fmm_source *src, int32_t nsrc, int32_t block, double stride, void *psi_dev,
                      void *hip_stream, const fmm_options *opt, fmm_stats *stats)
{
    try {
        fmm_options o;
        fmm_options_default(&o);
        if (opt) o = *opt;
        if (int rc = check_options(o)) return rc;
        if (int rc = validate_problem(nx, ny, nz, h, F_dev, psi_dev, src, nsrc, block, stride, "noalloc"))
            return rc;
        if (o.stride_mode != FMM_STRIDE_FIXED && !std::isfinite(stride))
            return fail(FMM_EINVAL, "fmm_solve_noalloc: learned or scheduled strides need a finite base stride");
        if (nsrc > kNoallocMaxSources)
            return fail(FMM_EINVAL, "fmm_solve_noalloc: at most 256 sources");
        const int W = o.waves_per_block <= 0 ? 1 : o.waves_per_block;
        if (W != 1 && W != 2 && W != 4) return fail(FMM_EINVAL, "waves_per_block must be 1, 2 or 4");
        NoallocFn fn = nullptr;
        if (dtype == FMM_F32) fn = pick_noalloc<float>(block, W);
        else if (dtype == FMM_F64) fn = pick_noalloc<double>(block, W);
        else return fail(FMM_EINVAL, "dtype must be FMM_F32 or FMM_F64");
        if (!fn) return fail(FMM_ENOTSUP, "unsupported block / waves combination");
        ProbDesc d;
        std::memset(&d, 0, sizeof(d));
        d.F = F_dev;
        d.psi = psi_dev;
        d.nx = (int32_t)nx;
        d.ny = (int32_t)ny;
        d.nz = (int32_t)nz;
        d.h = h;
        d.stride = stride;
        d.width = o.width;
        Ctl ctl;
        std::memset(&ctl, 0, sizeof(ctl));
        int grid = 0;
        const int rc = fn(d, src, nsrc, o, (hipStream_t)hip_stream, ctl, grid);
        if (stats && (rc == 0 || rc == FMM_ENOCONV)) {
            std::memset(stats, 0, sizeof(*stats));
            stats->restarts = ctl.restarts;
            stats->pops = (int64_t)ctl.pops;
            stats->march_calls = (int64_t)ctl.march_calls;
            stats->exchange_calls = (int64_t)ctl.exchange_calls;
            stats->tile_loads = (int64_t)ctl.tile_loads;
            stats->final_bound = ctl.final_bound;
            stats->grid = grid;
            stats->block = block;
            stats->waves_per_block = W;
        }
        return rc;
    } catch (...) {
        return fail(FMM_EHIP, "fmm_solve_noalloc: unexpected exception");
    }
}

int fmm_solve_batched(int32_t nsolves, const fmm_problem *problems, int32_t dtype, int32_t block,
                      const fmm_options *opt, void *hip_stream, fmm_stats *per_solve_stats)
{
    try {
        if (nsolves <= 0 || !problems) return fail(FMM_EINVAL, "fmm_solve_batched: no problems");
        fmm_options o;
        fmm_options_default(&o);
        if (opt) o = *opt;
        if (int rc = check_options(o)) return rc;
        if (o.stride_mode != FMM_STRIDE_FIXED)
            return fail(FMM_ENOTSUP, "fmm_solve_batched: fixed stride only");
        if (o.launch_mode != FMM_LAUNCH_PERSISTENT)
            return fail(FMM_ENOTSUP, "fmm_solve_batched: persistent launch only");
        std::vector<Prob> probs;
        if (int rc = build_batch(nsolves, problems, block, o.width, "fmm_solve_batched", probs)) return rc;
        RunOut out{};
        int rc = dispatch(dtype, block, o, probs, (hipStream_t)hip_stream, out);
        if (per_solve_stats && (rc == 0 || rc == FMM_ENOCONV)) {
            const int W = o.waves_per_block <= 0 ? 1 : o.waves_per_block;
            for (int32_t q = 0; q < nsolves; ++q) {
                const int64_t rq = nsolves > 1 ? (int64_t)out.lastr[q] + 1 : out.ctl.restarts;
                const int64_t pq = nsolves > 1 ? (int64_t)out.ppops[q] : (int64_t)out.ctl.pops;
                fill_stats(&per_solve_stats[q], out, block, W, rq, pq);
                per_solve_stats[q].final_bound =
                    std::min((double)rq * probs[q].d.stride, probs[q].d.width);
            }
        }
        return rc;
    } catch (const std::exception &e) {
        return fail(FMM_EHIP, std::string("fmm_solve_batched: ") + e.what());
    } catch (...) {
        return fail(FMM_EHIP, "fmm_solve_batched: unknown exception");
    }
}

int fmm_autotune(int32_t nsamples, const fmm_problem *samples, int32_t dtype, const char *cache_path,
                 void *hip_stream, fmm_tuning *out)
{
    try {
        if (nsamples <= 0 || !samples || !out) return fail(FMM_EINVAL, "fmm_autotune: bad arguments");
        if (dtype != FMM_F32 && dtype != FMM_F64) return fail(FMM_EINVAL, "fmm_autotune: bad dtype");
        Device dev;
        if (int rc = device_info(dev)) return rc;
        const std::string key = tune_key(dev.name, dtype, nsamples, samples);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && tuning_fits(it->second, nsamples, samples)) {
            *out = it->second;
            return 0;
        }
        fmm_tuning best{0, 0, INFINITY};
        if (tune_file_lookup(cache_path, key, best) && tuning_fits(best, nsamples, samples)) {
            g_tune_cache[key] = best;
            *out = best;
            return 0;
        }
        best = fmm_tuning{0, 0, INFINITY};
        const int blocks[3] = {8, 16, 32};
        const int waves[3] = {1, 2, 4};
        for (int B : blocks) {
            bool divides = true;
            for (int32_t q = 0; q < nsamples; ++q)
                if (samples[q].nx % B || samples[q].ny % B || samples[q].nz % B) divides = false;
            if (!divides) continue;
            for (int W : waves) {
                if (B == 32 && W != 1) continue;  // 32^3 blocks march with one wave
                fmm_options o;
                fmm_options_default(&o);
                o.waves_per_block = W;
                std::vector<Prob> probs;
                if (int rc = build_batch(nsamples, samples, B, o.width, "fmm_autotune", probs)) return rc;
                RunOut r1{}, r2{};
                if (int rc = dispatch(dtype, B, o, probs, (hipStream_t)hip_stream, r1)) return rc;
                if (int rc = dispatch(dtype, B, o, probs, (hipStream_t)hip_stream, r2)) return rc;
                if (r2.ms < best.ms) best = fmm_tuning{B, W, (double)r2.ms};
            }
        }
        if (best.block == 0) return fail(FMM_ENOTSUP, "fmm_autotune: no block size divides every sample");
        g_tune_cache[key] = best;
        tune_file_store(cache_path, key, best);
        *out = best;
        return 0;
    } catch (const std::exception &e) {
        return fail(FMM_EHIP, std::string("fmm_autotune: ") + e.what());
    }
}

int fmm_selftest_wave_min(const uint32_t *in_dev, uint32_t *out_dev, int32_t nwaves, void *hip_stream)
{
    if (!in_dev || !out_dev || nwaves <= 0) return fail(FMM_EINVAL, "fmm_selftest_wave_min: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    k_wave_min<<<nwaves, 64, 0, st>>>(in_dev, out_dev, nwaves);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return 0;
}


int fmm_selftest_band_argmin(int dtype, int32_t block, const void *psi_dev, const uint16_t *band_dev,
                             int32_t n, int32_t cap, void *val_out_dev, int32_t *idx_out_dev,
                             void *hip_stream)
{
    if (!psi_dev || !band_dev || !val_out_dev || !idx_out_dev)
        return fail(FMM_EINVAL, "fmm_selftest_band_argmin: null pointer");
    if (cap < 0 || cap % 512)
        return fail(FMM_EINVAL, "fmm_selftest_band_argmin: cap must be a non-negative multiple of 512");
    hipStream_t st = (hipStream_t)hip_stream;
    try {
        if (dtype == FMM_F32) {
            if (block == 4) return argmin_probe<float, 4>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
            if (block == 8) return argmin_probe<float, 8>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
            if (block == 16) return argmin_probe<float, 16>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
        } else if (dtype == FMM_F64) {
            if (block == 4) return argmin_probe<double, 4>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
            if (block == 8) return argmin_probe<double, 8>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
            if (block == 16) return argmin_probe<double, 16>(psi_dev, band_dev, n, cap, val_out_dev, idx_out_dev, st);
        }
        return fail(FMM_EINVAL, "fmm_selftest_band_argmin: dtype or block size not supported");
    } catch (const std::exception &ex) {
        return fail(FMM_EHIP, std::string("fmm_selftest_band_argmin: ") + ex.what());
    }
}

int fmm_release(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    // no device call at all when no solve ever ran (nothing to free on any device)
    const bool have_cur = !g_ws.empty() && hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : g_ws) {
        if (hipSetDevice(kv.first) != hipSuccess) continue;
        Workspace &ws = kv.second;
        if (ws.arena.p) (void)hipFree(ws.arena.p);
        hipEvent_t *evs[4] = {&ws.e0, &ws.e1, &ws.l0, &ws.l1};
        for (hipEvent_t *e : evs) {
            if (*e) (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    }
    g_ws.clear();
    if (have_cur) (void)hipSetDevice(cur);
    fmm_internal_mlp_release();
    g_tune_cache.clear();
    for (int d = 0; d < kMaxDevices; ++d) g_scratch_ptr[d] = nullptr;
    return 0;
}

const char *fmm_strerror(int code)
{
    switch (code) {
    case FMM_OK: return "ok";
    case FMM_EINVAL: return "invalid argument";
    case FMM_ENOMEM: return "out of memory";
    case FMM_EHIP: return "HIP runtime error";
    case FMM_ENOCONV: return "no convergence (restart cap or device watchdog)";
    case FMM_ENOTSUP: return "not supported";
    default: return "unknown error code";
    }
}

const char *fmm_last_error_detail(void) { return g_detail.c_str(); }

const char *fmm_version(void) { return "fmm-mi355x 0.1 (gfx950)"; }

#ifdef FMM_CYCLES
// Profiling build only.  out[k] = segment k summed over every work-group since the last
// reset (see the account's segments in fmm_device.hpp); out[16] = shader-clock ticks
// per second of s_memtime, measured against the 100 MHz constant clock.
int fmm_cycle_account(unsigned long long *out, int reset)
{
    static unsigned long long rows[kCycRows][kCycSegs];
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpyFromSymbol(rows, HIP_SYMBOL(fmm_cyc_rows), sizeof(rows)));
    for (int k = 0; k < kCycSegs; ++k) {
        unsigned long long acc = 0;
        for (int w = 0; w < kCycRows; ++w) acc += rows[w][k];
        out[k] = acc;
    }
    unsigned long long *clk = nullptr;
    HIPCHK(hipMalloc(&clk, 4 * sizeof(unsigned long long)));
    k_clock_rate<<<1, 64>>>(clk);
    HIPCHK(hipGetLastError());
    unsigned long long h[4];
    HIPCHK(hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost));
    (void)hipFree(clk);
    out[kCycSegs] = (unsigned long long)((double)(h[1] - h[0]) / (double)(h[3] - h[2]) * 1e8);
    if (reset) {
        std::memset(rows, 0, sizeof(rows));
        HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(fmm_cyc_rows), rows, sizeof(rows)));
    }
    return 0;
}
#endif

} // extern "C"
