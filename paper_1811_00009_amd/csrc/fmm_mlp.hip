// fmm_mlp.hip -- forward, backward and Adam kernels of the stride network
// (12-32-32-1 perceptron, ReLU hidden layers, output log m = ln(1/4) +
// sigmoid(z) ln 32).  FP32.  The paper leaves the restart stride a free
// parameter (Sec. 2.4, Sec. 3.5-3.6); the network that picks it per restart is
// this library's addition.
//
// Gradients are reduced deterministically: every work-group writes the partial
// gradient of its contiguous chunk of samples, and a second kernel sums the
// partials in work-group order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fmm.h"

void fmm_internal_set_detail(const std::string &msg);

namespace {

constexpr int NI = 12, NH = 32, NP = NH * NI + NH + NH * NH + NH + NH + 1;
static_assert(NP == FMM_MLP_NPARAMS, "parameter count");
constexpr float kLogMin = -1.3862943611198906f;
constexpr float kLogSpan = 3.4657359027997265f;
constexpr int kTile = 64;        // samples per LDS tile
constexpr int kThreads = 256;    // threads per work-group
constexpr int kGradGroups = 240; // work-groups of the gradient pass


// offsets into the parameter vector
constexpr int oW1 = 0, ob1 = oW1 + NH * NI, oW2 = ob1 + NH, ob2 = oW2 + NH * NH, oW3 = ob2 + NH,
              ob3 = oW3 + NH;

__device__ float forward_one(const float *P, const float *x, float *h1, float *h2, float *zout)
{
    for (int o = 0; o < NH; ++o) {
        float s = P[ob1 + o];
        for (int i = 0; i < NI; ++i) s += P[oW1 + o * NI + i] * x[i];
        h1[o] = s > 0.f ? s : 0.f;
    }
    for (int o = 0; o < NH; ++o) {
        float s = P[ob2 + o];
        for (int i = 0; i < NH; ++i) s += P[oW2 + o * NH + i] * h1[i];
        h2[o] = s > 0.f ? s : 0.f;
    }
    float z = P[ob3];
    for (int i = 0; i < NH; ++i) z += P[oW3 + i] * h2[i];
    *zout = z;
    const float sig = 1.0f / (1.0f + expf(-z));
    return kLogMin + kLogSpan * sig;
}

__global__ void k_forward(const float *P, const float *X, int64_t n, float *Y)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[NI], h1[NH], h2[NH], z;
    for (int i = 0; i < NI; ++i) x[i] = X[s * NI + i];
    Y[s] = forward_one(P, x, h1, h2, &z);
}

// Partial loss and gradient of the chunk of samples owned by this work-group.
__global__ void __launch_bounds__(kThreads) k_grad_partial(const float *P, const float *X, const float *Tg,
                                                     int64_t n, float *partial)
{
    __shared__ float sx[kTile][NI];
    __shared__ float sh1[kTile][NH];
    __shared__ float sh2[kTile][NH];
    __shared__ float sd1[kTile][NH];
    __shared__ float sd2[kTile][NH];
    __shared__ float sdz[kTile];
    __shared__ float sloss[kTile];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = blockIdx.x * chunk;
    const int64_t s1 = s0 + chunk < n ? s0 + chunk : n;
    constexpr int EPT = (NP + kThreads - 1) / kThreads;  // gradient entries per thread
    float acc[EPT];
    for (int k = 0; k < EPT; ++k) acc[k] = 0.f;
    float lacc = 0.f;
    const float inv_n = 1.0f / (float)n;
    for (int64_t base = s0; base < s1; base += kTile) {
        const int cnt = (int)((s1 - base) < kTile ? (s1 - base) : kTile);
        if (tid < kTile) {
            float x[NI], h1[NH], h2[NH], z;
            if (tid < cnt) {
                for (int i = 0; i < NI; ++i) x[i] = X[(base + tid) * NI + i];
                const float y = forward_one(P, x, h1, h2, &z);
                const float e = y - Tg[base + tid];
                const float sig = 1.0f / (1.0f + expf(-z));
                const float dz = (2.0f * e * inv_n) * kLogSpan * sig * (1.0f - sig);
                float d2[NH], d1[NH];
                for (int i = 0; i < NH; ++i) d2[i] = h2[i] > 0.f ? dz * P[oW3 + i] : 0.f;
                for (int i = 0; i < NH; ++i) {
                    float s = 0.f;
                    for (int o = 0; o < NH; ++o) s += d2[o] * P[oW2 + o * NH + i];
                    d1[i] = h1[i] > 0.f ? s : 0.f;
                }
                for (int i = 0; i < NI; ++i) sx[tid][i] = x[i];
                for (int i = 0; i < NH; ++i) {
                    sh1[tid][i] = h1[i];
                    sh2[tid][i] = h2[i];
                    sd1[tid][i] = d1[i];
                    sd2[tid][i] = d2[i];
                }
                sdz[tid] = dz;
                sloss[tid] = e * e;
            } else {
                for (int i = 0; i < NI; ++i) sx[tid][i] = 0.f;
                for (int i = 0; i < NH; ++i) sh1[tid][i] = sh2[tid][i] = sd1[tid][i] = sd2[tid][i] = 0.f;
                sdz[tid] = 0.f;
                sloss[tid] = 0.f;
            }
        }
        __syncthreads();
        for (int k = 0; k < EPT; ++k) {
            const int e = tid + k * kThreads;
            if (e >= NP) break;
            float s = 0.f;
            if (e < ob1) {
                const int o = e / NI, i = e % NI;
                for (int t = 0; t < kTile; ++t) s += sd1[t][o] * sx[t][i];
            } else if (e < oW2) {
                const int o = e - ob1;
                for (int t = 0; t < kTile; ++t) s += sd1[t][o];
            } else if (e < ob2) {
                const int o = (e - oW2) / NH, i = (e - oW2) % NH;
                for (int t = 0; t < kTile; ++t) s += sd2[t][o] * sh1[t][i];
            } else if (e < oW3) {
                const int o = e - ob2;
                for (int t = 0; t < kTile; ++t) s += sd2[t][o];
            } else if (e < ob3) {
                const int i = e - oW3;
                for (int t = 0; t < kTile; ++t) s += sdz[t] * sh2[t][i];
            } else {
                for (int t = 0; t < kTile; ++t) s += sdz[t];
            }
            acc[k] += s;
        }
        if (tid == 0)
            for (int t = 0; t < kTile; ++t) lacc += sloss[t];
        __syncthreads();
    }
    float *out = partial + (int64_t)blockIdx.x * (NP + 1);
    for (int k = 0; k < EPT; ++k) {
        const int e = tid + k * kThreads;
        if (e < NP) out[e] = acc[k];
    }
    if (tid == 0) out[NP] = lacc;
}

// Sum the partials in work-group order: grad[e] and loss = sum / n.
__global__ void k_grad_reduce(const float *partial, int groups, int64_t n, float *grad, float *loss)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e > NP) return;
    float s = 0.f;
    for (int g = 0; g < groups; ++g) s += partial[(int64_t)g * (NP + 1) + e];
    if (e < NP) grad[e] = s;
    else *loss = s / (float)n;
}

__global__ void k_adam(float *P, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_copy1(const float *src, float *dst) { *dst = *src; }

struct Scratch {
    float *partial = nullptr;
    float *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    bool ok = false;
};
Scratch g_scr;

int mlp_fail(int code, const std::string &msg)
{
    fmm_internal_set_detail(msg);
    return code;
}

#define MLPCHK(x)                                                                               \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return mlp_fail(FMM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

int scratch()
{
    if (g_scr.ok) return 0;
    MLPCHK(hipMalloc(&g_scr.partial, sizeof(float) * (size_t)kGradGroups * (NP + 1)));
    MLPCHK(hipMalloc(&g_scr.grad, sizeof(float) * NP));
    MLPCHK(hipMalloc(&g_scr.m, sizeof(float) * NP));
    MLPCHK(hipMalloc(&g_scr.v, sizeof(float) * NP));
    MLPCHK(hipMalloc(&g_scr.loss, sizeof(float)));
    g_scr.ok = true;
    return 0;
}

int launch_loss_grad(const float *P, const float *X, const float *T, int64_t n, float *loss,
                     float *grad, hipStream_t st)
{
    if (int rc = scratch()) return rc;
    const int groups = (int)std::min<int64_t>(kGradGroups, (n + kTile - 1) / kTile);
    k_grad_partial<<<groups, kThreads, 0, st>>>(P, X, T, n, g_scr.partial);
    k_grad_reduce<<<(NP + 1 + 255) / 256, 256, 0, st>>>(g_scr.partial, groups, n, grad, loss);
    MLPCHK(hipGetLastError());
    return 0;
}

} // namespace

// Frees the scratch (on the device it was allocated on); the next use allocates again.
void fmm_internal_mlp_release()
{
    float **bufs[5] = {&g_scr.partial, &g_scr.grad, &g_scr.m, &g_scr.v, &g_scr.loss};
    for (float **b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    g_scr.ok = false;
}

extern "C" {

int fmm_mlp_forward(const float *params_dev, const float *x_dev, int64_t n, float *y_dev, void *hip_stream)
{
    if (!params_dev || !x_dev || !y_dev || n <= 0) return mlp_fail(FMM_EINVAL, "fmm_mlp_forward: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    k_forward<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(params_dev, x_dev, n, y_dev);
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize(st));
    return 0;
}

int fmm_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n,
                      float *loss_dev, float *grad_dev, void *hip_stream)
{
    if (!params_dev || !x_dev || !t_dev || !loss_dev || !grad_dev || n <= 0)
        return mlp_fail(FMM_EINVAL, "fmm_mlp_loss_grad: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    if (int rc = launch_loss_grad(params_dev, x_dev, t_dev, n, loss_dev, grad_dev, st)) return rc;
    MLPCHK(hipStreamSynchronize(st));
    return 0;
}

int fmm_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, float lr,
                 float beta1, float beta2, float eps, int64_t t, void *hip_stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev || t < 1)
        return mlp_fail(FMM_EINVAL, "fmm_mlp_adam: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    k_adam<<<(NP + 255) / 256, 256, 0, st>>>(params_dev, grad_dev, m_dev, v_dev, lr, beta1, beta2, eps, c1, c2);
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize(st));
    return 0;
}

int fmm_mlp_train(float *params_dev, const float *x_dev, const float *t_dev, int64_t n, int64_t steps,
                  float lr, float *loss_hist_dev, void *hip_stream)
{
    if (!params_dev || !x_dev || !t_dev || n <= 0 || steps <= 0)
        return mlp_fail(FMM_EINVAL, "fmm_mlp_train: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    if (int rc = scratch()) return rc;
    MLPCHK(hipMemsetAsync(g_scr.m, 0, sizeof(float) * NP, st));
    MLPCHK(hipMemsetAsync(g_scr.v, 0, sizeof(float) * NP, st));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t t = 1; t <= steps; ++t) {
        if (int rc = launch_loss_grad(params_dev, x_dev, t_dev, n, g_scr.loss, g_scr.grad, st)) return rc;
        if (loss_hist_dev) k_copy1<<<1, 1, 0, st>>>(g_scr.loss, loss_hist_dev + (t - 1));
        const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
        const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
        k_adam<<<(NP + 255) / 256, 256, 0, st>>>(params_dev, g_scr.grad, g_scr.m, g_scr.v, lr, b1, b2, eps, c1, c2);
    }
    MLPCHK(hipGetLastError());
    MLPCHK(hipStreamSynchronize(st));
    return 0;
}

} // extern "C"
