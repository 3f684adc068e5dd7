// Training and inference kernels of the repair/rebuild selector network
// (6 features -> 64 ReLU -> 64 ReLU -> 2 logits), FP32, for gfx950.
//
//   k_mlp_fwd_bwd  one thread per sample, parameters staged in LDS: forward
//                  pass, weighted softmax cross-entropy, and backpropagation to
//                  the pre-activation gradients of every layer, stored
//                  feature-major ([unit][sample]) so that both this kernel's
//                  stores and the next kernel's loads are coalesced;
//   k_mlp_wgrad    one thread per parameter: its gradient as a dot product over
//                  the batch (deterministic: no atomics), plus the batch loss;
//   k_mlp_adam     the Adam update of every parameter;
//   k_mlp_forward  logits of a batch (inference).
// Parameter layout: W1 [64x6], b1 [64], W2 [64x64], b2 [64], W3 [2x64], b3 [2].
#include <math.h>

#include <mutex>

#include "internal.hpp"

namespace nnc {

namespace {

constexpr int NF = NNC_FEATURES, NH = 64, NO = 2, NP = NNC_SELECTOR_PARAMS;
constexpr int OW1 = 0, OB1 = OW1 + NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NO * NH;
static_assert(OB3 + NO == NP, "parameter layout");
constexpr int kT = 256;

__device__ __forceinline__ void stage_params(const float *__restrict__ p, float *sp)
{
    for (int k = threadIdx.x; k < NP; k += blockDim.x) sp[k] = p[k];
    __syncthreads();
}

// Forward pass of sample x; returns the logits.  If H1/H2 are given, the hidden
// activations are stored feature-major at column b of a batch of B.
__device__ __forceinline__ void forward(const float *sp, const float *x, float *o, float *H1, float *H2, int b, int B)
{
    float h1[NH];
#pragma unroll 8
    for (int j = 0; j < NH; ++j) {
        float z = sp[OB1 + j];
#pragma unroll
        for (int k = 0; k < NF; ++k) z += sp[OW1 + j * NF + k] * x[k];
        h1[j] = fmaxf(z, 0.0f);
        if (H1) H1[(size_t)j * B + b] = h1[j];
    }
    float o0 = sp[OB3], o1 = sp[OB3 + 1];
    for (int j = 0; j < NH; ++j) {
        float z = sp[OB2 + j];
#pragma unroll 8
        for (int i = 0; i < NH; ++i) z += sp[OW2 + j * NH + i] * h1[i];
        const float h = fmaxf(z, 0.0f);
        if (H2) H2[(size_t)j * B + b] = h;
        o0 += sp[OW3 + j] * h;
        o1 += sp[OW3 + NH + j] * h;
    }
    o[0] = o0;
    o[1] = o1;
}

// Workspace, feature-major over the batch: H1, H2, D1, D2 [64][B], D3 [2][B], L [B].
__global__ void __launch_bounds__(kT) k_mlp_fwd_bwd(const float *__restrict__ p, const float *__restrict__ X,
                                                    const int *__restrict__ y, const float *__restrict__ w, int B,
                                                    float *__restrict__ ws)
{
    __shared__ float sp[NP];
    stage_params(p, sp);
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= B) return;
    float *H1 = ws, *H2 = H1 + (size_t)NH * B, *D1 = H2 + (size_t)NH * B, *D2 = D1 + (size_t)NH * B;
    float *D3 = D2 + (size_t)NH * B, *L = D3 + (size_t)NO * B;
    float x[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) x[k] = X[(size_t)b * NF + k];
    float o[2];
    forward(sp, x, o, H1, H2, b, B);
    const float mx = fmaxf(o[0], o[1]);
    const float e0 = expf(o[0] - mx), e1 = expf(o[1] - mx);
    const float lse = mx + logf(e0 + e1);
    const int yb = y[b];
    const float wb = w[b] / (float)B;
    L[b] = wb * (lse - (yb ? o[1] : o[0]));
    const float p0 = e0 / (e0 + e1), p1 = e1 / (e0 + e1);
    const float g0 = wb * (p0 - (yb == 0 ? 1.0f : 0.0f));
    const float g1 = wb * (p1 - (yb == 1 ? 1.0f : 0.0f));
    D3[b] = g0;
    D3[(size_t)B + b] = g1;
    float dh1[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) dh1[i] = 0.0f;
    for (int j = 0; j < NH; ++j) {
        const float h2 = H2[(size_t)j * B + b];
        const float dz2 = h2 > 0.0f ? sp[OW3 + j] * g0 + sp[OW3 + NH + j] * g1 : 0.0f;
        D2[(size_t)j * B + b] = dz2;
#pragma unroll 8
        for (int i = 0; i < NH; ++i) dh1[i] += sp[OW2 + j * NH + i] * dz2;
    }
#pragma unroll 8
    for (int i = 0; i < NH; ++i) {
        const float h1 = H1[(size_t)i * B + b];
        D1[(size_t)i * B + b] = h1 > 0.0f ? dh1[i] : 0.0f;
    }
}

__global__ void __launch_bounds__(kT) k_mlp_wgrad(const float *__restrict__ X, int B, const float *__restrict__ ws,
                                                  float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k > NP) return;
    const float *H1 = ws, *H2 = H1 + (size_t)NH * B, *D1 = H2 + (size_t)NH * B, *D2 = D1 + (size_t)NH * B;
    const float *D3 = D2 + (size_t)NH * B, *L = D3 + (size_t)NO * B;
    float acc = 0.0f;
    if (k == NP) {
        for (int b = 0; b < B; ++b) acc += L[b];
        *loss = acc;
        return;
    }
    if (k < OB1) {
        const int j = k / NF, c = k % NF;
        for (int b = 0; b < B; ++b) acc += D1[(size_t)j * B + b] * X[(size_t)b * NF + c];
    } else if (k < OW2) {
        const int j = k - OB1;
        for (int b = 0; b < B; ++b) acc += D1[(size_t)j * B + b];
    } else if (k < OB2) {
        const int j = (k - OW2) / NH, i = (k - OW2) % NH;
        for (int b = 0; b < B; ++b) acc += D2[(size_t)j * B + b] * H1[(size_t)i * B + b];
    } else if (k < OW3) {
        const int j = k - OB2;
        for (int b = 0; b < B; ++b) acc += D2[(size_t)j * B + b];
    } else if (k < OB3) {
        const int c = (k - OW3) / NH, j = (k - OW3) % NH;
        for (int b = 0; b < B; ++b) acc += D3[(size_t)c * B + b] * H2[(size_t)j * B + b];
    } else {
        const int c = k - OB3;
        for (int b = 0; b < B; ++b) acc += D3[(size_t)c * B + b];
    }
    grad[k] = acc;
}

__global__ void __launch_bounds__(kT) k_mlp_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                                 const float *__restrict__ g, float c1, float c2, float lr, float b1,
                                                 float b2, float eps)
{
    const int k = blockIdx.x * kT + threadIdx.x;
    if (k >= NP) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void __launch_bounds__(kT) k_mlp_forward(const float *__restrict__ p, const float *__restrict__ X, int B,
                                                    float *__restrict__ logits)
{
    __shared__ float sp[NP];
    stage_params(p, sp);
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= B) return;
    float x[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) x[k] = X[(size_t)b * NF + k];
    float o[2];
    forward(sp, x, o, nullptr, nullptr, b, B);
    logits[(size_t)b * 2] = o[0];
    logits[(size_t)b * 2 + 1] = o[1];
}

inline int check() { return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP; }

}  // namespace

// Workspace of nnc_mlp_grad_static: H1, H2, D1, D2 [64][B], D3 [2][B], L [B] for
// B <= NNC_MLP_STATIC_MAX_B, one copy per device for the life of the process.
constexpr size_t kStaticFloats = (size_t)(4 * NH + NO + 1) * NNC_MLP_STATIC_MAX_B;
static __device__ __align__(256) float scratch[kStaticFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices];  // device address of scratch, per device

// The device address of this device's copy of scratch (looked up once per device,
// with that device current).  Null on failure.
float *scratch_on(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return nullptr;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = (float *)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

}  // namespace nnc

extern "C" {

size_t nnc_mlp_workspace_bytes(int B) { return B > 0 ? (size_t)(4 * 64 + 2 + 1) * (size_t)B * sizeof(float) : 0; }

int nnc_mlp_grad(const float *params, const float *X, const int32_t *y, const float *w, int B, void *workspace,
                 float *grad, float *loss, void *stream)
{
    if (!params || !X || !y || !w || !workspace || !grad || !loss || B <= 0) return NNC_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(nnc::k_mlp_fwd_bwd, dim3((B + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0, s, params, X, y, w,
                       B, (float *)workspace);
    hipLaunchKernelGGL(nnc::k_mlp_wgrad, dim3((nnc::NP + 1 + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0, s, X, B,
                       (const float *)workspace, grad, loss);
    return nnc::check();
}

int nnc_mlp_grad_static(const float *params, const float *X, const int32_t *y, const float *w, int B, float *grad,
                        float *loss, void *stream)
{
    if (!params || !X || !y || !w || !grad || !loss || B <= 0 || B > NNC_MLP_STATIC_MAX_B) return NNC_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    if (s ? hipStreamGetDevice(s, &dev) != hipSuccess : hipGetDevice(&dev) != hipSuccess) return NNC_E_HIP;
    float *ws = nnc::scratch_on(dev);
    if (!ws) return NNC_E_HIP;
    // every workspace entry the gradient kernel reads is written by the first kernel
    // for this B: nothing needs clearing between calls
    hipLaunchKernelGGL(nnc::k_mlp_fwd_bwd, dim3((B + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0, s, params, X, y, w,
                       B, ws);
    hipLaunchKernelGGL(nnc::k_mlp_wgrad, dim3((nnc::NP + 1 + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0, s, X, B,
                       (const float *)ws, grad, loss);
    return nnc::check();
}

int nnc_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1, float beta2,
                 float eps, void *stream)
{
    if (!params || !m || !v || !grad || step < 1) return NNC_E_INVAL;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(nnc::k_mlp_adam, dim3((nnc::NP + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0,
                       (hipStream_t)stream, params, m, v, grad, c1, c2, lr, beta1, beta2, eps);
    return nnc::check();
}

int nnc_mlp_forward(const float *params, const float *X, int B, float *logits, void *stream)
{
    if (!params || !X || !logits || B < 0) return NNC_E_INVAL;
    if (B == 0) return NNC_OK;
    hipLaunchKernelGGL(nnc::k_mlp_forward, dim3((B + nnc::kT - 1) / nnc::kT), dim3(nnc::kT), 0,
                       (hipStream_t)stream, params, X, B, logits);
    return nnc::check();
}

}  // extern "C"
