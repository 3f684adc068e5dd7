// Exact all-pairs top-2 (the naive full rebuild and the frontier ground truth
// of Section 3, six strategies; Table 2's brute-force pass), for gfx950.
//
// One workgroup owns 64 queries (one per lane) and S waves; wave w scans the
// j-range [w*L, (w+1)*L) in ascending order.  The j coordinates are
// wave-uniform, so they are fetched with scalar loads into SGPRs and fed to
// the VALU as scalar operands: no LDS traffic and no per-lane address work in
// the inner loop.  Per pair the VALU work is the fixed binary32 distance
// (3d-1 operations, no FMA) plus min, med3, compare and select for the
// running top-2.  Only the j-range that contains the wave's own queries runs
// the variant that excludes the self pair.  The S partial top-2s are merged in
// LDS in ascending j order with the lowest-index tie rule, then d1 = sqrtf(s1),
// d2 = sqrtf(s2).
#include "device_common.hpp"
#include "internal.hpp"

namespace nnc {

namespace {

template <int D, bool CHECK>
__device__ __forceinline__ void scan_range(const float *__restrict__ px, const float *__restrict__ py,
                                           const float *__restrict__ pz, int j0, int j1, float xi, float yi,
                                           float zi, int i, float &s1, float &s2, int &nn)
{
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
        float s = sqdist<D>(xi, yi, zi, px[j], py[j], D == 3 ? pz[j] : 0.0f);
        if constexpr (CHECK) s = (j == i) ? kInf : s;
        const bool b = s < s1;
        s2 = __builtin_amdgcn_fmed3f(s1, s2, s);
        s1 = fminf(s1, s);
        nn = b ? j : nn;
    }
}

template <int D, int S>
__global__ void __launch_bounds__(64 * S) k_allpairs(const float *__restrict__ pos, int n,
                                                     const int *__restrict__ qidx, int nq, int chunk,
                                                     int *__restrict__ nn_out, float *__restrict__ d1_out,
                                                     float *__restrict__ d2_out)
{
    __shared__ float s_s1[S][64];
    __shared__ float s_s2[S][64];
    __shared__ int s_nn[S][64];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 64 + lane;
    int i = q < nq ? (qidx ? qidx[q] : q) : -1;
    const bool active = i >= 0 && i < n;
    if (!active) i = -1;
    const float *__restrict__ px = pos;
    const float *__restrict__ py = pos + (size_t)n;
    const float *__restrict__ pz = pos + 2 * (size_t)n;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (active) {
        xi = px[i];
        yi = py[i];
        if constexpr (D == 3) zi = pz[i];
    }
    // span of this wave's query indices: the only j that need the self check
    int lo = active ? i : 0x7fffffff, hi = active ? i : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off, 64));
        hi = max(hi, __shfl_xor(hi, off, 64));
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    const int j0 = w * chunk;
    const int j1 = min(j0 + chunk, n);
    float s1 = kInf, s2 = kInf;
    int nn = -1;
    if (j0 < j1) {
        const int a = max(j0, min(j1, lo));   // [j0, a) unchecked
        const int b = max(a, min(j1, hi + 1));  // [a, b) checked, [b, j1) unchecked
        scan_range<D, false>(px, py, pz, j0, a, xi, yi, zi, i, s1, s2, nn);
        scan_range<D, true>(px, py, pz, a, b, xi, yi, zi, i, s1, s2, nn);
        scan_range<D, false>(px, py, pz, b, j1, xi, yi, zi, i, s1, s2, nn);
    }
    if constexpr (S == 1) {
        if (active) {
            nn_out[q] = nn;
            d1_out[q] = cert_sqrt(s1);
            d2_out[q] = cert_sqrt(s2);
        }
    } else {
        s_s1[w][lane] = s1;
        s_s2[w][lane] = s2;
        s_nn[w][lane] = nn;
        __syncthreads();
        if (w == 0 && active) {
            Top2 t;
            t.s1 = s_s1[0][lane];
            t.s2 = s_s2[0][lane];
            t.nn = s_nn[0][lane];
#pragma unroll
            for (int k = 1; k < S; ++k) t.merge(s_s1[k][lane], s_s2[k][lane], s_nn[k][lane]);
            nn_out[q] = t.nn;
            d1_out[q] = cert_sqrt(t.s1);
            d2_out[q] = cert_sqrt(t.s2);
        }
    }
}

template <int D>
int launch_d(const float *pos, int n, const int32_t *qidx, int nq, int32_t *nn, float *d1, float *d2,
             hipStream_t s)
{
    const int blocks = (nq + 63) / 64;
    // aim at about four waves per SIMD (256 CUs x 4 SIMDs)
    int S = 1;
    while (S < 16 && (long long)blocks * S * 2 <= 4096 && (long long)(S * 2) * 64 <= (long long)n) S *= 2;
    int chunk = (n + S - 1) / S;
    chunk = (chunk + 63) & ~63;
    switch (S) {
    case 1:
        hipLaunchKernelGGL((k_allpairs<D, 1>), dim3(blocks), dim3(64), 0, s, pos, n, qidx, nq, chunk, nn, d1, d2);
        break;
    case 2:
        hipLaunchKernelGGL((k_allpairs<D, 2>), dim3(blocks), dim3(128), 0, s, pos, n, qidx, nq, chunk, nn, d1, d2);
        break;
    case 4:
        hipLaunchKernelGGL((k_allpairs<D, 4>), dim3(blocks), dim3(256), 0, s, pos, n, qidx, nq, chunk, nn, d1, d2);
        break;
    case 8:
        hipLaunchKernelGGL((k_allpairs<D, 8>), dim3(blocks), dim3(512), 0, s, pos, n, qidx, nq, chunk, nn, d1, d2);
        break;
    default:
        hipLaunchKernelGGL((k_allpairs<D, 16>), dim3(blocks), dim3(1024), 0, s, pos, n, qidx, nq, chunk, nn, d1,
                           d2);
        break;
    }
    return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP;
}

__global__ void __launch_bounds__(256) k_sqrt(const float *__restrict__ x, float *__restrict__ out, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = cert_sqrt(x[i]);
}

}  // namespace

int launch_sqrt(const float *x, float *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return NNC_OK;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_sqrt, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, x, out,
                       (long long)n);
    return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP;
}

int launch_allpairs(const float *pos, int64_t n, int d, const int32_t *qidx, int64_t nq, int32_t *nn, float *d1,
                    float *d2, hipStream_t s)
{
    if (nq <= 0) return NNC_OK;
    return d == 2 ? launch_d<2>(pos, (int)n, qidx, (int)nq, nn, d1, d2, s)
                  : launch_d<3>(pos, (int)n, qidx, (int)nq, nn, d1, d2, s);
}

}  // namespace nnc
