// Device-side building blocks shared by the gfx950 kernels of libnncert.
//
// The file is compiled with -ffp-contract=off and the pragma below, so no
// expression is contracted into a fused multiply-add: the certificate
// arithmetic is the fixed binary32 formula stated in nncert.h (Definition 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace nnc {

constexpr float kInf = __builtin_inff();

// Square root of the certificates (d1, d2), of eps_t and of the predictor's
// displacements: binary32, correctly rounded (the gfx950 lowering of sqrtf without
// fast-math flags; nnc_sqrt_f32 exposes it so that its rounding can be checked).
__device__ __forceinline__ float cert_sqrt(float s) { return sqrtf(s); }

// Squared distance ((dx*dx) + (dy*dy)) + (dz*dz), dx = x_j - x_i, binary32.
template <int D>
__device__ __forceinline__ float sqdist(float xi, float yi, float zi, float xj, float yj, float zj)
{
    const float dx = xj - xi;
    const float dy = yj - yi;
    const float sx = dx * dx;
    const float sy = dy * dy;
    float s = sx + sy;
    if constexpr (D == 3) {
        const float dz = zj - zi;
        const float sz = dz * dz;
        s = s + sz;
    }
    return s;
}

// Running top-2 of one query in any scan order: (s1, nn) is the minimum with
// ties to the lowest index and s2 the second smallest value of the multiset.
// med3(s1, s2, s) is the second smallest of {s1, s2, s} because s1 <= s2.
struct Top2 {
    float s1, s2;
    int nn;
    __device__ __forceinline__ void init()
    {
        s1 = kInf;
        s2 = kInf;
        nn = -1;
    }
    __device__ __forceinline__ void push(float s, int j)
    {
        const bool better = (s < s1) || (s == s1 && j < nn);
        s2 = __builtin_amdgcn_fmed3f(s1, s2, s);
        s1 = fminf(s1, s);
        nn = better ? j : nn;
    }
    // Merge the top-2 of a disjoint set of points.
    __device__ __forceinline__ void merge(float o1, float o2, int onn)
    {
        const bool better = (o1 < s1) || (o1 == s1 && onn < nn && onn >= 0);
        const float hi = fmaxf(s1, o1);
        s2 = fminf(hi, fminf(s2, o2));
        s1 = fminf(s1, o1);
        nn = better ? onn : nn;
    }
};

// Cell coordinate on one axis: floor(fl32(x * G)) clamped to [0, G-1].
__device__ __forceinline__ int cell_axis(float x, int G)
{
    const float q = x * (float)G;
    const float f = floorf(q);
    const float c = fminf(fmaxf(f, 0.0f), (float)(G - 1));
    return (int)c;
}

template <int D>
__device__ __forceinline__ int cell_id(float x, float y, float z, int G)
{
    int id = cell_axis(x, G) + G * cell_axis(y, G);
    if constexpr (D == 3) id += G * G * cell_axis(z, G);
    return id;
}

// The domain box of a scene: cells of axis k cover [lo_k, hi_k) in G equal parts,
// s_k = fl32(G / (hi_k - lo_k)) (the division in binary64); w_k = (hi_k - lo_k) / G
// in binary64 for distance bounds.  The unit box is lo = 0, s = G, w = 1/G, with
// which the cell formula below is exactly floor(fl32(x * G)).
struct Box {
    float lo[3], s[3];
    double w[3];
};

// Cell coordinate on one axis of a box: floor(fl32(fl32(x - lo) * s)) clamped to
// [0, G-1].
__device__ __forceinline__ int cell_axis(float x, float lo, float s, int G)
{
    const float q = (x - lo) * s;
    const float f = floorf(q);
    const float c = fminf(fmaxf(f, 0.0f), (float)(G - 1));
    return (int)c;
}

template <int D>
__device__ __forceinline__ int cell_id(float x, float y, float z, int G, const Box &b)
{
    int id = cell_axis(x, b.lo[0], b.s[0], G) + G * cell_axis(y, b.lo[1], b.s[1], G);
    if constexpr (D == 3) id += G * G * cell_axis(z, b.lo[2], b.s[2], G);
    return id;
}

template <int D>
__device__ __forceinline__ bool all_finite(float x, float y, float z)
{
    bool ok = __builtin_isfinite(x) && __builtin_isfinite(y);
    if constexpr (D == 3) ok = ok && __builtin_isfinite(z);
    return ok;
}

// Expiry key of a certificate computed at clock S: S + (c - g*d2) * K, binary64;
// +inf without a second neighbour.
__device__ __forceinline__ double expiry(double S, float d1, float d2, double guard, double K)
{
    if (__builtin_isinf(d2)) return __builtin_inf();
    const float c = d2 - d1;
    const double gd = guard * (double)d2;
    const double num = (double)c - gd;
    const double off = num * K;
    return S + off;
}

// Agent-scope relaxed atomics on a 64-bit word: coherent across the XCDs'
// separate L2 caches without a cache-wide fence.
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Number of set bits of a 64-lane mask strictly below this lane.
__device__ __forceinline__ int rank_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// 64-bit mixing function (SplitMix64 finaliser, Steele, Lea & Flood 2014).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace nnc
