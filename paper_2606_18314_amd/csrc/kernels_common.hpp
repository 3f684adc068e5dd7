// Device routines shared by the single-scene kernels (grid.hip) and the batched
// kernels (batch.hip): workgroup scans, the clock advance, the entropy
// reduction, and the lane-group exact 2-NN query through the loose grid.
#pragma once
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace nnc {
namespace kc {

constexpr double kFuzz = 0x1p-20;  // cell-boundary rounding allowance (coordinates)
constexpr double kRel = 0x1p-20;   // relative allowance on drift and distances
constexpr double kCutSlack = 0x1p-16;  // relative slack of the repair cut-off

// Exclusive scan of one value per thread over a workgroup of NT threads.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int *s_w, int &total)
{
    const int lane = (int)lane_id(), w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int wbase = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        const int t = s_w[k];
        wbase += (k < w) ? t : 0;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return wbase + x - v;
}

// Add a per-lane change of the occupied-cell count with one atomic per wave.
__device__ __forceinline__ void add_C(DevScalars *sc, int delta)
{
    const int w = wave_sum(delta);
    if (lane_id() == 0 && w != 0) atomicAdd(&sc->C, w);
}

// Per-workgroup publication of the ingest results: the largest squared
// displacement and the change of the occupied-cell count, reduced over the
// workgroup first so that one atomic per quantity leaves each workgroup (the
// words are shared by every workgroup of the launch).
template <int NT>
__device__ __forceinline__ void publish_ingest(DevScalars *sc, int parity, float sq, int dC)
{
    constexpr int NW = NT / 64;
    __shared__ float s_sq[NW];
    __shared__ int s_dc[NW];
    sq = wave_max(sq);
    dC = wave_sum(dC);
    const int w = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
        s_sq[w] = sq;
        s_dc[w] = dC;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        int c = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            m = fmaxf(m, s_sq[k]);
            c += s_dc[k];
        }
        if (c != 0) atomicAdd(&sc->C, c);
        if (m > 0.0f) atomicMax(&sc->dmax[parity], __float_as_uint(m));
    }
}

// Clock advance shared by the filter variants, called by every thread of a full
// workgroup: each wave derives S_t from the displacement maximum (the shared
// word and its kSpread slots, one per lane); the leading wave publishes S_t,
// folds the occupied-cell changes into C and clears the other parity's words.
__device__ __forceinline__ double advance_clock(DevScalars *sc, int parity, float eps_decl, bool leader_wave)
{
    const int lane = (int)lane_id();
    const float m = fmaxf(wave_max(__uint_as_float(sc->dmax_part[parity][lane])), __uint_as_float(sc->dmax[parity]));
    const float eps = cert_sqrt(m);
    const double St = sc->S[parity ^ 1] + (double)eps;
    if (leader_wave) {
        const int dc = wave_sum(sc->dC_part[lane]);
        sc->dC_part[lane] = 0;
        sc->dmax_part[parity ^ 1][lane] = 0u;
        if (lane == 0) {
            sc->C += dc;
            sc->S[parity] = St;
            sc->eps = (double)eps;
            sc->dmax[parity ^ 1] = 0u;
            if (eps_decl >= 0.0f && (double)eps > (double)eps_decl * (1.0 + 0x1p-16) + 0x1p-20)
                atomicOr(&sc->err, kErrEps);
        }
    }
    return St;
}

// Ingest results of a workgroup into slot blockIdx % kSpread of the spread words
// (the launch may have thousands of workgroups; a slot sees few of them).
template <int NT>
__device__ __forceinline__ void publish_ingest_spread(DevScalars *sc, int parity, float sq, int dC)
{
    constexpr int NW = NT / 64;
    __shared__ float s_sq[NW];
    __shared__ int s_dc[NW];
    sq = wave_max(sq);
    dC = wave_sum(dC);
    const int w = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
        s_sq[w] = sq;
        s_dc[w] = dC;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        int c = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            m = fmaxf(m, s_sq[k]);
            c += s_dc[k];
        }
        const int slot = (int)(blockIdx.x & 63);
        if (c != 0) atomicAdd(&sc->dC_part[slot], c);
        if (m > 0.0f) atomicMax(&sc->dmax_part[parity][slot], __float_as_uint(m));
    }
}

// Normalised entropy (Definition 2) of the failures (which = 0) or candidates
// (which = 1) over the touched cells, computed by one workgroup of NT threads;
// clears the histogram entries and counters it consumed.
// Sum of a double over a workgroup of NT threads; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double s_acc[NT / 64];
    v = wave_sum(v);
    if (lane_id() == 0) s_acc[threadIdx.x >> 6] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) tot += s_acc[k];
    return tot;
}

// This thread's share (k = k0, k0 + stride, ...) of sum n_k ln n_k over the touched
// cells; clears the histogram entries it reads.
__device__ __forceinline__ double entropy_terms(int m, int *__restrict__ hist, const int *__restrict__ touched,
                                                int k0, int stride)
{
    double acc = 0.0;
    for (int k = k0; k < m; k += stride) {
        const int c = touched[k];
        const int nk = hist[c];
        hist[c] = 0;
        acc += (double)nk * log((double)nk);
    }
    return acc;
}

// H = (ln F - sum n ln n / F) / ln C (0 when F = 0 or C <= 1); publishes the
// result and resets the counters of the histogram it consumed.  One thread.
__device__ __forceinline__ void entropy_finish(int which, double tot, DevScalars *sc)
{
    const int m = which == 0 ? sc->ntouched : sc->ncand_touched;
    const int F = which == 0 ? sc->nfail : sc->nfront;
    const int C = sc->C;
    double H = 0.0;
    if (F > 0 && C > 1) H = (log((double)F) - tot / (double)F) / log((double)C);
    sc->H[which] = H;
    sc->m[which] = m;
    sc->F[which] = F;
    sc->Cres[which] = C;
    if (which == 0) {
        sc->nfail = 0;
        sc->ntouched = 0;
    } else {
        sc->ncand_touched = 0;
    }
}

// Normalised entropy (Definition 2) of the failures (which = 0) or candidates
// (which = 1) over the touched cells, computed by one workgroup of NT threads.
template <int NT>
__device__ void entropy_block(int which, int *__restrict__ hist, const int *__restrict__ touched, DevScalars *sc)
{
    const int m = which == 0 ? sc->ntouched : sc->ncand_touched;
    const double tot = block_sum<NT>(entropy_terms(m, hist, touched, (int)threadIdx.x, NT));
    if (threadIdx.x == 0) entropy_finish(which, tot, sc);
}

// Histogram-scan form of the entropy reduction, for a histogram without a list of
// touched cells: this thread's share of (F, m, sum n ln n) over the int4 groups
// k0, k0 + stride, ... of hist (zero-padded to a multiple of four cells); clears
// the nonzero groups it reads.  Four groups are loaded before any is cleared.
struct HistSums {
    double F, m, s;
};

__device__ __forceinline__ void hist_terms(int *__restrict__ hist, int ncell4, int k0, int stride, HistSums &r)
{
    int4 *h4 = reinterpret_cast<int4 *>(hist);
    for (int k = k0; k < ncell4; k += 4 * stride) {
        int4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = k + u * stride;
            v[u] = idx < ncell4 ? h4[idx] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if ((v[u].x | v[u].y | v[u].z | v[u].w) == 0) continue;
            h4[k + u * stride] = make_int4(0, 0, 0, 0);
            const int c[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (c[e] > 0) {
                    r.F += (double)c[e];
                    r.m += 1.0;
                    r.s += (double)c[e] * log((double)c[e]);
                }
            }
        }
    }
}

// Workgroup sum of HistSums; valid in thread 0.
template <int NT>
__device__ __forceinline__ HistSums block_sums(HistSums r)
{
    __shared__ double s_v[3][NT / 64];
    r.F = wave_sum(r.F);
    r.m = wave_sum(r.m);
    r.s = wave_sum(r.s);
    if (lane_id() == 0) {
        s_v[0][threadIdx.x >> 6] = r.F;
        s_v[1][threadIdx.x >> 6] = r.m;
        s_v[2][threadIdx.x >> 6] = r.s;
    }
    __syncthreads();
    HistSums t{0.0, 0.0, 0.0};
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) {
            t.F += s_v[0][k];
            t.m += s_v[1][k];
            t.s += s_v[2][k];
        }
    return t;
}

// H from the sums (F = number of items, m = cells they meet); one thread.
__device__ __forceinline__ void entropy_publish(int which, const HistSums &t, DevScalars *sc)
{
    const int F = (int)t.F, C = sc->C;
    double H = 0.0;
    if (F > 0 && C > 1) H = (log(t.F) - t.s / t.F) / log((double)C);
    sc->H[which] = H;
    sc->m[which] = (int)t.m;
    sc->F[which] = F;
    sc->Cres[which] = C;
}

// Slot of each lane with pred set in a list whose length is *counter: one atomic
// per wave (lanes that are not active take no part).  -1 where pred is false.
__device__ __forceinline__ int wave_append(int *counter, bool pred)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + rank_below(m) : -1;
}

struct QueryArgs {
    const float *pos;          // current coordinates, point order
    const float4 *slots;       // slot records {x, y, z, point index}, current coordinates
    const int *cell_start, *cell;
    const int *list, *count_dev;
    int list_cap;              // entries of list readable past the count (the library's own
                               // lists hold n; 0 for a caller's list)
    int n, G, all, init, t, parity;
    int *nn, *stamp, *hist;
    int *touched;              // a batch scene's list of touched cells (with its counters);
                               // null for a single scene, whose entropy scans hist
    float *d1, *d2;
    double *e;
    double *Si;                // clock of each certificate (per-point budget), or null
    uint8_t *cmask;            // tiled repair: candidates marked in slot order (cleared as read); else null
    double *qkey;              // expiry calendar: new key of list entry q written at qkey[q]; else null
    int tiled_from;            // > 0: candidate lists of at least this many entries go to the tiled
                               // repair (the pointwise query then skips them); 0: no such split
    uint8_t *fail;
    DevScalars *sc;
    double guard, K;
    Box box;                   // the scene's domain box
    double fuzz;               // cell-boundary rounding allowance for this box
};

// Lower bound on the distance from (x,y,z) to any point whose build-time cell
// lies outside the box of cells [g-r, g+r]^d; sides at the grid edge are open
// (no cell lies beyond them).  +inf when the box covers the whole grid.
template <int D>
__device__ __forceinline__ double outside_bound(float x, float y, float z, int gx, int gy, int gz, int r, int G)
{
    double B = __builtin_inf();
    const double invG = 1.0 / (double)G;
    const float pc[3] = {x, y, z};
    const int gc[3] = {gx, gy, gz};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (gc[k] - r > 0) B = fmin(B, (double)pc[k] - (double)(gc[k] - r) * invG);
        if (gc[k] + r < G - 1) B = fmin(B, (double)(gc[k] + r + 1) * invG - (double)pc[k]);
    }
    return B;
}

template <int D>
__device__ __forceinline__ double outside_bound(float x, float y, float z, int gx, int gy, int gz, int r, int G,
                                                const Box &b)
{
    double B = __builtin_inf();
    const float pc[3] = {x, y, z};
    const int gc[3] = {gx, gy, gz};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double lo = (double)b.lo[k], w = b.w[k];
        if (gc[k] - r > 0) B = fmin(B, (double)pc[k] - (lo + (double)(gc[k] - r) * w));
        if (gc[k] + r < G - 1) B = fmin(B, (lo + (double)(gc[k] + r + 1) * w) - (double)pc[k]);
    }
    return B;
}

template <int L>
__device__ __forceinline__ void group_reduce(Top2 &t)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) {
        const float o1 = __shfl_xor(t.s1, off, L);
        const float o2 = __shfl_xor(t.s2, off, L);
        const int on = __shfl_xor(t.nn, off, L);
        t.merge(o1, o2, on);
    }
}

template <int D>
__device__ __forceinline__ void visit_slot(const QueryArgs &a, int k, float x, float y, float z, int i, Top2 &t)
{
    const float4 r = a.slots[k];
    const int j = __float_as_int(r.w);
    const float s = sqdist<D>(x, y, z, r.x, r.y, r.z);
    if (j != i) t.push(s, j);
}

// Visit the `total` slots of a concatenation of runs, L lanes at a time;
// slot_of(k) maps position k of the concatenation to its slot (it may shuffle
// within the group, so every lane calls it).  Past the first L positions the
// positions are taken four strides at a time: the four slots are found first and
// their records loaded together, so a long walk waits for one memory round trip
// per 4L slots instead of one per L.  Positions past the end load the last slot
// (a valid address) and are not visited.  Used for the 3^3 block of a query in
// the cube, whose walks are long; the shorter walks of the plane and of the rings
// keep a plain stride-L loop, which measured faster there.
template <int D, int L, class SlotOf>
__device__ __forceinline__ void walk_slots(const QueryArgs &a, float x, float y, float z, int i, int total,
                                           int lane, Top2 &t, SlotOf slot_of)
{
    constexpr int U = 4;
    if (total <= 0) return;
    if (total <= L) {
        const int slot = slot_of(min(lane, total - 1));
        if (lane < total) visit_slot<D>(a, slot, x, y, z, i, t);
        return;
    }
    for (int b = 0; b < total; b += U * L) {
        int sl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sl[u] = slot_of(min(b + u * L + lane, total - 1));
        float4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = a.slots[sl[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = __float_as_int(r[u].w);
            const float s2 = sqdist<D>(x, y, z, r[u].x, r[u].y, r[u].z);
            if (b + u * L + lane < total && j != i) t.push(s2, j);
        }
    }
}

// Axis gaps from a query point to the faces of its own cell, binary64: glo[k] to
// the lower face, ghi[k] to the upper one (clamped at 0: the rounded cell id can
// put a point a hair outside its cell; the search margin covers that).  A cell
// of the block at offset -1 (+1) along axis k is at least glo[k] (ghi[k]) away
// along that axis.
template <int D, bool UNIT>
__device__ __forceinline__ void cell_gaps(const QueryArgs &a, float x, float y, float z, int gx, int gy, int gz,
                                          double (&glo)[3], double (&ghi)[3])
{
    const float pc[3] = {x, y, z};
    const int gc[3] = {gx, gy, gz};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double f0, f1;
        if constexpr (UNIT) {
            const double invG = 1.0 / (double)a.G;
            f0 = (double)gc[k] * invG;
            f1 = (double)(gc[k] + 1) * invG;
        } else {
            const double lo = (double)a.box.lo[k], w = a.box.w[k];
            f0 = lo + (double)gc[k] * w;
            f1 = lo + (double)(gc[k] + 1) * w;
        }
        glo[k] = fmax((double)pc[k] - f0, 0.0);
        ghi[k] = fmax(f1 - (double)pc[k], 0.0);
    }
}

// Squared distance bound from the query to the row of cells at offsets (dy, dz),
// over the y and z axes only.
template <int D>
__device__ __forceinline__ double row_gap2(const double (&glo)[3], const double (&ghi)[3], int dy, int dz)
{
    double g = dy < 0 ? glo[1] * glo[1] : dy > 0 ? ghi[1] * ghi[1] : 0.0;
    if constexpr (D == 3) g += dz < 0 ? glo[2] * glo[2] : dz > 0 ? ghi[2] * ghi[2] : 0.0;
    return g;
}

// The part of row (dy, dz) of the 3^d block that lies within T of the query
// (T2 = T^2; +inf keeps the whole block): x range [xlo, xhi] (empty when xlo >
// xhi); `cut` is set when a cell of the row inside the grid is left out.
template <int D>
__device__ __forceinline__ void block_row(const double (&glo)[3], const double (&ghi)[3], double T2, int gx, int G,
                                          int dy, int dz, int &xlo, int &xhi, bool &cut)
{
    xlo = max(gx - 1, 0);
    xhi = min(gx + 1, G - 1);
    cut = false;
    if (T2 == __builtin_inf()) return;
    const double yz = row_gap2<D>(glo, ghi, dy, dz);
    if (yz > T2) {
        xlo = 1;
        xhi = 0;
        cut = true;
        return;
    }
    if (gx > 0 && yz + glo[0] * glo[0] > T2) {
        xlo = gx;
        cut = true;
    }
    if (gx < G - 1 && yz + ghi[0] * ghi[0] > T2) {
        xhi = gx;
        cut = true;
    }
}

// The cells of the 3^d block around (gx,gy,gz) that lie within T of the query,
// clipped to the grid: 3^(d-1) rows, each a contiguous run of slots.  Lanes first
// fetch one row's bounds each, then walk the concatenated slots with stride L.
// Returns (to every lane of the group) whether a cell of the block was left out.
template <int D, int L>
__device__ __forceinline__ bool scan_block(const QueryArgs &a, float x, float y, float z, int i, int gx, int gy,
                                           int gz, const double (&glo)[3], const double (&ghi)[3], double T2,
                                           int lane, Top2 &t)
{
    constexpr int R = D == 3 ? 9 : 3;
    const int G = a.G;
    if constexpr (L == 1) {
        // one thread per query: walk the block's rows one after another
        bool any = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int dy = r % 3 - 1, dz = D == 3 ? r / 3 - 1 : 0;
            const int cy = gy + dy, cz = gz + dz;
            if (cy < 0 || cy >= G || cz < 0 || cz >= (D == 3 ? G : 1)) continue;
            int xlo, xhi;
            bool cut;
            block_row<D>(glo, ghi, T2, gx, G, dy, dz, xlo, xhi, cut);
            any |= cut;
            if (xlo > xhi) continue;
            const int row = (cz * G + cy) * G;
            const int k1 = a.cell_start[row + xhi + 1];
            for (int k = a.cell_start[row + xlo]; k < k1; ++k) visit_slot<D>(a, k, x, y, z, i, t);
        }
        return any;
    }
    // one lane per row; a group of 8 in the cube also gives its first lane the ninth row
    static_assert(L == 1 || L >= R || (D == 3 && L == 8), "a group needs a lane per row");
    constexpr int RL = R < L ? R : L;  // rows held one per lane
    auto row_bounds = [&](int r, int &rs_, int &rl_, bool &cut_) {
        const int dy = r % 3 - 1, dz = D == 3 ? r / 3 - 1 : 0;
        const int cy = gy + dy, cz = gz + dz;
        if (cy >= 0 && cy < G && cz >= 0 && cz < (D == 3 ? G : 1)) {
            int xlo, xhi;
            block_row<D>(glo, ghi, T2, gx, G, dy, dz, xlo, xhi, cut_);
            if (xlo <= xhi) {
                const int row = (cz * G + cy) * G;
                rs_ = a.cell_start[row + xlo];
                rl_ = a.cell_start[row + xhi + 1] - rs_;
            }
        }
    };
    int rs = 0, rl = 0;
    bool cut = false;
    if (lane < RL) row_bounds(lane, rs, rl, cut);
    int rs9 = 0, rl9 = 0;  // the ninth row of a group of 8 (its first lane)
    if constexpr (RL < R) {
        bool cut9 = false;
        if (lane == 0) row_bounds(8, rs9, rl9, cut9);
        cut |= cut9;
    }
    const unsigned long long gmask = L == 64 ? ~0ull : ((1ull << L) - 1) << (lane_id() & ~(unsigned)(L - 1));
    const bool any = (__ballot(cut) & gmask) != 0;
    int incl = rl;
#pragma unroll
    for (int off = 1; off < RL; off <<= 1) {
        const int v = __shfl_up(incl, off, L);
        if (lane >= off) incl += v;
    }
    if constexpr (RL < R) {
        // eight rows on the lanes, the ninth after them: its prefix is the others' sum
        const int pre9 = __shfl(incl, RL - 1, L);
        const int start9 = __shfl(rs9, 0, L);
        const int total = pre9 + __shfl(rl9, 0, L);
        const int pre = incl - rl;
        walk_slots<D, L>(a, x, y, z, i, total, lane, t, [&](int kk) {
            int lo = 0;
#pragma unroll
            for (int step = L / 2; step > 0; step >>= 1) {
                const int p = __shfl(pre, lo + step, L);
                if (p <= kk) lo += step;
            }
            const int in_row = __shfl(rs, lo, L) + (kk - __shfl(pre, lo, L));
            return kk >= pre9 ? start9 + (kk - pre9) : in_row;
        });
        return any;
    }
    const int total = __shfl(incl, R - 1, L);
    if constexpr (D == 3) {
        // nine rows: each slot finds its row by a binary search over the rows'
        // prefixes held by lanes 0..8 (lanes 9.. hold an empty row at the end)
        const int pre = lane < R ? incl - rl : total;
        walk_slots<D, L>(a, x, y, z, i, total, lane, t, [&](int kk) {
            int lo = 0;
#pragma unroll
            for (int step = 8; step > 0; step >>= 1) {
                const int p = __shfl(pre, lo + step, L);
                if (p <= kk) lo += step;
            }
            return __shfl(rs, lo, L) + (kk - __shfl(pre, lo, L));
        });
        return any;
    }
    int rstart[R], rpre[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rstart[r] = __shfl(rs, r, L);
        rpre[r] = __shfl(incl - rl, r, L);
    }
#pragma unroll 4
    for (int k = lane; k < total; k += L) {
        int sr = rstart[0], pr = rpre[0];
#pragma unroll
        for (int u = 1; u < R; ++u) {
            const bool in = k >= rpre[u];
            sr = in ? rstart[u] : sr;
            pr = in ? rpre[u] : pr;
        }
        visit_slot<D>(a, sr + (k - pr), x, y, z, i, t);
    }
    return any;
}

// One x-contiguous run of the ring of cells at Chebyshev distance exactly r
// (r >= 2) from (gx,gy,gz): returns false when the run lies outside the grid.
// With m = 2r+1, in d = 3 the runs are the 2m full rows of the two z faces,
// the 2(m-2) full rows of the two y faces between them, and the 2(m-2)^2
// single cells of the two x faces; in d = 2 the two full y rows and the
// 2(m-2) single cells of the x sides.
template <int D>
__device__ __forceinline__ bool ring_run(int u, int r, int gx, int gy, int gz, int G, int &row, int &xlo, int &xhi)
{
    const int m = 2 * r + 1, m2 = m - 2;
    int dy, dz = 0, x0, x1;
    if constexpr (D == 3) {
        if (u < 2 * m) {
            dz = u < m ? -r : r;
            dy = u % m - r;
            x0 = -r;
            x1 = r;
        } else if (u < 2 * m + 2 * m2) {
            const int v = u - 2 * m;
            dy = v < m2 ? -r : r;
            dz = v % m2 - (r - 1);
            x0 = -r;
            x1 = r;
        } else {
            const int v = u - 2 * m - 2 * m2;
            const int f = v / (m2 * m2), rem = v % (m2 * m2);
            dz = rem / m2 - (r - 1);
            dy = rem % m2 - (r - 1);
            x0 = x1 = f ? r : -r;
        }
    } else {
        if (u < 2) {
            dy = u ? r : -r;
            x0 = -r;
            x1 = r;
        } else {
            const int v = u - 2;
            dy = v % m2 - (r - 1);
            x0 = x1 = v < m2 ? -r : r;
        }
    }
    const int cy = gy + dy, cz = gz + dz;
    if (cy < 0 || cy >= G || (D == 3 && (cz < 0 || cz >= G))) return false;
    xlo = max(gx + x0, 0);
    xhi = min(gx + x1, G - 1);
    if (xlo > xhi) return false;
    row = (cz * G + cy) * G;
    return true;
}

// Visit every slot of a list of x-contiguous runs of cells; run(u, row, xlo,
// xhi) gives run u (false: empty).  Runs are taken L at a time: each lane
// fetches one run's slot range, a group scan concatenates them, and the lanes
// walk the concatenation with stride L, finding each slot's run by a binary
// search over the group (all loops are uniform over the group, so every
// shuffle reads an active lane).
template <int D, int L, class Run>
__device__ __forceinline__ void scan_runs(const QueryArgs &a, float x, float y, float z, int i, int nruns,
                                          int lane, Top2 &t, Run run)
{
    for (int c0 = 0; c0 < nruns; c0 += L) {
        const int u = c0 + lane;
        int rs = 0, rl = 0;
        int row, xlo, xhi;
        if (u < nruns && run(u, row, xlo, xhi)) {
            rs = a.cell_start[row + xlo];
            rl = a.cell_start[row + xhi + 1] - rs;
        }
        int incl = rl;
#pragma unroll
        for (int off = 1; off < L; off <<= 1) {
            const int v = __shfl_up(incl, off, L);
            if (lane >= off) incl += v;
        }
        const int total = __shfl(incl, L - 1, L);
        const int pre = incl - rl;
        for (int b = 0; b < total; b += L) {
            const int k = b + lane;
            const int kk = min(k, total - 1);
            int lo = 0;
#pragma unroll
            for (int step = L / 2; step > 0; step >>= 1) {
                const int p = __shfl(pre, lo + step, L);
                if (p <= kk) lo += step;
            }
            const int slot = __shfl(rs, lo, L) + (kk - __shfl(pre, lo, L));
            if (k < total) visit_slot<D>(a, slot, x, y, z, i, t);
        }
    }
}

// Every slot of the ring r >= 2.
template <int D, int L>
__device__ __forceinline__ void scan_ring(const QueryArgs &a, float x, float y, float z, int i, int gx, int gy,
                                          int gz, int r, int lane, Top2 &t)
{
    const int G = a.G;
    const int m2 = 2 * r - 1;
    const int nruns = D == 3 ? 2 * (2 * r + 1) + 2 * m2 + 2 * m2 * m2 : 2 + 2 * m2;
    scan_runs<D, L>(a, x, y, z, i, nruns, lane, t, [&](int u, int &row, int &xlo, int &xhi) {
        return ring_run<D>(u, r, gx, gy, gz, G, row, xlo, xhi);
    });
}

// The cells of the 3^d block that scan_block left out for the same T2: per row
// two runs, the whole row when it was cut entirely, else its cut end cells.
template <int D, int L>
__device__ __forceinline__ void scan_block_rest(const QueryArgs &a, float x, float y, float z, int i, int gx,
                                                int gy, int gz, const double (&glo)[3], const double (&ghi)[3],
                                                double T2, int lane, Top2 &t)
{
    constexpr int R = D == 3 ? 9 : 3;
    const int G = a.G;
    scan_runs<D, L>(a, x, y, z, i, 2 * R, lane, t, [&](int u, int &row, int &xlo, int &xhi) {
        const int r = u >> 1, side = u & 1;
        const int dy = r % 3 - 1, dz = D == 3 ? r / 3 - 1 : 0;
        const int cy = gy + dy, cz = gz + dz;
        if (cy < 0 || cy >= G || cz < 0 || cz >= (D == 3 ? G : 1)) return false;
        int klo, khi;
        bool cut;
        block_row<D>(glo, ghi, T2, gx, G, dy, dz, klo, khi, cut);
        if (!cut) return false;
        row = (cz * G + cy) * G;
        if (klo > khi) {  // the whole row was left out
            xlo = max(gx - 1, 0);
            xhi = min(gx + 1, G - 1);
            return side == 0;
        }
        if (side == 0) {
            xlo = max(gx - 1, 0);
            xhi = klo - 1;
        } else {
            xlo = khi + 1;
            xhi = min(gx + 1, G - 1);
        }
        return xlo <= xhi;
    });
}

// Cell of a query point and the enclosure bound: the unit box (UNIT, with the
// constants folded) or the scene's domain box.
template <bool UNIT>
__device__ __forceinline__ int query_cell(const QueryArgs &a, float x, int k)
{
    if constexpr (UNIT)
        return cell_axis(x, a.G);
    else
        return cell_axis(x, a.box.lo[k], a.box.s[k], a.G);
}

template <int D, bool UNIT>
__device__ __forceinline__ double query_bound(const QueryArgs &a, float x, float y, float z, int gx, int gy, int gz,
                                              int r)
{
    if constexpr (UNIT)
        return outside_bound<D>(x, y, z, gx, gy, gz, r, a.G);
    else
        return outside_bound<D>(x, y, z, gx, gy, gz, r, a.G, a.box);
}

// Exact top-2 of (x,y,z) (point i excluded).  T is a cut-off on cell distance:
// an upper bound on the distance to the second neighbour plus the search margin
// (+inf: no bound known).  The first pass scans only the cells of the 3^d block
// within T; if its result is not enclosed by the cells it scanned (a left-out
// cell's points are farther than T - margin), the rest of the block is scanned
// and the search widens ring by ring as without a bound.  The bound only decides
// the order of the work: the result is exact for any T.  Returns the linear id of
// the query's cell (the same formula as the cell ids of the ingest).
template <int D, int L, bool UNIT>
__device__ int group_search(const QueryArgs &a, float x, float y, float z, int i, double margin, double T,
                            int lane, Top2 &t)
{
    const int gx = query_cell<UNIT>(a, x, 0), gy = query_cell<UNIT>(a, y, 1);
    const int gz = D == 3 ? query_cell<UNIT>(a, z, 2) : 0;
    const int cell = gx + a.G * gy + (D == 3 ? a.G * a.G * gz : 0);
    double glo[3] = {0.0, 0.0, 0.0}, ghi[3] = {0.0, 0.0, 0.0};
    double T2 = __builtin_inf();
    if (T < __builtin_inf()) {
        cell_gaps<D, UNIT>(a, x, y, z, gx, gy, gz, glo, ghi);
        T2 = T * T;
    }
    const bool cut = scan_block<D, L>(a, x, y, z, i, gx, gy, gz, glo, ghi, T2, lane, t);
    group_reduce<L>(t);
    if (cut) {
        // the cells left out are farther than T, their points farther than T - margin
        const double B = query_bound<D, UNIT>(a, x, y, z, gx, gy, gz, 1);
        const double Be = fmin(B, T) - margin;
        if (Be > 0.0 && (double)t.s2 < Be * Be * (1.0 - kRel)) return cell;
        if (lane != 0) t.init();
        scan_block_rest<D, L>(a, x, y, z, i, gx, gy, gz, glo, ghi, T2, lane, t);
        group_reduce<L>(t);
    }
    for (int r = 1;; ++r) {
        const double B = query_bound<D, UNIT>(a, x, y, z, gx, gy, gz, r);
        if (__builtin_isinf(B)) break;  // the whole grid has been visited
        const double Be = B - margin;
        if (Be > 0.0 && (double)t.s2 < Be * Be * (1.0 - kRel)) break;
        // every lane holds the merged result: keep it in lane 0 only, so that the
        // next merge combines disjoint sets
        if (lane != 0) t.init();
        scan_ring<D, L>(a, x, y, z, i, gx, gy, gz, r + 1, lane, t);
        group_reduce<L>(t);
    }
    return cell;
}

// Search margin: cell-boundary rounding plus the motion accumulated since the
// grid was built (the clock difference bounds every point's displacement).
__device__ __forceinline__ double query_margin(double St, double S_grid, double fuzz)
{
    const double drift = St - S_grid;
    return fuzz + drift * (1.0 + kRel);
}

// The new certificate of point i from its exact top-2 (old: its previous nearest
// neighbour): distances, expiry key, stamp, failure flag, failure histogram (and,
// for a batch scene, its failure count and touched-cell list).  cell: the point's
// current cell id, or -1 to read it.
__device__ __forceinline__ double write_certificate(const QueryArgs &a, int i, const Top2 &t, double St, int old,
                                                   int cell)
{
    const float d1 = cert_sqrt(t.s1), d2 = cert_sqrt(t.s2);
    const double key = expiry(St, d1, d2, a.guard, a.K);
    a.nn[i] = t.nn;
    a.d1[i] = d1;
    a.d2[i] = d2;
    a.e[i] = key;
    if (a.Si) a.Si[i] = St;
    a.stamp[i] = a.t;
    const bool f = !a.init && t.nn != old;
    a.fail[i] = f ? 1 : 0;
    if (a.touched == nullptr) {
        // histogram only (the entropy scans it): no shared counters
        if (f) atomicAdd(&a.hist[cell >= 0 ? cell : a.cell[i]], 1);
        return key;
    }
    // failure count and first touch of each cell: one counter atomic per wave
    const unsigned long long fm = __ballot(f);
    if (fm != 0) {
        if ((int)lane_id() == __ffsll((long long)fm) - 1) atomicAdd(&a.sc->nfail, (int)__popcll(fm));
        int c = 0;
        bool first = false;
        if (f) {
            c = cell >= 0 ? cell : a.cell[i];
            first = atomicAdd(&a.hist[c], 1) == 0;
        }
        const int at = wave_append(&a.sc->ntouched, first);
        if (first) a.touched[at] = c;
    }
    return key;
}

// First-pass cut-off of a query (repair or rebuild) from the point's previous certificate
// (d1, d2, expiry key e, made at clock S_i): every point has moved at most
// S_t - S_i since (the clock sums the measured maximum steps), so the two old
// neighbours lie within d2 + 2 (S_t - S_i) of the query, which bounds its new
// second-neighbour distance.  S_i is recovered from the key (e - (c - g d2) K).
// The relative slack covers the rounding of the stored values; a bound that is
// still too small only costs the second pass of group_search.
__device__ __forceinline__ double repair_cutoff(float d1, float d2, double e, double St, double guard, double K,
                                                double margin)
{
    if (!(d2 < kInf) || !(e < __builtin_inf())) return __builtin_inf();
    const float c = d2 - d1;
    const double Si = e - ((double)c - guard * (double)d2) * K;
    const double dS = fmax(St - Si, 0.0);
    return ((double)d2 + 2.0 * dS) * (1.0 + kCutSlack) + margin;
}

// The cut-off of point i: from its stored certificate clock when the scene keeps
// one (its key may have been moved by the per-point budget), else from the key.
__device__ __forceinline__ double point_cutoff(const QueryArgs &a, int i, double St, double margin)
{
    if (a.Si) {
        const float d2 = a.d2[i];
        if (!(d2 < kInf)) return __builtin_inf();
        const double dS = fmax(St - a.Si[i], 0.0);
        return ((double)d2 + 2.0 * dS) * (1.0 + kCutSlack) + margin;
    }
    return repair_cutoff(a.d1[i], a.d2[i], a.e[i], St, a.guard, a.K, margin);
}

// Query q of a scene (the q-th candidate, or the q-th slot when recomputing all
// points) by the L lanes of one group; lane 0 writes the new certificate, its
// expiry key, stamp and failure flag, and counts a failure in the histogram.
template <int D, int L, bool UNIT>
__device__ __forceinline__ void query_one(const QueryArgs &a, int q, double St, double margin, int lane,
                                          bool have_i = false, int i_pre = 0)
{
    const size_t n1 = (size_t)a.n, n2 = 2 * (size_t)a.n;
    int i;
    float x, y, z = 0.f;
    if (a.all) {
        const float4 r = a.slots[q];
        i = __float_as_int(r.w);
        x = r.x;
        y = r.y;
        if constexpr (D == 3) z = r.z;
    } else {
        i = have_i ? i_pre : a.list[q];
        if (i < 0 || i >= a.n) return;  // caller-supplied lists are checked
        x = a.pos[i];
        y = a.pos[n1 + i];
        if constexpr (D == 3) z = a.pos[n2 + i];
    }
    const int old = lane == 0 ? a.nn[i] : 0;  // fetched early, used at the end
    double T = __builtin_inf();
    if (!a.init) T = point_cutoff(a, i, St, margin);
    Top2 t;
    t.init();
    const int cell = group_search<D, L, UNIT>(a, x, y, z, i, margin, T, lane, t);
    if (lane == 0) {
        const double key = write_certificate(a, i, t, St, old, cell);
        if (a.qkey && !a.all) a.qkey[q] = key;
    }
}

// Selector features of one scene-step (the same six numbers for a single scene
// and for a scene of a batch):
//   f0 = |F|/N, f1 = H of the candidates, f2 = ln N, f3 = d,
//   f4 = cells met by the candidates / G^d,
//   f5 = eps_t / median remaining motion budget e_i - S_{t-1} of the certificates of
//        the first kVSample points (a fixed sample: one pass of one workgroup),
// the median taken from a 64-bin power-of-two histogram (bin b: [2^(b-48), 2^(b-47))).
constexpr int kVBins = 64;
constexpr int kVSample = 1024;  // certificates whose budgets give the median of f5
constexpr int kVBias = 48;

__device__ __forceinline__ int validity_bin(double r) { return min(max(ilogb(r) + kVBias, 0), kVBins - 1); }

__device__ __forceinline__ double validity_median(const int *h)
{
    int V = 0;
    for (int b = 0; b < kVBins; ++b) V += h[b];
    int run = 0;
    for (int b = 0; b < kVBins; ++b) {
        run += h[b];
        if (V > 0 && 2 * run >= V) return ldexp(1.5, b - kVBias);
    }
    return 0.0;
}

__device__ __forceinline__ void scene_features(float *f, int n, int d, int ncell, int nfront, double Hc, int m,
                                               float eps, double radius)
{
    f[0] = n > 0 ? (float)nfront / (float)n : 0.0f;
    f[1] = (float)Hc;
    f[2] = n > 0 ? logf((float)n) : 0.0f;
    f[3] = (float)d;
    f[4] = (float)m / (float)ncell;
    f[5] = radius > 0.0 ? (float)((double)eps / radius) : 0.0f;
}

}  // namespace kc
}  // namespace nnc
