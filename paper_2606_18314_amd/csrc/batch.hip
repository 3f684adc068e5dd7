// Batched maintenance step: many independent scenes of uneven size and
// dimension advanced together, for gfx950.
//
// Every kernel spans all scenes, or, with scenes of both dimensions, all scenes of
// one dimension: the plane's kernels up to their queries form one chain, the cube's
// another, run side by side on two streams (forked from the batch's stream and
// joined back before the entropy).  Tiles and query chunks are dealt to the XCDs in
// contiguous shares.
//   k_b_ingest   one workgroup per 1024-point tile of a scene: displacement,
//                per-scene maximum (one atomic per wave), cells, occupancy,
//                current coordinates into the grid slots (and, with the
//                per-point budget, the step stamps of the cells moving points
//                leave and enter);
//   k_b_budget   (per-point budget only) the same tiles: the budget tests of
//                the expired certificates, moving the keys of those kept;
//   k_b_filter   one 1024-thread workgroup per scene: clock, safety filter,
//                ordered compaction, candidate-cell histogram and entropy, the
//                six selector features, and the strategy decision (threshold
//                rule or the selector network, evaluated by the workgroup);
//   k_b_grid     one workgroup per scene that needs a fresh grid (rebuild, or
//                repair after the motion budget of the loose grid is spent):
//                cell-start scan and counting-sort scatter; one extra workgroup
//                turns the per-scene query counts into offsets per dimension;
//   k_b_query    one launch per dimension (more waves than can be resident,
//                each a contiguous chunk of the list) over the
//                queries of all scenes of that dimension (candidates of
//                repaired scenes, every point of rebuilt ones), L lanes per
//                query, the same exact search as one scene;
//   k_b_entropy  one workgroup per scene: failure entropy (Definition 2).
// No workgroup waits for another: all cross-scene coordination is by kernel
// order, so the step is safe to capture in a graph.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "kernels_common.hpp"

namespace nnc {

namespace {

using namespace kc;

constexpr int kB = 256;       // point-parallel workgroup
constexpr int kIU = 4;        // points per thread of the ingest
constexpr int kTile = kB * kIU;  // points of a scene per ingest workgroup
constexpr int kFB = 1024;     // per-scene workgroup
constexpr int kFRows = NNC_BATCH_MAX_N / kFB;
constexpr int kH = 64;        // selector hidden width
constexpr int kLnTable = 256; // candidate counts per cell with tabulated ln n and 1/n

}  // namespace

struct SceneDesc {
    int n, d, G, ncell;
    long long poff, coff, goff, soff;  // point, coordinate, cell and cell-start offsets
    double refresh_w;
};

// Launch arguments of the step kernels.  Everything that changes from one step
// to the next lives in device memory (the step counter, the clocks, the previous
// coordinates in the slot records, whether selector parameters are loaded), so a
// captured step replays as a fresh call would run: only the position buffer, the
// policy and tau are fixed by the launch.
struct BatchArgs {
    const SceneDesc *desc;
    int scenes, init, policy;
    float tau;
    int features_on;
    double guard, K;
    DevScalars *sc;
    int *tdev;                // [0] completed steps, [1] selector parameters loaded
    unsigned long long *cost; // per scene [filter, grid, query] wall-clock ticks (NNC_BATCH_TIMING), or null
    const float *pos_cur;
    float4 *slots;  // slot records {x, y, z, point index}, indexed by poff + slot
    int *cell, *counts, *rank, *cell_start, *cursor;
    int *nn, *stamp, *frontier, *hist_fail, *touched_fail, *hist_cand, *touched_cand;
    float *d1, *d2;
    double *e;
    double *Si;      // certificate clocks (per-point budget), or null
    int *last_move;  // per cell: last step a moving point left or entered it (per-point budget), or null
    uint8_t *fail;
    const int *tile_scene, *tile_start;
    const int *dscene;     // scene indices ordered by dimension: the plane's, then the cube's
    int *strategy, *need_grid, *qcount, *qpre;
    float *features;
    const float *params;
    const kc::QueryArgs *qs;  // per scene: the fixed part of its query view
};

namespace {

// Step number t of the running launch (0 during initialisation); step t reads the
// clock of parity (t - 1) & 1 and writes that of parity t & 1.
__device__ __forceinline__ int step_number(const BatchArgs &a) { return a.init ? 0 : a.tdev[0] + 1; }

// Workgroup b of nb runs on XCD b mod 8 (workgroups are dealt to the eight XCDs in
// turn); it takes item b / 8 of that XCD's contiguous share of the nb items (tiles,
// query chunks), so neighbouring items, mostly of one scene, share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b & 7, k = b >> 3;
    const int full = nb >> 3, rem = nb & 7;
    return x * full + min(x, rem) + k;
}

__global__ void __launch_bounds__(kB) k_b_cells_init(BatchArgs a, int first)
{
    const int tb = first + xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int s = a.tile_scene[tb];
    const SceneDesc sd = a.desc[s];
    int dC = 0;
    for (int u = 0; u < kIU; ++u) {
        const int i = a.tile_start[tb] + (int)threadIdx.x + u * kB;
        if (i >= sd.n) break;
        const float *p = a.pos_cur + sd.coff;
        const size_t n1 = (size_t)sd.n;
        const float x = p[i], y = p[n1 + i], z = sd.d == 3 ? p[2 * n1 + i] : 0.f;
        int c = 0;
        const bool ok = sd.d == 3 ? all_finite<3>(x, y, z) : all_finite<2>(x, y, z);
        if (ok)
            c = sd.d == 3 ? cell_id<3>(x, y, z, sd.G) : cell_id<2>(x, y, z, sd.G);
        else
            atomicOr(&a.sc[s].err, kErrNonFinite);
        a.cell[sd.poff + i] = c;
        dC += atomicAdd(&a.counts[sd.goff + c], 1) == 0;
    }
    add_C(&a.sc[s], dC);
}

// kIU points per thread (thread t of the tile: points t, t + kB, ...), their
// loads issued together so that each wave waits for few memory round trips.
__global__ void __launch_bounds__(kB) k_b_ingest(BatchArgs a, int first)
{
    const int tb = first + xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int s = a.tile_scene[tb];
    const SceneDesc sd = a.desc[s];
    const int i0 = a.tile_start[tb] + (int)threadIdx.x;
    const int parity = step_number(a) & 1;
    const float *pn = a.pos_cur + sd.coff;
    const size_t n1 = (size_t)sd.n, n2 = 2 * (size_t)sd.n;
    const bool d3 = sd.d == 3;
    float4 *slots = a.slots + sd.poff;
    int rk[kIU], oc[kIU];
#pragma unroll
    for (int u = 0; u < kIU; ++u) {
        const int i = i0 + u * kB;
        rk[u] = i < sd.n ? a.rank[sd.poff + i] : 0;
        oc[u] = i < sd.n ? a.cell[sd.poff + i] : 0;
    }
    float4 old4[kIU];
    float x1[kIU], y1[kIU], z1[kIU];
#pragma unroll
    for (int u = 0; u < kIU; ++u) {
        const int i = i0 + u * kB;
        const bool in = i < sd.n;
        // the slot record holds the point's coordinates of the previous step
        old4[u] = in ? slots[rk[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
        x1[u] = in ? pn[i] : 0.f;
        y1[u] = in ? pn[n1 + i] : 0.f;
        z1[u] = in && d3 ? pn[n2 + i] : 0.f;
    }
    float sq = 0.0f;
    int dC = 0;
#pragma unroll
    for (int u = 0; u < kIU; ++u) {
        const int i = i0 + u * kB;
        if (i >= sd.n) continue;
        slots[rk[u]] = make_float4(x1[u], y1[u], z1[u], __int_as_float(i));
        const float x0 = old4[u].x, y0 = old4[u].y, z0 = old4[u].z;
        const bool ok = d3 ? all_finite<3>(x1[u], y1[u], z1[u]) && all_finite<3>(x0, y0, z0)
                           : all_finite<2>(x1[u], y1[u], z1[u]) && all_finite<2>(x0, y0, z0);
        if (ok) {
            sq = fmaxf(sq, d3 ? sqdist<3>(x0, y0, z0, x1[u], y1[u], z1[u]) : sqdist<2>(x0, y0, z0, x1[u], y1[u], z1[u]));
            const int c = d3 ? cell_id<3>(x1[u], y1[u], z1[u], sd.G) : cell_id<2>(x1[u], y1[u], z1[u], sd.G);
            if (c != oc[u]) {
                a.cell[sd.poff + i] = c;
                dC -= atomicSub(&a.counts[sd.goff + oc[u]], 1) == 1;
                dC += atomicAdd(&a.counts[sd.goff + c], 1) == 0;
            }
            if (a.last_move && (x1[u] != x0 || y1[u] != y0 || z1[u] != z0)) {
                // the cells a moving point leaves and enters; every writer stores the same value
                a.last_move[sd.goff + oc[u]] = step_number(a);
                a.last_move[sd.goff + c] = step_number(a);
            }
        } else {
            atomicOr(&a.sc[s].err, kErrNonFinite);
        }
    }
    publish_ingest<kB>(&a.sc[s], parity, sq, dC);
}

// Per-point motion budget of every expired certificate, before the filter (the
// same two tests as a single scene's): (1) block-local: no cell of the point's
// 3^d block was stamped after its certificate and (d2 + D)(1 + 2^-20) + fuzz is
// below the distance to the outside of the block (D = S_t - S_i) -- the key moves
// to the next binary64 value above S_t; (2) distance: the kept neighbour's
// current distance r is below d2 (1 - g) - 2 D (1 + g) -- the key moves to
// S_t + gap K.  Otherwise the point stays expired and the filter lists it.  S_t is
// computed as the filter will compute it, read-only.  Tiles as in the ingest.
__global__ void __launch_bounds__(kB) k_b_budget(BatchArgs a, int first)
{
    const int tb = first + xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int s = a.tile_scene[tb];
    const SceneDesc sd = a.desc[s];
    const int parity = step_number(a) & 1;
    const DevScalars *sc = &a.sc[s];
    const int lane = (int)lane_id();
    const float m = fmaxf(wave_max(__uint_as_float(sc->dmax_part[parity][lane])), __uint_as_float(sc->dmax[parity]));
    const double St = sc->S[parity ^ 1] + (double)cert_sqrt(m);
    const int G = sd.G, n = sd.n;
    const bool d3 = sd.d == 3;
    const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
    const float *p = a.pos_cur + sd.coff;
    const double w = 1.0 / (double)G;
    for (int u = 0; u < kIU; ++u) {
        const int i = a.tile_start[tb] + (int)threadIdx.x + u * kB;
        if (i >= n) break;
        double *ei = a.e + sd.poff + i;
        if (!(St >= *ei)) continue;
        const int j = a.nn[sd.poff + i];
        if (j < 0 || j >= n) continue;
        const double dS = St - a.Si[sd.poff + i];
        const float d2 = a.d2[sd.poff + i];
        const float xi = p[i], yi = p[n1 + i], zi = d3 ? p[n2 + i] : 0.0f;
        {
            const int id = a.cell[sd.poff + i], si = a.stamp[sd.poff + i];
            const int gc[3] = {id % G, (id / G) % G, d3 ? id / (G * G) : 0};
            const int *lm = a.last_move + sd.goff;
            bool quiet = true;
            for (int oz = (d3 ? -1 : 0); oz <= (d3 ? 1 : 0) && quiet; ++oz) {
                const int z = gc[2] + oz;
                if (z < 0 || z >= (d3 ? G : 1)) continue;
                for (int oy = -1; oy <= 1 && quiet; ++oy) {
                    const int y = gc[1] + oy;
                    if (y < 0 || y >= G) continue;
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int x = gc[0] + ox;
                        if (x < 0 || x >= G) continue;
                        if (lm[x + G * (y + G * z)] > si) {
                            quiet = false;
                            break;
                        }
                    }
                }
            }
            if (quiet) {
                double B = __builtin_inf();
                const float pc[3] = {xi, yi, zi};
                for (int k = 0; k < (d3 ? 3 : 2); ++k) {
                    const double x = (double)pc[k];
                    if (gc[k] - 1 > 0) B = fmin(B, x - (double)(gc[k] - 1) * w);
                    if (gc[k] + 1 < G - 1) B = fmin(B, (double)(gc[k] + 2) * w - x);
                }
                const double need = ((double)d2 + dS) * (1.0 + 0x1p-20) + kFuzz;
                if (need < B) {
                    // the next binary64 value above the clock (S_t >= 0): tested again once anything moves
                    *ei = __longlong_as_double(__double_as_longlong(St) + 1);
                    continue;
                }
            }
        }
        const float sq = d3 ? sqdist<3>(xi, yi, zi, p[j], p[n1 + j], p[n2 + j])
                            : sqdist<2>(xi, yi, 0.0f, p[j], p[n1 + j], 0.0f);
        const float r = cert_sqrt(sq);
        const double thr = (double)d2 * (1.0 - a.guard) - 2.0 * (dS * (1.0 + a.guard));
        const double gap = thr - (double)r;
        if (gap > 0.0) *ei = St + gap * a.K;
    }
}

// The selector network evaluated by the whole 1024-thread workgroup (every thread
// calls it): layer 1 by the first wave (lane j: hidden unit j), layer 2 by all
// threads, thread j * 16 + p summing inputs 4p .. 4p + 3 of unit j (the weights
// read in one coalesced sweep) and the 16 parts combined by shuffles, layer 3 by
// the first wave.  Returns (in thread 0) 1 for rebuild, 0 for repair.
__device__ int mlp_decide(const float *__restrict__ p, const float *x, float *s_h1, float *s_h2)
{
    static_assert(kFB == kH * 16, "one thread per (unit, quarter-row) of layer 2");
    const int t = (int)threadIdx.x;
    const float *W1 = p, *b1 = p + kH * NNC_FEATURES, *W2 = b1 + kH, *b2 = W2 + kH * kH, *W3 = b2 + kH,
                *b3 = W3 + 2 * kH;
    if (t < kH) {
        float h = b1[t];
#pragma unroll
        for (int k = 0; k < NNC_FEATURES; ++k) h += W1[t * NNC_FEATURES + k] * x[k];
        s_h1[t] = fmaxf(h, 0.0f);
    }
    __syncthreads();
    {
        const int j = t >> 4, part = t & 15;
        const float4 wv = *reinterpret_cast<const float4 *>(W2 + j * kH + part * 4);
        float z = wv.x * s_h1[part * 4] + wv.y * s_h1[part * 4 + 1] + wv.z * s_h1[part * 4 + 2] +
                  wv.w * s_h1[part * 4 + 3];
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) z += __shfl_xor(z, off, 16);
        if (part == 0) s_h2[j] = fmaxf(b2[j] + z, 0.0f);
    }
    __syncthreads();
    int dec = 0;
    if (t < 64) {
        const float h2 = s_h2[t];
        float o0 = W3[t] * h2, o1 = W3[kH + t] * h2;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            o0 += __shfl_xor(o0, off, 64);
            o1 += __shfl_xor(o1, off, 64);
        }
        o0 += b3[0];
        o1 += b3[1];
        dec = o1 > o0 ? 1 : 0;
    }
    return dec;
}

__global__ void __launch_bounds__(kFB) k_b_filter(BatchArgs a, int first)
{
    constexpr int NW = kFB / 64;
    constexpr int NC = kFRows * NW;
    constexpr int PER = (NC + kFB - 1) / kFB;
    __shared__ int s_cnt[NC];
    __shared__ int s_w[NW];
    __shared__ int s_vh[kVBins];
    __shared__ double s_acc[NW];
    __shared__ double s_inv[NW];
    __shared__ double s_ln[kLnTable], s_rcp[kLnTable];
    __shared__ float s_x[NNC_FEATURES];
    __shared__ float s_h[kH];
    __shared__ float s_h2[kH];
    __shared__ int s_dec;
    const int s = a.dscene[first + (int)blockIdx.x];
    const long long t_start = a.cost ? wall_clock64() : 0;
    const SceneDesc sd = a.desc[s];
    DevScalars *sc = &a.sc[s];
    const int n = sd.n;
    const int parity = step_number(a) & 1;
    if (threadIdx.x < kVBins) s_vh[threadIdx.x] = 0;
    const double Sprev = sc->S[parity ^ 1];
    const float eps = cert_sqrt(__uint_as_float(sc->dmax[parity]));
    const double St = advance_clock(sc, parity, -1.0f, threadIdx.x < 64);
    double ev[kFRows];
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        const int i = k * kFB + (int)threadIdx.x;
        ev[k] = i < n ? a.e[sd.poff + i] : __builtin_inf();
    }
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const unsigned lane = lane_id();
    unsigned long long masks[kFRows];
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        const int i = k * kFB + (int)threadIdx.x;
        if (i < n) a.fail[sd.poff + i] = 0;
        masks[k] = __ballot(St >= ev[k]);
        if (lane == 0) s_cnt[k * NW + w] = __popcll(masks[k]);
    }
    __syncthreads();
    int v[PER];
    int loc = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = (int)threadIdx.x * PER + u;
        v[u] = idx < NC ? s_cnt[idx] : 0;
        loc += v[u];
    }
    int tot;
    int ex = block_excl_scan<kFB>(loc, s_w, tot);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = (int)threadIdx.x * PER + u;
        if (idx < NC) s_cnt[idx] = ex;
        ex += v[u];
    }
    __syncthreads();
    int *front = a.frontier + sd.poff;
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        if ((masks[k] >> lane) & 1ull) {
            const int at = s_cnt[k * NW + w] + rank_below(masks[k]);
            const int i = k * kFB + (int)threadIdx.x;
            if (at < n) front[at] = i;
        }
    }
    // The features (candidate histogram and entropy, the budget median) are computed
    // when statistics are requested, or under the learned policy for a scene whose
    // candidate fraction lies in the network's band [lo, hi) (outside it the size rule
    // decides: repair below lo, rebuild from hi on).
    const float f0 = n > 0 ? (float)tot / (float)n : 0.0f;
    const bool learned = a.policy == NNC_POLICY_LEARNED && a.tdev[1];
    const float band_lo = __int_as_float(a.tdev[2]), band_hi = __int_as_float(a.tdev[3]);
    const bool in_band = learned && f0 >= band_lo && f0 < band_hi;
    const bool want = a.features_on || in_band;
    if (want) {
        // the budget histogram of the first kVSample certificates (the first row), one
        // LDS add per distinct bin of the wave
        static_assert(kVSample == kFB, "the sample is the first row");
        {
            const int i = (int)threadIdx.x;
            int bin = -1;
            if (i < n) {
                const double r = ev[0] - Sprev;  // remaining motion budget of the certificate
                if (r > 0.0 && r < __builtin_inf()) bin = validity_bin(r);
            }
            unsigned long long left = __ballot(bin >= 0);
            while (left) {
                const int b = __shfl(bin, __ffsll((long long)left) - 1, 64);
                const unsigned long long same = __ballot(bin == b) & left;
                if (lane == 0) atomicAdd(&s_vh[b], (int)__popcll(same));
                left &= ~same;
            }
        }
    }
    // candidate cells: Definition 2's sum over cells of n ln n is the sum over candidates
    // of ln n_(cell of the candidate), and the cells met number the sum of 1 / n_(cell);
    // so the histogram is built with atomics whose results are not waited for, read
    // back once per candidate and cleared (each thread keeps its candidates' cells)
    double acc = 0.0, inv = 0.0;
    if (want) {
        // ln n and 1/n of the small counts from a table (one evaluation per thread,
        // instead of one per candidate on this one CU)
        if (threadIdx.x < kLnTable) {
            s_ln[threadIdx.x] = threadIdx.x > 0 ? log((double)threadIdx.x) : 0.0;
            s_rcp[threadIdx.x] = threadIdx.x > 0 ? 1.0 / (double)threadIdx.x : 0.0;
        }
        const int *cell = a.cell + sd.poff;
        int *hist = a.hist_cand + sd.goff;
        int cs[kFRows];
#pragma unroll
        for (int k = 0; k < kFRows; ++k) {
            cs[k] = -1;
            if ((masks[k] >> lane) & 1ull) {
                cs[k] = cell[k * kFB + (int)threadIdx.x];
                atomicAdd(&hist[cs[k]], 1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kFRows; ++k) {
            if (cs[k] >= 0) {
                // the adds above completed at the L2 before the barrier, and no line of
                // hist was read earlier in this kernel, so plain loads see them
                const int nk = hist[cs[k]];
                acc += nk < kLnTable ? s_ln[nk] : log((double)nk);
                inv += nk < kLnTable ? s_rcp[nk] : 1.0 / (double)nk;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kFRows; ++k)
            if (cs[k] >= 0) hist[cs[k]] = 0;
    }
    acc = wave_sum(acc);
    inv = wave_sum(inv);
    if (lane == 0) {
        s_acc[w] = acc;
        s_inv[w] = inv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0, msum = 0.0;
        for (int k = 0; k < NW; ++k) {
            sum += s_acc[k];
            msum += s_inv[k];
        }
        const int m = (int)llround(msum);  // an integer: the error of the sum is far below 1/2
        const int C = sc->C;
        double Hc = 0.0;
        if (tot > 0 && C > 1) Hc = (log((double)tot) - sum / (double)tot) / log((double)C);
        float f[NNC_FEATURES];
        scene_features(f, n, sd.d, sd.ncell, tot, Hc, m, eps, validity_median(s_vh));
        for (int k = 0; k < NNC_FEATURES; ++k) {
            s_x[k] = f[k];
            a.features[s * NNC_FEATURES + k] = f[k];
        }
        sc->nfront = tot;
        sc->H[1] = Hc;
        sc->m[1] = m;
        sc->F[1] = tot;
        sc->Cres[1] = C;
        int dec = 0;
        if (a.policy == NNC_POLICY_REBUILD) dec = 1;
        else if (a.policy == NNC_POLICY_THRESHOLD || (a.policy == NNC_POLICY_LEARNED && !learned))
            dec = f[0] >= a.tau ? 1 : 0;
        else if (a.policy == NNC_POLICY_LEARNED) dec = f0 >= band_hi ? 1 : 0;  // replaced in the band
        s_dec = dec;
    }
    __syncthreads();
    if (in_band) {
        bool finite = true;
        for (int k = 0; k < NNC_FEATURES; ++k) finite = finite && __builtin_isfinite(s_x[k]);
        if (finite) {  // uniform over the workgroup (shared features)
            const int dec = mlp_decide(a.params, s_x, s_h, s_h2);
            if (threadIdx.x == 0) s_dec = dec;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int dec = s_dec;
        a.strategy[s] = dec;
        a.need_grid[s] = dec == 1 || (St - sc->S_grid > sd.refresh_w);
        a.qcount[s] = dec == 1 ? n : tot;
        if (a.cost) {
            a.cost[3 * s] = (unsigned long long)(wall_clock64() - t_start);
            a.cost[3 * s + 2] = 0;  // the query kernel adds into it
        }
    }
}

// Per-scene grid builds (workgroups 0..scenes-1) and the query offsets (last workgroup).
__global__ void __launch_bounds__(kFB) k_b_grid(BatchArgs a, int first, int count, int dmask)
{
    __shared__ int s_w[kFB / 64];
    if ((int)blockIdx.x == count) {
        // query offsets per dimension (dimension d when bit d - 2 of dmask is set):
        // qpre[(d - 2) * (scenes + 1) + s] counts the queries of the scenes of
        // dimension d before scene s
        for (int d = 2; d <= 3; ++d) {
            if (!((dmask >> (d - 2)) & 1)) continue;
            int *pre = a.qpre + (d - 2) * (a.scenes + 1);
            int run = 0;
            for (int base = 0; base < a.scenes; base += kFB) {
                const int s = base + (int)threadIdx.x;
                const int v = s < a.scenes && a.desc[s].d == d ? a.qcount[s] : 0;
                int tot;
                const int ex = block_excl_scan<kFB>(v, s_w, tot);
                if (s < a.scenes) pre[s] = run + ex;
                run += tot;
            }
            if (threadIdx.x == 0) pre[a.scenes] = run;
        }
        return;
    }
    const int s = a.dscene[first + (int)blockIdx.x];
    if (!a.need_grid[s]) {
        if (a.cost && threadIdx.x == 0) a.cost[3 * s + 1] = 0;
        return;
    }
    const long long t_start = a.cost ? wall_clock64() : 0;
    const SceneDesc sd = a.desc[s];
    // cell-start scan over groups of four cells (the scene's cell regions start on
    // 16-byte boundaries and are padded with empty cells): wave w owns one
    // contiguous segment of the groups; it sums its segment, the workgroup scans
    // the 16 sums, then the wave scans its segment 64 groups at a time with a
    // running carry, four rounds of loads in flight (no workgroup barrier per
    // chunk).  Every padding entry receives the total, the sentinel included.
    {
        constexpr int NW = kFB / 64, U = 4;
        const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
        const int nq = (sd.ncell + 3) >> 2;
        const int seg = (((nq + NW - 1) / NW) + 63) & ~63;
        const int q0 = min(w * seg, nq), q1 = min(q0 + seg, nq);
        const int4 *cnt = reinterpret_cast<const int4 *>(a.counts + sd.goff);
        int4 *cs4 = reinterpret_cast<int4 *>(a.cell_start + sd.soff);
        int4 *cu4 = reinterpret_cast<int4 *>(a.cursor + sd.goff);
        int part = 0;
        for (int b = q0; b < q1; b += U * 64) {
            int4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b + u * 64 + lane;
                v[u] = k < q1 ? cnt[k] : make_int4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) part += v[u].x + v[u].y + v[u].z + v[u].w;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
        if (lane == 0) s_w[w] = part;
        __syncthreads();
        int carry = 0, total = 0;
        for (int k = 0; k < NW; ++k) {
            const int v = s_w[k];
            carry += k < w ? v : 0;
            total += v;
        }
        for (int b = q0; b < q1; b += U * 64) {
            int4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b + u * 64 + lane;
                v[u] = k < q1 ? cnt[k] : make_int4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b + u * 64 + lane;
                const int sum = v[u].x + v[u].y + v[u].z + v[u].w;
                int incl = sum;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int o = __shfl_up(incl, off, 64);
                    if (lane >= off) incl += o;
                }
                const int ex = carry + incl - sum;
                const int4 st = make_int4(ex, ex + v[u].x, ex + v[u].x + v[u].y, ex + v[u].x + v[u].y + v[u].z);
                if (k < q1) {
                    cs4[k] = st;
                    cu4[k] = st;
                }
                carry += __shfl(incl, 63, 64);
            }
        }
        if (threadIdx.x == 0) {
            a.cell_start[sd.soff + sd.ncell] = total;
            a.sc[s].S_grid = a.sc[s].S[step_number(a) & 1];
        }
    }
    __syncthreads();
    // counting-sort scatter, four points per thread in flight
    const size_t n1 = (size_t)sd.n;
    const float *p = a.pos_cur + sd.coff;
    float4 *so = a.slots + sd.poff;
    constexpr int U = 4;
    for (int i0 = (int)threadIdx.x; i0 < sd.n; i0 += U * kFB) {
        int k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kFB;
            k[u] = i < sd.n ? atomicAdd(&a.cursor[sd.goff + a.cell[sd.poff + i]], 1) : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kFB;
            if (i >= sd.n) continue;
            if (k[u] >= sd.n) {
                atomicOr(&a.sc[s].err, kErrOverflow);
                continue;
            }
            a.rank[sd.poff + i] = k[u];
            so[k[u]] = make_float4(p[i], p[n1 + i], sd.d == 3 ? p[2 * n1 + i] : 0.0f, __int_as_float(i));
        }
    }
    if (a.cost) {
        __syncthreads();
        if (threadIdx.x == 0) a.cost[3 * s + 1] = (unsigned long long)(wall_clock64() - t_start);
    }
}

// Per-scene view of the concatenated arrays for the shared query routine: the
// fixed part was built on the host at creation (one record per scene, read with
// scalar loads), so the query kernel keeps only the scene's view live, not the
// batch's base pointers as well; the step fills in what changes.
__device__ __forceinline__ QueryArgs scene_view(const BatchArgs &a, int s, int init, int t)
{
    // read through the constant address space: the records never change during a
    // launch, so the compiler may use scalar loads (the view stays in SGPRs)
#if __HIP_DEVICE_COMPILE__
    using CView = const __attribute__((address_space(4))) QueryArgs;
    QueryArgs q = ((CView *)a.qs)[s];
#else
    QueryArgs q = a.qs[s];  // (the host pass only parses this function)
#endif
    q.pos = a.pos_cur + a.desc[s].coff;
    q.all = a.strategy[s];
    q.init = init;
    q.t = t;
    q.parity = t & 1;
    return q;
}

// Every wave takes one contiguous chunk of the concatenated query list (all
// scenes' queries, scene by scene) and works on one scene at a time: per step its
// 64 / L lane groups take the next queries of the current scene (fewer at the
// scene's end), then the wave moves on.  The scene index is uniform over the wave,
// so the scene's descriptor and pointers sit in scalar registers and a wave never
// runs the plane and the cube search side by side.
// In the cube the kernel is held to five waves per SIMD (96 VGPRs, a few bytes of spill;
// measured faster than four waves without spill).
template <int D, int L>
__global__ void __launch_bounds__(kB) __attribute__((amdgpu_waves_per_eu(D == 3 ? 5 : 1))) k_b_query(BatchArgs a, int init)
{
    constexpr int GPW = 64 / L;  // lane groups per wave
    const int *qpre = a.qpre + (D - 2) * (a.scenes + 1);
    const int total = qpre[a.scenes];
    const int lane = threadIdx.x & (L - 1);
    const int grp = (int)(threadIdx.x & 63) / L;
    const int nw = (int)gridDim.x * (kB / 64);
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int w = __builtin_amdgcn_readfirstlane(blk * (kB / 64) + (int)(threadIdx.x >> 6));
    const int per = (total + nw - 1) / nw;
    int g = w * per;
    const int q1 = min(g + per, total);
    if (g >= q1) return;
    int lo = 0, hi = a.scenes;  // the last s with qpre[s] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (qpre[mid] <= g) lo = mid;
        else hi = mid;
    }
    int s = __builtin_amdgcn_readfirstlane(lo);
    const int t = step_number(a), parity = t & 1;
    while (g < q1) {
        const int first = qpre[s], next = qpre[s + 1];
        if (g < next) {
            const QueryArgs q = scene_view(a, s, init, t);
            const double St = a.sc[s].S[parity];
            const double margin = query_margin(St, a.sc[s].S_grid, kFuzz);
            const int end = min(next, q1);
            const long long t_start = a.cost ? wall_clock64() : 0;
            // list mode: the next round's list entry is loaded before this round's
            // query, so its round trip overlaps the query's
            const bool lst = !q.all;
            int nxt = lst && g + grp < end ? q.list[g + grp - first] : 0;
            for (; g < end; g += GPW) {
                const int cur = nxt;
                if (lst && g + GPW + grp < end) nxt = q.list[g + GPW + grp - first];
                if (g + grp < end) query_one<D, L, true>(q, g + grp - first, St, margin, lane, lst, cur);
            }
            g = end;
            if (a.cost && (threadIdx.x & 63) == 0)
                atomicAdd(&a.cost[3 * s + 2], (unsigned long long)(wall_clock64() - t_start));
        }
        ++s;
    }
}

__global__ void __launch_bounds__(kB) k_b_entropy(BatchArgs a)
{
    const int s = blockIdx.x;
    const SceneDesc sd = a.desc[s];
    entropy_block<kB>(0, a.hist_fail + sd.goff, a.touched_fail + sd.poff, &a.sc[s]);
    // the last kernel of a step counts it (no other workgroup of this launch reads the counter)
    if (s == 0 && threadIdx.x == 0) a.tdev[0] = step_number(a);
}

// Init: every scene rebuilds, every grid is built, queries are all points.
__global__ void k_b_init_flags(BatchArgs a)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < a.scenes; s += gridDim.x * blockDim.x) {
        a.strategy[s] = 1;
        a.need_grid[s] = 1;
        a.qcount[s] = a.desc[s].n;
    }
}

inline int check() { return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP; }

}  // namespace

}  // namespace nnc

// ---- host side -----------------------------------------------------------------------

#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

struct nnc_batch {
    int S, lanes;
    int lanes2, lanes3;     // lanes per query in the plane and in the cube
    double guard, K;
    hipStream_t stream;
    std::vector<nnc::SceneDesc> desc;
    std::vector<int> tile_scene, tile_start, dscene;
    std::vector<long long> point_off, coord_off;
    long long P, Q, NC, NS;
    int ntiles;
    void *arena;
    nnc::BatchArgs a;       // device pointers, refreshed per call
    size_t arena_bytes;
    int inited, features_on, eager, budget;
    int has_d[2];           // scenes of dimension 2, 3 present
    int S2;                 // scenes of dimension 2 (the first S2 entries of dscene)
    int T2;                 // ingest tiles of those scenes (the first T2 tiles)
    // with scenes of both dimensions, the plane's query runs on a second stream beside
    // the cube's (forked from and joined back into the batch's stream, also in a graph)
    hipStream_t side;
    hipEvent_t ev_fork, ev_join;
    double tick_us;         // microseconds per wall-clock tick (NNC_BATCH_TIMING)
    // the step as a graph: instantiated on the first call and replayed while
    // (positions, policy, tau) repeat; another key re-captures and updates it
    hipGraphExec_t exec;
    const float *g_pos;
    int g_policy;
    float g_tau;
};

namespace {

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int default_grid_b(int64_t n, int d)
{
    if (n <= 0) return 1;
    const double w = d == 2 ? 2.0 / sqrt((double)n) : cbrt(4.0 / (double)n);
    const double g = floor(1.0 / w);
    return g < 1.0 ? 1 : (int)g;
}

template <int D>
void launch_query_d(const nnc_batch *b, const nnc::BatchArgs &a, int init, hipStream_t st)
{
    // more waves than can be resident, each with a shorter chunk of the query list:
    // the chunks with slow queries hold up less (2048 -> 6144 workgroups: 0.833 ->
    // 0.764 ms per step on the 512-scene workload; waves without a chunk return)
    const int blocks = 6144;
    switch (D == 2 ? b->lanes2 : b->lanes3) {
    case 1: hipLaunchKernelGGL((nnc::k_b_query<D, 1>), dim3(blocks), dim3(nnc::kB), 0, st, a, init); break;
    case 64: hipLaunchKernelGGL((nnc::k_b_query<D, 64>), dim3(blocks), dim3(nnc::kB), 0, st, a, init); break;
    case 32: hipLaunchKernelGGL((nnc::k_b_query<D, 32>), dim3(blocks), dim3(nnc::kB), 0, st, a, init); break;
    case 4:
        if constexpr (D == 2)
            hipLaunchKernelGGL((nnc::k_b_query<2, 4>), dim3(blocks), dim3(nnc::kB), 0, st, a, init);
        break;
    case 8: hipLaunchKernelGGL((nnc::k_b_query<D, 8>), dim3(blocks), dim3(nnc::kB), 0, st, a, init); break;
    default: hipLaunchKernelGGL((nnc::k_b_query<D, 16>), dim3(blocks), dim3(nnc::kB), 0, st, a, init); break;
    }
}

// One launch per dimension present (each kernel holds one search, so the plane's
// launch is not limited by the cube's register use); with both, the two run side by
// side, each filling the other's tail.
int launch_query_b(const nnc_batch *b, const nnc::BatchArgs &a, int init)
{
    if (b->has_d[0] && b->has_d[1] && b->side) {
        if (hipEventRecord(b->ev_fork, b->stream) != hipSuccess ||
            hipStreamWaitEvent(b->side, b->ev_fork, 0) != hipSuccess)
            return NNC_E_HIP;
        launch_query_d<2>(b, a, init, b->side);
        launch_query_d<3>(b, a, init, b->stream);
        if (hipEventRecord(b->ev_join, b->side) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev_join, 0) != hipSuccess)
            return NNC_E_HIP;
        return nnc::check();
    }
    if (b->has_d[0]) launch_query_d<2>(b, a, init, b->stream);
    if (b->has_d[1]) launch_query_d<3>(b, a, init, b->stream);
    return nnc::check();
}

// One dimension's part of a step on stream st: ingest (and the per-point budget) of
// tiles [t0, t0 + nt), filter and grid builds of the scenes dscene[s0, s0 + ns), and
// the query launch of dimension D (none when D is 0: the caller runs the queries).
template <int D>
void launch_chain(const nnc_batch *b, const nnc::BatchArgs &a, hipStream_t st, int t0, int nt, int s0, int ns,
                  int dmask)
{
    if (nt > 0) {
        hipLaunchKernelGGL(nnc::k_b_ingest, dim3(nt), dim3(nnc::kB), 0, st, a, t0);
        if (b->budget) hipLaunchKernelGGL(nnc::k_b_budget, dim3(nt), dim3(nnc::kB), 0, st, a, t0);
    }
    hipLaunchKernelGGL(nnc::k_b_filter, dim3(ns), dim3(nnc::kFB), 0, st, a, s0);
    hipLaunchKernelGGL(nnc::k_b_grid, dim3(ns + 1), dim3(nnc::kFB), 0, st, a, s0, ns, dmask);
    if constexpr (D != 0) launch_query_d<D>(b, a, 0, st);
}

// A step up to its queries.  With scenes of both dimensions each dimension's kernels
// form a chain of their own (the plane's on the second stream, forked from the
// batch's stream and joined back), so the two overlap: one dimension's queries run
// while the other's grids are still built.
int launch_chains(const nnc_batch *b, const nnc::BatchArgs &a)
{
    const int S = b->S, S2 = b->S2, T = b->ntiles, T2 = b->T2;
    if (b->has_d[0] && b->has_d[1] && b->side) {
        if (hipEventRecord(b->ev_fork, b->stream) != hipSuccess ||
            hipStreamWaitEvent(b->side, b->ev_fork, 0) != hipSuccess)
            return NNC_E_HIP;
        launch_chain<2>(b, a, b->side, 0, T2, 0, S2, 1);
        launch_chain<3>(b, a, b->stream, T2, T - T2, S2, S - S2, 2);
        if (hipEventRecord(b->ev_join, b->side) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev_join, 0) != hipSuccess)
            return NNC_E_HIP;
        return nnc::check();
    }
    launch_chain<0>(b, a, b->stream, 0, T, 0, S, 3);
    const int rc = nnc::check();
    return rc == NNC_OK ? launch_query_b(b, a, 0) : rc;
}

}  // namespace

extern "C" {

int nnc_batch_create(nnc_batch **out, const nnc_batch_config *cfg)
{
    if (!out || !cfg || cfg->scenes <= 0 || !cfg->n || !cfg->d) return NNC_E_INVAL;
    *out = nullptr;
    nnc_batch *b = new (std::nothrow) nnc_batch();
    if (!b) return NNC_E_NOMEM;
    b->S = cfg->scenes;
    b->lanes = cfg->lanes == 1 || cfg->lanes == 4 || cfg->lanes == 8 || cfg->lanes == 16 || cfg->lanes == 32 ||
                       cfg->lanes == 64
                   ? cfg->lanes
                   : 0;
    // a plane block has three rows, a cube block nine: groups of 4 serve the plane only
    // (narrow groups keep more queries in flight per wave; measured faster: the default
    // 4 in the plane and 8 in the cube)
    b->lanes2 = b->lanes == 0 ? 4 : b->lanes;
    b->lanes3 = b->lanes == 0 ? 8 : b->lanes == 4 ? 16 : b->lanes;
    b->features_on = (cfg->flags & NNC_BATCH_FEATURES) != 0;
    b->eager = (cfg->flags & NNC_BATCH_EAGER) != 0;
    b->budget = (cfg->flags & NNC_BATCH_BUDGET) != 0;
    b->guard = cfg->guard < 0.0 ? 0x1p-18 : cfg->guard;
    b->K = 1.0 / (4.0 + 4.0 * b->guard);
    b->stream = (hipStream_t)cfg->stream;
    // a batch's scenes are small: rebuilding a loose grid is cheap next to the wider
    // search margins of a stale one (measured: 0.125 cell widths beats 0.25 and 0.03)
    const double refresh = cfg->refresh > 0.0 ? cfg->refresh : 0.125;
    long long P = 0, Q = 0, NC = 0, NS = 0;
    b->desc.resize(b->S);
    b->point_off.resize(b->S + 1);
    b->coord_off.resize(b->S + 1);
    for (int s = 0; s < b->S; ++s) {
        const int64_t n = cfg->n[s];
        const int d = cfg->d[s];
        if ((d != 2 && d != 3) || n < 0 || n > NNC_BATCH_MAX_N) {
            delete b;
            return NNC_E_INVAL;
        }
        const int G = cfg->grid_g && cfg->grid_g[s] > 0 ? cfg->grid_g[s] : default_grid_b(n, d);
        const double cells = pow((double)G, (double)d);
        if (cells > (double)(1 << 22)) {
            delete b;
            return NNC_E_INVAL;
        }
        b->has_d[d - 2] = 1;
        nnc::SceneDesc &sd = b->desc[s];
        sd.n = (int)n;
        sd.d = d;
        sd.G = G;
        sd.ncell = (int)cells;
        sd.poff = P;
        sd.coff = Q;
        sd.goff = NC;
        sd.soff = NS;
        sd.refresh_w = refresh / (double)G;
        b->point_off[s] = P;
        b->coord_off[s] = Q;
        P += n;
        Q += n * d;
        NC += (sd.ncell + 3) & ~3;      // cell regions start on 16-byte boundaries
        NS += (sd.ncell + 1 + 3) & ~3;
        for (int64_t i0 = 0; i0 < n; i0 += nnc::kTile) {
            b->tile_scene.push_back(s);
            b->tile_start.push_back((int)i0);
        }
    }
    if (P >= (1ll << 31) || Q >= (1ll << 31) || NS >= (1ll << 31)) {
        delete b;
        return NNC_E_INVAL;
    }
    b->point_off[b->S] = P;
    b->coord_off[b->S] = Q;
    b->P = P;
    b->Q = Q;
    b->NC = NC;
    b->NS = NS;
    for (int s = 0; s < b->S; ++s)
        if (b->desc[s].d == 2) b->dscene.push_back(s);
    b->S2 = (int)b->dscene.size();
    for (int s = 0; s < b->S; ++s)
        if (b->desc[s].d == 3) b->dscene.push_back(s);
    // the ingest tiles in the same order: the plane's scenes' tiles first
    b->tile_scene.clear();
    b->tile_start.clear();
    for (int k = 0; k < b->S; ++k) {
        const int s = b->dscene[k];
        if (k == b->S2) b->T2 = (int)b->tile_scene.size();
        for (int64_t i0 = 0; i0 < cfg->n[s]; i0 += nnc::kTile) {
            b->tile_scene.push_back(s);
            b->tile_start.push_back((int)i0);
        }
    }
    if (b->S2 == b->S) b->T2 = (int)b->tile_scene.size();
    b->ntiles = (int)b->tile_scene.size();
    const size_t S = (size_t)b->S, Pp = (size_t)(P > 0 ? P : 1);
    const size_t T = (size_t)(b->ntiles > 0 ? b->ntiles : 1);
    size_t bytes = 0;
    bytes += al(S * sizeof(nnc::SceneDesc)) + al(S * sizeof(nnc::DevScalars));
    bytes += al(Pp * 16);                                      // slot records
    bytes += 3 * al(Pp * 4);                                   // cell, rank, nn
    bytes += 2 * al(Pp * 4) + al(Pp * 8) + al(Pp);             // d1, d2, e, fail
    bytes += 4 * al(Pp * 4);                                   // stamp, frontier, touched x2
    bytes += 4 * al((size_t)NC * 4) + al((size_t)NS * 4);      // counts, cursor, hist x2, cell_start
    bytes += 2 * al(T * 4) + 4 * al(S * 4) + al(2 * (S + 1) * 4);  // tiles, strategy/need/qcount/dscene, qpre
    bytes += al(S * NNC_FEATURES * 4) + al(NNC_SELECTOR_PARAMS * 4) + al(4 * 4) + al(S * 3 * 8);
    if (b->budget) bytes += al(Pp * 8) + al((size_t)NC * 4);   // certificate clocks, cell stamps
    bytes += al(S * sizeof(nnc::kc::QueryArgs));               // per-scene query views
    if (hipMalloc(&b->arena, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return NNC_E_NOMEM;
    }
    if (hipMemsetAsync(b->arena, 0, bytes, b->stream) != hipSuccess) {
        (void)hipFree(b->arena);
        delete b;
        return NNC_E_HIP;
    }
    char *p = (char *)b->arena;
    auto take = [&](size_t n) {
        char *r = p;
        p += al(n);
        return r;
    };
    nnc::BatchArgs &a = b->a;
    memset(&a, 0, sizeof(a));
    a.desc = (const nnc::SceneDesc *)take(S * sizeof(nnc::SceneDesc));
    a.sc = (nnc::DevScalars *)take(S * sizeof(nnc::DevScalars));
    a.slots = (float4 *)take(Pp * 16);
    a.cell = (int *)take(Pp * 4);
    a.rank = (int *)take(Pp * 4);
    a.nn = (int *)take(Pp * 4);
    a.d1 = (float *)take(Pp * 4);
    a.d2 = (float *)take(Pp * 4);
    a.e = (double *)take(Pp * 8);
    a.fail = (uint8_t *)take(Pp);
    a.stamp = (int *)take(Pp * 4);
    a.frontier = (int *)take(Pp * 4);
    a.touched_fail = (int *)take(Pp * 4);
    a.touched_cand = (int *)take(Pp * 4);
    a.counts = (int *)take((size_t)NC * 4);
    a.cursor = (int *)take((size_t)NC * 4);
    a.hist_fail = (int *)take((size_t)NC * 4);
    a.hist_cand = (int *)take((size_t)NC * 4);
    a.cell_start = (int *)take((size_t)NS * 4);
    a.tile_scene = (const int *)take(T * 4);
    a.tile_start = (const int *)take(T * 4);
    a.strategy = (int *)take(S * 4);
    a.need_grid = (int *)take(S * 4);
    a.qcount = (int *)take(S * 4);
    a.qpre = (int *)take(2 * (S + 1) * 4);
    a.dscene = (const int *)take(S * 4);
    a.features = (float *)take(S * NNC_FEATURES * 4);
    a.params = (const float *)take(NNC_SELECTOR_PARAMS * 4);
    a.tdev = (int *)take(4 * 4);
    unsigned long long *cost = (unsigned long long *)take(S * 3 * 8);
    if (b->budget) {
        a.Si = (double *)take(Pp * 8);
        a.last_move = (int *)take((size_t)NC * 4);
    }
    a.qs = (const nnc::kc::QueryArgs *)take(S * sizeof(nnc::kc::QueryArgs));
    a.cost = (cfg->flags & NNC_BATCH_TIMING) ? cost : nullptr;
    a.scenes = b->S;
    b->arena_bytes = bytes;
    b->tick_us = 0.01;
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            b->tick_us = 1e3 / (double)khz;
    }
    a.guard = b->guard;
    a.K = b->K;
    // the fixed part of every scene's query view (scenes of a batch live in the unit box)
    std::vector<nnc::kc::QueryArgs> qv(S);
    for (size_t s = 0; s < S; ++s) {
        const nnc::SceneDesc &sd = b->desc[s];
        nnc::kc::QueryArgs &q = qv[s];
        memset(&q, 0, sizeof(q));
        q.slots = a.slots + sd.poff;
        q.cell_start = a.cell_start + sd.soff;
        q.cell = a.cell + sd.poff;
        q.list = a.frontier + sd.poff;
        q.n = sd.n;
        q.G = sd.G;
        q.nn = a.nn + sd.poff;
        q.stamp = a.stamp + sd.poff;
        q.hist = a.hist_fail + sd.goff;
        q.touched = a.touched_fail + sd.poff;
        q.d1 = a.d1 + sd.poff;
        q.d2 = a.d2 + sd.poff;
        q.e = a.e + sd.poff;
        q.Si = a.Si ? a.Si + sd.poff : nullptr;
        q.fail = a.fail + sd.poff;
        q.sc = a.sc + s;
        q.guard = a.guard;
        q.K = a.K;
        for (int k = 0; k < 3; ++k) {
            q.box.lo[k] = 0.0f;
            q.box.s[k] = (float)sd.G;
            q.box.w[k] = 1.0 / (double)sd.G;
        }
        q.fuzz = nnc::kc::kFuzz;
    }
    int rc = NNC_OK;
    if (hipMemcpyAsync((void *)a.qs, qv.data(), S * sizeof(nnc::kc::QueryArgs), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync((void *)a.desc, b->desc.data(), S * sizeof(nnc::SceneDesc), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync((void *)a.dscene, b->dscene.data(), S * 4, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        (b->ntiles > 0 &&
         (hipMemcpyAsync((void *)a.tile_scene, b->tile_scene.data(), b->ntiles * 4, hipMemcpyHostToDevice,
                         b->stream) != hipSuccess ||
          hipMemcpyAsync((void *)a.tile_start, b->tile_start.data(), b->ntiles * 4, hipMemcpyHostToDevice,
                         b->stream) != hipSuccess)))
        rc = NNC_E_HIP;
    // the learned policy's band: the network decides at every candidate fraction
    if (rc == NNC_OK) rc = nnc::launch_fill(a.tdev + 3, __builtin_bit_cast(int, 2.0f), 1, b->stream);
    if (rc == NNC_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = NNC_E_HIP;
    if (rc == NNC_OK && b->has_d[0] && b->has_d[1] &&
        (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
         hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess))
        rc = NNC_E_HIP;
    if (rc != NNC_OK) {
        if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
        if (b->ev_join) (void)hipEventDestroy(b->ev_join);
        if (b->side) (void)hipStreamDestroy(b->side);
        (void)hipFree(b->arena);
        delete b;
        return rc;
    }
    *out = b;
    return NNC_OK;
}

void nnc_batch_destroy(nnc_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    (void)hipFree(b->arena);
    delete b;
}

int nnc_batch_offsets(const nnc_batch *b, int64_t *point_off, int64_t *coord_off)
{
    if (!b) return NNC_E_INVAL;
    for (int s = 0; s <= b->S; ++s) {
        if (point_off) point_off[s] = b->point_off[s];
        if (coord_off) coord_off[s] = b->coord_off[s];
    }
    return NNC_OK;
}

int nnc_batch_init(nnc_batch *b, const float *pos)
{
    if (!b || (!pos && b->P > 0)) return NNC_E_INVAL;
    nnc::BatchArgs &a = b->a;
    // clear the per-scene scalars, the step counter and the occupancy and histogram arrays
    if (hipMemsetAsync(a.sc, 0, b->S * sizeof(nnc::DevScalars), b->stream) != hipSuccess ||
        hipMemsetAsync(a.tdev, 0, 4, b->stream) != hipSuccess ||
        hipMemsetAsync(a.counts, 0, (size_t)b->NC * 4, b->stream) != hipSuccess ||
        hipMemsetAsync(a.hist_fail, 0, (size_t)b->NC * 4, b->stream) != hipSuccess ||
        hipMemsetAsync(a.hist_cand, 0, (size_t)b->NC * 4, b->stream) != hipSuccess ||
        hipMemsetAsync(a.nn, 0xff, (size_t)(b->P > 0 ? b->P : 1) * 4, b->stream) != hipSuccess ||
        (a.last_move && hipMemsetAsync(a.last_move, 0, (size_t)b->NC * 4, b->stream) != hipSuccess))
        return NNC_E_HIP;
    a.pos_cur = pos;
    a.init = 1;
    if (b->ntiles > 0) hipLaunchKernelGGL(nnc::k_b_cells_init, dim3(b->ntiles), dim3(nnc::kB), 0, b->stream, a, 0);
    hipLaunchKernelGGL(nnc::k_b_init_flags, dim3((b->S + 255) / 256), dim3(256), 0, b->stream, a);
    hipLaunchKernelGGL(nnc::k_b_grid, dim3(b->S + 1), dim3(nnc::kFB), 0, b->stream, a, 0, b->S, 3);
    int rc = nnc::check();
    if (rc == NNC_OK) rc = launch_query_b(b, a, 1);
    b->inited = rc == NNC_OK;
    return rc;
}

namespace {

// The kernels of one step, in order, on the batch's stream.
int launch_step(nnc_batch *b, const float *pos_new, int policy, float tau)
{
    nnc::BatchArgs a = b->a;
    a.pos_cur = pos_new;
    a.init = 0;
    a.policy = policy;
    a.tau = tau;
    a.features_on = b->features_on;
    int rc = launch_chains(b, a);
    if (rc == NNC_OK) {
        hipLaunchKernelGGL(nnc::k_b_entropy, dim3(b->S), dim3(nnc::kB), 0, b->stream, a);
        rc = nnc::check();
    }
    return rc;
}

// Capture the step into a graph and instantiate it (or update the existing
// executable graph in place).  Returns NNC_OK or an error; on error no graph is kept.
int capture_step(nnc_batch *b, const float *pos_new, int policy, float tau)
{
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return NNC_E_HIP;
    const int rc = launch_step(b, pos_new, policy, tau);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->stream, &graph);
    if (rc != NNC_OK || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc != NNC_OK ? rc : NNC_E_HIP;
    }
    bool ok = false;
    if (b->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        ok = hipGraphExecUpdate(b->exec, graph, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!ok) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
    }
    if (!ok) ok = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipGraphDestroy(graph);
    if (!ok) {
        (void)hipGetLastError();
        b->exec = nullptr;
        return NNC_E_HIP;
    }
    b->g_pos = pos_new;
    b->g_policy = policy;
    b->g_tau = tau;
    return NNC_OK;
}

}  // namespace

int nnc_batch_step(nnc_batch *b, const float *pos_new, int policy, float tau)
{
    if (!b || (!pos_new && b->P > 0)) return NNC_E_INVAL;
    if (!b->inited) return NNC_E_STATE;
    if (policy < NNC_POLICY_REPAIR || policy > NNC_POLICY_LEARNED) return NNC_E_INVAL;
    // a caller's own capture, the null stream, or NNC_BATCH_EAGER: launch the kernels
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (b->eager || !b->stream || hipStreamIsCapturing(b->stream, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return launch_step(b, pos_new, policy, tau);
    if (!b->exec || b->g_pos != pos_new || b->g_policy != policy || b->g_tau != tau) {
        const int rc = capture_step(b, pos_new, policy, tau);
        if (rc != NNC_OK) return rc;
    }
    return hipGraphLaunch(b->exec, b->stream) == hipSuccess ? NNC_OK : NNC_E_HIP;
}

int nnc_batch_selector_load(nnc_batch *b, const float *params)
{
    if (!b || !params) return NNC_E_INVAL;
    if (hipMemcpyAsync((void *)b->a.params, params, NNC_SELECTOR_PARAMS * 4, hipMemcpyDeviceToDevice, b->stream) !=
        hipSuccess)
        return NNC_E_HIP;
    return nnc::launch_fill(b->a.tdev + 1, 1, 1, b->stream);
}

int nnc_batch_selector_band(nnc_batch *b, float lo, float hi)
{
    if (!b || !(lo <= hi)) return NNC_E_INVAL;
    int rc = nnc::launch_fill(b->a.tdev + 2, __builtin_bit_cast(int, lo), 1, b->stream);
    if (rc == NNC_OK) rc = nnc::launch_fill(b->a.tdev + 3, __builtin_bit_cast(int, hi), 1, b->stream);
    return rc;
}

int nnc_batch_scene_stats(nnc_batch *b, nnc_scene_stats *out)
{
    if (!b || !out) return NNC_E_INVAL;
    std::vector<nnc::DevScalars> sc(b->S);
    std::vector<int> strat(b->S);
    std::vector<float> feat((size_t)b->S * NNC_FEATURES);
    std::vector<unsigned long long> cost(b->a.cost ? (size_t)b->S * 3 : 0);
    if (b->a.cost && hipMemcpyAsync(cost.data(), b->a.cost, cost.size() * 8, hipMemcpyDeviceToHost, b->stream) !=
                         hipSuccess)
        return NNC_E_HIP;
    int tdev = 0;
    if (hipMemcpyAsync(sc.data(), b->a.sc, b->S * sizeof(nnc::DevScalars), hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(&tdev, b->a.tdev, 4, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipMemcpyAsync(strat.data(), b->a.strategy, b->S * 4, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipMemcpyAsync(feat.data(), b->a.features, feat.size() * 4, hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return NNC_E_HIP;
    int rc = NNC_OK;
    for (int s = 0; s < b->S; ++s) {
        const nnc::DevScalars &h = sc[s];
        nnc_scene_stats &o = out[s];
        o.eps = h.eps;
        o.S = h.S[tdev & 1];
        o.H_fail = h.H[0];
        o.H_cand = h.H[1];
        o.n_cand = h.F[1];
        o.n_fail = h.F[0];
        o.m_cand = h.m[1];
        o.C = h.C;
        o.strategy = strat[s];
        o.err = h.err == 0u ? NNC_OK
                : (h.err & nnc::kErrNonFinite) ? NNC_E_NONFINITE
                : (h.err & nnc::kErrEps)       ? NNC_E_EPS
                                               : NNC_E_DEVICE;
        if (o.err != NNC_OK && rc == NNC_OK) rc = o.err;
        for (int k = 0; k < NNC_FEATURES; ++k) o.features[k] = feat[(size_t)s * NNC_FEATURES + k];
        o.t_filter_us = cost.empty() ? -1.0 : (double)cost[3 * (size_t)s] * b->tick_us;
        o.t_grid_us = cost.empty() ? -1.0 : (double)cost[3 * (size_t)s + 1] * b->tick_us;
        o.t_query_us = cost.empty() ? -1.0 : (double)cost[3 * (size_t)s + 2] * b->tick_us;
    }
    return rc;
}

struct nnc_batch_snap {
    size_t bytes;
    void *dev;
};

int nnc_batch_snapshot(nnc_batch *b, nnc_batch_snap **out)
{
    if (!b || !out) return NNC_E_INVAL;
    *out = nullptr;
    nnc_batch_snap *sn = new (std::nothrow) nnc_batch_snap();
    if (!sn) return NNC_E_NOMEM;
    sn->bytes = b->arena_bytes;
    if (hipMalloc(&sn->dev, sn->bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete sn;
        return NNC_E_NOMEM;
    }
    if (hipMemcpyAsync(sn->dev, b->arena, sn->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess) {
        (void)hipFree(sn->dev);
        delete sn;
        return NNC_E_HIP;
    }
    *out = sn;
    return NNC_OK;
}

int nnc_batch_snapshot_update(nnc_batch *b, nnc_batch_snap *sn)
{
    if (!b || !sn || sn->bytes != b->arena_bytes) return NNC_E_INVAL;
    return hipMemcpyAsync(sn->dev, b->arena, sn->bytes, hipMemcpyDeviceToDevice, b->stream) == hipSuccess ? NNC_OK
                                                                                                        : NNC_E_HIP;
}

int nnc_batch_restore(nnc_batch *b, const nnc_batch_snap *sn)
{
    if (!b || !sn || sn->bytes != b->arena_bytes) return NNC_E_INVAL;
    return hipMemcpyAsync(b->arena, sn->dev, sn->bytes, hipMemcpyDeviceToDevice, b->stream) == hipSuccess ? NNC_OK
                                                                                                        : NNC_E_HIP;
}

void nnc_batch_snap_free(nnc_batch_snap *sn)
{
    if (!sn) return;
    (void)hipFree(sn->dev);
    delete sn;
}

int nnc_batch_get_state(nnc_batch *b, nnc_state *v)
{
    if (!b || !v) return NNC_E_INVAL;
    v->nn = b->a.nn;
    v->d1 = b->a.d1;
    v->d2 = b->a.d2;
    v->e = b->a.e;
    v->cell = b->a.cell;
    v->fail = b->a.fail;
    v->n = b->P;
    v->d = 0;
    v->grid_g = 0;
    v->rho = nullptr;
    v->Si = nullptr;
    return NNC_OK;
}

}  // extern "C"
