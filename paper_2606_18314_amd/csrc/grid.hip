// Single-scene kernels of the maintenance step (Algorithm 1 with the appendix's
// clock) and of the O(N) grid rebuild, for gfx950.
//
//   k_ingest       per point: squared displacement, new cell id, occupancy
//                  counts, the point's current coordinates written to its grid
//                  slot; per workgroup one maximum and one occupied-cell change
//                  into one of 64 spread slots (folded by the filter).
//   k_filter*      clock advance and safety filter S_t >= e_i with an
//                  order-preserving compaction into an ascending candidate
//                  list (wave ballot + mbcnt, a per-tile scan in LDS): one
//                  workgroup for N <= 4096, a decoupled look-back across tiles
//                  up to 2^19 points, above that reduce-then-scan (counts per
//                  tile, one scan, ordered writes).
//   k_scan_cells   exclusive scan of the occupancy counts -> cell-start table.
//   k_scatter      counting-sort scatter: rank (point -> slot) and the slot
//                  records {x, y, z, point index}, in point order (the first
//                  build); k_scatter_slots the same from the previous slot
//                  order (every later build: runs of equal cells share one
//                  atomic and write in sequence), then k_copy4 copies back.
//   k_query        exact 2-NN of each query through the grid, one group of L
//                  lanes per query: the 3^d block's rows are spread over the
//                  lanes (contiguous slots, coalesced loads; with a previous
//                  certificate only the cells within its cut-off first),
//                  partial top-2s are merged by a butterfly, and the search
//                  widens ring by ring until the second neighbour is provably
//                  enclosed (Corollary 1); then the new certificate, expiry
//                  key, failure flag and failure histogram.
//   k_query_tiled  all-point query of large scenes: cell patches with their
//   k_finish_all   neighbourhood staged in LDS, point-order records, then the
//                  certificates.
//   k_entropy*     normalised entropy (Definition 2) from a scan of the cell
//                  histogram (one workgroup, or partial sums for large grids);
//   k_cand_hist    the candidates' histogram for the same.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "kernels_common.hpp"

namespace nnc {

namespace {

using namespace kc;

constexpr int kB = 256;            // threads per point-parallel workgroup
constexpr int kScanV = 16;              // consecutive cells per thread in the cell scan
constexpr int kScanTile = kB * kScanV;  // cells per cell-scan look-back tile
// filter look-back tiles: 512 items up to kFiltSmallTilesN points, 1024 above
// (measured: shorter tiles win at small N, longer chains lose as N grows; from
// kReduceScanMinN on the filter is reduce-then-scan)
constexpr int kFiltRowsSmall = 2, kFiltRowsLarge = 4;
constexpr long long kFiltSmallTilesN = 65536;
constexpr int kSmallB = 1024;      // one-workgroup filter: threads
constexpr int kSmallRows = 32;     // one-workgroup filter: items per thread (n <= 32768)
constexpr int kSmallMaxN = 4096;       // scenes up to this size use the one-workgroup filter
constexpr long long kReduceScanMinN = 1 << 19;  // above this, the reduce-then-scan filter
constexpr int kFlagA = 1, kFlagP = 2;
constexpr unsigned kSpinLimit = 1u << 24;
// automatic choice of the all-point query: tiled from these sizes on.  A rebuild's
// pointwise queries take the cut-off from the previous certificates, which keeps
// them ahead of the tiled pass up to 2^17 points in the plane and 2^19 in the cube
// (measured); initialisation has no certificates and tiles from 2^16.
constexpr long long kTiledMinN = 65536;
constexpr long long kTiledMinNRebuild2 = 1 << 17, kTiledMinNRebuild3 = 1 << 19;
// repairs go to the cell-tiled query of the marked candidates only under
// NNC_QUERY_TILED: measured at N = 2^20 in the plane it beats the pointwise repair
// only above about 40 % candidates (0.125 against 0.145 ms at 50 %) and loses below
// (5 %: 0.090 against 0.026 ms; the staged neighbourhood serves a dozen candidates
// per tile), and its launches cost about 18 us when the device-side gate skips it
constexpr int kEntropyOneGroup4 = 1 << 15;  // histograms up to 2^17 cells: one-workgroup entropy
constexpr int kIngestBlocks = 4096;  // at most 64 workgroups per spread slot

__device__ __forceinline__ unsigned long long pack_status(unsigned epoch, int flag, unsigned v)
{
    return ((unsigned long long)(epoch & 0x3fffffffu) << 34) | ((unsigned long long)flag << 32) | v;
}

// Decoupled look-back, run by all 64 lanes of wave 0: publish this tile's
// aggregate, then inspect the 64 nearest predecessors at once; if a
// predecessor nearer than the nearest inclusive prefix is not ready yet, wait
// and re-read, else add the aggregates up to (and including) that prefix and
// stop, or move 64 tiles further back.  Tickets are taken in launch order, so
// every predecessor is running or done; the wait is bounded all the same.
__device__ unsigned lookback(unsigned long long *status, int tile, unsigned agg, unsigned epoch, unsigned *err)
{
    const int lane = (int)lane_id();
    const unsigned ep = epoch & 0x3fffffffu;
    if (tile == 0) {
        if (lane == 0) st_agent(&status[0], pack_status(epoch, kFlagP, agg));
        return 0u;
    }
    if (lane == 0) st_agent(&status[tile], pack_status(epoch, kFlagA, agg));
    unsigned excl = 0;
    int base = tile - 1;
    unsigned spins = 0;
    for (;;) {
        const int p = base - lane;
        unsigned long long v = 0;
        int flag = kFlagP;  // before tile 0: an empty inclusive prefix
        if (p >= 0) {
            v = ld_agent(&status[p]);
            flag = (unsigned)(v >> 34) == ep ? (int)((v >> 32) & 3u) : 0;
        }
        const unsigned long long pm = __ballot(flag == kFlagP);
        const unsigned long long xm = __ballot(flag == 0);
        const int firstP = pm ? __ffsll((long long)pm) - 1 : 64;
        const int firstX = xm ? __ffsll((long long)xm) - 1 : 64;
        if (firstX < firstP) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(err, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const unsigned mine = (lane <= firstP && p >= 0) ? (unsigned)v : 0u;
        excl += (unsigned)wave_sum((int)mine);
        if (firstP < 64) break;
        base -= 64;
    }
    if (lane == 0) st_agent(&status[tile], pack_status(epoch, kFlagP, excl + agg));
    return excl;
}

// Ticket and epoch for a look-back scan.  The holder of the last ticket
// retires both: by the time its look-back ends every tile has published at
// least its aggregate, so every tile has read the epoch.
__device__ __forceinline__ void take_ticket(DevSync *sy, int *s_tile, unsigned *s_epoch)
{
    if (threadIdx.x == 0) {
        *s_tile = (int)atomicAdd(&sy->tile_ctr, 1u);
        *s_epoch = __hip_atomic_load(&sy->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

__device__ __forceinline__ void retire_ticket(DevSync *sy, unsigned epoch)
{
    sy->tile_ctr = 0u;
    __hip_atomic_store(&sy->epoch, epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fill(int *p, int value, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void __launch_bounds__(kB) k_copy4(const float4 *__restrict__ src, float4 *__restrict__ dst, int n)
{
    for (int k = blockIdx.x * kB + (int)threadIdx.x; k < n; k += gridDim.x * kB) dst[k] = src[k];
}

template <int D>
__global__ void __launch_bounds__(kB) k_cells_init(const float *__restrict__ pos, int n, int G, Box box,
                                                   int *__restrict__ cell, int *__restrict__ counts,
                                                   DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    int dC = 0;
    if (i < n) {
        const float x = pos[i], y = pos[(size_t)n + i], z = D == 3 ? pos[2 * (size_t)n + i] : 0.f;
        int c = 0;
        if (all_finite<D>(x, y, z))
            c = cell_id<D>(x, y, z, G, box);
        else
            atomicOr(&sc->err, kErrNonFinite);
        cell[i] = c;
        dC = atomicAdd(&counts[c], 1) == 0;
    }
    publish_ingest_spread<kB>(sc, 0, 0.0f, dC);  // C is folded by the first filter
}

template <int D>
__global__ void __launch_bounds__(kB) k_ingest(const float *__restrict__ pold, const float *__restrict__ pnew,
                                               int n, int G, Box box, int *__restrict__ cell, int *__restrict__ counts,
                                               const int *__restrict__ rank, float4 *__restrict__ slots,
                                               DevScalars *sc, int parity, int *__restrict__ last_move, int t)
{
    // grid-stride over at most kIngestBlocks workgroups, each adding its maximum and
    // cell-count change into one of the spread slots; with last_move (the per-point
    // budget), the cells a moving point leaves and enters are stamped with step t
    float s = 0.0f;
    int dC = 0;
    const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
    // U points per thread per pass, their loads issued together (large scenes run
    // many passes; one point per pass waits for each point's loads in turn)
    constexpr int U = 4;
    const int stride = gridDim.x * kB;
    for (int i0 = blockIdx.x * kB + (int)threadIdx.x; i0 < n; i0 += U * stride) {
        float x0[U], y0[U], z0[U], x1[U], y1[U], z1[U];
        int rk[U], oc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * stride;
            const bool in = i < n;
            x0[u] = in ? pold[i] : 0.f;
            y0[u] = in ? pold[n1 + i] : 0.f;
            z0[u] = in && D == 3 ? pold[n2 + i] : 0.f;
            x1[u] = in ? pnew[i] : 0.f;
            y1[u] = in ? pnew[n1 + i] : 0.f;
            z1[u] = in && D == 3 ? pnew[n2 + i] : 0.f;
            rk[u] = in ? rank[i] : 0;
            oc[u] = in ? cell[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * stride;
            if (i >= n) continue;
            slots[rk[u]] = make_float4(x1[u], y1[u], z1[u], __int_as_float(i));
            if (all_finite<D>(x1[u], y1[u], z1[u]) && all_finite<D>(x0[u], y0[u], z0[u])) {
                s = fmaxf(s, sqdist<D>(x0[u], y0[u], z0[u], x1[u], y1[u], z1[u]));
                const int c = cell_id<D>(x1[u], y1[u], z1[u], G, box);
                const int old = oc[u];
                if (c != old) {
                    cell[i] = c;
                    dC -= atomicSub(&counts[old], 1) == 1;
                    dC += atomicAdd(&counts[c], 1) == 0;
                }
                if (last_move && (x1[u] != x0[u] || y1[u] != y0[u] || z1[u] != z0[u])) {
                    last_move[old] = t;  // every writer stores the same value
                    last_move[c] = t;
                }
            } else {
                atomicOr(&sc->err, kErrNonFinite);
            }
        }
    }
    publish_ingest_spread<kB>(sc, parity, s, dC);
}

template <int kFiltRows>
__global__ void __launch_bounds__(kB) k_filter(const double *__restrict__ e, int n, DevScalars *sc, DevSync *sy,
                                               int parity, float eps_decl, int *__restrict__ frontier,
                                               uint8_t *__restrict__ fail, unsigned long long *status)
{
    __shared__ int s_tile;
    __shared__ unsigned s_epoch;
    __shared__ int s_cnt[kFiltRows][kB / 64];
    __shared__ unsigned s_base;
    take_ticket(sy, &s_tile, &s_epoch);
    const int tile = s_tile;
    const double St = advance_clock(sc, parity, eps_decl, tile == 0 && threadIdx.x < 64);
    const int w = threadIdx.x >> 6;
    const unsigned lane = lane_id();
    constexpr int kFiltTile = kB * kFiltRows;
    const long long base = (long long)tile * kFiltTile;
    unsigned long long masks[kFiltRows];
#pragma unroll
    for (int k = 0; k < kFiltRows; ++k) {
        const long long i = base + (long long)k * kB + threadIdx.x;
        bool cand = false;
        if (i < n) {
            cand = St >= e[i];
            fail[i] = 0;
        }
        masks[k] = __ballot(cand);
        if (lane == 0) s_cnt[k][w] = __popcll(masks[k]);
    }
    __syncthreads();
    __shared__ int s_run;
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < kFiltRows; ++k)
            for (int v = 0; v < kB / 64; ++v) {
                const int c = s_cnt[k][v];
                s_cnt[k][v] = run;
                run += c;
            }
        s_run = run;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int run = s_run;
        const unsigned excl = lookback(status, tile, (unsigned)run, s_epoch, &sc->err);
        if (threadIdx.x == 0) {
            s_base = excl;
            if (tile == (int)gridDim.x - 1) {
                sc->nfront = (int)(excl + (unsigned)run);
                retire_ticket(sy, s_epoch);
            }
        }
    }
    __syncthreads();
    const unsigned b = s_base;
#pragma unroll
    for (int k = 0; k < kFiltRows; ++k) {
        if ((masks[k] >> lane) & 1ull) {
            const long long i = base + (long long)k * kB + threadIdx.x;
            const unsigned at = b + s_cnt[k][w] + rank_below(masks[k]);
            if (at < (unsigned)n)
                frontier[at] = (int)i;
            else
                atomicOr(&sc->err, kErrOverflow);
        }
    }
}

// One workgroup filters and compacts all n <= kSmallB * kSmallRows points: no
// inter-workgroup communication at all.
__global__ void __launch_bounds__(kSmallB) k_filter_small(const double *__restrict__ e, int n, DevScalars *sc,
                                                          int parity, float eps_decl, int *__restrict__ frontier,
                                                          uint8_t *__restrict__ fail)
{
    constexpr int NW = kSmallB / 64;
    constexpr int NC = kSmallRows * NW;                 // (row, wave) counts, index order
    constexpr int PER = (NC + kSmallB - 1) / kSmallB;   // counts scanned per thread
    __shared__ int s_cnt[NC];
    __shared__ int s_w[NW];
    const double St = advance_clock(sc, parity, eps_decl, threadIdx.x < 64);
    const int w = threadIdx.x >> 6;
    const unsigned lane = lane_id();
    // all loads first, so that they are in flight together
    double ev[kSmallRows];
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) {
        const int i = k * kSmallB + threadIdx.x;
        ev[k] = i < n ? e[i] : __builtin_inf();
    }
    unsigned long long masks[kSmallRows];
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) {
        const int i = k * kSmallB + threadIdx.x;
        if (i < n) fail[i] = 0;
        masks[k] = __ballot(St >= ev[k]);
        if (lane == 0) s_cnt[k * NW + w] = __popcll(masks[k]);
    }
    __syncthreads();
    int v[PER];
    int loc = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x * PER + u;
        v[u] = idx < NC ? s_cnt[idx] : 0;
        loc += v[u];
    }
    int tot;
    int ex = block_excl_scan<kSmallB>(loc, s_w, tot);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x * PER + u;
        if (idx < NC) s_cnt[idx] = ex;
        ex += v[u];
    }
    __syncthreads();
    if (threadIdx.x == 0) sc->nfront = tot;
#pragma unroll
    for (int k = 0; k < kSmallRows; ++k) {
        if ((masks[k] >> lane) & 1ull) {
            const int i = k * kSmallB + threadIdx.x;
            const int at = s_cnt[k * NW + w] + rank_below(masks[k]);
            if (at < n)
                frontier[at] = i;
            else
                atomicOr(&sc->err, kErrOverflow);
        }
    }
}

// Reduce-then-scan filter for large N (no chain between tiles): k_filter_count
// advances the clock, stores each tile's candidate ballots (one bit per point)
// (each wave's as one contiguous run) and counts them, k_filter_offsets scans
// the counts in one workgroup,
// k_filter_write reads the ballots back (not the keys) and writes each tile's
// candidates at its offset, in index order.  The fail flags are cleared over the
// previous step's candidates (the only ones its repair could set) when that list
// is short, else all of them, as after a rebuild, a caller's list or a restore.
constexpr int kFRows = 16;                // items per thread in the counting tiles
constexpr int kFTile = kB * kFRows;       // 4096 items per tile
constexpr int kFMasks = kFRows * (kB / 64);  // ballot words per tile

__global__ void __launch_bounds__(kB) k_filter_count(const double *__restrict__ e, int n, DevScalars *sc, int parity,
                                                     float eps_decl, uint8_t *__restrict__ fail,
                                                     int *__restrict__ tcount, unsigned long long *__restrict__ fmask,
                                                     int clear_all, const int *__restrict__ prev_list)
{
    __shared__ int s_w[kB / 64];
    const long long base = (long long)blockIdx.x * kFTile;
    // the tile's keys are requested before the clock's dependent loads and stores
    double ev[kFRows];
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        const long long i = base + (long long)k * kB + threadIdx.x;
        ev[k] = i < n ? e[i] : __builtin_inf();
    }
    const double St = advance_clock(sc, parity, eps_decl, blockIdx.x == 0 && threadIdx.x < 64);
    const int w = (int)(threadIdx.x >> 6);
    const int lane = (int)lane_id();
    int c = 0;  // wave-uniform
    // a list longer than n / 64 costs more in scattered byte stores (a cache line
    // each) than streaming zeros over all n flags
    const int prev = min(sc->nfront, n);  // the count is rewritten only by the next kernel
    clear_all = clear_all || (long long)prev * 64 > (long long)n;
    if (!clear_all) {
        for (int q = blockIdx.x * kB + (int)threadIdx.x; q < prev; q += gridDim.x * kB) {
            const int i = prev_list[q];
            if (i >= 0 && i < n) fail[i] = 0;
        }
    }
    // the wave's kFRows ballots, lane k holding row k's, stored as one contiguous run
    unsigned long long mine = 0;
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        const long long i = base + (long long)k * kB + threadIdx.x;
        const unsigned long long m = __ballot(i < n && St >= ev[k]);
        c += __popcll(m);
        if (lane == k) mine = m;
    }
    if (lane < kFRows) fmask[(long long)blockIdx.x * kFMasks + w * kFRows + lane] = mine;
    if (clear_all) {
        // the tile's flags as 16-byte stores (fail is 256-byte aligned; a partial last tile
        // clears byte by byte)
        static_assert(kFTile % (16 * kB) == 0, "whole 16-byte stores per tile");
#pragma unroll
        for (int u = 0; u < kFTile / (16 * kB); ++u) {
            const long long f0 = base + 16ll * (u * kB + (int)threadIdx.x);
            if (f0 + 16 <= n)
                *reinterpret_cast<uint4 *>(fail + f0) = make_uint4(0u, 0u, 0u, 0u);
            else
                for (long long i = f0; i < n && i < f0 + 16; ++i) fail[i] = 0;
        }
    }
    if (lane == 0) s_w[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int v = 0; v < kB / 64; ++v) t += s_w[v];
        tcount[blockIdx.x] = t;
    }
}

// Each thread scans a contiguous run of the tile counts, four at a time (one
// workgroup scan in all; tcount is 256-byte aligned and holds at least
// tiles rounded up to four, with a zero beyond the last tile, see the sizing).
__global__ void __launch_bounds__(1024) k_filter_offsets(int *__restrict__ tcount, int tiles, DevScalars *sc)
{
    __shared__ int s_w[1024 / 64];
    const int t4 = (tiles + 3) >> 2;                       // groups of four
    const int per = (t4 + 1023) / 1024;
    const int g0 = min((int)threadIdx.x * per, t4), g1 = min(g0 + per, t4);
    int4 *tc4 = reinterpret_cast<int4 *>(tcount);
    auto get = [&](int g) {
        int4 v = tc4[g];
        const int t = 4 * g;  // entries past the last tile count as zero
        if (t + 1 >= tiles) v.y = 0;
        if (t + 2 >= tiles) v.z = 0;
        if (t + 3 >= tiles) v.w = 0;
        return v;
    };
    int sum = 0;
    for (int g = g0; g < g1; ++g) {
        const int4 v = get(g);
        sum += v.x + v.y + v.z + v.w;
    }
    int tot;
    int run = block_excl_scan<1024>(sum, s_w, tot);
    for (int g = g0; g < g1; ++g) {
        const int4 v = get(g);
        int4 o;
        o.x = run;
        o.y = run + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        run = o.w + v.w;
        const int t = 4 * g;
        if (t + 3 < tiles) {
            tc4[g] = o;
        } else {
            tcount[t] = o.x;
            if (t + 1 < tiles) tcount[t + 1] = o.y;
            if (t + 2 < tiles) tcount[t + 2] = o.z;
        }
    }
    if (threadIdx.x == 0) sc->nfront = tot;
}

__global__ void __launch_bounds__(kB) k_filter_write(int n, const unsigned long long *__restrict__ fmask,
                                                     const int *__restrict__ toff, int *__restrict__ frontier,
                                                     unsigned *err)
{
    __shared__ int s_cnt[kFRows][kB / 64];
    const int w = threadIdx.x >> 6;
    const unsigned lane = lane_id();
    const long long base = (long long)blockIdx.x * kFTile;
    const int t0 = threadIdx.x < 64 ? toff[blockIdx.x] : 0;  // requested with the ballots
    // the wave's ballots: one load (lane k: row k), then broadcast
    const unsigned long long mine =
        lane < (unsigned)kFRows ? fmask[(long long)blockIdx.x * kFMasks + w * kFRows + lane] : 0ull;
    unsigned long long masks[kFRows];
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        masks[k] = __shfl(mine, k, 64);
        if (lane == 0) s_cnt[k][w] = __popcll(masks[k]);
    }
    __syncthreads();
    // the tile's (row, wave) counts in index order: one exclusive scan by the first
    // wave, each lane taking CPL consecutive counts
    constexpr int CPL = kFRows * (kB / 64) / 64;
    static_assert(CPL * 64 == kFRows * (kB / 64), "whole counts per lane");
    if (threadIdx.x < 64) {
        int *flat = &s_cnt[0][0] + CPL * threadIdx.x;
        int v[CPL], sum = 0;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            v[u] = flat[u];
            sum += v[u];
        }
        int incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off, 64);
            if ((int)lane >= off) incl += o;
        }
        int run = t0 + incl - sum;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            flat[u] = run;
            run += v[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFRows; ++k) {
        if ((masks[k] >> lane) & 1ull) {
            const long long i = base + (long long)k * kB + threadIdx.x;
            const unsigned at = (unsigned)s_cnt[k][w] + rank_below(masks[k]);
            if (at < (unsigned)n)
                frontier[at] = (int)i;
            else
                atomicOr(err, kErrOverflow);
        }
    }
}

// Each thread scans kScanV consecutive cells (16-byte loads and stores where the
// run lies inside the table; the table is 256-byte aligned), one workgroup scan
// per tile of kScanTile cells, then the look-back across tiles.
__global__ void __launch_bounds__(kB) k_scan_cells(const int *__restrict__ counts, int ncell,
                                                   int *__restrict__ cell_start, int *__restrict__ cursor,
                                                   DevScalars *sc, DevSync *sy, int parity,
                                                   unsigned long long *status)
{
    __shared__ int s_tile;
    __shared__ unsigned s_epoch;
    __shared__ int s_w[kB / 64];
    __shared__ unsigned s_base;
    take_ticket(sy, &s_tile, &s_epoch);
    const int tile = s_tile;
    const long long c0 = (long long)tile * kScanTile + (long long)threadIdx.x * kScanV;
    const bool whole = c0 + kScanV <= ncell;
    int v[kScanV];
    if (whole) {
        const int4 *p4 = reinterpret_cast<const int4 *>(counts + c0);
#pragma unroll
        for (int q = 0; q < kScanV / 4; ++q) {
            const int4 w = p4[q];
            v[4 * q] = w.x;
            v[4 * q + 1] = w.y;
            v[4 * q + 2] = w.z;
            v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanV; ++k) v[k] = c0 + k < ncell ? counts[c0 + k] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanV; ++k) {
        const int x = v[k];
        v[k] = sum;  // exclusive prefix within the thread's run
        sum += x;
    }
    int run;
    const int ex = block_excl_scan<kB>(sum, s_w, run);
    if (threadIdx.x < 64) {
        const unsigned excl = lookback(status, tile, (unsigned)run, s_epoch, &sc->err);
        if (threadIdx.x == 0) {
            s_base = excl;
            if (tile == (int)gridDim.x - 1) {
                cell_start[ncell] = (int)(excl + (unsigned)run);
                retire_ticket(sy, s_epoch);
            }
            if (tile == 0) {
                sc->S_grid = sc->S[parity];
                sc->nwide = 0;
            }
        }
    }
    __syncthreads();
    const int b = (int)s_base + ex;
    if (whole) {
        int4 *cs4 = reinterpret_cast<int4 *>(cell_start + c0);
        int4 *cu4 = reinterpret_cast<int4 *>(cursor + c0);
#pragma unroll
        for (int q = 0; q < kScanV / 4; ++q) {
            const int4 w = make_int4(b + v[4 * q], b + v[4 * q + 1], b + v[4 * q + 2], b + v[4 * q + 3]);
            cs4[q] = w;
            cu4[q] = w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanV; ++k)
            if (c0 + k < ncell) {
                cell_start[c0 + k] = b + v[k];
                cursor[c0 + k] = b + v[k];
            }
    }
}

template <int D>
__global__ void __launch_bounds__(kB) k_scatter(const float *__restrict__ pos, const int *__restrict__ cell, int n,
                                                int *__restrict__ cursor, int *__restrict__ rank,
                                                float4 *__restrict__ slots, DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const int k = atomicAdd(&cursor[cell[i]], 1);
    if (k >= n) {  // unreachable while the counts match the cells
        atomicOr(&sc->err, kErrOverflow);
        return;
    }
    rank[i] = k;
    slots[k] = make_float4(pos[i], pos[(size_t)n + i], D == 3 ? pos[2 * (size_t)n + i] : 0.0f, __int_as_float(i));
}

// Counting-sort scatter from the previous slot order (every grid build after the
// first): slot k's record already holds its point's current coordinates, and
// neighbouring slots mostly land in one new cell, so each run of equal cells over
// consecutive lanes of a wave takes its slots with one atomic (by the run's last
// lane) and writes them in sequence.  The cell is the ingest's formula on the same
// coordinates (the maintained cell id for a non-finite point).  Records go to
// `out`, to be copied back over the slots; rank[i] to the new slot.
template <int D>
__global__ void __launch_bounds__(kB) k_scatter_slots(const float4 *__restrict__ slots,
                                                      const int *__restrict__ cell, int n, int G, Box box,
                                                      int *__restrict__ cursor, int *__restrict__ rank,
                                                      float4 *__restrict__ out, DevScalars *sc)
{
    const int k = blockIdx.x * kB + threadIdx.x;
    float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int c = -1, i = 0;
    bool act = k < n;
    if (act) {
        r = slots[k];
        i = __float_as_int(r.w);
        if (i < 0 || i >= n) {  // unreachable: the slots hold a permutation of the points
            atomicOr(&sc->err, kErrOverflow);
            act = false;
        } else {
            c = all_finite<D>(r.x, r.y, r.z) ? cell_id<D>(r.x, r.y, r.z, G, box) : cell[i];
        }
    }
    // runs of equal cells: every lane finds the first (h) and last (e) lane of its run
    const int lane = (int)lane_id();
    const int cp = __shfl_up(c, 1), cn = __shfl_down(c, 1);
    int h = lane == 0 || cp != c ? lane : 0;
    int e = lane == 63 || cn != c ? lane : 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int vh = __shfl_up(h, off), ve = __shfl_down(e, off);
        if (lane >= off) h = max(h, vh);
        if (lane + off < 64) e = min(e, ve);
    }
    int base = 0;
    if (act && lane == e) base = atomicAdd(&cursor[c], e - h + 1);
    base = __shfl(base, e);
    if (!act) return;
    const int kn = base + (lane - h);
    if (kn >= n) {  // unreachable while the counts match the cells
        atomicOr(&sc->err, kErrOverflow);
        return;
    }
    out[kn] = r;
    rank[i] = kn;
}

template <int D, int L, bool UNIT>
__global__ void __launch_bounds__(kB) k_query(QueryArgs a)
{
    const int lane = threadIdx.x & (L - 1);
    constexpr int GPB = kB / L;
    int q = blockIdx.x * GPB + (int)(threadIdx.x / L);
    // the first list entry is read in the same round trip as the count (an entry
    // past the count is never used)
    const bool pre = !a.all && q < a.list_cap;
    const int i_pre = pre ? a.list[q] : 0;
    const int count = a.all ? a.n : min(*a.count_dev, a.n);
    if (a.tiled_from > 0 && count >= a.tiled_from) return;  // the tiled repair takes this list
    const double St = a.sc->S[a.parity];
    const double margin = query_margin(St, a.sc->S_grid, a.fuzz);
    for (bool first = true; q < count; q += gridDim.x * GPB, first = false)
        query_one<D, L, UNIT>(a, q, St, margin, lane, first && pre, i_pre);
}

// All-point query (rebuild and initialisation, right after a grid build), tiled
// by cells: a tile is a patch of TX x TY cells of one grid plane (fixed z); the
// (TY + 2) x 3^(d-2) neighbouring row segments are contiguous slot ranges, staged
// once in LDS, and every point of the tile's cells scans its 3^d block from LDS,
// one thread per point.  A point whose second neighbour is not enclosed by the
// first block is appended to the widening list and finished by the pointwise
// query; a tile whose neighbourhood exceeds the LDS capacity runs the pointwise
// search for its points.  Results go to a 16-byte record per point in point
// order (one scattered 16-byte store, which costs about 32 bytes of HBM traffic),
// and k_finish_all turns the records into certificates reading them in sequence
// (a scattered 16-byte read would fetch a whole 128-byte line, and six scattered
// certificate stores a line each).  Tiles are dealt to XCDs in
// contiguous ranges (workgroups go to the eight XCDs round-robin), so
// neighbouring tiles share an L2.
constexpr int kTB = 512;       // threads per tile
constexpr int kNbMax = 3072;   // neighbourhood points staged in LDS
constexpr int kTXMax = 256;    // cells per tile row
constexpr int kTYMax = 8;      // rows per tile
constexpr int kCsMax = 2304;   // cell-start entries of a tile's neighbourhood rows

__device__ __forceinline__ int xcd_tile(int b, int nt)
{
    const int x = b & 7, k = b >> 3;
    const int full = nt >> 3, rem = nt & 7;
    return x * full + min(x, rem) + k;
}

template <int D, bool UNIT>
__global__ void __launch_bounds__(kTB) k_query_tiled(QueryArgs a, int TX, int TY, int nsx, int nsy,
                                                     int *__restrict__ wide, int4 *__restrict__ rec)
{
    constexpr int RMAX = D == 3 ? 3 * (kTYMax + 2) : kTYMax + 2;
    if (a.cmask && min(*a.count_dev, a.n) < a.tiled_from) return;  // a short list: the pointwise repair
    __shared__ float4 s_p[kNbMax];  // x, y, z (0 in the plane), point index bits
    __shared__ int s_cs[kCsMax];
    __shared__ int s_lo[RMAX], s_off[RMAX + 1], s_qoff[kTYMax + 1];
    const int G = a.G;
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int sx = tile % nsx, rest = tile / nsx;
    const int sy = rest % nsy, gz = D == 3 ? rest / nsy : 0;
    const int gx0 = sx * TX, gx1 = min(gx0 + TX, G);      // the tile's cells [gx0, gx1) x [gy0, gy1)
    const int gy0 = sy * TY, gy1 = min(gy0 + TY, G);
    const int ty = gy1 - gy0, ry = ty + 2;                // neighbourhood rows per plane
    const int R = D == 3 ? 3 * ry : ry;                   // row k: y = gy0 - 1 + k % ry, z = gz - 1 + k / ry
    const int gl = max(gx0 - 1, 0), gh = min(gx1, G - 1);  // neighbourhood cells [gl, gh] of each row
    const int w1 = gh - gl + 2;                           // cell-start entries per row
    const int kbase = D == 3 ? ry : 0;                    // first row of the middle plane
    for (int idx = (int)threadIdx.x; idx < R * w1; idx += kTB) {
        const int k = idx / w1, u = idx - k * w1;
        const int y = gy0 - 1 + k % ry, z = D == 3 ? gz - 1 + k / ry : 0;
        const bool in = y >= 0 && y < G && z >= 0 && z < G;
        s_cs[idx] = in ? a.cell_start[gl + u + G * (y + G * z)] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
        for (int k = 0; k < R; ++k) {
            s_lo[k] = s_cs[k * w1];
            s_off[k] = off;
            off += s_cs[k * w1 + w1 - 1] - s_cs[k * w1];
        }
        s_off[R] = off;
        int q = 0;
        for (int j = 0; j < ty; ++j) {
            const int k = kbase + 1 + j;
            s_qoff[j] = q;
            q += s_cs[k * w1 + gx1 - gl] - s_cs[k * w1 + gx0 - gl];
        }
        s_qoff[ty] = q;
    }
    __syncthreads();
    if (a.cmask) {
        // repair of the marked candidates only: nothing to do in a tile without one
        __shared__ int s_any;
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        const int qt = s_qoff[ty];
        int j0 = 0, any = 0;
        for (int qq = (int)threadIdx.x; qq < qt; qq += kTB) {
            while (s_qoff[j0 + 1] <= qq) ++j0;
            const int kq = kbase + 1 + j0;
            const int slot = s_cs[kq * w1 + gx0 - gl] + (qq - s_qoff[j0]);  // still slot numbers here
            any |= a.cmask[slot];
        }
        if (any) s_any = 1;
        __syncthreads();
        if (!s_any) return;
    }
    const int total = s_off[R];
    const bool staged = total <= kNbMax;
    // slot of LDS entry m of row k: s_lo[k] + (m - s_off[k]); cell starts become LDS positions
    for (int idx = (int)threadIdx.x; idx < R * w1; idx += kTB) s_cs[idx] += s_off[idx / w1] - s_lo[idx / w1];
    if (staged) {
        int k = 0;
        for (int m = (int)threadIdx.x; m < total; m += kTB) {
            while (s_off[k + 1] <= m) ++k;  // m increases, so k only moves forward
            const int slot = s_lo[k] + (m - s_off[k]);
            s_p[m] = a.slots[slot];
        }
    }
    __syncthreads();
    const double St = a.sc->S[a.parity];
    const double margin = query_margin(St, a.sc->S_grid, a.fuzz);
    const int qtotal = s_qoff[ty];
    int j = 0;
    for (int qq = (int)threadIdx.x; qq < qtotal; qq += kTB) {
        while (s_qoff[j + 1] <= qq) ++j;
        const int kq = kbase + 1 + j;
        const int q = s_cs[kq * w1 + gx0 - gl] + (qq - s_qoff[j]);  // LDS position
        const int slot = s_lo[kq] + (q - s_off[kq]);
        if (a.cmask) {
            if (!a.cmask[slot]) continue;
            a.cmask[slot] = 0;
        }
        float x, y, z = 0.0f;
        int i;
        if (staged) {
            const float4 v = s_p[q];
            x = v.x;
            y = v.y;
            z = v.z;
            i = __float_as_int(v.w);
        } else {
            const float4 v = a.slots[slot];
            x = v.x;
            y = v.y;
            if constexpr (D == 3) z = v.z;
            i = __float_as_int(v.w);
        }
        Top2 t;
        t.init();
        const int cx = query_cell<UNIT>(a, x, 0), cy = query_cell<UNIT>(a, y, 1);
        const int cz = D == 3 ? query_cell<UNIT>(a, z, 2) : 0;
        bool widen = false;
        if (staged && cx >= gx0 && cx < gx1 && cy >= gy0 && cy < gy1 && cz == gz) {
            // a rebuild in the cube scans only the block cells within the cut-off
            // from the point's previous certificate (initialisation, and the plane,
            // whose blocks hold few points: the whole block; measured)
            double T = __builtin_inf(), glo[3] = {0.0, 0.0, 0.0}, ghi[3] = {0.0, 0.0, 0.0};
            if (D == 3 && !a.init) {
                T = point_cutoff(a, i, St, margin);
                cell_gaps<D, UNIT>(a, x, y, z, cx, cy, cz, glo, ghi);
            }
            const double T2 = T < __builtin_inf() ? T * T : __builtin_inf();
            bool cut = false;
            const int k0 = cy - gy0;  // row of dy = -1 in each plane
#pragma unroll
            for (int pz = 0; pz < (D == 3 ? 3 : 1); ++pz) {
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int cyy = cy + dy - 1, czz = cz + pz - 1;
                    if (cyy < 0 || cyy >= G || (D == 3 && (czz < 0 || czz >= G))) continue;  // empty rows
                    int xlo, xhi;
                    bool rc;
                    block_row<D>(glo, ghi, T2, cx, G, dy - 1, pz - 1, xlo, xhi, rc);
                    cut |= rc;
                    if (xlo > xhi) continue;
                    const int k = k0 + dy + pz * ry;
                    const int lo = s_cs[k * w1 + xlo - gl], hi = s_cs[k * w1 + xhi - gl + 1];
                    for (int m = lo; m < hi; ++m) {
                        const float4 v = s_p[m];
                        const float s = sqdist<D>(x, y, z, v.x, v.y, v.z);
                        const int jj = __float_as_int(v.w);
                        if (jj != i) t.push(s, jj);
                    }
                }
            }
            const double B = query_bound<D, UNIT>(a, x, y, z, cx, cy, cz, 1);
            const double Be = (cut ? fmin(B, T) : B) - margin;
            widen = (cut || !__builtin_isinf(B)) && !(Be > 0.0 && (double)t.s2 < Be * Be * (1.0 - kRel));
        } else {
            group_search<D, 1, UNIT>(a, x, y, z, i, margin, __builtin_inf(), 0, t);
        }
        const int at = wave_append(&a.sc->nwide, widen);
        if (widen) {
            if (at < a.n)
                wide[at] = i;
            else
                atomicOr(&a.sc->err, kErrOverflow);
            if (!a.cmask) rec[i] = make_int4(-1, 0, 0, 0);  // finished by the widening pass
        } else if (a.cmask) {
            write_certificate(a, i, t, St, a.nn[i], -1);      // a repaired candidate, in place
        } else {
            rec[i] = make_int4(t.nn, __float_as_int(t.s1), __float_as_int(t.s2), 1);
        }
    }
}

// Candidates of a repair list marked in slot order for the tiled repair (when the
// list is long enough for it); resets the widening count.
__global__ void __launch_bounds__(kB) k_cand_mask(const int *__restrict__ list, const int *__restrict__ count_dev,
                                                  int n, int tiled_from, const int *__restrict__ rank,
                                                  uint8_t *__restrict__ cmask, DevScalars *sc)
{
    const int count = min(*count_dev, n);
    if (count < tiled_from) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->nwide = 0;
    for (int q = blockIdx.x * kB + (int)threadIdx.x; q < count; q += gridDim.x * kB) {
        const int i = list[q];
        if (i >= 0 && i < n) cmask[rank[i]] = 1;
    }
}

// Point-order completion of the tiled pass: certificate of point i from its
// record (skipped if the widening pass owns the point).
__global__ void __launch_bounds__(kB) k_finish_all(QueryArgs a, const int4 *__restrict__ rec)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= a.n) return;
    const int4 r = rec[i];
    if (r.w == 0) return;
    Top2 t;
    t.nn = r.x;
    t.s1 = __int_as_float(r.y);
    t.s2 = __int_as_float(r.z);
    const double St = a.sc->S[a.parity];
    write_certificate(a, i, t, St, a.nn[i], -1);
}

// Normalised entropy (Definition 2) of the failures (which = 0) or candidates
// (which = 1): one workgroup scans the cell histogram.
__global__ void __launch_bounds__(1024) k_entropy(int which, int *__restrict__ hist, int ncell4, DevScalars *sc)
{
    HistSums r{0.0, 0.0, 0.0};
    hist_terms(hist, ncell4, (int)threadIdx.x, 1024, r);
    const HistSums t = block_sums<1024>(r);
    if (threadIdx.x == 0) entropy_publish(which, t, sc);
}

__global__ void __launch_bounds__(kB) k_cand_hist(const int *__restrict__ frontier, const int *__restrict__ cell,
                                                  int *__restrict__ hist, const DevScalars *sc)
{
    const int count = sc->nfront;
    for (int q = blockIdx.x * kB + (int)threadIdx.x; q < count; q += gridDim.x * kB)
        atomicAdd(&hist[cell[frontier[q]]], 1);
}

// The same over a large histogram: per-workgroup partial sums, then one
// workgroup adds them up and publishes.
__global__ void __launch_bounds__(kB) k_entropy_part(int *__restrict__ hist, int ncell4, double *__restrict__ part)
{
    HistSums r{0.0, 0.0, 0.0};
    hist_terms(hist, ncell4, blockIdx.x * kB + (int)threadIdx.x, (int)gridDim.x * kB, r);
    const HistSums t = block_sums<kB>(r);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = t.F;
        part[3 * blockIdx.x + 1] = t.m;
        part[3 * blockIdx.x + 2] = t.s;
    }
}

__global__ void __launch_bounds__(kB) k_entropy_final(int which, int nparts, const double *__restrict__ part,
                                                      DevScalars *sc)
{
    HistSums r{0.0, 0.0, 0.0};
    for (int k = (int)threadIdx.x; k < nparts; k += kB) {
        r.F += part[3 * k];
        r.m += part[3 * k + 1];
        r.s += part[3 * k + 2];
    }
    const HistSums t = block_sums<kB>(r);
    if (threadIdx.x == 0) entropy_publish(which, t, sc);
}

// Selector features of the pending step (after the candidate entropy kernel).
__global__ void __launch_bounds__(1024) k_features(const double *__restrict__ e, int n, int d, int ncell,
                                                   DevScalars *sc, int parity, float *__restrict__ out)
{
    __shared__ int s_vh[kVBins];
    if (threadIdx.x < kVBins) s_vh[threadIdx.x] = 0;
    __syncthreads();
    const double Sprev = sc->S[parity ^ 1];
    for (int i = threadIdx.x; i < min(n, kVSample); i += 1024) {
        const double r = e[i] - Sprev;
        if (r > 0.0 && r < __builtin_inf()) atomicAdd(&s_vh[validity_bin(r)], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float eps = (float)sc->eps;
        float f[NNC_FEATURES];
        scene_features(f, n, d, ncell, sc->nfront, sc->H[1], sc->m[1], eps, validity_median(s_vh));
        for (int k = 0; k < NNC_FEATURES; ++k) out[k] = f[k];
    }
}

// Audit of the state against an all-pairs result (a_*): misses, value
// mismatches of certificates computed at this step, failures and an
// order-independent hash of nn[] (sum of SplitMix64(i << 32 | nn_i)).
__global__ void __launch_bounds__(kB) k_audit(int n, const int *__restrict__ nn, const float *__restrict__ d1,
                                              const float *__restrict__ d2, const int *__restrict__ stamp, int t,
                                              const uint8_t *__restrict__ fail, const int *__restrict__ a_nn,
                                              const float *__restrict__ a_d1, const float *__restrict__ a_d2,
                                              const uint8_t *__restrict__ rho, DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    int missed = 0, vm = 0, tf = 0, fresh = 0, hit = 0;
    unsigned long long h = 0;
    if (i < n) {
        missed = a_nn[i] != nn[i];
        fresh = stamp[i] == t;
        vm = fresh && (__float_as_uint(a_d1[i]) != __float_as_uint(d1[i]) ||
                       __float_as_uint(a_d2[i]) != __float_as_uint(d2[i]));
        tf = fail[i] != 0;
        hit = rho != nullptr && tf && rho[i] != 0;
        h = mix64(((unsigned long long)(unsigned)i << 32) | (unsigned)nn[i]);
    }
    missed = wave_sum(missed);
    hit = wave_sum(hit);
    vm = wave_sum(vm);
    tf = wave_sum(tf);
    fresh = wave_sum(fresh);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
    if (lane_id() == 0) {
        atomicAdd(&sc->audit[0], (unsigned long long)missed);
        atomicAdd(&sc->audit[1], (unsigned long long)vm);
        atomicAdd(&sc->audit[2], (unsigned long long)tf);
        atomicAdd(&sc->audit[3], (unsigned long long)fresh);
        atomicAdd(&sc->audit[4], h);
        if (hit) atomicAdd(&sc->audit[7], (unsigned long long)hit);
    }
}

// Per-point motion budget (the Limitations section's tighter safe set; Theorem 2
// applied to the kept certificate), for each point whose key has expired:
//  1. block-local: if no cell of the point's 3^d block was stamped (a moving point
//     left or entered it) after the point's certificate, neither the point nor any
//     point that was inside the block has moved; a point from outside is at least
//     B - fuzz away (B: distance to the outside of the block) and has moved at most
//     D = S_t - S_i, so if (d2 + D)(1 + 2^-20) + fuzz < B none can have come within
//     d2: the certificate is exact, the point is no candidate, and its key becomes
//     the next binary64 value above S_t (tested again once anything moves);
//  2. distance: every point has moved at most D since the certificate (nn = j, d2),
//     so every other point is at least d2 - 2 D from i now, while j is at its
//     current distance r; if r < d2 - 2 D (with the guard g:
//     gap = (d2 (1 - g) - 2 (D (1 + g))) - r > 0) the certificate is kept and its key
//     moves to S_t + gap * K -- the gap closes by at most 4 per unit of clock;
// otherwise the point stays expired and the filter makes it a candidate.  S_t is
// computed as the filter will (from the same ingest maxima), read-only.
template <int D>
__global__ void __launch_bounds__(kB) k_budget(const float *__restrict__ pos, int n, const int *__restrict__ nn,
                                               const float *__restrict__ d2, const double *__restrict__ Si,
                                               double *__restrict__ e, const DevScalars *__restrict__ sc, int parity,
                                               double guard, double K, const int *__restrict__ cell,
                                               const int *__restrict__ stamp, const int *__restrict__ last_move,
                                               int G, Box box, double fuzz)
{
    const int lane = (int)lane_id();
    const float m = fmaxf(wave_max(__uint_as_float(sc->dmax_part[parity][lane])), __uint_as_float(sc->dmax[parity]));
    const double St = sc->S[parity ^ 1] + (double)cert_sqrt(m);
    const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
    for (int i = blockIdx.x * kB + (int)threadIdx.x; i < n; i += gridDim.x * kB) {
        const double ei = e[i];
        if (!(St >= ei)) continue;
        const int j = nn[i];
        if (j < 0 || j >= n) continue;
        const double dS = St - Si[i];
        {
            const int id = cell[i], si = stamp[i];
            const int gc[3] = {id % G, (id / G) % G, D == 3 ? id / (G * G) : 0};
            bool quiet = true;
            for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0) && quiet; ++oz) {
                const int z = gc[2] + oz;
                if (z < 0 || z >= G) continue;
                for (int oy = -1; oy <= 1 && quiet; ++oy) {
                    const int y = gc[1] + oy;
                    if (y < 0 || y >= G) continue;
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int x = gc[0] + ox;
                        if (x < 0 || x >= G) continue;
                        if (last_move[x + G * (y + G * z)] > si) {
                            quiet = false;
                            break;
                        }
                    }
                }
            }
            if (quiet) {
                double B = __builtin_inf();
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double w = box.w[k], lo = (double)box.lo[k], x = (double)pos[(size_t)k * n1 + i];
                    if (gc[k] - 1 > 0) B = fmin(B, x - (lo + (double)(gc[k] - 1) * w));
                    if (gc[k] + 1 < G - 1) B = fmin(B, (lo + (double)(gc[k] + 2) * w) - x);
                }
                const double need = ((double)d2[i] + dS) * (1.0 + 0x1p-20) + fuzz;
                if (need < B) {
                    // the next binary64 value above the clock (S_t >= 0): tested again once anything moves
                    e[i] = __longlong_as_double(__double_as_longlong(St) + 1);
                    continue;
                }
            }
        }
        const float s = sqdist<D>(pos[i], pos[n1 + i], D == 3 ? pos[n2 + i] : 0.0f, pos[j], pos[n1 + j],
                                  D == 3 ? pos[n2 + j] : 0.0f);
        const float r = cert_sqrt(s);
        const double thr = (double)d2[i] * (1.0 - guard) - 2.0 * (dS * (1.0 + guard));
        const double gap = thr - (double)r;
        if (gap > 0.0) e[i] = St + gap * K;
    }
}

// Spatial spread of a frontier (the dataset's gyration descriptor): per workgroup,
// sums over the members -- the failed points (list == nullptr: fail[i] set) or the
// listed candidates -- of (x, y, z, 1) when cen is null, else of the squared
// distance to the centroid cen; binary64.  part[4 * blockIdx + k] receives them.
template <int D>
__global__ void __launch_bounds__(kB) k_shape(const float *__restrict__ pos, int n, const uint8_t *__restrict__ fail,
                                              const int *__restrict__ list, const int *__restrict__ count,
                                              const double *__restrict__ cen, double *__restrict__ part)
{
    constexpr int NW = kB / 64;
    __shared__ double s_v[4][NW];
    const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
    const int items = list ? *count : n;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = blockIdx.x * kB + (int)threadIdx.x; q < items; q += gridDim.x * kB) {
        int i = q;
        if (list) {
            i = list[q];
            if (i < 0 || i >= n) continue;
        } else if (!fail[i]) {
            continue;
        }
        const double x = pos[i], y = pos[n1 + i], z = D == 3 ? (double)pos[n2 + i] : 0.0;
        if (!cen) {
            v[0] += x;
            v[1] += y;
            v[2] += z;
            v[3] += 1.0;
        } else {
            const double dx = x - cen[0], dy = y - cen[1], dz = z - cen[2];
            v[0] += dx * dx + dy * dy + dz * dz;
        }
    }
    const int w = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = wave_sum(v[k]);
        if (lane_id() == 0) s_v[k][w] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int k = 0; k < NW; ++k) t += s_v[threadIdx.x][k];
        part[4 * blockIdx.x + threadIdx.x] = t;
    }
}

// The local failure predictor of the audit (Section 4, Table 1): point i is flagged
// when twice its last-step motion plus its kept neighbour's exceeds the kept
// certificate's clearance, 2 (|dp_i| + |dp_j|) > d2 - d1, all in binary32.
template <int D>
__global__ void __launch_bounds__(kB) k_rho(int n, const float *__restrict__ pold, const float *__restrict__ pnew,
                                            const int *__restrict__ nn, const float *__restrict__ d1,
                                            const float *__restrict__ d2, uint8_t *__restrict__ rho,
                                            DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    int f = 0;
    if (i < n) {
        const int j = nn[i];
        if (j >= 0 && j < n) {
            const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
            const float si = sqdist<D>(pold[i], pold[n1 + i], D == 3 ? pold[n2 + i] : 0.0f, pnew[i], pnew[n1 + i],
                                       D == 3 ? pnew[n2 + i] : 0.0f);
            const float sj = sqdist<D>(pold[j], pold[n1 + j], D == 3 ? pold[n2 + j] : 0.0f, pnew[j], pnew[n1 + j],
                                       D == 3 ? pnew[n2 + j] : 0.0f);
            const float delta = cert_sqrt(si) + cert_sqrt(sj);
            const float c = d2[i] - d1[i];
            f = 2.0f * delta > c ? 1 : 0;
        }
        rho[i] = (uint8_t)f;
    }
    f = wave_sum(f);
    if (lane_id() == 0 && f) atomicAdd(&sc->audit[6], (unsigned long long)f);
}

// Failures among the candidates (for the false-repair count).
__global__ void __launch_bounds__(kB) k_audit_cand(const int *__restrict__ frontier, const uint8_t *__restrict__ fail,
                                                   DevScalars *sc)
{
    const int count = sc->nfront;
    int k = 0;
    for (int q = blockIdx.x * kB + threadIdx.x; q < count; q += gridDim.x * kB) k += fail[frontier[q]] != 0;
    k = wave_sum(k);
    if (lane_id() == 0 && k) atomicAdd(&sc->audit[5], (unsigned long long)k);
}

inline int blocks_for(long long n, int per) { return (int)((n + per - 1) / per); }

inline int check() { return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP; }

template <int D, int L>
void launch_query_t(const QueryArgs &a, long long maxq, hipStream_t s, bool unit)
{
    // at most 8192 workgroups (32 per CU, more than can be resident) striding over
    // the queries: the waves queue behind the resident ones, so a wave held up by
    // slow queries delays little else (against 2048: the plane repair query at
    // 2^24 509 -> 428 us), and few are idle when the count on the device is far
    // below the bound maxq
    constexpr int GPB = kB / L;
    long long blocks = (maxq + GPB - 1) / GPB;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    if (unit)
        hipLaunchKernelGGL((k_query<D, L, true>), dim3((unsigned)blocks), dim3(kB), 0, s, a);
    else
        hipLaunchKernelGGL((k_query<D, L, false>), dim3((unsigned)blocks), dim3(kB), 0, s, a);
}

}  // namespace

int launch_fill(void *p, int value, size_t count, hipStream_t s)
{
    if (count == 0) return NNC_OK;
    const int blocks = (int)((count + kB - 1) / kB < 4096 ? (count + kB - 1) / kB : 4096);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kB), 0, s, (int *)p, value, count);
    return check();
}

int launch_cells_init(nnc_ctx *c, const float *pos)
{
    if (c->n == 0) return NNC_OK;
    const int blocks = blocks_for(c->n, kB);
    if (c->d == 2)
        hipLaunchKernelGGL(k_cells_init<2>, dim3(blocks), dim3(kB), 0, c->stream, pos, (int)c->n, c->G, c->box, c->cell,
                           c->grid.counts, c->sc);
    else
        hipLaunchKernelGGL(k_cells_init<3>, dim3(blocks), dim3(kB), 0, c->stream, pos, (int)c->n, c->G, c->box, c->cell,
                           c->grid.counts, c->sc);
    return check();
}

int launch_ingest(nnc_ctx *c, const float *pold, const float *pnew)
{
    if (c->n == 0) return NNC_OK;
    const int parity = (int)(c->t & 1);
    const int blocks = blocks_for(c->n, kB) < kIngestBlocks ? blocks_for(c->n, kB) : kIngestBlocks;
    int *lm = (c->flags & NNC_BUDGET) ? c->last_move : nullptr;
    if (c->d == 2)
        hipLaunchKernelGGL(k_ingest<2>, dim3(blocks), dim3(kB), 0, c->stream, pold, pnew, (int)c->n, c->G, c->box, c->cell,
                           c->grid.counts, c->grid.rank, c->grid.slots, c->sc, parity, lm, (int)c->t);
    else
        hipLaunchKernelGGL(k_ingest<3>, dim3(blocks), dim3(kB), 0, c->stream, pold, pnew, (int)c->n, c->G, c->box, c->cell,
                           c->grid.counts, c->grid.rank, c->grid.slots, c->sc, parity, lm, (int)c->t);
    return check();
}

int launch_filter(nnc_ctx *c, float eps_declared)
{
    const int parity = (int)(c->t & 1);
    if (c->n > (int64_t)kReduceScanMinN) {
        const int tiles = blocks_for(c->n, kFTile);
        if (tiles + 1 > c->ntcount) return NNC_E_INVAL;
        if ((long long)tiles * kFMasks > c->nfmask) return NNC_E_INVAL;
        hipLaunchKernelGGL(k_filter_count, dim3(tiles), dim3(kB), 0, c->stream, c->e, (int)c->n, c->sc, parity,
                           eps_declared, c->fail, c->tcount, c->fmask, c->fail_dirty ? 1 : 0,
                           (const int *)c->frontier);
        hipLaunchKernelGGL(k_filter_offsets, dim3(1), dim3(1024), 0, c->stream, c->tcount, tiles, c->sc);
        hipLaunchKernelGGL(k_filter_write, dim3(tiles), dim3(kB), 0, c->stream, (int)c->n,
                           (const unsigned long long *)c->fmask, (const int *)c->tcount, c->frontier, &c->sc->err);
        c->fail_dirty = 0;
        return check();
    }
    // one workgroup only for small scenes: above two tiles the look-back version,
    // whose tiles count in parallel, is faster (measured at N = 16000)
    const bool small = c->n <= (int64_t)kSmallMaxN;
    const bool small_tiles = c->n <= kFiltSmallTilesN;
    const int ftile = kB * (small_tiles ? kFiltRowsSmall : kFiltRowsLarge);
    if (!small && blocks_for(c->n, ftile) > c->nstatus) return NNC_E_INVAL;
    if (small) {
        hipLaunchKernelGGL(k_filter_small, dim3(1), dim3(kSmallB), 0, c->stream, c->e, (int)c->n, c->sc, parity,
                           eps_declared, c->frontier, c->fail);
    } else {
        const int tiles = blocks_for(c->n, ftile);
        if (small_tiles)
            hipLaunchKernelGGL(k_filter<kFiltRowsSmall>, dim3(tiles), dim3(kB), 0, c->stream, c->e, (int)c->n, c->sc,
                               c->sync, parity, eps_declared, c->frontier, c->fail, c->status);
        else
            hipLaunchKernelGGL(k_filter<kFiltRowsLarge>, dim3(tiles), dim3(kB), 0, c->stream, c->e, (int)c->n, c->sc,
                               c->sync, parity, eps_declared, c->frontier, c->fail, c->status);
    }
    return check();
}

int launch_grid_build(nnc_ctx *c, const float *pos, bool from_slots)
{
    const int parity = (int)(c->t & 1);
    const int tiles = blocks_for(c->ncell, kScanTile);
    if (tiles > c->nstatus) return NNC_E_INVAL;
    hipLaunchKernelGGL(k_scan_cells, dim3(tiles), dim3(kB), 0, c->stream, c->grid.counts, c->ncell,
                       c->grid.cell_start, c->grid.cursor, c->sc, c->sync, parity, c->status);
    if (c->n > 0 && from_slots) {
        // the tiled pass's record buffer (16 bytes per point) holds the new order
        // until it is copied back over the slots
        const int blocks = blocks_for(c->n, kB);
        float4 *tmp = reinterpret_cast<float4 *>(c->rec);
        if (c->d == 2)
            hipLaunchKernelGGL(k_scatter_slots<2>, dim3(blocks), dim3(kB), 0, c->stream,
                               (const float4 *)c->grid.slots, (const int *)c->cell, (int)c->n, c->G, c->box,
                               c->grid.cursor, c->grid.rank, tmp, c->sc);
        else
            hipLaunchKernelGGL(k_scatter_slots<3>, dim3(blocks), dim3(kB), 0, c->stream,
                               (const float4 *)c->grid.slots, (const int *)c->cell, (int)c->n, c->G, c->box,
                               c->grid.cursor, c->grid.rank, tmp, c->sc);
        hipLaunchKernelGGL(k_copy4, dim3(blocks < 4096 ? blocks : 4096), dim3(kB), 0, c->stream,
                           (const float4 *)tmp, c->grid.slots, (int)c->n);
    } else if (c->n > 0) {
        const int blocks = blocks_for(c->n, kB);
        if (c->d == 2)
            hipLaunchKernelGGL(k_scatter<2>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.rank, c->grid.slots, c->sc);
        else
            hipLaunchKernelGGL(k_scatter<3>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.rank, c->grid.slots, c->sc);
    }
    return check();
}

namespace {

QueryArgs query_args(nnc_ctx *c, const int32_t *list, const int32_t *count_dev, int all, int init)
{
    QueryArgs a;
    a.pos = c->pos_cur;
    a.slots = c->grid.slots;
    a.cell_start = c->grid.cell_start;
    a.cell = c->cell;
    a.list = list;
    a.count_dev = count_dev;
    a.list_cap = list == c->frontier || list == c->wide ? (int)c->n : 0;
    a.n = (int)c->n;
    a.G = c->G;
    a.all = all;
    a.init = init;
    a.t = (int)c->t;
    a.parity = (int)(c->t & 1);
    a.nn = c->nn;
    a.stamp = c->stamp;
    a.hist = c->hist_fail;
    a.touched = nullptr;  // the entropy scans the histogram
    a.d1 = c->d1;
    a.d2 = c->d2;
    a.e = c->e;
    a.Si = c->Si;
    a.cmask = nullptr;
    a.qkey = nullptr;
    a.tiled_from = 0;
    a.fail = c->fail;
    a.sc = c->sc;
    a.guard = c->guard;
    a.K = c->K;
    a.box = c->box;
    a.fuzz = c->fuzz;
    return a;
}

void launch_pointwise(nnc_ctx *c, const QueryArgs &a)
{
    const long long maxq = c->n;
    if (c->d == 2) {
        if (c->lanes == 64) launch_query_t<2, 64>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 32) launch_query_t<2, 32>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 1) launch_query_t<2, 1>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 4) launch_query_t<2, 4>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 8) launch_query_t<2, 8>(a, maxq, c->stream, c->unit_box);
        else launch_query_t<2, 16>(a, maxq, c->stream, c->unit_box);
    } else {
        if (c->lanes == 64) launch_query_t<3, 64>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 32) launch_query_t<3, 32>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 1) launch_query_t<3, 1>(a, maxq, c->stream, c->unit_box);
        else if (c->lanes == 8) launch_query_t<3, 8>(a, maxq, c->stream, c->unit_box);
        else launch_query_t<3, 16>(a, maxq, c->stream, c->unit_box);
    }
}

}  // namespace

namespace {

// Tile shape of the cell-tiled queries: the most queries per staged neighbour at
// the mean occupancy, within the LDS stage and the cell-start table.
void tile_shape(const nnc_ctx *c, int &TX, int &TY)
{
    const double occ = (double)c->n / (double)c->ncell > 1.0 ? (double)c->n / (double)c->ncell : 1.0;
    TX = TY = 1;
    double best = -1.0;
    for (int ty = 1; ty <= kTYMax && ty <= c->G; ty *= 2) {
        const int R = c->d == 3 ? 3 * (ty + 2) : ty + 2;
        int tx = (int)(0.6 * kNbMax / (R * occ)) - 2;
        tx = tx > kTXMax ? kTXMax : tx;
        tx = tx > c->G ? c->G : tx;
        tx = tx > kCsMax / R - 3 ? kCsMax / R - 3 : tx;
        if (tx < 1) continue;
        const double ratio = (double)tx * ty / ((double)R * (tx + 2));
        if (ratio > best) {
            best = ratio;
            TX = tx;
            TY = ty;
        }
    }
}

void launch_tiled(nnc_ctx *c, const QueryArgs &a, int TX, int TY, long long nsx, long long nsy, long long tiles)
{
    const dim3 grid((unsigned)tiles), block(kTB);
    if (c->d == 2 && c->unit_box)
        hipLaunchKernelGGL((k_query_tiled<2, true>), grid, block, 0, c->stream, a, TX, TY, (int)nsx, (int)nsy, c->wide,
                           c->rec);
    else if (c->d == 2)
        hipLaunchKernelGGL((k_query_tiled<2, false>), grid, block, 0, c->stream, a, TX, TY, (int)nsx, (int)nsy, c->wide,
                           c->rec);
    else if (c->unit_box)
        hipLaunchKernelGGL((k_query_tiled<3, true>), grid, block, 0, c->stream, a, TX, TY, (int)nsx, (int)nsy, c->wide,
                           c->rec);
    else
        hipLaunchKernelGGL((k_query_tiled<3, false>), grid, block, 0, c->stream, a, TX, TY, (int)nsx, (int)nsy, c->wide,
                           c->rec);
}

}  // namespace

int tiled_repair_from(const nnc_ctx *c)
{
    return (c->flags & NNC_QUERY_TILED) && !(c->flags & NNC_QUERY_POINTWISE) ? 1 : 0;
}

int launch_query(nnc_ctx *c, const int32_t *list, const int32_t *count_dev, int all, int init, double *qkey)
{
    if (c->n == 0) return NNC_OK;
    // a long repair list of a large scene: the cell-tiled query of the marked candidates
    // (the device picks it from the list's length: both launches check the count)
    const bool split = !all && !init && list && tiled_repair_from(c) > 0;
    if (!split) {
        QueryArgs a = query_args(c, list, count_dev, all, init);
        a.qkey = all ? nullptr : qkey;
        launch_pointwise(c, a);
        return check();
    }
    const int from = tiled_repair_from(c);
    int TX, TY;
    tile_shape(c, TX, TY);
    const long long nsx = (c->G + TX - 1) / TX, nsy = (c->G + TY - 1) / TY;
    const long long tiles = nsx * nsy * (c->d == 3 ? c->G : 1);
    if (tiles > 0x7fffffffLL) return NNC_E_INVAL;
    const int mb = blocks_for(c->n, kB) < 4096 ? blocks_for(c->n, kB) : 4096;
    hipLaunchKernelGGL(k_cand_mask, dim3(mb), dim3(kB), 0, c->stream, list, count_dev, (int)c->n, from, c->grid.rank,
                       c->cmask, c->sc);
    QueryArgs a = query_args(c, list, count_dev, 0, 0);
    a.cmask = c->cmask;
    a.tiled_from = from;
    launch_tiled(c, a, TX, TY, nsx, nsy, tiles);
    a.cmask = nullptr;
    a.qkey = qkey;
    launch_pointwise(c, a);   // the short lists
    // points of the tiled repair whose search must widen (none when it did not run)
    QueryArgs w = query_args(c, c->wide, &c->sc->nwide, 0, 0);
    w.tiled_from = 0;
    launch_pointwise(c, w);
    return check();
}

// All points, right after a grid build: tiled (then the widening pass over the
// points it left), or pointwise.
int launch_query_all(nnc_ctx *c, int init)
{
    if (c->n == 0) return NNC_OK;
    const long long from = init ? kTiledMinN : c->d == 3 ? kTiledMinNRebuild3 : kTiledMinNRebuild2;
    const bool tiled = (c->flags & NNC_QUERY_TILED) || (!(c->flags & NNC_QUERY_POINTWISE) && c->n >= from);
    if (!tiled) return launch_query(c, nullptr, nullptr, 1, init, nullptr);
    int TX, TY;
    tile_shape(c, TX, TY);
    const long long nsx = (c->G + TX - 1) / TX, nsy = (c->G + TY - 1) / TY;
    const long long tiles = nsx * nsy * (c->d == 3 ? c->G : 1);
    if (tiles > 0x7fffffffLL) return NNC_E_INVAL;
    const QueryArgs a = query_args(c, nullptr, nullptr, 1, init);
    launch_tiled(c, a, TX, TY, nsx, nsy, tiles);
    hipLaunchKernelGGL(k_finish_all, dim3(blocks_for(c->n, kB)), dim3(kB), 0, c->stream, a, (const int4 *)c->rec);
    launch_pointwise(c, query_args(c, c->wide, &c->sc->nwide, 0, init));
    return check();
}

int launch_entropy(nnc_ctx *c, int which)
{
    int *hist = which == 0 ? c->hist_fail : c->hist_cand;
    const int ncell4 = (c->ncell + 3) / 4;
    if (ncell4 > kEntropyOneGroup4) {
        hipLaunchKernelGGL(k_entropy_part, dim3(kEntropyParts), dim3(kB), 0, c->stream, hist, ncell4, c->ent_part);
        hipLaunchKernelGGL(k_entropy_final, dim3(1), dim3(kB), 0, c->stream, which, kEntropyParts,
                           (const double *)c->ent_part, c->sc);
    } else {
        hipLaunchKernelGGL(k_entropy, dim3(1), dim3(1024), 0, c->stream, which, hist, ncell4, c->sc);
    }
    return check();
}

int launch_cand_hist(nnc_ctx *c)
{
    const int blocks = c->n > 0 ? (blocks_for(c->n, kB) < 4096 ? blocks_for(c->n, kB) : 4096) : 1;
    hipLaunchKernelGGL(k_cand_hist, dim3(blocks), dim3(kB), 0, c->stream, c->frontier, c->cell, c->hist_cand,
                       c->sc);
    return check();
}

int launch_features(nnc_ctx *c, float *out)
{
    hipLaunchKernelGGL(k_features, dim3(1), dim3(1024), 0, c->stream, c->e, (int)c->n, c->d, c->ncell, c->sc,
                       (int)(c->t & 1), out);
    return check();
}

int launch_audit(nnc_ctx *c)
{
    if (c->n == 0) return NNC_OK;
    const int blocks = blocks_for(c->n, kB);
    hipLaunchKernelGGL(k_audit, dim3(blocks), dim3(kB), 0, c->stream, (int)c->n, c->nn, c->d1, c->d2, c->stamp,
                       (int)c->t, c->fail, c->a_nn, c->a_d1, c->a_d2,
                       (const uint8_t *)(c->rho_step == c->t ? c->rho : nullptr), c->sc);
    hipLaunchKernelGGL(k_audit_cand, dim3(blocks < 4096 ? blocks : 4096), dim3(kB), 0, c->stream, c->frontier,
                       c->fail, c->sc);
    return check();
}

int launch_shape(nnc_ctx *c, int which, const double *cen)
{
    const int *list = which == 1 ? c->frontier : nullptr;
    const int *count = which == 1 ? &c->sc->nfront : nullptr;
    if (c->d == 2)
        hipLaunchKernelGGL(k_shape<2>, dim3(kShapeParts), dim3(kB), 0, c->stream, c->pos_cur, (int)c->n, c->fail, list,
                           count, cen, c->shape_part);
    else
        hipLaunchKernelGGL(k_shape<3>, dim3(kShapeParts), dim3(kB), 0, c->stream, c->pos_cur, (int)c->n, c->fail, list,
                           count, cen, c->shape_part);
    return check();
}

int launch_budget(nnc_ctx *c)
{
    if (c->n == 0) return NNC_OK;
    const int parity = (int)(c->t & 1);
    const int b = blocks_for(c->n, kB);
    const int blocks = b < 4096 ? b : 4096;
    if (c->d == 2)
        hipLaunchKernelGGL(k_budget<2>, dim3(blocks), dim3(kB), 0, c->stream, c->pos_cur, (int)c->n, c->nn, c->d2,
                           c->Si, c->e, c->sc, parity, c->guard, c->K, c->cell, c->stamp, c->last_move, c->G, c->box,
                           c->fuzz);
    else
        hipLaunchKernelGGL(k_budget<3>, dim3(blocks), dim3(kB), 0, c->stream, c->pos_cur, (int)c->n, c->nn, c->d2,
                           c->Si, c->e, c->sc, parity, c->guard, c->K, c->cell, c->stamp, c->last_move, c->G, c->box,
                           c->fuzz);
    return check();
}

int launch_rho(nnc_ctx *c)
{
    if (c->n == 0) return NNC_OK;
    const int blocks = blocks_for(c->n, kB);
    if (c->d == 2)
        hipLaunchKernelGGL(k_rho<2>, dim3(blocks), dim3(kB), 0, c->stream, (int)c->n, c->pos_prev, c->pos_cur, c->nn,
                           c->d1, c->d2, c->rho, c->sc);
    else
        hipLaunchKernelGGL(k_rho<3>, dim3(blocks), dim3(kB), 0, c->stream, (int)c->n, c->pos_prev, c->pos_cur, c->nn,
                           c->d1, c->d2, c->rho, c->sc);
    return check();
}

}  // namespace nnc
