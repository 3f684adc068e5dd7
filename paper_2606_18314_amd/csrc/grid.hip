// Single-scene kernels of the maintenance step (Algorithm 1 with the appendix's
// clock) and of the O(N) grid rebuild, for gfx950.
//
//   k_ingest       per point: squared displacement (wave max -> one atomic per
//                  wave), new cell id, occupancy counts and the occupied-cell
//                  count C kept incrementally, and the point's current
//                  coordinates written to its grid slot.
//   k_filter*      clock advance and safety filter S_t >= e_i with an
//                  order-preserving compaction into an ascending candidate
//                  list (wave ballot + mbcnt, a per-tile scan in LDS; across
//                  tiles a decoupled look-back, or one workgroup for small N).
//   k_scan_cells   exclusive scan of the occupancy counts -> cell-start table.
//   k_scatter      counting-sort scatter: slot order (perm, rank) and the
//                  coordinates in slot order.
//   k_query        exact 2-NN of each query through the grid, one group of L
//                  lanes per query: the 3^d block's rows are spread over the
//                  lanes (contiguous slots, coalesced loads), partial top-2s
//                  are merged by a butterfly, and the search widens ring by
//                  ring until the second neighbour is provably enclosed
//                  (Corollary 1); then the new certificate, expiry key,
//                  failure flag and failure histogram.
//   k_entropy      normalised entropy (Definition 2) over the touched cells.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace nnc {

namespace {

constexpr int kB = 256;            // threads per point-parallel workgroup
constexpr int kRows = 8;           // items per thread in the tile scans
constexpr int kTile = kB * kRows;  // items per look-back tile
constexpr int kSmallB = 1024;      // one-workgroup filter: threads
constexpr int kSmallRows = 32;     // one-workgroup filter: items per thread (n <= 32768)
constexpr int kFlagA = 1, kFlagP = 2;
constexpr unsigned kSpinLimit = 1u << 24;
constexpr double kFuzz = 0x1p-20;  // cell-boundary rounding allowance (coordinates)
constexpr double kRel = 0x1p-20;   // relative allowance on drift and distances

__device__ __forceinline__ unsigned long long pack_status(unsigned epoch, int flag, unsigned v)
{
    return ((unsigned long long)(epoch & 0x3fffffffu) << 34) | ((unsigned long long)flag << 32) | v;
}

// Decoupled look-back (single thread): publish this tile's aggregate, walk
// predecessors until an inclusive prefix is found, publish the inclusive prefix
// and return the exclusive one.  Tickets are taken in launch order, so every
// predecessor is running or done; the wait is bounded all the same.
__device__ unsigned lookback(unsigned long long *status, int tile, unsigned agg, unsigned epoch, unsigned *err)
{
    if (tile == 0) {
        st_agent(&status[0], pack_status(epoch, kFlagP, agg));
        return 0u;
    }
    st_agent(&status[tile], pack_status(epoch, kFlagA, agg));
    unsigned excl = 0;
    int p = tile - 1;
    unsigned spins = 0;
    const unsigned ep = epoch & 0x3fffffffu;
    while (p >= 0) {
        const unsigned long long v = ld_agent(&status[p]);
        const int flag = (int)((v >> 32) & 3u);
        if ((unsigned)(v >> 34) != ep || flag == 0) {
            if (++spins > kSpinLimit) {
                atomicOr(err, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += (unsigned)v;
        if (flag == kFlagP) break;
        --p;
    }
    st_agent(&status[tile], pack_status(epoch, kFlagP, excl + agg));
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

__global__ void k_fill(int *p, int value, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Add a per-lane change of the occupied-cell count with one atomic per wave.
__device__ __forceinline__ void add_C(DevScalars *sc, int delta)
{
    const int w = wave_sum(delta);
    if (lane_id() == 0 && w != 0) atomicAdd(&sc->C, w);
}

template <int D>
__global__ void __launch_bounds__(kB) k_cells_init(const float *__restrict__ pos, int n, int G,
                                                   int *__restrict__ cell, int *__restrict__ counts,
                                                   DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    int dC = 0;
    if (i < n) {
        const float x = pos[i], y = pos[(size_t)n + i], z = D == 3 ? pos[2 * (size_t)n + i] : 0.f;
        int c = 0;
        if (all_finite<D>(x, y, z))
            c = cell_id<D>(x, y, z, G);
        else
            atomicOr(&sc->err, kErrNonFinite);
        cell[i] = c;
        dC = atomicAdd(&counts[c], 1) == 0;
    }
    add_C(sc, dC);
}

template <int D>
__global__ void __launch_bounds__(kB) k_ingest(const float *__restrict__ pold, const float *__restrict__ pnew,
                                               int n, int G, int *__restrict__ cell, int *__restrict__ counts,
                                               const int *__restrict__ rank, float *__restrict__ sorted,
                                               DevScalars *sc, int parity)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    float s = 0.0f;
    int dC = 0;
    if (i < n) {
        const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
        const float x0 = pold[i], y0 = pold[n1 + i], z0 = D == 3 ? pold[n2 + i] : 0.f;
        const float x1 = pnew[i], y1 = pnew[n1 + i], z1 = D == 3 ? pnew[n2 + i] : 0.f;
        const int k = rank[i];
        sorted[k] = x1;
        sorted[n1 + k] = y1;
        if constexpr (D == 3) sorted[n2 + k] = z1;
        if (all_finite<D>(x1, y1, z1) && all_finite<D>(x0, y0, z0)) {
            s = sqdist<D>(x0, y0, z0, x1, y1, z1);
            const int c = cell_id<D>(x1, y1, z1, G);
            const int old = cell[i];
            if (c != old) {
                cell[i] = c;
                dC -= atomicSub(&counts[old], 1) == 1;
                dC += atomicAdd(&counts[c], 1) == 0;
            }
        } else {
            atomicOr(&sc->err, kErrNonFinite);
        }
    }
    add_C(sc, dC);
    s = wave_max(s);
    if (lane_id() == 0 && s > 0.0f) atomicMax(&sc->dmax[parity], __float_as_uint(s));
}

// Clock advance shared by both filter variants: every workgroup derives S_t
// from the same two words; one leader publishes it.
__device__ __forceinline__ double advance_clock(DevScalars *sc, int parity, float eps_decl, bool leader)
{
    const float eps = sqrtf(__uint_as_float(sc->dmax[parity]));
    const double St = sc->S[parity ^ 1] + (double)eps;
    if (leader) {
        sc->S[parity] = St;
        sc->eps = (double)eps;
        sc->dmax[parity ^ 1] = 0u;
        if (eps_decl >= 0.0f && (double)eps > (double)eps_decl * (1.0 + 0x1p-16) + 0x1p-20)
            atomicOr(&sc->err, kErrEps);
    }
    return St;
}

__global__ void __launch_bounds__(kB) k_filter(const double *__restrict__ e, int n, DevScalars *sc, DevSync *sy,
                                               int parity, float eps_decl, int *__restrict__ frontier,
                                               uint8_t *__restrict__ fail, unsigned long long *status)
{
    __shared__ int s_tile;
    __shared__ unsigned s_epoch;
    __shared__ int s_cnt[kRows][kB / 64];
    __shared__ unsigned s_base;
    take_ticket(sy, &s_tile, &s_epoch);
    const int tile = s_tile;
    const double St = advance_clock(sc, parity, eps_decl, tile == 0 && threadIdx.x == 0);
    const int w = threadIdx.x >> 6;
    const unsigned lane = lane_id();
    const long long base = (long long)tile * kTile;
    unsigned long long masks[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
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
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < kRows; ++k)
            for (int v = 0; v < kB / 64; ++v) {
                const int c = s_cnt[k][v];
                s_cnt[k][v] = run;
                run += c;
            }
        const unsigned excl = lookback(status, tile, (unsigned)run, s_epoch, &sc->err);
        s_base = excl;
        if (tile == (int)gridDim.x - 1) {
            sc->nfront = (int)(excl + (unsigned)run);
            retire_ticket(sy, s_epoch);
        }
    }
    __syncthreads();
    const unsigned b = s_base;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
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
    const double St = advance_clock(sc, parity, eps_decl, threadIdx.x == 0);
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
    const long long base = (long long)tile * kTile;
    int pref[kRows];
    int run = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const long long c = base + (long long)k * kB + threadIdx.x;
        const int v = c < ncell ? counts[c] : 0;
        int tot;
        const int ex = block_excl_scan<kB>(v, s_w, tot);
        pref[k] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        const unsigned excl = lookback(status, tile, (unsigned)run, s_epoch, &sc->err);
        s_base = excl;
        if (tile == (int)gridDim.x - 1) {
            cell_start[ncell] = (int)(excl + (unsigned)run);
            retire_ticket(sy, s_epoch);
        }
        if (tile == 0) sc->S_grid = sc->S[parity];
    }
    __syncthreads();
    const int b = (int)s_base;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const long long c = base + (long long)k * kB + threadIdx.x;
        if (c < ncell) {
            cell_start[c] = b + pref[k];
            cursor[c] = b + pref[k];
        }
    }
}

template <int D>
__global__ void __launch_bounds__(kB) k_scatter(const float *__restrict__ pos, const int *__restrict__ cell, int n,
                                                int *__restrict__ cursor, int *__restrict__ perm,
                                                int *__restrict__ rank, float *__restrict__ sorted,
                                                DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const int k = atomicAdd(&cursor[cell[i]], 1);
    if (k >= n) {  // unreachable while the counts match the cells
        atomicOr(&sc->err, kErrOverflow);
        return;
    }
    perm[k] = i;
    rank[i] = k;
    sorted[k] = pos[i];
    sorted[(size_t)n + k] = pos[(size_t)n + i];
    if constexpr (D == 3) sorted[2 * (size_t)n + k] = pos[2 * (size_t)n + i];
}

// Normalised entropy (Definition 2) of the failures (which = 0) or candidates
// (which = 1) over the touched cells, computed by one workgroup of NT threads;
// clears the histogram entries and counters it consumed.
template <int NT>
__device__ void entropy_block(int which, int *__restrict__ hist, const int *__restrict__ touched, DevScalars *sc)
{
    __shared__ double s_acc[NT / 64];
    const int m = which == 0 ? sc->ntouched : sc->ncand_touched;
    const int F = which == 0 ? sc->nfail : sc->nfront;
    double acc = 0.0;
    for (int k = threadIdx.x; k < m; k += NT) {
        const int c = touched[k];
        const int nk = hist[c];
        hist[c] = 0;
        acc += (double)nk * log((double)nk);
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_acc[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < NT / 64; ++k) tot += s_acc[k];
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
}

struct QueryArgs {
    const float *pos;          // current coordinates, point order
    const float *sorted;       // current coordinates, slot order
    const int *cell_start, *perm, *cell;
    const int *list, *count_dev;
    int n, G, all, init, t, parity;
    int *nn, *stamp, *hist, *touched;
    float *d1, *d2;
    double *e;
    uint8_t *fail;
    DevScalars *sc;
    double guard, K;
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
    const size_t n1 = (size_t)a.n, n2 = 2 * (size_t)a.n;
    const float xj = a.sorted[k];
    const float yj = a.sorted[n1 + k];
    const float zj = D == 3 ? a.sorted[n2 + k] : 0.0f;
    const int j = a.perm[k];
    const float s = sqdist<D>(x, y, z, xj, yj, zj);
    if (j != i) t.push(s, j);
}

// Cells of the 3^d block around (gx,gy,gz), clipped to the grid: 3^(d-1) rows,
// each a contiguous run of slots.  Lanes first fetch one row's bounds each,
// then walk the concatenated slots with stride L.
template <int D, int L>
__device__ __forceinline__ void scan_block(const QueryArgs &a, float x, float y, float z, int i, int gx, int gy,
                                           int gz, int lane, Top2 &t)
{
    constexpr int R = D == 3 ? 9 : 3;
    static_assert(L >= R, "a group needs one lane per row");
    const int G = a.G;
    int rs = 0, rl = 0;
    if (lane < R) {
        const int cy = gy + lane % 3 - 1;
        const int cz = D == 3 ? gz + lane / 3 - 1 : 0;
        if (cy >= 0 && cy < G && cz >= 0 && cz < (D == 3 ? G : 1)) {
            const int row = (cz * G + cy) * G;
            const int xlo = max(gx - 1, 0), xhi = min(gx + 1, G - 1);
            rs = a.cell_start[row + xlo];
            rl = a.cell_start[row + xhi + 1] - rs;
        }
    }
    int incl = rl;
#pragma unroll
    for (int off = 1; off < R; off <<= 1) {
        const int v = __shfl_up(incl, off, L);
        if (lane >= off) incl += v;
    }
    const int total = __shfl(incl, R - 1, L);
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

// Visit every slot of the ring r >= 2.  Runs are taken L at a time: each lane
// fetches one run's slot range, a group scan concatenates them, and the lanes
// walk the concatenation with stride L, finding each slot's run by a binary
// search over the group (all loops are uniform over the group, so every
// shuffle reads an active lane).
template <int D, int L>
__device__ __forceinline__ void scan_ring(const QueryArgs &a, float x, float y, float z, int i, int gx, int gy,
                                          int gz, int r, int lane, Top2 &t)
{
    const int G = a.G;
    const int m2 = 2 * r - 1;
    const int nruns = D == 3 ? 2 * (2 * r + 1) + 2 * m2 + 2 * m2 * m2 : 2 + 2 * m2;
    for (int c0 = 0; c0 < nruns; c0 += L) {
        const int u = c0 + lane;
        int rs = 0, rl = 0;
        int row, xlo, xhi;
        if (u < nruns && ring_run<D>(u, r, gx, gy, gz, G, row, xlo, xhi)) {
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

template <int D, int L>
__device__ void group_search(const QueryArgs &a, float x, float y, float z, int i, double margin, int lane,
                             Top2 &t)
{
    const int G = a.G;
    const int gx = cell_axis(x, G), gy = cell_axis(y, G), gz = D == 3 ? cell_axis(z, G) : 0;
    scan_block<D, L>(a, x, y, z, i, gx, gy, gz, lane, t);
    group_reduce<L>(t);
    for (int r = 1;; ++r) {
        const double B = outside_bound<D>(x, y, z, gx, gy, gz, r, G);
        if (__builtin_isinf(B)) break;  // the whole grid has been visited
        const double Be = B - margin;
        if (Be > 0.0 && (double)t.s2 < Be * Be * (1.0 - kRel)) break;
        // every lane holds the merged result: keep it in lane 0 only, so that the
        // next merge combines disjoint sets
        if (lane != 0) t.init();
        scan_ring<D, L>(a, x, y, z, i, gx, gy, gz, r + 1, lane, t);
        group_reduce<L>(t);
    }
}

template <int D, int L>
__global__ void __launch_bounds__(kB) k_query(QueryArgs a)
{
    const int count = a.all ? a.n : min(*a.count_dev, a.n);
    const double St = a.sc->S[a.parity];
    const double drift = St - a.sc->S_grid;
    const double margin = kFuzz + drift * (1.0 + kRel);
    const size_t n1 = (size_t)a.n, n2 = 2 * (size_t)a.n;
    const int lane = threadIdx.x & (L - 1);
    constexpr int GPB = kB / L;
    for (int q = blockIdx.x * GPB + (int)(threadIdx.x / L); q < count; q += gridDim.x * GPB) {
        int i;
        float x, y, z = 0.f;
        if (a.all) {
            i = a.perm[q];
            x = a.sorted[q];
            y = a.sorted[n1 + q];
            if constexpr (D == 3) z = a.sorted[n2 + q];
        } else {
            i = a.list[q];
            if (i < 0 || i >= a.n) continue;  // caller-supplied lists are checked
            x = a.pos[i];
            y = a.pos[n1 + i];
            if constexpr (D == 3) z = a.pos[n2 + i];
        }
        const int old = lane == 0 ? a.nn[i] : 0;  // fetched early, used at the end
        Top2 t;
        t.init();
        group_search<D, L>(a, x, y, z, i, margin, lane, t);
        if (lane == 0) {
            const float d1 = sqrtf(t.s1), d2 = sqrtf(t.s2);
            a.nn[i] = t.nn;
            a.d1[i] = d1;
            a.d2[i] = d2;
            a.e[i] = expiry(St, d1, d2, a.guard, a.K);
            a.stamp[i] = a.t;
            const bool f = !a.init && t.nn != old;
            a.fail[i] = f ? 1 : 0;
            if (f) {
                atomicAdd(&a.sc->nfail, 1);
                const int c = a.cell[i];
                if (atomicAdd(&a.hist[c], 1) == 0) a.touched[atomicAdd(&a.sc->ntouched, 1)] = c;
            }
        }
    }
}

__global__ void __launch_bounds__(1024) k_entropy(int which, int *__restrict__ hist, const int *__restrict__ touched,
                                                  DevScalars *sc)
{
    entropy_block<1024>(which, hist, touched, sc);
}

__global__ void __launch_bounds__(kB) k_cand_hist(const int *__restrict__ frontier, const int *__restrict__ cell,
                                                  int *__restrict__ hist, int *__restrict__ touched, DevScalars *sc)
{
    const int count = sc->nfront;
    for (int q = blockIdx.x * kB + threadIdx.x; q < count; q += gridDim.x * kB) {
        const int c = cell[frontier[q]];
        if (atomicAdd(&hist[c], 1) == 0) touched[atomicAdd(&sc->ncand_touched, 1)] = c;
    }
}

// Audit of the state against an all-pairs result (a_*): misses, value
// mismatches of certificates computed at this step, failures and an
// order-independent hash of nn[] (sum of SplitMix64(i << 32 | nn_i)).
__global__ void __launch_bounds__(kB) k_audit(int n, const int *__restrict__ nn, const float *__restrict__ d1,
                                              const float *__restrict__ d2, const int *__restrict__ stamp, int t,
                                              const uint8_t *__restrict__ fail, const int *__restrict__ a_nn,
                                              const float *__restrict__ a_d1, const float *__restrict__ a_d2,
                                              DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    int missed = 0, vm = 0, tf = 0, fresh = 0;
    unsigned long long h = 0;
    if (i < n) {
        missed = a_nn[i] != nn[i];
        fresh = stamp[i] == t;
        vm = fresh && (__float_as_uint(a_d1[i]) != __float_as_uint(d1[i]) ||
                       __float_as_uint(a_d2[i]) != __float_as_uint(d2[i]));
        tf = fail[i] != 0;
        h = mix64(((unsigned long long)(unsigned)i << 32) | (unsigned)nn[i]);
    }
    missed = wave_sum(missed);
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
    }
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
void launch_query_t(const QueryArgs &a, long long maxq, hipStream_t s)
{
    constexpr int GPB = kB / L;
    long long blocks = (maxq + GPB - 1) / GPB;
    if (blocks < 1) blocks = 1;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL((k_query<D, L>), dim3((unsigned)blocks), dim3(kB), 0, s, a);
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
        hipLaunchKernelGGL(k_cells_init<2>, dim3(blocks), dim3(kB), 0, c->stream, pos, (int)c->n, c->G, c->cell,
                           c->grid.counts, c->sc);
    else
        hipLaunchKernelGGL(k_cells_init<3>, dim3(blocks), dim3(kB), 0, c->stream, pos, (int)c->n, c->G, c->cell,
                           c->grid.counts, c->sc);
    return check();
}

int launch_ingest(nnc_ctx *c, const float *pold, const float *pnew)
{
    if (c->n == 0) return NNC_OK;
    const int parity = (int)(c->t & 1);
    const int blocks = blocks_for(c->n, kB);
    if (c->d == 2)
        hipLaunchKernelGGL(k_ingest<2>, dim3(blocks), dim3(kB), 0, c->stream, pold, pnew, (int)c->n, c->G, c->cell,
                           c->grid.counts, c->grid.rank, c->grid.sorted, c->sc, parity);
    else
        hipLaunchKernelGGL(k_ingest<3>, dim3(blocks), dim3(kB), 0, c->stream, pold, pnew, (int)c->n, c->G, c->cell,
                           c->grid.counts, c->grid.rank, c->grid.sorted, c->sc, parity);
    return check();
}

int launch_filter(nnc_ctx *c, float eps_declared)
{
    const int parity = (int)(c->t & 1);
    if (c->n > (int64_t)kSmallB * kSmallRows && blocks_for(c->n, kTile) > c->nstatus) return NNC_E_INVAL;
    if (c->n <= (int64_t)kSmallB * kSmallRows) {
        hipLaunchKernelGGL(k_filter_small, dim3(1), dim3(kSmallB), 0, c->stream, c->e, (int)c->n, c->sc, parity,
                           eps_declared, c->frontier, c->fail);
    } else {
        const int tiles = blocks_for(c->n, kTile);
        hipLaunchKernelGGL(k_filter, dim3(tiles), dim3(kB), 0, c->stream, c->e, (int)c->n, c->sc, c->sync, parity,
                           eps_declared, c->frontier, c->fail, c->status);
    }
    return check();
}

int launch_grid_build(nnc_ctx *c, const float *pos)
{
    const int parity = (int)(c->t & 1);
    const int tiles = blocks_for(c->ncell, kTile);
    if (tiles > c->nstatus) return NNC_E_INVAL;
    hipLaunchKernelGGL(k_scan_cells, dim3(tiles), dim3(kB), 0, c->stream, c->grid.counts, c->ncell,
                       c->grid.cell_start, c->grid.cursor, c->sc, c->sync, parity, c->status);
    if (c->n > 0) {
        const int blocks = blocks_for(c->n, kB);
        if (c->d == 2)
            hipLaunchKernelGGL(k_scatter<2>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.perm, c->grid.rank, c->grid.sorted, c->sc);
        else
            hipLaunchKernelGGL(k_scatter<3>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.perm, c->grid.rank, c->grid.sorted, c->sc);
    }
    return check();
}

int launch_query(nnc_ctx *c, const int32_t *list, const int32_t *count_dev, int all, int init)
{
    if (c->n == 0) return NNC_OK;
    QueryArgs a;
    a.pos = c->pos_cur;
    a.sorted = c->grid.sorted;
    a.cell_start = c->grid.cell_start;
    a.perm = c->grid.perm;
    a.cell = c->cell;
    a.list = list;
    a.count_dev = count_dev;
    a.n = (int)c->n;
    a.G = c->G;
    a.all = all;
    a.init = init;
    a.t = (int)c->t;
    a.parity = (int)(c->t & 1);
    a.nn = c->nn;
    a.stamp = c->stamp;
    a.hist = c->hist_fail;
    a.touched = c->touched_fail;
    a.d1 = c->d1;
    a.d2 = c->d2;
    a.e = c->e;
    a.fail = c->fail;
    a.sc = c->sc;
    a.guard = c->guard;
    a.K = c->K;
    const long long maxq = c->n;
    if (c->d == 2) {
        if (c->lanes == 64) launch_query_t<2, 64>(a, maxq, c->stream);
        else if (c->lanes == 32) launch_query_t<2, 32>(a, maxq, c->stream);
        else launch_query_t<2, 16>(a, maxq, c->stream);
    } else {
        if (c->lanes == 64) launch_query_t<3, 64>(a, maxq, c->stream);
        else if (c->lanes == 32) launch_query_t<3, 32>(a, maxq, c->stream);
        else launch_query_t<3, 16>(a, maxq, c->stream);
    }
    return check();
}

int launch_entropy(nnc_ctx *c, int which)
{
    if (which == 0)
        hipLaunchKernelGGL(k_entropy, dim3(1), dim3(1024), 0, c->stream, 0, c->hist_fail, c->touched_fail, c->sc);
    else
        hipLaunchKernelGGL(k_entropy, dim3(1), dim3(1024), 0, c->stream, 1, c->hist_cand, c->touched_cand, c->sc);
    return check();
}

int launch_cand_hist(nnc_ctx *c)
{
    const int blocks = c->n > 0 ? (blocks_for(c->n, kB) < 4096 ? blocks_for(c->n, kB) : 4096) : 1;
    hipLaunchKernelGGL(k_cand_hist, dim3(blocks), dim3(kB), 0, c->stream, c->frontier, c->cell, c->hist_cand,
                       c->touched_cand, c->sc);
    return check();
}

int launch_audit(nnc_ctx *c)
{
    if (c->n == 0) return NNC_OK;
    const int blocks = blocks_for(c->n, kB);
    hipLaunchKernelGGL(k_audit, dim3(blocks), dim3(kB), 0, c->stream, (int)c->n, c->nn, c->d1, c->d2, c->stamp,
                       (int)c->t, c->fail, c->a_nn, c->a_d1, c->a_d2, c->sc);
    hipLaunchKernelGGL(k_audit_cand, dim3(blocks < 4096 ? blocks : 4096), dim3(kB), 0, c->stream, c->frontier,
                       c->fail, c->sc);
    return check();
}

}  // namespace nnc
