// Single-scene kernels of the maintenance step (Algorithm 1 with the appendix's
// clock) and of the O(N) grid rebuild, for gfx950.
//
//   k_ingest       eps_t candidates + cell update: squared displacement of every
//                  point, wave max -> one atomic per wave; new cell id; occupancy
//                  counts and the occupied-cell count C kept incrementally.
//   k_filter       clock advance and safety filter S_t >= e_i with an
//                  order-preserving compaction (wave ballot + mbcnt, a per-tile
//                  scan in LDS, decoupled look-back across tiles) -> ascending
//                  candidate list.  Also clears the failure flags.
//   k_scan_cells   exclusive scan of the occupancy counts -> cell-start table.
//   k_scatter      counting-sort scatter: grid order (perm) and the coordinates
//                  in grid order.
//   k_query        exact 2-NN of each query through the grid: the 3^d block
//                  around its cell, widened ring by ring until the second
//                  neighbour is provably enclosed (Corollary 1), then the new
//                  certificate, expiry key, failure flag and failure histogram.
//   k_entropy      normalised entropy (Definition 2) over the touched cells.
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace nnc {

namespace {

constexpr int kB = 256;            // threads per point-parallel workgroup
constexpr int kRows = 8;           // items per thread in the tile scans
constexpr int kTile = kB * kRows;  // items per look-back tile
constexpr int kFlagA = 1, kFlagP = 2;
constexpr unsigned kSpinLimit = 1u << 24;
constexpr double kFuzz = 0x1p-20;       // cell-boundary rounding allowance (coordinates)
constexpr double kRel = 0x1p-20;        // relative allowance on drift and distances

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

// Exclusive scan of one value per thread over a 256-thread workgroup.
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
    for (int k = 0; k < kB / 64; ++k) {
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

template <int D>
__global__ void __launch_bounds__(kB) k_cells_init(const float *__restrict__ pos, int n, int G,
                                                   int *__restrict__ cell, int *__restrict__ counts,
                                                   DevScalars *sc)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const float x = pos[i], y = pos[(size_t)n + i], z = D == 3 ? pos[2 * (size_t)n + i] : 0.f;
    if (!all_finite<D>(x, y, z)) {
        atomicOr(&sc->err, kErrNonFinite);
        cell[i] = 0;
        if (atomicAdd(&counts[0], 1) == 0) atomicAdd(&sc->C, 1);
        return;
    }
    const int c = cell_id<D>(x, y, z, G);
    cell[i] = c;
    if (atomicAdd(&counts[c], 1) == 0) atomicAdd(&sc->C, 1);
}

template <int D>
__global__ void __launch_bounds__(kB) k_ingest(const float *__restrict__ pold, const float *__restrict__ pnew,
                                               int n, int G, int *__restrict__ cell, int *__restrict__ counts,
                                               DevScalars *sc, int parity)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    float s = 0.0f;
    if (i < n) {
        const size_t n1 = (size_t)n, n2 = 2 * (size_t)n;
        const float x0 = pold[i], y0 = pold[n1 + i], z0 = D == 3 ? pold[n2 + i] : 0.f;
        const float x1 = pnew[i], y1 = pnew[n1 + i], z1 = D == 3 ? pnew[n2 + i] : 0.f;
        if (all_finite<D>(x1, y1, z1) && all_finite<D>(x0, y0, z0)) {
            s = sqdist<D>(x0, y0, z0, x1, y1, z1);
            const int c = cell_id<D>(x1, y1, z1, G);
            const int old = cell[i];
            if (c != old) {
                cell[i] = c;
                if (atomicSub(&counts[old], 1) == 1) atomicSub(&sc->C, 1);
                if (atomicAdd(&counts[c], 1) == 0) atomicAdd(&sc->C, 1);
            }
        } else {
            atomicOr(&sc->err, kErrNonFinite);
        }
    }
    s = wave_max(s);
    if (lane_id() == 0 && s > 0.0f) atomicMax(&sc->dmax[parity], __float_as_uint(s));
}

__global__ void __launch_bounds__(kB) k_filter(const double *__restrict__ e, int n, DevScalars *sc, int parity,
                                               float eps_decl, int *__restrict__ frontier,
                                               uint8_t *__restrict__ fail, unsigned long long *status,
                                               unsigned epoch)
{
    __shared__ int s_tile;
    __shared__ int s_cnt[kRows][kB / 64];
    __shared__ unsigned s_base;
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(&sc->tile_ctr, 1u);
    __syncthreads();
    const int tile = s_tile;
    const float eps = sqrtf(__uint_as_float(sc->dmax[parity]));
    const double St = sc->S[parity ^ 1] + (double)eps;
    if (tile == 0 && threadIdx.x == 0) {
        sc->S[parity] = St;
        sc->eps = (double)eps;
        sc->dmax[parity ^ 1] = 0u;
        if (eps_decl >= 0.0f && (double)eps > (double)eps_decl * (1.0 + 0x1p-16) + 0x1p-20)
            atomicOr(&sc->err, kErrEps);
    }
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
        const unsigned excl = lookback(status, tile, (unsigned)run, epoch, &sc->err);
        s_base = excl;
        if (tile == (int)gridDim.x - 1) {
            sc->nfront = (int)(excl + (unsigned)run);
            sc->tile_ctr = 0u;
        }
    }
    __syncthreads();
    const unsigned b = s_base;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        if ((masks[k] >> lane) & 1ull) {
            const long long i = base + (long long)k * kB + threadIdx.x;
            frontier[b + s_cnt[k][w] + rank_below(masks[k])] = (int)i;
        }
    }
}

__global__ void __launch_bounds__(kB) k_scan_cells(const int *__restrict__ counts, int ncell,
                                                   int *__restrict__ cell_start, int *__restrict__ cursor,
                                                   DevScalars *sc, int parity, unsigned long long *status,
                                                   unsigned epoch)
{
    __shared__ int s_tile;
    __shared__ int s_w[kB / 64];
    __shared__ unsigned s_base;
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(&sc->tile_ctr, 1u);
    __syncthreads();
    const int tile = s_tile;
    const long long base = (long long)tile * kTile;
    int pref[kRows];
    int run = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
        const long long c = base + (long long)k * kB + threadIdx.x;
        const int v = c < ncell ? counts[c] : 0;
        int tot;
        const int ex = block_excl_scan(v, s_w, tot);
        pref[k] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) {
        const unsigned excl = lookback(status, tile, (unsigned)run, epoch, &sc->err);
        s_base = excl;
        if (tile == (int)gridDim.x - 1) {
            cell_start[ncell] = (int)(excl + (unsigned)run);
            sc->tile_ctr = 0u;
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
                                                float *__restrict__ sorted)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const int k = atomicAdd(&cursor[cell[i]], 1);
    if (k >= n) return;  // unreachable while counts match cells
    perm[k] = i;
    sorted[k] = pos[i];
    sorted[(size_t)n + k] = pos[(size_t)n + i];
    if constexpr (D == 3) sorted[2 * (size_t)n + k] = pos[2 * (size_t)n + i];
}

struct QueryArgs {
    const float *pos;          // current coordinates, point order
    const float *sorted;       // coordinates in grid order (current when fresh)
    const int *cell_start, *perm, *cell;
    const int *list, *count_dev;
    int n, G, all, init, fresh, t, parity;
    int *nn, *stamp, *hist, *touched;
    float *d1, *d2;
    double *e;
    uint8_t *fail;
    DevScalars *sc;
    double guard, K;
};

template <int D, bool FRESH>
__device__ __forceinline__ void visit(const QueryArgs &a, int k0, int k1, float x, float y, float z, int i,
                                      Top2 &t)
{
    const size_t n1 = (size_t)a.n, n2 = 2 * (size_t)a.n;
    for (int k = k0; k < k1; ++k) {
        const int j = a.perm[k];
        float xj, yj, zj = 0.f;
        if constexpr (FRESH) {
            xj = a.sorted[k];
            yj = a.sorted[n1 + k];
            if constexpr (D == 3) zj = a.sorted[n2 + k];
        } else {
            xj = a.pos[j];
            yj = a.pos[n1 + j];
            if constexpr (D == 3) zj = a.pos[n2 + j];
        }
        const float s = sqdist<D>(x, y, z, xj, yj, zj);
        if (j != i) t.push(s, j);
    }
}

// Lower bound on the distance from (x,y,z) to any point binned outside the
// box of cells [g-r, g+r]^d (sides at the grid edge are open: no cell lies
// beyond them).  Returns +inf when the box covers the whole grid.
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

template <int D, bool FRESH>
__device__ void search(const QueryArgs &a, float x, float y, float z, int i, double margin, Top2 &t)
{
    const int G = a.G;
    const int gx = cell_axis(x, G), gy = cell_axis(y, G), gz = D == 3 ? cell_axis(z, G) : 0;
    for (int r = 1;; ++r) {
        const int zlo = D == 3 ? max(gz - r, 0) : 0, zhi = D == 3 ? min(gz + r, G - 1) : 0;
        const int ylo = max(gy - r, 0), yhi = min(gy + r, G - 1);
        const int xlo = max(gx - r, 0), xhi = min(gx + r, G - 1);
        for (int cz = zlo; cz <= zhi; ++cz) {
            const bool zface = (D == 3) && (cz - gz == r || gz - cz == r);
            for (int cy = ylo; cy <= yhi; ++cy) {
                const int row = (cz * G + cy) * G;
                if (r == 1 || zface || cy - gy == r || gy - cy == r) {
                    visit<D, FRESH>(a, a.cell_start[row + xlo], a.cell_start[row + xhi + 1], x, y, z, i, t);
                } else {
                    if (gx - r >= 0) {
                        const int c = row + gx - r;
                        visit<D, FRESH>(a, a.cell_start[c], a.cell_start[c + 1], x, y, z, i, t);
                    }
                    if (gx + r <= G - 1) {
                        const int c = row + gx + r;
                        visit<D, FRESH>(a, a.cell_start[c], a.cell_start[c + 1], x, y, z, i, t);
                    }
                }
            }
        }
        const double B = outside_bound<D>(x, y, z, gx, gy, gz, r, G);
        if (__builtin_isinf(B)) break;  // the whole grid has been visited
        const double Be = B - margin;
        if (Be > 0.0 && (double)t.s2 < Be * Be * (1.0 - kRel)) break;
    }
}

template <int D, bool FRESH>
__global__ void __launch_bounds__(kB) k_query(QueryArgs a)
{
    const int count = a.all ? a.n : min(*a.count_dev, a.n);
    const double St = a.sc->S[a.parity];
    const double drift = FRESH ? 0.0 : St - a.sc->S_grid;
    const double margin = kFuzz + drift * (1.0 + kRel);
    const size_t n1 = (size_t)a.n, n2 = 2 * (size_t)a.n;
    for (int q = blockIdx.x * kB + threadIdx.x; q < count; q += gridDim.x * kB) {
        const int i = a.all ? a.perm[q] : a.list[q];
        if (i < 0 || i >= a.n) continue;  // caller-supplied lists are checked
        float x, y, z = 0.f;
        if (FRESH && a.all) {
            x = a.sorted[q];
            y = a.sorted[n1 + q];
            if constexpr (D == 3) z = a.sorted[n2 + q];
        } else {
            x = a.pos[i];
            y = a.pos[n1 + i];
            if constexpr (D == 3) z = a.pos[n2 + i];
        }
        Top2 t;
        t.init();
        search<D, FRESH>(a, x, y, z, i, margin, t);
        const int old = a.nn[i];
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

__global__ void __launch_bounds__(1024) k_entropy(int which, int *__restrict__ hist, const int *__restrict__ touched,
                                                  DevScalars *sc)
{
    __shared__ double s_acc[16];
    const int m = which == 0 ? sc->ntouched : sc->ncand_touched;
    const int F = which == 0 ? sc->nfail : sc->nfront;
    double acc = 0.0;
    for (int k = threadIdx.x; k < m; k += 1024) {
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
        for (int k = 0; k < 16; ++k) tot += s_acc[k];
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

inline int grid_cap(long long n)
{
    const long long b = (n + kB - 1) / kB;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

inline int check() { return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP; }

inline unsigned next_epoch(nnc_ctx *c)
{
    c->epoch = (c->epoch + 1u) & 0x3fffffffu;
    if (c->epoch == 0u) c->epoch = 1u;
    return c->epoch;
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
                           c->grid.counts, c->sc, parity);
    else
        hipLaunchKernelGGL(k_ingest<3>, dim3(blocks), dim3(kB), 0, c->stream, pold, pnew, (int)c->n, c->G, c->cell,
                           c->grid.counts, c->sc, parity);
    return check();
}

int launch_filter(nnc_ctx *c, float eps_declared)
{
    const int parity = (int)(c->t & 1);
    const int tiles = c->n > 0 ? blocks_for(c->n, kTile) : 1;
    hipLaunchKernelGGL(k_filter, dim3(tiles), dim3(kB), 0, c->stream, c->e, (int)c->n, c->sc, parity, eps_declared,
                       c->frontier, c->fail, c->status, next_epoch(c));
    return check();
}

int launch_grid_build(nnc_ctx *c, const float *pos)
{
    const int parity = (int)(c->t & 1);
    const int tiles = blocks_for(c->ncell, kTile);
    hipLaunchKernelGGL(k_scan_cells, dim3(tiles), dim3(kB), 0, c->stream, c->grid.counts, c->ncell,
                       c->grid.cell_start, c->grid.cursor, c->sc, parity, c->status, next_epoch(c));
    if (c->n > 0) {
        const int blocks = blocks_for(c->n, kB);
        if (c->d == 2)
            hipLaunchKernelGGL(k_scatter<2>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.perm, c->grid.sorted);
        else
            hipLaunchKernelGGL(k_scatter<3>, dim3(blocks), dim3(kB), 0, c->stream, pos, c->cell, (int)c->n,
                               c->grid.cursor, c->grid.perm, c->grid.sorted);
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
    a.fresh = c->grid_fresh;
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
    const int blocks = grid_cap(c->n);
    if (c->d == 2) {
        if (c->grid_fresh)
            hipLaunchKernelGGL((k_query<2, true>), dim3(blocks), dim3(kB), 0, c->stream, a);
        else
            hipLaunchKernelGGL((k_query<2, false>), dim3(blocks), dim3(kB), 0, c->stream, a);
    } else {
        if (c->grid_fresh)
            hipLaunchKernelGGL((k_query<3, true>), dim3(blocks), dim3(kB), 0, c->stream, a);
        else
            hipLaunchKernelGGL((k_query<3, false>), dim3(blocks), dim3(kB), 0, c->stream, a);
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
    hipLaunchKernelGGL(k_cand_hist, dim3(grid_cap(c->n)), dim3(kB), 0, c->stream, c->frontier, c->cell, c->hist_cand,
                       c->touched_cand, c->sc);
    return check();
}

int launch_audit(nnc_ctx *c)
{
    if (c->n == 0) return NNC_OK;
    hipLaunchKernelGGL(k_audit, dim3(blocks_for(c->n, kB)), dim3(kB), 0, c->stream, (int)c->n, c->nn, c->d1, c->d2,
                       c->stamp, (int)c->t, c->fail, c->a_nn, c->a_d1, c->a_d2, c->sc);
    hipLaunchKernelGGL(k_audit_cand, dim3(grid_cap(c->n)), dim3(kB), 0, c->stream, c->frontier, c->fail, c->sc);
    return check();
}

}  // namespace nnc
