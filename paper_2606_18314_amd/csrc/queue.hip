// Expiry calendar queue for the safety filter, for gfx950 (NNC_QUEUE).
//
// The appendix keeps the points in a min-heap keyed by their expiry S_i + c_i/4
// and pops the expired keys each step, so that detection costs O(|F_t| log N)
// instead of a scan of all N keys (Theorem 3).  A heap is a sequential
// structure; its GPU counterpart here is a calendar: keys are filed in a ring of
// kQR buckets of width W in clock units, and a step pops the buckets the clock
// has reached.  The work of a step is proportional to the entries of those
// buckets and the filing of the repaired points, not to N.
//
//   k_q_clear      clear the fail flags of the previous step's candidates (the
//                  only ones its repair set) and the pop counters;
//   k_q_pop        advance the clock (as the filter does) and read the runs of
//                  the buckets [a_next, a_hi] the clock reached: an entry whose
//                  key is due becomes a candidate, one that is not (the last
//                  bucket is reached part way) is kept for filing again; when the
//                  clock ran past the ring or reached the far set's smallest key,
//                  every key is scanned instead and the calendar is rebuilt;
//   k_q_after_pop  publish the candidate count, empty the popped buckets;
// and after the repair (or rebuild) wrote the new keys:
//   k_q_file_begin choose between appending and rebuilding the calendar (pool or
//                  run table full, a fallback pop, or the host's request), and
//                  reset it for a rebuild with W = 2 eps_t;
//   k_q_file_count bucket of every item (candidates and kept entries, or all
//                  points for a rebuild), counted per bucket in LDS, the far set's
//                  smallest key;
//   k_q_file_runs  one workgroup: each bucket's new run in the pool;
//   k_q_file_put   the items written into their runs.
// Every entry carries its point's key, and the repair writes the new keys in
// list order (beside the candidate list), so pops and filings read and write
// contiguous runs and never gather keys by point index (except after a tiled
// repair, whose keys are read from the state).  Candidates come out in bucket
// order, not in index order.  A bucket is emptied when it is popped and every
// point is filed exactly once between builds (the host rebuilds the calendar
// after anything that changes keys of points that were not popped).
#include <math.h>

#include "device_common.hpp"
#include "internal.hpp"
#include "kernels_common.hpp"

namespace nnc {

namespace {

using namespace kc;

constexpr int kQB = 256;       // threads per workgroup (one entry each per chunk)
constexpr int kQPop = 512;     // workgroups of the pop and filing kernels

// Relative bucket of a key for filing: at least the clock's bucket a_hi; -1 for
// the far set (kQAhead or more buckets past a_hi); -2 for an infinite key.
__device__ __forceinline__ int file_bucket(double e, double W, long long a_epoch, int a_hi)
{
    if (!(e < __builtin_inf())) return -2;
    double a = floor(e / W) - (double)a_epoch;
    const double lo = (double)a_hi;
    if (a < lo) a = lo;
    if (a >= lo + (double)kQAhead) return -1;
    return (int)a;
}

// Point and key of filing item q: every point for a rebuild (mode 1), else the
// candidates (their new keys in list order, or from the state after a tiled
// repair) then the kept entries.  Point -1 past the end.
struct FileArgs {
    int mode, n, nf, nk;
    bool keys_in_list;
    const int *frontier, *keep;
    const double *e, *qkey, *keep_e;
};

__device__ __forceinline__ int file_item(int q, const FileArgs &f, double &key)
{
    if (f.mode) {
        if (q >= f.n) return -1;
        key = f.e[q];
        return q;
    }
    if (q < f.nf) {
        const int i = f.frontier[q];
        key = f.keys_in_list ? f.qkey[q] : (i >= 0 && i < f.n ? f.e[i] : 0.0);
        return i;
    }
    if (q - f.nf < f.nk) {
        key = f.keep_e[q - f.nf];
        return f.keep[q - f.nf];
    }
    return -1;
}

__device__ __forceinline__ FileArgs file_args(const QHead *qh, const DevScalars *sc, int n, int tiled_from,
                                              const int *frontier, const int *keep, const double *e,
                                              const double *qkey, const double *keep_e)
{
    FileArgs f;
    f.mode = qh->mode;
    f.n = n;
    f.nf = sc->nfront;
    f.nk = qh->nkeep;
    f.keys_in_list = !(tiled_from > 0 && min(f.nf, n) >= tiled_from);
    f.frontier = frontier;
    f.keep = keep;
    f.e = e;
    f.qkey = qkey;
    f.keep_e = keep_e;
    return f;
}

__global__ void __launch_bounds__(kQB) k_q_clear(const int *__restrict__ frontier, const int *__restrict__ count,
                                                 int n, uint8_t *__restrict__ fail, QHead *qh, int parity)
{
    const int m = *count;
    for (int q = blockIdx.x * kQB + (int)threadIdx.x; q < m; q += gridDim.x * kQB) {
        const int i = frontier[q];
        if (i >= 0 && i < n) fail[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        qh->cnt[parity] = 0;
        qh->nkeep = 0;
        qh->fallback = 0;
    }
}

// One chunk of up to kQB entries (i < 0: none) through the workgroup: due entries
// appended to the candidates, kept ones to the keep list, one atomic each.
__device__ __forceinline__ void append_chunk(int i, double key, bool due, bool kp, int n, QHead *qh, int parity,
                                             int *__restrict__ frontier, int *__restrict__ keep,
                                             double *__restrict__ keep_e, DevScalars *sc, int *s_w, int *s_base)
{
    int tot;
    const int ex = block_excl_scan<kQB>((due ? 1 : 0) + (kp ? 0x10000 : 0), s_w, tot);
    if (threadIdx.x == 0) {
        s_base[0] = (tot & 0xffff) ? atomicAdd(&qh->cnt[parity], tot & 0xffff) : 0;
        s_base[1] = (tot >> 16) ? atomicAdd(&qh->nkeep, tot >> 16) : 0;
    }
    __syncthreads();
    if (due) {
        const int at = s_base[0] + (ex & 0xffff);
        if (at < n) frontier[at] = i;
        else atomicOr(&sc->err, kErrOverflow);
    }
    if (kp) {
        const int at = s_base[1] + (ex >> 16);
        if (at < n) {
            keep[at] = i;
            keep_e[at] = key;
        } else {
            atomicOr(&sc->err, kErrOverflow);
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kQB) k_q_pop(const double *__restrict__ e, int n, DevScalars *sc, int parity,
                                               float eps_decl, QHead *qh, const int *__restrict__ pool,
                                               const double *__restrict__ pool_e, const int *__restrict__ nruns,
                                               const int *__restrict__ run_start, const int *__restrict__ run_len,
                                               int *__restrict__ frontier, int *__restrict__ keep,
                                               double *__restrict__ keep_e)
{
    __shared__ int s_w[kQB / 64];
    __shared__ int s_base[2];
    const double St = advance_clock(sc, parity, eps_decl, blockIdx.x == 0 && threadIdx.x < 64);
    const double ah = floor(St / qh->W) - (double)qh->a_epoch;
    const int a_lo = qh->a_next;
    const double far_min = __longlong_as_double((long long)qh->far_min);
    const bool scan_all = !(ah >= (double)a_lo) || ah - (double)a_lo >= (double)kQR || ah >= 1073741824.0 ||
                          !(far_min > St);
    if (scan_all) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            qh->fallback = 1;
            qh->n_scan += 1;
        }
        for (int base = blockIdx.x * kQB; base < n; base += gridDim.x * kQB) {
            const int i = base + (int)threadIdx.x;
            const bool due = i < n && St >= e[i];
            append_chunk(i, 0.0, due, false, n, qh, parity, frontier, keep, keep_e, sc, s_w, s_base);
        }
        return;
    }
    const int a_hi = (int)ah;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        qh->a_hi = a_hi;
        qh->n_pop += 1;
    }
    int chunk = 0;
    unsigned long long read = 0;
    for (int a = a_lo; a <= a_hi; ++a) {
        const int r = a & (kQR - 1);
        const int nr = nruns[r];
        for (int j = 0; j < nr; ++j) {
            const int st = run_start[r * kQRuns + j], len = run_len[r * kQRuns + j];
            for (int off = 0; off < len; off += kQB, ++chunk) {
                if (chunk % (int)gridDim.x != (int)blockIdx.x) continue;
                read += (unsigned long long)min(kQB, len - off);
                const int q = off + (int)threadIdx.x;
                int i = -1;
                double key = 0.0;
                bool due = false, kp = false;
                if (q < len) {
                    i = pool[st + q];
                    key = pool_e[st + q];
                    if (i >= 0 && i < n) {
                        due = St >= key;
                        kp = !due;
                    }
                }
                append_chunk(i, key, due, kp, n, qh, parity, frontier, keep, keep_e, sc, s_w, s_base);
            }
        }
    }
    if (threadIdx.x == 0 && read) atomicAdd(&qh->n_read, read);
}

__global__ void __launch_bounds__(kQB) k_q_after_pop(DevScalars *sc, QHead *qh, int parity, int *__restrict__ nruns)
{
    const int fb = qh->fallback;
    const int a_lo = qh->a_next, a_hi = qh->a_hi;
    __syncthreads();
    if (fb) {
        if (threadIdx.x == 0) {
            sc->nfront = qh->cnt[parity];
            qh->build = 1;
        }
        return;
    }
    for (int a = a_lo + (int)threadIdx.x; a <= a_hi; a += kQB) nruns[a & (kQR - 1)] = 0;
    if (threadIdx.x == 0) {
        sc->nfront = qh->cnt[parity];
        qh->a_next = a_hi;
    }
}

__global__ void __launch_bounds__(kQB) k_q_file_begin(const DevScalars *sc, QHead *qh, int parity, int force, int n,
                                                      int cap, int *__restrict__ nruns, int *__restrict__ bcnt)
{
    __shared__ int s_full;
    if (threadIdx.x == 0) s_full = 0;
    __syncthreads();
    int full = 0;
    for (int r = threadIdx.x; r < kQR; r += kQB) full |= nruns[r] >= kQRuns - 1;
    if (full) atomicOr(&s_full, 1);
    __syncthreads();
    const int items = sc->nfront + qh->nkeep;
    const bool build = force || qh->build || s_full || qh->pool_top + items > cap;
    for (int r = threadIdx.x; r < kQR; r += kQB) {
        bcnt[r] = 0;
        if (build) nruns[r] = 0;
    }
    if (threadIdx.x == 0) {
        qh->mode = build ? 1 : 0;
        if (build) {
            qh->n_build += 1;
            const double St = sc->S[parity];
            const double W = fmax(2.0 * sc->eps, 0x1p-40);
            qh->W = W;
            qh->a_epoch = (long long)floor(St / W);
            qh->pool_top = 0;
            qh->a_next = 0;
            qh->a_hi = 0;
            qh->far_min = (unsigned long long)__double_as_longlong(__builtin_inf());
            qh->far_count = 0;
            qh->build = 0;
        }
    }
}

__global__ void __launch_bounds__(kQB) k_q_file_count(const double *__restrict__ e, int n,
                                                      const DevScalars *__restrict__ sc, QHead *qh, int tiled_from,
                                                      const int *__restrict__ frontier, const int *__restrict__ keep,
                                                      const double *__restrict__ qkey,
                                                      const double *__restrict__ keep_e, int *__restrict__ bcnt)
{
    __shared__ int s_h[kQAhead];
    const FileArgs fa = file_args(qh, sc, n, tiled_from, frontier, keep, e, qkey, keep_e);
    const int items = fa.mode ? n : fa.nf + fa.nk;
    const double W = qh->W;
    const long long a_ep = qh->a_epoch;
    const int a_hi = qh->a_hi;
    for (int k = threadIdx.x; k < kQAhead; k += kQB) s_h[k] = 0;
    __syncthreads();
    double fmin_local = __builtin_inf();
    int nfar = 0;
    for (int q = blockIdx.x * kQB + (int)threadIdx.x; q < items; q += gridDim.x * kQB) {
        double ei = 0.0;
        const int i = file_item(q, fa, ei);
        if (i < 0 || i >= n) continue;
        const int b = file_bucket(ei, W, a_ep, a_hi);
        if (b >= 0) {
            atomicAdd(&s_h[b - a_hi], 1);
        } else if (b == -1) {
            fmin_local = fmin(fmin_local, ei);
            ++nfar;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) fmin_local = fmin(fmin_local, __shfl_xor(fmin_local, off, 64));
    nfar = wave_sum(nfar);
    if (lane_id() == 0) {
        if (fmin_local < __builtin_inf())
            atomicMin(&qh->far_min, (unsigned long long)__double_as_longlong(fmin_local));
        if (nfar) atomicAdd(&qh->far_count, nfar);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kQAhead; k += kQB)
        if (s_h[k]) atomicAdd(&bcnt[(a_hi + k) & (kQR - 1)], s_h[k]);
}

__global__ void __launch_bounds__(kQB) k_q_file_runs(QHead *qh, int cap, int *__restrict__ nruns,
                                                     int *__restrict__ run_start, int *__restrict__ run_len,
                                                     const int *__restrict__ bcnt, int *__restrict__ cursor,
                                                     DevScalars *sc)
{
    __shared__ int s_w[kQB / 64];
    const int top = qh->pool_top;
    int run = 0;
    for (int base = 0; base < kQR; base += kQB) {
        const int r = base + (int)threadIdx.x;
        const int v = r < kQR ? bcnt[r] : 0;
        int tot;
        const int ex = block_excl_scan<kQB>(v, s_w, tot);
        if (v > 0) {
            const int at = top + run + ex, j = nruns[r];
            if (at + v <= cap && j < kQRuns) {
                run_start[r * kQRuns + j] = at;
                run_len[r * kQRuns + j] = v;
                nruns[r] = j + 1;
                cursor[r] = at;
            } else {
                cursor[r] = -1;
                atomicOr(&sc->err, kErrOverflow);
            }
        }
        run += tot;
    }
    if (threadIdx.x == 0) qh->pool_top = top + run;
}

__global__ void __launch_bounds__(kQB) k_q_file_put(const double *__restrict__ e, int n,
                                                    const DevScalars *__restrict__ sc, const QHead *__restrict__ qh,
                                                    int tiled_from, const int *__restrict__ frontier,
                                                    const int *__restrict__ keep, const double *__restrict__ qkey,
                                                    const double *__restrict__ keep_e, int *__restrict__ cursor,
                                                    int *__restrict__ pool, double *__restrict__ pool_e, int cap)
{
    __shared__ int s_c[kQAhead];
    __shared__ int s_base[kQAhead];
    const FileArgs fa = file_args(qh, sc, n, tiled_from, frontier, keep, e, qkey, keep_e);
    const int items = fa.mode ? n : fa.nf + fa.nk;
    const double W = qh->W;
    const long long a_ep = qh->a_epoch;
    const int a_hi = qh->a_hi;
    for (int base = blockIdx.x * kQB; base < items; base += gridDim.x * kQB) {
        for (int k = threadIdx.x; k < kQAhead; k += kQB) s_c[k] = 0;
        __syncthreads();
        const int q = base + (int)threadIdx.x;
        double key = 0.0;
        const int i = q < items ? file_item(q, fa, key) : -1;
        int b = -1, rank = 0;
        if (i >= 0 && i < n) {
            b = file_bucket(key, W, a_ep, a_hi);
            if (b >= 0) rank = atomicAdd(&s_c[b - a_hi], 1);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kQAhead; k += kQB) {
            const int c = s_c[k];
            int at = -1;
            if (c) {
                const int r = (a_hi + k) & (kQR - 1);
                at = cursor[r] >= 0 ? atomicAdd(&cursor[r], c) : -1;
            }
            s_base[k] = at;
        }
        __syncthreads();
        if (b >= 0) {
            const int at = s_base[b - a_hi];
            if (at >= 0 && at + rank < cap) {
                pool[at + rank] = i;
                pool_e[at + rank] = key;
            }
        }
        __syncthreads();
    }
}

inline int check() { return hipGetLastError() == hipSuccess ? NNC_OK : NNC_E_HIP; }

}  // namespace

int launch_queue_pop(nnc_ctx *c, float eps_declared)
{
    const int parity = (int)(c->t & 1);
    const int n = (int)c->n;
    const int cb = (n + kQB - 1) / kQB;
    const int clear_blocks = cb < 1 ? 1 : (cb < 1024 ? cb : 1024);
    hipLaunchKernelGGL(k_q_clear, dim3(clear_blocks), dim3(kQB), 0, c->stream, c->frontier, &c->sc->nfront, n, c->fail,
                       c->qh, parity);
    hipLaunchKernelGGL(k_q_pop, dim3(kQPop), dim3(kQB), 0, c->stream, c->e, n, c->sc, parity, eps_declared, c->qh,
                       c->q_pool, c->q_pool_e, c->q_nruns, c->q_run_start, c->q_run_len, c->frontier, c->q_keep,
                       c->q_keep_e);
    hipLaunchKernelGGL(k_q_after_pop, dim3(1), dim3(kQB), 0, c->stream, c->sc, c->qh, parity, c->q_nruns);
    return check();
}

int launch_queue_file(nnc_ctx *c, int build)
{
    const int parity = (int)(c->t & 1);
    const int n = (int)c->n;
    hipLaunchKernelGGL(k_q_file_begin, dim3(1), dim3(kQB), 0, c->stream, c->sc, c->qh, parity, build, n, c->q_cap,
                       c->q_nruns, c->q_bcnt);
    const int from = tiled_repair_from(c);
    hipLaunchKernelGGL(k_q_file_count, dim3(kQPop), dim3(kQB), 0, c->stream, c->e, n, c->sc, c->qh, from, c->frontier,
                       c->q_keep, c->q_key, c->q_keep_e, c->q_bcnt);
    hipLaunchKernelGGL(k_q_file_runs, dim3(1), dim3(kQB), 0, c->stream, c->qh, c->q_cap, c->q_nruns, c->q_run_start,
                       c->q_run_len, c->q_bcnt, c->q_cursor, c->sc);
    hipLaunchKernelGGL(k_q_file_put, dim3(kQPop), dim3(kQB), 0, c->stream, c->e, n, c->sc, c->qh, from, c->frontier,
                       c->q_keep, c->q_key, c->q_keep_e, c->q_cursor, c->q_pool, c->q_pool_e, c->q_cap);
    return check();
}

}  // namespace nnc
