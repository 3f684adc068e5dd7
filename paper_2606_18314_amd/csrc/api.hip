// C ABI of libnncert: context lifetime, the maintenance step, repair, rebuild,
// verification, entropy and snapshots.  Host code only; every computation is
// in the kernels of grid.hip and allpairs.hip.
#include <math.h>
#include <cmath>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.hpp"

using nnc::DevScalars;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxCells = 1 << 24;
constexpr int kRefreshSteps = 8;   // grid refresh interval when no eps bound is declared

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Carver {
    char *base;
    size_t off;
    template <class T>
    T *take(size_t count)
    {
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off = align_up(off + count * sizeof(T));
        return p;
    }
};

// Lay out every buffer of the context in one arena (base == nullptr: measure).
// The state that a snapshot must copy comes first.
size_t carve(nnc_ctx *c, char *base)
{
    const size_t n = (size_t)c->n > 0 ? (size_t)c->n : 1;
    const size_t nc = (size_t)c->ncell;
    Carver k{base, 0};
    c->sc = k.take<DevScalars>(1);
    c->nn = k.take<int32_t>(n);
    c->cell = k.take<int32_t>(n);
    c->stamp = k.take<int32_t>(n);
    c->d1 = k.take<float>(n);
    c->d2 = k.take<float>(n);
    c->e = k.take<double>(n);
    c->Si = k.take<double>(n);
    c->fail = k.take<uint8_t>(n);
    c->frontier = k.take<int32_t>(n);
    c->grid.counts = k.take<int>(nc);
    c->grid.cell_start = k.take<int>(nc + 1);
    c->grid.rank = k.take<int>(n);
    c->grid.slots = k.take<float4>(n);
    // histograms padded to whole int4 groups (the entropy scans them four cells at a time)
    c->hist_fail = k.take<int32_t>((nc + 3) / 4 * 4);
    c->hist_cand = k.take<int32_t>((nc + 3) / 4 * 4);
    c->last_move = k.take<int32_t>(nc);
    c->state_bytes = k.off;
    c->sync = k.take<nnc::DevSync>(1);
    c->grid.cursor = k.take<int>(nc);
    // one descriptor per look-back tile (512 or 2048 items of the filter, 4096 of the cell
    // scan; sized for 2048 here, which covers both)
    const size_t tf = (n + 511) / 512, tc = (nc + 2047) / 2048;
    const size_t tiles = (tf > tc ? tf : tc) + 1;
    c->nstatus = (int)tiles;
    c->status = k.take<unsigned long long>(tiles);
    c->wide = k.take<int32_t>(n);
    c->rec = k.take<int4>(n);
    c->cmask = k.take<uint8_t>(n);
    c->ntcount = (int)(((n + 4095) / 4096 + 1 + 3) & ~3ll);  // whole groups of four (k_filter_offsets)
    c->tcount = k.take<int32_t>((size_t)c->ntcount);
    c->nfmask = (long long)((n + 4095) / 4096 + 1) * 64;
    c->fmask = k.take<unsigned long long>((size_t)c->nfmask);
    c->ent_part = k.take<double>(3 * nnc::kEntropyParts);
    c->shape_part = k.take<double>(4 * nnc::kShapeParts + 4);
    if (c->flags & NNC_QUEUE) {
        c->q_cap = (int)(4 * n + 1024);
        c->qh = k.take<nnc::QHead>(1);
        c->q_pool = k.take<int32_t>((size_t)c->q_cap);
        c->q_pool_e = k.take<double>((size_t)c->q_cap);
        c->q_keep_e = k.take<double>(n);
        c->q_key = k.take<double>(n);
        c->q_nruns = k.take<int32_t>(nnc::kQR);
        c->q_run_start = k.take<int32_t>((size_t)nnc::kQR * nnc::kQRuns);
        c->q_run_len = k.take<int32_t>((size_t)nnc::kQR * nnc::kQRuns);
        c->q_bcnt = k.take<int32_t>(nnc::kQR);
        c->q_cursor = k.take<int32_t>(nnc::kQR);
        c->q_keep = k.take<int32_t>(n);
    }
    c->a_nn = k.take<int32_t>(n);
    c->a_d1 = k.take<float>(n);
    c->a_d2 = k.take<float>(n);
    c->rho = k.take<uint8_t>(n);
    if (c->flags & NNC_COPY_POSITIONS) {
        c->pos_copy[0] = k.take<float>(n * (size_t)c->d);
        c->pos_copy[1] = k.take<float>(n * (size_t)c->d);
    } else {
        c->pos_copy[0] = c->pos_copy[1] = nullptr;
    }
    return k.off;
}

int default_grid(int64_t n, int d)
{
    if (n <= 0) return 1;
    const double w = d == 2 ? 2.0 / sqrt((double)n) : cbrt(4.0 / (double)n);
    const double g = floor(1.0 / w);
    return g < 1.0 ? 1 : (int)g;
}

int sync_scalars(nnc_ctx *c, DevScalars *h)
{
    if (hipMemcpyAsync(h, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return NNC_E_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return NNC_E_HIP;
    return NNC_OK;
}

// Map and clear latched device errors.
int take_error(nnc_ctx *c, const DevScalars &h)
{
    if (h.err == 0u) return NNC_OK;
    const unsigned zero = 0u;
    (void)hipMemcpyAsync(&c->sc->err, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    if (h.err & nnc::kErrNonFinite) return NNC_E_NONFINITE;
    if (h.err & nnc::kErrEps) return NNC_E_EPS;
    return NNC_E_DEVICE;
}

const float *adopt_positions(nnc_ctx *c, const float *pos)
{
    if (!(c->flags & NNC_COPY_POSITIONS)) return pos;
    float *dst = c->pos_copy[c->copy_slot];
    c->copy_slot ^= 1;
    (void)hipMemcpyAsync(dst, pos, (size_t)c->n * (size_t)c->d * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
    return dst;
}

void prof_fold(nnc_ctx *c)
{
    if (c->prof_used == 0) return;
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < c->prof_used; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->prof_ev[2 * k], c->prof_ev[2 * k + 1]) == hipSuccess) {
            c->prof_ms[c->prof_cls[k]] += (double)ms;
            c->prof_cnt[c->prof_cls[k]] += 1;
        }
    }
    c->prof_used = 0;
}

// Run one launcher, bracketed by timing events when profiling is on.
template <class F>
int timed(nnc_ctx *c, int cls, F &&launch)
{
    if (!c->prof_on) return launch();
    if (c->prof_used == c->prof_cap) prof_fold(c);
    const int k = c->prof_used;
    (void)hipEventRecord(c->prof_ev[2 * k], c->stream);
    const int rc = launch();
    (void)hipEventRecord(c->prof_ev[2 * k + 1], c->stream);
    c->prof_cls[k] = cls;
    c->prof_used = k + 1;
    return rc;
}

int build_grid(nnc_ctx *c, bool from_slots = true)
{
    const int rc = timed(c, NNC_K_GRID, [&] { return nnc::launch_grid_build(c, c->pos_cur, from_slots); });
    c->grid_fresh = 1;
    c->drift_host = 0.0;
    c->steps_since_grid = 0;
    return rc;
}

}  // namespace

extern "C" {

const char *nnc_strerror(int code)
{
    switch (code) {
    case NNC_OK: return "ok";
    case NNC_E_INVAL: return "invalid argument";
    case NNC_E_NOMEM: return "device allocation failed";
    case NNC_E_HIP: return "HIP runtime error";
    case NNC_E_EPS: return "measured step exceeds the declared eps";
    case NNC_E_NONFINITE: return "non-finite coordinate";
    case NNC_E_STATE: return "call out of order";
    case NNC_E_DEVICE: return "device-side wait expired";
    default: return "unknown error";
    }
}

int nnc_create(nnc_ctx **out, const nnc_config *cfg)
{
    if (!out || !cfg) return NNC_E_INVAL;
    *out = nullptr;
    if (cfg->d != 2 && cfg->d != 3) return NNC_E_INVAL;
    if (cfg->n < 0 || cfg->n >= (int64_t)1 << 31) return NNC_E_INVAL;
    if ((cfg->flags & NNC_QUEUE) && ((cfg->flags & NNC_BUDGET) || cfg->n >= (int64_t)1 << 28)) return NNC_E_INVAL;
    const int G = cfg->grid_g > 0 ? cfg->grid_g : default_grid(cfg->n, cfg->d);
    const double cells = pow((double)G, (double)cfg->d);
    if (G < 1 || cells > (double)kMaxCells) return NNC_E_INVAL;
    // domain box: all zero = the unit box; else finite with hi > lo on every used axis
    bool unit = true;
    for (int k = 0; k < 3; ++k) unit = unit && cfg->lo[k] == 0.0f && cfg->hi[k] == 0.0f;
    float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {1.0f, 1.0f, 1.0f};
    if (!unit)
        for (int k = 0; k < cfg->d; ++k) {
            if (!std::isfinite(cfg->lo[k]) || !std::isfinite(cfg->hi[k]) || !(cfg->hi[k] > cfg->lo[k]))
                return NNC_E_INVAL;
            lo[k] = cfg->lo[k];
            hi[k] = cfg->hi[k];
        }
    nnc_ctx *c = new (std::nothrow) nnc_ctx();
    if (!c) return NNC_E_NOMEM;
    c->d = cfg->d;
    c->n = cfg->n;
    c->G = G;
    c->ncell = (int)cells;
    c->block = 256;
    c->lanes = cfg->block == 1 || cfg->block == 16 || cfg->block == 32 || cfg->block == 64 ? cfg->block
               : cfg->block == 8 || (cfg->block == 4 && cfg->d == 2)                        ? cfg->block
                                                                                             : (cfg->d == 3 ? 32 : 16);
    c->guard = cfg->guard < 0.0 ? 0x1p-18 : cfg->guard;
    c->K = 1.0 / (4.0 + 4.0 * c->guard);
    // cells: s = fl32(G / (hi - lo)) with the division in binary64, w = (hi - lo) / G;
    // the boundary-rounding allowance grows with the coordinates' magnitude
    double wmin = 1.0, mag = 1.0;
    for (int k = 0; k < 3; ++k) {
        const double width = (double)hi[k] - (double)lo[k];
        c->box.lo[k] = lo[k];
        c->box.s[k] = (float)((double)G / width);
        c->box.w[k] = width / (double)G;
        if (k < cfg->d) {
            wmin = fmin(wmin, width);
            mag = fmax(mag, fmax(fabs((double)lo[k]), fabs((double)hi[k])));
        }
    }
    c->fuzz = 0x1p-20 * mag;
    c->unit_box = unit;
    c->refresh_w = (cfg->refresh > 0.0 ? cfg->refresh : 0.25) * wmin / (double)G;
    c->stream = (hipStream_t)cfg->stream;
    c->flags = cfg->flags;
    c->grid.G = G;
    c->grid.ncell = c->ncell;
    c->arena_bytes = carve(c, nullptr);
    if (hipMalloc(&c->arena, c->arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return NNC_E_NOMEM;
    }
    carve(c, (char *)c->arena);
    if (hipMemsetAsync(c->arena, 0, c->arena_bytes, c->stream) != hipSuccess) {
        (void)hipFree(c->arena);
        delete c;
        return NNC_E_HIP;
    }
    *out = c;
    return NNC_OK;
}

void nnc_destroy(nnc_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->prof_ev) {
        for (int k = 0; k < 2 * c->prof_cap; ++k) (void)hipEventDestroy(c->prof_ev[k]);
        free(c->prof_ev);
        free(c->prof_cls);
    }
    (void)hipFree(c->arena);
    delete c;
}

int nnc_init_certificates(nnc_ctx *c, const float *pos)
{
    if (!c || (!pos && c->n > 0)) return NNC_E_INVAL;
    c->pos_cur = adopt_positions(c, pos);
    c->pos_prev = nullptr;
    c->t = 0;
    c->pending = 0;
    c->rho_step = -1;
    c->queue_valid = 0;
    c->fail_dirty = 1;
    // everything but the status words (whose epochs keep increasing) starts at zero
    if (hipMemsetAsync(c->arena, 0, c->state_bytes, c->stream) != hipSuccess) return NNC_E_HIP;
    int rc = nnc::launch_cells_init(c, c->pos_cur);
    if (rc == NNC_OK) rc = build_grid(c, false);  // no slot records yet
    if (rc == NNC_OK) rc = timed(c, NNC_K_QUERY, [&] { return nnc::launch_query_all(c, 1); });
    c->inited = rc == NNC_OK;
    return rc;
}

int nnc_step(nnc_ctx *c, const float *pos_new, float eps_declared, nnc_frontier *out)
{
    if (!c || (!pos_new && c->n > 0)) return NNC_E_INVAL;
    if (!c->inited || c->pending) return NNC_E_STATE;
    c->t += 1;
    c->pos_prev = c->pos_cur;
    c->pos_cur = adopt_positions(c, pos_new);
    int rc = timed(c, NNC_K_INGEST, [&] { return nnc::launch_ingest(c, c->pos_prev, c->pos_cur); });
    if (rc == NNC_OK && (c->flags & NNC_BUDGET))
        rc = timed(c, NNC_K_FILTER, [&] { return nnc::launch_budget(c); });
    if (rc == NNC_OK) {
        if ((c->flags & NNC_QUEUE) && c->queue_valid)
            rc = timed(c, NNC_K_FILTER, [&] { return nnc::launch_queue_pop(c, eps_declared); });
        else
            rc = timed(c, NNC_K_FILTER, [&] { return nnc::launch_filter(c, eps_declared); });
    }
    if (rc != NNC_OK) return rc;
    c->grid_fresh = 0;
    if (eps_declared >= 0.0f && c->drift_host >= 0.0)
        c->drift_host += (double)eps_declared * (1.0 + 0x1p-16) + 0x1p-20;
    else
        c->drift_host = -1.0;
    c->pending = 1;
    if (out) {
        out->idx_dev = c->frontier;
        out->count_dev = &c->sc->nfront;
        out->count_host = -1;
        out->step = (int32_t)c->t;
    }
    if (c->flags & NNC_SYNC) {
        DevScalars h;
        rc = sync_scalars(c, &h);
        if (rc != NNC_OK) return rc;
        if (out) out->count_host = h.nfront;
        return take_error(c, h);
    }
    return NNC_OK;
}

int nnc_repair(nnc_ctx *c, const nnc_frontier *f)
{
    if (!c) return NNC_E_INVAL;
    if (!c->pending) return NNC_E_STATE;
    if (f && (!f->idx_dev || !f->count_dev)) return NNC_E_INVAL;
    int rc = NNC_OK;
    const bool refresh = c->drift_host < 0.0 ? c->steps_since_grid >= kRefreshSteps : c->drift_host > c->refresh_w;
    if (refresh) rc = build_grid(c);
    if (rc == NNC_OK)
        rc = timed(c, NNC_K_QUERY, [&] {
            return nnc::launch_query(c, f ? f->idx_dev : c->frontier, f ? f->count_dev : &c->sc->nfront, 0, 0,
                                     (c->flags & NNC_QUEUE) && !f ? c->q_key : nullptr);
        });
    if (rc == NNC_OK) rc = timed(c, NNC_K_ENTROPY, [&] { return nnc::launch_entropy(c, 0); });
    // the calendar files the new keys (anew when it was not valid); after a caller's
    // list, whose points were not popped and whose fail flags the next pop would not
    // clear, the next step scans every key and the calendar is filed anew
    if (f) c->fail_dirty = 1;  // the caller's list set fail flags outside the candidate list
    if (rc == NNC_OK && (c->flags & NNC_QUEUE)) {
        if (f) {
            c->queue_valid = 0;
        } else {
            rc = timed(c, NNC_K_FILTER, [&] { return nnc::launch_queue_file(c, !c->queue_valid); });
            c->queue_valid = rc == NNC_OK;
        }
    }
    c->pending = 0;
    c->steps_since_grid += 1;
    return rc;
}

int nnc_rebuild(nnc_ctx *c)
{
    if (!c) return NNC_E_INVAL;
    if (!c->pending) return NNC_E_STATE;
    int rc = build_grid(c);
    if (rc == NNC_OK) rc = timed(c, NNC_K_QUERY, [&] { return nnc::launch_query_all(c, 0); });
    if (rc == NNC_OK) rc = timed(c, NNC_K_ENTROPY, [&] { return nnc::launch_entropy(c, 0); });
    // every key and any fail flag changed: the next step scans all keys (clearing every
    // flag) and its repair files the calendar anew
    c->queue_valid = 0;
    c->fail_dirty = 1;
    c->pending = 0;
    return rc;
}

int nnc_oracle_verify(nnc_ctx *c, nnc_audit *out)
{
    if (!c || !out) return NNC_E_INVAL;
    if (!c->inited) return NNC_E_STATE;
    int rc = nnc::launch_allpairs(c->pos_cur, c->n, c->d, nullptr, c->n, c->a_nn, c->a_d1, c->a_d2, c->stream);
    if (rc != NNC_OK) return rc;
    // the rho counter ([6]) belongs to nnc_rho_predict
    if (hipMemsetAsync(c->sc->audit, 0, 6 * sizeof(c->sc->audit[0]), c->stream) != hipSuccess ||
        hipMemsetAsync(&c->sc->audit[7], 0, sizeof(c->sc->audit[7]), c->stream) != hipSuccess)
        return NNC_E_HIP;
    rc = nnc::launch_audit(c);
    if (rc != NNC_OK) return rc;
    DevScalars h;
    rc = sync_scalars(c, &h);
    if (rc != NNC_OK) return rc;
    out->n_checked = c->n;
    out->n_detect = h.nfront;
    out->n_true_fail = (int64_t)h.audit[2];
    out->n_missed = (int64_t)h.audit[0];
    out->n_false = (int64_t)h.nfront - (int64_t)h.audit[5];
    out->n_value_mismatch = (int64_t)h.audit[1];
    out->nn_hash = h.audit[4];
    const bool rho = c->rho_step == c->t;
    out->rho_flagged = rho ? (int64_t)h.audit[6] : -1;
    out->rho_hit = rho ? (int64_t)h.audit[7] : -1;
    return take_error(c, h);
}

int nnc_rho_predict(nnc_ctx *c)
{
    if (!c) return NNC_E_INVAL;
    if (!c->pending || !c->pos_prev) return NNC_E_STATE;
    if (hipMemsetAsync(&c->sc->audit[6], 0, sizeof(c->sc->audit[6]), c->stream) != hipSuccess) return NNC_E_HIP;
    const int rc = nnc::launch_rho(c);
    if (rc == NNC_OK) c->rho_step = c->t;
    return rc;
}

int nnc_frontier_entropy(nnc_ctx *c, int which, nnc_entropy *out)
{
    if (!c || !out || (which != NNC_FAILED && which != NNC_CANDIDATES)) return NNC_E_INVAL;
    if (!c->inited) return NNC_E_STATE;
    int rc = NNC_OK;
    if (which == NNC_CANDIDATES) {
        rc = nnc::launch_cand_hist(c);
        if (rc == NNC_OK) rc = nnc::launch_entropy(c, 1);
        if (rc != NNC_OK) return rc;
    }
    DevScalars h;
    rc = sync_scalars(c, &h);
    if (rc != NNC_OK) return rc;
    out->eps = h.eps;
    out->S = h.S[c->t & 1];
    out->H = h.H[which];
    out->m = h.m[which];
    out->C = h.Cres[which];
    out->count = h.F[which];
    return take_error(c, h);
}

int nnc_queue_stats(nnc_ctx *c, int64_t *out)
{
    if (!c || !out) return NNC_E_INVAL;
    if (!(c->flags & NNC_QUEUE)) return NNC_E_STATE;
    nnc::QHead h;
    if (hipMemcpyAsync(&h, c->qh, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return NNC_E_HIP;
    out[0] = (int64_t)h.n_pop;
    out[1] = (int64_t)h.n_scan;
    out[2] = (int64_t)h.n_build;
    out[3] = (int64_t)h.n_read;
    out[4] = (int64_t)h.pool_top;
    out[5] = (int64_t)h.far_count;
    return NNC_OK;
}

int nnc_frontier_gyration(nnc_ctx *c, int which, double *gyration, double *centroid)
{
    if (!c || !gyration || (which != NNC_FAILED && which != NNC_CANDIDATES)) return NNC_E_INVAL;
    if (!c->inited) return NNC_E_STATE;
    std::vector<double> part(4 * nnc::kShapeParts);
    double sums[4] = {0.0, 0.0, 0.0, 0.0}, cen[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t pbytes = part.size() * sizeof(double);
    int rc = c->n > 0 ? nnc::launch_shape(c, which, nullptr) : NNC_OK;
    if (rc == NNC_OK && c->n > 0) {
        if (hipMemcpyAsync(part.data(), c->shape_part, pbytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return NNC_E_HIP;
        for (int b = 0; b < nnc::kShapeParts; ++b)
            for (int k = 0; k < 4; ++k) sums[k] += part[4 * b + k];
    }
    if (rc != NNC_OK) return rc;
    double g = 0.0;
    if (sums[3] > 0.0) {
        for (int k = 0; k < 3; ++k) cen[k] = sums[k] / sums[3];
        double *cen_dev = c->shape_part + 4 * nnc::kShapeParts;
        if (hipMemcpyAsync(cen_dev, cen, 4 * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return NNC_E_HIP;
        rc = nnc::launch_shape(c, which, cen_dev);
        if (rc != NNC_OK) return rc;
        if (hipMemcpyAsync(part.data(), c->shape_part, pbytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return NNC_E_HIP;
        double ss = 0.0;
        for (int b = 0; b < nnc::kShapeParts; ++b) ss += part[4 * b];
        g = sqrt(ss / sums[3]);
    }
    *gyration = g;
    if (centroid)
        for (int k = 0; k < 3; ++k) centroid[k] = cen[k];
    return NNC_OK;
}

int nnc_features(nnc_ctx *c, float *out)
{
    if (!c || !out) return NNC_E_INVAL;
    if (!c->inited || !c->pending) return NNC_E_STATE;
    int rc = nnc::launch_cand_hist(c);
    if (rc == NNC_OK) rc = nnc::launch_entropy(c, 1);
    if (rc == NNC_OK) rc = nnc::launch_features(c, out);
    return rc;
}

int nnc_get_state(nnc_ctx *c, nnc_state *v)
{
    if (!c || !v) return NNC_E_INVAL;
    v->nn = c->nn;
    v->d1 = c->d1;
    v->d2 = c->d2;
    v->e = c->e;
    v->cell = c->cell;
    v->fail = c->fail;
    v->n = c->n;
    v->d = c->d;
    v->grid_g = c->G;
    v->rho = c->rho;
    v->Si = c->Si;
    return NNC_OK;
}

int nnc_snapshot(nnc_ctx *c, nnc_snap **out)
{
    if (!c || !out) return NNC_E_INVAL;
    nnc_snap *s = new (std::nothrow) nnc_snap();
    if (!s) return NNC_E_NOMEM;
    s->bytes = c->state_bytes;
    if (hipMalloc(&s->dev, s->bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return NNC_E_NOMEM;
    }
    if (hipMemcpyAsync(s->dev, c->arena, s->bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
        (void)hipFree(s->dev);
        delete s;
        return NNC_E_HIP;
    }
    s->t = c->t;
    s->pending = c->pending;
    s->grid_fresh = c->grid_fresh;
    s->drift_host = c->drift_host;
    s->steps_since_grid = c->steps_since_grid;
    s->pos_cur = c->pos_cur;
    s->pos_prev = c->pos_prev;
    *out = s;
    return NNC_OK;
}

int nnc_snapshot_update(nnc_ctx *c, nnc_snap *s)
{
    if (!c || !s || s->bytes != c->state_bytes) return NNC_E_INVAL;
    if (hipMemcpyAsync(s->dev, c->arena, s->bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return NNC_E_HIP;
    s->t = c->t;
    s->pending = c->pending;
    s->grid_fresh = c->grid_fresh;
    s->drift_host = c->drift_host;
    s->steps_since_grid = c->steps_since_grid;
    s->pos_cur = c->pos_cur;
    s->pos_prev = c->pos_prev;
    return NNC_OK;
}

int nnc_restore(nnc_ctx *c, const nnc_snap *s)
{
    if (!c || !s || s->bytes != c->state_bytes) return NNC_E_INVAL;
    if (hipMemcpyAsync(c->arena, s->dev, s->bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return NNC_E_HIP;
    c->t = s->t;
    c->pending = s->pending;
    c->grid_fresh = s->grid_fresh;
    c->drift_host = s->drift_host;
    c->pos_cur = s->pos_cur;
    c->pos_prev = s->pos_prev;
    c->steps_since_grid = s->steps_since_grid;
    c->rho_step = -1;
    c->queue_valid = 0;  // the calendar is not part of a snapshot: the next step scans every key
    c->fail_dirty = 1;
    return NNC_OK;
}

void nnc_snap_free(nnc_snap *s)
{
    if (!s) return;
    (void)hipFree(s->dev);
    delete s;
}

int nnc_profile_enable(nnc_ctx *c, int enable)
{
    if (!c) return NNC_E_INVAL;
    if (enable && !c->prof_ev) {
        const int cap = 256;
        c->prof_ev = (hipEvent_t *)calloc(2 * cap, sizeof(hipEvent_t));
        c->prof_cls = (int *)calloc(cap, sizeof(int));
        if (!c->prof_ev || !c->prof_cls) return NNC_E_NOMEM;
        for (int k = 0; k < 2 * cap; ++k)
            if (hipEventCreate(&c->prof_ev[k]) != hipSuccess) return NNC_E_HIP;
        c->prof_cap = cap;
    }
    if (!enable) prof_fold(c);
    c->prof_on = enable ? 1 : 0;
    return NNC_OK;
}

int nnc_profile_read(nnc_ctx *c, nnc_profile *out, int reset)
{
    if (!c || !out) return NNC_E_INVAL;
    prof_fold(c);
    for (int k = 0; k < NNC_K_COUNT; ++k) {
        out->ms[k] = c->prof_ms[k];
        out->count[k] = c->prof_cnt[k];
        if (reset) {
            c->prof_ms[k] = 0.0;
            c->prof_cnt[k] = 0;
        }
    }
    return NNC_OK;
}

int nnc_allpairs_top2(const float *pos, int64_t n, int32_t d, const int32_t *qidx, int64_t nq, int32_t *nn,
                      float *d1, float *d2, void *stream)
{
    if ((d != 2 && d != 3) || n < 0 || n >= (int64_t)1 << 31 || nq < 0) return NNC_E_INVAL;
    if (!qidx && nq != n) return NNC_E_INVAL;
    if (nq > 0 && (!pos || !nn || !d1 || !d2)) return NNC_E_INVAL;
    return nnc::launch_allpairs(pos, n, d, qidx, nq, nn, d1, d2, (hipStream_t)stream);
}

int nnc_sqrt_f32(const float *x, float *out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!x || !out))) return NNC_E_INVAL;
    return nnc::launch_sqrt(x, out, n, (hipStream_t)stream);
}

}  // extern "C"
