// Internal declarations of libnncert: the context, the device scalar block and
// the host-side launchers of each kernel family.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nncert.h"
#include "device_common.hpp"

namespace nnc {

// Bits of the device error word.
enum : unsigned { kErrNonFinite = 1u, kErrEps = 2u, kErrSpin = 4u, kErrOverflow = 8u };

constexpr int kEntropyParts = 256;  // workgroups of the split entropy reduction
constexpr int kShapeParts = 256;    // workgroups of the frontier gyration sums

// Scalars that live on the device so that a step never waits for the host.
// The clock and the displacement maximum are double-buffered by step parity:
// step t reads S[(t-1)&1], writes S[t&1]; its ingest accumulates into dmax[t&1].
struct DevScalars {
    double S[2];
    double S_grid;           // clock when the grid index was last built
    double eps;              // eps_t of the last step
    unsigned dmax[2];        // largest squared displacement (float bits), per parity
    int C;                   // occupied cells
    int nfront;              // candidates of the last step
    int nfail;               // failures of the last repair/rebuild
    int ntouched;            // cells met by those failures
    int ncand_touched;       // cells met by the candidates (on demand)
    unsigned err;            // kErr* bits
    int nwide;               // all-point query: points left to the widening pass
    int pad1;
    // results of the entropy kernel: [0] failures, [1] candidates
    double H[2];
    int m[2];
    int F[2];
    int Cres[2];
    // audit counters
    // [0] missed, [1] value mismatches, [2] failures, [3] fresh, [4] nn hash,
    // [5] candidates that failed, [6] rho-flagged points, [7] flagged that failed
    unsigned long long audit[8];
    // ingest results spread over kSpread words (workgroup b adds into slot b % kSpread),
    // folded by the filter's leading wave: displacement maxima per parity, and
    // changes of the occupied-cell count
    unsigned dmax_part[2][64];
    int dC_part[64];
};

// Ticket counter and epoch of the look-back scans.  Kept outside the state that
// init clears and snapshots copy: the epoch only ever increases, so tile
// descriptors left by earlier scans (or earlier graph replays) never match.
struct DevSync {
    unsigned epoch;
    unsigned tile_ctr;
};

// Expiry calendar queue (NNC_QUEUE): every finite expiry key is filed in a ring of
// kQR buckets of width W (clock units) starting at bucket a_epoch, or, more than
// kQAhead buckets past the clock, in a far set whose smallest key is kept.  A
// bucket is a list of runs (start, length) in an append-only pool; each filing
// adds at most one run per bucket.  See queue.hip.
constexpr int kQR = 512;        // ring buckets
constexpr int kQAhead = 256;    // buckets past the clock's bucket that the ring files
constexpr int kQRuns = 512;     // runs per bucket

struct QHead {
    double W;                   // bucket width
    long long a_epoch;          // absolute bucket floor(e / W) of relative bucket 0
    unsigned long long far_min; // bits of the smallest key in the far set (keys >= 0)
    int pool_top;               // entries used in the pool
    int a_next;                 // first relative bucket not yet fully popped
    int a_hi;                   // relative bucket of S_t at the last pop or build
    int cnt[2];                 // entries popped as candidates, by step parity
    int nkeep;                  // popped entries not yet due (filed again after the repair)
    int build;                  // 1: the next filing rebuilds the whole calendar
    int mode;                   // this filing: 0 appends, 1 rebuilds
    int far_count;
    int fallback;               // this step's pop scanned every key
    // counters since creation: steps that popped buckets, steps that scanned every
    // key, calendars filed anew, entries the pops read
    unsigned long long n_pop, n_scan, n_build, n_read;
};

// Loose uniform grid: slots are grouped by the cell each point had when the grid
// was last built; slot k holds one 16-byte record {x, y, z, point index} with the
// point's CURRENT coordinates (z = 0 in the plane; ingest rewrites the record
// every step through rank[]), and queries widen their search by the motion
// accumulated since the build.
struct Grid {
    int G, ncell;
    int *counts;        // [ncell] occupancy of current cells
    int *cell_start;    // [ncell+1] slot ranges of the build-time cells
    int *cursor;        // [ncell] scatter cursors
    int *rank;          // [n] point index -> slot
    float4 *slots;      // [n] slot records {x, y, z, bits of the point index}
};

}  // namespace nnc

struct nnc_snap {
    size_t bytes;
    void *dev;
    int64_t t;
    int pending;
    int grid_fresh;
    double drift_host;
    int steps_since_grid;
    const float *pos_cur;
    const float *pos_prev;
};

struct nnc_ctx {
    int d, G, ncell, block;
    int64_t n;
    double guard, K, refresh_w;
    nnc::Box box;                 // domain box of the cells
    bool unit_box;                // the box is [0,1]^d (queries use the folded formula)
    double fuzz;                  // cell-boundary rounding allowance of the queries
    hipStream_t stream;
    uint32_t flags;

    // state, original point order
    int32_t *nn, *cell, *stamp;
    float *d1, *d2;
    double *e;
    double *Si;                   // clock at which each certificate was computed
    uint8_t *fail;
    // grid index
    nnc::Grid grid;
    // frontier and histograms
    int32_t *frontier;
    int32_t *hist_fail, *hist_cand;   // per-cell counts of failures / candidates
    int32_t *last_move;           // per cell: last step a moving point left or entered it
    // expiry calendar queue (NNC_QUEUE)
    nnc::QHead *qh;
    int32_t *q_pool, *q_nruns, *q_run_start, *q_run_len, *q_bcnt, *q_cursor, *q_keep;
    double *q_pool_e, *q_keep_e, *q_key;  // keys beside the pool and keep entries; new keys in list order
    int q_cap;
    int queue_valid;              // host: the calendar holds every current key
    unsigned long long *status;   // look-back tile descriptors
    int nstatus;
    nnc::DevScalars *sc;
    nnc::DevSync *sync;
    // all-point query: points whose search must widen past the first block, and
    // the tiled pass's results in slot order (nn, d1, d2 bits, done flag)
    int32_t *wide;
    int4 *rec;
    uint8_t *cmask;               // tiled repair: candidates marked in slot order (all zero between repairs)
    // reduce-then-scan filter: candidates per tile, then their offsets
    int32_t *tcount;
    int ntcount;
    unsigned long long *fmask;    // its candidate ballots, one bit per point
    long long nfmask;
    int fail_dirty;               // host: fail flags may be set outside the last candidate list
    double *ent_part;             // partial sums of the split entropy reduction
    double *shape_part;           // partial sums of the gyration (4 per workgroup), then the centroid
    // audit scratch
    int32_t *a_nn;
    float *a_d1, *a_d2;
    uint8_t *rho;                 // local predictor flags of the step rho_step (-1: none)
    int64_t rho_step;
    // one arena holds every buffer above
    void *arena;
    size_t arena_bytes;
    size_t state_bytes;           // prefix of the arena that a snapshot copies

    const float *pos_cur, *pos_prev;
    float *pos_copy[2];
    int copy_slot;

    int64_t t;
    int pending;
    int grid_fresh;               // grid built at the current step (slot records current)
    double drift_host;            // accumulated declared eps since the grid build; <0 unknown
    int steps_since_grid;
    int lanes;                    // lanes per query (16, 32 or 64)
    int inited;

    // kernel timing (nnc_profile_enable)
    int prof_on, prof_cap, prof_used;
    hipEvent_t *prof_ev;
    int *prof_cls;
    double prof_ms[NNC_K_COUNT];
    int64_t prof_cnt[NNC_K_COUNT];
};

namespace nnc {

// grid.hip
int launch_cells_init(nnc_ctx *c, const float *pos);
int launch_ingest(nnc_ctx *c, const float *pold, const float *pnew);
int launch_filter(nnc_ctx *c, float eps_declared);
// from_slots: the slot records hold every point's current coordinates (any build
// after the first), and the scatter reads them in their previous order
int launch_grid_build(nnc_ctx *c, const float *pos, bool from_slots);
// qkey: with a list, the new key of entry q is also written at qkey[q] (the expiry
// calendar's filing), unless the tiled repair takes the list
int launch_query(nnc_ctx *c, const int32_t *list, const int32_t *count_dev, int all, int init, double *qkey);
// the list length from which a repair goes to the cell-tiled query (0: never)
int tiled_repair_from(const nnc_ctx *c);
int launch_query_all(nnc_ctx *c, int init);
int launch_entropy(nnc_ctx *c, int which);
int launch_cand_hist(nnc_ctx *c);
int launch_audit(nnc_ctx *c);
int launch_rho(nnc_ctx *c);
int launch_budget(nnc_ctx *c);
// queue.hip: the calendar's pop (in place of the filter) and its filing after a repair
// or rebuild (rebuilding the whole calendar when build is set)
int launch_queue_pop(nnc_ctx *c, float eps_declared);
int launch_queue_file(nnc_ctx *c, int build);
// which = 0: failed points, 1: candidates; cen: null for the first pass (sums of
// coordinates and count), else the centroid (sum of squared distances)
int launch_shape(nnc_ctx *c, int which, const double *cen);
int launch_features(nnc_ctx *c, float *out);
int launch_fill(void *p, int value, size_t count, hipStream_t s);

// allpairs.hip
int launch_allpairs(const float *pos, int64_t n, int d, const int32_t *qidx, int64_t nq,
                    int32_t *nn, float *d1, float *d2, hipStream_t s);
int launch_sqrt(const float *x, float *out, int64_t n, hipStream_t s);

}  // namespace nnc
