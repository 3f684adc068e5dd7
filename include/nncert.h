/*
 * nncert: exact nearest-neighbour certificates for moving points on MI355X.
 *
 * The operation (Section 2): every point i of a set of N points in R^d
 * (d = 2 or 3) keeps a certificate (nn_i, d1_i, d2_i) -- its nearest neighbour
 * and the two smallest neighbour distances (Definition 1) -- and the grid cell
 * that holds it.  Each step the points move; a certificate with clearance
 * c_i = d2_i - d1_i larger than four times the motion since it was computed
 * cannot have failed (Lemma 1, Theorem 2), so only the others -- the repair
 * frontier -- are recomputed (Algorithm 1).  Motion is accumulated on a clock
 * S = sum of per-step maximum displacements, and certificate i, computed at
 * clock S_i, is a repair candidate once S reaches its expiry key
 * S_i + c_i / 4 (appendix, per-step cost).  Competitors: a full O(N) grid
 * rebuild and an exact all-pairs brute force.
 *
 * Arithmetic, fixed so that results are reproducible bit for bit:
 *   squared distance s = ((dx*dx) + (dy*dy)) + (dz*dz), dx = x_j - x_i, every
 *   operation binary32 round-to-nearest-even, no fused multiply-add;
 *   nn = argmin_j s over j != i, ties to the lowest index; s2 = the second
 *   smallest value of {s(i,j)}; d1 = sqrtf(s1), d2 = sqrtf(s2) correctly
 *   rounded; +inf for missing neighbours, nn = -1 when N = 1;
 *   eps_t = sqrtf(max_i s(p_i(t-1), p_i(t)));  S_t = S_{t-1} + eps_t (binary64);
 *   expiry e_i = S_i + (c_i - g*d2_i) * K, K = 1/(4 + 4g), binary64, with a
 *   guard g (default 2^-18) that absorbs binary32 rounding; g = 0 is the
 *   paper's key;  candidate iff S_t >= e_i;
 *   cell of a point: per axis floor(fl32(x * G)) clamped to [0, G-1], linear id
 *   gx + G*(gy + G*gz) over the box [0,1]^d (points outside go to edge cells), or
 *   over a domain box given at creation (nnc_config.lo / hi).
 *
 * Conventions for every call:
 *   - return 0 on success or a negative NNC_E_* code; no exception crosses the ABI;
 *   - pointers documented "device" are device (HBM) addresses, e.g. the
 *     data_ptr() of a contiguous float32 CUDA tensor; positions are
 *     structure-of-arrays: pos[k*N + i] is coordinate k of point i;
 *   - work is ordered on the context's HIP stream; only calls that return host
 *     values synchronise with it (stated per call);
 *   - errors found on the device (a non-finite coordinate, a declared eps
 *     below the measured one) are latched in a device error word and returned
 *     by the next synchronising call;
 *   - a context is not thread-safe: one context per stream, one thread at a time.
 */
#ifndef NNCERT_H
#define NNCERT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define NNC_OK           0
#define NNC_E_INVAL     -1   /* bad argument or configuration */
#define NNC_E_NOMEM     -2   /* device allocation failed */
#define NNC_E_HIP       -3   /* a HIP runtime call failed */
#define NNC_E_EPS       -4   /* measured eps_t exceeded the declared bound */
#define NNC_E_NONFINITE -5   /* a coordinate was NaN or infinite */
#define NNC_E_STATE     -6   /* call out of order (e.g. repair without a pending step) */
#define NNC_E_DEVICE    -7   /* a device-side bounded wait expired (internal error) */

/* ---- configuration flags ------------------------------------------------ */
#define NNC_COPY_POSITIONS 1u  /* keep a private copy of each position frame */
#define NNC_SYNC           2u  /* nnc_step synchronises and fills count_host */
/* All-point queries (initialisation, rebuild) run tiled by grid cells with the
 * neighbourhood staged in LDS from N = 65536 on for initialisation and from
 * N = 2^17 (d = 2) or 2^19 (d = 3) on for a rebuild, pointwise below; these force one.
 * NNC_QUERY_TILED also sends repairs to the tiled query of the marked candidates
 * (faster only when about half of the points are candidates). */
#define NNC_QUERY_TILED     4u
#define NNC_QUERY_POINTWISE 8u
/* Per-point motion budget (the Limitations section's tighter safe set): each step,
 * a point whose key S_i + c_i/4 has expired is re-tested against its kept
 * certificate (nn = j, d2, made at clock S_i and step t_i), D = S_t - S_i:
 *  (1) block-local: if no cell of its 3^d block was left or entered by a moving
 *      point after step t_i and (d2 + D)(1 + 2^-20) + fuzz < B (B: distance to the
 *      outside of the block, fuzz the cell-boundary allowance 2^-20 max(1, |lo|, |hi|)),
 *      no point can have come within d2: kept, key = the next binary64 value
 *      above S_t (tested again at the next step in which anything moves);
 *  (2) distance: j is still the strict nearest neighbour while its current
 *      distance r (binary32 formula) is below d2 - 2 D; then the certificate is
 *      kept and its key moves to S_t + gap * K, gap = (d2 (1 - g) - 2 (D (1 + g))) - r
 *      in binary64 (g the guard, K = 1/(4 + 4g));
 * otherwise the point is a candidate.  The candidates are a subset of the clock
 * rule's, and motion confined to one region makes candidates only near it; no
 * failure is missed.  Costs a per-cell step stamp in the ingest. */
#define NNC_BUDGET          16u
/* Expiry calendar queue (appendix, per-step cost; Theorem 3): the keys are filed
 * in a ring of buckets of the clock, so a step reads only the buckets the clock
 * reached and files the repaired points' new keys, instead of scanning all N keys;
 * the calendar is rebuilt (O(N)) after init, a rebuild, a restore, a caller's
 * repair list, or when its pool fills.  The candidate SET is the same; the list
 * comes in bucket order, not ascending.  Not with NNC_BUDGET; n < 2^28. */
#define NNC_QUEUE           32u

/* nnc_frontier_entropy: which set */
#define NNC_FAILED     0      /* certificates whose nearest neighbour changed (Definition 2) */
#define NNC_CANDIDATES 1      /* the repair candidates of the last step */

typedef struct nnc_ctx nnc_ctx;
typedef struct nnc_snap nnc_snap;

typedef struct {
    int32_t  d;           /* 2 or 3 */
    int32_t  grid_g;      /* cells per axis over [0,1]^d; 0 = occupancy rule below */
    int64_t  n;           /* number of points, 0 <= n < 2^31 */
    double   guard;       /* expiry guard g; negative = default 2^-18 */
    double   refresh;     /* loose-grid refresh when accumulated motion since the last
                             index build exceeds refresh * cell width; <= 0 = 0.25 */
    void    *stream;      /* hipStream_t to order work on; NULL = the null stream */
    uint32_t flags;       /* NNC_COPY_POSITIONS | NNC_SYNC | NNC_QUERY_TILED | NNC_QUERY_POINTWISE |
                             NNC_BUDGET | NNC_QUEUE */
    int32_t  block;       /* lanes that share one 2-NN query: 1 (one thread per query,
                             for large N), 4 (d = 2 only; in d = 3 it means the
                             default), 8, 16, 32 or 64; 0 = 32 for d = 3 and 16 for d = 2 */
    /* Domain box of the grid: axis k is cut into grid_g equal cells over
     * [lo[k], hi[k]); a point's cell on axis k is floor(fl32(fl32(x - lo[k]) * s_k))
     * clamped to [0, grid_g - 1], s_k = fl32(grid_g / (hi[k] - lo[k])) with the
     * division in binary64 (points outside fall into edge cells).  All zero = the
     * unit box [0,1]^d, where the formula is floor(fl32(x * grid_g)).  Otherwise
     * every used axis needs finite lo < hi (else NNC_E_INVAL). */
    float    lo[3];
    float    hi[3];
} nnc_config;

/* Default grid_g: cell width w = 2/sqrt(N) (d = 2) or (4/N)^(1/3) (d = 3) and
 * G = max(1, floor(1/w)), a small constant mean occupancy (Section 2). */

typedef struct {
    const int32_t *idx_dev;    /* device: ascending candidate indices (in bucket order with
                                  NNC_QUEUE; library-owned, valid until the next step) */
    const int32_t *count_dev;  /* device: number of candidates */
    int32_t count_host;        /* filled when NNC_SYNC is set, else -1 */
    int32_t step;              /* step number t (1 = first step after init) */
} nnc_frontier;

typedef struct {
    const int32_t *nn;    /* device [n] */
    const float   *d1;    /* device [n] */
    const float   *d2;    /* device [n] */
    const double  *e;     /* device [n], expiry keys */
    const int32_t *cell;  /* device [n], current cell ids */
    const uint8_t *fail;  /* device [n], 1 if nn changed at the last repair/rebuild */
    int64_t n;
    int32_t d, grid_g;
    const uint8_t *rho;   /* device [n], flags of the local predictor (nnc_rho_predict) of
                             the last step; meaningful only after that call, NULL in a batch */
    const double *Si;     /* device [n], clock S_i at which each certificate was computed
                             (NULL in a batch) */
} nnc_state;

typedef struct {
    int64_t n_checked;        /* points whose nn was compared */
    int64_t n_detect;         /* candidates of the last step */
    int64_t n_true_fail;      /* points whose nn changed at the last step */
    int64_t n_missed;         /* points whose kept nn differs from brute force (must be 0) */
    int64_t n_false;          /* candidates that did not fail */
    int64_t n_value_mismatch; /* fresh certificates whose d1/d2 differ from brute force */
    uint64_t nn_hash;         /* 64-bit hash of nn[] (order-dependent, deterministic) */
    int64_t rho_flagged;      /* points the local predictor flagged for the last step
                                 (nnc_rho_predict), -1 if it was not evaluated */
    int64_t rho_hit;          /* flagged points that failed, -1 likewise */
} nnc_audit;

typedef struct {
    double  eps;      /* eps_t of the last step */
    double  S;        /* clock S_t */
    double  H;        /* normalised entropy of the chosen set */
    int32_t m;        /* occupied cells the set meets */
    int32_t C;        /* occupied cells */
    int32_t count;    /* |set| */
} nnc_entropy;

/* Create a context for cfg->n points in cfg->d dimensions (Section 2: the moving
 * point set, its per-point records and the uniform grid sized for a constant mean
 * occupancy); allocates all state.
 * Errors: NNC_E_INVAL (d not 2/3, n out of range, G^d over 2^24), NNC_E_NOMEM. */
int nnc_create(nnc_ctx **out, const nnc_config *cfg);

/* Release every buffer of the context created by nnc_create (Section 2's state),
 * after draining its stream.  NULL is ignored. */
void nnc_destroy(nnc_ctx *ctx);

/* Certificates (Definition 1) of every point at positions pos (device, float32
 * [d][n]) by a full grid build and 2-NN query; clock S = 0.  pos is borrowed: it must stay
 * unchanged until the next nnc_step returns (or is copied with
 * NNC_COPY_POSITIONS).  Asynchronous. */
int nnc_init_certificates(nnc_ctx *ctx, const float *pos);

/* One step of Algorithm 1 up to its repair loop: measure eps_t against the
 * previous frame, advance the clock (appendix, per-step cost), bring every cell
 * id up to date, and compact the candidates S_t >= e_i (Lemma 1, Theorem 2) into
 * an ascending list (out).
 * pos_new (device, float32 [d][n]) is borrowed like in init.  eps_declared < 0:
 * no check; else a measured eps_t > eps_declared * (1 + 2^-16) + 2^-20 (the
 * slack covers rounding of coordinates to binary32) is reported as NNC_E_EPS by
 * the next synchronising call, and the step still runs with the measured eps_t, so
 * certificates stay exact: the state IS advanced (the check runs on the device,
 * and holding the state back would need a synchronisation every step).  The
 * declared bound also paces the refresh of the grid index.  Asynchronous unless NNC_SYNC.  A step must be followed by exactly
 * one nnc_repair or nnc_rebuild before the next step (NNC_E_STATE otherwise). */
int nnc_step(nnc_ctx *ctx, const float *pos_new, float eps_declared, nnc_frontier *out);

/* Recompute the certificates of the pending step's candidates (f == NULL) or of
 * an explicit list (f->idx_dev, f->count_dev device pointers; any order,
 * duplicates not allowed), against the current positions through the grid
 * index, widening each query until its second neighbour is provably enclosed
 * (Corollary 1).  Sets fail flags, S_i = S_t, and the failure histogram used
 * by nnc_frontier_entropy.  Asynchronous. */
int nnc_repair(nnc_ctx *ctx, const nnc_frontier *f);

/* The competitor (Section 3's GPU grid rebuild; Theorem 3's Theta(N) side): rebin
 * all n points and recompute every certificate, in place of nnc_repair for the
 * pending step.  Asynchronous. */
int nnc_rebuild(nnc_ctx *ctx);

/* The exact frontier oracle (Section 3; the no-miss audit of Section 4 and
 * Corollary 1): tiled all-pairs top-2 of the current positions on the GPU,
 * compared with the state: nn of every point, d1/d2 bitwise of points certified
 * at the last step.  Synchronises. */
int nnc_oracle_verify(nnc_ctx *ctx, nnc_audit *out);

/* The local failure predictor the paper reports beside the safety rule (Section 4,
 * Table 1): rho_i = delta_i / c_i > 1/2, where c_i = d2 - d1 of point i's kept
 * certificate and delta_i the last step's motion of i plus that of its kept nearest
 * neighbour j (each the correctly rounded square root of the binary32 squared
 * displacement, summed in binary32); i is flagged iff 2 delta_i > c_i (never when
 * d2 = +inf or nn = -1).  Call after nnc_step and before nnc_repair or nnc_rebuild;
 * the next nnc_oracle_verify reports how many points were flagged and how many of
 * them failed.  An audit tool, not part of the maintenance step.  Asynchronous.
 * NNC_E_STATE without a pending step. */
int nnc_rho_predict(nnc_ctx *ctx);

/* Normalised entropy (Definition 2) of the failed set or of the last step's
 * candidates, over the current cells, with m and C (Theorem 4: m >= C^H), in one
 * struct with eps_t, S_t and the set's size.  Synchronises. */
int nnc_frontier_entropy(nnc_ctx *ctx, int which, nnc_entropy *out);

/* Work counters of the expiry calendar (NNC_QUEUE; appendix, per-step cost), since
 * creation: out[0] steps that popped buckets, out[1] steps that scanned every key
 * (the clock outran the calendar), out[2] calendars filed anew, out[3] entries the
 * pops read; out[4] pool entries in use, out[5] keys in the far set at the last
 * filing.  Synchronises.  NNC_E_STATE without NNC_QUEUE. */
int nnc_queue_stats(nnc_ctx *ctx, int64_t *out);

/* Spatial spread of the failed set (Definition 2's F_t) or of the last step's
 * candidates at the current positions: its radius of gyration
 * sqrt(mean |p_i - centroid|^2) and centroid (centroid[3] may be NULL; z = 0 in
 * the plane), in binary64; 0 for an empty set.  The gyration descriptor of the
 * dataset (Section 6).  Synchronises. */
int nnc_frontier_gyration(nnc_ctx *ctx, int which, double *gyration, double *centroid);

/* The six selector features of the pending step (after nnc_step, before
 * nnc_repair/nnc_rebuild); the selector predicts Section 3's best-strategy label
 * (the fastest strategy of the transition) from them, written to out (device float32 [NNC_FEATURES]):
 * |F|/N, H of the candidates, ln N, d, cells met by the candidates / G^d, and
 * eps_t / the median remaining motion budget e_i - S_{t-1} of the certificates of
 * points 0 .. min(N, 1024) - 1 (median from a
 * power-of-two histogram).  Asynchronous. */
int nnc_features(nnc_ctx *ctx, float *out);

/* Read-only device views of the state arrays: the per-point record of Section 2
 * (certificate of Definition 1, expiry key of the appendix, cell of Algorithm 1,
 * failure flag of Definition 2).  Does not synchronise. */
int nnc_get_state(nnc_ctx *ctx, nnc_state *v);

/* Device-side copy of the whole state, so that both strategies can be timed on one
 * transition (Section 3 labels each transition with its fastest strategy).
 * Allocates the snapshot; restore copies it back (asynchronous); snap_free
 * releases it (NULL ignored). */
int nnc_snapshot(nnc_ctx *ctx, nnc_snap **out);
int nnc_restore(nnc_ctx *ctx, const nnc_snap *snap);
/* Overwrite an existing snapshot of this context with the current state (no allocation). */
int nnc_snapshot_update(nnc_ctx *ctx, nnc_snap *snap);
void nnc_snap_free(nnc_snap *snap);

/* Standalone exact all-pairs top-2 (Section 3's full N x N pass and Table 2's brute
 * force; the ground truth of Definition 1):
 * for every point of pos (device float32 [d][n]) -- or for the nq listed points
 * when qidx (device int32 [nq]) is not NULL -- write nn (int32), d1, d2 (float32)
 * to device arrays of length n (or nq).  stream: hipStream_t or NULL.
 * Asynchronous. */
int nnc_allpairs_top2(const float *pos, int64_t n, int32_t d, const int32_t *qidx, int64_t nq,
                      int32_t *nn, float *d1, float *d2, void *stream);

/* Square root of every element of x (device float32 [n]) into out (device float32
 * [n]), by the routine that computes d1 = sqrt(s1), d2 = sqrt(s2) (Definition 1)
 * and eps_t in every kernel; the certificates are bit-exact only if it is
 * correctly rounded, which this call lets a test check over all binary32 inputs.
 * stream: hipStream_t or NULL.  Asynchronous.  NNC_E_INVAL for n < 0 or NULL arrays. */
int nnc_sqrt_f32(const float *x, float *out, int64_t n, void *stream);

/* ---- kernel timing ------------------------------------------------------ */
/* Kernel classes timed by the profiler. */
#define NNC_K_INGEST  0   /* displacement, eps_t, cell update */
#define NNC_K_FILTER  1   /* clock, safety filter, ordered compaction */
#define NNC_K_GRID    2   /* cell-start scan and counting-sort scatter */
#define NNC_K_QUERY   3   /* 2-NN queries: repair of candidates or rebuild of all */
#define NNC_K_ENTROPY 4   /* failure histogram entropy */
#define NNC_K_COUNT   5

typedef struct {
    double  ms[NNC_K_COUNT];     /* summed kernel durations, milliseconds */
    int64_t count[NNC_K_COUNT];  /* number of timed launches */
} nnc_profile;

/* Enable (1) or disable (0) HIP-event timing of every kernel the context
 * launches, per class (the per-strategy times of Section 3's cost comparison).  Events are recorded on the context's stream around each
 * launch; enabling adds an event pair per launch, so use it for measurement
 * passes only.  Not for use under stream capture. */
int nnc_profile_enable(nnc_ctx *ctx, int enable);

/* Synchronise, add up the recorded durations into out, and clear them if reset. */
int nnc_profile_read(nnc_ctx *ctx, nnc_profile *out, int reset);

/* ---- many independent scenes in one step --------------------------------- */
/* A batch advances S independent scenes of uneven size and dimension together:
 * every kernel of the step spans all scenes (scene tiles for the per-point
 * passes, one workgroup per scene for the filter, compaction, features and
 * strategy decision, one persistent grid-stride launch for the 2-NN queries of
 * all scenes).  Each scene follows exactly the single-scene semantics above;
 * the strategy (repair or rebuild) is chosen per scene and per step. */
typedef struct nnc_batch nnc_batch;

#define NNC_POLICY_REPAIR    0   /* repair the candidates of every scene */
#define NNC_POLICY_REBUILD   1   /* rebuild every scene */
#define NNC_POLICY_THRESHOLD 2   /* rebuild a scene iff |F|/N >= tau */
#define NNC_POLICY_LEARNED   3   /* the selector network decides; without loaded parameters,
                                    or for a scene whose features are not finite, the
                                    threshold rule decides */

#define NNC_FEATURES        6      /* per scene-step: |F|/N, H(F), ln N, d, m/G^d, eps/radius */
#define NNC_SELECTOR_PARAMS 4738   /* 6-64-64-2 network: W1 b1 W2 b2 W3 b3, row-major out x in */
#define NNC_BATCH_MAX_N     32768  /* points per scene */

typedef struct {
    int32_t scenes;
    const int64_t *n;        /* host [scenes]: points per scene, 0 <= n <= NNC_BATCH_MAX_N */
    const int32_t *d;        /* host [scenes]: 2 or 3 */
    const int32_t *grid_g;   /* host [scenes]: cells per axis; NULL or entries <= 0 = occupancy rule */
    int32_t lanes;           /* lanes per query: 1, 4, 8, 16, 32 or 64 (4 in the plane only;
                                cube scenes then use 16); 0 = 4 in the plane, 8 in the cube */
    double guard;            /* as in nnc_config */
    double refresh;          /* as in nnc_config, but <= 0 = 0.125 */
    void *stream;            /* hipStream_t */
    uint32_t flags;          /* NNC_BATCH_FEATURES | NNC_BATCH_EAGER | NNC_BATCH_TIMING | NNC_BATCH_BUDGET */
} nnc_batch_config;

/* Compute the candidate histogram, H of the candidates and the selector features
 * at every step (otherwise only under NNC_POLICY_LEARNED). */
#define NNC_BATCH_FEATURES 1u
/* Launch the step's kernels one by one instead of through the library's graph. */
#define NNC_BATCH_EAGER    2u
/* Per-scene cost accounting with the GPU's wall clock: the filter's and the grid
 * build's workgroup time and the query waves' summed busy time of each scene
 * (nnc_scene_stats.t_*_us), to label each scene-step with its cheaper strategy
 * inside the batch (Section 3's best-strategy label). */
#define NNC_BATCH_TIMING   4u
/* The per-point motion budget of NNC_BUDGET (Section 5, Limitations) in every
 * scene: before the filter, each expired certificate takes the block-local and
 * the distance test, and only the points that fail both are candidates.  Costs a
 * per-cell step stamp in the ingest, a binary64 certificate clock per point and
 * one pass over the expired points. */
#define NNC_BATCH_BUDGET   8u

typedef struct {
    double  eps;             /* eps_t of the last step */
    double  S;               /* clock */
    double  H_fail;          /* entropy of the failures (Definition 2) */
    double  H_cand;          /* entropy of the candidates */
    int32_t n_cand;          /* |candidates| */
    int32_t n_fail;          /* |failures| */
    int32_t m_cand;          /* cells met by the candidates (0 unless features are computed) */
    int32_t C;               /* occupied cells */
    int32_t strategy;        /* 0 repair, 1 rebuild */
    int32_t err;             /* NNC_OK or a negative code latched for this scene */
    float   features[NNC_FEATURES];
    double  t_filter_us;     /* with NNC_BATCH_TIMING (else -1): the scene's filter workgroup time, */
    double  t_grid_us;       /* its grid build's workgroup time (0 without a build), */
    double  t_query_us;      /* and the summed time of the query waves that worked on it */
} nnc_scene_stats;

/* Create a batch of independent scenes, each the point set of Section 2; allocates
 * every buffer.  Scene s's coordinates occupy a
 * float32 [d_s][n_s] block at offset coord_off[s] of the concatenated position
 * arrays, and its per-point state the range [point_off[s], point_off[s] + n_s)
 * of the concatenated state arrays (offsets from nnc_batch_offsets).
 * Errors: NNC_E_INVAL, NNC_E_NOMEM. */
int nnc_batch_create(nnc_batch **out, const nnc_batch_config *cfg);
void nnc_batch_destroy(nnc_batch *b);

/* Where each scene's points and coordinates sit in the concatenated arrays: host
 * arrays of scenes+1 entries each (the last entry is the total). */
int nnc_batch_offsets(const nnc_batch *b, int64_t *point_off, int64_t *coord_off);

/* Certificates (Definition 1) of every point of every scene (device, concatenated
 * positions, read during the call).  Asynchronous. */
int nnc_batch_init(nnc_batch *b, const float *pos);

/* One maintenance step of every scene (Algorithm 1 per scene, with the clock of
 * the appendix): measure eps_t, advance the clock, update the cells, filter and
 * compact, compute the features, choose the strategy by policy, rebuild or
 * refresh grids where needed, run every scene's queries in one launch per
 * dimension, and reduce the failure entropy (Definition 2).  With scenes of both
 * dimensions, the plane scenes' kernels up to their queries run on a stream the
 * library owns, forked from the batch's stream by an event and joined back into it
 * before the entropy, so the step stays ordered on the batch's stream (also under
 * capture, where the fork and join become graph edges).  pos_new (device, concatenated) is
 * read during the step only: the previous coordinates are kept by the library.
 * Asynchronous.  The step's kernels are captured into a HIP graph on the
 * first call and the graph is replayed while pos_new, policy and tau repeat
 * (write each new frame into the same buffer); another pointer, policy or tau
 * re-captures the graph (a host cost of tens of microseconds).  Under a caller's
 * own stream capture, on the null stream, or with NNC_BATCH_EAGER the kernels are
 * launched directly.  The step counter, the clocks and the previous coordinates
 * live in device memory, so a caller may also capture one call and replay it for
 * successive steps: each replay advances every scene by one step, reading the
 * positions from the captured pos_new buffer.  No allocation, memset or
 * synchronisation happens inside a step. */
int nnc_batch_step(nnc_batch *b, const float *pos_new, int policy, float tau);

/* Load the selector's parameters (device float32 [NNC_SELECTOR_PARAMS]); copied.
 * The network predicts Section 3's best-strategy label for NNC_POLICY_LEARNED. */
int nnc_batch_selector_load(nnc_batch *b, const float *params);

/* Band of candidate fractions [lo, hi) in which the learned policy computes the
 * features and asks the network; below lo it repairs, from hi on it rebuilds (the
 * size rule), so scene-steps outside the band cost no features.  Default [0, 2):
 * the network everywhere.  NNC_E_INVAL unless lo <= hi. */
int nnc_batch_selector_band(nnc_batch *b, float lo, float hi);

/* Per-scene results of the last step (host array [scenes]): eps_t and S_t
 * (appendix clock), sizes and entropies of the failed and candidate sets
 * (Definition 2), the features and the chosen strategy.  Synchronises. */
int nnc_batch_scene_stats(nnc_batch *b, nnc_scene_stats *out);

/* Device-side copy of a batch's whole state, to time both strategies on one step
 * of every scene (Section 3's label); allocates.  Restore copies it back
 * (asynchronous); snap_free releases it (NULL ignored). */
typedef struct nnc_batch_snap nnc_batch_snap;
int nnc_batch_snapshot(nnc_batch *b, nnc_batch_snap **out);
int nnc_batch_restore(nnc_batch *b, const nnc_batch_snap *snap);
/* Overwrite an existing snapshot of this batch with the current state (no allocation). */
int nnc_batch_snapshot_update(nnc_batch *b, nnc_batch_snap *snap);
void nnc_batch_snap_free(nnc_batch_snap *snap);

/* Device views of the concatenated per-point records (Section 2; n = total
 * points, d = 0, grid_g = 0, rho = NULL).  Does not synchronise. */
int nnc_batch_get_state(nnc_batch *b, nnc_state *v);

/* ---- selector network: training and inference kernels ----------------------- */
/* A 6-64-64-2 ReLU network in FP32 (layout as NNC_SELECTOR_PARAMS above) that
 * predicts Section 3's best-strategy label (repair or rebuild) from the features.
 * All pointers are device pointers; all calls are asynchronous on stream. */

/* Bytes of workspace nnc_mlp_grad needs for a batch of B samples. */
size_t nnc_mlp_workspace_bytes(int B);

/* Loss L = (1/B) sum_b w_b * CE(softmax(z_b), y_b) of a batch (X [B][6] float32,
 * y [B] int32 in {0,1}, w [B] float32) and its gradient grad [NNC_SELECTOR_PARAMS]
 * (overwritten), loss [1]. */
int nnc_mlp_grad(const float *params, const float *X, const int32_t *y, const float *w, int B, void *workspace,
                 float *grad, float *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): nnc_mlp_grad without a
 * workspace argument.  The workspace is a fixed device array inside the library
 * (4 MiB per device for NNC_MLP_STATIC_MAX_B samples, held until the process
 * ends); the call allocates nothing.  B above NNC_MLP_STATIC_MAX_B gives
 * NNC_E_INVAL.  Every call on one device shares that array: calls that overlap
 * on one device (on different streams) race and must be serialised by the
 * caller.  The stream's device (the current device for NULL) is used.  Results
 * equal nnc_mlp_grad's bit for bit.  Asynchronous. */
#define NNC_MLP_STATIC_MAX_B 4096
int nnc_mlp_grad_static(const float *params, const float *X, const int32_t *y, const float *w, int B, float *grad,
                        float *loss, void *stream);

/* One Adam step (step = 1, 2, ...) on params with moments m, v. */
int nnc_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1,
                 float beta2, float eps, void *stream);

/* Logits [B][2] of a batch of feature rows X [B][6]. */
int nnc_mlp_forward(const float *params, const float *X, int B, float *logits, void *stream);

/* Human-readable text of an error code (a static string; never NULL). */
const char *nnc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* NNCERT_H */
