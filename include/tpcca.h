/*
 * tpcca.h — C ABI of the MI355X TPC sector tracker.
 *
 * Computes the sector-tracking hot path of Rohr et al., "Track Reconstruction
 * in the ALICE TPC using GPUs for LHC Run 3" (arXiv:1811.11481), Section 2
 * (cellular-automaton seeding, Kalman-filter track following, final fit) with
 * the resolution changes of Section 3 (inward pass through the seed with
 * outlier rejection, chi2-based cluster rejection, three-pass refit):
 *   clusters per sector instance and pad row in,
 *   tracks with five parameters, covariance, chi2 and cluster lists out.
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer owned by the caller, unless a
 *    comment says "host". It must stay valid until the stream has completed
 *    the call.
 *  - Clusters are given per instance (one sector of one event or time frame)
 *    and pad row as a CSR over rows: row_start[k * n_rows + r] is the first
 *    cluster of row r of instance k; clusters of a row are contiguous and the
 *    cluster id used everywhere (outputs, exports) is the index into y/z.
 *    Coordinates are sector-local: x is the pad-row plane params.row_x[r], y
 *    along the row, z along the drift (any origin: only z differences are used).
 *  - All track arithmetic is IEEE binary32 in a fixed operation order: a
 *    fused multiply-add (one rounding) exactly where the written algorithm
 *    has one and nowhere else (no compiler contraction), correctly rounded
 *    division and square root; only cross-track sums are FP64.
 *  - Status codes are the only error channel; tpcca_last_error() gives text.
 *    Calls are asynchronous on `hip_stream` except where a host output is
 *    returned (track counts), which synchronises the stream once.
 *  - A context is used by one host thread at a time (not thread-safe) and owns
 *    scratch device memory that grows on demand and is reused.
 */
#ifndef TPCCA_H
#define TPCCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPCCA_OK = 0,
    TPCCA_E_ARG = 1,      /* invalid argument or malformed input (detected on host or device) */
    TPCCA_E_CAPACITY = 2, /* output capacity too small (required sizes are returned) or a
                             per-row / per-instance hard limit exceeded */
    TPCCA_E_DEVICE = 3,   /* HIP runtime error */
    TPCCA_E_OOM = 4,      /* device allocation failed */
    TPCCA_E_INTERNAL = 5
} tpcca_status;

typedef struct tpcca_ctx tpcca_ctx;

#define TPCCA_MAX_ROWS 255
#define TPCCA_MAX_ROW_CLUSTERS 16384   /* clusters of one pad row of one instance */
#define TPCCA_MAX_STARTS_PER_INST 1048576 /* tracklet ids are 20-bit per instance */

/* Tracking parameters. Defaults (tpcca_default_params) are the readings of
 * the paper recorded with the algorithm description; doubles are rounded to
 * binary32 once when a context is created. */
typedef struct {
    int32_t n_rows;               /* pad rows per instance (1..255), default 152 */
    float row_x[256];             /* pad-row plane x [cm], strictly increasing; default 85 + i*162/151 */
    double bz;                    /* solenoid field [T] (Bx = By = 0), default 0.5 */
    double sigma_y, sigma_z;      /* cluster errors [cm], default 0.1 */
    double win_ty, win_tz;        /* neighbour window slope terms, default 2.0, 1.1 */
    double win_ny, win_nz;        /* neighbour window constant terms [cm], default 0.5 */
    double nbr_score_max;         /* max straight-line deviation of a triplet [cm^2], 0.24 */
    double nsig;                  /* pickup window in sigmas, 3 */
    double chi2_pick;             /* pickup chi2 cut (2 dof), 16 */
    double chi2_rej;              /* refit rejection chi2 cut (2 dof), 25 */
    double sinphi_max;            /* |sin phi| guard, 0.95 */
    double cov_reset;             /* variance scale at a covariance reset, 100 */
    double q_max;                 /* |q/pT| clamp of the seed [c/GeV], 20 */
    double u_max;                 /* max |curvature * chord / 2| per step, 0.25 */
    double c0[5];                 /* seed covariance diagonal, (1, 1, 0.25, 0.25, 400) */
    int32_t n_min;                /* min clusters of a tracklet and of a track, 10 */
    int32_t max_miss;             /* consecutive empty rows ending the following, 8 */
    uint32_t flags;               /* TPCCA_FLAG_* */
    double chi2_merge;            /* cross-sector merge: max chi2 (five parameters) of a segment pair, 25 */
    int32_t merge_max_gap;        /* cross-sector merge: max rows between a segment's end and the next, 24 */
    /* Native cluster coordinates (tpcca_track_native; Sections 4 and 6: pad, row and time). */
    float pad_width[256];         /* pad pitch along local y per row [cm]; default 0.416 (rows 0-62), 0.42
                                     (63-126), 0.46 (127-151) */
    float pad_center[256];        /* pad coordinate of local y = 0 per row; default (n_pads - 1) / 2 with
                                     n_pads = 2 ceil(row_x tan(10 deg) / pad_width), the pads that cover the
                                     row's width */
    double z_per_bin;             /* drift length per time bin [cm], 0.516 (2.58 cm/us drift, 200 ns bins) */
    double z_readout;             /* |z| of the readout planes [cm], 250 */
} tpcca_params;

#define TPCCA_FLAG_STATS 1u       /* count work items (rows visited, candidates) for the byte model */
#define TPCCA_FLAG_TIMING 2u      /* batched form runs uncaptured with HIP events between stages */
#define TPCCA_FLAG_MERGE 8u       /* track calls keep what tpcca_merge needs (outward-pass states, rows) */

/* Launch/tiling choices. They never change results (tested bit-exact). */
typedef struct {
    int32_t hits_per_bin;     /* grid occupancy target per bin (>= 1), default 1 */
    int32_t block_links;      /* threads per block of the neighbour kernel (64..1024), default 256 */
    int32_t block_tracklet;   /* threads per block of the tracklet kernels (64..256), default 64 */
    int32_t block_refit;      /* threads per block of the refit kernel (64..256), default 128 */
    int32_t block_scan;       /* threads per block of scans/compactions, default 256 */
    int32_t sort_seeds;       /* order of the refit's tracks over its lanes (results identical): 0
                                 consecutive tracks; 1 (default): each workgroup hands its chunk of
                                 consecutive tracks to its lanes longest first; 2: a counting sort by
                                 estimated work over chunks of 1024 tracks, longest first (its lanes'
                                 cluster lists are then far apart). tpcca_autotune tries all three. */
    int32_t tape_mb;          /* device memory for the differentiable refit's tape [MiB], default 32768;
                                 a larger set is recomputed batch by batch in tpcca_refit_bwd */
    int32_t xcd_remap;        /* 1: workgroups renumbered so that each of the 8 XCDs (own L2) works on
                                 contiguous instances (neighbour and tracklet kernels), default 1 */
    int32_t ckpt;             /* differentiable refit: 0 = the forward records every operation on a tape
                                 (default); 1 = the forward keeps a checkpoint at the start of each of
                                 the three passes and the backward recomputes one pass at a time from
                                 it, last pass first (a third of the tape; same gradients bit for bit) */
    int32_t inward_wgs;       /* 0 (default): see inward_sort; > 0: the outward kernel stops at the turn and a
                                 persistent kernel of this many workgroups (block_tracklet threads, at
                                 most 65536) runs the inward passes, each lane taking the next tracklet
                                 as soon as its last one ends */
    int32_t inward_sort;      /* 1 (default; with inward_wgs = 0): the outward kernel stops at the turn; the
                                 tracklets are ordered within chunks of 1024 seeds by the row their outward
                                 following reached, and a second kernel runs the inward passes in that
                                 order (lanes of a wave then have passes of similar length); 0: one kernel
                                 runs each tracklet's outward and inward passes in one lane */
} tpcca_tuning;

/* Input clusters (device pointers, caller-owned). */
typedef struct {
    int32_t n_inst;             /* number of sector instances (>= 0) */
    const int32_t* inst_sector; /* [n_inst] geometric sector 0..35 (alpha = ((s mod 18) + 0.5) * 20 deg) */
    const int64_t* row_start;   /* [n_inst * n_rows + 1] CSR over (instance, row); row_start[0] = 0,
                                   non-decreasing, last = n_clusters */
    const float* y;             /* [n_clusters] local y [cm] */
    const float* z;             /* [n_clusters] z [cm] */
    int64_t n_clusters;         /* host value */
} tpcca_clusters;

/* Output tracks (device pointers with capacities, caller-owned). Tracks are
 * ordered by (instance, tracklet id); each track's clusters by ascending row. */
typedef struct {
    int64_t cap_tracks;   /* host: capacity of the per-track arrays */
    int64_t cap_hits;     /* host: capacity of hit_id */
    int32_t* inst;        /* [cap_tracks] instance */
    float* x_ref;         /* [cap_tracks] local x of the parameters (innermost cluster's row plane) */
    float* alpha;         /* [cap_tracks] sector rotation angle [rad] */
    float* param;         /* [cap_tracks * 5] y, z, sin phi, tan lambda, q/pT */
    float* cov;           /* [cap_tracks * 15] packed lower triangle 00,10,11,20,21,22,30,..,44 */
    float* chi2;          /* [cap_tracks] sum of accepted predicted chi2 of the last pass */
    int32_t* ndf;         /* [cap_tracks] 2 * clusters - 5 */
    int64_t* hit_start;   /* [cap_tracks + 1] CSR into hit_id */
    int32_t* hit_id;      /* [cap_hits] cluster ids */
    double* chi2_total;   /* [2] FP64: sum of chi2, sum of ndf (deterministic order) */
    float* z0;            /* [cap_tracks] or NULL: z of the track's closest approach to the beam line
                             (Section 4: the primary-vertex z, i.e. the collision time, of a track in
                             continuous readout), from the final fit's state, evaluated in FP64 */
    int16_t* residuals;   /* [cap_hits * 2] or NULL: track-model compression residuals (Section 5.1),
                             (y, z) per output cluster, parallel to hit_id: round((cluster - prediction)
                             / 2^residual_step_log2) where the prediction carries the track's output
                             parameters outward from x_ref row by row with the tracker's binary32 helix
                             step; -32768 marks a value outside int16 or after a failed step */
    int32_t residual_step_log2; /* host: quantisation step 2^k cm, k in [-20, 4] (e.g. -7) */
    int64_t n_tracks;     /* host, written on return: tracks found (even if above capacity) */
    int64_t n_hits;       /* host, written on return */
} tpcca_tracks;

/* Work counters collected when TPCCA_FLAG_STATS is set (host struct). */
typedef struct {
    int64_t n_clusters, n_segments, n_links, n_starts, n_chain_hits;
    int64_t tl_rows_visited, tl_candidates, tl_picks;
    int64_t n_selected, n_selected_hits, n_tracks, n_track_hits;
    int64_t rf_rows_visited, rf_hit_visits;
    int64_t nb_candidates_u, nb_pairs;
} tpcca_stats;

tpcca_status tpcca_default_params(tpcca_params* out);          /* host */
tpcca_status tpcca_default_tuning(tpcca_tuning* out);          /* host */

/* Create a context on HIP device `device` with copies of params and tuning
 * (tuning may be NULL = defaults). */
tpcca_status tpcca_create(const tpcca_params* params, const tpcca_tuning* tuning, int device,
                          tpcca_ctx** out);
void tpcca_destroy(tpcca_ctx* ctx);
const char* tpcca_last_error(const tpcca_ctx* ctx);
tpcca_status tpcca_set_tuning(tpcca_ctx* ctx, const tpcca_tuning* tuning);
tpcca_status tpcca_get_tuning(const tpcca_ctx* ctx, tpcca_tuning* out);

/* Plain form: the sector tracking of Section 2 (hit grid, cellular-automaton
 * neighbour finding and evolution, start hits, Kalman tracklets with the
 * inward pass of Section 3, selection) and the final three-pass fit of
 * Section 3, every stage launched once per instance, instances one after
 * another on `hip_stream`. Reads row_start back to the host once (CSR checks,
 * launch sizes) and the track counts once at the end (two synchronisations).
 * Errors: TPCCA_E_ARG (malformed CSR, non-finite coordinate, null pointers),
 * TPCCA_E_CAPACITY (out->n_tracks / n_hits then hold the required sizes, or a
 * per-row / per-instance limit above), TPCCA_E_DEVICE, TPCCA_E_OOM. */
tpcca_status tpcca_track(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, void* hip_stream);

/* Batched form of tpcca_track: the same computation with every stage launched
 * once over all instances (the paper fills a GPU by processing several events
 * at once, Section 2); the launch sequence is captured in a HIP graph and
 * replayed while every captured pointer, the sizes and the tuning are
 * unchanged. Output identical to tpcca_track (bit for bit); same errors. */
tpcca_status tpcca_track_batched(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out,
                                 void* hip_stream);

/* Batched form without any host synchronisation (Section 5's design keeps the
 * whole chain on the GPU with no host transfers between steps): the CSR is
 * checked on the device, and the counts stay on the device.
 *   counts: device int64[2], written with (n_tracks, n_hits) found (even when
 *           above capacity); status: device int32[1], written with a
 *           tpcca_status (TPCCA_OK, TPCCA_E_ARG, TPCCA_E_CAPACITY,
 *           TPCCA_E_INTERNAL) when the stream reaches the end of the call.
 * The host return value covers only what the host can see (null pointers,
 * sizes, launch failures, scratch allocation); out->n_tracks / n_hits are not
 * written. Sizes the neighbour kernel's LDS staging for the largest row
 * allowed (TPCCA_MAX_ROW_CLUSTERS), so it may run slower than the
 * synchronising forms. Output buffers identical to tpcca_track_batched. */
tpcca_status tpcca_track_async(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, int64_t* counts,
                               int32_t* status, void* hip_stream);

/* Clusters in native coordinates (Sections 4 and 6: the tracking reads pad,
 * row and time and transforms to space on the GPU). Device pointers,
 * caller-owned; the same CSR over (instance, row) as tpcca_clusters. */
typedef struct {
    int32_t n_inst;             /* number of sector instances (>= 0) */
    const int32_t* inst_sector; /* [n_inst] geometric sector 0..35 (0..17: A side, z > 0; 18..35: C side) */
    const int64_t* row_start;   /* [n_inst * n_rows + 1] CSR over (instance, row), as in tpcca_clusters */
    const float* pad;           /* [n_clusters] pad coordinate along the row (pad centres are integers) */
    const float* time;          /* [n_clusters] time since the start of the time frame [time bins] */
    int64_t n_clusters;         /* host value */
} tpcca_native_clusters;

/* The native-to-local transform, in binary32 with the operations in this
 * order: y = (pad - pad_center[row]) * pad_width[row];
 * z = side * (z_readout - z_per_bin * time), side = +1 on the A side, -1 on
 * the C side. The time is scaled linearly to z as if the chamber were
 * arbitrarily long (Section 4, the first step for continuous readout): the
 * clusters of a collision at time t_c appear shifted by -side * z_per_bin *
 * t_c, which the vertex z (tracks' z0) recovers. Writes y, z (device
 * [n_clusters] binary32, caller-owned). Errors: TPCCA_E_ARG (null pointers,
 * sizes; a malformed CSR leaves y, z of the clusters outside every row
 * unwritten), TPCCA_E_DEVICE. Does not synchronise. */
tpcca_status tpcca_native_to_local(tpcca_ctx* ctx, const tpcca_native_clusters* in, float* y, float* z,
                                   void* hip_stream);

/* Batched form of the track call on native clusters: no transformed copy of
 * the input is made; the grid kernel transforms each cluster as it reads it
 * (tpcca_native_to_local's arithmetic) and every later stage works on the
 * grid. Output bit for bit that of tpcca_track_batched on the clusters
 * tpcca_native_to_local gives, with z in the linear time scale (z0 is then
 * the vertex z in that scale). tpcca_merge may follow it as after the other
 * synchronous forms. Same errors and synchronisations as tpcca_track_batched. */
tpcca_status tpcca_track_native(tpcca_ctx* ctx, const tpcca_native_clusters* in, tpcca_tracks* out,
                                void* hip_stream);

/* Cross-sector merge (the second phase of Section 2: the track segments found
 * in the individual sectors are merged and fitted as one track; Section 4: the
 * fit follows the helix through rotations between sector frames) of the
 * output tracks of the last synchronous track call on ctx, which must have
 * been created with TPCCA_FLAG_MERGE (the track calls then keep the
 * outward-pass states and cluster rows the merge needs); that call's inputs
 * and outputs must still be valid.
 *   inst_event: device [n_inst] event (or time-frame) id of each instance:
 *     only segments of one event in phi-neighbouring sectors of one side are
 *     merged; an instance that is not the lowest of its (event, sector) is
 *     left as it is.
 * A segment continues as another when its state after the outward pass,
 * rotated into the other's frame and carried row by row (at most
 * params.merge_max_gap rows) to the other's reference row, agrees with the
 * other's fitted state within chi2 <= params.chi2_merge (five parameters);
 * mutual best pairs form chains of at most 8 segments, and each chain is
 * refitted over all its clusters with the three passes of the final fit,
 * rotating between frames. Output `merged` (tracks struct; z0, residuals
 * and chi2_total are not written): in sector-track order, a merged track at
 * its first segment (params in that segment's frame), other segments kept as
 * they are; a chain whose refit fails keeps its segments. nseg (device
 * [cap_tracks] or NULL): segments per output track. seg_next (device
 * [sector tracks] or NULL): the sector track each one was paired with as its
 * continuation (-1: none; also set for a chain whose refit failed).
 * Synchronises the stream once (the counts).
 * Errors: TPCCA_E_ARG (no usable previous call, flag missing, null
 * pointers), TPCCA_E_CAPACITY (merged->n_tracks / n_hits hold the sizes). */
tpcca_status tpcca_merge(tpcca_ctx* ctx, const int32_t* inst_event, tpcca_tracks* merged, int32_t* nseg,
                         int32_t* seg_next, void* hip_stream);

/* Allocation-free form of tpcca_track_async, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc. The same kernels and outputs as tpcca_track_async
 * (bit for bit), with every scratch buffer carved from one fixed static device
 * array of TPCCA_NOALLOC_SCRATCH_BYTES per device (resolved at context
 * creation, held until the process ends). It calls no hipMalloc, hipFree,
 * graph or stream creation and never waits: the kernels are enqueued on
 * hip_stream directly (the null stream is used as given). The caller still
 * passes inputs, outputs, counts and status (as for tpcca_track_async).
 * Limits: n_clusters <= TPCCA_NOALLOC_MAX_CLUSTERS and n_inst <=
 * TPCCA_NOALLOC_MAX_INST (these fit for n_rows <= 152; more pad rows need a
 * larger per-tracklet table); an input above them, or whose scratch layout
 * would exceed the array, returns TPCCA_E_CAPACITY before anything is
 * enqueued. Every call on one GPU, from any context, shares that GPU's array:
 * calls that overlap on one GPU race (serialise them on one stream). The
 * kernels clear what must start at zero themselves; exports are not
 * available after this call. */
#define TPCCA_NOALLOC_SCRATCH_BYTES (64u << 20)
#define TPCCA_NOALLOC_MAX_CLUSTERS 131072
#define TPCCA_NOALLOC_MAX_INST 64
tpcca_status tpcca_track_async_noalloc(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out,
                                       int64_t* counts, int32_t* status, void* hip_stream);

/* Autotuner of the batching form (a project extension: the paper gives no
 * tuning procedure). Time the batched form over candidate tunings on `sample`
 * (median of `repeats` runs each) and write the fastest to *out (also set on
 * ctx). Outputs go to internal buffers; results never depend on the tuning. */
tpcca_status tpcca_autotune(tpcca_ctx* ctx, const tpcca_clusters* sample, int32_t repeats,
                            tpcca_tuning* out, void* hip_stream);

/* ---- exports of intermediate results of the last track call (device
 * outputs in cluster-id space; sizes from tpcca_export_sizes). They expose
 * the per-stage results of Section 2 (grid, neighbour links before and after
 * the evolution step, tracklets, selected segments with the refit's accept
 * bits of Section 3) for stage-by-stage comparison. Each returns TPCCA_E_ARG
 * when no track call has completed on the context; asynchronous on
 * hip_stream. ---- */
/* host sizes[8]: n_clusters, n_segments, n_starts, n_selected, n_selected_hits, n_tracks, n_track_hits, n_rows */
tpcca_status tpcca_export_sizes(tpcca_ctx* ctx, int64_t* sizes, void* hip_stream);
/* sorted_id[n_clusters]: cluster id at each grid position; bin_start[n_clusters + n_segments + 1]
 * (segment s at offset row_start[s] + s); ny, nz[n_segments]; meta[n_segments*4]: ymin zmin inv_y inv_z */
tpcca_status tpcca_export_grid(tpcca_ctx* ctx, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz,
                               float* meta, void* hip_stream);
/* neighbour links and cleaned links per cluster id (-1 = none) */
tpcca_status tpcca_export_links(tpcca_ctx* ctx, int32_t* up, int32_t* dn, int32_t* up_clean, int32_t* dn_clean,
                                void* hip_stream);
/* per start (order instance, row, cluster id): start cluster, instance, tracklet id, nHits, rowhit
 * [n_starts * n_rows] (cluster id or -1), state [n_starts * 20] (p[5], C[15]), state row; weight[n_clusters] */
tpcca_status tpcca_export_tracklets(tpcca_ctx* ctx, int32_t* start_hit, int32_t* start_inst, int32_t* start_tid,
                                    int32_t* nhits, int32_t* rowhit, float* state, int32_t* state_row,
                                    uint32_t* weight, void* hip_stream);
/* per selected tracklet: tracklet index, hit_start[n_selected+1], owned cluster ids (ascending row),
 * refit accept bits per cluster (bit k = pass k+1), status (1 = output track) */
tpcca_status tpcca_export_selected(tpcca_ctx* ctx, int32_t* sel_tl, int64_t* hit_start, int32_t* hit_id,
                                   uint8_t* mask, int32_t* status, void* hip_stream);
tpcca_status tpcca_get_stats(tpcca_ctx* ctx, tpcca_stats* out); /* host out; syncs */
/* Stage timing of the last batched call (host out, ms): weights clear + grid, links, clean + starts,
 * tracklets, selection, refit, compaction into the outputs, FP64 totals. Filled only when the
 * context was created with TPCCA_FLAG_TIMING (the batched form then runs without graph capture). */
tpcca_status tpcca_get_stage_times(tpcca_ctx* ctx, float* ms8);

/* ---- Differentiable refit ----
 * The paper applies calibration corrections to the clusters between seeding
 * and the final fit (Sections 1 and 4). Here the chi2 of the three-pass refit
 * (Section 3) with FROZEN accept masks is a function of each track's start
 * state and of a smooth space-charge correction map; tpcca_refit_fwd evaluates
 * it and tpcca_refit_bwd returns its gradient (reverse mode, hand-written
 * adjoints of the row step, covariance reset and cluster update).
 *
 * Correction map: TPCCA_MAP_SIZE binary32 coefficients [comp][ir][iphi][iz]
 * (comp 0: delta r, 1: delta r*phi, 2: delta z, in cm), each component a
 * tricubic uniform B-spline with knots r_k = 84 + (k-1)*168/13 (k = 0..15),
 * phi_k = k*2pi/16 (periodic), z_k = -252 + (k-1)*504/29 (k = 0..31). A cluster
 * of row r with local (y, z) in a sector of angle alpha is corrected inside
 * its pad-row plane x = row_x[r]: R = sqrt(x^2 + y^2), phi = alpha + atan2(y, x),
 * y' = y - (dr*y + drphi*x)/R, z' = z - dz, with (dr, drphi, dz) the map at
 * (R, phi, z) (R and z clamped to the knot range).
 *
 * Refit per track (the refit of tpcca_track with masks given): start state
 * params0/cov0 at row0, step row by row to the outermost cluster, then passes
 * inward, outward, inward, each opening with a covariance reset; cluster i is
 * used in pass p iff bit p of hit_mask[i] is set. chi2 = sum of the predicted
 * chi2 of the clusters used in the last pass. A track whose row step leaves
 * the |sin phi| guard has chi2 0, track_ok 0 and zero gradient. */
#define TPCCA_MAP_SIZE (3 * 16 * 16 * 32)
#define TPCCA_FLAG_ADJOINT_F64 4u /* tpcca_refit_bwd: adjoint arithmetic in binary64 (default binary32) */

typedef struct {
    int64_t n_tracks;         /* host */
    int64_t n_hits;           /* host: hit_start[n_tracks] */
    const float* params0;     /* [n_tracks * 5] start state y, z, sin phi, tan lambda, q/pT */
    const float* cov0;        /* [n_tracks * 15] packed lower-triangular start covariance */
    const int32_t* row0;      /* [n_tracks] row of the start state, 0..n_rows-1 */
    const int32_t* inst;      /* [n_tracks] instance of the track's clusters */
    const int64_t* hit_start; /* [n_tracks + 1] CSR into hit_id; hit_start[0] = 0, at most n_rows per track */
    const int32_t* hit_id;    /* [n_hits] cluster ids of instance inst[t], rows strictly increasing */
    const uint8_t* hit_mask;  /* [n_hits] accept bits, bit p = used in pass p (p = 0, 1, 2) */
} tpcca_refit_set;

/* Forward. map_coef: device [TPCCA_MAP_SIZE] binary32, or NULL (no
 * correction). Outputs: chi2_track [n_tracks] (binary32, the refit's own
 * arithmetic: without a map it equals the tracker's chi2 bit for bit), track_ok
 * [n_tracks] (1/0, may be NULL), chi2_total [1] (FP64 sum, fixed order).
 * Validates the set on the device (ranges, cluster ids inside their instance,
 * strictly increasing rows): TPCCA_E_ARG otherwise. Synchronises the stream
 * twice (validation and operation counts, then errors).
 * record = 1 keeps what tpcca_refit_bwd needs: a tape of every operation's
 * inputs (covariance and operands, 76 bytes per operation, ~80 KB per track),
 * or, when the set's tape exceeds tuning.tape_mb, only the operation counts
 * (the backward then re-runs the forward batch by batch). The clusters, the set
 * and map_coef must then stay unchanged until tpcca_refit_bwd. record = 0:
 * forward only. */
tpcca_status tpcca_refit_fwd(tpcca_ctx* ctx, const tpcca_clusters* clusters, const tpcca_refit_set* set,
                             const float* map_coef, float* chi2_track, int32_t* track_ok, double* chi2_total,
                             int32_t record, void* hip_stream);

/* Backward of the last recorded tpcca_refit_fwd on this context, for the loss
 * L = sum_t grad_chi2[t] * chi2_track[t]. grad_chi2: device [n_tracks]
 * binary32. Outputs (FP64, device): grad_params0 [n_tracks * 5] = dL/dparams0;
 * grad_map [TPCCA_MAP_SIZE] = dL/dcoef (may be NULL; evaluated at the
 * forward's map, zero map if it was NULL; deterministic: every contribution is
 * rounded once to a 64-bit fixed-point integer scaled so that no partial sum can
 * exceed 2^61, the sums are exact integer additions in any order, and the result
 * is converted back to FP64); grad_hit_yz [n_hits * 2] =
 * dL/d(y', z') of each corrected cluster (may be NULL). Tracks whose refit
 * failed get zero gradients. Asynchronous; may be called again (another
 * grad_chi2) while the recorded forward stays valid. */
tpcca_status tpcca_refit_bwd(tpcca_ctx* ctx, const float* grad_chi2, double* grad_params0, double* grad_map,
                             double* grad_hit_yz, void* hip_stream);

/* Corrected final fit of the tracks of the last synchronous track call on ctx
 * (Section 4, continuous readout: with a track's vertex z, i.e. its collision
 * time, estimated, the space-point correction, which depends on the absolute
 * z, can be applied, and the track is fitted again). Per track: its output
 * clusters and its output state are moved to the absolute frame (z - z0), the
 * clusters corrected by the map in the form of tpcca_refit_fwd (none if
 * map_coef is NULL), and the three passes of the final fit (covariance reset,
 * chi2 <= chi2_rej acceptance) run again from that state. That call must have
 * written z0 (out->z0 not NULL); its inputs and outputs must still be valid.
 * Outputs (device, caller-owned, per track of that call): param [n*5] (z
 * absolute), cov [n*15], chi2 [n] (last pass), ndf [n] (2 accepted - 5, or -1
 * when a row step fails or fewer than n_min clusters are kept; the other
 * outputs of that track are then unspecified), x_ref [n], z0 [n] (refined:
 * the old z0 plus the closest approach of the new state), masks [n_hits] or
 * NULL (bit p: cluster used in pass p), hit_yz [n_hits * 2] or NULL (the
 * corrected coordinates, absolute z, binary32). Uses the differentiable refit's
 * scratch (a recorded forward is dropped). Does not synchronise. Errors:
 * TPCCA_E_ARG (no usable last call or no z0, null outputs), TPCCA_E_DEVICE,
 * TPCCA_E_OOM. */
tpcca_status tpcca_fit_corrected(tpcca_ctx* ctx, const float* map_coef, float* param, float* cov, float* chi2,
                                 int32_t* ndf, float* x_ref, float* z0, uint8_t* masks, float* hit_yz,
                                 void* hip_stream);

/* Arithmetic self-check: out_div[i] = a[i] / b[i], out_sqrt[i] = sqrt(|a[i]|) with the
 * library's binary32 operations (for bit comparison with a CPU). Synchronous. */
tpcca_status tpcca_fp32_selfcheck(const float* a, const float* b, float* out_div, float* out_sqrt, int64_t n,
                                  void* hip_stream);

/* Self-check of the square root in the helix step (Section 3's track model;
 * the step takes roots of 1 - sin^2 phi and of 1 + tan^2). It adds to
 * *count (device memory, caller-initialised) the number of binary32 bit
 * patterns x in [first, last] (as unsigned integers) for which that root
 * differs from the correctly rounded sqrtf; two NaN results count as equal.
 * The root is exact for +-0, for normal arguments of at least 2^-96, for +inf,
 * negative arguments and NaN. Synchronous. Errors: TPCCA_E_ARG (null count,
 * first > last), TPCCA_E_DEVICE. */
tpcca_status tpcca_sqrt_step_check(uint32_t first, uint32_t last, unsigned long long* count, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* TPCCA_H */
