// Internal interface between the host runtime (api.hip) and the kernels
// (kernels.hip). Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_device.h"

namespace tpcca {

// error bits raised by kernels
enum : uint32_t {
    ERR_ARG = 1u,        // malformed CSR / non-finite coordinate
    ERR_ROW_CAP = 2u,    // more than TPCCA_MAX_ROW_CLUSTERS on one row of one instance
    ERR_TID_CAP = 4u,    // more than 2^20 tracklets in one instance
    ERR_OUT_CAP = 8u,    // output capacity exceeded
    ERR_SCRATCH = 16u,   // internal scratch bound violated (should not happen)
    ERR_CSR = 32u,       // raised only by the device CSR check before any stage runs:
                         // every stage kernel then returns at entry (constant during them)
};

// statistics slots
enum {
    ST_LINKS = 0, ST_NB_CAND_U, ST_NB_PAIRS, ST_CHAIN_HITS, ST_TL_ROWS, ST_TL_CAND, ST_TL_PICKS,
    ST_RF_ROWS, ST_RF_HITS, ST_COUNT
};

// Running totals of the three compactions (starts, selected, tracks); each
// slot holds {running total, base of the current range, count of the current
// range} as packed (hi 32: items, lo 32: sub-items) 64-bit sums.
enum { SL_START = 0, SL_SEL = 1, SL_TRK = 2, SL_MRG = 3 };
struct Counters {
    unsigned long long slot[4][3];
    unsigned int err;
    unsigned int pad;
    unsigned int tlq[8];  // queues of the persistent inward-pass kernel (one per XCD)
    unsigned long long stats[ST_COUNT];
};

// Per-(instance, row) grid header, one 32-byte load: first grid position and
// count of the row's clusters, bin counts, lower corner and inverse bin sizes.
struct alignas(32) SegHdr {
    int32_t rs, n, ny, nz;
    float ymin, zmin, iy, iz;
};

// All device buffers of one call (scratch + caller arrays).
struct Bufs {
    const DevConsts* K;
    Counters* ctr;
    int n_rows;  // host copy of K->n_rows
    // input
    int32_t n_inst;
    int64_t n_clusters;
    const int32_t* inst_sector;
    const int64_t* row_start;
    const float* y;      // local y, or the pad coordinate when native
    const float* z;      // local z, or the time when native
    int native;          // 1: (y, z) hold native (pad, time), transformed where the grid reads them
    // grid
    float2* yz;        // (y, z) at grid position
    int32_t* sid;      // cluster id at grid position
    int32_t* pos_of;   // grid position of cluster id
    int32_t* bin_start;
    SegHdr* hdr;
    int hits_per_bin;
    // CA (grid-position space)
    int32_t* up;
    int32_t* dn;
    int32_t* upc;
    int32_t* dnc;
    uint8_t* start_flag; // [N] grid-position space: 1 at a start hit (written by the cleaning)
    // starts and tracklets
    int64_t cap_starts;
    int32_t* starts;     // grid position of the start hit
    int32_t* start_inst;
    int32_t* seed_order; // split form: processing order of the inward passes (permutation of the start range)
    int32_t* tl_last;    // last row with a cluster after the outward following
    int32_t* tl_nhits;
    int32_t* tl_tid;
    int32_t* tl_row;
    float* tl_state;     // [cap_starts * 20]
    int32_t* tl_pick_pos;  // [cap_starts * n_rows], stage-3 order (rows descending)
    uint8_t* tl_pick_row;
    uint32_t* weight;    // [N] grid-position space
    int32_t* tl_own;     // owned clusters per tracklet (0 if it has fewer than n_min hits)
    uint32_t* tl_ownmask;  // [cap_starts * 8] bit k: pick k is owned
    // selection
    int64_t cap_sel;
    int32_t* sel_tl;
    int32_t* sel_off;
    int32_t* sel_n;
    int32_t* sel_pos;    // [N]
    float2* sel_yz;      // [N] coordinates of the selected clusters (gathered for the refit)
    uint8_t* sel_row;    // [N]
    uint8_t* sel_mask;   // [N]
    // refit results per selected
    float* rf_state;     // [cap_sel * 20]
    float* rf_chi2;
    int32_t* rf_nacc;
    int32_t* rf_row;
    int32_t* rf_ok;
    int32_t* trk_t;      // [cap_sel] output track index of a selected tracklet (-1: none)
    int32_t* trk_ho;     // [cap_sel] its first output hit
    // scan scratch
    unsigned long long* scan_part;  // [kScanBlocks]
    // outputs
    int64_t cap_tracks, cap_hits;
    int32_t* o_inst;
    float* o_xref;
    float* o_alpha;
    float* o_param;
    float* o_cov;
    float* o_chi2;
    int32_t* o_ndf;
    int64_t* o_hit_start;
    int32_t* o_hit_id;
    double* o_chi2_total;
    float* o_z0;         // may be null
    int16_t* o_res;      // may be null: compression residuals [cap_hits * 2]
    float res_scale;     // 1 / residual step (a power of two)
    uint32_t* sel_res;   // [N] packed (y, z) int16 residuals per selected cluster
    // kept for the cross-sector merge (TPCCA_FLAG_MERGE)
    int keep_merge;
    float* rf_state2;    // [cap_sel * 20] state after the outward pass (absolute y, z)
    int32_t* rf_row2;    // [cap_sel] its row
    int32_t* trk_si;     // [cap_sel] selected index of output track t
    uint8_t* trk_hrow;   // [N] row of output cluster q
};

// The cross-sector merge of the last track call's output tracks.
struct MergeBufs {
    Bufs b;                       // the last track call (its inputs and outputs must still be valid)
    const int32_t* inst_event;    // [n_inst] event of each instance
    int64_t n_t;                  // sector tracks of that call
    int64_t n_h;                  // their output clusters
    // scratch
    int32_t* nb;                  // [n_inst * 2] neighbour instance per direction (-1: none)
    int32_t* rcnt;                // [n_inst * n_rows + 1] tracks per (instance, reference row)
    int32_t* rstart;              // [n_inst * n_rows + 1]
    int32_t* rfill;               // [n_inst * n_rows]
    int32_t* rids;                // [n_t] tracks bucketed by (instance, reference row)
    int32_t* best_out;            // [n_t]
    unsigned long long* best_in;  // [n_t] (chi2 bits << 32) | partner
    int32_t* next;                // [n_t]
    int32_t* prev;                // [n_t]
    int32_t* ok;                  // [n_t] merged refit of the chain starting here succeeded
    uint8_t* absorbed;            // [n_t] segment of a merged chain after its first
    float* state;                 // [n_t * 20]
    float* chi2;                  // [n_t]
    int32_t* nacc;                // [n_t]
    int32_t* row;                 // [n_t]
    int32_t* nseg;                // [n_t]
    uint8_t* acc3;                // [n_hits] kept by the merged refit's last pass
    float2* hyz;                  // [n_hits] coordinates of each output cluster
    int32_t* heads;               // [n_t] chain heads (first nheads entries)
    unsigned int* nheads;         // [1]
    int32_t* out_t;               // [n_t] output index
    int64_t* out_h;               // [n_t] first output cluster
    // outputs
    int64_t cap_tracks, cap_hits;
    int32_t* o_inst;
    float* o_xref;
    float* o_alpha;
    float* o_param;
    float* o_cov;
    float* o_chi2;
    int32_t* o_ndf;
    int64_t* o_hit_start;
    int32_t* o_hit_id;
    int32_t* o_nseg;              // may be null
    int32_t* seg_next;            // may be null: [n_t] outer partner of each sector track in the output
};

void enqueue_merge(const MergeBufs& m, hipStream_t st);

struct Launch {
    int block_links, block_tracklet, block_refit, block_scan, sort_seeds, xcd_remap, inward_wgs, inward_sort;
};

constexpr int kScanBlocks = 1024;

// Instance range [i0, i1) with its cluster range [c0, c1) (host values).
void enqueue_reset(const Bufs& b, hipStream_t st);
void enqueue_weights_clear(const Bufs& b, int64_t c0, int64_t c1, hipStream_t st);
void enqueue_grid(const Bufs& b, int i0, int i1, int max_row, hipStream_t st);  // max_row: largest row (bound)
void enqueue_links(const Bufs& b, const Launch& L, int i0, int i1, int max_row, hipStream_t st);
void enqueue_clean_starts(const Bufs& b, const Launch& L, int i0, int i1, int64_t c0, int64_t c1, hipStream_t st);
void enqueue_tracklets(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st);
void enqueue_select(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st);
void enqueue_refit(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st);
void enqueue_write(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st);
void enqueue_finish(const Bufs& b, hipStream_t st);
// device-side input check (the forms that do not read row_start to the host)
void enqueue_check_csr(const Bufs& b, hipStream_t st);
// counts (n_tracks, n_hits) and a tpcca_status code left on the device
void enqueue_async_status(const Bufs& b, int64_t* counts, int32_t* status, hipStream_t st);

// native (pad, time) -> local (y, z) of every cluster (b.native must be 1)
void enqueue_native_local(const Bufs& b, int64_t nseg, float* y, float* z, hipStream_t st);

// exports (cluster-id space)
void enqueue_export_grid(const Bufs& b, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz,
                         float* meta, int64_t nseg, hipStream_t st);
void enqueue_export_links(const Bufs& b, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc, hipStream_t st);
void enqueue_export_tracklets(const Bufs& b, int64_t n_starts, int32_t* start_hit, int32_t* start_inst,
                              int32_t* start_tid, int32_t* nhits, int32_t* rowhit, float* state,
                              int32_t* state_row, uint32_t* weight, hipStream_t st);
void enqueue_export_selected(const Bufs& b, int64_t n_sel, int32_t* sel_tl, int64_t* hit_start, int32_t* hit_id,
                             uint8_t* mask, int32_t* status, hipStream_t st);
void enqueue_fp32_selfcheck(const float* a, const float* bb, float* od, float* os, int64_t n, hipStream_t st);
void enqueue_sqrt_step_check(uint32_t first, uint32_t last, unsigned long long* count, hipStream_t st);

}  // namespace tpcca
