// Internal interface of the differentiable refit (adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_device.h"

namespace tpcca {

constexpr int kMapSize = 3 * 16 * 16 * 32;
constexpr int kTapeWords = 20;  // per operation: covariance (15), three operands, operation word, pad
constexpr int64_t kTapeBytesPerOp = 4 * kTapeWords;

enum : uint32_t {
    AERR_RANGE = 1u,  // hit_start, instance or start row out of range
    AERR_HIT = 2u,    // a cluster id outside its track's instance
    AERR_ROWS = 4u,   // cluster rows of a track not strictly increasing
    AERR_TAPE = 8u,   // operation count above the tape stride (never with valid rows)
};

// words of the small status block (device): error bits, max operation count
struct AdjStatus {
    uint32_t err;
    int32_t max_ops;      // operations of the whole refit, largest over the set
    int32_t max_seg_ops;  // operations of one pass segment (the walk belongs to the first), largest
    int32_t pad;
};

constexpr int kCkptWords = 24;  // per pass start: state (5 + 15), reference point (2), row, pad

struct AdjBufs {
    const DevConsts* K;
    int n_rows;
    int32_t n_inst;
    int64_t n_clusters;
    const int32_t* inst_sector;
    const int64_t* row_start;
    const float* y;
    const float* z;
    // refit set
    int64_t n_tracks, n_hits;
    const float* params0;
    const float* cov0;
    const int32_t* row0;
    const int32_t* inst;
    const int64_t* hit_start;
    const int32_t* hit_id;
    const uint8_t* hit_mask;
    const float* coef;  // may be null: no correction
    // scratch
    int32_t* hit_inst;    // [n_hits]
    uint8_t* hit_row;     // [n_hits]
    float2* hit_yz;       // [n_hits] corrected coordinates
    double2* hit_grad;    // [3][n_hits] d/d(y', z') per pass
    int32_t* nops;        // [n_tracks] operations of the last recorded forward (-1: failed)
    uint32_t* tape;       // operation k of batch track b at word (b * tape_ops + k) * kTapeWords
    int32_t tape_ops;     // operations per track the tape holds (the set's maximum, or a segment's)
    float* ckpt;          // [3][n_tracks][kCkptWords] pass-start checkpoints, or null (full tape)
    int32_t* seg_nops;    // [n_tracks] operations of the last recomputed segment
    double* carry;        // [n_tracks][20] adjoint of (state, covariance) between segments
    AdjStatus* status;
    // outputs
    float* chi2_track;
    int32_t* track_ok;
    double* chi2_total;
    // backward
    const float* grad_chi2;
    double* grad_params;
    double* grad_map;
    int32_t adj_f64;
};

// Enqueue validation, corrected coordinates and operation counts (status
// block: error bits and the largest operation count, for the host to size
// the tape).
void enqueue_refit_prepare(const AdjBufs& a, hipStream_t st);
// Forward over tracks [t0, t1): chi2 per track (when `outputs`), operation
// counts, and the tape of those tracks when a.tape is set. With a.ckpt set the
// full forward stores each pass's starting point there.
void enqueue_refit_forward(const AdjBufs& a, int64_t t0, int64_t t1, bool outputs, hipStream_t st);
// Recompute pass `seg` (seg 0 includes the walk to the outermost cluster) of
// tracks [t0, t1) from its checkpoint, recording its operations on the tape.
void enqueue_refit_segment(const AdjBufs& a, int64_t t0, int64_t t1, int seg, hipStream_t st);
void enqueue_refit_total(const AdjBufs& a, hipStream_t st);
// Reverse sweep over the taped tracks [t0, t1): the whole refit (seg < 0), or
// one recomputed pass segment, whose adjoint is carried to the next (earlier)
// segment in a.carry.
void enqueue_refit_reverse(const AdjBufs& a, int64_t t0, int64_t t1, int seg, hipStream_t st);
// The corrected final fit of the last track call's tracks (tpcca_fit_corrected).
struct CorrBufs {
    const DevConsts* K;
    int n_rows;
    const int32_t* inst_sector;
    const int64_t* row_start;
    const float2* yz;        // grid coordinates of the last call
    const int32_t* pos_of;   // grid position of each cluster id
    int64_t n_tracks, n_hits;
    const int32_t* inst;     // the last call's outputs
    const float* param;
    const float* cov;
    const float* xref;
    const float* z0;
    const int64_t* hit_start;
    const int32_t* hit_id;
    const float* coef;       // may be null: no correction
    float2* cyz;             // scratch [n_hits]: corrected coordinates, absolute frame
    uint8_t* crow;           // scratch [n_hits]: pad row
    float* o_param;          // outputs
    float* o_cov;
    float* o_chi2;
    int32_t* o_ndf;
    float* o_xref;
    float* o_z0;
    uint8_t* o_mask;         // may be null
    float* o_hit_yz;         // may be null: corrected coordinates [n_hits * 2]
};

void enqueue_fit_corrected(const CorrBufs& c, hipStream_t st);

// Map gradient (grad_map) and per-cluster gradient (sum over passes) from the
// reverse sweeps; the map gradient uses map_grad_scratch_bytes(n_hits) of scratch.
size_t map_grad_scratch_bytes(int64_t n_hits);
void enqueue_refit_map_grad(const AdjBufs& a, void* scratch, hipStream_t st);
void enqueue_refit_hit_grad(const AdjBufs& a, double* out, hipStream_t st);

}  // namespace tpcca
