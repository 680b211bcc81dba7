// Internal interface of the differentiable refit (adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_device.h"

namespace tpcca {

constexpr int kMapSize = 3 * 16 * 16 * 32;
constexpr int kCk = 32;         // refit operations per checkpoint segment
constexpr int kCkWords = 26;    // iterator (4) + state (5) + covariance (15) + reference point (2)
constexpr int kTapeWords = 19;  // covariance (15) + three operands + operation word

enum : uint32_t {
    AERR_RANGE = 1u,  // hit_start, instance or start row out of range
    AERR_HIT = 2u,    // a cluster id outside its track's instance
    AERR_ROWS = 4u,   // cluster rows of a track not strictly increasing
    AERR_CKPT = 8u,   // checkpoint bound exceeded (never with valid rows)
};

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
    // scratch (SoA over tracks: word f of slot k of track t at (k * words + f) * n_tracks + t)
    int32_t* hit_inst;
    uint8_t* hit_row;
    float2* hit_yz;
    double2* hit_grad;
    int32_t* nops;
    uint32_t* ckpt;
    uint32_t* tape;
    int32_t max_ck;
    uint32_t* err;
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

int64_t adj_max_ops(int n_rows);
void enqueue_adj_clear(const AdjBufs& a, hipStream_t st);
void enqueue_refit_fwd(const AdjBufs& a, hipStream_t st);
void enqueue_refit_bwd(const AdjBufs& a, hipStream_t st);

}  // namespace tpcca
