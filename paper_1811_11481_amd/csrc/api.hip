// Host runtime of the TPC sector tracker: the C ABI declared in
// include/tpcca.h. Owns the per-context constants and scratch arena, checks
// inputs, enqueues the stage kernels (per instance for the plain form, once
// over all instances for the batched form), captures the batched sequence in
// a HIP graph, and reads back the track counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpcca.h"
#include "adjoint.h"
#include "internal.h"

using namespace tpcca;

// Scratch of the allocation-free entry point: one fixed array per device,
// held by every device the library is loaded on until the process ends. Host
// code never uses this name as an address: the per-device address comes from
// hipGetSymbolAddress at context creation.
static __device__ __align__(256) unsigned char scratch[TPCCA_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr double kPi = 3.14159265358979323846;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Arena {
    void* base = nullptr;
    size_t bytes = 0;
    int64_t N = -1, nseg = -1, ninst = -1;
    int nr = 0;
};

// Everything a captured launch sequence depends on: every device pointer its
// kernels take (each in its own slot), the stream, sizes and tuning.
struct GraphKey {
    const void* p[21];
    int64_t v[10];
    bool operator==(const GraphKey& o) const {
        return std::memcmp(p, o.p, sizeof(p)) == 0 && std::memcmp(v, o.v, sizeof(v)) == 0;
    }
};

}  // namespace

struct tpcca_ctx {
    int device = 0;
    tpcca_params params{};
    tpcca_tuning tuning{};
    DevConsts hK{};
    DevConsts* dK = nullptr;
    Counters* dctr = nullptr;
    Counters* hctr = nullptr;  // pinned
    int64_t* h_rowstart = nullptr;  // pinned
    size_t h_rowstart_cap = 0;
    Arena arena;
    std::string err;
    // last call
    bool has_last = false;
    Bufs last{};
    int64_t last_nseg = 0;
    Counters last_ctr{};
    // graph of the batched form
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey{};
    bool has_graph = false;
    // stage timing
    hipEvent_t ev[9] = {};
    hipStream_t own_stream = nullptr;
    bool events = false;
    float stage_ms[8] = {};
    void* noalloc = nullptr;  // this device's address of the static scratch array
    void* mg_base = nullptr;  // scratch of the cross-sector merge, grown on demand
    size_t mg_bytes = 0;
    // differentiable refit: per-track / per-cluster scratch, tape, status, last forward
    void* adj_base = nullptr;
    size_t adj_bytes = 0;
    int64_t adj_cap_t = -1, adj_cap_h = -1;
    void* tape_base = nullptr;
    size_t tape_bytes = 0;
    AdjStatus* h_adj_status = nullptr;  // pinned
    AdjBufs adj{};
    bool adj_valid = false;   // a recorded forward is available to tpcca_refit_bwd
    bool adj_taped = false;   // ... and its tape covers the whole set
    int64_t adj_batch = 0;    // tracks per batch when the backward recomputes
};

namespace {

tpcca_status fail(tpcca_ctx* c, tpcca_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

tpcca_status hip_fail(tpcca_ctx* c, hipError_t e, const char* where) {
    return fail(c, e == hipErrorOutOfMemory ? TPCCA_E_OOM : TPCCA_E_DEVICE,
                std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

void build_consts(const tpcca_params& p, DevConsts& K) {
    std::memset(&K, 0, sizeof(K));
    K.n_rows = p.n_rows;
    K.n_min = p.n_min;
    K.max_miss = p.max_miss;
    K.stats = (p.flags & TPCCA_FLAG_STATS) ? 1 : 0;
    for (int i = 0; i < p.n_rows; ++i) K.X[i] = p.row_x[i];
    const float ty = (float)p.win_ty, tz = (float)p.win_tz, ny = (float)p.win_ny, nz = (float)p.win_nz;
    for (int r = 1; r + 1 < p.n_rows; ++r) {
        const float du = K.X[r + 1] - K.X[r];
        const float dd = K.X[r] - K.X[r - 1];
        K.wyu[r] = du * ty + ny;
        K.wzu[r] = du * tz + nz;
        K.wyd[r] = dd * ty + ny;
        K.wzd[r] = dd * tz + nz;
        K.tr[r] = (K.X[r] - K.X[r - 1]) / (K.X[r + 1] - K.X[r - 1]);
    }
    for (int s = 0; s < 18; ++s) K.alpha[s] = (float)((s + 0.5) * 20.0 * kPi / 180.0);
    K.kB = (float)(-0.00299792458 * p.bz);
    K.kB_f64 = -0.00299792458 * p.bz;
    K.chi2_merge = (float)p.chi2_merge;
    K.merge_max_gap = p.merge_max_gap;
    for (int i = 0; i < p.n_rows; ++i) {
        K.pad_w[i] = p.pad_width[i];
        K.pad_c[i] = p.pad_center[i];
    }
    K.z_per_bin = (float)p.z_per_bin;
    K.z_readout = (float)p.z_readout;
    K.rot_c = (float)std::cos(20.0 * kPi / 180.0);
    K.rot_s = (float)std::sin(20.0 * kPi / 180.0);
    const float sy = (float)p.sigma_y, sz = (float)p.sigma_z;
    K.vy = sy * sy;
    K.vz = sz * sz;
    K.smax = (float)p.nbr_score_max;
    K.nsig = (float)p.nsig;
    K.chi2_pick = (float)p.chi2_pick;
    K.chi2_rej = (float)p.chi2_rej;
    K.sinphi_max = (float)p.sinphi_max;
    K.cov_reset = (float)p.cov_reset;
    K.q_max = (float)p.q_max;
    const float um = (float)p.u_max;
    K.u_max2 = um * um;
    for (int i = 0; i < 5; ++i) K.c0[i] = (float)p.c0[i];
}

tpcca_status check_params(tpcca_ctx* ctx, const tpcca_params& p) {
    if (p.n_rows < 3 || p.n_rows > TPCCA_MAX_ROWS) return fail(ctx, TPCCA_E_ARG, "n_rows must be in [3, 255]");
    for (int i = 1; i < p.n_rows; ++i)
        if (!(p.row_x[i] > p.row_x[i - 1])) return fail(ctx, TPCCA_E_ARG, "row_x must be strictly increasing");
    if (!(p.sigma_y > 0) || !(p.sigma_z > 0)) return fail(ctx, TPCCA_E_ARG, "cluster errors must be positive");
    if (!(p.sinphi_max > 0 && p.sinphi_max < 1)) return fail(ctx, TPCCA_E_ARG, "sinphi_max must be in (0, 1)");
    if (p.n_min < 3 || p.n_min > p.n_rows) return fail(ctx, TPCCA_E_ARG, "n_min must be in [3, n_rows]");
    if (p.max_miss < 1) return fail(ctx, TPCCA_E_ARG, "max_miss must be >= 1");
    if (!(p.u_max > 0 && p.u_max <= 0.5)) return fail(ctx, TPCCA_E_ARG, "u_max must be in (0, 0.5]");
    if (!(p.chi2_merge > 0)) return fail(ctx, TPCCA_E_ARG, "chi2_merge must be positive");
    if (p.merge_max_gap < 0 || p.merge_max_gap > 255) return fail(ctx, TPCCA_E_ARG, "merge_max_gap must be in [0, 255]");
    for (int i = 0; i < p.n_rows; ++i)
        if (!(p.pad_width[i] > 0.0f && p.pad_width[i] < 1e30f) || !(std::fabs(p.pad_center[i]) < 1e30f))
            return fail(ctx, TPCCA_E_ARG, "pad_width must be positive and pad_center finite on every row");
    if (!(p.z_per_bin > 0 && p.z_per_bin < 1e30) || !(std::fabs(p.z_readout) < 1e30))
        return fail(ctx, TPCCA_E_ARG, "z_per_bin must be positive and z_readout finite");
    return TPCCA_OK;
}

tpcca_status check_tuning(tpcca_ctx* ctx, const tpcca_tuning& t) {
    auto okb = [](int v) { return v >= 64 && v <= 1024 && (v % 64) == 0; };
    if (t.hits_per_bin < 1 || t.hits_per_bin > 64) return fail(ctx, TPCCA_E_ARG, "hits_per_bin must be in [1, 64]");
    if (!okb(t.block_links) || !okb(t.block_tracklet) || !okb(t.block_refit) || !okb(t.block_scan))
        return fail(ctx, TPCCA_E_ARG, "block sizes must be multiples of 64 in [64, 1024]");
    if (t.block_tracklet > 256 || t.block_refit > 256)
        return fail(ctx, TPCCA_E_ARG, "tracklet and refit blocks hold at most 256 threads");
    if (t.tape_mb < 1) return fail(ctx, TPCCA_E_ARG, "tape_mb must be >= 1");
    if (t.xcd_remap != 0 && t.xcd_remap != 1) return fail(ctx, TPCCA_E_ARG, "xcd_remap must be 0 or 1");
    if (t.ckpt != 0 && t.ckpt != 1) return fail(ctx, TPCCA_E_ARG, "ckpt must be 0 or 1");
    if (t.inward_wgs < 0 || t.inward_wgs > 65536) return fail(ctx, TPCCA_E_ARG, "inward_wgs must be in [0, 65536]");
    if (t.inward_sort != 0 && t.inward_sort != 1) return fail(ctx, TPCCA_E_ARG, "inward_sort must be 0 or 1");
    if (t.sort_seeds < 0 || t.sort_seeds > 2) return fail(ctx, TPCCA_E_ARG, "sort_seeds must be 0, 1 or 2");
    return TPCCA_OK;
}

// Scratch layout for N clusters, nseg segments, ninst instances.
struct Layout {
    size_t off[64];
    int k = 0;
    size_t total = 0;
    size_t add(size_t bytes) {
        off[k] = total;
        total += align256(bytes ? bytes : 1);
        return off[k++];
    }
};

void carve(tpcca_ctx* ctx, Bufs& b, int64_t N, int64_t nseg, int64_t ninst, bool really, size_t* total,
           void* at = nullptr) {
    const int nr = ctx->params.n_rows;
    const int64_t cap_s = N / 3 + ninst + 1;
    const int64_t cap_sel = N / std::max(1, ctx->params.n_min) + ninst + 1;
    Layout L;
    size_t o_yz = L.add(8 * N), o_sid = L.add(4 * N), o_pos = L.add(4 * N);
    size_t o_bs = L.add(4 * (N + nseg + 1)), o_hdr = L.add(sizeof(SegHdr) * nseg);
    size_t o_up = L.add(4 * N), o_dn = L.add(4 * N), o_upc = L.add(4 * N), o_dnc = L.add(4 * N), o_sf = L.add(N);
    size_t o_st = L.add(4 * cap_s), o_sti = L.add(4 * cap_s), o_so = L.add(4 * cap_s), o_sl = L.add(4 * cap_s);
    size_t o_tn = L.add(4 * cap_s), o_tt = L.add(4 * cap_s), o_tr = L.add(4 * cap_s), o_ts = L.add(80 * cap_s);
    size_t o_tpp = L.add(4 * cap_s * nr), o_tpr = L.add((size_t)cap_s * nr);
    size_t o_w = L.add(4 * N), o_own = L.add(4 * cap_s), o_ownm = L.add(32 * cap_s);
    size_t o_sel = L.add(4 * cap_sel), o_soff = L.add(4 * cap_sel), o_sn = L.add(4 * cap_sel);
    size_t o_spos = L.add(4 * N), o_syz = L.add(8 * N), o_srow = L.add(N), o_smask = L.add(N), o_sres = L.add(4 * N);
    size_t o_rs = L.add(80 * cap_sel), o_rc = L.add(4 * cap_sel), o_rn = L.add(4 * cap_sel),
           o_rr = L.add(4 * cap_sel), o_rok = L.add(4 * cap_sel), o_kt = L.add(4 * cap_sel), o_kho = L.add(4 * cap_sel);
    size_t o_part = L.add(8 * kScanBlocks);
    const bool km = (ctx->params.flags & TPCCA_FLAG_MERGE) != 0;
    size_t o_rs2 = L.add(km ? 80 * cap_sel : 0), o_rr2 = L.add(km ? 4 * cap_sel : 0),
           o_tsi = L.add(km ? 4 * cap_sel : 0), o_thr = L.add(km ? N : 0);
    *total = L.total;
    if (!really) return;
    char* base = (char*)(at ? at : ctx->arena.base);
    b.yz = (float2*)(base + o_yz);
    b.sid = (int32_t*)(base + o_sid);
    b.pos_of = (int32_t*)(base + o_pos);
    b.bin_start = (int32_t*)(base + o_bs);
    b.hdr = (SegHdr*)(base + o_hdr);
    b.up = (int32_t*)(base + o_up);
    b.dn = (int32_t*)(base + o_dn);
    b.upc = (int32_t*)(base + o_upc);
    b.dnc = (int32_t*)(base + o_dnc);
    b.start_flag = (uint8_t*)(base + o_sf);
    b.cap_starts = cap_s;
    b.starts = (int32_t*)(base + o_st);
    b.start_inst = (int32_t*)(base + o_sti);
    b.seed_order = (int32_t*)(base + o_so);
    b.tl_last = (int32_t*)(base + o_sl);
    b.tl_nhits = (int32_t*)(base + o_tn);
    b.tl_tid = (int32_t*)(base + o_tt);
    b.tl_row = (int32_t*)(base + o_tr);
    b.tl_state = (float*)(base + o_ts);
    b.tl_pick_pos = (int32_t*)(base + o_tpp);
    b.tl_pick_row = (uint8_t*)(base + o_tpr);
    b.weight = (uint32_t*)(base + o_w);
    b.tl_own = (int32_t*)(base + o_own);
    b.tl_ownmask = (uint32_t*)(base + o_ownm);
    b.cap_sel = cap_sel;
    b.sel_tl = (int32_t*)(base + o_sel);
    b.sel_off = (int32_t*)(base + o_soff);
    b.sel_n = (int32_t*)(base + o_sn);
    b.sel_pos = (int32_t*)(base + o_spos);
    b.sel_yz = (float2*)(base + o_syz);
    b.sel_row = (uint8_t*)(base + o_srow);
    b.sel_mask = (uint8_t*)(base + o_smask);
    b.sel_res = (uint32_t*)(base + o_sres);
    b.rf_state = (float*)(base + o_rs);
    b.rf_chi2 = (float*)(base + o_rc);
    b.rf_nacc = (int32_t*)(base + o_rn);
    b.rf_row = (int32_t*)(base + o_rr);
    b.rf_ok = (int32_t*)(base + o_rok);
    b.trk_t = (int32_t*)(base + o_kt);
    b.trk_ho = (int32_t*)(base + o_kho);
    b.scan_part = (unsigned long long*)(base + o_part);
    b.keep_merge = km ? 1 : 0;
    b.rf_state2 = (float*)(base + o_rs2);
    b.rf_row2 = (int32_t*)(base + o_rr2);
    b.trk_si = (int32_t*)(base + o_tsi);
    b.trk_hrow = (uint8_t*)(base + o_thr);
}

tpcca_status ensure_arena(tpcca_ctx* ctx, int64_t N, int64_t nseg, int64_t ninst) {
    Arena& A = ctx->arena;
    if (A.base && N <= A.N && nseg <= A.nseg && ninst <= A.ninst && A.nr == ctx->params.n_rows) return TPCCA_OK;
    const int64_t n2 = std::max(N, A.N), s2 = std::max(nseg, A.nseg), i2 = std::max(ninst, A.ninst);
    Bufs tmp{};
    size_t total = 0;
    carve(ctx, tmp, n2, s2, i2, false, &total);
    if (A.base) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(A.base));
        A.base = nullptr;
    }
    if (ctx->has_graph) {
        (void)hipGraphExecDestroy(ctx->gexec);
        (void)hipGraphDestroy(ctx->graph);
        ctx->has_graph = false;
    }
    ctx->has_last = false;
    hipError_t e = hipMalloc(&A.base, total);
    if (e != hipSuccess) {
        A.base = nullptr;
        A.N = A.nseg = A.ninst = -1;
        return hip_fail(ctx, e, "scratch allocation");
    }
    A.bytes = total;
    A.N = n2;
    A.nseg = s2;
    A.ninst = i2;
    A.nr = ctx->params.n_rows;
    return TPCCA_OK;
}

tpcca_status check_io(tpcca_ctx* ctx, const tpcca_clusters* in, const tpcca_tracks* out) {
    if (!ctx) return TPCCA_E_ARG;
    if (!in || !out) return fail(ctx, TPCCA_E_ARG, "null clusters or tracks");
    if (in->n_inst < 0 || in->n_clusters < 0) return fail(ctx, TPCCA_E_ARG, "negative sizes");
    if (in->n_clusters >= (int64_t)1 << 31) return fail(ctx, TPCCA_E_ARG, "more than 2^31-1 clusters");
    if (in->n_inst > 0 && (!in->row_start || !in->inst_sector))
        return fail(ctx, TPCCA_E_ARG, "null row_start or inst_sector");
    if (in->n_clusters > 0 && (!in->y || !in->z)) return fail(ctx, TPCCA_E_ARG, "null cluster coordinates");
    if (out->cap_tracks < 0 || out->cap_hits < 0) return fail(ctx, TPCCA_E_ARG, "negative capacities");
    if (!out->hit_start || !out->chi2_total) return fail(ctx, TPCCA_E_ARG, "null hit_start or chi2_total");
    if (out->cap_tracks > 0 && (!out->inst || !out->x_ref || !out->alpha || !out->param || !out->cov ||
                                !out->chi2 || !out->ndf))
        return fail(ctx, TPCCA_E_ARG, "null track arrays");
    if (out->cap_hits > 0 && !out->hit_id) return fail(ctx, TPCCA_E_ARG, "null hit_id");
    if (out->residuals && (out->residual_step_log2 < -20 || out->residual_step_log2 > 4))
        return fail(ctx, TPCCA_E_ARG, "residual_step_log2 must be in [-20, 4]");
    return TPCCA_OK;
}

// Read row_start to the host and check the CSR (monotone, within [0, N]).
tpcca_status load_rowstart(tpcca_ctx* ctx, const tpcca_clusters* in, hipStream_t st) {
    const int64_t n = (int64_t)in->n_inst * ctx->params.n_rows + 1;
    if (in->n_inst == 0) return TPCCA_OK;
    if ((size_t)n > ctx->h_rowstart_cap) {
        if (ctx->h_rowstart) hipHostFree(ctx->h_rowstart);
        ctx->h_rowstart = nullptr;
        HIP_TRY(hipHostMalloc((void**)&ctx->h_rowstart, n * sizeof(int64_t), hipHostMallocDefault));
        ctx->h_rowstart_cap = n;
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_rowstart, in->row_start, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t* rs = ctx->h_rowstart;
    if (rs[0] != 0) return fail(ctx, TPCCA_E_ARG, "row_start[0] must be 0");
    for (int64_t i = 1; i < n; ++i)
        if (rs[i] < rs[i - 1]) return fail(ctx, TPCCA_E_ARG, "row_start must be non-decreasing");
    if (rs[n - 1] != in->n_clusters) return fail(ctx, TPCCA_E_ARG, "row_start[last] must equal n_clusters");
    for (int64_t i = 1; i < n; ++i)
        if (rs[i] - rs[i - 1] > TPCCA_MAX_ROW_CLUSTERS)
            return fail(ctx, TPCCA_E_CAPACITY, "a pad row of one instance holds more than TPCCA_MAX_ROW_CLUSTERS clusters");
    return TPCCA_OK;
}

Bufs make_bufs(tpcca_ctx* ctx, const tpcca_clusters* in, const tpcca_tracks* out, void* at = nullptr,
               int64_t N = -1, int64_t nseg = -1, int64_t ninst = -1, int native = 0) {
    Bufs b{};
    size_t total;
    if (at) carve(ctx, b, N, nseg, ninst, true, &total, at);
    else carve(ctx, b, ctx->arena.N, ctx->arena.nseg, ctx->arena.ninst, true, &total);
    b.K = ctx->dK;
    b.ctr = ctx->dctr;
    b.n_rows = ctx->params.n_rows;
    b.n_inst = in->n_inst;
    b.n_clusters = in->n_clusters;
    b.inst_sector = in->inst_sector;
    b.row_start = in->row_start;
    b.y = in->y;
    b.z = in->z;
    b.native = native;
    b.hits_per_bin = ctx->tuning.hits_per_bin;
    b.cap_tracks = out->cap_tracks;
    b.cap_hits = out->cap_hits;
    b.o_inst = out->inst;
    b.o_xref = out->x_ref;
    b.o_alpha = out->alpha;
    b.o_param = out->param;
    b.o_cov = out->cov;
    b.o_chi2 = out->chi2;
    b.o_ndf = out->ndf;
    b.o_hit_start = out->hit_start;
    b.o_hit_id = out->hit_id;
    b.o_chi2_total = out->chi2_total;
    b.o_z0 = out->z0;
    b.o_res = out->residuals;
    b.res_scale = std::ldexp(1.0f, -out->residual_step_log2);
    return b;
}

Launch make_launch(const tpcca_tuning& t) {
    return Launch{t.block_links, t.block_tracklet, t.block_refit, t.block_scan, t.sort_seeds, t.xcd_remap,
                  t.inward_wgs, t.inward_sort};
}

// The whole pipeline for instances [i0, i1) with clusters [c0, c1).
void enqueue_range(const Bufs& b, const Launch& L, int i0, int i1, int64_t c0, int64_t c1, int n_min, int max_row,
                   hipStream_t st, tpcca_ctx* timing) {
    auto mark = [&](int k) {
        if (timing) hipEventRecord(timing->ev[k], st);
    };
    enqueue_weights_clear(b, c0, c1, st);
    mark(0);
    enqueue_grid(b, i0, i1, max_row, st);
    mark(1);
    enqueue_links(b, L, i0, i1, max_row, st);
    mark(2);
    enqueue_clean_starts(b, L, i0, i1, c0, c1, st);
    mark(3);
    const int64_t ninst = i1 - i0;
    enqueue_tracklets(b, L, (c1 - c0) / 3 + ninst, st);
    mark(4);
    enqueue_select(b, L, (c1 - c0) / 3 + ninst, st);
    mark(5);
    enqueue_refit(b, L, (c1 - c0) / std::max(1, n_min) + ninst, st);
    mark(6);
    enqueue_write(b, L, (c1 - c0) / std::max(1, n_min) + ninst, st);
    mark(7);
}

tpcca_status finish_call(tpcca_ctx* ctx, const Bufs& b, tpcca_tracks* out, int64_t nseg) {
    const Counters& c = *ctx->hctr;
    ctx->last_ctr = c;
    ctx->last = b;
    ctx->last_nseg = nseg;
    ctx->has_last = true;
    const unsigned long long tot = c.slot[SL_TRK][0];
    out->n_tracks = (int64_t)(tot >> 32);
    out->n_hits = (int64_t)(tot & 0xFFFFFFFFull);
    if (c.err & ERR_ARG) return fail(ctx, TPCCA_E_ARG, "non-finite cluster coordinate or malformed row ranges");
    if (c.err & ERR_ROW_CAP)
        return fail(ctx, TPCCA_E_CAPACITY, "a pad row of one instance holds more than TPCCA_MAX_ROW_CLUSTERS clusters");
    if (c.err & ERR_TID_CAP)
        return fail(ctx, TPCCA_E_CAPACITY, "an instance has more than TPCCA_MAX_STARTS_PER_INST tracklets");
    if (c.err & ERR_SCRATCH) return fail(ctx, TPCCA_E_INTERNAL, "internal scratch bound exceeded");
    if ((c.err & ERR_OUT_CAP) || out->n_tracks > out->cap_tracks || out->n_hits > out->cap_hits)
        return fail(ctx, TPCCA_E_CAPACITY, "output capacity too small (n_tracks / n_hits hold the required sizes)");
    ctx->err.clear();
    return TPCCA_OK;
}

// Everything a captured launch sequence depends on: every device pointer its
// kernels take, the stream, the sizes and the tuning.
GraphKey graph_key(const tpcca_ctx* ctx, const tpcca_clusters* in, const tpcca_tracks* out, hipStream_t st,
                   const int64_t* counts, const int32_t* status, int mrow, int native = 0) {
    GraphKey key{};
    const void* ps[21] = {in->inst_sector, in->row_start, in->y,        in->z,        out->inst,
                          out->x_ref,       out->alpha,     out->param,   out->cov,     out->chi2,
                          out->ndf,         out->hit_start, out->hit_id,  out->chi2_total,
                          ctx->arena.base,  (void*)st,      (void*)ctx->dK, counts,     status, out->z0,
                          out->residuals};
    std::memcpy(key.p, ps, sizeof(ps));
    const int64_t vs[10] = {in->n_inst, in->n_clusters, out->cap_tracks, out->cap_hits, mrow,
                           ((ctx->tuning.inward_wgs * 2LL + ctx->tuning.inward_sort) * 64 + ctx->tuning.hits_per_bin) * 8 +
                               ctx->tuning.xcd_remap * 4 + ctx->tuning.sort_seeds,
                           ctx->tuning.block_links * 100000LL + ctx->tuning.block_tracklet,
                           ctx->tuning.block_refit * 100000LL + ctx->tuning.block_scan,
                           (counts != nullptr ? 1 : 0) + 2 * native, out->residual_step_log2};
    std::memcpy(key.v, vs, sizeof(vs));
    return key;
}

// Launch the context's graph, capturing `enqueue` first when the key differs
// from the captured one.
template <class F>
tpcca_status replay_graph(tpcca_ctx* ctx, const GraphKey& key, hipStream_t st, F&& enqueue) {
    if (!ctx->has_graph || !(ctx->gkey == key)) {
        if (ctx->has_graph) {
            (void)hipGraphExecDestroy(ctx->gexec);
            (void)hipGraphDestroy(ctx->graph);
            ctx->has_graph = false;
        }
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        enqueue();
        hipError_t e = hipStreamEndCapture(st, &ctx->graph);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(ctx->graph);
            return hip_fail(ctx, e, "hipGraphInstantiate");
        }
        ctx->has_graph = true;
        ctx->gkey = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->gexec, st));
    return TPCCA_OK;
}

// Kernels of the asynchronous forms: counters cleared, the CSR checked on the
// device (a malformed input turns every stage into a no-op), all stages over
// all instances with the neighbour staging sized for the largest row allowed,
// then the counts and the status.
void enqueue_async_body(const Bufs& b, const Launch& L, const tpcca_clusters* in, int64_t N, int n_min,
                        int64_t* counts, int32_t* status, hipStream_t st) {
    enqueue_reset(b, st);
    enqueue_check_csr(b, st);
    enqueue_range(b, L, 0, in->n_inst, 0, N, n_min, TPCCA_MAX_ROW_CLUSTERS, st, nullptr);
    enqueue_finish(b, st);
    enqueue_async_status(b, counts, status, st);
}

tpcca_status run(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, void* stream, bool batched,
                 int native = 0) {
    tpcca_status s = check_io(ctx, in, out);
    if (s != TPCCA_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int nr = ctx->params.n_rows;
    const int64_t N = in->n_clusters, nseg = (int64_t)in->n_inst * nr;
    s = load_rowstart(ctx, in, st);
    if (s != TPCCA_OK) return s;
    s = ensure_arena(ctx, std::max<int64_t>(N, 1), std::max<int64_t>(nseg, 1), std::max<int64_t>(in->n_inst, 1));
    if (s != TPCCA_OK) return s;
    const Bufs b = make_bufs(ctx, in, out, nullptr, -1, -1, -1, native);
    const Launch L = make_launch(ctx->tuning);
    const bool timing = (ctx->params.flags & TPCCA_FLAG_TIMING) != 0;
    if (timing && !ctx->events) {
        for (auto& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        ctx->events = true;
    }
    const int64_t* rs = ctx->h_rowstart;
    auto max_row = [&](int i0, int i1) {
        int64_t m = 0;
        for (int64_t g = (int64_t)i0 * nr; g < (int64_t)i1 * nr; ++g) m = std::max(m, rs[g + 1] - rs[g]);
        return (int)m;
    };
    if (!batched) {
        enqueue_reset(b, st);
        for (int i = 0; i < in->n_inst; ++i)
            enqueue_range(b, L, i, i + 1, rs[(int64_t)i * nr], rs[(int64_t)(i + 1) * nr], ctx->params.n_min,
                          max_row(i, i + 1), st, nullptr);
        enqueue_finish(b, st);
        HIP_TRY(hipMemcpyAsync(ctx->hctr, ctx->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
        return finish_call(ctx, b, out, nseg);
    }
    if (timing) {  // uncaptured, with stage events
        enqueue_reset(b, st);
        enqueue_range(b, L, 0, in->n_inst, 0, N, ctx->params.n_min, max_row(0, in->n_inst), st, ctx);
        enqueue_finish(b, st);
        (void)hipEventRecord(ctx->ev[8], st);
        HIP_TRY(hipMemcpyAsync(ctx->hctr, ctx->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
        for (int k = 0; k < 8; ++k) hipEventElapsedTime(&ctx->stage_ms[k], ctx->ev[k], ctx->ev[k + 1]);
        return finish_call(ctx, b, out, nseg);
    }
    if (st == nullptr) {  // the legacy null stream cannot be captured: use the context's blocking stream
        if (!ctx->own_stream) HIP_TRY(hipStreamCreate(&ctx->own_stream));
        st = ctx->own_stream;
    }
    const int mrow = max_row(0, in->n_inst);  // sizes the neighbour kernel's LDS staging
    const GraphKey key = graph_key(ctx, in, out, st, nullptr, nullptr, mrow, native);
    s = replay_graph(ctx, key, st, [&] {
        enqueue_reset(b, st);
        enqueue_range(b, L, 0, in->n_inst, 0, N, ctx->params.n_min, mrow, st, nullptr);
        enqueue_finish(b, st);
        (void)hipMemcpyAsync(ctx->hctr, ctx->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st);
    });
    if (s != TPCCA_OK) return s;
    HIP_TRY(hipStreamSynchronize(st));
    return finish_call(ctx, b, out, nseg);
}

// Device addresses of the static scratch array, one per device, resolved once
// per device with that device current.
std::mutex g_scratch_mu;
void* g_scratch_at[64] = {};

tpcca_status resolve_scratch(tpcca_ctx* ctx) {
    if (ctx->device >= 64) return TPCCA_OK;  // the allocation-free form then reports an error
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[ctx->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_at[ctx->device] = p;
    }
    ctx->noalloc = g_scratch_at[ctx->device];
    return TPCCA_OK;
}

// The asynchronous sequence on the static scratch array: kernels enqueued
// directly on the caller's stream (no graph, no allocation, no wait).
tpcca_status run_noalloc(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, int64_t* counts,
                         int32_t* status, void* stream) {
    tpcca_status s = check_io(ctx, in, out);
    if (s != TPCCA_OK) return s;
    if (!counts || !status) return fail(ctx, TPCCA_E_ARG, "null counts or status");
    if (!ctx->noalloc) return fail(ctx, TPCCA_E_DEVICE, "static scratch address not resolved for this device");
    if (in->n_inst > 0 && !in->row_start) return fail(ctx, TPCCA_E_ARG, "null row_start");
    const int64_t N = in->n_clusters;
    if (N > TPCCA_NOALLOC_MAX_CLUSTERS || in->n_inst > TPCCA_NOALLOC_MAX_INST)
        return fail(ctx, TPCCA_E_CAPACITY, "input above the allocation-free form's limits "
                                           "(TPCCA_NOALLOC_MAX_CLUSTERS, TPCCA_NOALLOC_MAX_INST)");
    const int64_t N1 = std::max<int64_t>(N, 1), nseg1 = std::max<int64_t>((int64_t)in->n_inst * ctx->params.n_rows, 1),
                  ninst1 = std::max<int64_t>(in->n_inst, 1);
    Bufs probe{};
    size_t total = 0;
    carve(ctx, probe, N1, nseg1, ninst1, false, &total);
    if (total > (size_t)TPCCA_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, TPCCA_E_CAPACITY, "input needs more than TPCCA_NOALLOC_SCRATCH_BYTES of scratch");
    HIP_TRY(hipSetDevice(ctx->device));
    const Bufs b = make_bufs(ctx, in, out, ctx->noalloc, N1, nseg1, ninst1);
    const Launch L = make_launch(ctx->tuning);
    ctx->has_last = false;  // exports need the host counts of a synchronising call
    hipStream_t st = (hipStream_t)stream;
    enqueue_async_body(b, L, in, N, ctx->params.n_min, counts, status, st);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

// The batched sequence with the input checked on the device and the counts
// and status left on the device: nothing is read back, nothing waits.
tpcca_status run_async(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, int64_t* counts,
                       int32_t* status, void* stream) {
    tpcca_status s = check_io(ctx, in, out);
    if (s != TPCCA_OK) return s;
    if (!counts || !status) return fail(ctx, TPCCA_E_ARG, "null counts or status");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t N = in->n_clusters;
    if (in->n_inst > 0 && !in->row_start) return fail(ctx, TPCCA_E_ARG, "null row_start");
    s = ensure_arena(ctx, std::max<int64_t>(N, 1), std::max<int64_t>((int64_t)in->n_inst * ctx->params.n_rows, 1),
                     std::max<int64_t>(in->n_inst, 1));
    if (s != TPCCA_OK) return s;
    const Bufs b = make_bufs(ctx, in, out);
    const Launch L = make_launch(ctx->tuning);
    ctx->has_last = false;  // exports need the host counts of a synchronising call
    if (st == nullptr) {
        if (!ctx->own_stream) HIP_TRY(hipStreamCreate(&ctx->own_stream));
        st = ctx->own_stream;
    }
    const GraphKey key = graph_key(ctx, in, out, st, counts, status, TPCCA_MAX_ROW_CLUSTERS);
    return replay_graph(ctx, key, st, [&] { enqueue_async_body(b, L, in, N, ctx->params.n_min, counts, status, st); });
}

}  // namespace

// ---------------------------------------------------------------- differentiable refit
namespace {

struct AdjLayout {
    size_t o_inst, o_row, o_yz, o_grad, o_rec, o_nops, o_status, o_ckpt, o_segn, o_carry, total;
};

AdjLayout adj_layout(int64_t cap_t, int64_t cap_h) {
    Layout L;
    AdjLayout a;
    a.o_inst = L.add(4 * cap_h);
    a.o_row = L.add(cap_h);
    a.o_yz = L.add(8 * cap_h);
    a.o_grad = L.add(3 * 16 * cap_h);
    a.o_rec = L.add(map_grad_scratch_bytes(cap_h));
    a.o_nops = L.add(4 * cap_t);
    a.o_status = L.add(256);
    a.o_ckpt = L.add(3 * 4 * kCkptWords * cap_t);
    a.o_segn = L.add(4 * cap_t);
    a.o_carry = L.add(8 * 20 * cap_t);
    a.total = L.total;
    return a;
}

tpcca_status ensure_adj_arena(tpcca_ctx* ctx, int64_t nt, int64_t nh) {
    if (ctx->adj_base && nt <= ctx->adj_cap_t && nh <= ctx->adj_cap_h) return TPCCA_OK;
    const int64_t ct = std::max(nt, ctx->adj_cap_t), ch = std::max(nh, ctx->adj_cap_h);
    const AdjLayout L = adj_layout(ct, ch);
    ctx->adj_valid = false;
    if (ctx->adj_base) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(ctx->adj_base));
        ctx->adj_base = nullptr;
        ctx->adj_cap_t = ctx->adj_cap_h = -1;
    }
    hipError_t e = hipMalloc(&ctx->adj_base, L.total);
    if (e != hipSuccess) {
        ctx->adj_base = nullptr;
        return hip_fail(ctx, e, "refit scratch allocation");
    }
    ctx->adj_bytes = L.total;
    ctx->adj_cap_t = ct;
    ctx->adj_cap_h = ch;
    return TPCCA_OK;
}

tpcca_status ensure_tape(tpcca_ctx* ctx, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (ctx->tape_base && bytes <= ctx->tape_bytes) return TPCCA_OK;
    ctx->adj_valid = false;
    if (ctx->tape_base) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(ctx->tape_base));
        ctx->tape_base = nullptr;
        ctx->tape_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->tape_base, bytes);
    if (e != hipSuccess) {
        ctx->tape_base = nullptr;
        return hip_fail(ctx, e, "refit tape allocation");
    }
    ctx->tape_bytes = bytes;
    return TPCCA_OK;
}

tpcca_status read_adj_status(tpcca_ctx* ctx, const AdjBufs& a, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(ctx->h_adj_status, a.status, sizeof(AdjStatus), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    const uint32_t err = ctx->h_adj_status->err;
    if (err & AERR_RANGE)
        return fail(ctx, TPCCA_E_ARG, "refit set: hit_start, instance, start row or row_start out of range");
    if (err & AERR_HIT) return fail(ctx, TPCCA_E_ARG, "refit set: a cluster id lies outside its track's instance");
    if (err & AERR_ROWS) return fail(ctx, TPCCA_E_ARG, "refit set: cluster rows of a track not strictly increasing");
    if (err) return fail(ctx, TPCCA_E_INTERNAL, "refit tape bound exceeded");
    return TPCCA_OK;
}

}  // namespace

extern "C" {

tpcca_status tpcca_default_params(tpcca_params* p) {
    if (!p) return TPCCA_E_ARG;
    std::memset(p, 0, sizeof(*p));
    p->n_rows = 152;
    for (int i = 0; i < p->n_rows; ++i) p->row_x[i] = (float)(85.0 + i * 162.0 / 151.0);
    p->bz = 0.5;
    p->sigma_y = p->sigma_z = 0.1;
    p->win_ty = 2.0;
    p->win_tz = 1.1;
    p->win_ny = p->win_nz = 0.5;
    p->nbr_score_max = 0.24;
    p->nsig = 3.0;
    p->chi2_pick = 16.0;
    p->chi2_rej = 25.0;
    p->sinphi_max = 0.95;
    p->cov_reset = 100.0;
    p->q_max = 20.0;
    p->u_max = 0.25;
    p->c0[0] = 1.0;
    p->c0[1] = 1.0;
    p->c0[2] = 0.25;
    p->c0[3] = 0.25;
    p->c0[4] = 400.0;
    p->n_min = 10;
    p->max_miss = 8;
    p->flags = 0;
    p->chi2_merge = 25.0;
    p->merge_max_gap = 24;
    // pad widths of the four readout regions (63, 34, 30 and 25 rows), pads
    // covering each row's full width (2 x tan(10 deg) at the plane)
    const double tan10 = std::tan(10.0 * kPi / 180.0);
    for (int i = 0; i < 256; ++i) {
        const double w = i < 63 ? 0.416 : i < 127 ? 0.42 : 0.46;
        const double x = i < p->n_rows ? (double)p->row_x[i] : 0.0;
        const double np = 2.0 * std::ceil(x * tan10 / w);
        p->pad_width[i] = (float)w;
        p->pad_center[i] = (float)((np - 1.0) * 0.5);
    }
    p->z_per_bin = 2.58 * 0.2;
    p->z_readout = 250.0;
    return TPCCA_OK;
}

tpcca_status tpcca_default_tuning(tpcca_tuning* t) {
    if (!t) return TPCCA_E_ARG;
    t->hits_per_bin = 1;
    t->block_links = 256;
    t->block_tracklet = 64;
    t->block_refit = 128;
    t->block_scan = 256;
    t->sort_seeds = 1;
    t->tape_mb = 32768;
    t->xcd_remap = 1;
    t->ckpt = 0;
    t->inward_wgs = 0;
    t->inward_sort = 1;
    return TPCCA_OK;
}

tpcca_status tpcca_create(const tpcca_params* params, const tpcca_tuning* tuning, int device, tpcca_ctx** out) {
    if (!params || !out) return TPCCA_E_ARG;
    *out = nullptr;
    tpcca_ctx* ctx = new tpcca_ctx;
    ctx->params = *params;
    if (tuning) ctx->tuning = *tuning;
    else tpcca_default_tuning(&ctx->tuning);
    tpcca_status s = check_params(ctx, ctx->params);
    if (s == TPCCA_OK) s = check_tuning(ctx, ctx->tuning);
    if (s != TPCCA_OK) {
        fprintf(stderr, "tpcca_create: %s\n", ctx->err.c_str());
        delete ctx;
        return s;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete ctx;
        return TPCCA_E_DEVICE;
    }
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return TPCCA_E_DEVICE;
    }
    build_consts(ctx->params, ctx->hK);
    if (hipMalloc((void**)&ctx->dK, sizeof(DevConsts)) != hipSuccess ||
        hipMalloc((void**)&ctx->dctr, sizeof(Counters)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->hctr, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        tpcca_destroy(ctx);
        return TPCCA_E_OOM;
    }
    if (hipMemcpy(ctx->dK, &ctx->hK, sizeof(DevConsts), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->dctr, 0, sizeof(Counters)) != hipSuccess) {
        tpcca_destroy(ctx);
        return TPCCA_E_DEVICE;
    }
    std::memset(ctx->hctr, 0, sizeof(Counters));
    if (resolve_scratch(ctx) != TPCCA_OK) {
        fprintf(stderr, "tpcca_create: %s\n", ctx->err.c_str());
        tpcca_destroy(ctx);
        return TPCCA_E_DEVICE;
    }
    *out = ctx;
    return TPCCA_OK;
}

void tpcca_destroy(tpcca_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->mg_base) (void)hipFree(ctx->mg_base);
    (void)hipDeviceSynchronize();
    if (ctx->has_graph) {
        (void)hipGraphExecDestroy(ctx->gexec);
        (void)hipGraphDestroy(ctx->graph);
    }
    if (ctx->events)
        for (auto& e : ctx->ev) hipEventDestroy(e);
    if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
    if (ctx->arena.base) hipFree(ctx->arena.base);
    if (ctx->adj_base) hipFree(ctx->adj_base);
    if (ctx->tape_base) hipFree(ctx->tape_base);
    if (ctx->h_adj_status) hipHostFree(ctx->h_adj_status);
    if (ctx->dK) hipFree(ctx->dK);
    if (ctx->dctr) hipFree(ctx->dctr);
    if (ctx->hctr) hipHostFree(ctx->hctr);
    if (ctx->h_rowstart) hipHostFree(ctx->h_rowstart);
    delete ctx;
}

const char* tpcca_last_error(const tpcca_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

tpcca_status tpcca_set_tuning(tpcca_ctx* ctx, const tpcca_tuning* t) {
    if (!ctx || !t) return TPCCA_E_ARG;
    tpcca_status s = check_tuning(ctx, *t);
    if (s != TPCCA_OK) return s;
    ctx->tuning = *t;
    return TPCCA_OK;
}

tpcca_status tpcca_get_tuning(const tpcca_ctx* ctx, tpcca_tuning* out) {
    if (!ctx || !out) return TPCCA_E_ARG;
    *out = ctx->tuning;
    return TPCCA_OK;
}

tpcca_status tpcca_track(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    return run(ctx, in, out, hip_stream, false);
}

tpcca_status tpcca_track_batched(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    return run(ctx, in, out, hip_stream, true);
}

// The native clusters seen through the local-coordinate struct: pad and time
// take the places of y and z (the kernels know them by Bufs::native).
tpcca_clusters native_view(const tpcca_native_clusters* in) {
    tpcca_clusters c{};
    c.n_inst = in->n_inst;
    c.inst_sector = in->inst_sector;
    c.row_start = in->row_start;
    c.y = in->pad;
    c.z = in->time;
    c.n_clusters = in->n_clusters;
    return c;
}

tpcca_status tpcca_track_native(tpcca_ctx* ctx, const tpcca_native_clusters* in, tpcca_tracks* out,
                                void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!in) return fail(ctx, TPCCA_E_ARG, "null clusters");
    const tpcca_clusters c = native_view(in);
    return run(ctx, &c, out, hip_stream, true, 1);
}

tpcca_status tpcca_native_to_local(tpcca_ctx* ctx, const tpcca_native_clusters* in, float* y, float* z,
                                   void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!in) return fail(ctx, TPCCA_E_ARG, "null clusters");
    if (in->n_inst < 0 || in->n_clusters < 0) return fail(ctx, TPCCA_E_ARG, "negative sizes");
    if (in->n_clusters >= (int64_t)1 << 31) return fail(ctx, TPCCA_E_ARG, "more than 2^31-1 clusters");
    if (in->n_inst > 0 && (!in->row_start || !in->inst_sector))
        return fail(ctx, TPCCA_E_ARG, "null row_start or inst_sector");
    if (in->n_clusters > 0 && (!in->pad || !in->time || !y || !z))
        return fail(ctx, TPCCA_E_ARG, "null cluster coordinates");
    if (in->n_inst == 0) return TPCCA_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    Bufs b{};
    b.K = ctx->dK;
    b.n_rows = ctx->params.n_rows;
    b.n_inst = in->n_inst;
    b.n_clusters = in->n_clusters;
    b.inst_sector = in->inst_sector;
    b.row_start = in->row_start;
    b.y = in->pad;
    b.z = in->time;
    b.native = 1;
    enqueue_native_local(b, (int64_t)in->n_inst * ctx->params.n_rows, y, z, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_track_async(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, int64_t* counts,
                               int32_t* status, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    return run_async(ctx, in, out, counts, status, hip_stream);
}

tpcca_status tpcca_track_async_noalloc(tpcca_ctx* ctx, const tpcca_clusters* in, tpcca_tracks* out, int64_t* counts,
                                       int32_t* status, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    return run_noalloc(ctx, in, out, counts, status, hip_stream);
}

tpcca_status tpcca_merge(tpcca_ctx* ctx, const int32_t* inst_event, tpcca_tracks* merged, int32_t* nseg,
                         int32_t* seg_next, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!(ctx->params.flags & TPCCA_FLAG_MERGE))
        return fail(ctx, TPCCA_E_ARG, "the context was created without TPCCA_FLAG_MERGE");
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "tpcca_merge needs a completed synchronous track call");
    if (!merged || !merged->hit_start) return fail(ctx, TPCCA_E_ARG, "null merged tracks or hit_start");
    const Bufs& lb = ctx->last;
    if (lb.n_inst > 0 && !inst_event) return fail(ctx, TPCCA_E_ARG, "null inst_event");
    const unsigned long long tot = ctx->last_ctr.slot[SL_TRK][0];
    const int64_t nt = (int64_t)(tot >> 32), nh = (int64_t)(tot & 0xFFFFFFFFull);
    if (nt > lb.cap_tracks || nh > lb.cap_hits)
        return fail(ctx, TPCCA_E_ARG, "the last track call did not fit its outputs");
    if (merged->cap_tracks > 0 && (!merged->inst || !merged->x_ref || !merged->alpha || !merged->param ||
                                   !merged->cov || !merged->chi2 || !merged->ndf))
        return fail(ctx, TPCCA_E_ARG, "null merged track arrays");
    if (merged->cap_hits > 0 && !merged->hit_id) return fail(ctx, TPCCA_E_ARG, "null merged hit_id");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t nkeys = (int64_t)lb.n_inst * lb.n_rows;
    const int64_t t1 = std::max<int64_t>(nt, 1);
    Layout L;
    const size_t o_nb = L.add(8 * std::max<int64_t>(lb.n_inst, 1)), o_rc = L.add(4 * (nkeys + 1)),
                 o_rs = L.add(4 * (nkeys + 1)), o_rf = L.add(4 * (nkeys + 1)), o_ri = L.add(4 * t1),
                 o_bo = L.add(4 * t1), o_bi = L.add(8 * t1), o_nx = L.add(4 * t1), o_pv = L.add(4 * t1),
                 o_ok = L.add(4 * t1), o_ab = L.add(t1), o_st = L.add(80 * t1), o_c2 = L.add(4 * t1),
                 o_na = L.add(4 * t1), o_rw = L.add(4 * t1), o_ns = L.add(4 * t1),
                 o_a3 = L.add(std::max<int64_t>(nh, 1)), o_ot = L.add(4 * t1), o_oh = L.add(8 * t1),
                 o_hyz = L.add(8 * std::max<int64_t>(nh, 1)), o_hd = L.add(4 * t1), o_nhd = L.add(4);
    if (L.total > ctx->mg_bytes) {
        if (ctx->mg_base) {
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipFree(ctx->mg_base));
            ctx->mg_base = nullptr;
            ctx->mg_bytes = 0;
        }
        const hipError_t e = hipMalloc(&ctx->mg_base, L.total);
        if (e != hipSuccess) {
            ctx->mg_base = nullptr;
            return hip_fail(ctx, e, "merge scratch allocation");
        }
        ctx->mg_bytes = L.total;
    }
    char* base = (char*)ctx->mg_base;
    MergeBufs m{};
    m.b = lb;
    m.inst_event = inst_event;
    m.n_t = nt;
    m.n_h = nh;
    m.nb = (int32_t*)(base + o_nb);
    m.rcnt = (int32_t*)(base + o_rc);
    m.rstart = (int32_t*)(base + o_rs);
    m.rfill = (int32_t*)(base + o_rf);
    m.rids = (int32_t*)(base + o_ri);
    m.best_out = (int32_t*)(base + o_bo);
    m.best_in = (unsigned long long*)(base + o_bi);
    m.next = (int32_t*)(base + o_nx);
    m.prev = (int32_t*)(base + o_pv);
    m.ok = (int32_t*)(base + o_ok);
    m.absorbed = (uint8_t*)(base + o_ab);
    m.state = (float*)(base + o_st);
    m.chi2 = (float*)(base + o_c2);
    m.nacc = (int32_t*)(base + o_na);
    m.row = (int32_t*)(base + o_rw);
    m.nseg = (int32_t*)(base + o_ns);
    m.acc3 = (uint8_t*)(base + o_a3);
    m.out_t = (int32_t*)(base + o_ot);
    m.out_h = (int64_t*)(base + o_oh);
    m.hyz = (float2*)(base + o_hyz);
    m.heads = (int32_t*)(base + o_hd);
    m.nheads = (unsigned int*)(base + o_nhd);
    m.cap_tracks = merged->cap_tracks;
    m.cap_hits = merged->cap_hits;
    m.o_inst = merged->inst;
    m.o_xref = merged->x_ref;
    m.o_alpha = merged->alpha;
    m.o_param = merged->param;
    m.o_cov = merged->cov;
    m.o_chi2 = merged->chi2;
    m.o_ndf = merged->ndf;
    m.o_hit_start = merged->hit_start;
    m.o_hit_id = merged->hit_id;
    m.o_nseg = nseg;
    m.seg_next = seg_next;
    enqueue_merge(m, st);
    HIP_TRY(hipMemcpyAsync(ctx->hctr, ctx->dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    const unsigned long long mt = ctx->hctr->slot[SL_MRG][0];
    merged->n_tracks = (int64_t)(mt >> 32);
    merged->n_hits = (int64_t)(mt & 0xFFFFFFFFull);
    if (merged->n_tracks > merged->cap_tracks || merged->n_hits > merged->cap_hits)
        return fail(ctx, TPCCA_E_CAPACITY, "merged output capacity too small (n_tracks / n_hits hold the sizes)");
    ctx->err.clear();
    return TPCCA_OK;
}

tpcca_status tpcca_autotune(tpcca_ctx* ctx, const tpcca_clusters* sample, int32_t repeats, tpcca_tuning* out,
                            void* hip_stream) {
    if (!ctx || !sample || !out) return TPCCA_E_ARG;
    if (repeats < 1) repeats = 1;
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t N = sample->n_clusters;
    const int64_t cap_t = N / std::max(1, ctx->params.n_min) + sample->n_inst + 1;
    // internal output buffers
    size_t bytes = 0;
    Layout L;
    size_t o_inst = L.add(4 * cap_t), o_x = L.add(4 * cap_t), o_a = L.add(4 * cap_t), o_p = L.add(20 * cap_t),
           o_c = L.add(60 * cap_t), o_chi = L.add(4 * cap_t), o_ndf = L.add(4 * cap_t),
           o_hs = L.add(8 * (cap_t + 1)), o_hid = L.add(4 * std::max<int64_t>(N, 1)), o_tot = L.add(16);
    bytes = L.total;
    char* mem = nullptr;
    HIP_TRY(hipMalloc((void**)&mem, bytes));
    tpcca_tracks tr{};
    tr.cap_tracks = cap_t;
    tr.cap_hits = std::max<int64_t>(N, 1);
    tr.inst = (int32_t*)(mem + o_inst);
    tr.x_ref = (float*)(mem + o_x);
    tr.alpha = (float*)(mem + o_a);
    tr.param = (float*)(mem + o_p);
    tr.cov = (float*)(mem + o_c);
    tr.chi2 = (float*)(mem + o_chi);
    tr.ndf = (int32_t*)(mem + o_ndf);
    tr.hit_start = (int64_t*)(mem + o_hs);
    tr.hit_id = (int32_t*)(mem + o_hid);
    tr.chi2_total = (double*)(mem + o_tot);
    const uint32_t saved_flags = ctx->params.flags;
    ctx->params.flags &= ~TPCCA_FLAG_TIMING;  // time the captured form
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    tpcca_tuning best = ctx->tuning;
    auto time_it = [&](const tpcca_tuning& t, float* ms_out) -> tpcca_status {
        tpcca_status s = tpcca_set_tuning(ctx, &t);
        if (s != TPCCA_OK) return s;
        s = run(ctx, sample, &tr, hip_stream, true);  // warm-up and capture
        if (s != TPCCA_OK) return s;
        std::vector<float> ms;
        for (int r = 0; r < repeats; ++r) {
            (void)hipEventRecord(e0, st);
            s = run(ctx, sample, &tr, hip_stream, true);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            if (s != TPCCA_OK) return s;
            float m = 0;
            (void)hipEventElapsedTime(&m, e0, e1);
            ms.push_back(m);
        }
        std::sort(ms.begin(), ms.end());
        *ms_out = ms[ms.size() / 2];
        return TPCCA_OK;
    };
    float best_ms = 0;
    tpcca_status s = time_it(best, &best_ms);
    const int hpb[] = {1, 2, 3, 4, 6, 8};
    const int blk[] = {64, 128, 256};
    const int rord[] = {0, 1, 2};  // the refit's track order over its lanes
    for (int dim = 0; dim < 5 && s == TPCCA_OK; ++dim) {
        const int* vals = dim == 0 ? hpb : dim == 4 ? rord : blk;
        const int nv = dim == 0 ? 6 : 3;
        for (int k = 0; k < nv && s == TPCCA_OK; ++k) {
            tpcca_tuning t = best;
            int* field = dim == 0   ? &t.hits_per_bin
                         : dim == 1 ? &t.block_tracklet
                         : dim == 2 ? &t.block_refit
                         : dim == 3 ? &t.block_links
                                    : &t.sort_seeds;
            if (*field == vals[k]) continue;
            *field = vals[k];
            float m = 0;
            s = time_it(t, &m);
            if (s == TPCCA_OK && m < best_ms) {
                best_ms = m;
                best = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->params.flags = saved_flags;
    tpcca_set_tuning(ctx, &best);
    *out = best;
    ctx->has_last = false;  // internal buffers are about to go away
    (void)hipStreamSynchronize(st);
    (void)hipFree(mem);
    if (ctx->has_graph) {  // graph refers to the freed buffers
        (void)hipGraphExecDestroy(ctx->gexec);
        (void)hipGraphDestroy(ctx->graph);
        ctx->has_graph = false;
    }
    return s;
}

tpcca_status tpcca_export_sizes(tpcca_ctx* ctx, int64_t* sizes, void* hip_stream) {
    (void)hip_stream;
    if (!ctx || !sizes) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result to export");
    const Counters& c = ctx->last_ctr;
    sizes[0] = ctx->last.n_clusters;
    sizes[1] = ctx->last_nseg;
    sizes[2] = (int64_t)(c.slot[SL_START][0] & 0xFFFFFFFFull);
    sizes[3] = (int64_t)(c.slot[SL_SEL][0] >> 32);
    sizes[4] = (int64_t)(c.slot[SL_SEL][0] & 0xFFFFFFFFull);
    sizes[5] = (int64_t)(c.slot[SL_TRK][0] >> 32);
    sizes[6] = (int64_t)(c.slot[SL_TRK][0] & 0xFFFFFFFFull);
    sizes[7] = ctx->params.n_rows;
    return TPCCA_OK;
}

tpcca_status tpcca_export_grid(tpcca_ctx* ctx, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz,
                               float* meta, void* hip_stream) {
    if (!ctx || !sorted_id || !bin_start || !ny || !nz || !meta) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result to export");
    enqueue_export_grid(ctx->last, sorted_id, bin_start, ny, nz, meta, ctx->last_nseg, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_export_links(tpcca_ctx* ctx, int32_t* up, int32_t* dn, int32_t* up_clean, int32_t* dn_clean,
                                void* hip_stream) {
    if (!ctx || !up || !dn || !up_clean || !dn_clean) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result to export");
    enqueue_export_links(ctx->last, up, dn, up_clean, dn_clean, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_export_tracklets(tpcca_ctx* ctx, int32_t* start_hit, int32_t* start_inst, int32_t* start_tid,
                                    int32_t* nhits, int32_t* rowhit, float* state, int32_t* state_row,
                                    uint32_t* weight, void* hip_stream) {
    if (!ctx || !weight) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result to export");
    const int64_t ns = (int64_t)(ctx->last_ctr.slot[SL_START][0] & 0xFFFFFFFFull);
    if (ns > 0 && (!start_hit || !start_inst || !start_tid || !nhits || !rowhit || !state || !state_row))
        return TPCCA_E_ARG;
    enqueue_export_tracklets(ctx->last, ns, start_hit, start_inst, start_tid, nhits, rowhit, state, state_row, weight,
                             (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_export_selected(tpcca_ctx* ctx, int32_t* sel_tl, int64_t* hit_start, int32_t* hit_id,
                                   uint8_t* mask, int32_t* status, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result to export");
    const int64_t nsel = (int64_t)(ctx->last_ctr.slot[SL_SEL][0] >> 32);
    if (nsel > 0 && (!sel_tl || !hit_start || !hit_id || !mask || !status)) return TPCCA_E_ARG;
    enqueue_export_selected(ctx->last, nsel, sel_tl, hit_start, hit_id, mask, status, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_get_stats(tpcca_ctx* ctx, tpcca_stats* o) {
    if (!ctx || !o) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "no tracking result");
    const Counters& c = ctx->last_ctr;
    std::memset(o, 0, sizeof(*o));
    o->n_clusters = ctx->last.n_clusters;
    o->n_segments = ctx->last_nseg;
    o->n_links = (int64_t)c.stats[ST_LINKS];
    o->n_starts = (int64_t)(c.slot[SL_START][0] & 0xFFFFFFFFull);
    o->n_chain_hits = (int64_t)c.stats[ST_CHAIN_HITS];
    o->tl_rows_visited = (int64_t)c.stats[ST_TL_ROWS];
    o->tl_candidates = (int64_t)c.stats[ST_TL_CAND];
    o->tl_picks = (int64_t)c.stats[ST_TL_PICKS];
    o->n_selected = (int64_t)(c.slot[SL_SEL][0] >> 32);
    o->n_selected_hits = (int64_t)(c.slot[SL_SEL][0] & 0xFFFFFFFFull);
    o->n_tracks = (int64_t)(c.slot[SL_TRK][0] >> 32);
    o->n_track_hits = (int64_t)(c.slot[SL_TRK][0] & 0xFFFFFFFFull);
    o->rf_rows_visited = (int64_t)c.stats[ST_RF_ROWS];
    o->rf_hit_visits = (int64_t)c.stats[ST_RF_HITS];
    o->nb_candidates_u = (int64_t)c.stats[ST_NB_CAND_U];
    o->nb_pairs = (int64_t)c.stats[ST_NB_PAIRS];
    return TPCCA_OK;
}

tpcca_status tpcca_get_stage_times(tpcca_ctx* ctx, float* ms8) {
    if (!ctx || !ms8) return TPCCA_E_ARG;
    for (int k = 0; k < 8; ++k) ms8[k] = ctx->stage_ms[k];
    return TPCCA_OK;
}

tpcca_status tpcca_fp32_selfcheck(const float* a, const float* b, float* out_div, float* out_sqrt, int64_t n,
                                  void* hip_stream) {
    if (n < 0 || (n > 0 && (!a || !b || !out_div || !out_sqrt))) return TPCCA_E_ARG;
    enqueue_fp32_selfcheck(a, b, out_div, out_sqrt, n, (hipStream_t)hip_stream);
    if (hipGetLastError() != hipSuccess) return TPCCA_E_DEVICE;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return TPCCA_E_DEVICE;
    return TPCCA_OK;
}

tpcca_status tpcca_sqrt_step_check(uint32_t first, uint32_t last, unsigned long long* count, void* hip_stream) {
    if (!count || first > last) return TPCCA_E_ARG;
    enqueue_sqrt_step_check(first, last, count, (hipStream_t)hip_stream);
    if (hipGetLastError() != hipSuccess) return TPCCA_E_DEVICE;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return TPCCA_E_DEVICE;
    return TPCCA_OK;
}

tpcca_status tpcca_fit_corrected(tpcca_ctx* ctx, const float* map_coef, float* param, float* cov, float* chi2,
                                 int32_t* ndf, float* x_ref, float* z0, uint8_t* masks, float* hit_yz,
                                 void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!ctx->has_last) return fail(ctx, TPCCA_E_ARG, "tpcca_fit_corrected needs a completed synchronous track call");
    const Bufs& lb = ctx->last;
    if (!lb.o_z0) return fail(ctx, TPCCA_E_ARG, "the last track call did not write z0");
    const unsigned long long tot = ctx->last_ctr.slot[SL_TRK][0];
    const int64_t nt = (int64_t)(tot >> 32), nh = (int64_t)(tot & 0xFFFFFFFFull);
    if (nt > lb.cap_tracks || nh > lb.cap_hits)
        return fail(ctx, TPCCA_E_ARG, "the last track call did not fit its outputs");
    if (nt > 0 && (!param || !cov || !chi2 || !ndf || !x_ref || !z0))
        return fail(ctx, TPCCA_E_ARG, "null output arrays");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->adj_valid = false;  // its scratch is reused
    tpcca_status s = ensure_adj_arena(ctx, std::max<int64_t>(nt, 1), std::max<int64_t>(nh, 1));
    if (s != TPCCA_OK) return s;
    const AdjLayout L = adj_layout(ctx->adj_cap_t, ctx->adj_cap_h);
    char* base = (char*)ctx->adj_base;
    CorrBufs c{};
    c.K = ctx->dK;
    c.n_rows = ctx->params.n_rows;
    c.inst_sector = lb.inst_sector;
    c.row_start = lb.row_start;
    c.yz = lb.yz;
    c.pos_of = lb.pos_of;
    c.n_tracks = nt;
    c.n_hits = nh;
    c.inst = lb.o_inst;
    c.param = lb.o_param;
    c.cov = lb.o_cov;
    c.xref = lb.o_xref;
    c.z0 = lb.o_z0;
    c.hit_start = lb.o_hit_start;
    c.hit_id = lb.o_hit_id;
    c.coef = map_coef;
    c.cyz = (float2*)(base + L.o_yz);
    c.crow = (uint8_t*)(base + L.o_row);
    c.o_param = param;
    c.o_cov = cov;
    c.o_chi2 = chi2;
    c.o_ndf = ndf;
    c.o_xref = x_ref;
    c.o_z0 = z0;
    c.o_mask = masks;
    c.o_hit_yz = hit_yz;
    enqueue_fit_corrected(c, st);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

tpcca_status tpcca_refit_fwd(tpcca_ctx* ctx, const tpcca_clusters* in, const tpcca_refit_set* set,
                             const float* map_coef, float* chi2_track, int32_t* track_ok, double* chi2_total,
                             int32_t record, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    ctx->adj_valid = false;
    if (!in || !set || !chi2_total) return fail(ctx, TPCCA_E_ARG, "null clusters, refit set or chi2_total");
    const int64_t nt = set->n_tracks, nh = set->n_hits;
    if (nt < 0 || nh < 0 || nt >= ((int64_t)1 << 31) || nh >= ((int64_t)1 << 31))
        return fail(ctx, TPCCA_E_ARG, "refit set sizes must be in [0, 2^31)");
    if (in->n_inst < 0 || in->n_clusters < 0) return fail(ctx, TPCCA_E_ARG, "negative cluster sizes");
    if (nt > 0 && (!set->params0 || !set->cov0 || !set->row0 || !set->inst || !set->hit_start || !chi2_track))
        return fail(ctx, TPCCA_E_ARG, "null refit-set array or chi2_track");
    if (nt > 0 && (in->n_inst == 0 || !in->row_start || !in->inst_sector))
        return fail(ctx, TPCCA_E_ARG, "tracks given without cluster instances");
    if (nh > 0 && (!set->hit_id || !set->hit_mask || !in->y || !in->z))
        return fail(ctx, TPCCA_E_ARG, "null hit_id, hit_mask or cluster coordinates");
    if (nt == 0 && nh != 0) return fail(ctx, TPCCA_E_ARG, "clusters given without tracks");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->h_adj_status)
        HIP_TRY(hipHostMalloc((void**)&ctx->h_adj_status, sizeof(AdjStatus), hipHostMallocDefault));
    tpcca_status s = ensure_adj_arena(ctx, std::max<int64_t>(nt, 1), std::max<int64_t>(nh, 1));
    if (s != TPCCA_OK) return s;
    const AdjLayout L = adj_layout(ctx->adj_cap_t, ctx->adj_cap_h);
    char* base = (char*)ctx->adj_base;
    AdjBufs a{};
    a.K = ctx->dK;
    a.n_rows = ctx->params.n_rows;
    a.n_inst = in->n_inst;
    a.n_clusters = in->n_clusters;
    a.inst_sector = in->inst_sector;
    a.row_start = in->row_start;
    a.y = in->y;
    a.z = in->z;
    a.n_tracks = nt;
    a.n_hits = nh;
    a.params0 = set->params0;
    a.cov0 = set->cov0;
    a.row0 = set->row0;
    a.inst = set->inst;
    a.hit_start = set->hit_start;
    a.hit_id = set->hit_id;
    a.hit_mask = set->hit_mask;
    a.coef = map_coef;
    a.hit_inst = (int32_t*)(base + L.o_inst);
    a.hit_row = (uint8_t*)(base + L.o_row);
    a.hit_yz = (float2*)(base + L.o_yz);
    a.hit_grad = (double2*)(base + L.o_grad);
    a.nops = (int32_t*)(base + L.o_nops);
    a.status = (AdjStatus*)(base + L.o_status);
    a.chi2_track = chi2_track;
    a.track_ok = track_ok;
    a.chi2_total = chi2_total;
    a.adj_f64 = (ctx->params.flags & TPCCA_FLAG_ADJOINT_F64) ? 1 : 0;
    const bool ckpt = ctx->tuning.ckpt != 0;
    a.seg_nops = (int32_t*)(base + L.o_segn);
    a.carry = (double*)(base + L.o_carry);
    if (ckpt && record) a.ckpt = (float*)(base + L.o_ckpt);
    // validation, corrected clusters, operation counts; the host sizes the tape
    enqueue_refit_prepare(a, st);
    s = read_adj_status(ctx, a, st);
    if (s != TPCCA_OK) return s;
    // the tape holds a whole refit per track, or with checkpoints one pass segment
    a.tape_ops = ckpt ? ctx->h_adj_status->max_seg_ops : ctx->h_adj_status->max_ops;
    const int64_t per_track = std::max<int64_t>(1, (int64_t)a.tape_ops * kTapeBytesPerOp);
    const int64_t budget = (int64_t)ctx->tuning.tape_mb << 20;
    const int64_t batch = std::min<int64_t>(std::max<int64_t>(1, budget / per_track), std::max<int64_t>(nt, 1));
    const bool taped = record && !ckpt && batch >= nt;
    if (taped) {
        s = ensure_tape(ctx, (size_t)(per_track * std::max<int64_t>(nt, 1)));
        if (s != TPCCA_OK) return s;
        a.tape = (uint32_t*)ctx->tape_base;
    }
    enqueue_refit_forward(a, 0, nt, true, st);
    enqueue_refit_total(a, st);
    s = read_adj_status(ctx, a, st);
    if (s != TPCCA_OK) return s;
    ctx->adj = a;
    ctx->adj_valid = record != 0;
    ctx->adj_taped = taped;
    ctx->adj_batch = batch;
    ctx->err.clear();
    return TPCCA_OK;
}

tpcca_status tpcca_refit_bwd(tpcca_ctx* ctx, const float* grad_chi2, double* grad_params0, double* grad_map,
                             double* grad_hit_yz, void* hip_stream) {
    if (!ctx) return TPCCA_E_ARG;
    if (!ctx->adj_valid) return fail(ctx, TPCCA_E_ARG, "no recorded tpcca_refit_fwd to differentiate");
    AdjBufs a = ctx->adj;
    if (a.n_tracks > 0 && (!grad_chi2 || !grad_params0))
        return fail(ctx, TPCCA_E_ARG, "null grad_chi2 or grad_params0");
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipSetDevice(ctx->device));
    a.grad_chi2 = grad_chi2;
    a.grad_params = grad_params0;
    a.grad_map = grad_map;
    if (ctx->adj_taped) {
        enqueue_refit_reverse(a, 0, a.n_tracks, -1, st);
    } else {
        // record and reverse batch by batch: the whole refit when the set's
        // tape exceeds the budget, or one pass segment at a time, last pass
        // first, recomputed from its checkpoint
        const int64_t per_track = std::max<int64_t>(1, (int64_t)a.tape_ops * kTapeBytesPerOp);
        tpcca_status s = ensure_tape(ctx, (size_t)(per_track * ctx->adj_batch));
        if (s != TPCCA_OK) return s;
        a.tape = (uint32_t*)ctx->tape_base;
        for (int64_t t0 = 0; t0 < a.n_tracks; t0 += ctx->adj_batch) {
            const int64_t t1 = std::min(a.n_tracks, t0 + ctx->adj_batch);
            if (a.ckpt) {
                for (int seg = 2; seg >= 0; --seg) {
                    enqueue_refit_segment(a, t0, t1, seg, st);
                    enqueue_refit_reverse(a, t0, t1, seg, st);
                }
            } else {
                enqueue_refit_forward(a, t0, t1, false, st);
                enqueue_refit_reverse(a, t0, t1, -1, st);
            }
        }
    }
    if (grad_map) {
        const AdjLayout L = adj_layout(ctx->adj_cap_t, ctx->adj_cap_h);
        enqueue_refit_map_grad(a, (char*)ctx->adj_base + L.o_rec, st);
    }
    if (grad_hit_yz) enqueue_refit_hit_grad(a, grad_hit_yz, st);
    HIP_TRY(hipGetLastError());
    return TPCCA_OK;
}

}  // extern "C"
