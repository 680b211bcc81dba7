// Cross-sector merge (gfx950) of the sector tracks of the last track call:
// the second phase of Section 2 of arXiv:1811.11481 (segments found in the
// individual sectors are merged, then fitted as one track), with the refit
// following the helix through rotations between sector frames (Section 4).
//
// Segment A continues as segment B (same event, phi-neighbouring sector of the
// same side) when A's state after the outward pass of its refit, rotated into
// B's frame and carried row by row from the first row plane outward of the
// rotated point to B's reference row (at most merge_max_gap rows), agrees with
// B's fitted state: chi2 of the five parameter differences with the summed
// covariance <= chi2_merge (pairs whose z or tan(lambda) difference alone
// exceeds the cut are rejected before the solve). Mutual best pairs (smallest
// chi2, ties to the smaller track index) form chains of at most kMaxChain
// segments (a closed loop is opened at its smallest track index); each chain
// is refitted over all its clusters with the sector refit's three passes,
// rotating between frames. Output in sector-track order: a merged track at its
// first segment, the other segments omitted; a chain whose refit fails keeps
// its segments as sector tracks. Every decision and value is binary32 in the
// oracle's operation order (bit-exact parity).
//
// Work mapping: one lane per sector track for the pair search (its candidate
// partners bucketed by (instance, reference row), so the lane carries its
// rotated state outward one row at a time and tests only the tracks that start
// on that row; the partner's best is an order-free 64-bit atomicMin of (chi2
// bits, index)), one lane per chain for the merged refit, a deterministic scan
// for the output positions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "kf_device.h"

#pragma clang fp contract(off)

namespace tpcca {

namespace {

constexpr int kMaxChain = 8;

__device__ __forceinline__ int sector_step(int sa, int sb) {
    if (sa / 18 != sb / 18) return 0;
    const int a = sa % 18, b = sb % 18;
    if (b == (a + 1) % 18) return 1;
    if (a == (b + 1) % 18) return -1;
    return 0;
}

// Rotation of the state into the frame turned by d (cos ca, sin sa): the point
// (x, y) to (x ca + y sa, -x sa + y ca), phi to phi - d, taken at the point's
// new x; covariance J C J^T with dy'/dy = cos phi / cos phi',
// dz'/dy = -sa tan(lambda) / cos phi', d sin phi'/dy = -c sa (curvature c),
// d sin phi'/d sin phi = cos phi' / cos phi. Fails unless the track still
// moves outward with |sin phi'| below the guard.
__device__ __forceinline__ bool kf_rotate(KState& s, float& x, float ca, float sa, const KfConsts& K) {
    const float sf = s.p[2];
    const float cf = __builtin_sqrtf(__builtin_fmaf(-sf, sf, 1.0f));
    const float sn = __builtin_fmaf(sf, ca, -(cf * sa));
    const float cn = __builtin_fmaf(cf, ca, sf * sa);
    if (!(cn > 0.0f) || !(__builtin_fabsf(sn) < K.sinphi_max)) return false;
    const float xn = __builtin_fmaf(x, ca, s.p[0] * sa);
    const float yn = __builtin_fmaf(-x, sa, s.p[0] * ca);
    const float icn = 1.0f / cn;
    const float j00 = cf * icn;
    const float j10 = -((sa * s.p[3]) * icn);
    const float j20 = -((K.kB * s.p[4]) * sa);
    const float j22 = cn / cf;
    float B[5][5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float c0 = s.C[pk(0, j)], c1 = s.C[pk(1, j)], c2 = s.C[pk(2, j)];
        B[0][j] = j00 * c0;
        B[1][j] = __builtin_fmaf(j10, c0, c1);
        B[2][j] = __builtin_fmaf(j20, c0, j22 * c2);
        B[3][j] = s.C[pk(3, j)];
        B[4][j] = s.C[pk(4, j)];
    }
    float Cn[15];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Cn[pk(i, 0)] = B[i][0] * j00;
        if (i >= 1) Cn[pk(i, 1)] = __builtin_fmaf(B[i][0], j10, B[i][1]);
        if (i >= 2) Cn[pk(i, 2)] = __builtin_fmaf(B[i][0], j20, B[i][2] * j22);
        if (i >= 3) Cn[pk(i, 3)] = B[i][3];
        if (i >= 4) Cn[pk(i, 4)] = B[i][4];
    }
#pragma unroll
    for (int q = 0; q < 15; ++q) s.C[q] = Cn[q];
    x = xn;
    s.p[0] = yn;
    s.p[2] = sn;
    return true;
}

// chi2 of d = b - a with covariance Ca + Cb by LDL^T in a fixed order; the z
// and tan(lambda) marginals are tested against the cut first.
__device__ __forceinline__ bool pair_chi2(const KState& a, const float* bp, const float* bc, float cut, float& chi2) {
    float C[5][5], L[5][5], D[5], d[5], zz[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        d[i] = bp[i] - a.p[i];
#pragma unroll
        for (int j = 0; j <= i; ++j) C[i][j] = a.C[pk(i, j)] + bc[pk(i, j)];
    }
    if (!(d[1] * d[1] <= cut * C[1][1]) || !(d[3] * d[3] <= cut * C[3][3])) return false;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        float v = C[j][j];
#pragma unroll
        for (int q = 0; q < j; ++q) v = v - (L[j][q] * L[j][q]) * D[q];
        if (!(v > 0.0f)) return false;
        D[j] = v;
#pragma unroll
        for (int i = j + 1; i < 5; ++i) {
            float w = C[i][j];
#pragma unroll
            for (int q = 0; q < j; ++q) w = w - (L[i][q] * L[j][q]) * D[q];
            L[i][j] = w / v;
        }
    }
    float c = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        float v = d[i];
#pragma unroll
        for (int q = 0; q < i; ++q) v = v - L[i][q] * zz[q];
        zz[i] = v;
        c = c + (v * v) / D[i];
    }
    chi2 = c;
    return true;
}

__device__ __forceinline__ int plane_towards(const float* sX, int nr, float x, int dir) {
    if (dir > 0) {
        for (int r = 0; r < nr; ++r)
            if (sX[r] >= x) return r;
    } else {
        for (int r = nr - 1; r >= 0; --r)
            if (sX[r] <= x) return r;
    }
    return -1;
}

__device__ __forceinline__ void load_state(KState& s, const float* p20) {
#pragma unroll
    for (int q = 0; q < 5; ++q) s.p[q] = p20[q];
#pragma unroll
    for (int q = 0; q < 15; ++q) s.C[q] = p20[5 + q];
}

__global__ void k_mrg_clear(int32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// -------------------------------------------------------------- neighbours
// For every instance, the lowest instance of the same event in the
// phi-neighbouring sector of the same side, one per direction; an instance
// that is not the lowest of its (event, sector) takes no part in the merge.
constexpr int kNbLds = 4096;  // instances whose (event, sector) a workgroup stages in LDS

__global__ __launch_bounds__(256) void k_mrg_neighbours(MergeBufs m) {
    const Bufs& b = m.b;
    __shared__ int2 es[kNbLds];  // (event, sector) per instance
    const int n = b.n_inst;
    const bool lds = n <= kNbLds;
    if (lds)
        for (int j = threadIdx.x; j < n; j += blockDim.x) es[j] = make_int2(m.inst_event[j], b.inst_sector[j]);
    __syncthreads();
    auto at = [&](int j) { return lds ? es[j] : make_int2(m.inst_event[j], b.inst_sector[j]); };
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int2 me = at(i);
        const int sec = me.y, side = sec / 18, phi = sec % 18;
        int canon = 1;
        for (int j = 0; j < i && canon; ++j) {
            const int2 o = at(j);
            if (o.x == me.x && o.y == sec) canon = 0;
        }
        for (int k = 0; k < 2; ++k) {
            const int want = side * 18 + (phi + (k ? 1 : -1) + 18) % 18;
            int best = -1;
            for (int j = 0; j < n && canon; ++j) {
                const int2 o = at(j);
                if (j != i && o.x == me.x && o.y == want) {
                    best = j;
                    break;
                }
            }
            m.nb[2 * i + k] = canon ? best : -1;
        }
    }
}

// tracks bucketed by (instance, reference row): counts, scan, fill
__global__ void k_mrg_count(MergeBufs m) {
    const Bufs& b = m.b;
    const int nr = b.n_rows;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m.n_t; t += (int64_t)gridDim.x * blockDim.x) {
        const int key = b.o_inst[t] * nr + b.rf_row[b.trk_si[t]];
        atomicAdd(&m.rcnt[key], 1);
        m.best_out[t] = -1;
        m.best_in[t] = ~0ull;
        m.next[t] = -1;
        m.prev[t] = -1;
        m.ok[t] = 0;
        m.absorbed[t] = 0;
    }
}

// exclusive scan of the bucket counts, one workgroup of 1024 threads, each a
// contiguous run of buckets
__global__ __launch_bounds__(1024) void k_mrg_rscan(MergeBufs m, int nkeys) {
    __shared__ int sh[1024];
    const int per = (nkeys + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(lo + per, nkeys);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += m.rcnt[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < 1024; ++w) {
            const int v = sh[w];
            sh[w] = run;
            run += v;
        }
    }
    __syncthreads();
    int run = sh[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        m.rstart[i] = run;
        m.rfill[i] = run;
        run += m.rcnt[i];
    }
    if (hi == nkeys && lo < hi) m.rstart[nkeys] = run;
    if (nkeys == 0 && threadIdx.x == 0) m.rstart[0] = 0;
}

__global__ void k_mrg_fill(MergeBufs m) {
    const Bufs& b = m.b;
    const int nr = b.n_rows;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m.n_t; t += (int64_t)gridDim.x * blockDim.x) {
        const int key = b.o_inst[t] * nr + b.rf_row[b.trk_si[t]];
        m.rids[atomicAdd(&m.rfill[key], 1)] = (int32_t)t;
    }
}

// -------------------------------------------------------------- pair search
// One lane per track A: for each neighbouring sector, rotate A's outward state
// into that frame, carry it outward row by row and test the tracks whose
// reference row is the current row.
__global__ __launch_bounds__(256) void k_mrg_match(MergeBufs m) {
    const Bufs& b = m.b;
    const DevConsts& K = *b.K;
    const KfConsts kc = kf_consts(K);
    __shared__ float sX[kMaxRows];
    kf_load_rows(sX, K);
    const int nr = K.n_rows;
    const float cut = K.chi2_merge;
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < m.n_t; a += (int64_t)gridDim.x * blockDim.x) {
        const int32_t si = b.trk_si[a];
        const int inst = b.o_inst[a];
        int32_t best = -1;
        float bchi = 0.0f;
        for (int k = 0; k < 2; ++k) {
            const int j = m.nb[2 * inst + k];
            if (j < 0) continue;
            KState s;
            load_state(s, b.rf_state2 + (int64_t)si * 20);
            float x = sX[b.rf_row2[si]];
            if (!kf_rotate(s, x, K.rot_c, k ? K.rot_s : -K.rot_s, kc)) continue;
            const int r1 = plane_towards(sX, nr, x, +1);
            if (r1 < 0) continue;
            if (!kf_propagate(s, x, sX[r1], kc)) continue;
            const int rmax = min(r1 + K.merge_max_gap, nr - 1);
            for (int r = r1; r <= rmax; ++r) {
                if (r > r1 && !kf_propagate(s, sX[r - 1], sX[r], kc)) break;
                const int key = j * nr + r;
                for (int q = m.rstart[key]; q < m.rstart[key + 1]; ++q) {
                    const int32_t bt = m.rids[q];
                    float c;
                    if (!pair_chi2(s, b.o_param + (int64_t)bt * 5, b.o_cov + (int64_t)bt * 15, cut, c) || !(c <= cut))
                        continue;
                    if (best < 0 || c < bchi || (c == bchi && bt < best)) {
                        best = bt;
                        bchi = c;
                    }
                    atomicMin(&m.best_in[bt], ((unsigned long long)__float_as_uint(c) << 32) | (unsigned long long)a);
                }
            }
        }
        m.best_out[a] = best;
    }
}

__global__ void k_mrg_link(MergeBufs m) {
    for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < m.n_t; a += (int64_t)gridDim.x * blockDim.x) {
        const int32_t bt = m.best_out[a];
        if (bt >= 0 && (int64_t)(m.best_in[bt] & 0xFFFFFFFFull) == a) {
            m.next[a] = bt;
            m.prev[bt] = (int32_t)a;
        }
    }
}

// a closed loop of links is opened at its smallest track index (every member
// finds the same index; the writes are identical)
__global__ void k_mrg_cycles(MergeBufs m) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m.n_t; t += (int64_t)gridDim.x * blockDim.x) {
        if (m.prev[t] < 0) continue;
        int64_t u = m.prev[t], mn = t;
        int steps = 0;
        while (u >= 0 && u != t && steps++ < 64) {
            mn = min(mn, u);
            u = m.prev[u];
        }
        if (u == t) {
            const int32_t p = m.prev[mn];
            if (p >= 0) m.next[p] = -1;
            m.prev[mn] = -1;
        }
    }
}

// -------------------------------------------------------------- merged refit
// Coordinates of every output cluster of the last track call, gathered once in
// cluster order (as the grid holds them: native input transformed), so that a
// chain's refit reads one array at a computed index.
__global__ void k_mrg_gather(MergeBufs m, int64_t nh) {
    const Bufs& b = m.b;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nh; q += (int64_t)gridDim.x * blockDim.x)
        m.hyz[q] = b.yz[b.pos_of[b.o_hit_id[q]]];
}

// The chain heads (a segment with a partner and none before it), in any order:
// each chain's refit depends on its own segments only.
__global__ void k_mrg_heads(MergeBufs m) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m.n_t; t += (int64_t)gridDim.x * blockDim.x)
        if (m.prev[t] < 0 && m.next[t] >= 0) m.heads[atomicAdd(m.nheads, 1u)] = (int32_t)t;
}

// Position in a chain's cluster stream: the segment, its index in the chain
// (its frame), the output cluster and the segment's cluster range.
struct ChainCursor {
    int32_t seg;
    int f;
    int64_t q, lo, hi;
};

__device__ __forceinline__ void cursor_at(const MergeBufs& m, ChainCursor& c, int32_t seg, int f, bool last) {
    c.seg = seg;
    c.f = f;
    c.lo = m.b.o_hit_start[seg];
    c.hi = m.b.o_hit_start[seg + 1];
    c.q = last ? c.hi - 1 : c.lo;
}

// the next cluster inward (towards the chain's first segment) or outward
__device__ __forceinline__ void cursor_step(const MergeBufs& m, ChainCursor& c, bool inward) {
    if (inward) {
        if (c.q > c.lo) --c.q;
        else cursor_at(m, c, m.prev[c.seg], c.f - 1, true);
    } else {
        if (c.q + 1 < c.hi) ++c.q;
        else cursor_at(m, c, m.next[c.seg], c.f + 1, false);
    }
}

// One lane per chain: the three passes of the sector refit over all clusters
// of the chain, rotating between frames; the next cluster's row and
// coordinates are loaded one step ahead.
__global__ __launch_bounds__(128) void k_mrg_refit(MergeBufs m) {
    const Bufs& b = m.b;
    const DevConsts& K = *b.K;
    const KfConsts kc = kf_consts(K);
    __shared__ float sX[kMaxRows];
    __shared__ int skey[128], sorder[128];
    kf_load_rows(sX, K);
    const int nr = K.n_rows;
    const int64_t nheads = (int64_t)*m.nheads;
    const int nt = blockDim.x;
    for (int64_t c0 = blockIdx.x * (int64_t)nt; c0 < nheads; c0 += (int64_t)gridDim.x * nt) {  // uniform
        int key = -1;  // the chain's clusters: three passes over them
        if (c0 + threadIdx.x < nheads) {
            const int32_t h = m.heads[c0 + threadIdx.x];
            int nk = (int)(b.o_hit_start[h + 1] - b.o_hit_start[h]), sk = 1;
            for (int32_t u = m.next[h]; u >= 0 && sk < kMaxChain; u = m.next[u], ++sk)
                nk += (int)(b.o_hit_start[u + 1] - b.o_hit_start[u]);
            key = nk;
        }
        const int64_t k = chunk_item_by_work(skey, sorder, c0, key);
        if (k >= nheads) continue;
        const int32_t t = m.heads[k];
        // the chain: at most kMaxChain segments from t along next
        int nseg = 1, n = (int)(b.o_hit_start[t + 1] - b.o_hit_start[t]);
        int32_t tail = t;
        for (int32_t u = m.next[t]; u >= 0 && nseg < kMaxChain; u = m.next[u]) {
            tail = u;
            n += (int)(b.o_hit_start[u + 1] - b.o_hit_start[u]);
            ++nseg;
        }
        {
            int32_t u = t;
            for (int f = 0; f < nseg; ++f, u = m.next[u])
                for (int64_t q = b.o_hit_start[u]; q < b.o_hit_start[u + 1]; ++q) m.acc3[q] = 0;
        }
        const int32_t tail_si = b.trk_si[tail];
        KState s;
        load_state(s, b.rf_state2 + (int64_t)tail_si * 20);
        int cur = b.rf_row2[tail_si];
        int frame = nseg - 1;
        int32_t frame_seg = tail;  // the segment whose frame the state is in
        float ref_y = s.p[0], ref_z = s.p[1];
        s.p[0] = 0.0f;
        s.p[1] = 0.0f;
        auto move_to = [&](int target, int tframe, int32_t tseg) -> bool {
            if (tframe != frame) {
                s.p[0] = ref_y + s.p[0];
                s.p[1] = ref_z + s.p[1];
                float x = sX[cur];
                const int sa = b.inst_sector[b.o_inst[frame_seg]], sb = b.inst_sector[b.o_inst[tseg]];
                const int dir = tframe > frame ? sector_step(sa, sb) : -sector_step(sb, sa);
                if (!kf_rotate(s, x, K.rot_c, dir > 0 ? K.rot_s : -K.rot_s, kc)) return false;
                frame = tframe;
                frame_seg = tseg;
                ref_y = s.p[0];
                ref_z = s.p[1];
                s.p[0] = 0.0f;
                s.p[1] = 0.0f;
                const int r1 = plane_towards(sX, nr, x, sX[target] >= x ? +1 : -1);
                if (r1 < 0 || !kf_propagate(s, x, sX[r1], kc)) return false;
                cur = r1;
            }
            while (cur != target) {
                const int nx = cur < target ? cur + 1 : cur - 1;
                if (!kf_propagate(s, sX[cur], sX[nx], kc)) return false;
                cur = nx;
            }
            return true;
        };
        bool ok = n > 0;
        if (ok) {  // to the chain's last cluster, in the tail's frame
            const int64_t q = b.o_hit_start[tail + 1] - 1;
            ok = move_to(b.trk_hrow[q], nseg - 1, tail);
        }
        float chi2sum = 0.0f;
        int nacc = 0;
        for (int pass = 0; pass < 3 && ok; ++pass) {
            kf_reset(s, kc);
            const bool inward = pass != 1;
            ChainCursor cu;
            if (inward) cursor_at(m, cu, tail, nseg - 1, true);
            else cursor_at(m, cu, t, 0, false);
            int row_n = b.trk_hrow[cu.q];
            float2 c_n = m.hyz[cu.q];
            for (int qq = 0; qq < n; ++qq) {
                const ChainCursor cc = cu;
                const int row = row_n;
                const float2 c = c_n;
                if (qq + 1 < n) {
                    cursor_step(m, cu, inward);
                    row_n = b.trk_hrow[cu.q];
                    c_n = m.hyz[cu.q];
                }
                if (!move_to(row, cc.f, cc.seg)) {
                    ok = false;
                    break;
                }
                const float y = c.x, z = c.y;
                const Innov inn = kf_innovation(s, y - ref_y, z - ref_z, kc);
                if (inn.chi2 <= kc.chi2_rej) {
                    kf_update(s, inn);
                    s.p[0] = s.p[0] + (ref_y - y);
                    s.p[1] = s.p[1] + (ref_z - z);
                    ref_y = y;
                    ref_z = z;
                    if (pass == 2) {
                        chi2sum = chi2sum + inn.chi2;
                        ++nacc;
                        m.acc3[cc.q] = 1;
                    }
                }
            }
        }
        ok = ok && frame == 0 && nacc >= kc.n_min;
        if (!ok) continue;
        float* o = m.state + (int64_t)t * 20;
        o[0] = ref_y + s.p[0];
        o[1] = ref_z + s.p[1];
#pragma unroll
        for (int q = 2; q < 5; ++q) o[q] = s.p[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) o[5 + q] = s.C[q];
        m.chi2[t] = chi2sum;
        m.nacc[t] = nacc;
        m.row[t] = cur;
        m.nseg[t] = nseg;
        m.ok[t] = 1;
        {
            int32_t u = m.next[t];
            for (int f = 1; f < nseg; ++f, u = m.next[u]) m.absorbed[u] = 1;
        }
    }
}

// -------------------------------------------------------------- output
// Output position of every sector track (deterministic scan over packed
// (tracks, clusters)); the three-phase scan of the tracker's compactions.
struct MergeOp {
    MergeBufs m;
    __device__ int64_t begin() const { return 0; }
    __device__ int64_t end() const { return m.n_t; }
    __device__ unsigned long long value(int64_t t) const {
        if (m.absorbed[t]) return 0ull;
        const int nh = m.ok[t] ? m.nacc[t] : (int)(m.b.o_hit_start[t + 1] - m.b.o_hit_start[t]);
        return (1ull << 32) | (unsigned long long)nh;
    }
    __device__ void write(int64_t t, unsigned long long prefix, unsigned long long) const {
        m.out_t[t] = (int32_t)(prefix >> 32);
        m.out_h[t] = (int64_t)(prefix & 0xFFFFFFFFull);
    }
};

__device__ __forceinline__ unsigned long long mrg_block_scan(unsigned long long v, unsigned long long* sh,
                                                             unsigned long long* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned long long incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int w = 0; w < nw; ++w) {
            const unsigned long long t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[16] = run;
    }
    __syncthreads();
    const unsigned long long r = sh[wid] + incl - v;
    *total = sh[16];
    __syncthreads();
    return r;
}

constexpr int kMrgScanBlocks = 256;

__global__ __launch_bounds__(256) void k_mrg_scan_part(MergeOp op, unsigned long long* part) {
    __shared__ unsigned long long sh[17];
    const int64_t n = op.end();
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, n);
    unsigned long long s = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += op.value(i);
    unsigned long long tot;
    mrg_block_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_mrg_scan_top(unsigned long long* part, Counters* ctr) {
    __shared__ unsigned long long sh[17];
    unsigned long long tot;
    const unsigned long long ex = mrg_block_scan(part[threadIdx.x], sh, &tot);
    part[threadIdx.x] = ex;
    if (threadIdx.x == 0) ctr->slot[SL_MRG][0] = tot;
}

__global__ __launch_bounds__(256) void k_mrg_scan_apply(MergeOp op, const unsigned long long* part) {
    __shared__ unsigned long long sh[17];
    const int64_t n = op.end();
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, n);
    unsigned long long run = part[blockIdx.x];
    for (int64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
        const int64_t i = t0 + threadIdx.x;
        const unsigned long long v = (i < hi) ? op.value(i) : 0ull;
        unsigned long long tot;
        const unsigned long long ex = mrg_block_scan(v, sh, &tot);
        if (i < hi && v) op.write(i, run + ex, v);
        run += tot;
    }
}

// merged outputs (one lane per sector track with an output)
__global__ void k_mrg_write(MergeBufs m) {
    const Bufs& b = m.b;
    const DevConsts& K = *b.K;
    const unsigned long long tot = m.b.ctr->slot[SL_MRG][0];
    const int64_t ntot = (int64_t)(tot >> 32), htot = (int64_t)(tot & 0xFFFFFFFFull);
    const bool fits = ntot <= m.cap_tracks && htot <= m.cap_hits;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m.n_t; t += (int64_t)gridDim.x * blockDim.x) {
        if (m.seg_next) m.seg_next[t] = m.next[t];
        if (m.absorbed[t] || !fits) continue;
        const int64_t o = m.out_t[t], h = m.out_h[t];
        m.o_inst[o] = b.o_inst[t];
        m.o_alpha[o] = b.o_alpha[t];
        m.o_hit_start[o] = h;
        if (m.ok[t]) {
            m.o_xref[o] = K.X[m.row[t]];
            for (int q = 0; q < 5; ++q) m.o_param[o * 5 + q] = m.state[t * 20 + q];
            for (int q = 0; q < 15; ++q) m.o_cov[o * 15 + q] = m.state[t * 20 + 5 + q];
            m.o_chi2[o] = m.chi2[t];
            m.o_ndf[o] = 2 * m.nacc[t] - 5;
            m.o_nseg[o] = m.nseg[t];
            int64_t w = h;
            int n = 0;
            for (int64_t u = t; u >= 0 && n < kMaxChain; u = m.next[u], ++n)
                for (int64_t q = b.o_hit_start[u]; q < b.o_hit_start[u + 1]; ++q)
                    if (m.acc3[q]) m.o_hit_id[w++] = b.o_hit_id[q];
        } else {
            m.o_xref[o] = b.o_xref[t];
            for (int q = 0; q < 5; ++q) m.o_param[o * 5 + q] = b.o_param[t * 5 + q];
            for (int q = 0; q < 15; ++q) m.o_cov[o * 15 + q] = b.o_cov[t * 15 + q];
            m.o_chi2[o] = b.o_chi2[t];
            m.o_ndf[o] = b.o_ndf[t];
            m.o_nseg[o] = 1;
            int64_t w = h;
            for (int64_t q = b.o_hit_start[t]; q < b.o_hit_start[t + 1]; ++q) m.o_hit_id[w++] = b.o_hit_id[q];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && fits) m.o_hit_start[ntot] = htot;
}

inline int grid_of(int64_t n, int block, int cap) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

void enqueue_merge(const MergeBufs& m, hipStream_t st) {
    const int nkeys = m.b.n_inst * m.b.n_rows;
    hipLaunchKernelGGL(k_mrg_neighbours, dim3(grid_of(m.b.n_inst, 256, 1024)), dim3(256), 0, st, m);
    // bucket counts cleared by a kernel (graph-capture safe)
    hipLaunchKernelGGL(k_mrg_clear, dim3(grid_of(nkeys + 1, 256, 1024)), dim3(256), 0, st, m.rcnt, (int64_t)nkeys + 1);
    if (m.n_t > 0) {
        const unsigned g = grid_of(m.n_t, 256, 4096);
        hipLaunchKernelGGL(k_mrg_count, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_rscan, dim3(1), dim3(1024), 0, st, m, nkeys);
        hipLaunchKernelGGL(k_mrg_fill, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_match, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_link, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_cycles, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_gather, dim3(grid_of(m.n_h, 256, 16384)), dim3(256), 0, st, m, m.n_h);
        hipLaunchKernelGGL(k_mrg_clear, dim3(1), dim3(64), 0, st, (int32_t*)m.nheads, (int64_t)1);
        hipLaunchKernelGGL(k_mrg_heads, dim3(g), dim3(256), 0, st, m);
        hipLaunchKernelGGL(k_mrg_refit, dim3(grid_of(m.n_t, 128, 4096)), dim3(128), 0, st, m);
    }
    MergeOp op{m};
    hipLaunchKernelGGL(k_mrg_scan_part, dim3(kMrgScanBlocks), dim3(256), 0, st, op, m.b.scan_part);
    hipLaunchKernelGGL(k_mrg_scan_top, dim3(1), dim3(kMrgScanBlocks), 0, st, m.b.scan_part, m.b.ctr);
    hipLaunchKernelGGL(k_mrg_scan_apply, dim3(kMrgScanBlocks), dim3(256), 0, st, op,
                       (const unsigned long long*)m.b.scan_part);
    hipLaunchKernelGGL(k_mrg_write, dim3(grid_of(m.n_t, 256, 4096)), dim3(256), 0, st, m);
}

}  // namespace tpcca
