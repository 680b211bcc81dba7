// HIP kernels (gfx950, wave64) of the TPC sector tracker.
//
// Stages (Section 2 of arXiv:1811.11481, with the resolution changes of
// Section 3): per-row hit grid, cellular-automaton neighbour links, mutual
// link cleaning and start hits, Kalman tracklets (seed fit, outward
// following, inward re-pick through the seed), ownership selection, the
// three-pass refit with chi2 rejection, compaction into the caller's track
// arrays and FP64 totals.
//
// Work mapping: one workgroup per (instance, row) for the grid and the links
// (the paper parallelises the cellular automaton over hits), one lane per
// tracklet and one lane per track for the Kalman stages (parallel over
// tracks). Compactions are deterministic three-phase scans. No result depends
// on the grid bin size, the launch shape or thread order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "kf_device.h"

#pragma clang fp contract(off)

namespace tpcca {

namespace {

constexpr float kBinMargin = 0.01f;  // cm: bin ranges of window queries are widened by this
constexpr int kCandChunk = 8;         // window candidates loaded per memory round trip
// neighbour candidates in row r-1 kept in registers per hit: 8 where both
// adjacent rows hold at most kDenseRow clusters, 16 in denser rows (more
// registers, which slow the sparse rows down)
constexpr int kNbKeep = 8;
constexpr int kNbKeepDense = 16;
constexpr int kDenseRow = 512;
constexpr int kSmallRow = 4096;
constexpr int kLargeRow = 16384;      // TPCCA_MAX_ROW_CLUSTERS
constexpr int kKeyShift = 14;         // key = bin << 14 | local index (both < 16384)

__device__ __forceinline__ void raise_err(Counters* c, unsigned int bit) { atomicOr(&c->err, bit); }

// The device CSR check (run before every stage when the host does not check
// the input) found a malformed input: the stage kernels then do nothing. The
// flag is written only by that check, so it is the same for every thread of
// every later kernel.
__device__ __forceinline__ bool input_rejected(const Counters* c) { return (c->err & ERR_CSR) != 0u; }

__device__ __forceinline__ void stat_add(Counters* c, int slot, unsigned long long v) {
    // wave-aggregated add
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&c->stats[slot], v);
}

// Bin index of coordinate v: trunc((v - vmin) * inv) clamped to [0, nb - 1]
// (a NaN maps to bin 0, so a malformed input never indexes out of range).
__device__ __forceinline__ int bin_of(float v, float vmin, float inv, int nb) {
    const float t = (v - vmin) * inv;
    if (!(t > 0.0f)) return 0;
    if (t >= (float)(nb - 1)) return nb - 1;
    return (int)t;
}

// Row of a grid position / cluster id inside instance `inst` (binary search).
__device__ __forceinline__ int row_of(const int64_t* row_start, int64_t seg0, int nr, int64_t pos) {
    int lo = 0, hi = nr;  // find last r with row_start[seg0 + r] <= pos
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row_start[seg0 + mid] <= pos) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct GridView {
    int64_t rs;        // first grid position of the segment
    const int32_t* bs; // bin starts (relative positions)
    int ny, nz, n;
    float ymin, zmin, iy, iz;
};

__device__ __forceinline__ SegHdr load_hdr(const Bufs& b, int64_t seg) { return b.hdr[seg]; }

__device__ __forceinline__ GridView grid_view(const Bufs& b, int64_t seg, const SegHdr& h) {
    GridView g;
    g.rs = h.rs;
    g.n = h.n;
    g.bs = b.bin_start + (int64_t)h.rs + seg;
    g.ny = h.ny;
    g.nz = h.nz;
    g.ymin = h.ymin;
    g.zmin = h.zmin;
    g.iy = h.iy;
    g.iz = h.iz;
    return g;
}

__device__ __forceinline__ GridView grid_view(const Bufs& b, int64_t seg) { return grid_view(b, seg, load_hdr(b, seg)); }

// ------------------------------------------------------------------ native coordinates
// Per-row constants of the native-to-local transform (side: +1 on the A
// side, sectors 0..17, -1 on the C side).
struct NativeRow {
    float pc, pw, zr, zpb, side;
    int on;
};

__device__ __forceinline__ NativeRow native_row(const Bufs& b, int64_t seg) {
    NativeRow t{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, b.native};
    if (t.on) {
        const DevConsts& K = *b.K;
        const int nr = K.n_rows;
        const int row = (int)(seg % nr);
        t.pc = K.pad_c[row];
        t.pw = K.pad_w[row];
        t.zr = K.z_readout;
        t.zpb = K.z_per_bin;
        t.side = b.inst_sector[seg / nr] < 18 ? 1.0f : -1.0f;
    }
    return t;
}

// Local (y, z) of cluster i: the input as it is, or native (pad, time)
// transformed (pad offset times pitch; time scaled linearly to the drift
// length from the readout plane).
__device__ __forceinline__ float2 cluster_yz(const Bufs& b, const NativeRow& t, int64_t i) {
    const float u = b.y[i], v = b.z[i];
    if (!t.on) return make_float2(u, v);
    return make_float2((u - t.pc) * t.pw, t.side * (t.zr - t.zpb * v));
}

__global__ __launch_bounds__(256) void k_native_local(Bufs b, int64_t nseg, float* y, float* z) {
    for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int64_t a = b.row_start[seg], e = b.row_start[seg + 1];
        if (a < 0 || e < a || e > b.n_clusters) continue;  // malformed CSR: nothing written
        const NativeRow t = native_row(b, seg);
        for (int64_t i = a + threadIdx.x; i < e; i += blockDim.x) {
            const float2 c = cluster_yz(b, t, i);
            y[i] = c.x;
            z[i] = c.y;
        }
    }
}

// ------------------------------------------------------------------ grid
// Bitonic sort of the 256 R keys key[0 .. 256 R) by 256 threads, thread t
// holding keys t + 256 r (r < R) in registers: partners at a distance of 256
// or more are in the same thread, 64 and 128 in another wave of the block
// (exchanged through LDS), below 64 in the same wave (lane shuffles). The
// network is unrolled, so every register index is a constant. Keys at and
// beyond `count` read as the largest key. All 256 threads must call it.
template <int R>
__device__ __forceinline__ void bitonic_regs(uint32_t* key, int count, int tid) {
    constexpr int N = 256 * R;
    uint32_t x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = (tid + 256 * r < count) ? key[tid + 256 * r] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 256) {
                const int jr = j >> 8;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r & jr) continue;
                    const bool asc = ((tid + 256 * r) & k) == 0;
                    const uint32_t lo = x[r], hi = x[r | jr];
                    const uint32_t mn = lo < hi ? lo : hi, mx = lo < hi ? hi : lo;
                    x[r] = asc ? mn : mx;
                    x[r | jr] = asc ? mx : mn;
                }
            } else {
                uint32_t y[R];
                if (j < 64) {
#pragma unroll
                    for (int r = 0; r < R; ++r) y[r] = __shfl_xor(x[r], j, 64);
                } else {
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) key[tid + 256 * r] = x[r];
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) y[r] = key[(tid ^ j) + 256 * r];
                }
                const bool low = (tid & j) == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool asc = ((tid + 256 * r) & k) == 0;
                    const uint32_t mn = x[r] < y[r] ? x[r] : y[r], mx = x[r] < y[r] ? y[r] : x[r];
                    x[r] = (low == asc) ? mn : mx;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) key[tid + 256 * r] = x[r];
    __syncthreads();
}

// One workgroup per (instance, row): exact ranges, bin layout, stable sort of
// (bin, cluster index) keys by a bitonic network in LDS, gather of the sorted
// coordinates, bin starts.
template <int MAXN>
__global__ __launch_bounds__(256) void k_grid(Bufs b, int64_t seg0) {
    __shared__ uint32_t key[MAXN];
    __shared__ float red[4][4];
    __shared__ int sh_i[4];
    __shared__ float sh_f[4];
    if (input_rejected(b.ctr)) return;
    const int64_t seg = seg0 + blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    int64_t a = b.row_start[seg], e = b.row_start[seg + 1];
    bool bad = (a < 0) || (e < a) || (e > b.n_clusters);
    int64_t n64 = bad ? 0 : e - a;
    if (MAXN == kSmallRow) {
        if (n64 > kSmallRow) return;  // handled by the large variant
    } else {
        if (n64 <= kSmallRow) return;
        if (n64 > kLargeRow) {
            if (tid == 0) raise_err(b.ctr, ERR_ROW_CAP);
            return;
        }
    }
    if (bad && tid == 0) raise_err(b.ctr, ERR_ARG);
    const int n = (int)n64;
    const int nr = b.K->n_rows;
    const NativeRow nat = native_row(b, seg);
    // ranges
    float ymn = __builtin_inff(), ymx = -__builtin_inff(), zmn = __builtin_inff(), zmx = -__builtin_inff();
    bool nonfinite = false;
    for (int i = tid; i < n; i += nt) {
        const float2 c = cluster_yz(b, nat, a + i);
        const float yv = c.x, zv = c.y;
        nonfinite |= !(__builtin_fabsf(yv) <= 3.0e38f) || !(__builtin_fabsf(zv) <= 3.0e38f);
        ymn = fminf(ymn, yv); ymx = fmaxf(ymx, yv);
        zmn = fminf(zmn, zv); zmx = fmaxf(zmx, zv);
    }
    if (nonfinite) raise_err(b.ctr, ERR_ARG);
    for (int o = 32; o > 0; o >>= 1) {
        ymn = fminf(ymn, __shfl_xor(ymn, o, 64)); ymx = fmaxf(ymx, __shfl_xor(ymx, o, 64));
        zmn = fminf(zmn, __shfl_xor(zmn, o, 64)); zmx = fmaxf(zmx, __shfl_xor(zmx, o, 64));
    }
    const int wid = tid >> 6;
    if ((tid & 63) == 0) {
        red[wid][0] = ymn; red[wid][1] = ymx; red[wid][2] = zmn; red[wid][3] = zmx;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < (nt >> 6); ++w) {
            ymn = fminf(ymn, red[w][0]); ymx = fmaxf(ymx, red[w][1]);
            zmn = fminf(zmn, red[w][2]); zmx = fmaxf(zmx, red[w][3]);
        }
        int ny = 1, nz = 1;
        float iy = 0.0f, iz = 0.0f;
        if (n == 0) {
            ymn = zmn = 0.0f;
        } else {
            const float ly = ymx - ymn, lz = zmx - zmn;
            const int tb = max(1, n / b.hits_per_bin);
            if (ly > 0.0f && lz > 0.0f) {
                const float f = __builtin_sqrtf((float)tb * (ly / lz));
                ny = (f >= (float)tb) ? tb : max(1, (int)f);
            } else if (ly > 0.0f) {
                ny = tb;
            } else {
                ny = 1;
            }
            nz = max(1, tb / ny);
            iy = ly > 0.0f ? (float)ny / ly : 0.0f;
            iz = lz > 0.0f ? (float)nz / lz : 0.0f;
        }
        SegHdr h;
        h.rs = (int32_t)a;
        h.n = n;
        h.ny = ny;
        h.nz = nz;
        h.ymin = ymn;
        h.zmin = zmn;
        h.iy = iy;
        h.iz = iz;
        b.hdr[seg] = h;
        sh_i[0] = ny; sh_i[1] = nz;
        sh_f[0] = ymn; sh_f[1] = zmn; sh_f[2] = iy; sh_f[3] = iz;
    }
    __syncthreads();
    const int ny = sh_i[0], nz = sh_i[1];
    const float ymin = sh_f[0], zmin = sh_f[1], iy = sh_f[2], iz = sh_f[3];
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = tid; i < P; i += nt) {
        if (i < n) {
            const float2 c = cluster_yz(b, nat, a + i);
            const int by = bin_of(c.x, ymin, iy, ny);
            const int bz = bin_of(c.y, zmin, iz, nz);
            key[i] = ((uint32_t)(bz * ny + by) << kKeyShift) | (uint32_t)i;
        } else {
            key[i] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    // keys in registers (padded to 256 R) up to 2048 keys; larger rows sort in
    // LDS with a barrier per stage
    if (nt == 256 && P <= 256) {
        bitonic_regs<1>(key, P, tid);
    } else if (nt == 256 && P == 512) {
        bitonic_regs<2>(key, P, tid);
    } else if (nt == 256 && P == 1024) {
        bitonic_regs<4>(key, P, tid);
    } else if (nt == 256 && P == 2048 && MAXN >= 2048) {
        bitonic_regs<8>(key, P, tid);
    } else {
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < P; i += nt) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const uint32_t x = key[i], w = key[ixj];
                        const bool asc = (i & k) == 0;
                        if ((x > w) == asc) {
                            key[i] = w;
                            key[ixj] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    int32_t* bs = b.bin_start + a + seg;
    const int nb = ny * nz;
    for (int p = tid; p < n; p += nt) {
        const uint32_t kk = key[p];
        const int i = (int)(kk & ((1u << kKeyShift) - 1));
        const int bin = (int)(kk >> kKeyShift);
        b.yz[a + p] = cluster_yz(b, nat, a + i);
        b.sid[a + p] = (int32_t)(a + i);
        b.pos_of[a + i] = (int32_t)(a + p);
        const int prev = (p == 0) ? -1 : (int)(key[p - 1] >> kKeyShift);
        for (int q = prev + 1; q <= bin; ++q) bs[q] = p;
    }
    if (tid == 0) {
        const int last = (n == 0) ? -1 : (int)(key[n - 1] >> kKeyShift);
        for (int q = last + 1; q <= nb; ++q) bs[q] = n;
    }
    (void)nr;
}

// The GPU hands consecutive workgroups to its 8 XCDs in turn (workgroup g
// runs on XCD g mod 8), and every XCD has its own L2. Renumbering physical
// workgroup g of a period P (a multiple of 8) to logical workgroup
// (g mod 8) * P/8 + g/8 gives XCD x the contiguous logical range
// [x P/8, (x+1) P/8): work that is adjacent in the logical order (the rows of
// one sector instance, the seeds of one instance) then shares one L2 instead
// of being spread over all eight.
__device__ __forceinline__ int64_t xcd_logical(int64_t g, int64_t P) { return (g & 7) * (P >> 3) + (g >> 3); }

// ------------------------------------------------------------------ links
// One workgroup per (instance, row); one lane per hit of the row. Candidate
// pairs (u on row+1, d on row-1) inside the windows; the minimum straight-line
// deviation score wins, ties to the smaller (id_u, id_d). When both adjacent
// rows fit in `cap` clusters, their coordinates and bin starts are staged in
// LDS once per workgroup and every candidate read is an LDS read.
// rows: 0 every row; 1 the rows whose adjacent rows both hold at most
// kDenseRow clusters (and the first and last rows); 2 the others.
template <int KEEP>
__global__ __launch_bounds__(1024) void k_links(Bufs b, int64_t seg0, int64_t nseg, int cap, int remap, int rows) {
    extern __shared__ unsigned char smem[];
    const DevConsts& K = *b.K;
    const int nr = K.n_rows;
    const int64_t l = remap ? xcd_logical(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    if (l >= nseg || input_rejected(b.ctr)) return;
    const int64_t seg = seg0 + l;
    const int r = (int)(seg % nr);
    const int64_t a = b.row_start[seg], e = b.row_start[seg + 1];
    if (r == 0 || r == nr - 1) {
        if (rows == 2) return;
        for (int64_t p = a + threadIdx.x; p < e; p += blockDim.x) {
            b.up[p] = -1;
            b.dn[p] = -1;
        }
        return;
    }
    const GridView gu = grid_view(b, seg + 1);
    const GridView gd = grid_view(b, seg - 1);
    if (rows != 0 && ((gu.n > kDenseRow || gd.n > kDenseRow) != (rows == 2))) return;  // uniform: the other launch
    const int nbu = gu.ny * gu.nz, nbd = gd.ny * gd.nz;
    const bool lds = cap > 0 && gu.n <= cap && gd.n <= cap;  // uniform over the workgroup
    float2* su = reinterpret_cast<float2*>(smem);
    float2* sd = su + cap;
    int32_t* sbu = reinterpret_cast<int32_t*>(sd + cap);
    int32_t* sbd = sbu + cap + 1;
    if (lds) {
        for (int i = threadIdx.x; i < gu.n; i += blockDim.x) su[i] = b.yz[gu.rs + i];
        for (int i = threadIdx.x; i < gd.n; i += blockDim.x) sd[i] = b.yz[gd.rs + i];
        for (int i = threadIdx.x; i <= nbu; i += blockDim.x) sbu[i] = gu.bs[i];
        for (int i = threadIdx.x; i <= nbd; i += blockDim.x) sbd[i] = gd.bs[i];
        __syncthreads();
    }
    const float2* cu = lds ? su : b.yz + gu.rs;
    const float2* cd = lds ? sd : b.yz + gd.rs;
    const int32_t* bsu = lds ? sbu : gu.bs;
    const int32_t* bsd = lds ? sbd : gd.bs;
    const float wyu = K.wyu[r], wzu = K.wzu[r], wyd = K.wyd[r], wzd = K.wzd[r], tr = K.tr[r], smax = K.smax;
    unsigned long long n_links = 0, n_cu = 0, n_pairs = 0;
    for (int64_t p = a + threadIdx.x; p < e; p += blockDim.x) {
        const float2 ph = b.yz[p];
        const float yh = ph.x, zh = ph.y;
        bool found = false;
        float best = 0.0f;
        int32_t bu = -1, bd = -1;  // relative positions in rows r+1 and r-1
        if (gu.n > 0 && gd.n > 0) {
            const int uy0 = bin_of((yh - wyu) - kBinMargin, gu.ymin, gu.iy, gu.ny);
            const int uy1 = bin_of((yh + wyu) + kBinMargin, gu.ymin, gu.iy, gu.ny);
            const int uz0 = bin_of((zh - wzu) - kBinMargin, gu.zmin, gu.iz, gu.nz);
            const int uz1 = bin_of((zh + wzu) + kBinMargin, gu.zmin, gu.iz, gu.nz);
            const int dy0 = bin_of((yh - wyd) - kBinMargin, gd.ymin, gd.iy, gd.ny);
            const int dy1 = bin_of((yh + wyd) + kBinMargin, gd.ymin, gd.iy, gd.ny);
            const int dz0 = bin_of((zh - wzd) - kBinMargin, gd.zmin, gd.iz, gd.nz);
            const int dz1 = bin_of((zh + wzd) + kBinMargin, gd.zmin, gd.iz, gd.nz);
            // a candidate pair (u, d) that passed both boxes
            auto pair = [&](int q, float yu, float zu, int t, float yd, float zd) {
                ++n_pairs;
                const float ey = (yd + (yu - yd) * tr) - yh;
                const float ez = (zd + (zu - zd) * tr) - zh;
                const float sc = ey * ey + ez * ez;
                if (!(sc <= smax)) return;
                bool take = !found || sc < best;
                if (!take && sc == best) {  // ids decide only exact ties
                    const int32_t uid = b.sid[gu.rs + q], did = b.sid[gd.rs + t];
                    const int32_t buid = b.sid[gu.rs + bu], bdid = b.sid[gd.rs + bd];
                    take = uid < buid || (uid == buid && did < bdid);
                }
                if (take) {
                    found = true;
                    best = sc;
                    bu = q;
                    bd = t;
                }
            };
            // the d candidates inside their box, scanned once: up to KEEP kept
            // in registers (a shift register, no indexed register access)
            int nd = 0;
            int dt[KEEP];
            float2 dc[KEEP];
#pragma unroll
            for (int i = 0; i < KEEP; ++i) {
                dt[i] = 0;
                dc[i] = make_float2(0.0f, 0.0f);
            }
            const bool short_d = dz1 - dz0 <= 1;
            if (short_d) {
                const int d00 = bsd[dz0 * gd.ny + dy0], d01 = bsd[dz0 * gd.ny + dy1 + 1];
                int d10 = 0, d11 = 0;
                if (dz1 > dz0) {
                    d10 = bsd[(dz0 + 1) * gd.ny + dy0];
                    d11 = bsd[(dz0 + 1) * gd.ny + dy1 + 1];
                }
                const int na = max(d01 - d00, 0), n2 = na + max(d11 - d10, 0);
                for (int k = 0; k < n2; ++k) {
                    const int t = k < na ? d00 + k : d10 + (k - na);
                    const float2 pd = cd[t];
                    if (!(__builtin_fabsf(pd.x - yh) <= wyd && __builtin_fabsf(pd.y - zh) <= wzd)) continue;
#pragma unroll
                    for (int i = KEEP - 1; i > 0; --i) {
                        dt[i] = dt[i - 1];
                        dc[i] = dc[i - 1];
                    }
                    dt[0] = t;
                    dc[0] = pd;
                    ++nd;
                }
            } else {
                // a window over three or more bin rows (small bins of dense
                // rows): the same collection row by row, given up as soon as
                // more than KEEP candidates are inside
                for (int dz = dz0; dz <= dz1 && nd <= KEEP; ++dz) {
                    const int t0 = bsd[dz * gd.ny + dy0], t1 = bsd[dz * gd.ny + dy1 + 1];
                    for (int t = t0; t < t1 && nd <= KEEP; ++t) {
                        const float2 pd = cd[t];
                        if (!(__builtin_fabsf(pd.x - yh) <= wyd && __builtin_fabsf(pd.y - zh) <= wzd)) continue;
#pragma unroll
                        for (int i = KEEP - 1; i > 0; --i) {
                            dt[i] = dt[i - 1];
                            dc[i] = dc[i - 1];
                        }
                        dt[0] = t;
                        dc[0] = pd;
                        ++nd;
                    }
                }
            }
            const bool kept = nd <= KEEP;
            for (int uz = uz0; uz <= uz1; ++uz) {
                const int q0 = bsu[uz * gu.ny + uy0], q1 = bsu[uz * gu.ny + uy1 + 1];
                for (int q = q0; q < q1; ++q) {
                    const float2 pu = cu[q];
                    const float yu = pu.x, zu = pu.y;
                    if (!(__builtin_fabsf(yu - yh) <= wyu && __builtin_fabsf(zu - zh) <= wzu)) continue;
                    ++n_cu;
                    if (kept) {
#pragma unroll
                        for (int i = 0; i < KEEP; ++i)
                            if (nd > i) pair(q, yu, zu, dt[i], dc[i].x, dc[i].y);
                        continue;
                    }
                    for (int dz = dz0; dz <= dz1; ++dz) {
                        const int t0 = bsd[dz * gd.ny + dy0], t1 = bsd[dz * gd.ny + dy1 + 1];
                        for (int t = t0; t < t1; ++t) {
                            const float2 pd = cd[t];
                            if (!(__builtin_fabsf(pd.x - yh) <= wyd && __builtin_fabsf(pd.y - zh) <= wzd)) continue;
                            pair(q, yu, zu, t, pd.x, pd.y);
                        }
                    }
                }
            }
        }
        b.up[p] = found ? (int32_t)(gu.rs + bu) : -1;
        b.dn[p] = found ? (int32_t)(gd.rs + bd) : -1;
        n_links += found ? 1 : 0;
    }
    if (K.stats) {
        stat_add(b.ctr, ST_LINKS, n_links);
        stat_add(b.ctr, ST_NB_CAND_U, n_cu);
        stat_add(b.ctr, ST_NB_PAIRS, n_pairs);
    }
}

// ------------------------------------------------------------------ clean
__global__ void k_clean(Bufs b, int64_t c0, int64_t c1) {
    if (input_rejected(b.ctr)) return;
    for (int64_t p = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < c1;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = b.up[p], d = b.dn[p];
        const int32_t uc = (u >= 0 && b.dn[u] == p) ? u : -1;
        const int32_t dc = (d >= 0 && b.up[d] == p) ? d : -1;
        b.upc[p] = uc;
        b.dnc[p] = dc;
        // a start hit: no cleaned link down, and cleaned links up twice (the
        // next hit's cleaned up link, from the same uncleaned links)
        bool start = false;
        if (dc == -1 && uc != -1) {
            const int32_t w = b.up[uc];
            start = w >= 0 && b.dn[w] == uc;
        }
        b.start_flag[p] = start ? 1 : 0;
    }
}

// ------------------------------------------------------------------ scans
// Deterministic three-phase exclusive scan over [begin, end) of 64-bit packed
// values (hi 32 bits: items, lo 32 bits: sub-items), split into kScanBlocks
// contiguous chunks. Phase 3 hands each element its exclusive prefix
// (including the running total of earlier ranges) to Op::write.
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v, unsigned long long* sh,
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

// Elements per thread and tile of the scan kernels, Op::kVec: a thread takes
// kVec consecutive elements, so their value() loads are in flight together
// and a block-wide scan runs once per tile of kVec * blockDim elements (8 for
// the start hits, a cheap value over every cluster; 1 where write() is heavy
// and a block's chunk short).

template <class Op>
__global__ void k_scan_part(Op op, unsigned long long* part) {
    constexpr int kScanVec = Op::kVec;
    __shared__ unsigned long long sh[17];
    if (input_rejected(op.b.ctr)) return;
    const int64_t b0 = op.begin(), e0 = op.end();
    const int64_t n = e0 > b0 ? e0 - b0 : 0;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = b0 + blockIdx.x * chunk;
    const int64_t hi = min(lo + chunk, e0);
    unsigned long long s = 0;
    for (int64_t t0 = lo + (int64_t)threadIdx.x * kScanVec; t0 < hi; t0 += (int64_t)blockDim.x * kScanVec) {
        unsigned long long v[kScanVec];
#pragma unroll
        for (int k = 0; k < kScanVec; ++k) v[k] = (t0 + k < hi) ? op.value(t0 + k) : 0ull;
#pragma unroll
        for (int k = 0; k < kScanVec; ++k) s += v[k];
    }
    unsigned long long tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single workgroup of kScanBlocks threads
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long* part, Counters* ctr, int slot) {
    __shared__ unsigned long long sh[17];
    if (input_rejected(ctr)) return;  // the range counts stay zero: no later stage has work
    const unsigned long long v = part[threadIdx.x];
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan(v, sh, &tot);
    part[threadIdx.x] = ex;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long base = ctr->slot[slot][0];
        ctr->slot[slot][1] = base;
        ctr->slot[slot][2] = tot;
        ctr->slot[slot][0] = base + tot;
    }
}

template <class Op>
__global__ void k_scan_apply(Op op, const unsigned long long* part, const Counters* ctr, int slot) {
    constexpr int kScanVec = Op::kVec;
    __shared__ unsigned long long sh[17];
    if (input_rejected(ctr)) return;
    const int64_t b0 = op.begin(), e0 = op.end();
    const int64_t n = e0 > b0 ? e0 - b0 : 0;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = b0 + blockIdx.x * chunk;
    const int64_t hi = min(lo + chunk, e0);
    const int64_t tile = (int64_t)blockDim.x * kScanVec;
    unsigned long long run = ctr->slot[slot][1] + part[blockIdx.x];
    // per-block context for write() (the start hits: the instance of the
    // block's first cluster, found once)
    __shared__ int s_hint;
    if (threadIdx.x == 0) s_hint = lo < hi ? op.hint(lo) : 0;
    __syncthreads();
    const int hint = s_hint;
    for (int64_t t0 = lo; t0 < hi; t0 += tile) {  // uniform trip count per block
        const int64_t i0 = t0 + (int64_t)threadIdx.x * kScanVec;  // this thread's consecutive elements
        unsigned long long v[kScanVec], s = 0;
#pragma unroll
        for (int k = 0; k < kScanVec; ++k) {
            v[k] = (i0 + k < hi) ? op.value(i0 + k) : 0ull;
            s += v[k];
        }
        unsigned long long tot;
        unsigned long long ex = block_excl_scan(s, sh, &tot);
#pragma unroll
        for (int k = 0; k < kScanVec; ++k) {
            if (v[k]) op.write(i0 + k, run + ex, v[k], hint);
            ex += v[k];
        }
        run += tot;
    }
}

// Start hits, over cluster ids [c0, c1) of an instance range.
struct StartOp {
    static constexpr int kVec = 8;
    Bufs b;
    int64_t c0, c1;
    int i0, i1;
    __device__ int64_t begin() const { return c0; }
    __device__ int64_t end() const { return c1; }
    __device__ unsigned long long value(int64_t id) const { return b.start_flag[b.pos_of[id]]; }
    // instance of cluster id: the last k with row_start[k * n_rows] <= id
    __device__ int hint(int64_t id) const {
        const int nr = b.n_rows;
        int lo = i0, hi = i1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.row_start[(int64_t)mid * nr] <= id) lo = mid;
            else hi = mid;
        }
        return lo;
    }
    // inst0: the instance of an earlier cluster of the block's chunk (a chunk
    // rarely crosses an instance boundary, so this walks at most a few steps)
    __device__ void write(int64_t id, unsigned long long prefix, unsigned long long, int inst0) const {
        const int64_t j = (int64_t)(prefix & 0xFFFFFFFFull);
        if (j >= b.cap_starts) {
            raise_err(b.ctr, ERR_SCRATCH);
            return;
        }
        const int nr = b.n_rows;
        int inst = inst0;
        while (inst + 1 < i1 && b.row_start[(int64_t)(inst + 1) * nr] <= id) ++inst;
        b.starts[j] = b.pos_of[id];
        b.start_inst[j] = inst;
    }
};

// Selection, over tracklets of the current start range.
__device__ __forceinline__ uint32_t packed_weight(int nh, int tid) {
    return ((uint32_t)nh << 20) | (uint32_t)(0xFFFFF - tid);
}

struct SelectOp {
    static constexpr int kVec = 1;
    Bufs b;
    __device__ int64_t begin() const { return (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull); }
    __device__ int64_t end() const {
        const int64_t e = begin() + (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
        return e < b.cap_starts ? e : b.cap_starts;
    }
    __device__ unsigned long long value(int64_t j) const {
        const int own = b.tl_own[j];
        return own >= b.K->n_min ? ((1ull << 32) | (unsigned long long)own) : 0ull;
    }
    __device__ int hint(int64_t) const { return 0; }
    __device__ void write(int64_t j, unsigned long long prefix, unsigned long long v, int) const {
        const int64_t si = (int64_t)(prefix >> 32);
        const int64_t ho = (int64_t)(prefix & 0xFFFFFFFFull);
        const int own = (int)(v & 0xFFFFFFFFull);
        if (si >= b.cap_sel || ho + own > b.n_clusters) {
            raise_err(b.ctr, ERR_SCRATCH);
            return;
        }
        b.sel_tl[si] = (int32_t)j;
        b.sel_off[si] = (int32_t)ho;
        b.sel_n[si] = own;
    }
};

// Owned picks of every tracklet of the current range: count and bitmask. One
// wave per tracklet, one lane per pick (the picks' weight reads are
// independent, so they overlap instead of queueing behind one lane).
// A contiguous block of items for each wave, the workgroups numbered per
// XCD: the waves of one XCD cover one contiguous share of the items. In the
// ownership test the items are tracklets in instance order, so one XCD
// gathers the weights of a contiguous share of the instances and they stay in
// its L2 (C3, dense instances: 0.74 -> 0.54 ms; the selection-list and output
// kernels balance better with the interleaved loop). The range is uniform
// over the wave.
struct WaveBlock {
    int64_t lo, hi;
};
__device__ __forceinline__ WaveBlock wave_block(int64_t cnt) {
    const int64_t wpb = blockDim.x >> 6;
    const int64_t P = gridDim.x >= 8 ? (int64_t)(gridDim.x & ~7u) : (int64_t)gridDim.x;
    if ((int64_t)blockIdx.x >= P) return WaveBlock{0, 0};
    const int64_t lg = gridDim.x >= 8 ? xcd_logical(blockIdx.x, P) : (int64_t)blockIdx.x;
    const int64_t nw = P * wpb, w = lg * wpb + (threadIdx.x >> 6);
    const int64_t per = (cnt + nw - 1) / nw;
    const int64_t lo = min(cnt, w * per);
    return WaveBlock{lo, min(cnt, lo + per)};
}

__global__ void k_own(Bufs b) {
    const int nr = b.K->n_rows, n_min = b.K->n_min;
    const int64_t base = (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;
    const int lane = threadIdx.x & 63;
    const WaveBlock wb = wave_block(cnt);
    for (int64_t k0 = wb.lo; k0 < wb.hi; ++k0) {
        const int64_t j = base + k0;
        const int nh = b.tl_nhits[j];
        uint32_t mk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int own = 0;
        if (nh >= n_min) {
            const uint32_t w = packed_weight(nh, b.tl_tid[j]);
#pragma unroll
            for (int c = 0; c < 256; c += 64) {
                if (c >= nh) break;
                const int k = c + lane;
                const bool o = k < nh && b.weight[b.tl_pick_pos[j * nr + k]] == w;
                const unsigned long long bal = __ballot(o);
                mk[c >> 5] = (uint32_t)bal;
                mk[(c >> 5) + 1] = (uint32_t)(bal >> 32);
                own += __popcll(bal);
            }
        }
        if (lane == 0) {
            b.tl_own[j] = own;
            uint4* dst = reinterpret_cast<uint4*>(b.tl_ownmask + j * 8);  // 32-byte aligned rows
            dst[0] = make_uint4(mk[0], mk[1], mk[2], mk[3]);
            dst[1] = make_uint4(mk[4], mk[5], mk[6], mk[7]);
        }
    }
}

// Cluster lists of the selected tracklets (offsets from the selection scan):
// one wave per tracklet, one lane per pick. Owned pick k goes to position
// (owned picks after k) of the list, i.e. rows ascending, as the picks are
// stored rows descending.
__global__ void k_sel_fill(Bufs b) {
    const int nr = b.K->n_rows;
    const int64_t base = (int64_t)(b.ctr->slot[SL_SEL][1] >> 32);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_SEL][2] >> 32);
    if (base + cnt > b.cap_sel) cnt = b.cap_sel > base ? b.cap_sel - base : 0;
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; k0 < cnt; k0 += nwave) {
        const int64_t si = base + k0;
        const int32_t j = b.sel_tl[si];
        const int64_t ho = b.sel_off[si];
        const int own = b.sel_n[si];
        if (ho + own > b.n_clusters) continue;  // flagged by the scan
        const int nh = b.tl_nhits[j];
        const uint32_t* mask = b.tl_ownmask + (int64_t)j * 8;
        int run = 0;  // owned picks in the chunks before this one
        for (int c = 0; c < nh; c += 64) {
            const int k = c + lane;
            const bool o = k < nh && ((mask[k >> 5] >> (k & 31)) & 1u);
            const unsigned long long bal = __ballot(o);
            const int before = run;
            run += __popcll(bal);
            if (!o) continue;
            const int le = before + __popcll(bal & ((2ull << lane) - 1ull));  // owned picks with index <= k
            const int64_t m = ho + (own - le);
            const int32_t pos = b.tl_pick_pos[(int64_t)j * nr + k];
            b.sel_pos[m] = pos;
            b.sel_yz[m] = b.yz[pos];
            b.sel_row[m] = b.tl_pick_row[(int64_t)j * nr + k];
        }
    }
}


// Output tracks, over the current range of selected tracklets.
struct TrackOp {
    static constexpr int kVec = 1;
    Bufs b;
    __device__ int64_t begin() const { return (int64_t)(b.ctr->slot[SL_SEL][1] >> 32); }
    __device__ int64_t end() const {
        const int64_t e = begin() + (int64_t)(b.ctr->slot[SL_SEL][2] >> 32);
        return e < b.cap_sel ? e : b.cap_sel;
    }
    __device__ unsigned long long value(int64_t si) const {
        return b.rf_ok[si] ? ((1ull << 32) | (unsigned long long)b.rf_nacc[si]) : 0ull;
    }
    __device__ int hint(int64_t) const { return 0; }
    __device__ void write(int64_t si, unsigned long long prefix, unsigned long long v, int) const {
        const int64_t t = (int64_t)(prefix >> 32);
        const int64_t ho = (int64_t)(prefix & 0xFFFFFFFFull);
        const int nacc = (int)(v & 0xFFFFFFFFull);
        if (t >= b.cap_tracks || ho + nacc > b.cap_hits) {
            raise_err(b.ctr, ERR_OUT_CAP);
            b.trk_t[si] = -1;
            return;
        }
        b.trk_t[si] = (int32_t)t;
        b.trk_ho[si] = (int32_t)ho;
        const DevConsts& K = *b.K;
        const int32_t tl = b.sel_tl[si];
        const int32_t inst = b.start_inst[tl];
        b.o_inst[t] = inst;
        b.o_xref[t] = K.X[b.rf_row[si]];
        const int sec = b.inst_sector[inst];
        b.o_alpha[t] = K.alpha[((sec % 18) + 18) % 18];
        for (int q = 0; q < 5; ++q) b.o_param[t * 5 + q] = b.rf_state[si * 20 + q];
        for (int q = 0; q < 15; ++q) b.o_cov[t * 15 + q] = b.rf_state[si * 20 + 5 + q];
        b.o_chi2[t] = b.rf_chi2[si];
        b.o_ndf[t] = 2 * nacc - 5;
        b.o_hit_start[t] = ho;
        if (b.keep_merge) b.trk_si[t] = (int32_t)si;
        if (b.o_z0) b.o_z0[t] = vertex_z(K.kB_f64, (double)K.X[b.rf_row[si]], b.rf_state + si * 20);
    }
};

// Cluster ids of the output tracks: one wave per selected tracklet, one lane
// per cluster; the clusters used in the last pass keep their order (ballot
// prefix counts).
__global__ void k_trk_fill(Bufs b) {
    const int64_t base = (int64_t)(b.ctr->slot[SL_SEL][1] >> 32);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_SEL][2] >> 32);
    if (base + cnt > b.cap_sel) cnt = b.cap_sel > base ? b.cap_sel - base : 0;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; k0 < cnt; k0 += nwave) {
        const int64_t si = base + k0;
        if (!b.rf_ok[si]) continue;
        const int32_t t = b.trk_t[si];
        if (t < 0) continue;  // capacity exceeded: flagged by the scan
        const int64_t ho = b.trk_ho[si];
        const int off = b.sel_off[si], n = b.sel_n[si];
        int run = 0;
        for (int c = 0; c < n; c += 64) {
            const int i = c + lane;
            const bool use = i < n && (b.sel_mask[off + i] & 4);
            const unsigned long long bal = __ballot(use);
            if (use) {
                const int64_t at = ho + run + __popcll(bal & below);
                b.o_hit_id[at] = b.sid[b.sel_pos[off + i]];
                if (b.o_res) reinterpret_cast<uint32_t*>(b.o_res)[at] = b.sel_res[off + i];
                if (b.keep_merge) b.trk_hrow[at] = b.sel_row[off + i];
            }
            run += __popcll(bal);
        }
    }
}

// ------------------------------------------------------------------ tracklets
struct Pick {
    int32_t pos;
    Innov inn;
};

// Best cluster on the row of segment `seg` for the predicted state.
__device__ __forceinline__ bool pick_on_row(const Bufs& b, const KfConsts& K, const KState& s, int64_t seg,
                                            const SegHdr& h, Pick& out, unsigned int& ncand) {
    const GridView g = grid_view(b, seg, h);
    if (g.n == 0) return false;
    const float s00 = s.C[0] + K.vy, s01 = s.C[1], s11 = s.C[2] + K.vz;
    const float wy = K.nsig * __builtin_sqrtf(s00), wz = K.nsig * __builtin_sqrtf(s11);
    const float det = __builtin_fmaf(s00, s11, -(s01 * s01));
    const float idet = 1.0f / det;
    const float a00 = s11 * idet, a01 = (-s01) * idet, a11 = s00 * idet;
    const float py = s.p[0], pz = s.p[1];
    const int y0 = bin_of((py - wy) - kBinMargin, g.ymin, g.iy, g.ny);
    const int y1 = bin_of((py + wy) + kBinMargin, g.ymin, g.iy, g.ny);
    const int z0 = bin_of((pz - wz) - kBinMargin, g.zmin, g.iz, g.nz);
    const int z1 = bin_of((pz + wz) + kBinMargin, g.zmin, g.iz, g.nz);
    bool found = false;
    auto consider = [&](int64_t pos, float2 c) {
        const float r0 = c.x - py, r1 = c.y - pz;
        if (!(__builtin_fabsf(r0) <= wy && __builtin_fabsf(r1) <= wz)) return;
        const float w0 = __builtin_fmaf(a00, r0, a01 * r1);
        const float w1 = __builtin_fmaf(a01, r0, a11 * r1);
        const float chi2 = __builtin_fmaf(r0, w0, r1 * w1);
        if (!(chi2 <= K.chi2_pick)) return;
        // cluster ids decide only exact chi2 ties: load them only then
        if (!found || chi2 < out.inn.chi2 || (chi2 == out.inn.chi2 && b.sid[pos] < b.sid[out.pos])) {
            found = true;
            out.pos = (int32_t)pos;
            out.inn.a00 = a00;
            out.inn.a01 = a01;
            out.inn.a11 = a11;
            out.inn.r0 = r0;
            out.inn.r1 = r1;
            out.inn.chi2 = chi2;
        }
    };
    // bin-row ranges of the window: the first two rows' bounds are loaded together
    const int q00 = g.bs[z0 * g.ny + y0], q01 = g.bs[z0 * g.ny + y1 + 1];
    int q10 = 0, q11 = 0;
    if (z1 > z0) {
        q10 = g.bs[(z0 + 1) * g.ny + y0];
        q11 = g.bs[(z0 + 1) * g.ny + y1 + 1];
    }
    // the candidates of those two rows as one list, kCandChunk per memory
    // round trip: a wave then runs as many candidate tests as its longest list
    // needs, not the sum of per-row chunks and remainders
    const int na = max(q01 - q00, 0), n2 = na + max(q11 - q10, 0);
    for (int k = 0; k < n2; k += kCandChunk) {
        int64_t pos[kCandChunk];
        float2 c[kCandChunk];
#pragma unroll
        for (int i = 0; i < kCandChunk; ++i) {
            const int kk = min(k + i, n2 - 1);  // past the end: a repeat of the last, not tested
            pos[i] = g.rs + (kk < na ? q00 + kk : q10 + (kk - na));
            c[i] = b.yz[pos[i]];
        }
        // slots past the end get an infinite y: the window test rejects them
        // without a branch of their own (an infinite y passes only an infinite
        // window, whose s00 = inf makes a00 zero and the chi2 NaN)
#pragma unroll
        for (int i = 0; i < kCandChunk; ++i) {
            float2 ci = c[i];
            if (k + i >= n2) ci.x = __builtin_inff();
            consider(pos[i], ci);
        }
        ncand += (unsigned)min(kCandChunk, n2 - k);
    }
    // further rows of a tall window, one row at a time
    for (int bz = z0 + 2; bz <= z1; ++bz) {
        const int q0 = g.bs[bz * g.ny + y0], q1 = g.bs[bz * g.ny + y1 + 1];
        for (int q = q0; q < q1; q += kCandChunk) {
            int64_t pos[kCandChunk];
            float2 c[kCandChunk];
#pragma unroll
            for (int i = 0; i < kCandChunk; ++i) {
                pos[i] = g.rs + min(q + i, q1 - 1);
                c[i] = b.yz[pos[i]];
            }
#pragma unroll
            for (int i = 0; i < kCandChunk; ++i) {
                float2 ci = c[i];
                if (q + i >= q1) ci.x = __builtin_inff();
                consider(pos[i], ci);
            }
            ncand += (unsigned)min(kCandChunk, q1 - q);
        }
    }
    return found;
}

__device__ __forceinline__ bool seed_from_chain(const DevConsts& K, float x0, float y0, float z0, float xm, float ym,
                                                float xe, float ye, float ze, KState& s) {
    const float ax = xm - x0, ay = ym - y0, bx = xe - x0, by = ye - y0, cx = xe - xm, cy = ye - ym;
    const float cr = ax * by - ay * bx;
    const float d01 = __builtin_sqrtf(ax * ax + ay * ay);
    const float d02 = __builtin_sqrtf(bx * bx + by * by);
    const float d12 = __builtin_sqrtf(cx * cx + cy * cy);
    const float kap = (2.0f * cr) / ((d01 * d02) * d12);
    float v = (kap * d02) * 0.5f;
    if (v > 1.0f) v = 1.0f;
    if (v < -1.0f) v = -1.0f;
    const float sn = by / d02, cs = bx / d02;
    const float s0 = sn * __builtin_sqrtf(1.0f - v * v) - cs * v;
    const float arc = d02 * asin_over_u(v);
    const float t0 = (ze - z0) / arc;
    float q0 = (K.kB != 0.0f) ? kap / K.kB : 0.0f;
    if (q0 > K.q_max) q0 = K.q_max;
    if (q0 < -K.q_max) q0 = -K.q_max;
    if (!(__builtin_fabsf(s0) < K.sinphi_max)) return false;
    s.p[0] = y0;
    s.p[1] = z0;
    s.p[2] = s0;
    s.p[3] = t0;
    s.p[4] = q0;
#pragma unroll
    for (int q = 0; q < 15; ++q) s.C[q] = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) s.C[pk(i, i)] = K.c0[i];
    return true;
}

__device__ __forceinline__ int lower_bound_inst(const int32_t* a, int64_t lo, int64_t hi, int32_t v) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo;
}

// One lane per start hit: seed, stage 1 (chain), stage 2 (outward), turn,
// stage 3 (inward re-pick), weights.
// Stage-3 pick store: picks leave four at a time (one 16-byte and one 4-byte
// store) from a shift register, newest in p0; rows pack oldest-lowest.
struct PickRing {
    int32_t p0, p1, p2, p3;
    uint32_t rows4;
};

__device__ __forceinline__ void pick_store(const Bufs& b, int64_t j, int nr, int nh, int32_t pos, int r, bool vec,
                                           PickRing& pr) {
    if (vec) {
        pr.p3 = pr.p2;
        pr.p2 = pr.p1;
        pr.p1 = pr.p0;
        pr.p0 = pos;
        pr.rows4 = (pr.rows4 >> 8) | ((uint32_t)r << 24);
        if (((nh + 1) & 3) == 0) {
            *reinterpret_cast<int4*>(b.tl_pick_pos + j * nr + nh - 3) = make_int4(pr.p3, pr.p2, pr.p1, pr.p0);
            *reinterpret_cast<uint32_t*>(b.tl_pick_row + j * nr + nh - 3) = pr.rows4;
        }
    } else {
        b.tl_pick_pos[j * nr + nh] = pos;
        b.tl_pick_row[j * nr + nh] = (uint8_t)r;
    }
}

// The last picks (fewer than four), the pick count and the packed weights of
// a finished tracklet.
__device__ __forceinline__ void tracklet_finish(const Bufs& b, int64_t j, int nr, int nh, int tid, bool vec,
                                                const PickRing& pr, int n_min) {
    if (vec) {
        const int k = nh & 3;
        int32_t* pp = b.tl_pick_pos + j * nr + (nh - k);
        uint8_t* prow = b.tl_pick_row + j * nr + (nh - k);
        if (k == 3) {
            pp[0] = pr.p2;
            pp[1] = pr.p1;
            pp[2] = pr.p0;
        } else if (k == 2) {
            pp[0] = pr.p1;
            pp[1] = pr.p0;
        } else if (k == 1) {
            pp[0] = pr.p0;
        }
        for (int i = 0; i < k; ++i) prow[i] = (uint8_t)(pr.rows4 >> (8 * (4 - k + i)));
    }
    b.tl_nhits[j] = nh;
    if (nh >= n_min) {
        // weights: the picks are read back eight per memory round trip
        // (atomic max: the order of the tracklets does not matter)
        const uint32_t w = packed_weight(nh, tid);
        const int32_t* pp = b.tl_pick_pos + j * nr;
        if ((nr & 3) == 0) {
            for (int q = 0; q < nh; q += 8) {
                const int4 a = *reinterpret_cast<const int4*>(pp + q);
                int4 c = make_int4(0, 0, 0, 0);
                if (q + 4 < nh) c = *reinterpret_cast<const int4*>(pp + q + 4);  // q + 8 <= nr
                const int32_t v[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (q + i < nh) atomicMax(&b.weight[v[i]], w);
            }
        } else {
            for (int q = 0; q < nh; ++q) atomicMax(&b.weight[pp[q]], w);
        }
    }
}

// The turn and stage 3 of one tracklet: covariance reset, the state carried
// from the row the outward following reached down to its last cluster's row,
// then the inward re-pick down to row 0 (or max_miss empty rows); picks,
// pick count and weights written. A failed step on the way down leaves the
// tracklet without picks.
__device__ __forceinline__ void inward_pass(const Bufs& b, const KfConsts& kc, const float* sX, KState& s, int cur,
                                            int last, int64_t seg0, int64_t j, int nr, int tid, unsigned int& st_rows,
                                            unsigned int& st_cand, unsigned int& st_picks) {
    kf_reset(s, kc);
    bool down_ok = true;
    for (int r = cur - 1; r >= last; --r) {
        if (!kf_propagate(s, sX[r + 1], sX[r], kc)) {
            down_ok = false;
            break;
        }
        cur = r;
    }
    if (!down_ok) {
        b.tl_nhits[j] = 0;
        return;
    }
    int nh = 0, miss = 0;
    const bool vec = (nr & 3) == 0;  // 16-byte aligned per-tracklet rows
    PickRing pr{0, 0, 0, 0, 0u};
    SegHdr hn3 = load_hdr(b, seg0 + last);
    for (int r = last; r >= 0; --r) {
        const SegHdr h = hn3;
        hn3 = load_hdr(b, seg0 + max(r - 1, 0));
        if (r != cur) {
            if (!kf_propagate(s, sX[cur], sX[r], kc)) break;
            cur = r;
        }
        ++st_rows;
        Pick pk_;
        if (pick_on_row(b, kc, s, seg0 + r, h, pk_, st_cand)) {
            kf_update(s, pk_.inn);
            pick_store(b, j, nr, nh, pk_.pos, r, vec, pr);
            ++nh;
            miss = 0;
        } else if (++miss >= kc.max_miss) {
            break;
        }
    }
    tracklet_finish(b, j, nr, nh, tid, vec, pr, kc.n_min);
    st_picks += nh;
}

// kSplit = 1: stop at the turn (the state, the row it reached and the last
// row with a cluster are stored) and leave the inward stage to k_tracklet_in
// or k_tracklet_inward.
template <int kSplit>
__global__ __launch_bounds__(256) void k_tracklet(Bufs b, int remap) {
    const DevConsts& K = *b.K;
    const int nr = K.n_rows;
    const KfConsts kc = kf_consts(K);
    const int stats = K.stats;
    __shared__ float sX[kMaxRows];
    kf_load_rows(sX, K);
    const int64_t base = (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;  // never hit: N/3 bound
    if (blockIdx.x == 0 && threadIdx.x < 8) b.ctr->tlq[threadIdx.x] = 0u;  // queues of k_tracklet_in
    unsigned int st_chain = 0, st_rows = 0, st_cand = 0, st_picks = 0;  // per lane: 32 bits suffice
    // logical workgroup (seeds are ordered by instance): with the XCD
    // renumbering over the workgroups that have seeds, each XCD follows the
    // seeds of about one eighth of the instances
    int64_t lg = blockIdx.x, period = gridDim.x;
    if (remap && gridDim.x >= 8) {
        const int64_t active = (cnt + blockDim.x - 1) / blockDim.x;
        period = min((active + 7) / 8 * 8, (int64_t)(gridDim.x & ~7u));
        lg = blockIdx.x < period ? xcd_logical(blockIdx.x, period) : cnt;  // past the period: no seeds
    }
    for (int64_t k = lg * blockDim.x + threadIdx.x; k < cnt; k += period * blockDim.x) {
        const int64_t j = base + k;
        const int32_t pos0 = b.starts[j];
        const int32_t inst = b.start_inst[j];
        const int tid = (int)(j - lower_bound_inst(b.start_inst, base, base + cnt, inst));
        b.tl_tid[j] = tid;
        b.tl_nhits[j] = 0;
        b.tl_row[j] = -1;
        if (tid >= (1 << 20)) {
            raise_err(b.ctr, ERR_TID_CAP);
            continue;
        }
        const int64_t seg0 = (int64_t)inst * nr;
        const int r0 = row_of(b.row_start, seg0, nr, pos0);
        // walk the chain once, keeping its positions in the tracklet's pick
        // buffer (overwritten by stage 3) so that later reads do not chase links
        int32_t* chain = b.tl_pick_pos + j * nr;
        int L = 1;
        int32_t pe = pos0;
        chain[0] = pos0;
        while (b.upc[pe] >= 0) {
            pe = b.upc[pe];
            chain[L++] = pe;
        }
        const int m = (L - 1) / 2;
        const int32_t pm = chain[m];
        KState s;
        const float2 c0 = b.yz[pos0], cm = b.yz[pm], ce = b.yz[pe];
        const bool seeded = seed_from_chain(K, sX[r0], c0.x, c0.y, sX[r0 + m], cm.x, sX[r0 + L - 1], ce.x, ce.y, s);
        int cur = r0, last = r0, miss = 0;
        bool ok = seeded;
        int nh = 0;
        if (ok) {
            // stages 1 and 2 in one outward loop: rows of the chain take the
            // chain's hit, rows beyond it pick a cluster. Each lane runs the
            // same operations in the same order as two separate loops would,
            // but a wave no longer waits for its longest chain and then again
            // for its longest outward pick run: it waits for its longest sum.
            st_chain += L;
            // two-deep prefetch along the chain: the coordinates of the next
            // hit and the position of the one after are in flight
            float2 cn = c0;
            int32_t pn = L > 2 ? chain[2] : pos0;
            {
                const Innov n = kf_innovation(s, cn.x, cn.y, kc);
                if (L > 1) cn = b.yz[chain[1]];
                kf_update(s, n);
            }
            const int rc = r0 + L;  // first row after the chain
            // a pick row's grid header does not depend on the state: it is
            // loaded one row ahead so that its latency hides behind the propagation
            SegHdr hn = load_hdr(b, seg0 + min(r0 + 1, nr - 1));
            for (int r = r0 + 1; r < nr && miss < kc.max_miss; ++r) {
                const bool in_chain = r < rc;
                const SegHdr h = hn;
                if (r + 1 >= rc) hn = load_hdr(b, seg0 + min(r + 1, nr - 1));
                if (!kf_propagate(s, sX[r - 1], sX[r], kc)) {
                    ok = ok && !in_chain;  // a failed step inside the chain voids the tracklet
                    break;
                }
                cur = r;
                Innov inn;
                bool have;
                if (in_chain) {
                    const float2 cp = cn;
                    const int i = r - r0;
                    if (i + 1 < L) {
                        cn = b.yz[pn];
                        if (i + 2 < L) pn = chain[i + 2];
                    }
                    inn = kf_innovation(s, cp.x, cp.y, kc);
                    have = true;
                    last = r;
                } else {
                    ++st_rows;
                    Pick pk_;
                    have = pick_on_row(b, kc, s, seg0 + r, h, pk_, st_cand);
                    inn = pk_.inn;
                    if (have) {
                        last = r;
                        miss = 0;
                    } else {
                        ++miss;
                    }
                }
                if (have) kf_update(s, inn);
            }
        }
        if (ok) {
            // the state at the end of the outward following is the
            // tracklet's output: the refit starts from it
            float* o = b.tl_state + j * 20;
#pragma unroll
            for (int q = 0; q < 5; ++q) o[q] = s.p[q];
#pragma unroll
            for (int q = 0; q < 15; ++q) o[5 + q] = s.C[q];
            b.tl_row[j] = cur;
            if (kSplit) b.tl_last[j] = last;
            if (!kSplit) {
                // turn, stage 3: the operations of inward_pass, written out here
                // (called, it needs 7 more VGPRs here: 2 waves per SIMD instead of 3)
                kf_reset(s, kc);
                bool down_ok = true;
                for (int r = cur - 1; r >= last; --r) {
                    if (!kf_propagate(s, sX[r + 1], sX[r], kc)) {
                        down_ok = false;
                        break;
                    }
                    cur = r;
                }
                if (down_ok) {
                    miss = 0;
                    const bool vec = (nr & 3) == 0;  // 16-byte aligned per-tracklet rows
                    PickRing pr{0, 0, 0, 0, 0u};
                    SegHdr hn3 = load_hdr(b, seg0 + last);
                    for (int r = last; r >= 0; --r) {
                        const SegHdr h = hn3;
                        hn3 = load_hdr(b, seg0 + max(r - 1, 0));
                        if (r != cur) {
                            if (!kf_propagate(s, sX[cur], sX[r], kc)) break;
                            cur = r;
                        }
                        ++st_rows;
                        Pick pk_;
                        if (pick_on_row(b, kc, s, seg0 + r, h, pk_, st_cand)) {
                            kf_update(s, pk_.inn);
                            pick_store(b, j, nr, nh, pk_.pos, r, vec, pr);
                            ++nh;
                            miss = 0;
                        } else if (++miss >= kc.max_miss) {
                            break;
                        }
                    }
                    tracklet_finish(b, j, nr, nh, tid, vec, pr, kc.n_min);
                    st_picks += nh;
                    continue;
                }
            }
        }
        b.tl_nhits[j] = nh;
        if (!ok) {
            float* o = b.tl_state + j * 20;
#pragma unroll
            for (int q = 0; q < 20; ++q) o[q] = 0.0f;
        }
    }
    if (stats) {
        stat_add(b.ctr, ST_CHAIN_HITS, st_chain);
        stat_add(b.ctr, ST_TL_ROWS, st_rows);
        stat_add(b.ctr, ST_TL_CAND, st_cand);
        stat_add(b.ctr, ST_TL_PICKS, st_picks);
    }
}

// Order of the inward passes in the split form: within each chunk of
// kOrderChunk consecutive seeds (one instance or a few: the grid stays in
// the XCD's L2), the tracklets by the row their outward following reached,
// highest first, so that the lanes of a wave have inward passes of similar
// length; failed tracklets last. Any order gives the same results (each
// tracklet's pass is its own; weights are an atomic max).
constexpr int kOrderChunk = 1024;

__global__ __launch_bounds__(256) void k_tl_order(Bufs b) {
    __shared__ int hist[kMaxRows + 1];
    const int nr = b.n_rows;
    const int64_t base = (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;
    for (int64_t c0 = (int64_t)blockIdx.x * kOrderChunk; c0 < cnt; c0 += (int64_t)gridDim.x * kOrderChunk) {
        const int n = (int)min((int64_t)kOrderChunk, cnt - c0);
        for (int i = threadIdx.x; i <= nr; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int row = b.tl_row[base + c0 + i];
            atomicAdd(&hist[row >= 0 ? nr - 1 - row : nr], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int run = 0;
            for (int k = 0; k <= nr; ++k) {
                const int v = hist[k];
                hist[k] = run;
                run += v;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int row = b.tl_row[base + c0 + i];
            const int at = atomicAdd(&hist[row >= 0 ? nr - 1 - row : nr], 1);
            b.seed_order[base + c0 + at] = (int32_t)(c0 + i);
        }
        __syncthreads();
    }
}

// The inward passes of the split form, one lane per tracklet in the order of
// k_tl_order (workgroups renumbered per XCD as in k_tracklet).
__global__ __launch_bounds__(256) void k_tracklet_inward(Bufs b, int remap) {
    const DevConsts& K = *b.K;
    const int nr = K.n_rows;
    const KfConsts kc = kf_consts(K);
    const int stats = K.stats;
    __shared__ float sX[kMaxRows];
    kf_load_rows(sX, K);
    const int64_t base = (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;
    unsigned int st_rows = 0, st_cand = 0, st_picks = 0;
    int64_t lg = blockIdx.x, period = gridDim.x;
    if (remap && gridDim.x >= 8) {
        const int64_t active = (cnt + blockDim.x - 1) / blockDim.x;
        period = min((active + 7) / 8 * 8, (int64_t)(gridDim.x & ~7u));
        lg = blockIdx.x < period ? xcd_logical(blockIdx.x, period) : cnt;
    }
    for (int64_t k = lg * blockDim.x + threadIdx.x; k < cnt; k += period * blockDim.x) {
        const int64_t j = base + b.seed_order[base + k];
        const int cur = b.tl_row[j];
        if (cur < 0) continue;
        KState s;
        const float* st = b.tl_state + j * 20;
#pragma unroll
        for (int i = 0; i < 5; ++i) s.p[i] = st[i];
#pragma unroll
        for (int i = 0; i < 15; ++i) s.C[i] = st[5 + i];
        inward_pass(b, kc, sX, s, cur, b.tl_last[j], (int64_t)b.start_inst[j] * nr, j, nr, b.tl_tid[j], st_rows,
                    st_cand, st_picks);
    }
    if (stats) {
        stat_add(b.ctr, ST_TL_ROWS, st_rows);
        stat_add(b.ctr, ST_TL_CAND, st_cand);
        stat_add(b.ctr, ST_TL_PICKS, st_picks);
    }
}

// The inward pass (stage 3) of the tracklets that k_tracklet<1> stopped at the
// turn. Persistent: a lane whose tracklet ends takes the next one at once, so
// that a wave is not held by its longest tracklet. Every lane runs the same
// operations on a tracklet, in the same order, as the single-kernel form.
// The tracklets are split into eight queues of consecutive seeds (seeds are
// ordered by instance); a workgroup drains the queue of its own XCD first
// (workgroups are dispatched to the XCDs round robin), then the others, so an
// XCD's L2 mostly holds the grid of about one eighth of the instances.
__global__ __launch_bounds__(256) void k_tracklet_in(Bufs b) {
    const DevConsts& K = *b.K;
    const int nr = K.n_rows;
    const KfConsts kc = kf_consts(K);
    const int stats = K.stats;
    __shared__ float sX[kMaxRows];
    kf_load_rows(sX, K);
    const int64_t base = (int64_t)(b.ctr->slot[SL_START][1] & 0xFFFFFFFFull);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_START][2] & 0xFFFFFFFFull);
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;
    const bool vec = (nr & 3) == 0;
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned int st_rows = 0, st_cand = 0, st_picks = 0;
    // wave-uniform queue cursor
    int q = (int)(blockIdx.x & 7), tried = 0;
    // lane state: 0 = needs a tracklet, 1 = down to the last row, 2 = inward
    // picking, 3 = the queues are empty, 4 = ended, its picks and weights not
    // yet written. Ended lanes wait until kRefill lanes of the wave are idle:
    // the stores, the weight atomics and the loads of the next tracklets then
    // run once for all of them instead of once per lane.
    constexpr int kRefill = 16;
    int phase = 0;
    int64_t j = 0, seg0 = 0;
    int cur = 0, last = 0, r = 0, miss = 0, nh = 0, tid = 0;
    KState s;
    PickRing pr{0, 0, 0, 0, 0u};
    SegHdr hn3{};
    while (true) {
        const unsigned long long act = __ballot(phase == 1 || phase == 2);
        if (act == 0ull || __popcll(__ballot(phase == 0 || phase == 4)) >= kRefill) {
            if (phase == 4) {
                tracklet_finish(b, j, nr, nh, tid, vec, pr, kc.n_min);
                st_picks += nh;
                phase = 0;
            }
            // idle lanes take the next tracklets of the current queue; a
            // queue found empty moves the whole wave to the next
            unsigned long long need = __ballot(phase == 0);
            while (need != 0ull) {
                if (tried == 8) {
                    if (phase == 0) phase = 3;
                    break;
                }
                const int64_t qlo = (int64_t)q * cnt / 8, qhi = (int64_t)(q + 1) * cnt / 8;
                const int leader = __ffsll((long long)need) - 1;
                unsigned int got = 0u;
                if (lane == leader) got = atomicAdd(&b.ctr->tlq[q], (unsigned int)__popcll(need));
                got = __shfl(got, leader, 64);
                if (qlo + (int64_t)got + __popcll(need) > qhi) {  // the queue ran out while taking
                    q = (q + 1) & 7;
                    ++tried;
                }
                if (phase == 0) {
                    const int64_t k = qlo + (int64_t)got + __popcll(need & below);
                    if (k < qhi) {
                        j = base + k;
                        cur = b.tl_row[j];
                        if (cur >= 0) {  // a tracklet whose outward following ended well
                            const float* st = b.tl_state + j * 20;
#pragma unroll
                            for (int i = 0; i < 5; ++i) s.p[i] = st[i];
#pragma unroll
                            for (int i = 0; i < 15; ++i) s.C[i] = st[5 + i];
                            kf_reset(s, kc);
                            last = b.tl_last[j];
                            tid = b.tl_tid[j];
                            seg0 = (int64_t)b.start_inst[j] * nr;
                            r = cur - 1 >= last ? cur - 1 : last;
                            phase = cur - 1 >= last ? 1 : 2;
                            miss = 0;
                            nh = 0;
                            hn3 = load_hdr(b, seg0 + last);
                        }
                    }
                }
                need = __ballot(phase == 0);
            }
            if (__ballot(phase == 1 || phase == 2) == 0ull) break;
        }
        // one row: propagate (both phases), then pick (inward phase)
        if (phase == 1 || phase == 2) {
            bool end = false;
            if (r != cur) {
                if (!kf_propagate(s, sX[cur], sX[r], kc)) end = true;
                else cur = r;
            }
            if (phase == 1 && !end) {
                if (r == last) phase = 2;  // the inward picking starts on this row
                else --r;
            }
            if (phase == 2 && !end) {
                const SegHdr h = hn3;
                hn3 = load_hdr(b, seg0 + max(r - 1, 0));
                ++st_rows;
                Pick pk_;
                if (pick_on_row(b, kc, s, seg0 + r, h, pk_, st_cand)) {
                    kf_update(s, pk_.inn);
                    pick_store(b, j, nr, nh, pk_.pos, r, vec, pr);
                    ++nh;
                    miss = 0;
                } else if (++miss >= kc.max_miss) {
                    end = true;
                }
                if (--r < 0) end = true;
            }
            // a failed step on the way down leaves the tracklet without picks
            if (end) phase = phase == 2 ? 4 : 0;
        }
    }
    if (stats) {
        stat_add(b.ctr, ST_TL_ROWS, st_rows);
        stat_add(b.ctr, ST_TL_CAND, st_cand);
        stat_add(b.ctr, ST_TL_PICKS, st_picks);
    }
}

// ------------------------------------------------------------------ refit
// One lane per selected tracklet: move to the outermost hit, then three
// passes inward, outward, inward, each after a covariance reset; a hit is
// used iff its predicted chi2 <= chi2_rej.
//
// A wave lasts as long as its longest track, and track lengths vary from ten
// to a few hundred row steps. Each workgroup takes a chunk of consecutive
// tracks (their cluster lists are adjacent in memory). With rank_by_work = 1
// it hands them to its lanes longest first (a rank by an estimate of the row
// steps of the walk and the three passes, plus the updates); with 2 the lanes
// take the tracks of a chunk of kOrderChunk in the order of k_rf_order (the
// same estimate), so that the tracks of one wave have similar lengths. Every
// track is independent and writes its own slots: the assignment changes no
// result. The first is the default; the second pays where few tracks fill
// the GPU and loses a little on dense batches (the lists of a wave's tracks
// are then far apart in memory).
__device__ __forceinline__ int refit_work(const Bufs& b, int64_t si) {
    const int off = b.sel_off[si], n = b.sel_n[si];
    if (n <= 0) return 0;
    const int lo = b.sel_row[off], hi = b.sel_row[off + n - 1];
    return abs(b.tl_row[b.sel_tl[si]] - hi) + 3 * (hi - lo) + 3 * n;
}

// With rank_by_work = 2 the refit reads its tracks in the order this kernel
// writes into seed_order (free once the tracklet stage has run): per chunk of
// kOrderChunk consecutive selected tracks, a counting sort by the work
// estimate (in steps of four, longest first). Order within a bucket follows
// the LDS atomics; every track still writes only its own slots.
constexpr int kRefitBuckets = 512;

__global__ __launch_bounds__(256) void k_rf_order(Bufs b) {
    __shared__ int hist[kRefitBuckets];
    const int64_t base = (int64_t)(b.ctr->slot[SL_SEL][1] >> 32);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_SEL][2] >> 32);
    if (base + cnt > b.cap_sel) cnt = b.cap_sel > base ? b.cap_sel - base : 0;
    if (base + cnt > b.cap_starts) cnt = b.cap_starts > base ? b.cap_starts - base : 0;  // never hit: sel <= starts
    for (int64_t c0 = (int64_t)blockIdx.x * kOrderChunk; c0 < cnt; c0 += (int64_t)gridDim.x * kOrderChunk) {
        const int n = (int)min((int64_t)kOrderChunk, cnt - c0);
        for (int i = threadIdx.x; i < kRefitBuckets; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        int key[kOrderChunk / 256];
#pragma unroll
        for (int u = 0; u < kOrderChunk / 256; ++u) {
            const int i = threadIdx.x + 256 * u;
            key[u] = 0;
            if (i < n) {
                key[u] = kRefitBuckets - 1 - min(refit_work(b, base + c0 + i) >> 2, kRefitBuckets - 1);
                atomicAdd(&hist[key[u]], 1);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int run = 0;
            for (int k = 0; k < kRefitBuckets; ++k) {
                const int v = hist[k];
                hist[k] = run;
                run += v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kOrderChunk / 256; ++u) {
            const int i = threadIdx.x + 256 * u;
            if (i < n) b.seed_order[base + c0 + atomicAdd(&hist[key[u]], 1)] = (int32_t)(c0 + i);
        }
        __syncthreads();
    }
}

// Accept bits in the refit. Bit j of a lane's bitmap stands for the track
// list's entry j - (off & 3) (off = the list's first index in the selected-hit
// arrays), so that four consecutive bits starting at a multiple of four are
// the four mask bytes of one aligned word. A list holds at most one cluster per
// pad row, so n_rows + 3 bits cover it.
__host__ __device__ constexpr int refit_bit_words(int n_rows) { return (n_rows + 3 + 31) >> 5; }

// Bits 0..3 of x moved to bits 0, 8, 16 and 24 (the four shifted copies of a
// 4-bit value do not overlap, so the product has no carries).
__device__ __forceinline__ uint32_t spread4(uint32_t x) { return ((x & 15u) * 0x00204081u) & 0x01010101u; }

__global__ __launch_bounds__(256) void k_refit(Bufs b, int rank_by_work, int remap) {
    const DevConsts& K = *b.K;
    const KfConsts kc = kf_consts(K);
    const int stats = K.stats;
    __shared__ float sX[kMaxRows];
    __shared__ int skey[256];
    __shared__ int sorder[256];
    // [pass][word][lane]: the accept bits of each lane's current track
    extern __shared__ uint32_t rf_bits[];
    const int nbw = refit_bit_words(K.n_rows);
    kf_load_rows(sX, K);
    const int64_t base = (int64_t)(b.ctr->slot[SL_SEL][1] >> 32);
    int64_t cnt = (int64_t)(b.ctr->slot[SL_SEL][2] >> 32);
    if (base + cnt > b.cap_sel) cnt = b.cap_sel > base ? b.cap_sel - base : 0;  // never hit: N/n_min bound
    unsigned int st_rows = 0, st_hits = 0;
    const int nt = blockDim.x, tid = threadIdx.x;
    const int64_t nchunk = (cnt + nt - 1) / nt;
    // in work order (rank_by_work = 2), workgroups renumbered per XCD as in
    // the tracklet kernels: the chunks one XCD runs are consecutive, so the
    // tracks of one sort chunk and their cluster lists share one L2 (in chunk
    // order, the interleaved numbering balances the XCDs better)
    int64_t lg = blockIdx.x, period = gridDim.x;
    if (remap && rank_by_work == 2 && gridDim.x >= 8) {
        period = min((nchunk + 7) / 8 * 8, (int64_t)(gridDim.x & ~7u));
        lg = blockIdx.x < period ? xcd_logical(blockIdx.x, period) : nchunk;  // past the period: no tracks
    }
    for (int64_t chunk = lg; chunk < nchunk; chunk += period) {  // uniform over the workgroup
        const int64_t k0 = chunk * nt;
        int64_t k = k0 + tid;
        if (rank_by_work == 2) {
            if (k < cnt) k = b.seed_order[base + k];
        } else if (rank_by_work) {  // uniform
            k = chunk_item_by_work(skey, sorder, k0, (k0 + tid < cnt) ? refit_work(b, base + k0 + tid) : -1);
        }
        if (k >= cnt) continue;
        const int64_t si = base + k;
        const int32_t tl = b.sel_tl[si];
        const int off = b.sel_off[si], n = b.sel_n[si];
        KState s;
        const float* st = b.tl_state + (int64_t)tl * 20;
#pragma unroll
        for (int q = 0; q < 5; ++q) s.p[q] = st[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) s.C[q] = st[5 + q];
        // y and z are carried as offsets from a reference that moves to each
        // accepted cluster: binary32 residuals are then formed from small values
        float ref_y = s.p[0], ref_z = s.p[1];
        s.p[0] = 0.0f;
        s.p[1] = 0.0f;
        int cur = b.tl_row[tl];
        bool ok = (n > 0);
        const int outer = ok ? (int)b.sel_row[off + n - 1] : 0;
        while (ok && cur != outer) {
            const int nx = cur < outer ? cur + 1 : cur - 1;
            if (!kf_propagate(s, sX[cur], sX[nx], kc)) ok = false;
            else cur = nx;
            ++st_rows;
        }
        // the mask byte of entry i: bit p set iff pass p reached and accepted
        // it; collected as bits and written once after the passes
        const int bsh = off & 3, nbt = (bsh + n + 31) >> 5;
        for (int w = 0; w < 3 * nbw; w += nbw)
            for (int v = 0; v < nbt; ++v) rf_bits[(w + v) * nt + tid] = 0u;
        float chi2sum = 0.0f;
        int nacc = 0;
        for (int pass = 0; pass < 3 && ok; ++pass) {
            kf_reset(s, kc);
            const bool inward = (pass != 1);
            // the next cluster's row and coordinates are loaded one iteration
            // ahead, so no row step waits on memory
            int i_n = inward ? n - 1 : 0;
            int t_n = b.sel_row[off + i_n];
            float2 c_n = b.sel_yz[off + i_n];
            // this pass's bits of one bitmap word, stored when the pass moves
            // to the next word and at its end
            uint32_t bits = 0u;
            int bw = (bsh + i_n) >> 5;
            for (int q = 0; q < n && ok; ++q) {
                const int i = i_n, target = t_n;
                const float2 c = c_n;
                if (q + 1 < n) {
                    i_n = inward ? n - 2 - q : q + 1;
                    t_n = b.sel_row[off + i_n];
                    c_n = b.sel_yz[off + i_n];
                }
                while (cur != target) {
                    const int nx = cur < target ? cur + 1 : cur - 1;
                    if (!kf_propagate(s, sX[cur], sX[nx], kc)) {
                        ok = false;
                        break;
                    }
                    cur = nx;
                    ++st_rows;
                }
                if (!ok) break;
                const float my = c.x, mz = c.y;
                const Innov inn = kf_innovation(s, my - ref_y, mz - ref_z, kc);
                ++st_hits;
                const bool acc = inn.chi2 <= kc.chi2_rej;
                if (acc) {
                    kf_update(s, inn);
                    s.p[0] = s.p[0] + (ref_y - my);
                    s.p[1] = s.p[1] + (ref_z - mz);
                    ref_y = my;
                    ref_z = mz;
                    if (pass == 2) {
                        chi2sum = chi2sum + inn.chi2;
                        ++nacc;
                    }
                }
                const int j = bsh + i;
                if ((j >> 5) != bw) {
                    rf_bits[(pass * nbw + bw) * nt + tid] = bits;
                    bits = 0u;
                    bw = j >> 5;
                }
                bits |= (acc ? 1u : 0u) << (j & 31);
            }
            rf_bits[(pass * nbw + bw) * nt + tid] = bits;  // also after a failed step
            if (pass == 1 && b.keep_merge && ok) {  // the outward pass ends at the outermost cluster
                float* o2 = b.rf_state2 + si * 20;
                o2[0] = ref_y + s.p[0];
                o2[1] = ref_z + s.p[1];
#pragma unroll
                for (int q = 2; q < 5; ++q) o2[q] = s.p[q];
#pragma unroll
                for (int q = 0; q < 15; ++q) o2[5 + q] = s.C[q];
                b.rf_row2[si] = cur;
            }
        }
        {
            // the list's mask bytes, four per aligned word: bits 4k..4k+3 of
            // each pass give the bytes of the word at off - bsh + 4k; words
            // that the list shares with a neighbour are written byte by byte
            const int je = bsh + n;
            uint32_t* const mword = reinterpret_cast<uint32_t*>(b.sel_mask);  // 256-byte aligned
            const int64_t g0 = (int64_t)off - bsh;
            for (int w = 0; w < nbt; ++w) {
                const uint32_t a0 = rf_bits[w * nt + tid], a1 = rf_bits[(nbw + w) * nt + tid],
                               a2 = rf_bits[(2 * nbw + w) * nt + tid];
                for (int k = 0; k < 8; ++k) {
                    const int j = w * 32 + 4 * k;
                    if (j >= je) break;
                    const int sft = 4 * k;
                    const uint32_t v = spread4(a0 >> sft) | (spread4(a1 >> sft) << 1) | (spread4(a2 >> sft) << 2);
                    if (j >= bsh && j + 4 <= je) {
                        mword[(g0 + j) >> 2] = v;
                    } else {
                        for (int t = 0; t < 4; ++t)
                            if (j + t >= bsh && j + t < je) b.sel_mask[g0 + j + t] = (uint8_t)(v >> (8 * t));
                    }
                }
            }
        }
        s.p[0] = ref_y + s.p[0];
        s.p[1] = ref_z + s.p[1];
        float* o = b.rf_state + si * 20;
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q] = s.p[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) o[5 + q] = s.C[q];
        b.rf_chi2[si] = chi2sum;
        b.rf_nacc[si] = nacc;
        b.rf_row[si] = cur;
        b.rf_ok[si] = (ok && nacc >= kc.n_min) ? 1 : 0;
        if (b.o_res && ok && nacc >= kc.n_min) {
            // track-model compression residuals of the clusters the last pass
            // kept: the output parameters carried outward row by row from
            // the output row by the same helix step
            float q[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) q[c] = s.p[c];
            int rc = cur;
            bool okc = true;
            for (int i = 0; i < n; ++i) {
                if (!(b.sel_mask[off + i] & 4)) continue;
                const int r = b.sel_row[off + i];
                while (okc && rc < r) {
                    if (!kf_step_state(q, sX[rc], sX[rc + 1], kc)) okc = false;
                    else ++rc;
                }
                uint32_t packed = 0x80008000u;  // both escaped
                if (okc) {
                    const float2 c = b.sel_yz[off + i];
                    const float qy = __builtin_rintf((c.x - q[0]) * b.res_scale);
                    const float qz = __builtin_rintf((c.y - q[1]) * b.res_scale);
                    const uint32_t uy = (qy >= -32767.0f && qy <= 32767.0f) ? (uint32_t)(uint16_t)(int16_t)qy : 0x8000u;
                    const uint32_t uz = (qz >= -32767.0f && qz <= 32767.0f) ? (uint32_t)(uint16_t)(int16_t)qz : 0x8000u;
                    packed = uy | (uz << 16);
                }
                b.sel_res[off + i] = packed;
            }
        }
    }
    if (stats) {
        stat_add(b.ctr, ST_RF_ROWS, st_rows);
        stat_add(b.ctr, ST_RF_HITS, st_hits);
    }
}

// ------------------------------------------------------------------ finish
// FP64 totals in a fixed order: kFinishParts workgroups each sum a fixed
// contiguous chunk of the tracks (strided per-lane sums, then a fixed tree),
// one workgroup sums the parts by the same tree; it also writes the closing
// entry of the output CSR.
constexpr int kFinishParts = 256;

__device__ __forceinline__ void tree_sum2(double* shc, double* shn) {
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            shc[threadIdx.x] += shc[threadIdx.x + s];
            shn[threadIdx.x] += shn[threadIdx.x + s];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_finish_part(Bufs b) {
    __shared__ double shc[256];
    __shared__ double shn[256];
    const unsigned long long tot = b.ctr->slot[SL_TRK][0];
    const int64_t nt = (int64_t)(tot >> 32);
    const int64_t n = nt < b.cap_tracks ? nt : b.cap_tracks;
    const int64_t chunk = (n + kFinishParts - 1) / kFinishParts;
    const int64_t lo = blockIdx.x * chunk, hi = min(lo + chunk, n);
    double c = 0.0, d = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) {
        c += (double)b.o_chi2[t];
        d += (double)b.o_ndf[t];
    }
    shc[threadIdx.x] = c;
    shn[threadIdx.x] = d;
    __syncthreads();
    tree_sum2(shc, shn);
    if (threadIdx.x == 0) {
        double* part = reinterpret_cast<double*>(b.scan_part);  // free once the scans are done
        part[2 * blockIdx.x] = shc[0];
        part[2 * blockIdx.x + 1] = shn[0];
    }
}

__global__ __launch_bounds__(kFinishParts) void k_finish(Bufs b) {
    __shared__ double shc[kFinishParts];
    __shared__ double shn[kFinishParts];
    const unsigned long long tot = b.ctr->slot[SL_TRK][0];
    const int64_t nt = (int64_t)(tot >> 32);
    const int64_t nh = (int64_t)(tot & 0xFFFFFFFFull);
    const double* part = reinterpret_cast<const double*>(b.scan_part);
    shc[threadIdx.x] = part[2 * threadIdx.x];
    shn[threadIdx.x] = part[2 * threadIdx.x + 1];
    __syncthreads();
    tree_sum2(shc, shn);
    if (threadIdx.x == 0) {
        if (b.o_chi2_total) {
            b.o_chi2_total[0] = shc[0];
            b.o_chi2_total[1] = shn[0];
        }
        if (nt <= b.cap_tracks && nh <= b.cap_hits) b.o_hit_start[nt] = nh;
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_reset_counters(Counters* c) {
    unsigned long long* w = reinterpret_cast<unsigned long long*>(c);
    const int nw = (int)(sizeof(Counters) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;
}

// ------------------------------------------------------------------ device input check
// CSR over (instance, row): row_start[0] = 0, non-decreasing, last entry =
// n_clusters, at most TPCCA_MAX_ROW_CLUSTERS per row (the host check of the
// synchronising forms, done where the data already is).
__global__ void k_check_csr(Bufs b, int64_t n_entries) {
    const int64_t* rs = b.row_start;
    unsigned int bits = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_entries;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = rs[i];
        if (i == 0 && v != 0) bits |= ERR_ARG;
        if (i == n_entries - 1 && v != b.n_clusters) bits |= ERR_ARG;
        if (i + 1 < n_entries) {
            const int64_t d = rs[i + 1] - v;
            if (d < 0) bits |= ERR_ARG;
            else if (d > kLargeRow) bits |= ERR_ROW_CAP;
        }
    }
    if (bits) raise_err(b.ctr, bits | ERR_CSR);
}

// Counts and status of the whole call, left on the device (one thread).
__global__ void k_async_status(Bufs b, int64_t* counts, int32_t* status) {
    if (threadIdx.x != 0) return;
    const unsigned long long tot = b.ctr->slot[SL_TRK][0];
    const int64_t nt = (int64_t)(tot >> 32), nh = (int64_t)(tot & 0xFFFFFFFFull);
    counts[0] = nt;
    counts[1] = nh;
    const unsigned int e = b.ctr->err;
    int32_t s = 0;                                         // TPCCA_OK
    if (e & ERR_ARG) s = 1;                                // TPCCA_E_ARG
    else if (e & (ERR_ROW_CAP | ERR_TID_CAP)) s = 2;       // TPCCA_E_CAPACITY
    else if (e & ERR_SCRATCH) s = 5;                       // TPCCA_E_INTERNAL
    else if ((e & ERR_OUT_CAP) || nt > b.cap_tracks || nh > b.cap_hits) s = 2;
    *status = s;
}

// ------------------------------------------------------------------ exports
__global__ void k_export_grid(Bufs b, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz, float* meta,
                              int64_t nseg) {
    const int64_t N = b.n_clusters;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < N; i += stride) sorted_id[i] = b.sid[i];
    for (int64_t i = i0; i < N + nseg + 1; i += stride) bin_start[i] = b.bin_start[i];
    for (int64_t s = i0; s < nseg; s += stride) {
        const SegHdr h = b.hdr[s];
        ny[s] = h.ny;
        nz[s] = h.nz;
        meta[4 * s] = h.ymin;
        meta[4 * s + 1] = h.zmin;
        meta[4 * s + 2] = h.iy;
        meta[4 * s + 3] = h.iz;
    }
}

__global__ void k_export_links(Bufs b, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < b.n_clusters;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t id = b.sid[p];
        const int32_t u = b.up[p], d = b.dn[p], uc = b.upc[p], dc = b.dnc[p];
        up[id] = u >= 0 ? b.sid[u] : -1;
        dn[id] = d >= 0 ? b.sid[d] : -1;
        upc[id] = uc >= 0 ? b.sid[uc] : -1;
        dnc[id] = dc >= 0 ? b.sid[dc] : -1;
    }
}

__global__ void k_export_tracklets(Bufs b, int64_t ns, int32_t* start_hit, int32_t* start_inst, int32_t* start_tid,
                                   int32_t* nhits, int32_t* rowhit, float* state, int32_t* state_row,
                                   uint32_t* weight) {
    const int nr = b.K->n_rows;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t j = i0; j < ns; j += stride) {
        start_hit[j] = b.sid[b.starts[j]];
        start_inst[j] = b.start_inst[j];
        start_tid[j] = b.tl_tid[j];
        const int nh = b.tl_nhits[j];
        nhits[j] = nh;
        for (int r = 0; r < nr; ++r) rowhit[j * nr + r] = -1;
        for (int k = 0; k < nh; ++k) rowhit[j * nr + b.tl_pick_row[j * nr + k]] = b.sid[b.tl_pick_pos[j * nr + k]];
        for (int q = 0; q < 20; ++q) state[j * 20 + q] = b.tl_state[j * 20 + q];
        state_row[j] = b.tl_row[j];
    }
    for (int64_t p = i0; p < b.n_clusters; p += stride) weight[b.sid[p]] = b.weight[p];
}

__global__ void k_export_selected(Bufs b, int64_t nsel, int32_t* sel_tl, int64_t* hit_start, int32_t* hit_id,
                                  uint8_t* mask, int32_t* status) {
    for (int64_t si = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; si < nsel; si += (int64_t)gridDim.x * blockDim.x) {
        sel_tl[si] = b.sel_tl[si];
        const int off = b.sel_off[si], n = b.sel_n[si];
        hit_start[si] = off;
        if (si == nsel - 1) hit_start[nsel] = off + n;
        for (int i = 0; i < n; ++i) {
            hit_id[off + i] = b.sid[b.sel_pos[off + i]];
            mask[off + i] = b.sel_mask[off + i];
        }
        status[si] = b.rf_ok[si];
    }
}

__global__ void k_fp32_selfcheck(const float* a, const float* bb, float* od, float* os, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        od[i] = a[i] / bb[i];
        os[i] = __builtin_sqrtf(__builtin_fabsf(a[i]));
    }
}

// Counts the binary32 bit patterns x in [first, last] for which the helix
// step's square root differs from sqrtf (two NaN results count as equal).
// Lanes add to the counter only for a difference.
__global__ void k_sqrt_step_check(uint32_t first, uint32_t last, unsigned long long* count) {
    const uint64_t n = (uint64_t)last - first + 1;
    unsigned long long bad = 0;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const float x = __uint_as_float(first + (uint32_t)k);
        const float r = sqrt_step(x), e = __builtin_sqrtf(x);
        const bool same = __float_as_uint(r) == __float_as_uint(e) || (r != r && e != e);
        bad += same ? 0ull : 1ull;
    }
    if (bad != 0ull) atomicAdd(count, bad);
}

inline int grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <class Op>
void launch_scan(const Op& op, const Bufs& b, int slot, int block, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_part<Op>, dim3(kScanBlocks), dim3(block), 0, st, op, b.scan_part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlocks), 0, st, b.scan_part, b.ctr, slot);
    hipLaunchKernelGGL(k_scan_apply<Op>, dim3(kScanBlocks), dim3(block), 0, st, op, (const unsigned long long*)b.scan_part,
                       (const Counters*)b.ctr, slot);
}

}  // namespace

// ------------------------------------------------------------------ launchers
void enqueue_reset(const Bufs& b, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, st, b.ctr);
}

void enqueue_weights_clear(const Bufs& b, int64_t c0, int64_t c1, hipStream_t st) {
    if (c1 > c0)
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(c1 - c0, 256, 4096)), dim3(256), 0, st, b.weight + c0, c1 - c0, 0u);
}

void enqueue_native_local(const Bufs& b, int64_t nseg, float* y, float* z, hipStream_t st) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_native_local, dim3((unsigned)(nseg < 65536 ? nseg : 65536)), dim3(256), 0, st, b, nseg, y, z);
}

void enqueue_grid(const Bufs& b, int i0, int i1, int max_row, hipStream_t st) {
    const int64_t seg0 = (int64_t)i0 * b.n_rows, nseg = (int64_t)(i1 - i0) * b.n_rows;
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_grid<kSmallRow>, dim3((unsigned)nseg), dim3(256), 0, st, b, seg0);
    // the large-row variant only when a row may exceed the small one's capacity
    if (max_row > kSmallRow)
        hipLaunchKernelGGL(k_grid<kLargeRow>, dim3((unsigned)nseg), dim3(256), 0, st, b, seg0);
}

void enqueue_links(const Bufs& b, const Launch& L, int i0, int i1, int max_row, hipStream_t st) {
    const int64_t seg0 = (int64_t)i0 * b.n_rows, nseg = (int64_t)(i1 - i0) * b.n_rows;
    if (nseg <= 0) return;
    // LDS: two rows of (y, z) and two bin-start arrays (bins <= clusters), for
    // rows of up to `cap` clusters (64 KB per workgroup); a workgroup whose
    // neighbour rows are larger reads them from global memory
    const int cap_lds = (int)((64 * 1024 - 2 * sizeof(int32_t)) / (2 * sizeof(float2) + 2 * sizeof(int32_t)));
    const int cap = max_row < 1 ? 1 : min(max_row, cap_lds);
    const size_t bytes = (size_t)cap * 2 * sizeof(float2) + (size_t)(cap + 1) * 2 * sizeof(int32_t);
    const int64_t grid = L.xcd_remap ? (nseg + 7) / 8 * 8 : nseg;
    if (max_row <= kDenseRow) {
        hipLaunchKernelGGL(k_links<kNbKeep>, dim3((unsigned)grid), dim3(L.block_links), bytes, st, b, seg0, nseg, cap,
                           L.xcd_remap, 0);
        return;
    }
    hipLaunchKernelGGL(k_links<kNbKeep>, dim3((unsigned)grid), dim3(L.block_links), bytes, st, b, seg0, nseg, cap,
                       L.xcd_remap, 1);
    hipLaunchKernelGGL(k_links<kNbKeepDense>, dim3((unsigned)grid), dim3(L.block_links), bytes, st, b, seg0, nseg,
                       cap, L.xcd_remap, 2);
}

void enqueue_clean_starts(const Bufs& b, const Launch& L, int i0, int i1, int64_t c0, int64_t c1, hipStream_t st) {
    if (c1 > c0) hipLaunchKernelGGL(k_clean, dim3(grid_for(c1 - c0, 256, 8192)), dim3(256), 0, st, b, c0, c1);
    StartOp op{b, c0, c1, i0, i1};
    launch_scan(op, b, SL_START, L.block_scan, st);
}

void enqueue_tracklets(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st) {
    const dim3 grid(grid_for(bound, L.block_tracklet, 16384));
    if (L.inward_wgs > 0) {
        hipLaunchKernelGGL(k_tracklet<1>, grid, dim3(L.block_tracklet), 0, st, b, L.xcd_remap);
        hipLaunchKernelGGL(k_tracklet_in, dim3(L.inward_wgs), dim3(L.block_tracklet), 0, st, b);
    } else if (L.inward_sort) {
        hipLaunchKernelGGL(k_tracklet<1>, grid, dim3(L.block_tracklet), 0, st, b, L.xcd_remap);
        hipLaunchKernelGGL(k_tl_order, dim3(grid_for(bound, kOrderChunk, 4096)), dim3(256), 0, st, b);
        hipLaunchKernelGGL(k_tracklet_inward, grid, dim3(L.block_tracklet), 0, st, b, L.xcd_remap);
    } else {
        hipLaunchKernelGGL(k_tracklet<0>, grid, dim3(L.block_tracklet), 0, st, b, L.xcd_remap);
    }
}

void enqueue_select(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st) {
    hipLaunchKernelGGL(k_own, dim3(grid_for(bound * 64, 256, 16384)), dim3(256), 0, st, b);
    SelectOp op{b};
    launch_scan(op, b, SL_SEL, L.block_scan, st);
    hipLaunchKernelGGL(k_sel_fill, dim3(grid_for(bound * 64, 256, 16384)), dim3(256), 0, st, b);
}

void enqueue_refit(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st) {
    if (L.sort_seeds == 2)
        hipLaunchKernelGGL(k_rf_order, dim3(grid_for(bound, kOrderChunk, 4096)), dim3(256), 0, st, b);
    // three accept bitmaps per lane (at most 3 x 9 words x 256 lanes = 27 KB)
    const size_t bits = (size_t)3 * refit_bit_words(b.n_rows) * L.block_refit * sizeof(uint32_t);
    hipLaunchKernelGGL(k_refit, dim3(grid_for(bound, L.block_refit, 16384)), dim3(L.block_refit), bits, st, b,
                       L.sort_seeds, L.xcd_remap);
}

void enqueue_write(const Bufs& b, const Launch& L, int64_t bound, hipStream_t st) {
    TrackOp op{b};
    launch_scan(op, b, SL_TRK, L.block_scan, st);
    hipLaunchKernelGGL(k_trk_fill, dim3(grid_for(bound * 64, 256, 16384)), dim3(256), 0, st, b);
}

void enqueue_finish(const Bufs& b, hipStream_t st) {
    static_assert(2 * kFinishParts <= kScanBlocks, "finish parts live in the scan scratch");
    hipLaunchKernelGGL(k_finish_part, dim3(kFinishParts), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kFinishParts), 0, st, b);
}

void enqueue_check_csr(const Bufs& b, hipStream_t st) {
    const int64_t n = (int64_t)b.n_inst * b.n_rows + 1;
    hipLaunchKernelGGL(k_check_csr, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, b, n);
}

void enqueue_async_status(const Bufs& b, int64_t* counts, int32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(k_async_status, dim3(1), dim3(64), 0, st, b, counts, status);
}

void enqueue_export_grid(const Bufs& b, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz,
                         float* meta, int64_t nseg, hipStream_t st) {
    hipLaunchKernelGGL(k_export_grid, dim3(grid_for(b.n_clusters + nseg + 1, 256, 8192)), dim3(256), 0, st, b,
                       sorted_id, bin_start, ny, nz, meta, nseg);
}

void enqueue_export_links(const Bufs& b, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc, hipStream_t st) {
    hipLaunchKernelGGL(k_export_links, dim3(grid_for(b.n_clusters, 256, 8192)), dim3(256), 0, st, b, up, dn, upc, dnc);
}

void enqueue_export_tracklets(const Bufs& b, int64_t n_starts, int32_t* start_hit, int32_t* start_inst,
                              int32_t* start_tid, int32_t* nhits, int32_t* rowhit, float* state,
                              int32_t* state_row, uint32_t* weight, hipStream_t st) {
    const int64_t n = n_starts > b.n_clusters ? n_starts : b.n_clusters;
    hipLaunchKernelGGL(k_export_tracklets, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, b, n_starts, start_hit,
                       start_inst, start_tid, nhits, rowhit, state, state_row, weight);
}

void enqueue_export_selected(const Bufs& b, int64_t n_sel, int32_t* sel_tl, int64_t* hit_start, int32_t* hit_id,
                             uint8_t* mask, int32_t* status, hipStream_t st) {
    if (n_sel <= 0) return;
    hipLaunchKernelGGL(k_export_selected, dim3(grid_for(n_sel, 256, 8192)), dim3(256), 0, st, b, n_sel, sel_tl,
                       hit_start, hit_id, mask, status);
}

void enqueue_sqrt_step_check(uint32_t first, uint32_t last, unsigned long long* count, hipStream_t st) {
    hipLaunchKernelGGL(k_sqrt_step_check, dim3(grid_for((int64_t)last - first + 1, 256, 16384)), dim3(256), 0, st, first,
                       last, count);
}

void enqueue_fp32_selfcheck(const float* a, const float* bb, float* od, float* os, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fp32_selfcheck, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, a, bb, od, os, n);
}

}  // namespace tpcca
