// Differentiable refit (gfx950): the chi2 of the three-pass Kalman refit with
// frozen accept masks, as a function of each track's start state and of a
// smooth space-charge correction map applied to the clusters between seeding
// and fitting (the paper applies such calibration corrections there,
// Sections 1 and 4), and its hand-written reverse-mode adjoint.
//
// Forward (binary32, the refit's own arithmetic and operation order): one lane
// per track. Every operation (row step, covariance reset, cluster update)
// records its inputs on a tape in HBM: the covariance before it and its
// operands, 76 bytes, stored structure-of-arrays over the tracks of a batch so
// that a wave's stores coalesce. A 1e5-track set needs ~8 GB of tape, which
// the 288 GB of HBM3E hold without recomputation; a set above the tape budget
// is recomputed batch by batch in the backward call.
// Backward: each lane reads its tape last operation first, prefetching one
// operation ahead, and applies the adjoints of the recorded operations in
// binary32 or binary64.
//
// Map: components (delta r, delta r*phi, delta z), each a tricubic uniform
// B-spline with 16 x 16 (periodic in phi) x 32 coefficients [comp][r][phi][z],
// knots r_k = 84 + (k - 1) 168/13, phi_k = k 2 pi/16, z_k = -252 + (k - 1) 504/29.
// A cluster on pad-row plane x with local (y, z) is corrected inside that
// plane: y' = y - (dr y + drphi x) / r, z' = z - dz, with r = sqrt(x^2 + y^2)
// and the map taken at (r, alpha + atan2(y, x), z).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adjoint.h"

#pragma clang fp contract(off)

namespace tpcca {

namespace {

constexpr int kMapNr = 16, kMapNphi = 16, kMapNz = 32;

// ------------------------------------------------------------ map
__device__ __forceinline__ void bspline_basis(float t, float w[4]) {
    const float t2 = t * t, t3 = t2 * t, s = 1.0f - t;
    w[0] = (s * s * s) * (1.0f / 6.0f);
    w[1] = ((3.0f * t3 - 6.0f * t2) + 4.0f) * (1.0f / 6.0f);
    w[2] = (((-3.0f * t3 + 3.0f * t2) + 3.0f * t) + 1.0f) * (1.0f / 6.0f);
    w[3] = t3 * (1.0f / 6.0f);
}

struct MapCell {
    int ir, iphi, iz;  // first of the four coefficients along each axis
    float wr[4], wphi[4], wz[4];
};

__device__ __forceinline__ MapCell map_cell(float r, float phi, float z) {
    const float pi2 = 6.2831853071795865f;
    MapCell c;
    float ur = 1.0f + (r - 84.0f) * (13.0f / 168.0f);
    float uz = 1.0f + (z + 252.0f) * (29.0f / 504.0f);
    ur = fminf(fmaxf(ur, 1.0f), 13.999999f);
    uz = fminf(fmaxf(uz, 1.0f), 29.999998f);
    float ph = fmodf(phi, pi2);
    if (ph < 0.0f) ph += pi2;
    float up = ph * ((float)kMapNphi / pi2);
    if (!(up < (float)kMapNphi)) up = 0.0f;
    if (!(up >= 0.0f)) up = 0.0f;
    const int ir = (int)ur, iz = (int)uz, ip = (int)up;
    bspline_basis(ur - (float)ir, c.wr);
    bspline_basis(uz - (float)iz, c.wz);
    bspline_basis(up - (float)ip, c.wphi);
    c.ir = ir - 1;
    c.iz = iz - 1;
    c.iphi = ip - 1;
    return c;
}

__device__ __forceinline__ int map_index(int comp, int ir, int iphi, int iz) {
    iphi = (iphi + kMapNphi) % kMapNphi;
    return ((comp * kMapNr + ir) * kMapNphi + iphi) * kMapNz + iz;
}

struct ClusterGeo {
    float x, r, phi;
};

__device__ __forceinline__ ClusterGeo cluster_geo(const AdjBufs& a, int row, int32_t inst, float y) {
    const DevConsts& K = *a.K;
    ClusterGeo g;
    g.x = K.X[row];
    g.r = __builtin_sqrtf(g.x * g.x + y * y);
    const int sec = a.inst_sector[inst];
    g.phi = K.alpha[((sec % 18) + 18) % 18] + atan2f(y, g.x);
    return g;
}

// The cluster (y, z) of geometry g moved by the map: (delta r, delta r*phi,
// delta z) at (r, phi, z), applied inside the pad-row plane.
__device__ __forceinline__ void map_correct(const float* coef, const ClusterGeo& g, float& y, float& z) {
    const MapCell c = map_cell(g.r, g.phi, z);
    float d[3];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        float acc = 0.0f;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const float wij = c.wr[i] * c.wphi[j];
                const float* cf = coef + map_index(comp, c.ir + i, c.iphi + j, c.iz);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc = acc + (wij * c.wz[e]) * cf[e];
            }
        d[comp] = acc;
    }
    y = y - (d[0] * y + d[1] * g.x) / g.r;
    z = z - d[2];
}

// ------------------------------------------------------------ tape
enum : int { OP_PROP = 1, OP_RESET = 2, OP_UPD = 3 };

__device__ __forceinline__ uint32_t op_word(int kind, int pass, int from, int to, int hit) {
    return (uint32_t)kind | ((uint32_t)pass << 2) | ((uint32_t)from << 4) | ((uint32_t)to << 12) |
           ((uint32_t)hit << 20);
}

// ------------------------------------------------------------ dual numbers
// value and derivatives with respect to (sin phi, tan lambda, q/pT) before a row step
template <class A>
struct D3 {
    A v, d0, d1, d2;
};
template <class A>
__device__ __forceinline__ D3<A> dc(A v) {
    return D3<A>{v, A(0), A(0), A(0)};
}
template <class A>
__device__ __forceinline__ D3<A> operator+(D3<A> a, D3<A> b) {
    return D3<A>{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2};
}
template <class A>
__device__ __forceinline__ D3<A> operator-(D3<A> a, D3<A> b) {
    return D3<A>{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2};
}
template <class A>
__device__ __forceinline__ D3<A> operator*(D3<A> a, D3<A> b) {
    return D3<A>{a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
template <class A>
__device__ __forceinline__ D3<A> operator*(D3<A> a, A k) {
    return D3<A>{a.v * k, a.d0 * k, a.d1 * k, a.d2 * k};
}
// The reverse sweep needs derivatives, not the forward's rounding: in binary32
// it divides and takes square roots with the hardware reciprocal and square
// root (about 1 ulp) instead of the correctly rounded sequences.
__device__ __forceinline__ float rcp_a(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_a(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_a(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_a(double x) { return sqrt(x); }

template <class A>
__device__ __forceinline__ D3<A> operator/(D3<A> a, D3<A> b) {
    const A ib = rcp_a(b.v), q = a.v * ib;
    return D3<A>{q, (a.d0 - q * b.d0) * ib, (a.d1 - q * b.d1) * ib, (a.d2 - q * b.d2) * ib};
}
template <class A>
__device__ __forceinline__ D3<A> dsqrt(D3<A> a) {
    const A s = sqrt_a(a.v), h = A(0.5) * rcp_a(s);
    return D3<A>{s, a.d0 * h, a.d1 * h, a.d2 * h};
}

// asin(u)/u and its derivative, the same truncated Maclaurin series as the refit
template <class A>
__device__ __forceinline__ D3<A> g_series(D3<A> u) {
    const D3<A> w = u * u;
    D3<A> h = dc(A(231.0 / 13312.0));
    h = dc(A(63.0 / 2816.0)) + w * h;
    h = dc(A(35.0 / 1152.0)) + w * h;
    h = dc(A(5.0 / 112.0)) + w * h;
    h = dc(A(3.0 / 40.0)) + w * h;
    h = dc(A(1.0 / 6.0)) + w * h;
    return dc(A(1)) + w * h;
}
template <class A>
__device__ __forceinline__ D3<A> gp_series(D3<A> u) {
    const D3<A> w = u * u;
    D3<A> h = dc(A(2772.0 / 13312.0));
    h = dc(A(630.0 / 2816.0)) + w * h;
    h = dc(A(280.0 / 1152.0)) + w * h;
    h = dc(A(30.0 / 112.0)) + w * h;
    h = dc(A(12.0 / 40.0)) + w * h;
    h = dc(A(2.0 / 6.0)) + w * h;
    return u * h;
}

// The variable Jacobian entries of one row step, F02, F04, F12, F13, F14, F24,
// with their derivatives with respect to (sin phi, tan lambda, q/pT).
template <class A>
__device__ __forceinline__ void step_jacobian(A s1v, A tv, A qv, A dx, A kB, D3<A> f[6]) {
    const D3<A> s1{s1v, A(1), A(0), A(0)}, t{tv, A(0), A(1), A(0)}, q{qv, A(0), A(0), A(1)};
    const D3<A> one = dc(A(1));
    const D3<A> kq = q * kB;
    const D3<A> s2 = s1 + kq * dx;
    const D3<A> c1 = dsqrt(one - s1 * s1), c2 = dsqrt(one - s2 * s2);
    const D3<A> tt = (s1 + s2) / (c1 + c2);
    const D3<A> w = one + tt * tt;
    const D3<A> lc = dsqrt(w) * dx;
    const D3<A> u = (kq * lc) * A(0.5);
    const D3<A> g = g_series(u), gp = gp_series(u);
    f[0] = ((w * dx) * (one / c1 + one / c2)) * A(0.5);
    f[1] = ((w * dx) * (dc(kB * dx) / c2)) * A(0.5);
    f[2] = t * ((tt * dx) / (c1 * c2));
    f[3] = lc * g;
    const D3<A> dlc = ((lc * (kB * dx)) * tt) / (c2 * A(2));
    const D3<A> du = (lc * kB + kq * dlc) * A(0.5);
    f[4] = t * (dlc * g + (lc * gp) * du);
    f[5] = dc(kB * dx);
}

// v <- F^T v for the row-step Jacobian F (identity plus the six entries)
template <class A>
__device__ __forceinline__ void ft_apply(A v[5], const A f[6]) {
    const A v0 = v[0], v1 = v[1], v2 = v[2];
    v[2] = v2 + f[0] * v0 + f[2] * v1;
    v[3] = v[3] + f[3] * v1;
    v[4] = v[4] + f[1] * v0 + f[4] * v1 + f[5] * v2;
}

// v <- F v
template <class A>
__device__ __forceinline__ void f_apply(A v[5], const A f[6]) {
    v[0] = v[0] + f[0] * v[2] + f[1] * v[4];
    v[1] = v[1] + f[2] * v[2] + f[3] * v[3] + f[4] * v[4];
    v[2] = v[2] + f[5] * v[4];
}

// Adjoint of a row step with input (sin phi, tan lambda, q/pT) and covariance
// C: pbar <- F^T pbar + 2 sum_bc M_bc dF_bc/dp (M = Cbar F C), Cbar <- F^T Cbar F.
template <class A, class KC>
__device__ __forceinline__ void adj_prop(const float C[15], float s1, float t, float q, float dx, A pb[5], A Cb[15],
                                         const KC& K) {
    D3<A> fd[6];
    step_jacobian<A>(A(s1), A(t), A(q), A(dx), A(K.kB), fd);
    A f[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) f[e] = fd[e].v;
    // columns 2..4 of B = F C
    A B[3][5];  // B[c - 2][k]
#pragma unroll
    for (int c = 2; c < 5; ++c) {
        A col[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) col[k] = A(C[pk(k, c)]);
        f_apply(col, f);
#pragma unroll
        for (int k = 0; k < 5; ++k) B[c - 2][k] = col[k];
    }
    // M_bc = sum_k Cbar_bk B_kc at the six variable entries
    auto M = [&](int b, int c) {
        A acc = A(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) acc = acc + Cb[pk(b, k)] * B[c - 2][k];
        return acc;
    };
    const A m02 = M(0, 2), m04 = M(0, 4), m12 = M(1, 2), m13 = M(1, 3), m14 = M(1, 4), m24 = M(2, 4);
    const A g0 = m02 * fd[0].d0 + m04 * fd[1].d0 + m12 * fd[2].d0 + m13 * fd[3].d0 + m14 * fd[4].d0 + m24 * fd[5].d0;
    const A g1 = m02 * fd[0].d1 + m04 * fd[1].d1 + m12 * fd[2].d1 + m13 * fd[3].d1 + m14 * fd[4].d1 + m24 * fd[5].d1;
    const A g2 = m02 * fd[0].d2 + m04 * fd[1].d2 + m12 * fd[2].d2 + m13 * fd[3].d2 + m14 * fd[4].d2 + m24 * fd[5].d2;
    ft_apply(pb, f);
    pb[2] = pb[2] + A(2) * g0;
    pb[3] = pb[3] + A(2) * g1;
    pb[4] = pb[4] + A(2) * g2;
    // Cbar <- F^T Cbar F: F^T on every column, then on every row
    A X[5][5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        A col[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) col[k] = Cb[pk(k, j)];
        ft_apply(col, f);
#pragma unroll
        for (int k = 0; k < 5; ++k) X[k][j] = col[k];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        ft_apply(X[i], f);
#pragma unroll
        for (int j = 0; j <= i; ++j) Cb[pk(i, j)] = X[i][j];
    }
}

// Adjoint of a covariance reset: variances scaled, correlations dropped.
template <class A, class KC>
__device__ __forceinline__ void adj_reset(A Cb[15], const KC& K) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) Cb[pk(i, j)] = A(0);
        Cb[pk(i, i)] = Cb[pk(i, i)] * A(K.cov_reset);
    }
}

// Adjoint of a cluster update with covariance C and residual r = m - (y, z):
// with G = C H^T (columns 0, 1 of C), A = S^-1, S = H C H^T + V,
// p+ = p + G A r, C+ = C - G A G^T, chi2 = r^T A r (weight cb):
//   rbar = A (G^T pbar+ + 2 cb r)      -> measurement, and -H^T rbar -> pbar
//   Gbar = pbar+ (A r)^T - 2 Cbar+ G A
//   Abar = (G^T pbar+) r^T - G^T Cbar+ G + cb r r^T,  Sbar = -A Abar A
//   Cbar = Cbar+ + sym(H^T Sbar H) + sym(Gbar H)
template <class A, class KC>
__device__ __forceinline__ void adj_upd(const float C[15], float r0f, float r1f, A pb[5], A Cb[15], A& mb0, A& mb1,
                                        A cb, const KC& K) {
    const A r0 = A(r0f), r1 = A(r1f);
    const A s00 = A(C[0]) + A(K.vy), s01 = A(C[1]), s11 = A(C[2]) + A(K.vz);
    const A idet = rcp_a(s00 * s11 - s01 * s01);
    const A a00 = s11 * idet, a01 = -s01 * idet, a11 = s00 * idet;
    A G0[5], G1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        G0[i] = A(C[pk(i, 0)]);
        G1[i] = A(C[pk(i, 1)]);
    }
    const A v0 = a00 * r0 + a01 * r1, v1 = a01 * r0 + a11 * r1;
    A gp0 = A(0), gp1 = A(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        gp0 = gp0 + G0[i] * pb[i];
        gp1 = gp1 + G1[i] * pb[i];
    }
    const A b0 = gp0 + A(2) * cb * r0, b1 = gp1 + A(2) * cb * r1;
    const A rb0 = a00 * b0 + a01 * b1, rb1 = a01 * b0 + a11 * b1;
    mb0 = mb0 + rb0;
    mb1 = mb1 + rb1;
    A CG0[5], CG1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        A x0 = A(0), x1 = A(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            x0 = x0 + Cb[pk(i, k)] * G0[k];
            x1 = x1 + Cb[pk(i, k)] * G1[k];
        }
        CG0[i] = x0;
        CG1[i] = x1;
    }
    A Gb0[5], Gb1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Gb0[i] = pb[i] * v0 - A(2) * (CG0[i] * a00 + CG1[i] * a01);
        Gb1[i] = pb[i] * v1 - A(2) * (CG0[i] * a01 + CG1[i] * a11);
    }
    A q00 = A(0), q01 = A(0), q10 = A(0), q11 = A(0);  // G^T Cbar+ G
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        q00 = q00 + G0[i] * CG0[i];
        q01 = q01 + G0[i] * CG1[i];
        q10 = q10 + G1[i] * CG0[i];
        q11 = q11 + G1[i] * CG1[i];
    }
    const A ab00 = gp0 * r0 - q00 + cb * r0 * r0;
    const A ab01 = gp0 * r1 - q01 + cb * r0 * r1;
    const A ab10 = gp1 * r0 - q10 + cb * r1 * r0;
    const A ab11 = gp1 * r1 - q11 + cb * r1 * r1;
    const A t00 = ab00 * a00 + ab01 * a01, t01 = ab00 * a01 + ab01 * a11;
    const A t10 = ab10 * a00 + ab11 * a01, t11 = ab10 * a01 + ab11 * a11;
    const A sb00 = -(a00 * t00 + a01 * t10);
    const A sb01 = -(a00 * t01 + a01 * t11);
    const A sb10 = -(a01 * t00 + a11 * t10);
    const A sb11 = -(a01 * t01 + a11 * t11);
    // symmetric part of Gbar H (Gbar in columns 0 and 1)
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const A eij = j == 0 ? Gb0[i] : (j == 1 ? Gb1[i] : A(0));
            const A eji = i == 0 ? Gb0[j] : (i == 1 ? Gb1[j] : A(0));
            Cb[pk(i, j)] = Cb[pk(i, j)] + A(0.5) * (eij + eji);
        }
    Cb[0] = Cb[0] + sb00;
    Cb[1] = Cb[1] + A(0.5) * (sb01 + sb10);
    Cb[2] = Cb[2] + sb11;
    pb[0] = pb[0] - rb0;
    pb[1] = pb[1] - rb1;
}

// ------------------------------------------------------------ kernels
__device__ __forceinline__ void set_err(AdjStatus* st, uint32_t bit) { atomicOr(&st->err, bit); }

// Per track: validate the refit set, tag every cluster slot with its instance.
__global__ void k_adj_prep(AdjBufs a) {
    const int nr = a.n_rows;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < a.n_tracks;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t h0 = a.hit_start[t], h1 = a.hit_start[t + 1];
        const int32_t inst = a.inst[t], row0 = a.row0[t];
        bool ok = h0 >= 0 && h0 <= h1 && h1 <= a.n_hits && h1 - h0 <= nr && inst >= 0 && inst < a.n_inst &&
                  row0 >= 0 && row0 < nr;
        if (t == 0 && h0 != 0) ok = false;
        if (t == a.n_tracks - 1 && h1 != a.n_hits) ok = false;
        if (!ok) {
            set_err(a.status, AERR_RANGE);
            continue;
        }
        const int64_t lo = a.row_start[(int64_t)inst * nr], hi = a.row_start[(int64_t)(inst + 1) * nr];
        if (!(lo >= 0 && lo <= hi && hi <= a.n_clusters)) {
            set_err(a.status, AERR_RANGE);
            continue;
        }
        for (int64_t h = h0; h < h1; ++h) {
            const int32_t id = a.hit_id[h];
            if (id < lo || id >= hi) set_err(a.status, AERR_HIT);
            a.hit_inst[h] = inst;
        }
    }
}

// Per cluster slot: pad row (search in the instance's row ranges) and the
// corrected coordinates.
__global__ void k_map_correct(AdjBufs a) {
    if (a.status->err) return;
    const int nr = a.n_rows;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < a.n_hits;
         h += (int64_t)gridDim.x * blockDim.x) {
        const int32_t id = a.hit_id[h];
        const int32_t inst = a.hit_inst[h];
        const int64_t* rs = a.row_start + (int64_t)inst * nr;
        int lo = 0, hi = nr;  // rs[lo] <= id < rs[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rs[mid] <= id) lo = mid;
            else hi = mid;
        }
        a.hit_row[h] = (uint8_t)lo;
        float y = a.y[id], z = a.z[id];
        if (a.coef) {
            const ClusterGeo g = cluster_geo(a, lo, inst, y);
            map_correct(a.coef, g, y, z);
        }
        a.hit_yz[h] = make_float2(y, z);
    }
}

// Per track: rows strictly increasing, and the number of operations of its
// refit: |row0 - outermost row| row steps and a reset, then per pass the row
// span in steps, one update per set mask bit and (passes 2 and 3) a reset.
__global__ void k_adj_count(AdjBufs a) {
    if (a.status->err) return;
    int32_t m = 0, mseg = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < a.n_tracks;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t off = a.hit_start[t];
        const int n = (int)(a.hit_start[t + 1] - off);
        if (n <= 0) continue;
        const uint8_t* rows = a.hit_row + off;
        int used = 0;
        bool inc = true;
        for (int i = 0; i < n; ++i) {
            if (i > 0 && rows[i] <= rows[i - 1]) inc = false;
            const uint8_t mk = a.hit_mask[off + i];
            used += (mk & 1u) + ((mk >> 1) & 1u) + ((mk >> 2) & 1u);
        }
        if (!inc) {
            set_err(a.status, AERR_ROWS);
            continue;
        }
        const int span = rows[n - 1] - rows[0];
        const int d0 = a.row0[t] - rows[n - 1];
        m = max(m, (d0 < 0 ? -d0 : d0) + 3 + 3 * span + used);
        int u0 = 0, u1 = 0, u2 = 0;
        for (int i = 0; i < n; ++i) {
            const uint8_t mk = a.hit_mask[off + i];
            u0 += mk & 1u;
            u1 += (mk >> 1) & 1u;
            u2 += (mk >> 2) & 1u;
        }
        mseg = max(mseg, max((d0 < 0 ? -d0 : d0) + 1 + span + u0, 1 + span + max(u1, u2)));
    }
    if (m > 0) atomicMax(&a.status->max_ops, m);
    if (mseg > 0) atomicMax(&a.status->max_seg_ops, mseg);
}

// Record operation k of a track: five 16-byte words (covariance before it in
// the first 15 floats, three operands, the operation word); the covariance is
// skipped for a reset.
__device__ __forceinline__ void rec_op(uint4* tp, int k, const float* C, bool cov, float o0, float o1, float o2,
                                       uint32_t ow) {
    uint4* p = tp + (int64_t)k * (kTapeWords / 4);
    if (cov) {
        p[0] = make_uint4(__float_as_uint(C[0]), __float_as_uint(C[1]), __float_as_uint(C[2]), __float_as_uint(C[3]));
        p[1] = make_uint4(__float_as_uint(C[4]), __float_as_uint(C[5]), __float_as_uint(C[6]), __float_as_uint(C[7]));
        p[2] = make_uint4(__float_as_uint(C[8]), __float_as_uint(C[9]), __float_as_uint(C[10]),
                          __float_as_uint(C[11]));
        p[3] = make_uint4(__float_as_uint(C[12]), __float_as_uint(C[13]), __float_as_uint(C[14]),
                          __float_as_uint(o0));
    }
    p[4] = make_uint4(__float_as_uint(o1), __float_as_uint(o2), ow, 0u);
}

// The refit of the tracker with given masks, on corrected clusters, over
// tracks [t0, t1): row steps to the outermost cluster, then three passes
// (inward, outward, inward) each opening with a covariance reset; the next
// cluster's row, coordinates and mask are loaded one cluster ahead.
__device__ __forceinline__ float* ckpt_at(const AdjBufs& a, int pass, int64_t t) {
    return a.ckpt + ((int64_t)pass * a.n_tracks + t) * kCkptWords;
}

// Passes [pass_lo, pass_hi) of the refit. pass_lo = 0 starts from the start
// state and walks to the outermost cluster first; pass_lo > 0 starts from
// that pass's checkpoint (a segment recompute, which then counts its own
// operations in seg_nops). With a.ckpt set, the full run (0, 3) stores the
// state, reference point and row at the start of every pass.
template <bool kTape>
__global__ __launch_bounds__(256) void k_refit_fwd(AdjBufs a, int64_t t0, int64_t t1, int outputs, int pass_lo,
                                                   int pass_hi) {
    const DevConsts& K = *a.K;
    const KfConsts kc = kf_consts(K);
    __shared__ float sX[kMaxRows];
    __shared__ int skey[256], sorder[256], s_err;
    kf_load_rows(sX, K);
    // the error flag read once per workgroup (other workgroups may raise it
    // meanwhile): the return, like the barriers below, is uniform
    if (threadIdx.x == 0) s_err = a.status->err;
    __syncthreads();
    if (s_err) return;
    const int cap = a.tape_ops;
    const int nt = blockDim.x;
    for (int64_t c0 = t0 + blockIdx.x * (int64_t)nt; c0 < t1; c0 += (int64_t)gridDim.x * nt) {  // uniform
        int key = -1;  // row steps of the walk and the three passes, plus the updates
        if (c0 + threadIdx.x < t1) {
            const int64_t tk = c0 + threadIdx.x, o = a.hit_start[tk];
            const int nk = (int)(a.hit_start[tk + 1] - o);
            key = nk > 0 ? abs(a.row0[tk] - (int)a.hit_row[o + nk - 1]) +
                               3 * abs((int)a.hit_row[o + nk - 1] - (int)a.hit_row[o]) + 3 * nk
                         : 0;
        }
        const int64_t t = chunk_item_by_work(skey, sorder, c0, key);
        if (t >= t1) continue;
        const int64_t off = a.hit_start[t];
        const int n = (int)(a.hit_start[t + 1] - off);
        const uint8_t* rows = a.hit_row + off;
        const uint8_t* masks = a.hit_mask + off;
        const float2* yz = a.hit_yz + off;
        uint4* tp = kTape ? (uint4*)a.tape + (t - t0) * (int64_t)cap * (kTapeWords / 4) : nullptr;
        const bool segment = !(pass_lo == 0 && pass_hi == 3);
        if (segment && a.nops[t] < 0) {  // the recorded forward failed: nothing to recompute
            a.seg_nops[t] = -1;
            continue;
        }
        KState s;
        float ref_y, ref_z;
        int cur;
        if (pass_lo == 0) {
#pragma unroll
            for (int q = 0; q < 5; ++q) s.p[q] = a.params0[t * 5 + q];
#pragma unroll
            for (int q = 0; q < 15; ++q) s.C[q] = a.cov0[t * 15 + q];
            ref_y = s.p[0];
            ref_z = s.p[1];
            s.p[0] = 0.0f;
            s.p[1] = 0.0f;
            cur = a.row0[t];
        } else {
            const float* c = ckpt_at(a, pass_lo, t);
#pragma unroll
            for (int q = 0; q < 5; ++q) s.p[q] = c[q];
#pragma unroll
            for (int q = 0; q < 15; ++q) s.C[q] = c[5 + q];
            ref_y = c[20];
            ref_z = c[21];
            cur = __float_as_int(c[22]);
        }
        int k = 0;
        bool ok = n > 0;
        float chi2 = 0.0f;
        auto step_to = [&](int target) {
            while (ok && cur != target) {
                const int nx = cur < target ? cur + 1 : cur - 1;
                if (kTape) {
                    if (k < cap) rec_op(tp, k, s.C, true, s.p[2], s.p[3], s.p[4], op_word(OP_PROP, 0, cur, nx, 0));
                    else set_err(a.status, AERR_TAPE);
                }
                ++k;
                if (!kf_propagate(s, sX[cur], sX[nx], kc)) ok = false;
                else cur = nx;
            }
        };
        if (ok && pass_lo == 0) step_to(rows[n - 1]);
        for (int pass = pass_lo; pass < pass_hi && ok; ++pass) {
            if (a.ckpt && !segment) {
                float* c = ckpt_at(a, pass, t);
#pragma unroll
                for (int q = 0; q < 5; ++q) c[q] = s.p[q];
#pragma unroll
                for (int q = 0; q < 15; ++q) c[5 + q] = s.C[q];
                c[20] = ref_y;
                c[21] = ref_z;
                c[22] = __int_as_float(cur);
            }
            if (kTape) {
                if (k < cap) rec_op(tp, k, s.C, false, 0.0f, 0.0f, 0.0f, op_word(OP_RESET, pass, 0, 0, 0));
                else set_err(a.status, AERR_TAPE);
            }
            ++k;
            kf_reset(s, kc);
            const bool inward = pass != 1;
            int i_n = inward ? n - 1 : 0;
            int t_n = rows[i_n];
            float2 c_n = yz[i_n];
            uint8_t m_n = masks[i_n];
            for (int q = 0; q < n && ok; ++q) {
                const int i = i_n, target = t_n;
                const float2 c = c_n;
                const uint8_t mk = m_n;
                if (q + 1 < n) {
                    i_n = inward ? n - 2 - q : q + 1;
                    t_n = rows[i_n];
                    c_n = yz[i_n];
                    m_n = masks[i_n];
                }
                step_to(target);
                if (!ok || !((mk >> pass) & 1u)) continue;
                const Innov inn = kf_innovation(s, c.x - ref_y, c.y - ref_z, kc);
                if (kTape) {
                    if (k < cap) rec_op(tp, k, s.C, true, inn.r0, inn.r1, 0.0f, op_word(OP_UPD, pass, 0, 0, i));
                    else set_err(a.status, AERR_TAPE);
                }
                ++k;
                kf_update(s, inn);
                s.p[0] = s.p[0] + (ref_y - c.x);
                s.p[1] = s.p[1] + (ref_z - c.y);
                ref_y = c.x;
                ref_z = c.y;
                if (pass == 2) chi2 = chi2 + inn.chi2;
            }
        }
        if (segment) a.seg_nops[t] = ok ? k : -1;
        else a.nops[t] = ok ? k : -1;
        if (outputs) {
            a.chi2_track[t] = ok ? chi2 : 0.0f;
            if (a.track_ok) a.track_ok[t] = ok ? 1 : 0;
        }
    }
}

__device__ __forceinline__ void load_op(const uint4* tp, int k, uint4 w[kTapeWords / 4]) {
    const uint4* p = tp + (int64_t)k * (kTapeWords / 4);
#pragma unroll
    for (int f = 0; f < kTapeWords / 4; ++f) w[f] = p[f];
}

// Reverse sweep over the taped tracks [t0, t1), one lane per track.
template <class A>
__global__ __launch_bounds__(256) void k_refit_bwd(AdjBufs a, int64_t t0, int64_t t1, int seg) {
    const DevConsts& K = *a.K;
    const KfConsts kc = kf_consts(K);
    __shared__ float sX[kMaxRows];
    __shared__ int skey[256], sorder[256];
    kf_load_rows(sX, K);
    const int64_t NH = a.n_hits;
    const int nt = blockDim.x;
    for (int64_t c0 = t0 + blockIdx.x * (int64_t)nt; c0 < t1; c0 += (int64_t)gridDim.x * nt) {  // uniform
        int key = -1;  // the recorded operations: the exact length of the reverse sweep
        if (c0 + threadIdx.x < t1) {
            const int64_t tk = c0 + threadIdx.x;
            key = max(seg < 0 ? a.nops[tk] : a.seg_nops[tk], 0);
        }
        const int64_t t = chunk_item_by_work(skey, sorder, c0, key);
        if (t >= t1) continue;
        const int64_t off = a.hit_start[t];
        const int n = (int)(a.hit_start[t + 1] - off);
        const bool first = seg < 0 || seg == 2;  // the last operations of the refit come first
        const bool last = seg <= 0;              // ... and its start last
        if (first)
            for (int p = 0; p < 3; ++p)
                for (int i = 0; i < n; ++i) a.hit_grad[p * NH + off + i] = make_double2(0.0, 0.0);
        double* gp = a.grad_params + t * 5;
        if (a.nops[t] <= 0) {
            if (last)
                for (int q = 0; q < 5; ++q) gp[q] = 0.0;
            continue;
        }
        const int nops = seg < 0 ? a.nops[t] : a.seg_nops[t];
        const uint4* tp = (const uint4*)a.tape + (t - t0) * (int64_t)a.tape_ops * (kTapeWords / 4);
        const A cb = A(a.grad_chi2[t]);
        A pb[5], Cb[15];
        double* cy = a.carry ? a.carry + t * 20 : nullptr;
#pragma unroll
        for (int q = 0; q < 5; ++q) pb[q] = first ? A(0) : A(cy[q]);
#pragma unroll
        for (int q = 0; q < 15; ++q) Cb[q] = first ? A(0) : A(cy[5 + q]);
        if (nops <= 0) {  // a segment without operations passes its adjoint on
            if (last) {
                for (int q = 0; q < 5; ++q) gp[q] = (double)pb[q];
            } else {
                for (int q = 0; q < 5; ++q) cy[q] = (double)pb[q];
                for (int q = 0; q < 15; ++q) cy[5 + q] = (double)Cb[q];
            }
            continue;
        }
        uint4 nxt[kTapeWords / 4];
        load_op(tp, nops - 1, nxt);
        for (int k = nops - 1; k >= 0; --k) {
            uint4 v[kTapeWords / 4];
#pragma unroll
            for (int f = 0; f < kTapeWords / 4; ++f) v[f] = nxt[f];
            if (k > 0) load_op(tp, k - 1, nxt);  // in flight while this operation is differentiated
            const uint32_t ow = v[4].z;
            const int kind = (int)(ow & 3u);
            if (kind == OP_RESET) {
                adj_reset(Cb, kc);
                continue;
            }
            const float C[15] = {__uint_as_float(v[0].x), __uint_as_float(v[0].y), __uint_as_float(v[0].z),
                                 __uint_as_float(v[0].w), __uint_as_float(v[1].x), __uint_as_float(v[1].y),
                                 __uint_as_float(v[1].z), __uint_as_float(v[1].w), __uint_as_float(v[2].x),
                                 __uint_as_float(v[2].y), __uint_as_float(v[2].z), __uint_as_float(v[2].w),
                                 __uint_as_float(v[3].x), __uint_as_float(v[3].y), __uint_as_float(v[3].z)};
            const float o0 = __uint_as_float(v[3].w), o1 = __uint_as_float(v[4].x);
            if (kind == OP_PROP) {
                const int from = (int)((ow >> 4) & 255u), to = (int)((ow >> 12) & 255u);
                adj_prop<A>(C, o0, o1, __uint_as_float(v[4].y), sX[to] - sX[from], pb, Cb, kc);
            } else {
                const int hit = (int)((ow >> 20) & 255u), pass = (int)((ow >> 2) & 3u);
                A mb0 = A(0), mb1 = A(0);
                adj_upd<A>(C, o0, o1, pb, Cb, mb0, mb1, pass == 2 ? cb : A(0), kc);
                a.hit_grad[pass * NH + off + hit] = make_double2((double)mb0, (double)mb1);
            }
        }
        if (last) {
#pragma unroll
            for (int q = 0; q < 5; ++q) gp[q] = (double)pb[q];
        } else {
#pragma unroll
            for (int q = 0; q < 5; ++q) cy[q] = (double)pb[q];
#pragma unroll
            for (int q = 0; q < 15; ++q) cy[5 + q] = (double)Cb[q];
        }
    }
}

__device__ __forceinline__ double2 hit_grad_sum(const AdjBufs& a, int64_t h) {
    const double2 g0 = a.hit_grad[h], g1 = a.hit_grad[a.n_hits + h], g2 = a.hit_grad[2 * a.n_hits + h];
    return make_double2((g0.x + g1.x) + g2.x, (g0.y + g1.y) + g2.y);
}

__global__ void k_hit_grad_out(AdjBufs a, double2* out) {
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < a.n_hits;
         h += (int64_t)gridDim.x * blockDim.x)
        out[h] = hit_grad_sum(a, h);
}

// d loss / d coef: each cluster slot adds its (d/dy', d/dz') times the
// derivative of (y', z') with respect to the 3 x 64 coefficients of its map
// cell. Two kernels:
// * k_grad_cells, one lane per cluster slot: cell, the 12 B-spline weights and
//   the three component factors into an 80-byte record (cell -1: no gradient);
// * k_map_scatter, kMapScatterHits slots per workgroup: the box of coefficients
//   the slots touch (r, phi relative to the first slot's cell, z) accumulates
//   in LDS, cut into z slabs when it exceeds kMapGradLds doubles; each wave
//   stages 64 records in LDS with one coalesced load, then takes one slot at
//   a time and its 64 lanes add the slot's 4 x 4 x 4 cube (lane = (i, j, e)),
//   so a wave's LDS atomics never share an address (a z stride of 4 mod 16
//   doubles spreads them evenly over the banks); the box's non-zero entries
//   then go to the global gradient with FP64 atomics.
// Tracks of one sector touch ~5 of 16 phi and half of the z coefficients: the
// global atomics drop from 192 per cluster to about one box per workgroup.
//
// Deterministic order: every contribution is rounded once to a fixed-point
// integer (a multiple of 2^-S) and all sums, in LDS and in global memory, are
// 64-bit integer additions, which are exact and associative, so the result
// does not depend on the order in which waves and workgroups add. The scale
// is chosen from an order-independent bound: no partial sum of a coefficient
// exceeds the sum over slots of |g| (the B-spline weights of a slot are
// non-negative and add up to one), which is at most n_slots * max|g|; S puts
// that bound at 2^61. The integers are converted back to FP64 at the end.
struct MapFixed {
    unsigned long long max_bits;  // max |g| over slots and components, as the bits of a non-negative double
    double scale;                 // 2^S
    double inv_scale;             // 2^-S
    unsigned long long sum[kMapSize];
};
constexpr int kMapScatterHits = 4096;
constexpr int kMapScatterThreads = 256;
constexpr int kMapGradLds = 7168;  // doubles (56 KB; with the staging buffer two workgroups fit a CU)

struct GradRec {  // 80 bytes
    int32_t cell;  // ir | iphi << 8 | iz << 16 (first coefficient along each axis, iphi + 1 in 0..15), -1: none
    float wr[4], wphi[4], wz[4];
    int32_t pad;
    double gc[3];
};

__global__ void k_grad_cells(AdjBufs a, GradRec* rec, MapFixed* fx) {
    double gmax = 0.0;
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < a.n_hits;
         h += (int64_t)gridDim.x * blockDim.x) {
        const double2 g = hit_grad_sum(a, h);
        GradRec r;
        if (g.x == 0.0 && g.y == 0.0) {
            r.cell = -1;
            for (int i = 0; i < 4; ++i) r.wr[i] = r.wphi[i] = r.wz[i] = 0.0f;
            r.gc[0] = r.gc[1] = r.gc[2] = 0.0;
        } else {
            const int32_t id = a.hit_id[h];
            const float y = a.y[id], z = a.z[id];
            const ClusterGeo geo = cluster_geo(a, a.hit_row[h], a.hit_inst[h], y);
            const MapCell c = map_cell(geo.r, geo.phi, z);
            r.cell = c.ir | ((c.iphi + 1) << 8) | (c.iz << 16);
            for (int i = 0; i < 4; ++i) {
                r.wr[i] = c.wr[i];
                r.wphi[i] = c.wphi[i];
                r.wz[i] = c.wz[i];
            }
            // y' = y - (dr y + drphi x) / r, z' = z - dz
            r.gc[0] = -g.x * (double)y / (double)geo.r;
            r.gc[1] = -g.x * (double)geo.x / (double)geo.r;
            r.gc[2] = -g.y;
            gmax = fmax(gmax, fmax(fabs(r.gc[0]), fmax(fabs(r.gc[1]), fabs(r.gc[2]))));
        }
        r.pad = 0;
        rec[h] = r;
    }
    // the maximum is order-independent; non-negative doubles order as their bit patterns
    for (int o = 32; o > 0; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    if ((threadIdx.x & 63) == 0 && gmax > 0.0) atomicMax(&fx->max_bits, (unsigned long long)__double_as_longlong(gmax));
}

__global__ void k_map_scale(MapFixed* fx, int64_t n_slots) {
    if (threadIdx.x != 0) return;
    const double bound = __longlong_as_double((long long)fx->max_bits) * (double)(n_slots > 0 ? n_slots : 1);
    int e = 0;
    if (bound > 0.0) frexp(bound, &e);  // bound < 2^e
    const int S = 61 - e;
    fx->scale = ldexp(1.0, S);
    fx->inv_scale = ldexp(1.0, -S);
}

__device__ __forceinline__ unsigned long long to_fixed(double v, double scale) {
    return (unsigned long long)__double2ll_rn(v * scale);
}

__global__ void k_map_from_fixed(AdjBufs a, const MapFixed* fx) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kMapSize; i += gridDim.x * blockDim.x)
        a.grad_map[i] = (double)(long long)fx->sum[i] * fx->inv_scale;
}

__device__ __forceinline__ int wrap_dphi(int ip, int ref) {
    return ((ip - ref + 2 * kMapNphi + kMapNphi / 2) % kMapNphi) - kMapNphi / 2;  // in [-8, 8)
}

__global__ __launch_bounds__(kMapScatterThreads) void k_map_scatter(AdjBufs a, const GradRec* rec, MapFixed* fx) {
    __shared__ unsigned long long acc[kMapGradLds + 192];  // the box, then one discard slot per lane and component
    __shared__ GradRec stage[kMapScatterThreads / 64][64];
    __shared__ int lo[3], hi[3], ref;
    const int64_t h0 = (int64_t)blockIdx.x * kMapScatterHits;
    const int64_t h1 = min(h0 + (int64_t)kMapScatterHits, a.n_hits);
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = 1 << 30;
            hi[d] = -(1 << 30);
        }
        ref = -1;
    }
    __syncthreads();
    // reference phi cell: that of the first slot with a gradient (any one would do)
    for (int64_t h = h0 + threadIdx.x; h < h1; h += blockDim.x)
        if (rec[h].cell >= 0) {
            if (ref < 0) atomicCAS(&ref, -1, (rec[h].cell >> 8) & 255);
            break;
        }
    __syncthreads();
    const int rf = ref;
    if (rf < 0) return;  // no slot with a gradient (uniform)
    for (int64_t h = h0 + threadIdx.x; h < h1; h += blockDim.x) {
        const int cell = rec[h].cell;
        if (cell < 0) continue;
        const int ir = cell & 255, ip = (cell >> 8) & 255, iz = cell >> 16;
        const int dp = wrap_dphi(ip, rf);
        atomicMin(&lo[0], ir);
        atomicMax(&hi[0], ir + 3);
        atomicMin(&lo[1], dp - 1);
        atomicMax(&hi[1], dp + 2);
        atomicMin(&lo[2], iz);
        atomicMax(&hi[2], iz + 3);
    }
    __syncthreads();
    const int lr = lo[0], nr = hi[0] - lo[0] + 1;
    const bool full_phi = hi[1] - lo[1] + 1 >= kMapNphi;
    const int lp = full_phi ? 0 : lo[1], np = full_phi ? kMapNphi : hi[1] - lo[1] + 1;
    const int lz = lo[2], hz = hi[2];
    const int slab = 3 * nr * np;  // <= 3 * 16 * 16 = 768
    // z stride of the box: 4 mod 16 doubles (a wave's 4 z lanes x 4 phi lanes
    // then cover every LDS bank once), as small as the z extent allows
    int nzs = 4;
    while (nzs < hz - lz + 1 && (nzs + 16) * slab <= kMapGradLds) nzs += 16;
    const int cstride = nr * np * nzs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int li = lane >> 4, lj = (lane >> 2) & 3, le = lane & 3;
    const double scale = fx->scale;
    for (int z0 = lz; z0 <= hz; z0 += nzs) {
        const int nz = min(nzs, hz - z0 + 1);
        const int size = 3 * cstride;
        for (int i = threadIdx.x; i < size; i += blockDim.x) acc[i] = 0ull;
        __syncthreads();
        // each wave stages 64 records with one coalesced load, then adds
        // them one at a time from LDS; the next record's fields are read
        // before this one's adds are issued, so no read waits for the adds
        for (int64_t hw = h0 + (int64_t)wave * 64; hw < h1; hw += (int64_t)nwave * 64) {
            const int64_t hl = hw + lane;
            if (hl < h1) stage[wave][lane] = rec[hl];
            __builtin_amdgcn_wave_barrier();
            const int cnt = (int)min((int64_t)64, h1 - hw);
            int cell = stage[wave][0].cell;
            float wr = stage[wave][0].wr[li], wp = stage[wave][0].wphi[lj], wz = stage[wave][0].wz[le];
            double g0 = stage[wave][0].gc[0], g1 = stage[wave][0].gc[1], g2 = stage[wave][0].gc[2];
            for (int k = 0; k < cnt; ++k) {
                const int kn = min(k + 1, cnt - 1);
                const int cell_n = stage[wave][kn].cell;
                const float wr_n = stage[wave][kn].wr[li], wp_n = stage[wave][kn].wphi[lj], wz_n = stage[wave][kn].wz[le];
                const double g0_n = stage[wave][kn].gc[0], g1_n = stage[wave][kn].gc[1], g2_n = stage[wave][kn].gc[2];
                // every lane always issues its three adds (a lane with nothing
                // to add adds zero to a slot of its own past the box), so the
                // compiler can count them and the next record's reads do not
                // wait for them
                const int ir = cell & 255, ip = (cell >> 8) & 255, iz = cell >> 16;
                const int zz = iz + le - z0;
                const bool ok = (cell >= 0) & (zz >= 0) & (zz < nz);
                const int pj = full_phi ? (ip - 1 + lj + kMapNphi) % kMapNphi : wrap_dphi(ip, rf) - 1 + lj - lp;
                const double w = ok ? (double)wr * (double)wp * (double)wz : 0.0;
                const int base = ((ir + li - lr) * np + pj) * nzs + zz;
                atomicAdd(&acc[ok ? base : kMapGradLds + lane], to_fixed(g0 * w, scale));
                atomicAdd(&acc[ok ? cstride + base : kMapGradLds + 64 + lane], to_fixed(g1 * w, scale));
                atomicAdd(&acc[ok ? 2 * cstride + base : kMapGradLds + 128 + lane], to_fixed(g2 * w, scale));
                cell = cell_n;
                wr = wr_n;
                wp = wp_n;
                wz = wz_n;
                g0 = g0_n;
                g1 = g1_n;
                g2 = g2_n;
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        for (int i = threadIdx.x; i < size; i += blockDim.x) {
            const unsigned long long v = acc[i];
            if (v == 0ull) continue;
            const int zz = i % nzs, rest = i / nzs;
            const int pj = rest % np, rest2 = rest / np;
            const int rr = rest2 % nr, comp = rest2 / nr;
            const int iphi = full_phi ? pj : rf + lp + pj;  // map_index wraps it
            atomicAdd(fx->sum + map_index(comp, lr + rr, iphi, z0 + zz), v);
        }
        __syncthreads();
    }
}

// Total chi2 in FP64, one block, fixed order.
__global__ void k_sum_chi2(AdjBufs a) {
    __shared__ double sh[1024];
    double acc = 0.0;
    if (!a.status->err)
        for (int64_t t = threadIdx.x; t < a.n_tracks; t += blockDim.x) acc += (double)a.chi2_track[t];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.chi2_total[0] = sh[0];
}

__global__ void k_fill_f64(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_clear_status(AdjStatus* st) {
    if (threadIdx.x == 0) {
        st->err = 0u;
        st->max_ops = 0;
        st->max_seg_ops = 0;
    }
}

inline int blocks_for(int64_t n, int block, int cap) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

void enqueue_refit_prepare(const AdjBufs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, a.status);
    if (a.n_tracks == 0) return;
    hipLaunchKernelGGL(k_adj_prep, dim3(blocks_for(a.n_tracks, 256, 16384)), dim3(256), 0, st, a);
    if (a.n_hits > 0)
        hipLaunchKernelGGL(k_map_correct, dim3(blocks_for(a.n_hits, 256, 16384)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_count, dim3(blocks_for(a.n_tracks, 256, 4096)), dim3(256), 0, st, a);
}

void enqueue_refit_forward(const AdjBufs& a, int64_t t0, int64_t t1, bool outputs, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g(blocks_for(t1 - t0, 128, 16384)), b(128);
    if (a.tape)
        hipLaunchKernelGGL(k_refit_fwd<true>, g, b, 0, st, a, t0, t1, outputs ? 1 : 0, 0, 3);
    else
        hipLaunchKernelGGL(k_refit_fwd<false>, g, b, 0, st, a, t0, t1, outputs ? 1 : 0, 0, 3);
}

void enqueue_refit_segment(const AdjBufs& a, int64_t t0, int64_t t1, int seg, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g(blocks_for(t1 - t0, 128, 16384)), b(128);
    hipLaunchKernelGGL(k_refit_fwd<true>, g, b, 0, st, a, t0, t1, 0, seg, seg + 1);
}

void enqueue_refit_total(const AdjBufs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_chi2, dim3(1), dim3(1024), 0, st, a);
}

void enqueue_refit_reverse(const AdjBufs& a, int64_t t0, int64_t t1, int seg, hipStream_t st) {
    if (t1 <= t0) return;
    const dim3 g(blocks_for(t1 - t0, 128, 16384)), b(128);
    if (a.adj_f64)
        hipLaunchKernelGGL(k_refit_bwd<double>, g, b, 0, st, a, t0, t1, seg);
    else
        hipLaunchKernelGGL(k_refit_bwd<float>, g, b, 0, st, a, t0, t1, seg);
}

size_t map_grad_scratch_bytes(int64_t n_hits) {
    return (sizeof(MapFixed) + 255) / 256 * 256 + sizeof(GradRec) * (size_t)n_hits;
}

void enqueue_refit_map_grad(const AdjBufs& a, void* scratch, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(kMapSize, 256, 1024)), dim3(256), 0, st, a.grad_map,
                       (int64_t)kMapSize);
    if (a.n_hits <= 0) return;
    MapFixed* fx = (MapFixed*)scratch;
    GradRec* rec = (GradRec*)((char*)scratch + (sizeof(MapFixed) + 255) / 256 * 256);
    // zero the fixed-point block (a fill kernel: also safe under graph capture)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(sizeof(MapFixed) / 8, 256, 1024)), dim3(256), 0, st,
                       (double*)fx, (int64_t)(sizeof(MapFixed) / 8));
    hipLaunchKernelGGL(k_grad_cells, dim3(blocks_for(a.n_hits, 256, 16384)), dim3(256), 0, st, a, rec, fx);
    hipLaunchKernelGGL(k_map_scale, dim3(1), dim3(64), 0, st, fx, a.n_hits);
    hipLaunchKernelGGL(k_map_scatter, dim3((unsigned)((a.n_hits + kMapScatterHits - 1) / kMapScatterHits)),
                       dim3(kMapScatterThreads), 0, st, a, (const GradRec*)rec, fx);
    hipLaunchKernelGGL(k_map_from_fixed, dim3(blocks_for(kMapSize, 256, 1024)), dim3(256), 0, st, a,
                       (const MapFixed*)fx);
}

void enqueue_refit_hit_grad(const AdjBufs& a, double* out, hipStream_t st) {
    if (a.n_hits > 0)
        hipLaunchKernelGGL(k_hit_grad_out, dim3(blocks_for(a.n_hits, 256, 16384)), dim3(256), 0, st, a,
                           (double2*)out);
}

namespace {

// Corrected final fit, first step: every output cluster of the last track
// call in its track's absolute frame (z minus the track's vertex z) and
// corrected by the map; one wave per track, one lane per cluster.
__global__ __launch_bounds__(256) void k_corr_clusters(CorrBufs c) {
    const DevConsts& K = *c.K;
    const int nr = c.n_rows;
    const int lane = threadIdx.x & 63;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; t < c.n_tracks; t += nwave) {
        const int32_t inst = c.inst[t];
        const int64_t* rs = c.row_start + (int64_t)inst * nr;
        const int sec = c.inst_sector[inst];
        const float zv = c.z0[t];
        for (int64_t q = c.hit_start[t] + lane; q < c.hit_start[t + 1]; q += 64) {
            const int32_t id = c.hit_id[q];
            int lo = 0, hi = nr;  // rs[lo] <= id < rs[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rs[mid] <= id) lo = mid;
                else hi = mid;
            }
            const float2 p = c.yz[c.pos_of[id]];
            float y = p.x, z = p.y - zv;
            if (c.coef) {
                ClusterGeo g;
                g.x = K.X[lo];
                g.r = __builtin_sqrtf(g.x * g.x + y * y);
                g.phi = K.alpha[((sec % 18) + 18) % 18] + atan2f(y, g.x);
                map_correct(c.coef, g, y, z);
            }
            c.cyz[q] = make_float2(y, z);
            c.crow[q] = (uint8_t)lo;
            if (c.o_hit_yz) {
                c.o_hit_yz[2 * q] = y;
                c.o_hit_yz[2 * q + 1] = z;
            }
        }
    }
}

// Corrected final fit, second step: one lane per track, the three passes of
// the final fit (covariance reset, chi2 rejection, reference point moved to
// each accepted cluster) over the corrected clusters, from the track's output
// state moved to the absolute frame; the next cluster is loaded one step
// ahead. ndf = 2 accepted - 5, or -1 when a step fails or fewer than n_min
// clusters are kept (the other outputs are then unspecified).
__global__ __launch_bounds__(128) void k_fit_corrected(CorrBufs c) {
    const DevConsts& K = *c.K;
    const KfConsts kc = kf_consts(K);
    __shared__ float sX[kMaxRows];
    __shared__ int skey[128], sorder[128];
    kf_load_rows(sX, K);
    const int nr = c.n_rows;
    const int nt = blockDim.x;
    for (int64_t c0 = blockIdx.x * (int64_t)nt; c0 < c.n_tracks; c0 += (int64_t)gridDim.x * nt) {  // uniform
        int key = -1;  // row steps of the three passes, plus the updates
        if (c0 + threadIdx.x < c.n_tracks) {
            const int64_t tk = c0 + threadIdx.x, hk = c.hit_start[tk];
            const int nk = (int)(c.hit_start[tk + 1] - hk);
            key = nk > 0 ? 3 * abs((int)c.crow[hk + nk - 1] - (int)c.crow[hk]) + 3 * nk : 0;
        }
        const int64_t t = chunk_item_by_work(skey, sorder, c0, key);
        if (t >= c.n_tracks) continue;
        const int64_t h0 = c.hit_start[t];
        const int n = (int)(c.hit_start[t + 1] - h0);
        const float zv = c.z0[t];
        KState s;
#pragma unroll
        for (int q = 0; q < 5; ++q) s.p[q] = c.param[t * 5 + q];
#pragma unroll
        for (int q = 0; q < 15; ++q) s.C[q] = c.cov[t * 15 + q];
        s.p[1] = s.p[1] - zv;
        int cur = 0;  // the row of x_ref (pad-row planes ascending)
        {
            const float x = c.xref[t];
            int lo = 0, hi = nr - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sX[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            cur = lo;
        }
        float ref_y = s.p[0], ref_z = s.p[1];
        s.p[0] = 0.0f;
        s.p[1] = 0.0f;
        bool ok = n > 0;
        const int outer = ok ? (int)c.crow[h0 + n - 1] : 0;
        while (ok && cur != outer) {
            const int nx = cur < outer ? cur + 1 : cur - 1;
            if (!kf_propagate(s, sX[cur], sX[nx], kc)) ok = false;
            else cur = nx;
        }
        if (c.o_mask)
            for (int i = 0; i < n; ++i) c.o_mask[h0 + i] = 0;
        float chi2sum = 0.0f;
        int nacc = 0;
        for (int pass = 0; pass < 3 && ok; ++pass) {
            kf_reset(s, kc);
            const bool inward = pass != 1;
            int i_n = inward ? n - 1 : 0;
            int t_n = c.crow[h0 + i_n];
            float2 c_n = c.cyz[h0 + i_n];
            for (int q = 0; q < n && ok; ++q) {
                const int i = i_n, target = t_n;
                const float2 cc = c_n;
                if (q + 1 < n) {
                    i_n = inward ? n - 2 - q : q + 1;
                    t_n = c.crow[h0 + i_n];
                    c_n = c.cyz[h0 + i_n];
                }
                while (cur != target) {
                    const int nx = cur < target ? cur + 1 : cur - 1;
                    if (!kf_propagate(s, sX[cur], sX[nx], kc)) {
                        ok = false;
                        break;
                    }
                    cur = nx;
                }
                if (!ok) break;
                const Innov inn = kf_innovation(s, cc.x - ref_y, cc.y - ref_z, kc);
                if (inn.chi2 <= kc.chi2_rej) {
                    kf_update(s, inn);
                    s.p[0] = s.p[0] + (ref_y - cc.x);
                    s.p[1] = s.p[1] + (ref_z - cc.y);
                    ref_y = cc.x;
                    ref_z = cc.y;
                    if (c.o_mask) c.o_mask[h0 + i] = (uint8_t)(c.o_mask[h0 + i] | (1u << pass));
                    if (pass == 2) {
                        chi2sum = chi2sum + inn.chi2;
                        ++nacc;
                    }
                }
            }
        }
        s.p[0] = ref_y + s.p[0];
        s.p[1] = ref_z + s.p[1];
        ok = ok && nacc >= kc.n_min;
#pragma unroll
        for (int q = 0; q < 5; ++q) c.o_param[t * 5 + q] = s.p[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) c.o_cov[t * 15 + q] = s.C[q];
        c.o_chi2[t] = chi2sum;
        c.o_ndf[t] = ok ? 2 * nacc - 5 : -1;
        c.o_xref[t] = sX[cur];
        c.o_z0[t] = ok ? zv + vertex_z(K.kB_f64, (double)sX[cur], s.p) : zv;
    }
}

}  // namespace

void enqueue_fit_corrected(const CorrBufs& c, hipStream_t st) {
    if (c.n_tracks <= 0) return;
    const int64_t w = c.n_tracks * 64;
    const int64_t g1 = (w + 255) / 256, g2 = (c.n_tracks + 127) / 128;
    hipLaunchKernelGGL(k_corr_clusters, dim3((unsigned)(g1 < 16384 ? g1 : 16384)), dim3(256), 0, st, c);
    hipLaunchKernelGGL(k_fit_corrected, dim3((unsigned)(g2 < 16384 ? g2 : 16384)), dim3(128), 0, st, c);
}

}  // namespace tpcca
