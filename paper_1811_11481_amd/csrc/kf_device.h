// Binary32 Kalman-filter primitives for the tracklet and refit kernels.
//
// State (y, z, sin phi, tan lambda, q/pT) at a pad-row plane x; covariance in
// packed lower-triangular order 00,10,11,20,21,22,30,31,32,33,40,41,42,43,44.
// Every expression is evaluated in the written order in IEEE binary32: the
// library is built with -ffp-contract=off and this header forbids contraction
// as well, so a multiply-add is fused exactly where __builtin_fmaf is written
// (one rounding, as IEEE fma) and nowhere else; / and sqrt are correctly rounded.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace tpcca {

constexpr int kMaxRows = 256;

// Per-context constants (binary32), built once on the host.
struct DevConsts {
    int n_rows, n_min, max_miss, stats;
    float X[kMaxRows];                        // pad-row plane x
    float wyu[kMaxRows], wzu[kMaxRows];       // neighbour windows towards row r+1
    float wyd[kMaxRows], wzd[kMaxRows];       // ... towards row r-1
    float tr[kMaxRows];                       // (X[r]-X[r-1]) / (X[r+1]-X[r-1])
    float alpha[18];                          // sector rotation angles
    float kB, vy, vz, smax, nsig, chi2_pick, chi2_rej, sinphi_max, cov_reset, q_max, u_max2;
    float c0[5];
    double kB_f64;                            // -0.00299792458 * Bz in FP64 (vertex z only)
    float chi2_merge, rot_c, rot_s;           // cross-sector merge cut; cos, sin of 20 degrees
    int merge_max_gap;                        // rows between a continued segment's end and the next
    float pad_w[kMaxRows], pad_c[kMaxRows];   // native input: pad pitch, pad coordinate of y = 0
    float z_per_bin, z_readout;               // native input: drift length per time bin, |z| of the readout
};

// The scalar constants of the row steps, copied into registers once per
// kernel (before any store, so they come in as uniform scalar loads). A step
// that read them from global memory would wait on each of those loads, and a
// wait on the vector-memory counter also waits for every load issued before
// it, prefetches included.
struct KfConsts {
    float kB, vy, vz, nsig, chi2_pick, chi2_rej, sinphi_max, cov_reset, u_max2;
    int max_miss, n_min;
};

__device__ __forceinline__ KfConsts kf_consts(const DevConsts& K) {
    KfConsts c;
    c.kB = K.kB;
    c.vy = K.vy;
    c.vz = K.vz;
    c.nsig = K.nsig;
    c.chi2_pick = K.chi2_pick;
    c.chi2_rej = K.chi2_rej;
    c.sinphi_max = K.sinphi_max;
    c.cov_reset = K.cov_reset;
    c.u_max2 = K.u_max2;
    c.max_miss = K.max_miss;
    c.n_min = K.n_min;
    return c;
}

// Pad-row radii in LDS for one workgroup (indexed per lane without touching
// the vector-memory counter). Every thread of the block must call it.
__device__ __forceinline__ void kf_load_rows(float* sX, const DevConsts& K) {
    for (int i = threadIdx.x; i < K.n_rows; i += blockDim.x) sX[i] = K.X[i];
    __syncthreads();
}

struct KState {
    float p[5];
    float C[15];
};

__device__ __forceinline__ int pk(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Correctly rounded binary32 square root, the same value as sqrtf, for the
// arguments of the helix step: +-0, normal numbers of at least 2^-96, +inf,
// negative numbers and NaN. The hardware square root is within one ulp; the
// result is its neighbour below or above when the residual x - s'*s of that
// neighbour s', formed by one fused multiply-add, shows the exact root to lie
// past the midpoint (the one-ulp correction of a faithful square root). The
// library call adds a scaling of arguments below 2^-96, where the residuals
// would lose bits, and a class test for 0 and inf (both come out right here
// without it). The helix step never takes a root there: 1 - s^2 of a binary32
// sine s below 1 in magnitude is at least 2^-23, and 1 + t^2 is at least 1.
__device__ __forceinline__ float sqrt_step(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float sd = __int_as_float(__float_as_int(s) - 1);
    const float su = __int_as_float(__float_as_int(s) + 1);
    float r = s;
    if (__builtin_fmaf(-sd, s, x) <= 0.0f) r = sd;
    if (__builtin_fmaf(-su, s, x) > 0.0f) r = su;
    return r;
}

// asin(u)/u by its Maclaurin series through u^12 (coefficients (2n)!/(4^n (n!)^2 (2n+1))).
__device__ __forceinline__ float asin_over_u(float u) {
    const float w = u * u;
    const float c1 = (float)(1.0 / 6.0), c2 = (float)(3.0 / 40.0), c3 = (float)(5.0 / 112.0),
                c4 = (float)(35.0 / 1152.0), c5 = (float)(63.0 / 2816.0), c6 = (float)(231.0 / 13312.0);
    float h = __builtin_fmaf(w, c6, c5);
    h = __builtin_fmaf(w, h, c4);
    h = __builtin_fmaf(w, h, c3);
    h = __builtin_fmaf(w, h, c2);
    h = __builtin_fmaf(w, h, c1);
    return __builtin_fmaf(w, h, 1.0f);
}

// Its derivative from the same series.
__device__ __forceinline__ float asin_over_u_deriv(float u) {
    const float w = u * u;
    const float d1 = (float)(2.0 / 6.0), d2 = (float)(12.0 / 40.0), d3 = (float)(30.0 / 112.0),
                d4 = (float)(280.0 / 1152.0), d5 = (float)(630.0 / 2816.0), d6 = (float)(2772.0 / 13312.0);
    float h = __builtin_fmaf(w, d6, d5);
    h = __builtin_fmaf(w, h, d4);
    h = __builtin_fmaf(w, h, d3);
    h = __builtin_fmaf(w, h, d2);
    h = __builtin_fmaf(w, h, d1);
    return u * h;
}

// One helix step x1 -> x2 in a uniform field along z: sin phi advances by
// kB*q*dx, y by dx times the tangent of the mean direction, z by tan(lambda)
// times the arc (signed chord * asin(u)/u). Covariance: C <- F C F^T with the
// exact Jacobian of this step. Returns false and leaves the state unchanged
// when |sin phi| would reach the guard or the step bends too much.
template <class KC>
__device__ __forceinline__ bool kf_propagate(KState& s, float x1, float x2, const KC& K) {
    const float dx = x2 - x1;
    const float s1 = s.p[2];
    const float kq = K.kB * s.p[4];
    const float s2 = __builtin_fmaf(kq, dx, s1);
    if (!(__builtin_fabsf(s2) < K.sinphi_max)) return false;
    const float c1 = sqrt_step(__builtin_fmaf(-s1, s1, 1.0f));
    const float c2 = sqrt_step(__builtin_fmaf(-s2, s2, 1.0f));
    const float tt = (s1 + s2) / (c1 + c2);
    const float w = __builtin_fmaf(tt, tt, 1.0f);
    const float lc = dx * sqrt_step(w);
    const float u = (kq * lc) * 0.5f;
    if (!(u * u <= K.u_max2)) return false;
    const float g = asin_over_u(u);
    const float arc = lc * g;
    const float t = s.p[3];
    const float ic1 = 1.0f / c1, ic2 = 1.0f / c2;  // two reciprocals serve four Jacobian terms
    const float f02 = ((dx * w) * (ic1 + ic2)) * 0.5f;
    const float f04 = ((dx * w) * ((K.kB * dx) * ic2)) * 0.5f;
    const float f12 = t * ((dx * tt) * (ic1 * ic2));
    const float f13 = arc;
    const float dlc = (((K.kB * dx) * lc) * tt) * (0.5f * ic2);
    const float du = __builtin_fmaf(K.kB, lc, kq * dlc) * 0.5f;
    const float f14 = t * __builtin_fmaf(dlc, g, (lc * asin_over_u_deriv(u)) * du);
    const float f24 = K.kB * dx;
    s.p[0] = __builtin_fmaf(dx, tt, s.p[0]);
    s.p[1] = __builtin_fmaf(t, arc, s.p[1]);
    s.p[2] = s2;
    // B = F C; only rows 0, 1, 2 differ from C.
    float B0[5], B1[5], B2[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float c0j = s.C[pk(0, j)], c1j = s.C[pk(1, j)], c2j = s.C[pk(2, j)], c3j = s.C[pk(3, j)],
                    c4j = s.C[pk(4, j)];
        B0[j] = __builtin_fmaf(f04, c4j, __builtin_fmaf(f02, c2j, c0j));
        B1[j] = __builtin_fmaf(f14, c4j, __builtin_fmaf(f13, c3j, __builtin_fmaf(f12, c2j, c1j)));
        B2[j] = __builtin_fmaf(f24, c4j, c2j);
    }
    // C' = B F^T (lower triangle). Rows 3, 4 of B are rows 3, 4 of C.
    float B3[5], B4[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        B3[j] = s.C[pk(3, j)];
        B4[j] = s.C[pk(4, j)];
    }
    float* Bi[5] = {B0, B1, B2, B3, B4};
    float Cn[15];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float* b = Bi[i];
        Cn[pk(i, 0)] = __builtin_fmaf(f04, b[4], __builtin_fmaf(f02, b[2], b[0]));
        if (i >= 1) Cn[pk(i, 1)] = __builtin_fmaf(f14, b[4], __builtin_fmaf(f13, b[3], __builtin_fmaf(f12, b[2], b[1])));
        if (i >= 2) Cn[pk(i, 2)] = __builtin_fmaf(f24, b[4], b[2]);
        if (i >= 3) Cn[pk(i, 3)] = b[3];
        if (i >= 4) Cn[pk(i, 4)] = b[4];
    }
#pragma unroll
    for (int q = 0; q < 15; ++q) s.C[q] = Cn[q];
    return true;
}

// The state part of kf_propagate alone (the same expressions, so the same
// binary32 results): the track model of the compression residuals.
template <class KC>
__device__ __forceinline__ bool kf_step_state(float* p, float x1, float x2, const KC& K) {
    const float dx = x2 - x1;
    const float s1 = p[2];
    const float kq = K.kB * p[4];
    const float s2 = __builtin_fmaf(kq, dx, s1);
    if (!(__builtin_fabsf(s2) < K.sinphi_max)) return false;
    const float c1 = sqrt_step(__builtin_fmaf(-s1, s1, 1.0f));
    const float c2 = sqrt_step(__builtin_fmaf(-s2, s2, 1.0f));
    const float tt = (s1 + s2) / (c1 + c2);
    const float w = __builtin_fmaf(tt, tt, 1.0f);
    const float lc = dx * sqrt_step(w);
    const float u = (kq * lc) * 0.5f;
    if (!(u * u <= K.u_max2)) return false;
    const float arc = lc * asin_over_u(u);
    p[0] = __builtin_fmaf(dx, tt, p[0]);
    p[1] = __builtin_fmaf(p[3], arc, p[1]);
    p[2] = s2;
    return true;
}

// Innovation of a measurement (my, mz): residual, inverse of S = C[0:2,0:2]+V
// and the predicted chi2.
struct Innov {
    float a00, a01, a11, r0, r1, chi2;
};

template <class KC>
__device__ __forceinline__ Innov kf_innovation(const KState& s, float my, float mz, const KC& K) {
    Innov n;
    const float s00 = s.C[0] + K.vy, s01 = s.C[1], s11 = s.C[2] + K.vz;
    const float det = __builtin_fmaf(s00, s11, -(s01 * s01));
    const float idet = 1.0f / det;
    n.a00 = s11 * idet;
    n.a01 = (-s01) * idet;
    n.a11 = s00 * idet;
    n.r0 = my - s.p[0];
    n.r1 = mz - s.p[1];
    const float w0 = __builtin_fmaf(n.a00, n.r0, n.a01 * n.r1);
    const float w1 = __builtin_fmaf(n.a01, n.r0, n.a11 * n.r1);
    n.chi2 = __builtin_fmaf(n.r0, w0, n.r1 * w1);
    return n;
}

// Kalman update with gain K = C H^T S^-1 (H picks y and z).
__device__ __forceinline__ void kf_update(KState& s, const Innov& n) {
    float c0j[5], c1j[5], K0[5], K1[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        c0j[j] = s.C[pk(0, j)];
        c1j[j] = s.C[pk(1, j)];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        K0[i] = __builtin_fmaf(c0j[i], n.a00, c1j[i] * n.a01);
        K1[i] = __builtin_fmaf(c0j[i], n.a01, c1j[i] * n.a11);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) s.p[i] = s.p[i] + __builtin_fmaf(K0[i], n.r0, K1[i] * n.r1);
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            s.C[pk(i, j)] = s.C[pk(i, j)] - __builtin_fmaf(K0[i], c0j[j], K1[i] * c1j[j]);
}

// z of the point of closest approach of the helix (state p at local x) to
// the beam line, the z axis of every sector frame: the turning angle d from
// the state solves A cos d + (B + 1/c) sin d = 0 with A = x cos phi + y sin phi,
// B = -x sin phi + y cos phi and curvature c = kB q/pT, so d = atan2(-A c,
// 1 + B c) and z0 = z + tan(lambda) d / c (as A/(1 + B c) atan(w)/w, w = -A c /
// (1 + B c), where 1 + B c > 0: exact in the straight-line limit). FP64: a
// derived output, evaluated once per track, not part of the Kalman filter.
__device__ __forceinline__ float vertex_z(double kB, double x, const float* p) {
    const double y = p[0], z = p[1], sp = p[2], tl = p[3], q = p[4];
    const double cp = sqrt(1.0 - sp * sp);
    const double c = kB * q;
    const double A = x * cp + y * sp, B = -x * sp + y * cp;
    const double den = 1.0 + B * c;
    double s;
    if (den > 0.0) {
        const double w = -A * c / den;
        const double g = (w == 0.0) ? 1.0 : atan(w) / w;
        s = -A / den * g;
    } else {
        s = atan2(-A * c, den) / c;
    }
    return (float)(z + tl * s);
}

// Lanes take the items (tracks, chains) of their workgroup's chunk
// [c0, c0 + blockDim.x) longest first (key: an estimate of the item's serial
// work, -1 past the end; equal keys in chunk order), so that the lanes of one
// wave end at similar times. Each item is independent and writes its own
// slots: the assignment changes no result. All threads of the workgroup must
// call it; skey and sorder hold blockDim.x ints in LDS.
__device__ __forceinline__ int64_t chunk_item_by_work(int* skey, int* sorder, int64_t c0, int key) {
    const int tid = threadIdx.x, nt = blockDim.x;
    skey[tid] = key;
    __syncthreads();
    int rank = 0;
    for (int j = 0; j < nt; ++j) {
        const int kj = skey[j];
        rank += (kj > key || (kj == key && j < tid)) ? 1 : 0;
    }
    sorder[rank] = tid;
    __syncthreads();
    const int64_t k = c0 + sorder[tid];
    __syncthreads();  // skey and sorder are rewritten for the next chunk
    return k;
}

// Covariance reset at a turn or pass start: variances scaled, correlations dropped.
template <class KC>
__device__ __forceinline__ void kf_reset(KState& s, const KC& K) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) s.C[pk(i, j)] = 0.0f;
        s.C[pk(i, i)] = s.C[pk(i, i)] * K.cov_reset;
    }
}

}  // namespace tpcca
