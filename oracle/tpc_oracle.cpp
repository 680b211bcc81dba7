// TPC track-finding ORACLE — test infrastructure only.
//
// A plain, slow CPU implementation of the sector-tracking hot path of
// Rohr, Gorbunov, Schmidt, Shahoyan, "Track Reconstruction in the ALICE TPC
// using GPUs for LHC Run 3" (arXiv:1811.11481). Only tests, the smoke check and
// the benchmark's CPU-baseline leg may load it; the product path never does.
// It shares no code with the GPU library.
//
// What it computes, in the paper's order (Section 2, "TPC Tracking Algorithm
// and Implementation"; Section 3, "Improvements of Tracking Resolution"):
//   1. per-(instance, pad row) hit grid (an exported artefact only: every
//      search below is brute force over the whole row, so no result depends on
//      the grid);
//   2. cellular automaton: links between hit triplets on adjacent rows that lie
//      close to a straight line (neighbour finding), then keeping only mutual
//      links (the evolution step that concatenates consecutive links), then the
//      start hits of chains of >= 3 hits;
//   3. tracklets: a simplified Kalman filter over each chain, extrapolation
//      outward with pickup of the best hit per row (no multiple hypotheses),
//      then an inward pass that propagates through the seed again and re-picks
//      every row (outlier rejection, Section 3);
//   4. selection: each cluster goes to the tracklet with the largest packed
//      (nHits, -id) weight; a tracklet survives with >= N_MIN owned clusters;
//   5. refit: the full Kalman filter iterated inward, outward, inward, with
//      clusters rejected on their predicted chi2 (Section 3).
// Numerical readings the paper leaves open (windows, cuts, initial covariance,
// tie-breaks, the helix step) follow the written algorithm description of this
// project; every number below is a parameter.
//
// Two instantiations: T = double (the FP64 oracle, exact asin in the helix
// step) and T = float (binary32 in a fixed operation order, no contraction, no
// library transcendentals: a power series for asin(u)/u).
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -shared -fPIC
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

extern "C" {
// Tracking parameters (all physics/geometry numbers; FP64 storage, each mode
// rounds them to its own precision once).
typedef struct {
    int32_t n_rows;        // pad rows (152)
    double bz;             // solenoid field [T]
    double sigma_y, sigma_z;  // cluster errors [cm]
    double win_ty, win_tz, win_ny, win_nz;  // neighbour window: dx * T + N [cm]
    double nbr_score_max;  // max straight-line deviation score [cm^2]
    double nsig;           // pickup window in sigmas
    double chi2_pick;      // pickup chi2 cut (2 dof)
    double chi2_rej;       // refit rejection chi2 cut (2 dof)
    double sinphi_max;     // |sin phi| guard
    double cov_reset;      // diagonal scale at a covariance reset
    double q_max;          // |q/pT| clamp of the seed estimate [c/GeV]
    double u_max;          // max |kappa * chord / 2| of one helix step
    double c0[5];          // initial covariance diagonal
    int32_t n_min;         // minimum clusters of a tracklet / track
    int32_t max_miss;      // consecutive empty rows that end the following
    int32_t hits_per_bin;  // grid occupancy target
    int32_t n_threads;     // CPU worker threads over instances (0 = 1)
    int32_t planes_f32;    // 1: pad-row planes at their binary32 positions in both
                           // modes (the positions the tracker is given), 0: exact
    double chi2_merge;     // cross-sector merge: max chi2 (5 parameters) of a segment pair
    int32_t merge_max_gap; // cross-sector merge: max rows between the continued segment's end and the next
} orc_params;

void orc_default_params(orc_params* p) {
    p->n_rows = 152;
    p->bz = 0.5;
    p->sigma_y = p->sigma_z = 0.1;
    p->win_ty = 2.0; p->win_tz = 1.1; p->win_ny = 0.5; p->win_nz = 0.5;
    p->nbr_score_max = 0.24;
    p->nsig = 3.0;
    p->chi2_pick = 16.0;
    p->chi2_rej = 25.0;
    p->sinphi_max = 0.95;
    p->cov_reset = 100.0;
    p->q_max = 20.0;
    p->u_max = 0.25;
    p->c0[0] = 1.0; p->c0[1] = 1.0; p->c0[2] = 0.25; p->c0[3] = 0.25; p->c0[4] = 400.0;
    p->n_min = 10;
    p->max_miss = 8;
    p->hits_per_bin = 1;
    p->n_threads = 1;
    p->planes_f32 = 0;
    p->chi2_merge = 25.0;
    p->merge_max_gap = 24;
}
}

namespace {

// Pad-row plane position: 152 rows evenly spaced between 85 and 247 cm.
double plane_x(int i) { return 85.0 + i * 162.0 / 151.0; }

// ----------------------------------------------------------------------------
// Constants of one precision mode.
template <class T>
struct Consts {
    int n_rows;
    std::vector<T> X;            // row plane x
    std::vector<T> dxu, dxd;     // X[r+1]-X[r], X[r]-X[r-1]
    std::vector<T> wyu, wzu, wyd, wzd, tr;
    T kB;                        // d(sin phi)/dx per unit q/pT
    T vy, vz;                    // sigma^2
    T smax, nsig, chi2_pick, chi2_rej, sinphi_max, cov_reset, q_max, u_max2;
    T c0[5];
    int n_min, max_miss, hpb;
    T chi2_merge, rot_c, rot_s;  // merge cut; cos and sin of one sector's opening (20 degrees)
    int merge_max_gap;
    explicit Consts(const orc_params& p) {
        n_rows = p.n_rows;
        X.resize(n_rows);
        // the binary32 mode always sees the rounded planes; the FP64 mode sees
        // them too when it replays a binary32 result, so that both evaluate
        // the same detector and differ only in their arithmetic
        for (int i = 0; i < n_rows; ++i) X[i] = p.planes_f32 ? (T)(float)plane_x(i) : (T)plane_x(i);
        dxu.assign(n_rows, 0); dxd.assign(n_rows, 0);
        wyu.assign(n_rows, 0); wzu.assign(n_rows, 0); wyd.assign(n_rows, 0); wzd.assign(n_rows, 0);
        tr.assign(n_rows, 0);
        const T ty = (T)p.win_ty, tz = (T)p.win_tz, ny = (T)p.win_ny, nz = (T)p.win_nz;
        for (int r = 1; r + 1 < n_rows; ++r) {
            dxu[r] = X[r + 1] - X[r];
            dxd[r] = X[r] - X[r - 1];
            wyu[r] = dxu[r] * ty + ny;
            wzu[r] = dxu[r] * tz + nz;
            wyd[r] = dxd[r] * ty + ny;
            wzd[r] = dxd[r] * tz + nz;
            tr[r] = (X[r] - X[r - 1]) / (X[r + 1] - X[r - 1]);
        }
        kB = (T)(-0.00299792458 * p.bz);
        const T sy = (T)p.sigma_y, sz = (T)p.sigma_z;
        vy = sy * sy;
        vz = sz * sz;
        smax = (T)p.nbr_score_max;
        nsig = (T)p.nsig;
        chi2_pick = (T)p.chi2_pick;
        chi2_rej = (T)p.chi2_rej;
        sinphi_max = (T)p.sinphi_max;
        cov_reset = (T)p.cov_reset;
        q_max = (T)p.q_max;
        const T um = (T)p.u_max;
        u_max2 = um * um;
        for (int i = 0; i < 5; ++i) c0[i] = (T)p.c0[i];
        n_min = p.n_min;
        max_miss = p.max_miss;
        hpb = p.hits_per_bin < 1 ? 1 : p.hits_per_bin;
        chi2_merge = (T)p.chi2_merge;
        merge_max_gap = p.merge_max_gap;
        rot_c = (T)std::cos(20.0 * 3.14159265358979323846 / 180.0);
        rot_s = (T)std::sin(20.0 * 3.14159265358979323846 / 180.0);
    }
};

// ----------------------------------------------------------------------------
// Track state: (y, z, sin phi, tan lambda, q/pT) at a local x, and the
// covariance in packed lower-triangular order 00,10,11,20,21,22,30,...,44.
template <class T>
struct State {
    T p[5];
    T C[15];
};

inline int pk(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// asin(u)/u. FP64: the library arcsine. FP32: its Maclaurin series
// sum_n (2n)! / (4^n (n!)^2 (2n+1)) u^(2n) through u^12, in Horner form.
inline double asin_over(double u) { return u == 0.0 ? 1.0 : std::asin(u) / u; }
inline float asin_over(float u) {
    const float w = u * u;
    const float c1 = (float)(1.0 / 6.0), c2 = (float)(3.0 / 40.0), c3 = (float)(5.0 / 112.0),
                c4 = (float)(35.0 / 1152.0), c5 = (float)(63.0 / 2816.0), c6 = (float)(231.0 / 13312.0);
    float h = std::fma(w, c6, c5);
    h = std::fma(w, h, c4);
    h = std::fma(w, h, c3);
    h = std::fma(w, h, c2);
    h = std::fma(w, h, c1);
    return std::fma(w, h, 1.0f);
}
// d/du of asin(u)/u from the same series (both precisions; it only enters the
// Jacobian): u * sum_n 2n c_n u^(2n-2).
template <class T>
T asin_over_deriv(T u) {
    const T w = u * u;
    const T d1 = (T)(2.0 / 6.0), d2 = (T)(12.0 / 40.0), d3 = (T)(30.0 / 112.0), d4 = (T)(280.0 / 1152.0),
            d5 = (T)(630.0 / 2816.0), d6 = (T)(2772.0 / 13312.0);
    T h = std::fma(w, d6, d5);
    h = std::fma(w, h, d4);
    h = std::fma(w, h, d3);
    h = std::fma(w, h, d2);
    h = std::fma(w, h, d1);
    return u * h;
}

// Helix step x1 -> x2 in a uniform field along z (Section 3 uses the full field;
// here Bx = By = 0). The turning rate is d(sin phi)/dx = kB * q/pT; y moves by
// dx * tan of the mean direction, z by tan(lambda) times the arc length, which
// is the signed chord times asin(u)/u with u = curvature * chord / 2.
// Returns false (state untouched) if |sin phi| leaves the guard or u is too big.
template <class T>
bool propagate(State<T>& s, T x1, T x2, const Consts<T>& k) {
    const T one = (T)1, half = (T)0.5;
    const T dx = x2 - x1;
    const T s1 = s.p[2];
    const T kq = k.kB * s.p[4];
    const T s2 = std::fma(kq, dx, s1);
    if (!(std::fabs(s2) < k.sinphi_max)) return false;
    const T c1 = std::sqrt(std::fma(-s1, s1, one));
    const T c2 = std::sqrt(std::fma(-s2, s2, one));
    const T tt = (s1 + s2) / (c1 + c2);      // tan of the mean direction
    const T w = std::fma(tt, tt, one);
    const T lc = dx * std::sqrt(w);           // signed chord
    const T u = (kq * lc) * half;
    if (!(u * u <= k.u_max2)) return false;
    const T g = asin_over(u);
    const T arc = lc * g;
    const T t = s.p[3];
    // Jacobian F (identity plus these entries), the derivative of this step:
    // d tan(mean dir) = (1 + tt^2) (dphi1 + dphi2) / 2 with dphi = d(sin phi) / cos,
    // d arc / d sin(phi1) = dx tt / (c1 c2), and for q/pT the chord and u terms.
    const T ic1 = one / c1, ic2 = one / c2;
    const T f02 = ((dx * w) * (ic1 + ic2)) * half;
    const T f04 = ((dx * w) * ((k.kB * dx) * ic2)) * half;
    const T f12 = t * ((dx * tt) * (ic1 * ic2));
    const T f13 = arc;
    const T dlc = (((k.kB * dx) * lc) * tt) * (half * ic2);  // d chord / d(q/pT)
    const T du = std::fma(k.kB, lc, kq * dlc) * half;      // d u / d(q/pT)
    const T f14 = t * std::fma(dlc, g, (lc * asin_over_deriv(u)) * du);
    const T f24 = k.kB * dx;
    s.p[0] = std::fma(dx, tt, s.p[0]);
    s.p[1] = std::fma(t, arc, s.p[1]);
    s.p[2] = s2;
    // C <- F C F^T: first B = F C (full 5x5), then the lower triangle of B F^T.
    T Cf[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Cf[i][j] = s.C[pk(i, j)];
    T B[5][5];
    for (int j = 0; j < 5; ++j) {
        B[0][j] = std::fma(f04, Cf[4][j], std::fma(f02, Cf[2][j], Cf[0][j]));
        B[1][j] = std::fma(f14, Cf[4][j], std::fma(f13, Cf[3][j], std::fma(f12, Cf[2][j], Cf[1][j])));
        B[2][j] = std::fma(f24, Cf[4][j], Cf[2][j]);
        B[3][j] = Cf[3][j];
        B[4][j] = Cf[4][j];
    }
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j <= i; ++j) {
            T v;
            if (j == 0) v = std::fma(f04, B[i][4], std::fma(f02, B[i][2], B[i][0]));
            else if (j == 1) v = std::fma(f14, B[i][4], std::fma(f13, B[i][3], std::fma(f12, B[i][2], B[i][1])));
            else if (j == 2) v = std::fma(f24, B[i][4], B[i][2]);
            else v = B[i][j];
            s.C[pk(i, j)] = v;
        }
    }
    return true;
}

// Rotation of the state into the frame of a neighbouring sector (the second
// phase of Section 2 merges segments across sectors; Section 4: the refit
// follows the helix through arbitrary rotations). The frame turns by d
// (cos d = ca, sin d = sa): the point (x, y) becomes (x ca + y sa, -x sa + y ca),
// the direction angle phi becomes phi - d; z, tan lambda and q/pT are frame
// independent. The new state is taken at the new x of the point. Covariance:
// with the new reference plane fixed, a shift dy of the point moves it by
// (dy sa, dy ca) in the new frame; going back along the track (direction phi'
// in the new frame) to the plane changes y' by dy ca - dy sa tan phi' =
// dy cos phi / cos phi', z' by -dy sa tan(lambda) / cos phi' and, along the
// curved path, sin phi' by -c sa dy (c = kB q/pT the curvature); a change of
// sin phi gives d sin phi' = (cos phi' / cos phi) d sin phi. Fails (state
// unchanged) unless the track still moves outward in the new frame with
// |sin phi'| below the guard.
template <class T>
bool rotate(State<T>& s, T& x, T ca, T sa, const Consts<T>& k) {
    const T one = (T)1;
    const T sf = s.p[2];
    const T cf = std::sqrt(std::fma(-sf, sf, one));
    const T sn = std::fma(sf, ca, -(cf * sa));
    const T cn = std::fma(cf, ca, sf * sa);
    if (!(cn > (T)0) || !(std::fabs(sn) < k.sinphi_max)) return false;
    const T xn = std::fma(x, ca, s.p[0] * sa);
    const T yn = std::fma(-x, sa, s.p[0] * ca);
    const T icn = one / cn;
    const T j00 = cf * icn;
    const T j10 = -((sa * s.p[3]) * icn);
    const T j20 = -((k.kB * s.p[4]) * sa);
    const T j22 = cn / cf;
    // C' = J C J^T; J is the identity except rows 0, 1, 2 (y', z', sin phi'),
    // whose entries are j00 (y), j10 and 1 (y, z), j20 and j22 (y, sin phi).
    T Cf[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) Cf[i][j] = s.C[pk(i, j)];
    T B[5][5];  // J C
    for (int j = 0; j < 5; ++j) {
        B[0][j] = j00 * Cf[0][j];
        B[1][j] = std::fma(j10, Cf[0][j], Cf[1][j]);
        B[2][j] = std::fma(j20, Cf[0][j], j22 * Cf[2][j]);
        B[3][j] = Cf[3][j];
        B[4][j] = Cf[4][j];
    }
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j <= i; ++j) {
            T v;
            if (j == 0) v = B[i][0] * j00;
            else if (j == 1) v = std::fma(B[i][0], j10, B[i][1]);
            else if (j == 2) v = std::fma(B[i][0], j20, B[i][2] * j22);
            else v = B[i][j];
            s.C[pk(i, j)] = v;
        }
    }
    x = xn;
    s.p[0] = yn;
    s.p[2] = sn;
    return true;
}

// Predicted chi2 of a measurement (my, mz) with V = diag(vy, vz): r^T S^-1 r,
// S = C[0:2,0:2] + V, with the explicit 2x2 inverse.
template <class T>
struct Innov {
    T a00, a01, a11, r0, r1, chi2;
};

template <class T>
Innov<T> innovation(const State<T>& s, T my, T mz, const Consts<T>& k) {
    const T one = (T)1;
    Innov<T> n;
    const T s00 = s.C[0] + k.vy, s01 = s.C[1], s11 = s.C[2] + k.vz;
    const T det = std::fma(s00, s11, -(s01 * s01));
    const T idet = one / det;
    n.a00 = s11 * idet;
    n.a01 = (-s01) * idet;
    n.a11 = s00 * idet;
    n.r0 = my - s.p[0];
    n.r1 = mz - s.p[1];
    const T w0 = std::fma(n.a00, n.r0, n.a01 * n.r1);
    const T w1 = std::fma(n.a01, n.r0, n.a11 * n.r1);
    n.chi2 = std::fma(n.r0, w0, n.r1 * w1);
    return n;
}

// Kalman update with gain K = C H^T S^-1 (H selects y, z).
template <class T>
void update(State<T>& s, const Innov<T>& n) {
    T c0j[5], c1j[5], K0[5], K1[5];
    for (int j = 0; j < 5; ++j) {
        c0j[j] = s.C[pk(0, j)];
        c1j[j] = s.C[pk(1, j)];
    }
    for (int i = 0; i < 5; ++i) {
        K0[i] = std::fma(c0j[i], n.a00, c1j[i] * n.a01);
        K1[i] = std::fma(c0j[i], n.a01, c1j[i] * n.a11);
    }
    for (int i = 0; i < 5; ++i) s.p[i] = s.p[i] + std::fma(K0[i], n.r0, K1[i] * n.r1);
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) s.C[pk(i, j)] = s.C[pk(i, j)] - std::fma(K0[i], c0j[j], K1[i] * c1j[j]);
}

// Covariance reset at a change of direction or a pass start: keep the
// variances scaled up, drop the correlations.
template <class T>
void reset_cov(State<T>& s, const Consts<T>& k) {
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < i; ++j) s.C[pk(i, j)] = (T)0;
    for (int i = 0; i < 5; ++i) s.C[pk(i, i)] = s.C[pk(i, i)] * k.cov_reset;
}

// ----------------------------------------------------------------------------
struct Input {
    int32_t n_inst;
    const int32_t* inst_sector;
    const int64_t* row_start;  // [n_inst * n_rows + 1]
    const float* y;
    const float* z;
};

template <class T>
struct Result {
    using value_type = T;
    int n_rows = 0;
    // grid
    std::vector<int32_t> sorted_id;   // [N] input id at each sorted position
    std::vector<int32_t> bin_start;   // [N + n_seg + 1]; segment s at row_start[s] + s
    std::vector<int32_t> g_ny, g_nz;  // [n_seg]
    std::vector<T> g_ymin, g_zmin, g_invy, g_invz;
    // CA (input-id space)
    std::vector<int32_t> up, dn, upc, dnc;
    // starts and tracklets (global order: instance, row, input id)
    std::vector<int32_t> start_hit, start_inst, start_tid;
    std::vector<int32_t> tl_nhits, tl_rowhit;  // rowhit [N_s * n_rows], -1 = none
    std::vector<T> tl_state;                  // [N_s * 20]: p[5], C[15]
    std::vector<int32_t> tl_row;              // row of the state
    std::vector<uint32_t> weight;             // [N]
    // selected tracks (instance, tid order)
    std::vector<int32_t> sel_tl;              // tracklet index
    std::vector<int64_t> sel_hit_start;       // CSR over owned hits (ascending row)
    std::vector<int32_t> sel_hit;             // input ids
    std::vector<uint8_t> sel_mask;            // refit accept bits per owned hit (b0,b1,b2 = pass 1..3)
    std::vector<int32_t> sel_status;          // 1 = output track, 0 = dropped
    // output tracks
    std::vector<int32_t> trk_inst, trk_sel, trk_ndf;
    std::vector<T> trk_x, trk_alpha, trk_param, trk_cov, trk_chi2;
    std::vector<int64_t> trk_hit_start;
    std::vector<int32_t> trk_hit;
    std::vector<T> trk_state2;                // [n_t * 20] state after the outward pass
    std::vector<int32_t> trk_row, trk_row2;   // rows of the output state and of state2
    double chi2_total = 0;
    // cross-sector merge (filled by merge_tracks)
    std::vector<int32_t> mrg_next;            // [n_t] outer partner track (-1: none)
    std::vector<int32_t> mrg_src;             // per merged track: first (head) sector track
    std::vector<int32_t> mrg_nseg;            // per merged track: segments
    std::vector<int32_t> mrg_inst, mrg_ndf;
    std::vector<T> mrg_x, mrg_alpha, mrg_param, mrg_cov, mrg_chi2;
    std::vector<int64_t> mrg_hit_start;
    std::vector<int32_t> mrg_hit;
    int64_t ndf_total = 0;
};

// ------------------------------------------------------------------ 1. grid
// Per (instance, row): exact y/z ranges; T = max(1, n / hits_per_bin) target
// bins split as ny ~ sqrt(T * Ly / Lz), nz = T / ny; bin = bz * ny + by with
// b = min(n - 1, trunc((v - vmin) * n / L)); stable counting sort by
// (bin, input order).
template <class T>
void build_grid(const Input& in, const Consts<T>& k, Result<T>& R, int64_t seg) {
    const int64_t a = in.row_start[seg], b = in.row_start[seg + 1];
    const int64_t n = b - a;
    int32_t* bs = R.bin_start.data() + a + seg;
    if (n == 0) {
        R.g_ny[seg] = R.g_nz[seg] = 1;
        R.g_ymin[seg] = R.g_zmin[seg] = R.g_invy[seg] = R.g_invz[seg] = (T)0;
        bs[0] = 0;  // single empty bin
        bs[1] = 0;
        return;
    }
    T ymin = (T)in.y[a], ymax = ymin, zmin = (T)in.z[a], zmax = zmin;
    for (int64_t i = a; i < b; ++i) {
        ymin = std::min(ymin, (T)in.y[i]); ymax = std::max(ymax, (T)in.y[i]);
        zmin = std::min(zmin, (T)in.z[i]); zmax = std::max(zmax, (T)in.z[i]);
    }
    const T ly = ymax - ymin, lz = zmax - zmin;
    const int tb = std::max<int64_t>(1, n / k.hpb);
    int ny, nz;
    if (ly > (T)0 && lz > (T)0) {
        const T f = std::sqrt((T)tb * (ly / lz));
        ny = (f >= (T)tb) ? tb : std::max(1, (int)f);
    } else if (ly > (T)0) {
        ny = tb;
    } else {
        ny = 1;
    }
    nz = std::max(1, tb / ny);
    const T invy = ly > (T)0 ? (T)ny / ly : (T)0;
    const T invz = lz > (T)0 ? (T)nz / lz : (T)0;
    R.g_ny[seg] = ny; R.g_nz[seg] = nz;
    R.g_ymin[seg] = ymin; R.g_zmin[seg] = zmin; R.g_invy[seg] = invy; R.g_invz[seg] = invz;
    auto bin_of = [&](T v, T vmin, T inv, int nb) {
        const T t = (v - vmin) * inv;
        if (t >= (T)(nb - 1)) return nb - 1;
        if (t <= (T)0) return 0;
        return (int)t;
    };
    const int nbins = ny * nz;
    std::vector<int32_t> cnt(nbins + 1, 0), bin(n);
    for (int64_t i = 0; i < n; ++i) {
        const int by = bin_of((T)in.y[a + i], ymin, invy, ny);
        const int bz = bin_of((T)in.z[a + i], zmin, invz, nz);
        bin[i] = bz * ny + by;
        cnt[bin[i] + 1]++;
    }
    for (int q = 0; q < nbins; ++q) cnt[q + 1] += cnt[q];
    for (int q = 0; q <= nbins; ++q) bs[q] = cnt[q];
    for (int64_t i = 0; i < n; ++i) R.sorted_id[a + cnt[bin[i]]++] = (int32_t)(a + i);
}

// ------------------------------------------------------ 2. neighbour links
// For hit h on row r (1 <= r <= n_rows - 2): candidates u on r+1 and d on r-1
// inside |dy| <= dx * TY + NY, |dz| <= dx * TZ + NZ; the pair whose linear
// interpolation at X_r misses h by the least squared distance wins, ties by
// (id_u, id_d); no link if that score exceeds the cut.
template <class T>
void find_links(const Input& in, const Consts<T>& k, Result<T>& R, int inst) {
    const int nr = k.n_rows;
    for (int r = 1; r + 1 < nr; ++r) {
        const int64_t seg = (int64_t)inst * nr + r;
        const int64_t a = in.row_start[seg], b = in.row_start[seg + 1];
        const int64_t ua = in.row_start[seg + 1], ub = in.row_start[seg + 2];
        const int64_t da = in.row_start[seg - 1], db = in.row_start[seg];
        for (int64_t h = a; h < b; ++h) {
            const T yh = (T)in.y[h], zh = (T)in.z[h];
            bool found = false;
            T best = (T)0;
            int64_t bu = -1, bd = -1;
            for (int64_t u = ua; u < ub; ++u) {
                const T yu = (T)in.y[u], zu = (T)in.z[u];
                if (!(std::fabs(yu - yh) <= k.wyu[r] && std::fabs(zu - zh) <= k.wzu[r])) continue;
                for (int64_t d = da; d < db; ++d) {
                    const T yd = (T)in.y[d], zd = (T)in.z[d];
                    if (!(std::fabs(yd - yh) <= k.wyd[r] && std::fabs(zd - zh) <= k.wzd[r])) continue;
                    const T ey = (yd + (yu - yd) * k.tr[r]) - yh;
                    const T ez = (zd + (zu - zd) * k.tr[r]) - zh;
                    const T sc = ey * ey + ez * ez;
                    if (!(sc <= k.smax)) continue;
                    if (!found || sc < best || (sc == best && (u < bu || (u == bu && d < bd)))) {
                        found = true;
                        best = sc;
                        bu = u;
                        bd = d;
                    }
                }
            }
            R.up[h] = (int32_t)bu;
            R.dn[h] = (int32_t)bd;
        }
    }
}

// ------------------------------------------- 3./4. cleaning and start hits
template <class T>
void clean_links(const Input& in, Result<T>& R, int inst, int nr) {
    const int64_t a = in.row_start[(int64_t)inst * nr], b = in.row_start[(int64_t)(inst + 1) * nr];
    for (int64_t h = a; h < b; ++h) {
        const int32_t u = R.up[h], d = R.dn[h];
        R.upc[h] = (u >= 0 && R.dn[u] == h) ? u : -1;
        R.dnc[h] = (d >= 0 && R.up[d] == h) ? d : -1;
    }
}

// ------------------------------------------------------------ 5. tracklets
struct Pick {
    int32_t row;
    int32_t hit;
};

// Best hit on a row for the predicted state: inside NSIG * sqrt(S_ii) in y and
// z, predicted chi2 <= cut, minimum chi2, ties to the smaller input id.
template <class T>
int64_t pick_on_row(const Input& in, const Consts<T>& k, const State<T>& s, int64_t seg, Innov<T>* out) {
    const T s00 = s.C[0] + k.vy, s11 = s.C[2] + k.vz;
    const T wy = k.nsig * std::sqrt(s00), wz = k.nsig * std::sqrt(s11);
    int64_t best = -1;
    Innov<T> bi{};
    for (int64_t c = in.row_start[seg]; c < in.row_start[seg + 1]; ++c) {
        const Innov<T> n = innovation(s, (T)in.y[c], (T)in.z[c], k);
        if (!(std::fabs(n.r0) <= wy && std::fabs(n.r1) <= wz)) continue;
        if (!(n.chi2 <= k.chi2_pick)) continue;
        if (best < 0 || n.chi2 < bi.chi2) {  // equal chi2: the earlier (smaller) id stays
            best = c;
            bi = n;
        }
    }
    if (best >= 0) *out = bi;
    return best;
}

// Seed from a chain h_0..h_{L-1} (rows r0..r0+L-1): circle through the first,
// middle and last hit in (x, y) gives the curvature and sin(phi) at h_0; the
// z slope over the arc gives tan(lambda).
template <class T>
bool seed_state(const Consts<T>& k, T x0, T y0, T z0, T xm, T ym, T xe, T ye, T ze, State<T>& s) {
    const T one = (T)1, half = (T)0.5, two = (T)2;
    const T ax = xm - x0, ay = ym - y0, bx = xe - x0, by = ye - y0, cx = xe - xm, cy = ye - ym;
    const T cr = ax * by - ay * bx;
    const T d01 = std::sqrt(ax * ax + ay * ay);
    const T d02 = std::sqrt(bx * bx + by * by);
    const T d12 = std::sqrt(cx * cx + cy * cy);
    const T kap = (two * cr) / ((d01 * d02) * d12);
    T v = (kap * d02) * half;
    if (v > one) v = one;
    if (v < -one) v = -one;
    const T sn = by / d02, cs = bx / d02;
    const T s0 = sn * std::sqrt(one - v * v) - cs * v;
    const T arc = d02 * asin_over(v);
    const T t0 = (ze - z0) / arc;
    T q0 = (k.kB != (T)0) ? kap / k.kB : (T)0;
    if (q0 > k.q_max) q0 = k.q_max;
    if (q0 < -k.q_max) q0 = -k.q_max;
    if (!(std::fabs(s0) < k.sinphi_max)) return false;
    s.p[0] = y0; s.p[1] = z0; s.p[2] = s0; s.p[3] = t0; s.p[4] = q0;
    for (int i = 0; i < 15; ++i) s.C[i] = (T)0;
    for (int i = 0; i < 5; ++i) s.C[pk(i, i)] = k.c0[i];
    return true;
}

template <class T>
void build_tracklet(const Input& in, const Consts<T>& k, Result<T>& R, int64_t sidx) {
    const int nr = k.n_rows;
    const int inst = R.start_inst[sidx];
    const int64_t seg0 = (int64_t)inst * nr;
    int32_t* rowhit = R.tl_rowhit.data() + sidx * nr;
    for (int r = 0; r < nr; ++r) rowhit[r] = -1;
    R.tl_nhits[sidx] = 0;
    R.tl_row[sidx] = -1;
    // chain via the cleaned up-links
    std::vector<int32_t> chain;
    for (int32_t h = R.start_hit[sidx]; h >= 0; h = R.upc[h]) chain.push_back(h);
    const int L = (int)chain.size();
    auto row_of = [&](int64_t h) {
        return (int)(std::upper_bound(in.row_start + seg0, in.row_start + seg0 + nr + 1, (int64_t)h) -
                     (in.row_start + seg0)) - 1;
    };
    const int r0 = row_of(chain[0]);
    const int m = (L - 1) / 2, e = L - 1;
    State<T> s;
    const int32_t h0 = chain[0], hm = chain[m], he = chain[e];
    if (!seed_state(k, k.X[r0], (T)in.y[h0], (T)in.z[h0], k.X[r0 + m], (T)in.y[hm], k.X[r0 + e], (T)in.y[he],
                    (T)in.z[he], s))
        return;
    // stage 1: simplified filter over the chain, no gating
    for (int i = 0; i < L; ++i) {
        if (i > 0 && !propagate(s, k.X[r0 + i - 1], k.X[r0 + i], k)) return;
        const Innov<T> n = innovation(s, (T)in.y[chain[i]], (T)in.z[chain[i]], k);
        update(s, n);
    }
    // stage 2: outward following
    int cur = r0 + e, last = r0 + e, miss = 0;
    for (int r = cur + 1; r < nr && miss < k.max_miss; ++r) {
        if (!propagate(s, k.X[r - 1], k.X[r], k)) break;
        cur = r;
        Innov<T> n;
        if (pick_on_row(in, k, s, seg0 + r, &n) >= 0) {
            update(s, n);
            last = r;
            miss = 0;
        } else {
            ++miss;
        }
    }
    // The state at the end of the outward following is the tracklet's output:
    // the refit starts from it.
    const State<T> s_out = s;
    const int row_out = cur;
    // turn, stage 3: inward through the seed, re-picking every row
    reset_cov(s, k);
    bool ok = true;
    for (int r = cur - 1; r >= last; --r) {
        if (!propagate(s, k.X[r + 1], k.X[r], k)) { ok = false; break; }
        cur = r;
    }
    int nh = 0;
    if (ok) {
        miss = 0;
        for (int r = last; r >= 0; --r) {
            if (r != cur) {
                if (!propagate(s, k.X[cur], k.X[r], k)) break;
                cur = r;
            }
            Innov<T> n;
            const int64_t c = pick_on_row(in, k, s, seg0 + r, &n);
            if (c >= 0) {
                update(s, n);
                rowhit[r] = (int32_t)c;
                ++nh;
                miss = 0;
            } else if (++miss >= k.max_miss) {
                break;
            }
        }
    }
    R.tl_nhits[sidx] = nh;
    R.tl_row[sidx] = row_out;
    T* st = R.tl_state.data() + sidx * 20;
    for (int i = 0; i < 5; ++i) st[i] = s_out.p[i];
    for (int i = 0; i < 15; ++i) st[5 + i] = s_out.C[i];
}

// ---------------------------------------------------------------- 7. refit
// Three passes inward, outward, inward over the hit rows, each starting with a
// covariance reset; a hit whose predicted chi2 exceeds the cut is skipped in
// that pass. Propagation is row by row. With `replay` set the accept decisions
// are read from it instead of being taken (FP64 replay of an FP32 result).
template <class T>
struct RefitOut {
    bool ok;
    State<T> s;
    T chi2;
    int nacc;
    int row;     // row of the output state (innermost hit)
    State<T> s2; // state after the outward pass (at the outermost hit), absolute y and z
    int row2;
};

// The refit carries y and z as offsets from a reference point that moves to
// each accepted cluster, so that binary32 residuals are formed from small
// numbers (the paper keeps parameters at coordinates where single precision
// stays accurate, Section 4).
template <class T>
RefitOut<T> refit(const Consts<T>& k, State<T> s, int row, int n, const int32_t* rows, const T* ys, const T* zs,
                  uint8_t* masks, const uint8_t* replay) {
    RefitOut<T> o{};
    o.ok = false;
    T ref_y = s.p[0], ref_z = s.p[1];
    s.p[0] = (T)0;
    s.p[1] = (T)0;
    int cur = row;
    auto move_to = [&](int target) {
        while (cur != target) {
            const int nx = cur < target ? cur + 1 : cur - 1;
            if (!propagate(s, k.X[cur], k.X[nx], k)) return false;
            cur = nx;
        }
        return true;
    };
    if (n <= 0 || !move_to(rows[n - 1])) return o;
    for (int i = 0; i < n; ++i) masks[i] = 0;
    T chi2sum = (T)0;
    int nacc = 0;
    for (int pass = 0; pass < 3; ++pass) {
        reset_cov(s, k);
        const bool inward = (pass != 1);
        for (int q = 0; q < n; ++q) {
            const int i = inward ? n - 1 - q : q;
            if (!move_to(rows[i])) return o;
            const Innov<T> in = innovation(s, ys[i] - ref_y, zs[i] - ref_z, k);
            const bool acc = replay ? ((replay[i] >> pass) & 1) != 0 : (in.chi2 <= k.chi2_rej);
            if (acc) {
                update(s, in);
                s.p[0] = s.p[0] + (ref_y - ys[i]);  // re-centre on the accepted cluster
                s.p[1] = s.p[1] + (ref_z - zs[i]);
                ref_y = ys[i];
                ref_z = zs[i];
                masks[i] |= (uint8_t)(1u << pass);
                if (pass == 2) {
                    chi2sum = chi2sum + in.chi2;
                    ++nacc;
                }
            }
        }
        if (pass == 1) {  // the outward pass ends at the outermost hit: the state there
            o.s2 = s;
            o.s2.p[0] = ref_y + s.p[0];
            o.s2.p[1] = ref_z + s.p[1];
            o.row2 = cur;
        }
    }
    s.p[0] = ref_y + s.p[0];
    s.p[1] = ref_z + s.p[1];
    o.ok = true;
    o.s = s;
    o.chi2 = chi2sum;
    o.nacc = nacc;
    o.row = cur;
    return o;
}

// ----------------------------------------------------------------- driver
template <class T>
void run_instance_ca(const Input& in, const Consts<T>& k, Result<T>& R, int inst) {
    const int nr = k.n_rows;
    for (int r = 0; r < nr; ++r) build_grid(in, k, R, (int64_t)inst * nr + r);
    find_links(in, k, R, inst);
}

template <class T>
Result<T>* run(const orc_params& p, const Input& in) {
    const Consts<T> k(p);
    const int nr = k.n_rows;
    auto* R = new Result<T>;
    R->n_rows = nr;
    const int64_t nseg = (int64_t)in.n_inst * nr;
    const int64_t N = in.row_start[nseg];
    R->sorted_id.assign(N, -1);
    R->bin_start.assign(N + nseg + 1, 0);
    R->g_ny.assign(nseg, 0); R->g_nz.assign(nseg, 0);
    R->g_ymin.assign(nseg, 0); R->g_zmin.assign(nseg, 0); R->g_invy.assign(nseg, 0); R->g_invz.assign(nseg, 0);
    R->up.assign(N, -1); R->dn.assign(N, -1); R->upc.assign(N, -1); R->dnc.assign(N, -1);
    R->weight.assign(N, 0);
    const int nthreads = std::max(1, p.n_threads);
    auto parallel_over = [&](int64_t count, auto fn) {
        if (nthreads == 1 || count < 2) {
            for (int64_t i = 0; i < count; ++i) fn(i);
            return;
        }
        std::vector<std::thread> th;
        for (int t = 0; t < nthreads; ++t)
            th.emplace_back([&, t]() {
                for (int64_t i = t; i < count; i += nthreads) fn(i);
            });
        for (auto& x : th) x.join();
    };
    parallel_over(in.n_inst, [&](int64_t i) { run_instance_ca(in, k, *R, (int)i); });
    parallel_over(in.n_inst, [&](int64_t i) { clean_links(in, *R, (int)i, nr); });
    // start hits, ordered by (instance, row, input id)
    for (int inst = 0; inst < in.n_inst; ++inst) {
        int32_t tid = 0;
        const int64_t a = in.row_start[(int64_t)inst * nr], b = in.row_start[(int64_t)(inst + 1) * nr];
        for (int64_t h = a; h < b; ++h) {
            const int32_t u = R->upc[h];
            if (R->dnc[h] == -1 && u != -1 && R->upc[u] != -1) {
                R->start_hit.push_back((int32_t)h);
                R->start_inst.push_back(inst);
                R->start_tid.push_back(tid++);
            }
        }
    }
    const int64_t ns = (int64_t)R->start_hit.size();
    R->tl_nhits.assign(ns, 0);
    R->tl_row.assign(ns, -1);
    R->tl_rowhit.assign(ns * nr, -1);
    R->tl_state.assign(ns * 20, 0);
    parallel_over(ns, [&](int64_t i) { build_tracklet(in, k, *R, i); });
    // weights: max over tracklets of (nHits << 20) | (0xFFFFF - tid)
    for (int64_t i = 0; i < ns; ++i) {
        const int nh = R->tl_nhits[i];
        if (nh < k.n_min) continue;
        const uint32_t w = ((uint32_t)nh << 20) | (uint32_t)(0xFFFFF - R->start_tid[i]);
        for (int r = 0; r < nr; ++r) {
            const int32_t h = R->tl_rowhit[i * nr + r];
            if (h >= 0) R->weight[h] = std::max(R->weight[h], w);
        }
    }
    // selection
    R->sel_hit_start.push_back(0);
    for (int64_t i = 0; i < ns; ++i) {
        const int nh = R->tl_nhits[i];
        if (nh < k.n_min) continue;
        const uint32_t w = ((uint32_t)nh << 20) | (uint32_t)(0xFFFFF - R->start_tid[i]);
        std::vector<int32_t> own;
        for (int r = 0; r < nr; ++r) {
            const int32_t h = R->tl_rowhit[i * nr + r];
            if (h >= 0 && R->weight[h] == w) own.push_back(h);
        }
        if ((int)own.size() < k.n_min) continue;
        R->sel_tl.push_back((int32_t)i);
        R->sel_hit.insert(R->sel_hit.end(), own.begin(), own.end());
        R->sel_hit_start.push_back((int64_t)R->sel_hit.size());
    }
    // refit
    const int64_t nsel = (int64_t)R->sel_tl.size();
    R->sel_mask.assign(R->sel_hit.size(), 0);
    R->sel_status.assign(nsel, 0);
    std::vector<RefitOut<T>> outs(nsel);
    parallel_over(nsel, [&](int64_t t) {
        const int64_t tl = R->sel_tl[t];
        const int inst = R->start_inst[tl];
        const int64_t a = R->sel_hit_start[t], b = R->sel_hit_start[t + 1];
        const int n = (int)(b - a);
        std::vector<int32_t> rows(n);
        std::vector<T> ys(n), zs(n);
        const int64_t seg0 = (int64_t)inst * nr;
        for (int i = 0; i < n; ++i) {
            const int32_t h = R->sel_hit[a + i];
            rows[i] = (int)(std::upper_bound(in.row_start + seg0, in.row_start + seg0 + nr + 1, (int64_t)h) -
                            (in.row_start + seg0)) - 1;
            ys[i] = (T)in.y[h];
            zs[i] = (T)in.z[h];
        }
        State<T> s;
        const T* st = R->tl_state.data() + tl * 20;
        for (int i = 0; i < 5; ++i) s.p[i] = st[i];
        for (int i = 0; i < 15; ++i) s.C[i] = st[5 + i];
        outs[t] = refit(k, s, R->tl_row[tl], n, rows.data(), ys.data(), zs.data(), R->sel_mask.data() + a, nullptr);
        R->sel_status[t] = (outs[t].ok && outs[t].nacc >= k.n_min) ? 1 : 0;
    });
    R->trk_hit_start.push_back(0);
    for (int64_t t = 0; t < nsel; ++t) {
        if (!R->sel_status[t]) continue;
        const RefitOut<T>& o = outs[t];
        const int64_t tl = R->sel_tl[t];
        const int inst = R->start_inst[tl];
        R->trk_inst.push_back(inst);
        R->trk_sel.push_back((int32_t)t);
        R->trk_x.push_back(k.X[o.row]);
        const int sec = in.inst_sector[inst];
        R->trk_alpha.push_back((T)(((sec % 18) + 0.5) * 20.0 * 3.14159265358979323846 / 180.0));
        for (int i = 0; i < 5; ++i) R->trk_param.push_back(o.s.p[i]);
        for (int i = 0; i < 15; ++i) R->trk_cov.push_back(o.s.C[i]);
        for (int i = 0; i < 5; ++i) R->trk_state2.push_back(o.s2.p[i]);
        for (int i = 0; i < 15; ++i) R->trk_state2.push_back(o.s2.C[i]);
        R->trk_row.push_back(o.row);
        R->trk_row2.push_back(o.row2);
        R->trk_chi2.push_back(o.chi2);
        R->trk_ndf.push_back(2 * o.nacc - 5);
        for (int64_t q = R->sel_hit_start[t]; q < R->sel_hit_start[t + 1]; ++q)
            if (R->sel_mask[q] & 4) R->trk_hit.push_back(R->sel_hit[q]);
        R->trk_hit_start.push_back((int64_t)R->trk_hit.size());
        R->chi2_total += (double)o.chi2;
        R->ndf_total += 2 * o.nacc - 5;
    }
    return R;
}

// ---------------------------------------------------------------- 8. merge
// The second phase of Section 2: the track segments found in the individual
// sectors are merged, then fitted as one track (Section 4: the refit follows
// the helix through rotations between sector frames). Reading of this
// project (the paper gives no procedure): a segment A continues as segment B
// of the same event in a phi-neighbouring sector of the same side when A's
// state after the outward pass, rotated into B's frame and carried to B's
// reference row (from the first row plane outward of the rotated point, row by
// row, at most merge_max_gap rows), agrees with B's fitted state: chi2 of the
// five parameter differences with the summed covariance <= chi2_merge. Pairs
// are kept when each is the other's best (smallest chi2, ties to the smaller
// track index); chains of pairs form merged tracks (a closed loop is opened
// at its smallest track index). A merged track is refitted over all its
// segments' clusters: the same three passes as the sector refit, from the last
// segment's outward state, and between segments the state is rotated into the
// next segment's frame (reference point restarted at the rotated position) and
// carried to the first row plane towards the target before the row steps.

// chi2 of d = b - a with covariance Ca + Cb (LDL^T, fixed order); false if
// the summed covariance is not positive definite or if the z or tan(lambda)
// difference alone already exceeds `cut` (a quadratic form is at least any of
// its one-parameter marginals, so such a pair is rejected before the solve).
template <class T>
bool pair_chi2(const State<T>& a, const State<T>& b, T cut, T& chi2) {
    T C[5][5], L[5][5], D[5], d[5], zz[5];
    for (int i = 0; i < 5; ++i) {
        d[i] = b.p[i] - a.p[i];
        for (int j = 0; j <= i; ++j) C[i][j] = a.C[pk(i, j)] + b.C[pk(i, j)];
    }
    if (!(d[1] * d[1] <= cut * C[1][1]) || !(d[3] * d[3] <= cut * C[3][3])) return false;
    for (int j = 0; j < 5; ++j) {
        T v = C[j][j];
        for (int q = 0; q < j; ++q) v = v - (L[j][q] * L[j][q]) * D[q];
        if (!(v > (T)0)) return false;
        D[j] = v;
        for (int i = j + 1; i < 5; ++i) {
            T w = C[i][j];
            for (int q = 0; q < j; ++q) w = w - (L[i][q] * L[j][q]) * D[q];
            L[i][j] = w / v;
        }
    }
    T c = (T)0;
    for (int i = 0; i < 5; ++i) {
        T v = d[i];
        for (int q = 0; q < i; ++q) v = v - L[i][q] * zz[q];
        zz[i] = v;
        c = c + (v * v) / D[i];
    }
    chi2 = c;
    return true;
}

// rotation direction from sector sa to sector sb (phi-neighbours of one side):
// +1 if sb is the next sector counter-clockwise, -1 the previous, 0 otherwise
inline int sector_step(int sa, int sb) {
    if (sa / 18 != sb / 18) return 0;
    const int a = sa % 18, b = sb % 18;
    if (b == (a + 1) % 18) return 1;
    if (a == (b + 1) % 18) return -1;
    return 0;
}

// first row plane at or beyond x (dir > 0) or at or before x (dir < 0); -1 if none
template <class T>
int plane_towards(const Consts<T>& k, T x, int dir) {
    if (dir > 0) {
        for (int r = 0; r < k.n_rows; ++r)
            if (k.X[r] >= x) return r;
    } else {
        for (int r = k.n_rows - 1; r >= 0; --r)
            if (k.X[r] <= x) return r;
    }
    return -1;
}

// chi2 of segment A continuing as segment B (rotation step dir), or false
template <class T>
bool match_pair(const Consts<T>& k, const Result<T>& R, int64_t a, int64_t b, int dir, T& chi2) {
    State<T> s;
    for (int i = 0; i < 5; ++i) s.p[i] = R.trk_state2[a * 20 + i];
    for (int i = 0; i < 15; ++i) s.C[i] = R.trk_state2[a * 20 + 5 + i];
    T x = k.X[R.trk_row2[a]];
    if (!rotate(s, x, k.rot_c, dir > 0 ? k.rot_s : -k.rot_s, k)) return false;
    const int r1 = plane_towards(k, x, +1);
    const int rb = R.trk_row[b];
    if (r1 < 0 || rb < r1 || rb > r1 + k.merge_max_gap) return false;
    if (!propagate(s, x, k.X[r1], k)) return false;
    for (int r = r1; r < rb; ++r)
        if (!propagate(s, k.X[r], k.X[r + 1], k)) return false;
    State<T> sb;
    for (int i = 0; i < 5; ++i) sb.p[i] = R.trk_param[b * 5 + i];
    for (int i = 0; i < 15; ++i) sb.C[i] = R.trk_cov[b * 15 + i];
    return pair_chi2(s, sb, k.chi2_merge, chi2);
}

constexpr int kMaxChain = 8;  // segments of one merged track; a longer chain is cut after the eighth

template <class T>
struct MergedHit {
    int row, frame;
    T y, z;
    int32_t id;
};

// Three-pass refit of a merged track (hits in order along the track, frames
// 0..nf-1 with dirs[f] the rotation step from frame f to f+1), from state s
// (absolute y, z) at row `row` of the last frame. Outputs the state at the
// innermost hit (frame 0), chi2 and the pass-3 accepted hits.
template <class T>
bool refit_merged(const Consts<T>& k, State<T> s, int row, const std::vector<MergedHit<T>>& hits,
                  const std::vector<int>& dirs, State<T>& out, T& chi2_out, int& nacc_out, int& row_out,
                  std::vector<uint8_t>& acc3) {
    const int n = (int)hits.size();
    int frame = hits.empty() ? 0 : hits[n - 1].frame;
    T ref_y = s.p[0], ref_z = s.p[1];
    s.p[0] = (T)0;
    s.p[1] = (T)0;
    int cur = row;
    auto move_to = [&](int target, int tframe) {
        if (tframe != frame) {
            // absolute position, into the neighbouring frame, reference restarted there
            s.p[0] = ref_y + s.p[0];
            s.p[1] = ref_z + s.p[1];
            T x = k.X[cur];
            const int dir = tframe > frame ? dirs[frame] : -dirs[tframe];
            if (!rotate(s, x, k.rot_c, dir > 0 ? k.rot_s : -k.rot_s, k)) return false;
            frame = tframe;
            ref_y = s.p[0];
            ref_z = s.p[1];
            s.p[0] = (T)0;
            s.p[1] = (T)0;
            const int r1 = plane_towards(k, x, k.X[target] >= x ? +1 : -1);
            if (r1 < 0 || !propagate(s, x, k.X[r1], k)) return false;
            cur = r1;
        }
        while (cur != target) {
            const int nx = cur < target ? cur + 1 : cur - 1;
            if (!propagate(s, k.X[cur], k.X[nx], k)) return false;
            cur = nx;
        }
        return true;
    };
    if (n <= 0 || !move_to(hits[n - 1].row, hits[n - 1].frame)) return false;
    acc3.assign(n, 0);
    T chi2sum = (T)0;
    int nacc = 0;
    for (int pass = 0; pass < 3; ++pass) {
        reset_cov(s, k);
        const bool inward = (pass != 1);
        for (int q = 0; q < n; ++q) {
            const int i = inward ? n - 1 - q : q;
            if (!move_to(hits[i].row, hits[i].frame)) return false;
            const Innov<T> in = innovation(s, hits[i].y - ref_y, hits[i].z - ref_z, k);
            if (in.chi2 <= k.chi2_rej) {
                update(s, in);
                s.p[0] = s.p[0] + (ref_y - hits[i].y);
                s.p[1] = s.p[1] + (ref_z - hits[i].z);
                ref_y = hits[i].y;
                ref_z = hits[i].z;
                if (pass == 2) {
                    chi2sum = chi2sum + in.chi2;
                    ++nacc;
                    acc3[i] = 1;
                }
            }
        }
    }
    s.p[0] = ref_y + s.p[0];
    s.p[1] = ref_z + s.p[1];
    out = s;
    chi2_out = chi2sum;
    nacc_out = nacc;
    row_out = cur;
    return frame == 0 && nacc >= k.n_min;
}

template <class T>
void merge_tracks(const Consts<T>& k, const Input& in, const int32_t* inst_event, Result<T>& R) {
    const int64_t nt = (int64_t)R.trk_inst.size();
    const int nr = k.n_rows;
    // instance of each (event, sector): the lowest instance index
    std::vector<std::pair<int64_t, int>> key(in.n_inst);
    for (int i = 0; i < in.n_inst; ++i) key[i] = {(int64_t)inst_event[i] * 64 + in.inst_sector[i], i};
    auto inst_of = [&](int64_t ev, int sec) -> int {
        int best = -1;
        for (int i = 0; i < in.n_inst; ++i)
            if (key[i].first == ev * 64 + sec && (best < 0 || i < best)) best = i;
        return best;
    };
    // tracks of each instance: [first, last) in output order
    std::vector<int64_t> tfirst(in.n_inst + 1, nt);
    for (int64_t t = nt - 1; t >= 0; --t) tfirst[R.trk_inst[t]] = t;
    std::vector<int64_t> tend(in.n_inst, 0);
    for (int64_t t = 0; t < nt; ++t) tend[R.trk_inst[t]] = t + 1;
    auto candidates = [&](int64_t t, int side_dir, auto fn) {
        // side_dir +1: tracks that may continue t outward (t is A); -1: tracks t may continue (t is B)
        const int inst = R.trk_inst[t];
        // an instance that is not the lowest of its (event, sector) takes no part
        if (inst_of(inst_event[inst], in.inst_sector[inst]) != inst) return;
        const int sec = in.inst_sector[inst], side = sec / 18, phi = sec % 18;
        for (int dir = -1; dir <= 1; dir += 2) {
            const int nsec = side * 18 + (phi + dir + 18) % 18;
            const int j = inst_of(inst_event[inst], nsec);
            if (j < 0 || j == inst || tend[j] <= tfirst[j]) continue;
            for (int64_t u = tfirst[j]; u < tend[j]; ++u) {
                if (R.trk_inst[u] != j) continue;
                fn(u, side_dir > 0 ? dir : -dir);
            }
        }
    };
    std::vector<int64_t> best_out(nt, -1), best_in(nt, -1);
    for (int64_t a = 0; a < nt; ++a) {
        T bc = (T)0;
        candidates(a, +1, [&](int64_t b, int dir) {
            T c;
            if (!match_pair(k, R, a, b, dir, c) || !(c <= k.chi2_merge)) return;
            if (best_out[a] < 0 || c < bc || (c == bc && b < best_out[a])) {
                best_out[a] = b;
                bc = c;
            }
        });
    }
    for (int64_t b = 0; b < nt; ++b) {
        T bc = (T)0;
        candidates(b, -1, [&](int64_t a, int dir) {
            T c;
            // a continues as b: a's frame turns by -dir' where dir' is b -> a
            if (!match_pair(k, R, a, b, dir, c) || !(c <= k.chi2_merge)) return;
            if (best_in[b] < 0 || c < bc || (c == bc && a < best_in[b])) {
                best_in[b] = a;
                bc = c;
            }
        });
    }
    R.mrg_next.assign(nt, -1);
    std::vector<int64_t> prev(nt, -1);
    for (int64_t a = 0; a < nt; ++a) {
        const int64_t b = best_out[a];
        if (b >= 0 && best_in[b] == a) {
            R.mrg_next[a] = (int32_t)b;
            prev[b] = a;
        }
    }
    // a closed loop is opened at its smallest track index
    for (int64_t t = 0; t < nt; ++t) {
        if (prev[t] < 0) continue;
        int64_t u = prev[t], m = t;
        int steps = 0;
        while (u >= 0 && u != t && steps++ < 64) {
            m = std::min(m, u);
            u = prev[u];
        }
        if (u == t) {
            R.mrg_next[prev[m]] = -1;
            prev[m] = -1;
        }
    }
    // merged tracks in the order of their first segment
    R.mrg_hit_start.assign(1, 0);
    auto emit = [&](int32_t src, int nseg, int inst, T x, T alpha, const State<T>& s, T chi2, int ndf,
                    const std::vector<int32_t>& hits) {
        R.mrg_src.push_back(src);
        R.mrg_nseg.push_back(nseg);
        R.mrg_inst.push_back(inst);
        R.mrg_x.push_back(x);
        R.mrg_alpha.push_back(alpha);
        for (int i = 0; i < 5; ++i) R.mrg_param.push_back(s.p[i]);
        for (int i = 0; i < 15; ++i) R.mrg_cov.push_back(s.C[i]);
        R.mrg_chi2.push_back(chi2);
        R.mrg_ndf.push_back(ndf);
        R.mrg_hit.insert(R.mrg_hit.end(), hits.begin(), hits.end());
        R.mrg_hit_start.push_back((int64_t)R.mrg_hit.size());
    };
    auto emit_single = [&](int64_t t) {
        State<T> s;
        for (int i = 0; i < 5; ++i) s.p[i] = R.trk_param[t * 5 + i];
        for (int i = 0; i < 15; ++i) s.C[i] = R.trk_cov[t * 15 + i];
        std::vector<int32_t> h(R.trk_hit.begin() + R.trk_hit_start[t], R.trk_hit.begin() + R.trk_hit_start[t + 1]);
        emit((int32_t)t, 1, R.trk_inst[t], R.trk_x[t], R.trk_alpha[t], s, R.trk_chi2[t], R.trk_ndf[t], h);
    };
    // refit every chain first; a chain whose refit fails leaves its segments
    // as sector tracks. Output in track order: a merged track at its first
    // segment, the other segments of a merged chain omitted.
    struct Merged {
        bool ok = false;
        int nseg = 0;
        State<T> s;
        T chi2;
        int ndf, row;
        std::vector<int32_t> hits;
    };
    std::vector<Merged> mg(nt);
    std::vector<uint8_t> absorbed(nt, 0);
    for (int64_t t = 0; t < nt; ++t) {
        if (prev[t] >= 0 || R.mrg_next[t] < 0) continue;  // not the first segment of a chain
        std::vector<int64_t> chain;
        for (int64_t u = t; u >= 0 && (int)chain.size() < kMaxChain; u = R.mrg_next[u]) chain.push_back(u);
        std::vector<MergedHit<T>> hits;
        std::vector<int> dirs;
        for (size_t f = 0; f < chain.size(); ++f) {
            const int64_t u = chain[f];
            const int inst = R.trk_inst[u];
            const int64_t seg0 = (int64_t)inst * nr;
            for (int64_t q = R.trk_hit_start[u]; q < R.trk_hit_start[u + 1]; ++q) {
                const int32_t h = R.trk_hit[q];
                const int row = (int)(std::upper_bound(in.row_start + seg0, in.row_start + seg0 + nr + 1,
                                                       (int64_t)h) - (in.row_start + seg0)) - 1;
                hits.push_back({row, (int)f, (T)in.y[h], (T)in.z[h], h});
            }
            if (f + 1 < chain.size())
                dirs.push_back(sector_step(in.inst_sector[inst], in.inst_sector[R.trk_inst[chain[f + 1]]]));
        }
        const int64_t tail = chain.back();
        State<T> s;
        for (int i = 0; i < 5; ++i) s.p[i] = R.trk_state2[tail * 20 + i];
        for (int i = 0; i < 15; ++i) s.C[i] = R.trk_state2[tail * 20 + 5 + i];
        State<T> out;
        T chi2;
        int nacc, row;
        std::vector<uint8_t> acc3;
        if (refit_merged(k, s, R.trk_row2[tail], hits, dirs, out, chi2, nacc, row, acc3)) {
            Merged& M = mg[t];
            M.ok = true;
            M.nseg = (int)chain.size();
            M.s = out;
            M.chi2 = chi2;
            M.ndf = 2 * nacc - 5;
            M.row = row;
            for (size_t i = 0; i < hits.size(); ++i)
                if (acc3[i]) M.hits.push_back(hits[i].id);
            for (size_t f = 1; f < chain.size(); ++f) absorbed[chain[f]] = 1;
        }
    }
    for (int64_t t = 0; t < nt; ++t) {
        if (absorbed[t]) continue;
        if (mg[t].ok) {
            const Merged& M = mg[t];
            emit((int32_t)t, M.nseg, R.trk_inst[t], k.X[M.row], R.trk_alpha[t], M.s, M.chi2, M.ndf, M.hits);
        } else {
            emit_single(t);
        }
    }
}

struct Handle {
    int prec;  // 32 or 64
    void* r;
};

template <class T>
Result<T>* res(void* h) { return (Result<T>*)((Handle*)h)->r; }

template <class T, class U>
void copy_out(const std::vector<T>& v, U* dst) {
    if (dst)
        for (size_t i = 0; i < v.size(); ++i) dst[i] = (U)v[i];
}

// state: p[5] then C[15] as double (values are rounded to T on load).
template <class T>
void load_state(const double* st, State<T>& s) {
    for (int i = 0; i < 5; ++i) s.p[i] = (T)st[i];
    for (int i = 0; i < 15; ++i) s.C[i] = (T)st[5 + i];
}
template <class T>
void store_state(const State<T>& s, double* st) {
    for (int i = 0; i < 5; ++i) st[i] = (double)s.p[i];
    for (int i = 0; i < 15; ++i) st[5 + i] = (double)s.C[i];
}

}  // namespace

extern "C" {

void* orc_run(const orc_params* p, int32_t precision, int32_t n_inst, const int32_t* inst_sector,
              const int64_t* row_start, const float* y, const float* z) {
    Input in{n_inst, inst_sector, row_start, y, z};
    auto* h = new Handle;
    h->prec = precision;
    if (precision == 32) h->r = run<float>(*p, in);
    else h->r = run<double>(*p, in);
    return h;
}

void orc_free(void* h) {
    if (!h) return;
    Handle* H = (Handle*)h;
    if (H->prec == 32) delete res<float>(h);
    else delete res<double>(h);
    delete H;
}

// sizes: [0] N, [1] n_starts, [2] n_selected, [3] n_selected_hits, [4] n_tracks, [5] n_track_hits
void orc_sizes(void* h, int64_t* s) {
    auto f = [&](auto* R) {
        s[0] = (int64_t)R->up.size();
        s[1] = (int64_t)R->start_hit.size();
        s[2] = (int64_t)R->sel_tl.size();
        s[3] = (int64_t)R->sel_hit.size();
        s[4] = (int64_t)R->trk_inst.size();
        s[5] = (int64_t)R->trk_hit.size();
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

void orc_get_grid(void* h, int32_t* sorted_id, int32_t* bin_start, int32_t* ny, int32_t* nz, double* ymin,
                  double* zmin, double* invy, double* invz) {
    auto f = [&](auto* R) {
        copy_out(R->sorted_id, sorted_id); copy_out(R->bin_start, bin_start);
        copy_out(R->g_ny, ny); copy_out(R->g_nz, nz); copy_out(R->g_ymin, ymin); copy_out(R->g_zmin, zmin);
        copy_out(R->g_invy, invy); copy_out(R->g_invz, invz);
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

void orc_get_links(void* h, int32_t* up, int32_t* dn, int32_t* upc, int32_t* dnc) {
    auto f = [&](auto* R) { copy_out(R->up, up); copy_out(R->dn, dn); copy_out(R->upc, upc); copy_out(R->dnc, dnc); };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

void orc_get_tracklets(void* h, int32_t* start_hit, int32_t* start_inst, int32_t* start_tid, int32_t* nhits,
                       int32_t* rowhit, double* state, int32_t* state_row, uint32_t* weight) {
    auto f = [&](auto* R) {
        copy_out(R->start_hit, start_hit); copy_out(R->start_inst, start_inst); copy_out(R->start_tid, start_tid);
        copy_out(R->tl_nhits, nhits); copy_out(R->tl_rowhit, rowhit); copy_out(R->tl_state, state);
        copy_out(R->tl_row, state_row); copy_out(R->weight, weight);
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

void orc_get_selected(void* h, int32_t* sel_tl, int64_t* hit_start, int32_t* hit, uint8_t* mask, int32_t* status) {
    auto f = [&](auto* R) {
        copy_out(R->sel_tl, sel_tl); copy_out(R->sel_hit_start, hit_start); copy_out(R->sel_hit, hit);
        copy_out(R->sel_mask, mask); copy_out(R->sel_status, status);
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

void orc_get_tracks(void* h, int32_t* inst, int32_t* sel, double* x, double* alpha, double* param, double* cov,
                    double* chi2, int32_t* ndf, int64_t* hit_start, int32_t* hit, double* totals) {
    auto f = [&](auto* R) {
        copy_out(R->trk_inst, inst); copy_out(R->trk_sel, sel); copy_out(R->trk_x, x); copy_out(R->trk_alpha, alpha);
        copy_out(R->trk_param, param); copy_out(R->trk_cov, cov); copy_out(R->trk_chi2, chi2);
        copy_out(R->trk_ndf, ndf); copy_out(R->trk_hit_start, hit_start); copy_out(R->trk_hit, hit);
        if (totals) {
            totals[0] = R->chi2_total;
            totals[1] = (double)R->ndf_total;
        }
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

// Cross-sector merge of the tracks of a finished run (same inputs as orc_run;
// inst_event: the event of each instance). Returns the number of merged tracks.
int64_t orc_merge(void* h, const orc_params* p, int32_t n_inst, const int32_t* inst_sector, const int32_t* inst_event,
                  const int64_t* row_start, const float* y, const float* z) {
    Input in{n_inst, inst_sector, row_start, y, z};
    auto f = [&](auto* R) -> int64_t {
        using T = typename std::remove_pointer<decltype(R)>::type::value_type;
        Consts<T> k(*p);
        R->mrg_src.clear(); R->mrg_nseg.clear(); R->mrg_inst.clear(); R->mrg_ndf.clear(); R->mrg_x.clear();
        R->mrg_alpha.clear(); R->mrg_param.clear(); R->mrg_cov.clear(); R->mrg_chi2.clear();
        R->mrg_hit.clear(); R->mrg_hit_start.clear();
        merge_tracks(k, in, inst_event, *R);
        return (int64_t)R->mrg_src.size();
    };
    return ((Handle*)h)->prec == 32 ? f(res<float>(h)) : f(res<double>(h));
}

// n_hits of the merged tracks
int64_t orc_merged_hits(void* h) {
    auto f = [&](auto* R) -> int64_t { return (int64_t)R->mrg_hit.size(); };
    return ((Handle*)h)->prec == 32 ? f(res<float>(h)) : f(res<double>(h));
}

void orc_get_merged(void* h, int32_t* next, int32_t* src, int32_t* nseg, int32_t* inst, double* x, double* alpha,
                    double* param, double* cov, double* chi2, int32_t* ndf, int64_t* hit_start, int32_t* hit,
                    double* state2) {
    auto f = [&](auto* R) {
        copy_out(R->mrg_next, next); copy_out(R->mrg_src, src); copy_out(R->mrg_nseg, nseg);
        copy_out(R->mrg_inst, inst); copy_out(R->mrg_x, x); copy_out(R->mrg_alpha, alpha);
        copy_out(R->mrg_param, param); copy_out(R->mrg_cov, cov); copy_out(R->mrg_chi2, chi2);
        copy_out(R->mrg_ndf, ndf); copy_out(R->mrg_hit_start, hit_start); copy_out(R->mrg_hit, hit);
        copy_out(R->trk_state2, state2);
    };
    if (((Handle*)h)->prec == 32) f(res<float>(h)); else f(res<double>(h));
}

// ---- primitives (for pinning the oracle against closed forms) -----------
int32_t orc_propagate(const orc_params* p, int32_t precision, double* st, double x1, double x2) {
    auto f = [&](auto zero) -> int32_t {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        load_state(st, s);
        if (!propagate(s, (T)x1, (T)x2, k)) return 0;
        store_state(s, st);
        return 1;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

// Rotate a state (20 values) at local x by the frame angle d; x is updated.
int32_t orc_rotate(const orc_params* p, int32_t precision, double* st, double* x, double d) {
    auto f = [&](auto zero) -> int32_t {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        load_state(st, s);
        T xx = (T)*x;
        if (!rotate(s, xx, (T)std::cos(d), (T)std::sin(d), k)) return 0;
        store_state(s, st);
        *x = (double)xx;
        return 1;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

double orc_update(const orc_params* p, int32_t precision, double* st, double my, double mz) {
    auto f = [&](auto zero) -> double {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        load_state(st, s);
        const Innov<T> n = innovation(s, (T)my, (T)mz, k);
        update(s, n);
        store_state(s, st);
        return (double)n.chi2;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

double orc_asin_over(int32_t precision, double u) {
    return precision == 32 ? (double)asin_over((float)u) : asin_over(u);
}

int32_t orc_seed(const orc_params* p, int32_t precision, const double* pts /* x0 y0 z0 xm ym xe ye ze */,
                 double* st) {
    auto f = [&](auto zero) -> int32_t {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        if (!seed_state(k, (T)pts[0], (T)pts[1], (T)pts[2], (T)pts[3], (T)pts[4], (T)pts[5], (T)pts[6],
                        (T)pts[7], s))
            return 0;
        store_state(s, st);
        return 1;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

// The pick rule of the track following on one row: candidates (ys, zs) of
// the row in input order, the predicted state st (p[5], C[15]). Returns the
// index of the chosen candidate or -1; *chi2 gets its predicted chi2.
int64_t orc_pick(const orc_params* p, int32_t precision, const double* st, int64_t n, const float* ys,
                 const float* zs, double* chi2) {
    auto f = [&](auto zero) -> int64_t {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        load_state(st, s);
        const int64_t rs[2] = {0, n};
        const int32_t sec = 0;
        const Input in{1, &sec, rs, ys, zs};
        Innov<T> out{};
        const int64_t c = pick_on_row(in, k, s, 0, &out);
        if (c >= 0 && chi2) *chi2 = (double)out.chi2;
        return c;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

// Refit of one hit list (rows ascending) from a start state at `row`.
// out: state[20] at the innermost hit; out_scalars: chi2, nacc, row.
// replay (may be NULL): accept bits per hit to reproduce instead of deciding.
int32_t orc_refit(const orc_params* p, int32_t precision, const double* st0, int32_t row, int32_t n,
                  const int32_t* rows, const double* ys, const double* zs, const uint8_t* replay, uint8_t* masks,
                  double* st_out, double* scalars) {
    auto f = [&](auto zero) -> int32_t {
        using T = decltype(zero);
        Consts<T> k(*p);
        State<T> s;
        load_state(st0, s);
        std::vector<T> y(n), z(n);
        for (int i = 0; i < n; ++i) {
            y[i] = (T)ys[i];
            z[i] = (T)zs[i];
        }
        RefitOut<T> o = refit(k, s, row, n, rows, y.data(), z.data(), masks, replay);
        if (!o.ok) return 0;
        store_state(o.s, st_out);
        scalars[0] = (double)o.chi2;
        scalars[1] = (double)o.nacc;
        scalars[2] = (double)o.row;
        return 1;
    };
    return precision == 32 ? f(0.0f) : f(0.0);
}

// FP64 replay of selected tracks: start states (FP32 tracklet states) and
// accept masks are given; returns params/cov/chi2 of pass 3 in double.
void orc_replay_f64(const orc_params* p, int64_t n_tracks, const double* st0, const int32_t* row0,
                    const int64_t* hit_start, const int32_t* hit_rows, const double* ys, const double* zs,
                    const uint8_t* masks, double* st_out, double* chi2_out, int32_t* ok_out) {
    Consts<double> k(*p);
    for (int64_t t = 0; t < n_tracks; ++t) {
        State<double> s;
        load_state(st0 + 20 * t, s);
        const int64_t a = hit_start[t];
        const int n = (int)(hit_start[t + 1] - a);
        std::vector<uint8_t> m(n);
        RefitOut<double> o = refit(k, s, row0[t], n, hit_rows + a, ys + a, zs + a, m.data(), masks + a);
        ok_out[t] = o.ok ? 1 : 0;
        if (o.ok) {
            store_state(o.s, st_out + 20 * t);
            chi2_out[t] = o.chi2;
        }
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiable refit: a smooth space-charge correction map and the refit with
// frozen accept masks as a function of it (the paper applies calibration
// corrections between seeding and fitting, Sections 1 and 4).
//
// Map: three components (delta r, delta r*phi, delta z) [cm], each a tricubic
// uniform B-spline with 16 (r) x 16 (phi, periodic) x 32 (z) coefficients,
// coefficient layout [comp][ir][iphi][iz]. Knots: r_k = 84 + (k - 1) * 168/13,
// phi_k = k * 2 pi / 16, z_k = -252 + (k - 1) * 504/29, so the data range maps to
// u in [1, 14) in r and [1, 30) in z and no index is ever clamped.
namespace {
constexpr int kMapNr = 16, kMapNphi = 16, kMapNz = 32;

void bspline_basis(double t, double w[4]) {
    const double t2 = t * t, t3 = t2 * t, s = 1.0 - t;
    w[0] = s * s * s / 6.0;
    w[1] = (3.0 * t3 - 6.0 * t2 + 4.0) / 6.0;
    w[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) / 6.0;
    w[3] = t3 / 6.0;
}

struct MapCell {
    int ir, iphi, iz;  // index of the first of the 4 coefficients per axis
    double wr[4], wphi[4], wz[4];
};

MapCell map_cell(double r, double phi, double z) {
    const double pi2 = 2.0 * 3.14159265358979323846;
    MapCell c;
    double ur = 1.0 + (r - 84.0) / (168.0 / 13.0);
    double uz = 1.0 + (z + 252.0) / (504.0 / 29.0);
    ur = std::min(std::max(ur, 1.0), 14.0 - 1e-9);
    uz = std::min(std::max(uz, 1.0), 30.0 - 1e-9);
    double ph = std::fmod(phi, pi2);
    if (ph < 0) ph += pi2;
    const double up = ph / (pi2 / kMapNphi);
    const int ir = (int)std::floor(ur), iz = (int)std::floor(uz), ip = (int)std::floor(up);
    bspline_basis(ur - ir, c.wr);
    bspline_basis(uz - iz, c.wz);
    bspline_basis(up - ip, c.wphi);
    c.ir = ir - 1;
    c.iz = iz - 1;
    c.iphi = ip - 1;
    return c;
}

inline int64_t map_index(int comp, int ir, int iphi, int iz) {
    iphi = ((iphi % kMapNphi) + kMapNphi) % kMapNphi;
    return (((int64_t)comp * kMapNr + ir) * kMapNphi + iphi) * kMapNz + iz;
}

double map_value(const double* coef, int comp, const MapCell& c) {
    double v = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 4; ++d)
                v += c.wr[a] * c.wphi[b] * c.wz[d] * coef[map_index(comp, c.ir + a, c.iphi + b, c.iz + d)];
    return v;
}

// Cluster on the row plane x with local (y, z) in a sector of angle alpha,
// corrected by the map inside its pad-row plane.
void correct_cluster(const double* coef, double alpha, double x, double y, double z, double* yc, double* zc) {
    const double r = std::sqrt(x * x + y * y);
    const double phi = alpha + std::atan2(y, x);
    const MapCell c = map_cell(r, phi, z);
    const double dr = map_value(coef, 0, c), drphi = map_value(coef, 1, c), dz = map_value(coef, 2, c);
    *yc = y - (dr * y + drphi * x) / r;
    *zc = z - dz;
}
}  // namespace

extern "C" {

void orc_map_eval(const double* coef, int64_t n, const double* r, const double* phi, const double* z, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        const MapCell c = map_cell(r[i], phi[i], z[i]);
        for (int comp = 0; comp < 3; ++comp) out[3 * i + comp] = map_value(coef, comp, c);
    }
}

void orc_correct(const double* coef, int64_t n, const double* alpha, const double* x, const double* y,
                 const double* z, double* yc, double* zc) {
    for (int64_t i = 0; i < n; ++i) correct_cluster(coef, alpha[i], x[i], y[i], z[i], yc + i, zc + i);
}

// Pass-3 chi2 of the three-pass refit with frozen accept masks, in FP64, on
// clusters corrected by `coef` (NULL: uncorrected), per track.
void orc_refit_frozen_f64(const orc_params* p, int64_t n_tracks, const double* st0, const int32_t* row0,
                          const double* alpha, const int64_t* hit_start, const int32_t* hit_rows, const double* ys,
                          const double* zs, const uint8_t* masks, const double* coef, double* chi2_out,
                          int32_t* ok_out) {
    Consts<double> k(*p);
    for (int64_t t = 0; t < n_tracks; ++t) {
        State<double> s;
        load_state(st0 + 20 * t, s);
        const int64_t a = hit_start[t];
        const int n = (int)(hit_start[t + 1] - a);
        std::vector<double> yc(n), zc(n);
        for (int i = 0; i < n; ++i) {
            if (coef) correct_cluster(coef, alpha[t], k.X[hit_rows[a + i]], ys[a + i], zs[a + i], &yc[i], &zc[i]);
            else { yc[i] = ys[a + i]; zc[i] = zs[a + i]; }
        }
        std::vector<uint8_t> m(n);
        RefitOut<double> o = refit(k, s, row0[t], n, hit_rows + a, yc.data(), zc.data(), m.data(), masks + a);
        ok_out[t] = o.ok ? 1 : 0;
        chi2_out[t] = o.ok ? o.chi2 : 0.0;
    }
}

}  // extern "C"

// ---------------------------------------------------------------- vertex z
// Continuous readout (Section 4): a track's collision time is unknown, and the
// position of closest approach to the beam line, taken as the z of its primary
// vertex, stands in for it. Sector frames share the beam line as their z axis,
// so the local frame of the state is used directly.
//
// The helix through (x, y) with direction angle phi and curvature c = kB q/pT
// passes its point closest to the beam line where its direction is
// perpendicular to the position: with A = x cos phi + y sin phi and
// B = -x sin phi + y cos phi, the turning angle d from the state to that point
// solves A cos d + (B + 1/c) sin d = 0, i.e. d = atan2(-A c, 1 + B c) (the
// solution nearest to the state). The transverse path is s = d / c, written
// as s = -A / (1 + B c) * atan(w) / w with w = -A c / (1 + B c) where
// 1 + B c > 0 (straight line: s = -A), and z0 = z + tan(lambda) s.
extern "C" {

// Native cluster coordinates to local ones (Sections 4 and 6: the tracker is
// to take pad, row and time and transform them to space itself). In binary32,
// one rounding per operation: y = (pad - pad_center[row]) * pad_width[row];
// z = side * (z_readout - z_per_bin * time) with side +1 for sectors 0..17
// (A side) and -1 for 18..35 (C side). The time is scaled linearly to z as
// for an arbitrarily long chamber (Section 4, continuous readout): a
// collision at time t shifts its clusters by -side * z_per_bin * t.
void orc_native_to_local(int32_t n_rows, int32_t n_inst, const int32_t* inst_sector, const int64_t* row_start,
                         const float* pad_width, const float* pad_center, float z_per_bin, float z_readout,
                         const float* pad, const float* time, float* y, float* z) {
    for (int32_t i = 0; i < n_inst; ++i) {
        const float side = inst_sector[i] < 18 ? 1.0f : -1.0f;
        for (int32_t r = 0; r < n_rows; ++r) {
            const int64_t seg = (int64_t)i * n_rows + r;
            for (int64_t c = row_start[seg]; c < row_start[seg + 1]; ++c) {
                const float u = pad[c] - pad_center[r];
                y[c] = u * pad_width[r];
                const float drift = z_per_bin * time[c];
                z[c] = side * (z_readout - drift);
            }
        }
    }
}

double orc_vertex_z(const orc_params* p, double x, const double* state5) {
    const double kB = -0.00299792458 * p->bz;
    const double y = state5[0], z = state5[1], sp = state5[2], tl = state5[3], q = state5[4];
    const double cp = std::sqrt(1.0 - sp * sp);
    const double c = kB * q;
    const double A = x * cp + y * sp, B = -x * sp + y * cp;
    const double den = 1.0 + B * c;
    double s;
    if (den > 0.0) {
        const double w = -A * c / den;
        const double g = (w == 0.0) ? 1.0 : std::atan(w) / w;
        s = -A / den * g;
    } else {
        s = std::atan2(-A * c, den) / c;
    }
    return z + tl * s;
}

// The corrected final fit of continuous readout (Section 4: a track's vertex z
// from its closest approach to the beam line stands for the collision time;
// with it known, the space-point correction, which depends on the absolute z,
// can be applied, and the track is fitted again). Per track: the clusters and
// the start state are moved to the absolute frame (z - z0), the clusters
// corrected by the map inside their pad-row planes (none if coef is null),
// and the three passes of the final fit run with chi2 rejection from the
// start state at its row. Outputs: state, chi2 and count of the last pass's
// accepted clusters, the row of the output state, the refined vertex z (z0
// plus the closest approach of the new state) and the accept masks.
void orc_fit_corrected(const orc_params* p, int64_t n_tracks, const double* st0, const int32_t* row0,
                       const double* z0, const double* alpha, const int64_t* hit_start, const int32_t* hit_rows,
                       const double* ys, const double* zs, const double* coef, double* st_out, double* chi2_out,
                       int32_t* nacc_out, int32_t* row_out, double* z0_out, int32_t* ok_out, uint8_t* mask_out) {
    Consts<double> k(*p);
    for (int64_t t = 0; t < n_tracks; ++t) {
        State<double> s;
        load_state(st0 + 20 * t, s);
        s.p[1] = s.p[1] - z0[t];
        const int64_t a = hit_start[t];
        const int n = (int)(hit_start[t + 1] - a);
        std::vector<double> yc(n), zc(n);
        for (int i = 0; i < n; ++i) {
            const double za = zs[a + i] - z0[t];
            if (coef) correct_cluster(coef, alpha[t], k.X[hit_rows[a + i]], ys[a + i], za, &yc[i], &zc[i]);
            else {
                yc[i] = ys[a + i];
                zc[i] = za;
            }
        }
        RefitOut<double> o = refit(k, s, row0[t], n, hit_rows + a, yc.data(), zc.data(), mask_out + a, nullptr);
        ok_out[t] = o.ok ? 1 : 0;
        if (!o.ok) continue;
        store_state(o.s, st_out + 20 * t);
        chi2_out[t] = o.chi2;
        nacc_out[t] = o.nacc;
        row_out[t] = o.row;
        z0_out[t] = z0[t] + orc_vertex_z(p, k.X[o.row], st_out + 20 * t);
    }
}

}  // extern "C"

// ---------------------------------------------------------------- track-model compression
// Section 5.1: the entropy of the stored clusters is reduced by keeping, for
// clusters attached to tracks, only their residuals to the track model; the
// model is the track fitted in the coordinates the clusters are stored in
// (no calibration correction). Encoder and decoder must predict the same
// positions, so the model is evaluated in binary32 in the tracker's own
// operation order: from the track parameters at their reference row (the
// final fit's innermost row, at or below the first cluster), the helix step of
// the tracker moves the state row by row outward, and each cluster (rows
// ascending) is predicted where the state crosses its row.
// Residual = cluster - prediction, in units of a step that is a power of two
// (so the scaling is exact), rounded to the nearest integer (ties to even).
// kResEscape marks a residual outside int16 or a cluster after a step that
// fails (the cluster would then be stored uncompressed).
extern "C" {

enum { kResEscape = -32768 };

int32_t orc_track_residuals(const orc_params* p, const double* params5, int32_t row0, int32_t n, const int32_t* rows,
                            const double* ys, const double* zs, int32_t step_log2, int16_t* q_out) {
    Consts<float> k(*p);
    State<float> s{};
    for (int i = 0; i < 5; ++i) s.p[i] = (float)params5[i];
    const float scale = std::ldexp(1.0f, -step_log2);  // 1 / step, exact
    int cur = row0;
    bool ok = true;
    int32_t n_esc = 0;
    for (int i = 0; i < n; ++i) {
        while (ok && cur < rows[i]) {
            if (!propagate(s, k.X[cur], k.X[cur + 1], k)) ok = false;
            else ++cur;
        }
        if (!ok || rows[i] < cur) {
            q_out[2 * i] = q_out[2 * i + 1] = (int16_t)kResEscape;
            n_esc += 1;
            continue;
        }
        const float r[2] = {(float)ys[i] - s.p[0], (float)zs[i] - s.p[1]};
        for (int c = 0; c < 2; ++c) {
            const float q = std::nearbyint(r[c] * scale);
            const bool fits = q >= -32767.0f && q <= 32767.0f;
            q_out[2 * i + c] = fits ? (int16_t)q : (int16_t)kResEscape;
            n_esc += fits ? 0 : 1;
        }
    }
    return n_esc;
}

// Decoder: the clusters back from the parameters, the rows and the residuals
// (the same model; an escaped residual decodes to NaN).
void orc_track_decode(const orc_params* p, const double* params5, int32_t row0, int32_t n, const int32_t* rows,
                      const int16_t* q, int32_t step_log2, double* ys, double* zs) {
    Consts<float> k(*p);
    State<float> s{};
    for (int i = 0; i < 5; ++i) s.p[i] = (float)params5[i];
    const float step = std::ldexp(1.0f, step_log2);
    int cur = row0;
    bool ok = true;
    for (int i = 0; i < n; ++i) {
        while (ok && cur < rows[i]) {
            if (!propagate(s, k.X[cur], k.X[cur + 1], k)) ok = false;
            else ++cur;
        }
        const bool esc_y = !ok || q[2 * i] == kResEscape, esc_z = !ok || q[2 * i + 1] == kResEscape;
        ys[i] = esc_y ? std::nan("") : (double)(s.p[0] + (float)q[2 * i] * step);
        zs[i] = esc_z ? std::nan("") : (double)(s.p[1] + (float)q[2 * i + 1] * step);
    }
}

}  // extern "C"
