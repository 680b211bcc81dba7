// Seeded synthetic TPC clusters from helices in a uniform solenoidal field.
//
// This module only produces inputs (clusters, Monte-Carlo labels, truth
// helices). It holds none of the track-finding arithmetic and is shared by the
// CPU oracle tests and the GPU tests alike.
//
// Geometry (readings of Sections 1 and 2 of the paper: 152 pad rows, 36
// trapezoidal sectors): 18 sectors in azimuth per side, sector s has centre
// angle alpha = ((s mod 18) + 0.5) * 20 deg; sectors 0..17 hold z >= 0 (A
// side), 18..35 hold z < 0 (C side). Pad row i is the plane x_local = X_i with
// X_i = 85 + i * 162 / 151 cm. A crossing of plane X_i belongs to the sector
// iff |y_local| <= X_i * tan(10 deg).
//
// Helix (FP64, exact): a particle of charge q and transverse momentum pT [GeV]
// in Bz [T] moves on a circle of radius R = pT / (0.00299792458 * Bz) cm and
// turns with d(phi)/ds = -q / R (clockwise seen from +z for q > 0, Bz > 0).
// z grows linearly with the transverse path length s: z = vz + tan(lambda) s.
// Every plane crossing inside the active volume gives one cluster; the track
// ends when it leaves the outer boundary, when |z| exceeds the drift length,
// or when it re-enters the inner radius (at most one turn).
//
// Build: g++ -O2 -std=c++17 -shared -fPIC helix_gen.cpp -o libtpcsynth.so
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr int kRows = 152;
constexpr double kPi = 3.14159265358979323846;
constexpr double kDrift = 250.0;  // |z| limit [cm]

double row_x(int i) { return 85.0 + i * 162.0 / 151.0; }

// ---------------------------------------------------------------- RNG
// splitmix64 seeds xoshiro256**; both are public-domain generators (Vigna).
struct Rng {
    uint64_t s[4];
    double cached = 0;
    bool has_cached = false;
    static uint64_t splitmix(uint64_t& x) {
        uint64_t z = (x += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    }
    explicit Rng(uint64_t seed) {
        uint64_t x = seed;
        for (auto& v : s) v = splitmix(x);
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next() {
        uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
        s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
        s[2] ^= t; s[3] = rotl(s[3], 45);
        return r;
    }
    double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }  // [0,1)
    double uniform(double a, double b) { return a + (b - a) * uniform(); }
    double normal() {  // Box-Muller
        if (has_cached) { has_cached = false; return cached; }
        double u1 = 1.0 - uniform(), u2 = uniform();
        double r = std::sqrt(-2.0 * std::log(u1));
        cached = r * std::sin(2 * kPi * u2);
        has_cached = true;
        return r * std::cos(2 * kPi * u2);
    }
    double exponential(double mean) { return -mean * std::log(1.0 - uniform()); }
    int64_t below(int64_t n) { return (int64_t)(uniform() * (double)n); }
};

struct Helix {
    double vx, vy, vz, pt, tanl, phi0;
    int q;
};

struct Hit {
    int32_t sector, row;
    double y, z, tau;
};

double wrap2pi(double a) {
    a = std::fmod(a, 2 * kPi);
    if (a < 0) a += 2 * kPi;
    return a;
}

// All valid pad-row plane crossings of one helix, in order of turning angle.
void trace(const Helix& h, double bz, std::vector<Hit>& out, int only_phi_sector = -1) {
    out.clear();
    if (h.pt <= 0 || bz == 0) {
        // Straight line (Bz = 0): x = vx + t cos(phi0), y = vy + t sin(phi0).
        double c = std::cos(h.phi0), s = std::sin(h.phi0);
        double tmax = 1e30;
        if (h.tanl > 0) tmax = (kDrift - h.vz) / h.tanl;
        if (h.tanl < 0) tmax = (-kDrift - h.vz) / h.tanl;
        for (int sec = 0; sec < 18; ++sec) {
            if (only_phi_sector >= 0 && sec != only_phi_sector) continue;
            double al = (sec + 0.5) * 20.0 * kPi / 180.0;
            double ca = std::cos(al), sa = std::sin(al);
            double dn = c * ca + s * sa;
            if (dn <= 0) continue;
            for (int i = 0; i < kRows; ++i) {
                double X = row_x(i);
                double t = (X - (h.vx * ca + h.vy * sa)) / dn;
                if (t < 0 || t > tmax) continue;
                double px = h.vx + t * c, py = h.vy + t * s;
                double yl = -px * sa + py * ca;
                if (std::fabs(yl) > X * std::tan(10.0 * kPi / 180.0)) continue;
                double z = h.vz + h.tanl * t;
                out.push_back({sec + (z < 0 ? 18 : 0), i, yl, z, t});
            }
        }
        std::sort(out.begin(), out.end(), [](const Hit& a, const Hit& b) { return a.tau < b.tau; });
        return;
    }
    const double R = h.pt / (0.00299792458 * bz);  // radius [cm]
    const double sigma = (bz > 0) ? -(double)h.q : (double)h.q;  // sign of d(phi)/ds
    const double rho = sigma * R;                                 // signed 1/omega
    const double cx = h.vx - rho * std::sin(h.phi0), cy = h.vy + rho * std::cos(h.phi0);
    const double cc = std::hypot(cx, cy);
    const double A = cc * cc + rho * rho, B = 2.0 * R * cc;
    const double gam = std::atan2(cy, cx);
    const double delta = sigma * (h.phi0 - gam);
    const double tan10 = std::tan(10.0 * kPi / 180.0);
    const double r_in = row_x(0), r_out = row_x(kRows - 1) / std::cos(10.0 * kPi / 180.0);
    // r^2(tau) = A + B sin(tau + delta); tau = turning angle (>= 0).
    if (B <= 0 || A + B < r_in * r_in) return;  // never reaches the inner radius
    double w_in = (r_in * r_in - A) / B;
    if (w_in < -1.0) return;  // (cannot happen for vertices inside r_in)
    double tau_in = wrap2pi(std::asin(w_in) - delta);
    double tau_end;
    if (A + B > r_out * r_out) {
        double w_out = (r_out * r_out - A) / B;
        tau_end = tau_in + (std::asin(w_out) - std::asin(w_in));
    } else {
        tau_end = tau_in + (kPi - 2.0 * std::asin(w_in));  // re-entry below r_in
    }
    if (h.tanl != 0) {
        double sz = (h.tanl > 0) ? (kDrift - h.vz) / h.tanl : (-kDrift - h.vz) / h.tanl;
        tau_end = std::min(tau_end, sz / R);
    }
    for (int sec = 0; sec < 18; ++sec) {
        if (only_phi_sector >= 0 && sec != only_phi_sector) continue;
        double al = (sec + 0.5) * 20.0 * kPi / 180.0;
        double ca = std::cos(al), sa = std::sin(al);
        double cn = cx * ca + cy * sa;
        for (int i = 0; i < kRows; ++i) {
            double X = row_x(i);
            double w = (X - cn) / rho;
            if (w < -1.0 || w > 1.0) continue;
            double as = std::asin(w);
            const double roots[2] = {as + al, kPi - as + al};  // theta values
            for (int k = 0; k < 4; ++k) {
                // each root recurs every full turn; tau_end can exceed 2 pi
                double tau = wrap2pi(sigma * (roots[k & 1] - h.phi0)) + (k >> 1) * 2.0 * kPi;
                if (tau > tau_end) continue;
                double thc = h.phi0 + sigma * tau;
                double px = cx + rho * std::sin(thc), py = cy - rho * std::cos(thc);
                double yl = -px * sa + py * ca;
                if (std::fabs(yl) > X * tan10) continue;
                double z = h.vz + h.tanl * R * tau;
                if (std::fabs(z) > kDrift) continue;
                out.push_back({sec + (z < 0 ? 18 : 0), i, yl, z, tau});
            }
        }
    }
    std::sort(out.begin(), out.end(), [](const Hit& a, const Hit& b) { return a.tau < b.tau; });
}

// Smooth synthetic space-charge displacement (cm) at global (r, phi, z):
// components along r, along r*phi and along z, amplitude <= 0.5 cm.
void true_distortion(double r, double phi, double z, double* dr, double* drphi, double* dz) {
    const double a = kPi * (r - 85.0) / 166.0, zz = z / kDrift;
    *dr = 0.5 * std::sin(a) * (0.6 + 0.4 * std::cos(phi)) * (1.0 - zz * zz);
    *drphi = 0.3 * std::cos(2.0 * a) * std::sin(2.0 * phi) * zz;
    *dz = 0.2 * std::sin(kPi * zz) * std::cos(a);
}

double sample_pt(Rng& rng, double mean, double lo, double hi) {
    // Exponential law truncated to [lo, hi] by resampling.
    for (;;) {
        double p = rng.exponential(mean);
        if (p >= lo && p <= hi) return p;
    }
}

}  // namespace

extern "C" {

// Generator modes.
//   0: sector instances. Instance j covers sector unit_sector[j] only and holds
//      unit_ntracks[j] primaries with phi0 uniform inside that sector and eta on
//      that sector's side, (0, eta_max) or (-eta_max, 0).
//   1: full events. Event e fills instances 36 e .. 36 e + 35 (instance =
//      sector); unit_ntracks[e] primaries over the full azimuth with
//      |eta| < eta_max plus round(sec_frac * primaries) secondaries whose vertex
//      lies at radius U(0, sec_rmax), azimuth U(0, 2 pi), z = 0.
//   2: time frame. n_units collisions into 36 instances; collision k has
//      unit_ntracks[k] primaries and a drift shift dz_k ~ U(0, zshift_max);
//      the apparent z is z - side * dz_k (side = +1 on A, -1 on C).
//   3: explicit helices (given by the caller), full event layout, one event.
typedef struct {
    int32_t mode;
    int32_t n_units;
    const int32_t* unit_sector;
    const int32_t* unit_ntracks;
    double bz;
    double pt_mean, pt_min, pt_max;
    double eta_max;
    double sec_frac, sec_rmax;
    double noise_frac;
    double sigma_y, sigma_z;
    double zshift_max;
    int32_t shuffle;
    uint64_t seed;
    // mode 3 only: explicit helices
    int32_t n_explicit;
    const double* ex_vx; const double* ex_vy; const double* ex_vz;
    const double* ex_pt; const double* ex_tanl; const double* ex_phi0;
    const int32_t* ex_q;
    // 1: displace every cluster by the smooth "true" space-charge map below
    // (before the smear), keeping it on its pad-row plane
    int32_t distort;
} syn_config;

typedef struct {
    int32_t n_inst;
    int64_t n_clusters;
    int64_t n_tracks;
    std::vector<int32_t>* inst_sector;
    std::vector<int64_t>* row_start;
    std::vector<float>* x;
    std::vector<float>* y;
    std::vector<float>* z;
    std::vector<int32_t>* row;
    std::vector<int32_t>* label;
    std::vector<double>* truth;  // per track: vx vy vz pt tanl phi0 q dz
} syn_result;

syn_result* syn_generate(const syn_config* cfg) {
    Rng rng(cfg->seed);
    std::vector<Helix> tracks;
    std::vector<double> track_dz;
    std::vector<int32_t> track_unit;
    int n_inst = 0;
    std::vector<int32_t> inst_sector;
    const double deg = kPi / 180.0;
    auto eta_to_tanl = [](double eta) { return std::sinh(eta); };

    if (cfg->mode == 0) {
        n_inst = cfg->n_units;
        for (int j = 0; j < n_inst; ++j) {
            int sec = cfg->unit_sector[j];
            inst_sector.push_back(sec);
            double al = ((sec % 18) + 0.5) * 20.0 * deg;
            double side = sec < 18 ? 1.0 : -1.0;
            for (int t = 0; t < cfg->unit_ntracks[j]; ++t) {
                Helix h;
                h.vx = h.vy = h.vz = 0;
                h.pt = sample_pt(rng, cfg->pt_mean, cfg->pt_min, cfg->pt_max);
                h.tanl = eta_to_tanl(side * rng.uniform(0.0, cfg->eta_max));
                h.phi0 = al + rng.uniform(-10.0 * deg, 10.0 * deg);
                h.q = rng.uniform() < 0.5 ? -1 : 1;
                tracks.push_back(h);
                track_dz.push_back(0);
                track_unit.push_back(j);
            }
        }
    } else if (cfg->mode == 1 || cfg->mode == 2 || cfg->mode == 3) {
        int n_events = (cfg->mode == 1) ? cfg->n_units : 1;
        n_inst = 36 * n_events;
        for (int e = 0; e < n_events; ++e)
            for (int s = 0; s < 36; ++s) inst_sector.push_back(s);
        if (cfg->mode == 3) {
            for (int t = 0; t < cfg->n_explicit; ++t) {
                Helix h{cfg->ex_vx[t], cfg->ex_vy[t], cfg->ex_vz[t], cfg->ex_pt[t],
                        cfg->ex_tanl[t], cfg->ex_phi0[t], cfg->ex_q[t]};
                tracks.push_back(h);
                track_dz.push_back(0);
                track_unit.push_back(0);
            }
        } else {
            int n_coll = cfg->n_units;
            for (int e = 0; e < n_coll; ++e) {
                double dz = (cfg->mode == 2) ? rng.uniform(0.0, cfg->zshift_max) : 0.0;
                int np = cfg->unit_ntracks[e];
                int ns = (cfg->mode == 1) ? (int)std::lround(cfg->sec_frac * np) : 0;
                for (int t = 0; t < np + ns; ++t) {
                    Helix h;
                    h.vx = h.vy = h.vz = 0;
                    if (t >= np) {
                        double rv = rng.uniform(0.0, cfg->sec_rmax);
                        double ps = rng.uniform(0.0, 2 * kPi);
                        h.vx = rv * std::cos(ps);
                        h.vy = rv * std::sin(ps);
                    }
                    h.pt = sample_pt(rng, cfg->pt_mean, cfg->pt_min, cfg->pt_max);
                    h.tanl = eta_to_tanl(rng.uniform(-cfg->eta_max, cfg->eta_max));
                    h.phi0 = rng.uniform(0.0, 2 * kPi);
                    h.q = rng.uniform() < 0.5 ? -1 : 1;
                    tracks.push_back(h);
                    track_dz.push_back(dz);
                    track_unit.push_back(cfg->mode == 1 ? e : 0);
                }
            }
        }
    } else {
        return nullptr;
    }

    struct Cl {
        int32_t inst, row, label;
        float y, z;
    };
    std::vector<Cl> cls;
    std::vector<Hit> hits;
    for (size_t t = 0; t < tracks.size(); ++t) {
        trace(tracks[t], cfg->bz, hits, cfg->mode == 0 ? inst_sector[track_unit[t]] % 18 : -1);
        for (const Hit& h : hits) {
            int inst;
            if (cfg->mode == 0) {
                if (h.sector != inst_sector[track_unit[t]]) continue;
                inst = track_unit[t];
            } else {
                inst = 36 * track_unit[t] + h.sector;
            }
            double side = h.sector < 18 ? 1.0 : -1.0;
            double yt = h.y, zt = h.z;
            if (cfg->distort) {
                const double X = row_x(h.row), r = std::hypot(X, h.y);
                const double phi = ((h.sector % 18) + 0.5) * 20.0 * kPi / 180.0 + std::atan2(h.y, X);
                double dr, drphi, dz;
                true_distortion(r, phi, h.z, &dr, &drphi, &dz);
                yt += (dr * h.y + drphi * X) / r;  // local-y component of the displacement
                zt += dz;
            }
            double y = yt + cfg->sigma_y * rng.normal();
            double z = zt + cfg->sigma_z * rng.normal() - side * track_dz[t];
            cls.push_back({inst, h.row, (int32_t)t, (float)y, (float)z});
        }
    }
    // Uniform noise: per instance round(noise_frac * signal) clusters, uniform
    // in row, in y over the sector width and in z over that instance's signal
    // z range (or the side's drift range if the instance holds no signal).
    if (cfg->noise_frac > 0) {
        std::vector<int64_t> nsig(n_inst, 0);
        std::vector<double> zlo(n_inst, 1e30), zhi(n_inst, -1e30);
        for (const Cl& c : cls) {
            nsig[c.inst]++;
            zlo[c.inst] = std::min(zlo[c.inst], (double)c.z);
            zhi[c.inst] = std::max(zhi[c.inst], (double)c.z);
        }
        for (int j = 0; j < n_inst; ++j) {
            int64_t nn = std::llround(cfg->noise_frac * (double)nsig[j]);
            double lo = zlo[j], hi = zhi[j];
            if (nsig[j] == 0) {
                lo = inst_sector[j] < 18 ? 0.0 : -kDrift;
                hi = lo + kDrift;
            }
            for (int64_t k = 0; k < nn; ++k) {
                int row = (int)rng.below(kRows);
                double X = row_x(row);
                double w = X * std::tan(10.0 * deg);
                double y = rng.uniform(-w, w);
                double z = rng.uniform(lo, hi);
                cls.push_back({j, row, -1, (float)y, (float)z});
            }
        }
    }
    // Input order: sorted by (instance, row); inside a row either generator
    // order (stable) or a seeded shuffle.
    std::stable_sort(cls.begin(), cls.end(), [](const Cl& a, const Cl& b) {
        return a.inst != b.inst ? a.inst < b.inst : a.row < b.row;
    });
    int64_t nseg = (int64_t)n_inst * kRows;
    auto* res = new syn_result;
    res->n_inst = n_inst;
    res->n_clusters = (int64_t)cls.size();
    res->n_tracks = (int64_t)tracks.size();
    res->inst_sector = new std::vector<int32_t>(inst_sector);
    res->row_start = new std::vector<int64_t>(nseg + 1, 0);
    for (const Cl& c : cls) (*res->row_start)[(int64_t)c.inst * kRows + c.row + 1]++;
    for (int64_t s = 0; s < nseg; ++s) (*res->row_start)[s + 1] += (*res->row_start)[s];
    if (cfg->shuffle) {
        for (int64_t s = 0; s < nseg; ++s) {
            int64_t a = (*res->row_start)[s], b = (*res->row_start)[s + 1];
            for (int64_t i = b - 1; i > a; --i) {  // Fisher-Yates
                int64_t j = a + rng.below(i - a + 1);
                std::swap(cls[i], cls[j]);
            }
        }
    }
    res->x = new std::vector<float>(cls.size());
    res->y = new std::vector<float>(cls.size());
    res->z = new std::vector<float>(cls.size());
    res->row = new std::vector<int32_t>(cls.size());
    res->label = new std::vector<int32_t>(cls.size());
    for (size_t i = 0; i < cls.size(); ++i) {
        (*res->x)[i] = (float)row_x(cls[i].row);
        (*res->y)[i] = cls[i].y;
        (*res->z)[i] = cls[i].z;
        (*res->row)[i] = cls[i].row;
        (*res->label)[i] = cls[i].label;
    }
    res->truth = new std::vector<double>(tracks.size() * 8);
    for (size_t t = 0; t < tracks.size(); ++t) {
        double* o = res->truth->data() + 8 * t;
        o[0] = tracks[t].vx; o[1] = tracks[t].vy; o[2] = tracks[t].vz;
        o[3] = tracks[t].pt; o[4] = tracks[t].tanl; o[5] = tracks[t].phi0;
        o[6] = tracks[t].q; o[7] = track_dz[t];
    }
    return res;
}

void syn_sizes(const syn_result* r, int64_t* n_inst, int64_t* n_clusters, int64_t* n_tracks) {
    *n_inst = r->n_inst;
    *n_clusters = r->n_clusters;
    *n_tracks = r->n_tracks;
}

void syn_copy(const syn_result* r, int32_t* inst_sector, int64_t* row_start, float* x, float* y,
              float* z, int32_t* row, int32_t* label, double* truth) {
    std::memcpy(inst_sector, r->inst_sector->data(), r->inst_sector->size() * 4);
    std::memcpy(row_start, r->row_start->data(), r->row_start->size() * 8);
    std::memcpy(x, r->x->data(), r->x->size() * 4);
    std::memcpy(y, r->y->data(), r->y->size() * 4);
    std::memcpy(z, r->z->data(), r->z->size() * 4);
    std::memcpy(row, r->row->data(), r->row->size() * 4);
    std::memcpy(label, r->label->data(), r->label->size() * 4);
    std::memcpy(truth, r->truth->data(), r->truth->size() * 8);
}

void syn_free(syn_result* r) {
    if (!r) return;
    delete r->inst_sector; delete r->row_start; delete r->x; delete r->y; delete r->z;
    delete r->row; delete r->label; delete r->truth;
    delete r;
}

}  // extern "C"
