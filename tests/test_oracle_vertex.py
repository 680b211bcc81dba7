"""Pins of the oracle's vertex-z estimate (closest approach to the beam line,
Section 4 of the paper: continuous readout has no absolute z, so the z of a
track's closest approach stands in for the primary vertex z and thus for the
collision time). Independent of the formula: closed-form helices from known
vertices (tests/helix_truth.py), the textbook straight-line closest approach,
and a brute-force minimisation over the helix for displaced vertices."""
import math

import numpy as np
import pytest

import oracle
from helix_truth import LocalHelix, plane_x


@pytest.mark.parametrize("q", [1, -1])
@pytest.mark.parametrize("pt", [0.12, 0.5, 2.0, 10.0])
def test_primary_helix_gives_its_vertex_z(q, pt):
    for zv, tanl, phi0, alpha in ((0.0, 0.3, 0.1, 0.0), (-87.5, -0.8, -0.15, 0.0), (140.0, 0.05, 1.2, 1.0)):
        h = LocalHelix(pt, q, tanl, phi0, alpha, vz=zv)
        for r in (0, 40, 100):
            st = h.at(plane_x(r))
            if st is None or abs(st[2]) > 0.95:
                continue
            z0 = oracle.vertex_z(plane_x(r), [st])[0]
            assert z0 == pytest.approx(zv, abs=1e-9), (pt, q, r, z0, zv)


def test_straight_line_is_the_textbook_closest_approach():
    p = oracle.default_params(bz=0.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        x, y = rng.uniform(85, 247), rng.uniform(-30, 30)
        sp, tl, z = rng.uniform(-0.9, 0.9), rng.uniform(-1, 1), rng.uniform(-200, 200)
        cp = math.sqrt(1 - sp * sp)
        # foot of the perpendicular from the axis: P - ((P . d) d), z moves by tan(lambda) per unit path
        s = -(x * cp + y * sp)
        assert oracle.vertex_z(x, [[y, z, sp, tl, rng.uniform(-5, 5)]], params=p)[0] == pytest.approx(z + tl * s,
                                                                                                         abs=1e-9)


def _brute_force_pca_z(h: LocalHelix, tau_state):
    """z at the point of the helix closest to the beam line, nearest to the
    state along the helix (turning angle within half a turn), by dense sampling
    and golden-section refinement of |P(tau)|."""
    rho = h.sigma * h.R

    def pos(tau):
        th = h.phi + h.sigma * tau
        return np.array([h.xc + rho * math.sin(th), h.yc - rho * math.cos(th)])

    taus = np.linspace(tau_state - math.pi, tau_state + math.pi, 20001)
    d = np.array([np.linalg.norm(pos(t)) for t in taus])
    k = int(np.argmin(d))
    a, b = taus[max(k - 1, 0)], taus[min(k + 1, len(taus) - 1)]
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c, e = b - g * (b - a), a + g * (b - a)
        if np.linalg.norm(pos(c)) < np.linalg.norm(pos(e)):
            b = e
        else:
            a = c
    t = 0.5 * (a + b)
    return h.zv + h.tanl * h.R * t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_displaced_vertex_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    checked = 0
    while checked < 6:
        rv, psi = rng.uniform(5, 50), rng.uniform(0, 2 * math.pi)
        h = LocalHelix(rng.uniform(0.3, 3.0), rng.choice([-1, 1]), rng.uniform(-0.8, 0.8),
                       rng.uniform(-0.3, 0.3), 0.0, vx=rv * math.cos(psi), vy=rv * math.sin(psi),
                       vz=rng.uniform(-100, 100))
        st = h.at(plane_x(20))
        if st is None or abs(st[2]) > 0.9:
            continue
        # turning angle of the state from the vertex: its z is zv + tanl R tau
        tau_state = (st[1] - h.zv) / (h.tanl * h.R) if h.tanl != 0 else None
        if tau_state is None or tau_state > math.pi:
            continue
        z_bf = _brute_force_pca_z(h, tau_state)
        assert oracle.vertex_z(plane_x(20), [st])[0] == pytest.approx(z_bf, abs=1e-6)
        checked += 1


def test_continuous_readout_tracks_find_their_collision_z():
    """QA on a small continuous-readout slice (six collisions, each shifted in
    drift by a random time): the closest-approach z of a found track (from the
    binary32 oracle's final state) recovers its collision's apparent vertex z,
    vertex z minus side times the drift shift. Gates frozen from the first
    run; low-pT loopers, whose returning legs carry no vertex information, are
    reported but not gated (the paper notes the estimate is wrong by design for
    tracks that do not come from the primary vertex)."""
    import synth
    cs = synth.generate_raw(2, 6, [150] * 6, pt_min=0.05, noise_frac=0.02, zshift_max=250.0, seed=77, name="ts")
    r = oracle.run(cs, 32, threads=4)
    z0 = oracle.vertex_z(r.trk_x, r.trk_param)
    lab = np.full(r.n_tracks, -1)
    for t in range(r.n_tracks):
        l = cs.label[r.trk_hit[r.trk_hit_start[t]:r.trk_hit_start[t + 1]]]
        l = l[l >= 0]
        if len(l):
            v, c = np.unique(l, return_counts=True)
            lab[t] = v[np.argmax(c)]
    ok = lab >= 0
    tr = cs.truth[lab[ok]]
    side = np.where(cs.inst_sector[r.trk_inst[ok]] < 18, 1.0, -1.0)
    d = np.abs(z0[ok] - (tr[:, 2] - side * tr[:, 7]))
    pt = tr[:, 3]
    assert np.mean(d[pt >= 0.5] < 1.0) >= 0.95
    assert np.mean(d[(pt >= 0.2) & (pt < 0.5)] < 1.0) >= 0.85
    assert np.median(d[pt >= 0.2]) < 0.1
