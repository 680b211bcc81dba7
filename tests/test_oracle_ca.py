"""Pins of the oracle's cellular automaton, grid, tracklet selection and full
tracker: hand-worked cases, brute force in FP64 on tiny inputs, structural
invariants, exact recovery, metamorphic checks and QA regression gates.

Section 2 of the paper: links between hit triplets close to a straight line,
an evolution step concatenating consecutive links into segments, a
simplified-KF seed fit, track following without multiple hypotheses, then the
final fit. QA definitions follow the footnote of Section 4.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth import N_ROWS, qa
from util import chains_from_links, make_clusterset, row_of_ids

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    return synth.generate("C1")


@pytest.fixture(scope="module")
def c1_run(c1):
    return oracle.run(c1, 32)


@pytest.fixture(scope="module")
def c2s():
    return synth.generate("C2").subset([0, 7, 20, 33])


@pytest.fixture(scope="module")
def c2s_run(c2s):
    return oracle.run(c2s, 32, threads=4)


# ------------------------------------------------------------ hand cases
def test_golden_neighbour_cases():
    cases = json.load(open(os.path.join(GOLDEN, "neighbour_cases.json")))["cases"]
    for case in cases:
        cs = make_clusterset([(0, r, y, z) for r, y, z in case["hits"]])
        for prec in (32, 64):
            res = oracle.run(cs, prec)
            m = case["middle"]
            assert (res.up[m], res.dn[m]) == (case["expect"]["up"], case["expect"]["dn"]), case["name"]


def _window(params, r_lo, r_hi, t, n):
    x = np.float32(synth.row_plane_x(r_hi)) - np.float32(synth.row_plane_x(r_lo))
    return np.float32(np.float32(x * np.float32(t)) + np.float32(n))


def test_window_edge_is_inclusive():
    p = oracle.default_params()
    wyu = _window(p, 10, 11, p.win_ty, p.win_ny)
    wyd = _window(p, 9, 10, p.win_ty, p.win_ny)
    # a straight line through the middle hit with both outer hits exactly on
    # the window edge is linked; one float step further is not a candidate
    yd = -wyd
    inside = make_clusterset([(0, 9, yd, 0.0), (0, 10, 0.0, 0.0), (0, 11, wyu, 0.0)])
    res = oracle.run(inside, 32)
    assert res.up[1] == 2 and res.dn[1] == 0
    out = make_clusterset([(0, 9, yd, 0.0), (0, 10, 0.0, 0.0), (0, 11, np.nextafter(wyu, np.float32(9)), 0.0)])
    res = oracle.run(out, 32)
    assert res.up[1] == -1 and res.dn[1] == -1


def test_edge_rows_and_empty_input():
    cs = make_clusterset([(0, 0, 0.0, 1.0), (0, 1, 0.0, 1.0), (0, 2, 0.0, 1.0), (0, 149, 0.0, 1.0),
                          (0, 150, 0.0, 1.0), (0, 151, 0.0, 1.0)])
    res = oracle.run(cs, 32)
    # rows 0 and 151 never hold a middle hit; their hits only appear as partners
    assert res.up[0] == -1 and res.dn[0] == -1 and res.up[5] == -1 and res.dn[5] == -1
    assert res.up[1] == 2 and res.dn[1] == 0 and res.up[4] == 5 and res.dn[4] == 3
    # a partner on row 0 has no up-link of its own, so cleaning removes the pair
    assert res.dnc[1] == -1 and res.upc[0] == -1
    empty = make_clusterset([], n_inst=2)
    r = oracle.run(empty, 32)
    assert r.n_tracks == 0 and len(r.start_hit) == 0 and len(r.up) == 0


# ------------------------------------------------------------ brute force
def _brute_links_f64(cs, p, sample=None):
    """Exhaustive FP64 search over all (u, d) pairs with the exact predicate.
    Returns up, dn and a flag per hit marking near-ties (ambiguous between
    binary32 and binary64)."""
    rows = row_of_ids(cs)
    X = synth.row_plane_x(np.arange(N_ROWS))
    y, z = cs.y.astype(np.float64), cs.z.astype(np.float64)
    n = len(y)
    up, dn = np.full(n, -1), np.full(n, -1)
    amb = np.zeros(n, bool)
    ids = range(n) if sample is None else sample
    rs = cs.row_start
    for h in ids:
        r = rows[h]
        if r < 1 or r > N_ROWS - 2:
            continue
        inst = int(np.searchsorted(rs, h, side="right") - 1) // N_ROWS
        seg = inst * N_ROWS + r
        U = range(rs[seg + 1], rs[seg + 2])
        D = range(rs[seg - 1], rs[seg])
        du, dd = X[r + 1] - X[r], X[r] - X[r - 1]
        tr = dd / (X[r + 1] - X[r - 1])
        cands = []
        for u in U:
            ddy, ddz = abs(y[u] - y[h]) - (du * p.win_ty + p.win_ny), abs(z[u] - z[h]) - (du * p.win_tz + p.win_nz)
            if max(ddy, ddz) > 1e-5:
                continue
            if abs(ddy) <= 1e-5 or abs(ddz) <= 1e-5:
                amb[h] = True
            for d in D:
                ey_, ez_ = abs(y[d] - y[h]) - (dd * p.win_ty + p.win_ny), abs(z[d] - z[h]) - (dd * p.win_tz + p.win_nz)
                if max(ey_, ez_) > 1e-5:
                    continue
                if abs(ey_) <= 1e-5 or abs(ez_) <= 1e-5:
                    amb[h] = True
                ey = y[d] + (y[u] - y[d]) * tr - y[h]
                ez = z[d] + (z[u] - z[d]) * tr - z[h]
                sc = ey * ey + ez * ez
                if abs(sc - p.nbr_score_max) < 1e-5:
                    amb[h] = True
                if sc <= p.nbr_score_max:
                    cands.append((sc, u, d))
        if cands:
            cands.sort()
            up[h], dn[h] = cands[0][1], cands[0][2]
            if len(cands) > 1 and cands[1][0] - cands[0][0] < 1e-5 * (1 + cands[0][0]):
                amb[h] = True
    return up, dn, amb


@pytest.mark.parametrize("seed", range(8))
def test_links_match_fp64_brute_force_on_tiny_inputs(seed):
    rng = np.random.default_rng(seed)
    hits = []
    for r in range(20, 25):
        for _ in range(rng.integers(5, 40)):
            hits.append((0, r, rng.uniform(-3, 3), rng.uniform(0, 4)))
    # a few exact straight lines through the block
    for _ in range(4):
        y0, z0, sy, sz = rng.uniform(-2, 2), rng.uniform(0.5, 3.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4)
        for r in range(20, 25):
            x = synth.row_plane_x(r) - synth.row_plane_x(20)
            hits.append((0, r, y0 + sy * x, z0 + sz * x))
    cs = make_clusterset(hits)
    p = oracle.default_params()
    res = oracle.run(cs, 32, p)
    up, dn, amb = _brute_links_f64(cs, p)
    ok = ~amb
    assert ok.sum() > 0.9 * len(ok)
    assert np.array_equal(res.up[ok], up[ok]) and np.array_equal(res.dn[ok], dn[ok])
    # FP64 oracle mode agrees too
    r64 = oracle.run(cs, 64, p)
    assert np.array_equal(r64.up[ok], up[ok]) and np.array_equal(r64.dn[ok], dn[ok])


def test_links_on_real_density_match_brute_force_sample(c1, c1_run):
    p = oracle.default_params()
    rng = np.random.default_rng(3)
    sample = rng.choice(len(c1.y), size=400, replace=False)
    up, dn, amb = _brute_links_f64(c1, p, sample)
    s = np.array([i for i in sample if not amb[i]])
    assert len(s) > 380
    assert np.array_equal(c1_run.up[s], up[s]) and np.array_equal(c1_run.dn[s], dn[s])


# ------------------------------------------------------------ invariants
def _check_ca_invariants(cs, res):
    rows = row_of_ids(cs)
    inst = cs.instance_of()
    up, dn, upc, dnc = res.up, res.dn, res.upc, res.dnc
    linked = up >= 0
    assert np.all((up >= 0) == (dn >= 0))
    assert np.all(rows[up[linked]] == rows[linked] + 1) and np.all(rows[dn[linked]] == rows[linked] - 1)
    assert np.all(inst[up[linked]] == inst[linked]) and np.all(inst[dn[linked]] == inst[linked])
    m = upc >= 0
    assert np.all(dnc[upc[m]] == np.nonzero(m)[0])  # mutual
    m = dnc >= 0
    assert np.all(upc[dnc[m]] == np.nonzero(m)[0])
    assert np.all((upc < 0) | (upc == up)) and np.all((dnc < 0) | (dnc == dn))
    chains = chains_from_links(upc, dnc)
    members = np.concatenate([np.array(c) for c in chains]) if chains else np.zeros(0, int)
    assert len(members) == len(np.unique(members))  # disjoint chains
    long_heads = sorted(c[0] for c in chains if len(c) >= 3)
    assert sorted(res.start_hit.tolist()) == long_heads  # one start per chain of >= 3
    # starts ordered by (instance, row, id); tid counts per instance from 0
    # (input ids are themselves ordered by instance and row)
    assert np.all(np.diff(res.start_hit) > 0)
    assert np.array_equal(res.start_inst, inst[res.start_hit])
    for i in np.unique(res.start_inst):
        t = res.start_tid[res.start_inst == i]
        assert np.array_equal(t, np.arange(len(t)))


def test_ca_invariants(c1, c1_run, c2s, c2s_run):
    _check_ca_invariants(c1, c1_run)
    _check_ca_invariants(c2s, c2s_run)
    # segments are "usually 4 to 10 hits" (Section 2): the median chain is short
    lens = [len(c) for c in chains_from_links(c2s_run.upc, c2s_run.dnc) if len(c) >= 3]
    assert len(lens) > 100


def _check_grid(cs, res, hpb):
    rs = cs.row_start
    for seg in range(len(rs) - 1):
        a, b = rs[seg], rs[seg + 1]
        n = b - a
        bs = res.bin_start[a + seg:]
        ny, nz = res.g_ny[seg], res.g_nz[seg]
        assert ny * nz <= max(1, n // hpb)
        nb = ny * nz
        assert bs[0] == 0 and bs[nb] == n and np.all(np.diff(bs[:nb + 1]) >= 0)
        ids = res.sorted_id[a:b]
        assert np.array_equal(np.sort(ids), np.arange(a, b))
        if n == 0:
            continue
        ymin, zmin, iy, iz = (np.float32(v) for v in res.g_meta[seg])
        ty = (cs.y[ids] - ymin) * iy
        tz = (cs.z[ids] - zmin) * iz
        by = np.where(ty >= ny - 1, ny - 1, np.where(ty <= 0, 0, np.floor(ty))).astype(int)
        bz = np.where(tz >= nz - 1, nz - 1, np.where(tz <= 0, 0, np.floor(tz))).astype(int)
        binid = bz * ny + by
        pos = np.arange(n)
        for q in range(nb):
            sel = pos[bs[q]:bs[q + 1]]
            assert np.all(binid[sel] == q)
            assert np.all(np.diff(ids[sel]) > 0)  # stable within a bin


def test_grid_invariants(c1, c1_run):
    _check_grid(c1, c1_run, 1)
    for hpb in (2, 5):
        r = oracle.run(c1, 32, oracle.default_params(hits_per_bin=hpb))
        _check_grid(c1, r, hpb)


def test_results_do_not_depend_on_grid(c2s, c2s_run):
    for hpb in (2, 3, 8):
        r = oracle.run(c2s, 32, oracle.default_params(hits_per_bin=hpb), threads=4)
        assert np.array_equal(r.up, c2s_run.up) and np.array_equal(r.start_hit, c2s_run.start_hit)
        assert np.array_equal(r.trk_hit, c2s_run.trk_hit) and np.array_equal(r.trk_param, c2s_run.trk_param)


def _packed(nh, tid):
    return (np.uint32(nh) << np.uint32(20)) | np.uint32(0xFFFFF - tid)


def _check_selection(cs, res, n_min=10):
    nr = res.n_rows
    # weights are the max packed (nHits, -tid) over tracklets with >= n_min hits
    w = np.zeros(len(cs.y), np.uint32)
    for i in range(len(res.start_hit)):
        if res.tl_nhits[i] < n_min:
            continue
        hs = res.tl_rowhit[i][res.tl_rowhit[i] >= 0]
        assert len(hs) == res.tl_nhits[i]
        w[hs] = np.maximum(w[hs], _packed(res.tl_nhits[i], res.start_tid[i]))
    assert np.array_equal(w, res.weight)
    # selected tracks own exactly their winning hits, in row order
    sel_expect = []
    for i in range(len(res.start_hit)):
        if res.tl_nhits[i] < n_min:
            continue
        hs = res.tl_rowhit[i][res.tl_rowhit[i] >= 0]
        own = hs[w[hs] == _packed(res.tl_nhits[i], res.start_tid[i])]
        if len(own) >= n_min:
            sel_expect.append((i, own))
    assert [s[0] for s in sel_expect] == res.sel_tl.tolist()
    for t, (_, own) in enumerate(sel_expect):
        assert np.array_equal(res.sel_hit[res.sel_hit_start[t]:res.sel_hit_start[t + 1]], own)
    # every cluster in at most one output track; rows strictly ascending
    assert len(np.unique(res.trk_hit)) == len(res.trk_hit)
    rows = row_of_ids(cs)
    for t in range(res.n_tracks):
        hs = res.trk_hit[res.trk_hit_start[t]:res.trk_hit_start[t + 1]]
        assert len(hs) >= n_min and np.all(np.diff(rows[hs]) > 0)
        assert res.trk_ndf[t] == 2 * len(hs) - 5
        C = np.zeros((5, 5))
        k = 0
        for i in range(5):
            for j in range(i + 1):
                C[i, j] = C[j, i] = res.trk_cov[t, k]
                k += 1
        np.linalg.cholesky(C)
    assert res.chi2_total == pytest.approx(float(np.sum(res.trk_chi2)), rel=1e-12)


def test_selection_and_track_invariants(c1, c1_run, c2s, c2s_run):
    _check_selection(c1, c1_run)
    _check_selection(c2s, c2s_run)


# ------------------------------------------------------------ end to end
def test_exact_recovery_of_noiseless_helices():
    # well separated helices through one sector, no smear, no noise
    truth = dict(vx=[0, 0, 0], vy=[0, 0, 0], vz=[0, 0, 0], pt=[2.0, 0.8, 5.0], tanl=[0.2, 0.5, 0.8],
                 phi0=[math.radians(8.0), math.radians(12.0), math.radians(4.0)], q=[1, -1, 1])
    cs = synth.generate_raw(3, 1, [0], explicit=truth, sigma=0.0, noise_frac=0.0, shuffle=False)
    cs = cs.subset([0])  # sector 0 (A side)
    for prec, tol in ((64, 1e-6), (32, 2e-4)):
        res = oracle.run(cs, prec)
        labels = [np.unique(cs.label[res.trk_hit[res.trk_hit_start[t]:res.trk_hit_start[t + 1]]])
                  for t in range(res.n_tracks)]
        assert all(len(l) == 1 for l in labels)
        assert sorted(int(l[0]) for l in labels) == [0, 1, 2]
        assert len(res.trk_hit) == len(cs.y)  # every cluster assigned
        from helix_truth import LocalHelix
        for t in range(res.n_tracks):
            k = int(labels[t][0])
            h = LocalHelix(truth["pt"][k], truth["q"][k], truth["tanl"][k], truth["phi0"][k],
                           math.radians(10.0))
            ref = h.at(res.trk_x[t])
            assert np.allclose(res.trk_param[t], ref, rtol=tol, atol=tol)


def test_fp32_and_fp64_oracles_agree(c1, c1_run):
    r64 = oracle.run(c1, 64)
    assert np.array_equal(r64.up, c1_run.up) and np.array_equal(r64.start_hit, c1_run.start_hit)
    assert np.array_equal(r64.trk_hit, c1_run.trk_hit)
    floors = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
    d = np.abs(r64.trk_param - c1_run.trk_param)
    assert np.all(d <= 1e-4 * np.maximum(np.abs(r64.trk_param), floors))


def test_qa_regression_gates(c1, c1_run, c2s, c2s_run):
    # thresholds frozen from the first oracle run (the paper's efficiency
    # figures are not available): findable = >= 70 clusters in the sector
    q1 = qa.evaluate(c1, c1_run.trk_hit_start, c1_run.trk_hit)
    assert q1["efficiency"] >= 0.98 and q1["clone_rate"] <= 0.01 and q1["fake_rate"] <= 0.01
    q2 = qa.evaluate(c2s, c2s_run.trk_hit_start, c2s_run.trk_hit)
    assert q2["efficiency"] >= 0.99 and q2["clone_rate"] <= 0.01 and q2["fake_rate"] <= 0.01
    assert c2s_run.chi2_total / c2s_run.ndf_total == pytest.approx(1.0, abs=0.06)


def test_time_shift_invariance(c2s, c2s_run):
    """Continuous readout: tracking without an absolute z (Section 4) finds the
    same tracks when every cluster of an instance is shifted in z."""
    shifted = synth.ClusterSet(c2s.n_inst, c2s.inst_sector, c2s.row_start, c2s.x, c2s.y,
                               (c2s.z.astype(np.float64) - 137.0).astype(np.float32), c2s.row, c2s.label,
                               c2s.truth)
    r = oracle.run(shifted, 32, threads=4)
    q0 = qa.evaluate(c2s, c2s_run.trk_hit_start, c2s_run.trk_hit)
    q1 = qa.evaluate(shifted, r.trk_hit_start, r.trk_hit)
    assert abs(q0["efficiency"] - q1["efficiency"]) < 0.005
    assert abs(r.n_tracks - c2s_run.n_tracks) <= 0.01 * c2s_run.n_tracks


def test_binary32_parameters_within_1e4_of_fp64_replay(c2s, c2s_run):
    """Every selected track of the binary32 oracle against the binary64 replay of
    its own cluster list, start state and accept masks (same detector: binary32
    pad-row planes): |dp| <= 1e-4 max(|p|, floor) for every parameter."""
    inp = oracle.refit_inputs(c2s_run, c2s)
    ok, out, _ = oracle.replay_f64(inp["st0"], inp["row0"], inp["hit_start"], inp["hit_rows"], inp["ys"],
                                   inp["zs"], inp["masks"])
    assert ok.all() and len(ok) == c2s_run.n_tracks
    floors = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
    d = np.abs(c2s_run.trk_param - out[:, :5])
    assert np.all(d <= 1e-4 * np.maximum(np.abs(out[:, :5]), floors)), (d / np.maximum(np.abs(out[:, :5]), floors)).max(0)
