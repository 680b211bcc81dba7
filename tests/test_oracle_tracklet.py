"""Pins of the oracle's track following (tracklet construction).

Paper, Section 2: after the cellular automaton, each segment is fitted with a
simplified Kalman filter, extrapolated row by row and the best hit of each row
is attached (no multiple hypotheses). Section 3: the filter then turns and
propagates inward through the initial seed, rejecting outlier clusters.

Pinned here, against values fixed by hand or by an independent derivation:
* the pick rule on one row (hand-worked cases in tests/golden/pick_cases.json:
  inclusive window on sqrt(C + V), inclusive chi2 cut, minimum chi2, ties to
  the smaller input id, correlated covariance);
* the stop after exactly MAX_MISS empty rows, outward and inward;
* the turn at the last picked row (stage 3 picks nothing beyond it);
* the inward pass through the seed dropping or replacing an outlier seed hit;
* the weight rule of overlapping tracklets (more hits win, then the lower id);
* a second FP64 derivation of whole tracklets (tests/tracklet_fp64.py: exact
  circle steps, numeric Jacobian, matrix Kalman update) on real-density input.
Clusters of the hand cases are noiseless points of closed-form helices
(tests/helix_truth.py), so every expectation follows from the construction.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
import tracklet_fp64 as T
from helix_truth import LocalHelix, plane_x
from util import make_clusterset, row_of_ids

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA0 = math.radians(10.0)  # centre of sector 0


def _cand(c):
    if isinstance(c[0], str):
        op, y, z = c
        y, z = np.float32(y), np.float32(z)
        if op == "y_next_up":
            y = np.nextafter(y, np.float32(np.inf) * np.sign(y))
        elif op == "z_next_down":
            z = np.nextafter(z, np.float32(np.inf) * np.sign(z))
        else:
            raise ValueError(op)
        return y, z
    return np.float32(c[0]), np.float32(c[1])


@pytest.mark.parametrize("prec", [32, 64])
def test_golden_pick_cases(prec):
    cases = json.load(open(os.path.join(GOLDEN, "pick_cases.json")))["cases"]
    for case in cases:
        st = np.zeros(20)
        st[:5] = case["p"]
        st[5 + 0], st[5 + 1], st[5 + 2] = case["C00"], case["C10"], case["C11"]
        st[5 + 5] = st[5 + 9] = 0.01  # other variances: irrelevant to the pick, kept positive
        st[5 + 14] = 1.0
        cands = [_cand(c) for c in case["cands"]]
        ys = np.array([c[0] for c in cands], np.float32)
        zs = np.array([c[1] for c in cands], np.float32)
        params = oracle.default_params(**case.get("params", {}))
        idx, chi2 = oracle.pick(st, ys, zs, precision=prec, params=params)
        assert idx == case["expect"], (case["name"], prec, idx)
        if "chi2" in case and prec == 32:
            assert chi2 == case["chi2"], (case["name"], chi2)
        elif "chi2" in case:
            assert abs(chi2 - case["chi2"]) <= 1e-12 * case["chi2"], (case["name"], chi2)


# ------------------------------------------------------------ hand-built tracks
def _helix(pt=5.0, q=1, tanl=0.3, dphi=0.02):
    return LocalHelix(pt, q, tanl, ALPHA0 + dphi, ALPHA0)


def _hits(h, rows, dy=None):
    dy = dy or {}
    out = []
    for r in rows:
        v = h.at(plane_x(r))
        out.append((0, r, float(v[0]) + dy.get(r, 0.0), float(v[1])))
    return out


def _run(hits, prec):
    cs = make_clusterset(hits)
    return cs, oracle.run(cs, prec)


def _tracklet_rows(cs, res, start_row):
    """Rows picked by the tracklet whose start hit lies on start_row."""
    rows = row_of_ids(cs)
    k = [i for i, h in enumerate(res.start_hit) if rows[h] == start_row]
    assert len(k) == 1, (start_row, [rows[h] for h in res.start_hit])
    k = k[0]
    rh = res.tl_rowhit[k]
    return k, {r: int(rh[r]) for r in range(len(rh)) if rh[r] >= 0}


def _id_on(cs, row, index_in_row=0):
    return int(cs.row_start[row] + index_in_row)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("gap", [7, 8])
def test_outward_following_stops_after_max_miss_empty_rows(prec, gap):
    # track on rows 20..59, `gap` empty rows, then rows up to 120; the chain of
    # the first segment is rows 21..58 (row 20 and 59 have no neighbour pair)
    rows = list(range(20, 60)) + list(range(60 + gap, 121))
    cs, res = _run(_hits(_helix(), rows), prec)
    k, picked = _tracklet_rows(cs, res, 21)
    if gap < 8:  # 7 misses: the following goes on across the gap
        assert sorted(picked) == rows
    else:  # the 8th consecutive miss ends the outward following at row 67
        assert sorted(picked) == list(range(20, 60))
        assert res.tl_row[k] == 59 + 8
    assert res.tl_nhits[k] == len(picked)
    for r, h in picked.items():
        assert h == _id_on(cs, r)


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("gap", [7, 8])
def test_inward_pass_stops_after_max_miss_empty_rows(prec, gap):
    # rows 10..40, `gap` empty rows, rows above up to 130: the tracklet seeded in
    # the upper segment runs inward through the gap only if it is under 8 rows
    lo = list(range(10, 41))
    hi0 = 41 + gap
    rows = lo + list(range(hi0, 131))
    cs, res = _run(_hits(_helix(pt=3.0, q=-1), rows), prec)
    k, picked = _tracklet_rows(cs, res, hi0 + 1)
    if gap < 8:
        assert sorted(picked) == rows
    else:
        assert sorted(picked) == list(range(hi0, 131))


@pytest.mark.parametrize("prec", [32, 64])
def test_inward_pass_starts_at_the_last_picked_row(prec):
    # the track ends at row 99; a stray cluster 1 cm off the track on row 101
    # is outside the outward window, but inside the inflated window after the
    # turn: the inward pass must not look at rows beyond the last pick
    h = _helix()
    rows = list(range(20, 100))
    hits = _hits(h, rows)
    v = h.at(plane_x(101))
    hits.append((0, 101, float(v[0]) + 1.0, float(v[1])))
    cs, res = _run(hits, prec)
    k, picked = _tracklet_rows(cs, res, 21)
    assert sorted(picked) == rows
    assert res.tl_row[k] == 99 + 8  # the state is where the outward following ended
    # the stray cluster would qualify for the pick rule with the state after the
    # turn (covariance reset at row 107, then moved row by row to row 101)
    st = _reset(res.tl_state[k])
    for r in range(107, 101, -1):
        ok, st = oracle.propagate(st, plane_x(r), plane_x(r - 1), precision=64)
        assert ok
    idx, _ = oracle.pick(st, np.array([hits[-1][2]], np.float32), np.array([hits[-1][3]], np.float32))
    assert idx == 0


def _reset(state20):
    """The turn's covariance reset: correlations dropped, variances scaled."""
    st = np.array(state20, np.float64)
    scale = oracle.default_params().cov_reset
    for i in range(5):
        for j in range(i + 1):
            q = 5 + i * (i + 1) // 2 + j
            st[q] = st[q] * scale if i == j else 0.0
    return st


@pytest.mark.parametrize("prec", [32, 64])
def test_inward_pass_drops_an_outlier_seed_hit(prec):
    # the cluster on row 40 is 0.45 cm off: close enough to a straight line for
    # the cellular automaton (deviation 0.2 cm^2 <= 0.24), so the seed chain runs
    # through it, but outside the 3 sigma window of the fitted track
    rows = list(range(20, 101))
    cs, res = _run(_hits(_helix(), rows, dy={40: 0.45}), prec)
    o = _id_on(cs, 40)
    assert res.upc[_id_on(cs, 39)] == o and res.upc[o] == _id_on(cs, 41)
    k, picked = _tracklet_rows(cs, res, 21)
    assert 40 not in picked
    assert sorted(picked) == [r for r in rows if r != 40]


@pytest.mark.parametrize("prec", [32, 64])
def test_inward_pass_replaces_an_outlier_seed_hit(prec):
    # rows 39, 40, 41 are 0.25 cm off, so the automaton links the displaced
    # cluster O of row 40 (a straight line through its displaced neighbours);
    # the true cluster R of row 40 (input after O) is left unlinked. The inward
    # pass re-picks row 40 and takes R, the better fit to the whole track.
    h = _helix()
    rows = list(range(20, 101))
    hits = _hits(h, rows, dy={39: 0.25, 40: 0.25, 41: 0.25})
    v = h.at(plane_x(40))
    hits.append((0, 40, float(v[0]), float(v[1])))
    cs, res = _run(hits, prec)
    o, r_true = _id_on(cs, 40, 0), _id_on(cs, 40, 1)
    assert res.upc[_id_on(cs, 39)] == o and res.upc[o] == _id_on(cs, 41)
    assert res.upc[r_true] == -1 and res.dnc[r_true] == -1
    k, picked = _tracklet_rows(cs, res, 21)
    assert picked[40] == r_true
    assert picked[39] == _id_on(cs, 39) and picked[41] == _id_on(cs, 41)
    assert sorted(picked) == rows


@pytest.mark.parametrize("prec", [32, 64])
def test_overlapping_tracklets_weight_and_ownership(prec):
    # gap of 7: two chains (rows 21..58 and 68..119) grow into the same 94-hit
    # tracklet; equal hit counts, so the lower tracklet id owns every cluster
    rows = list(range(20, 60)) + list(range(67, 121))
    cs, res = _run(_hits(_helix(), rows), prec)
    assert len(res.start_hit) == 2
    assert list(res.tl_nhits) == [len(rows), len(rows)]
    w0 = (len(rows) << 20) | (0xFFFFF - 0)
    assert np.all(res.weight == w0)
    assert list(res.sel_tl) == [0]
    assert res.n_tracks == 1


# ------------------------------------------------ independent FP64 derivation
@pytest.fixture(scope="module")
def c1_f64():
    cs = synth.generate("C1")
    return cs, oracle.run(cs, 64)


def test_tracklets_match_an_independent_fp64_derivation(c1_f64):
    cs, res = c1_f64
    P = T.Params()
    rows = row_of_ids(cs)
    nr = synth.N_ROWS
    row_y = [cs.y[cs.row_start[r]:cs.row_start[r + 1]].astype(np.float64) for r in range(nr)]
    row_z = [cs.z[cs.row_start[r]:cs.row_start[r + 1]].astype(np.float64) for r in range(nr)]
    rng = np.random.default_rng(7)
    sample = rng.choice(len(res.start_hit), size=min(60, len(res.start_hit)), replace=False)
    compared = 0
    for k in sample:
        chain = [int(res.start_hit[k])]
        while res.upc[chain[-1]] >= 0:
            chain.append(int(res.upc[chain[-1]]))
        crow = [int(rows[h]) for h in chain]
        ref = T.tracklet(crow, cs.y[chain].astype(np.float64), cs.z[chain].astype(np.float64), row_y, row_z, P)
        if ref is None:
            assert res.tl_nhits[k] == 0
            continue
        if ref["margin"] < 1e-6:  # a decision within rounding of its threshold
            continue
        compared += 1
        got = {r: int(h - cs.row_start[r]) for r, h in enumerate(res.tl_rowhit[k]) if h >= 0}
        assert got == ref["rowpick"], k
        assert res.tl_nhits[k] == ref["nhits"]
        assert res.tl_row[k] == ref["state_row"]
        st = res.tl_state[k]
        scale = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
        assert np.all(np.abs(st[:5] - ref["state"][:5]) <= 1e-7 * np.maximum(np.abs(ref["state"][:5]), scale)), k
        cov = ref["state"][5:]
        assert np.all(np.abs(st[5:] - cov) <= 1e-6 * np.sqrt(np.abs(np.outer(np.diag(_unpack(cov)),
                                                                           np.diag(_unpack(cov))))[
            np.tril_indices(5)]) + 1e-12), k
    assert compared >= 0.9 * len(sample), compared


def _unpack(c15):
    C = np.zeros((5, 5))
    C[np.tril_indices(5)] = c15
    return C + np.tril(C, -1).T
