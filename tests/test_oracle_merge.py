"""Pins of the oracle's cross-sector merge (the second phase of Section 2:
segments found in the individual sectors are merged and fitted as one
track). Independent references: closed-form helices crossing sector
boundaries (tests/helix_truth.py, the generator's exact plane crossings), the
Monte-Carlo labels of the central event, and event separation."""
import math

import numpy as np
import pytest

import oracle
import synth
from helix_truth import LocalHelix


def _phi0_crossing(pt, q, r_cross, boundary_deg):
    """Vertex direction of a helix from the origin whose position angle reaches
    the sector boundary at radius r_cross (a positive charge turns clockwise)."""
    R = pt / (0.00299792458 * 0.5)
    return math.radians(boundary_deg) + (1 if q > 0 else -1) * math.asin(r_cross / (2 * R))


HELICES = [  # pt, q, tanl, vz, crossing radius, boundary (deg)
    (0.5, 1, 0.3, 0.0, 150.0, 0.0),
    (0.6, -1, 0.5, 0.0, 170.0, 20.0),
    (0.8, 1, -0.4, 5.0, 120.0, 220.0),
    (2.0, -1, 0.1, -3.0, 200.0, 100.0),
]


def _event(helices, sigma=0.0, seed=5):
    ex = dict(vx=[0.0] * len(helices), vy=[0.0] * len(helices), vz=[h[3] for h in helices],
              pt=[h[0] for h in helices], tanl=[h[2] for h in helices], q=[h[1] for h in helices],
              phi0=[_phi0_crossing(h[0], h[1], h[4], h[5]) for h in helices])
    return synth.generate_raw(3, 1, [len(helices)], explicit=ex, sigma=sigma, noise_frac=0.0, seed=seed)


def test_noiseless_helices_crossing_sector_boundaries_merge_exactly():
    cs = _event(HELICES)
    for t in range(len(HELICES)):
        assert len(np.unique(cs.instance_of()[cs.label == t])) == 2  # each crosses one boundary
    r = oracle.run(cs, 64, inst_event=np.zeros(cs.n_inst, np.int32))
    m = r.merged
    assert r.n_tracks == 2 * len(HELICES)
    assert len(m["src"]) == len(HELICES) and np.all(m["nseg"] == 2)
    for j in range(len(HELICES)):
        hits = m["hit_id"][m["hit_start"][j]:m["hit_start"][j + 1]]
        lab = cs.label[hits]
        assert np.all(lab == lab[0]) and len(hits) == np.sum(cs.label == lab[0])  # every cluster, one helix
        assert m["chi2"][j] < 1e-6
        pt, q, tanl, vz = cs.truth[lab[0], 3], cs.truth[lab[0], 6], cs.truth[lab[0], 4], cs.truth[lab[0], 2]
        h = LocalHelix(pt, q, tanl, cs.truth[lab[0], 5], m["alpha"][j], vz=vz)
        assert np.allclose(m["param"][j], h.at(m["x_ref"][j]), rtol=1e-7, atol=1e-7)
    # binary32: the same merged cluster lists, parameters to binary32 accuracy
    r32 = oracle.run(cs, 32, inst_event=np.zeros(cs.n_inst, np.int32))
    assert np.array_equal(r32.merged["hit_id"], m["hit_id"]) and np.array_equal(r32.merged["nseg"], m["nseg"])
    assert np.allclose(r32.merged["param"], m["param"], rtol=1e-4, atol=1e-4)


def test_segments_of_different_events_are_not_merged():
    one = _event(HELICES[:2])
    two = _event(HELICES[2:], seed=6)
    # two events side by side: instances 0..35 event 0, 36..71 event 1
    cs = synth.ClusterSet(72, np.concatenate([one.inst_sector, two.inst_sector]),
                          np.concatenate([one.row_start, two.row_start[1:] + one.row_start[-1]]),
                          np.concatenate([one.x, two.x]), np.concatenate([one.y, two.y]),
                          np.concatenate([one.z, two.z]), np.concatenate([one.row, two.row]),
                          np.concatenate([one.label, two.label + 100]), one.truth)
    ev = np.repeat([0, 1], 36).astype(np.int32)
    r = oracle.run(cs, 64, inst_event=ev)
    assert len(r.merged["src"]) == 4 and np.all(r.merged["nseg"] == 2)
    for j in range(4):
        hits = r.merged["hit_id"][r.merged["hit_start"][j]:r.merged["hit_start"][j + 1]]
        assert len(np.unique(cs.label[hits])) == 1
    # the same data as one event: the segments of the two events now share
    # sectors, and the merge still pairs each with its own continuation
    r1 = oracle.run(cs, 64, inst_event=np.zeros(72, np.int32))
    for j in range(len(r1.merged["src"])):
        hits = r1.merged["hit_id"][r1.merged["hit_start"][j]:r1.merged["hit_start"][j + 1]]
        assert len(np.unique(cs.label[hits])) == 1


def test_merge_qa_on_central_event_sectors():
    """Sectors 0-5 and 18-23 of the central event (adjacent sectors of both
    sides): every link joins segments of one Monte-Carlo track, most segments
    of a track in adjacent sectors are linked, and merged tracks fit with
    chi2/ndf near one. Gates frozen from the first run."""
    c2 = synth.generate("C2")
    cs = c2.subset(list(range(0, 6)) + list(range(18, 24)))
    r = oracle.run(cs, 32, threads=4, inst_event=np.zeros(cs.n_inst, np.int32))
    m = r.merged
    nt = r.n_tracks

    def label(hits):
        lab = cs.label[hits]
        lab = lab[lab >= 0]
        if not len(lab):
            return -1
        v, c = np.unique(lab, return_counts=True)
        return v[np.argmax(c)]

    tl = np.array([label(r.trk_hit[r.trk_hit_start[t]:r.trk_hit_start[t + 1]]) for t in range(nt)])
    a = np.nonzero(m["next"] >= 0)[0]
    assert len(a) > 500
    assert np.mean(tl[a] == tl[m["next"][a]]) >= 0.995
    sec = cs.inst_sector[r.trk_inst]
    ideal = 0
    for lab in np.unique(tl[tl >= 0]):
        s = sorted(set(sec[tl == lab].tolist()))
        ideal += sum(1 for x, y in zip(s, s[1:]) if y - x == 1 and x // 18 == y // 18)
    assert len(a) >= 0.85 * ideal, (len(a), ideal)
    multi = m["nseg"] > 1
    assert abs(np.sum(m["chi2"][multi]) / np.sum(m["ndf"][multi]) - 1.0) < 0.06
