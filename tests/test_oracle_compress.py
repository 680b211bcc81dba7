"""Pins of the oracle's track-model residual codec (Section 5.1 of the paper:
clusters attached to tracks are stored as residuals to the track model).
Independent references: closed-form helices (tests/helix_truth.py) with known
offsets, the round trip through the decoder, and the entropy of a Gaussian
of the generator's smear."""
import math

import numpy as np
import pytest

import oracle
import synth
from helix_truth import LocalHelix, plane_x

STEP = 2.0 ** -7  # cm


def _helix_track(pt=1.5, q=1, rows=np.arange(10, 110)):
    h = LocalHelix(pt, q, tanl=0.4, phi0=0.05, alpha=0.0)
    truth = np.array([h.at(plane_x(r)) for r in rows])
    return rows, truth


def test_noiseless_helix_has_zero_residuals():
    rows, truth = _helix_track()
    ys, zs = truth[:, 0].astype(np.float32), truth[:, 1].astype(np.float32)
    q, n_esc = oracle.track_residuals(truth[0], rows, ys, zs)
    assert n_esc == 0 and np.abs(q).max() <= 1


def test_known_offset_is_its_residual():
    rows, truth = _helix_track(pt=0.7, q=-1)
    ys, zs = truth[:, 0].copy(), truth[:, 1].copy()
    ys[37] += 0.3125     # 40 steps
    zs[61] -= 0.078125   # 10 steps
    q, n_esc = oracle.track_residuals(truth[0], rows, ys, zs)
    assert n_esc == 0
    assert q[37, 0] == 40 and q[61, 1] == -10
    others = np.ones(len(rows), bool)
    others[[37, 61]] = False
    assert np.abs(q[others]).max() <= 1


def test_escape_for_large_residuals_and_failed_steps():
    rows, truth = _helix_track()
    ys = truth[:, 0].copy()
    ys[5] += 1000.0
    q, n_esc = oracle.track_residuals(truth[0], rows, ys, truth[:, 1])
    assert q[5, 0] == oracle.RES_ESCAPE and n_esc == 1
    # a state that leaves the |sin phi| guard within a few rows: every later cluster escapes
    st = truth[0].copy()
    st[2], st[4] = 0.94, -8.0
    q, n_esc = oracle.track_residuals(st, rows, truth[:, 0], truth[:, 1])
    assert (q[:, 0] == oracle.RES_ESCAPE).sum() > 50 and q[0, 0] != oracle.RES_ESCAPE


def test_round_trip_and_entropy_on_found_tracks():
    cs = synth.generate("C1")
    r = oracle.run(cs, 32)
    seg = np.searchsorted(cs.row_start, r.trk_hit, side="right") - 1
    rows = (seg % 152).astype(np.int32)
    xplanes = np.array([np.float32(plane_x(i)) for i in range(152)])
    allq = []
    for t in range(r.n_tracks):
        a, b = r.trk_hit_start[t], r.trk_hit_start[t + 1]
        ids = r.trk_hit[a:b]
        row0 = int(np.nonzero(xplanes == np.float32(r.trk_x[t]))[0][0])  # the final fit's reference row
        assert row0 <= rows[a]
        q, n_esc = oracle.track_residuals(r.trk_param[t], rows[a:b], cs.y[ids], cs.z[ids], row0=row0)
        assert n_esc == 0
        yd, zd = oracle.track_decode(r.trk_param[t], rows[a:b], q, row0=row0)
        assert np.all(np.abs(yd - cs.y[ids]) <= STEP / 2 + 1e-5)
        assert np.all(np.abs(zd - cs.z[ids]) <= STEP / 2 + 1e-5)
        allq.append(q)
    q = np.concatenate(allq)
    # smear sigma 0.1 cm in STEP units: a Gaussian's entropy log2(sigma/step sqrt(2 pi e))
    h_gauss = math.log2(0.1 / STEP * math.sqrt(2 * math.pi * math.e))
    for c in range(2):
        v, n = np.unique(q[:, c], return_counts=True)
        p = n / n.sum()
        h = -(p * np.log2(p)).sum()
        assert h_gauss - 0.6 <= h <= h_gauss + 0.2, (c, h, h_gauss)
