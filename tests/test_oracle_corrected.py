"""Pins of the oracle's corrected final fit (Section 4: with a track's vertex
z, i.e. its collision time, known, the z-dependent space-point correction is
applied and the track fitted again). Independent of the fit's own code: the
result cannot depend on the frame the vertex z moves it to; a map that is
constant in one component must act as that constant shift of every cluster
(the B-spline weights sum to one), checked against the closed-form in-plane
corrections written out here; the refined vertex z of a frame-shifted fit."""
import math

import numpy as np
import pytest

import oracle
import synth

MAP = 3 * 16 * 16 * 32


@pytest.fixture(scope="module")
def tracks():
    cs = synth.generate("C1")
    r = oracle.run(cs, 64)
    hs = r.trk_hit_start
    ids = r.trk_hit
    rows = cs.row[ids]
    st0 = np.concatenate([r.trk_param, r.trk_cov], axis=1)
    X = np.array([float(np.float32(85.0 + i * 162.0 / 151.0)) for i in range(152)])
    row0 = np.array([int(np.argmin(np.abs(X - x))) for x in r.trk_x], np.int32)
    alpha = np.asarray(r.trk_alpha, np.float64)
    return dict(st0=st0, row0=row0, alpha=alpha, hs=hs, rows=rows, ys=cs.y[ids].astype(np.float64),
                zs=cs.z[ids].astype(np.float64), X=X, n=len(st0))


def _fit(t, z0, coef=None, ys=None, zs=None, st0=None):
    return oracle.fit_corrected(t["st0"] if st0 is None else st0, t["row0"], z0, t["alpha"], t["hs"], t["rows"],
                                t["ys"] if ys is None else ys, t["zs"] if zs is None else zs, coef=coef)


def test_result_does_not_depend_on_the_frame(tracks):
    t = tracks
    a = _fit(t, np.zeros(t["n"]))
    assert a["ok"].all() and t["n"] > 50
    for c in (37.5, -120.0):
        b = _fit(t, np.full(t["n"], c))
        assert np.array_equal(a["ok"], b["ok"]) and np.array_equal(a["masks"], b["masks"])
        assert np.array_equal(a["nacc"], b["nacc"]) and np.array_equal(a["row"], b["row"])
        d = a["state"] - b["state"]
        d[:, 1] -= c  # the output z is in the absolute frame, moved by the vertex z
        np.testing.assert_allclose(d, 0.0, atol=1e-9 * (1 + abs(c)))
        np.testing.assert_allclose(a["chi2"], b["chi2"], rtol=1e-9, atol=1e-9)
        # the refined vertex z is frame-free: the closest approach moves with the frame
        np.testing.assert_allclose(a["z0"], b["z0"], atol=1e-9 * (1 + abs(c)))


def test_constant_dz_map_is_a_z_shift_of_every_cluster(tracks):
    t = tracks
    c = 0.37
    coef = np.zeros(MAP)
    coef[2 * 8192:] = c
    st = t["st0"].copy()
    st[:, 1] -= c
    a = _fit(t, np.zeros(t["n"]), coef=coef, st0=st)
    b = _fit(t, np.zeros(t["n"]), zs=t["zs"] - c, st0=st)
    assert np.array_equal(a["masks"], b["masks"])
    np.testing.assert_allclose(a["state"], b["state"], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("comp", [0, 1])
def test_constant_in_plane_maps_match_the_closed_form(tracks, comp):
    t = tracks
    c = 0.21
    coef = np.zeros(MAP)
    coef[comp * 8192:(comp + 1) * 8192] = c
    x = t["X"][t["rows"]]
    y = t["ys"]
    R = np.sqrt(x * x + y * y)
    # comp 0: radial shift dr (y moves by dr * y / R); comp 1: azimuthal r*dphi (y moves by r dphi * x / R)
    yc = y - (c * y / R if comp == 0 else c * x / R)
    a = _fit(t, np.zeros(t["n"]), coef=coef)
    b = _fit(t, np.zeros(t["n"]), ys=yc)
    assert np.array_equal(a["masks"], b["masks"])
    np.testing.assert_allclose(a["state"], b["state"], rtol=1e-10, atol=1e-12)
    assert np.abs(a["state"][:, 0] - _fit(t, np.zeros(t["n"]))["state"][:, 0]).max() > 1e-3  # the map acted


def test_refined_vertex_z_of_primaries(tracks):
    # C1 helices come from the origin: the refined vertex z of a frame
    # shifted by any z0 lands back near z = 0 in the original frame
    t = tracks
    for c in (0.0, 55.0):
        b = _fit(t, np.full(t["n"], c))
        assert np.median(np.abs(b["z0"])) < 0.2
