"""Pins of the synthetic input generator: noiseless clusters lie on the
analytic helix, workloads have the stated sizes and structure."""
import math

import numpy as np
import pytest

import synth


def _global_xy(x_loc, y_loc, sector):
    al = np.radians((sector % 18 + 0.5) * 20.0)
    return x_loc * np.cos(al) - y_loc * np.sin(al), x_loc * np.sin(al) + y_loc * np.cos(al)


def test_noiseless_clusters_lie_on_their_helix():
    ev = synth.generate_raw(1, 1, [300], sec_frac=0.2, sigma=0.0, noise_frac=0.0, seed=77)
    inst = ev.instance_of()
    gx, gy = _global_xy(ev.x.astype(np.float64), ev.y.astype(np.float64), ev.inst_sector[inst])
    for t in np.unique(ev.label):
        m = ev.label == t
        vx, vy, vz, pt, tanl, phi0, q, dz = ev.truth[t]
        R = pt / (0.00299792458 * 0.5)
        sigma = -q  # positive charges turn clockwise in +Bz
        cx, cy = vx - sigma * R * math.sin(phi0), vy + sigma * R * math.cos(phi0)
        # on the circle (float32 storage of the local coordinates)
        d = np.hypot(gx[m] - cx, gy[m] - cy)
        assert np.all(np.abs(d - R) < 2e-4 * max(1.0, R / 250.0))
        # z = vz + tan(lambda) * arc length from the vertex along the motion
        ang0 = math.atan2(vy - cy, vx - cx)
        ang = np.arctan2(gy[m] - cy, gx[m] - cx)
        turn = np.mod((ang - ang0) * sigma, 2 * math.pi)
        assert np.allclose(ev.z[m], vz + tanl * R * turn, atol=2e-4 * (1 + abs(tanl) * R / 250))
        # x on the pad-row plane, |y| inside the sector
        assert np.all(np.abs(ev.y[m]) <= ev.x[m] * math.tan(math.radians(10)) + 1e-4)


def test_workload_sizes():
    c2 = synth.generate("C2")
    assert 1.2e6 < c2.n_clusters < 1.5e6 and c2.n_inst == 36
    assert len(c2.truth) == 8800
    noise = np.mean(c2.label < 0)
    assert noise == pytest.approx(0.02 / 1.02, rel=0.05)
    c1 = synth.generate("C1")
    # one 20-degree sector keeps ~50 clusters per helix: low-pT helices leave it
    assert 8e3 < c1.n_clusters < 13e3 and c1.n_inst == 1
    assert np.all(c1.z >= -1.0)  # A side
    # CSR is consistent with the row array
    rows = np.repeat(np.arange(c1.n_inst * 152) % 152, np.diff(c1.row_start))
    assert np.array_equal(rows, c1.row)


def test_generator_is_seeded():
    a = synth.generate("C1")
    b = synth.generate("C1")
    c = synth.generate("C1", event=1)
    assert np.array_equal(a.y, b.y) and np.array_equal(a.z, b.z)
    assert a.n_clusters != c.n_clusters or not np.array_equal(a.y, c.y)


def test_distortion_displaces_clusters_by_the_stated_field():
    """Same seed with and without the space-charge displacement: the clusters
    move by the local-y and z components of the stated smooth field."""
    a = synth.generate_raw(0, 1, [200], [0], noise_frac=0.0, seed=7, shuffle=False)
    b = synth.generate_raw(0, 1, [200], [0], noise_frac=0.0, seed=7, shuffle=False, distort=True)
    assert np.array_equal(a.label, b.label) and np.array_equal(a.row, b.row)
    x = synth.row_plane_x(a.row)
    y = a.y.astype(np.float64)
    z = a.z.astype(np.float64)
    r = np.hypot(x, y)
    phi = 0.5 * 20.0 * np.pi / 180.0 + np.arctan2(y, x)
    ang, zz = np.pi * (r - 85.0) / 166.0, z / 250.0
    dr = 0.5 * np.sin(ang) * (0.6 + 0.4 * np.cos(phi)) * (1.0 - zz * zz)
    drphi = 0.3 * np.cos(2.0 * ang) * np.sin(2.0 * phi) * zz
    dz = 0.2 * np.sin(np.pi * zz) * np.cos(ang)
    # evaluated at the smeared position: error ~ field gradient x smear
    assert np.abs((b.y - a.y) - (dr * y + drphi * x) / r).max() < 3e-3
    assert np.abs((b.z - a.z) - dz).max() < 3e-3
    assert np.abs(b.z - a.z).max() > 0.1
