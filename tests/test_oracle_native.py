"""Pins of the oracle's native-coordinate transform (Sections 4 and 6: the
tracker takes pad, row and time and computes space points itself; the time is
scaled linearly to z as for an arbitrarily long chamber). Independent of the
transform's own code: exact values at the pad centre and at the readout plane,
exact binary32 products for whole pad offsets, the side symmetry, the pad
geometry against the sector width, the shift a collision time gives, and the
round trip through the generator's FP64 readout model."""
import math

import numpy as np
import pytest

import oracle
import synth


def _one_row(sector, row, pad, time, geo):
    n_rows = 152
    rs = np.zeros(n_rows + 1, np.int64)
    rs[row + 1:] = len(pad)
    return oracle.native_to_local(n_rows, [sector], rs, np.asarray(pad, np.float32), np.asarray(time, np.float32), geo)


def test_pad_centre_and_readout_plane_are_exact():
    g = oracle.native_geometry()
    for row in (0, 62, 63, 126, 127, 151):
        c = g["pad_center"][row]
        for sector, side in ((0, 1.0), (17, 1.0), (18, -1.0), (35, -1.0)):
            y, z = _one_row(sector, row, [c], [0.0], g)
            assert y[0] == 0.0 and z[0] == np.float32(side * 250.0)


@pytest.mark.parametrize("row", [0, 40, 63, 100, 127, 151])
def test_whole_pad_offsets_give_pitch_multiples(row):
    g = oracle.native_geometry()
    c, w = g["pad_center"][row], g["pad_width"][row]
    k = np.arange(-20, 21, dtype=np.float32)
    y, _ = _one_row(3, row, c + k, np.zeros_like(k), g)
    # c + k is exact (half-integers below 2^23) and so is the subtraction: one rounding, of k * w
    assert np.array_equal(y, (k * w).astype(np.float32))
    assert np.all(np.diff(y) > 0)


def test_sides_are_mirror_images():
    g = oracle.native_geometry()
    t = np.linspace(0.0, 480.0, 97, dtype=np.float32)
    _, za = _one_row(5, 10, np.full_like(t, 7.0), t, g)
    _, zc = _one_row(23, 10, np.full_like(t, 7.0), t, g)
    assert np.array_equal(za, -zc)
    # z decreases along the drift on the A side; the drift of the full length
    # (250 cm / 0.516 cm per bin) reaches the central electrode
    assert np.all(np.diff(za) < 0)
    _, z0 = _one_row(5, 10, [0.0], [250.0 / 0.516], g)
    assert abs(z0[0]) < 1e-4


def test_pad_geometry_covers_each_row_exactly():
    g = oracle.native_geometry()
    t10 = math.tan(math.radians(10.0))
    for row in range(152):
        x = 85.0 + row * 162.0 / 151.0
        w, n = float(g["pad_width"][row]), int(g["n_pads"][row])
        assert n % 2 == 0
        assert n * w >= 2 * x * t10 - 1e-5 and (n - 2) * w < 2 * x * t10
        assert float(g["pad_center"][row]) == (n - 1) / 2
    assert g["pad_width"][0] == np.float32(0.416) and g["pad_width"][63] == np.float32(0.42)
    assert g["pad_width"][127] == np.float32(0.46)
    # the outermost pads reach the sector edge |y| = x tan(10 deg)
    y, _ = _one_row(0, 151, [0.0, float(g["n_pads"][151] - 1)], [0.0, 0.0], g)
    xe = 85.0 + 162.0
    assert -y[0] == pytest.approx(y[1]) and abs(y[1]) <= xe * t10 and abs(y[1]) > xe * t10 - 0.46


def test_collision_time_shifts_z_linearly():
    # continuous readout: the same track from a collision dt bins later is seen
    # shifted by -side * z_per_bin * dt (the convention of the C3 generator)
    g = oracle.native_geometry()
    t = np.array([10.0, 100.0, 300.0], np.float32)
    for sector, side in ((2, 1.0), (20, -1.0)):
        _, z1 = _one_row(sector, 30, [5.0] * 3, t, g)
        _, z2 = _one_row(sector, 30, [5.0] * 3, t + np.float32(64.0), g)
        np.testing.assert_allclose(z2 - z1, -side * 0.516 * 64.0, atol=1e-4)


def test_round_trip_through_the_readout_model():
    cs = synth.generate("C1")
    g = oracle.native_geometry()
    pad, time = synth.to_native(cs, g["pad_width"], g["pad_center"], float(g["z_per_bin"]), float(g["z_readout"]))
    y, z = oracle.native_to_local(152, cs.inst_sector, cs.row_start, pad, time, g)
    # binary32 pad and time round the FP64 readout model (pad ~ 1e2, time ~ 5e2): a few 1e-5 cm
    assert np.max(np.abs(y - cs.y)) < 2e-5 * 0.46 * 64 and np.max(np.abs(z - cs.z)) < 2e-4
    assert np.max(np.abs(y - cs.y)) > 0  # the round trip is not the identity: the tracker sees the transform
