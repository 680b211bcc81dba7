"""Pins of the oracle's differentiable refit: the B-spline correction map, the
cluster correction, the frozen-mask FP64 refit and its finite-difference
reference gradient.

* The map against scipy's B-spline design matrices (an independent
  implementation of the same tensor-product cubic B-splines, periodic in phi
  by wrapped coefficients).
* Partition of unity: constant coefficients give a constant map, and the
  cluster correction then has a closed form.
* The frozen refit reduces to the FP64 replay (and the FP64 run) with no map.
* Translation invariance of the refit in y and z (it uses only differences),
  which fixes the identity sum_k dchi2/dcoef(dz, k) = sum_t dchi2_t/dz0_t.
* The finite-difference gradient is a true derivative: the Taylor remainder
  along a random direction shrinks as h^2.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
import synth

HR, HZ, HP = 168.0 / 13.0, 504.0 / 29.0, 2.0 * np.pi / 16.0


def _design(x, knots, ncoef):
    return BSpline.design_matrix(x, knots, 3, extrapolate=False).toarray()[:, :ncoef]


def scipy_map(coef, r, phi, z):
    coef = np.asarray(coef).reshape(3, 16, 16, 32)
    tr = 84.0 + (np.arange(20) - 3) * HR
    tz = -252.0 + (np.arange(36) - 3) * HZ
    tp = (np.arange(23) - 3) * HP  # 19 wrapped coefficients: column j is coefficient (j - 1) mod 16
    Br = _design(r, tr, 16)
    Bz = _design(z, tz, 32)
    Bp_ext = _design(np.mod(phi, 2 * np.pi), tp, 19)
    Bp = np.zeros((len(phi), 16))
    for j in range(19):
        Bp[:, (j - 1) % 16] += Bp_ext[:, j]
    return np.einsum("na,nb,nc,kabc->nk", Br, Bp, Bz, coef)


def test_map_matches_scipy_bsplines():
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(oracle.MAP_SIZE)
    n = 2000
    r = rng.uniform(84.0, 251.9, n)
    z = rng.uniform(-252.0, 251.9, n)
    phi = rng.uniform(-2 * np.pi, 4 * np.pi, n)  # periodic: any branch
    got = oracle.map_eval(coef, r, phi, z)
    ref = scipy_map(coef, r, phi, z)
    assert np.allclose(got, ref, rtol=0, atol=1e-11), np.abs(got - ref).max()


def test_constant_map_and_closed_form_correction():
    rng = np.random.default_rng(2)
    n = 500
    x = rng.uniform(85.0, 247.0, n)
    y = rng.uniform(-40.0, 40.0, n)
    z = rng.uniform(-250.0, 250.0, n)
    alpha = rng.uniform(0, 2 * np.pi, n)
    c = np.zeros(oracle.MAP_SHAPE)
    c[0], c[1], c[2] = 0.3, -0.7, 1.25
    m = oracle.map_eval(c, np.hypot(x, y), alpha + np.arctan2(y, x), z)
    assert np.allclose(m, [0.3, -0.7, 1.25], atol=1e-13)
    yc, zc = oracle.correct(c, alpha, x, y, z)
    r = np.hypot(x, y)
    assert np.allclose(yc, y - (0.3 * y - 0.7 * x) / r, atol=1e-12)
    assert np.allclose(zc, z - 1.25, atol=1e-12)
    # zero map: identity, exactly
    yc0, zc0 = oracle.correct(np.zeros(oracle.MAP_SIZE), alpha, x, y, z)
    assert np.array_equal(yc0, y) and np.array_equal(zc0, z)


@pytest.fixture(scope="module")
def c1_inputs():
    cs = synth.generate("C1")
    res = oracle.run(cs, 64)
    return cs, res, oracle.refit_inputs(res, cs)


def _f(inp, st0=None, ys=None, zs=None, coef=None):
    return oracle.refit_frozen_f64(inp["st0"] if st0 is None else st0, inp["row0"], inp["alpha"], inp["hit_start"],
                                   inp["hit_rows"], inp["ys"] if ys is None else ys, inp["zs"] if zs is None else zs,
                                   inp["masks"], coef)


def test_frozen_refit_without_map_is_the_replay(c1_inputs):
    cs, res, inp = c1_inputs
    ok, chi2 = _f(inp)
    ok0, chi2_0 = _f(inp, coef=np.zeros(oracle.MAP_SIZE))
    okr, _, chi2_r = oracle.replay_f64(inp["st0"], inp["row0"], inp["hit_start"], inp["hit_rows"], inp["ys"],
                                       inp["zs"], inp["masks"], planes_f32=False)
    assert ok.all() and ok0.all() and okr.all()
    assert np.array_equal(chi2, chi2_0) and np.array_equal(chi2, chi2_r)
    assert np.array_equal(chi2, res.trk_chi2)  # same decisions as the FP64 run itself


def test_refit_is_translation_invariant(c1_inputs):
    _, _, inp = c1_inputs
    _, chi2 = _f(inp)
    for k, key in ((0, "ys"), (1, "zs")):
        st = inp["st0"].copy()
        st[:, k] += 0.37
        kw = {key: inp[key] + 0.37}
        ok, c = _f(inp, st0=st, **kw)
        assert ok.all()
        assert np.allclose(c, chi2, rtol=1e-9, atol=1e-9)
    # and the start state does matter, if very little (three covariance resets)
    st = inp["st0"].copy()
    st[:, 1] += 0.37
    assert not np.allclose(_f(inp, st0=st)[1], chi2, rtol=1e-13, atol=0)


def _touched_coefs(inp, comp):
    """Flat indices of map coefficients whose B-spline support holds a cluster."""
    x = synth.row_plane_x(inp["hit_rows"])
    r = np.hypot(x, inp["ys"])
    phi = np.mod(np.repeat(inp["alpha"], np.diff(inp["hit_start"])) + np.arctan2(inp["ys"], x), 2 * np.pi)
    ir = np.floor(1 + (r - 84.0) / HR).astype(int) - 1
    iz = np.floor(1 + (inp["zs"] + 252.0) / HZ).astype(int) - 1
    ip = np.floor(phi / HP).astype(int) - 1
    out = set()
    for a in range(4):
        for b in range(4):
            for e in range(4):
                out.update((((comp * 16 + ir + a) * 16 + (ip + b) % 16) * 32 + iz + e).tolist())
    return np.array(sorted(out))


def _subset(inp, tracks):
    hs = inp["hit_start"]
    pos = np.concatenate([np.arange(hs[t], hs[t + 1]) for t in tracks])
    lens = hs[np.asarray(tracks) + 1] - hs[np.asarray(tracks)]
    out = {k: inp[k][tracks] for k in ("st0", "row0", "alpha", "inst")}
    out.update({k: inp[k][pos] for k in ("hit_rows", "hit_id", "ys", "zs", "masks")})
    out["hit_start"] = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return out


def test_fd_gradient_invariant_and_locality(c1_inputs):
    _, _, inp = c1_inputs
    sub = _subset(inp, [0, 7, 21])
    touched = _touched_coefs(sub, 2)
    far = np.array([2 * 8192 + 5, 2 * 8192 + 8191, 0])  # r/z corners no cluster reaches
    ok, gp, gc = oracle.frozen_chi2_grad_fd(sub, coef_index=np.concatenate([touched, far]))
    assert ok.all()
    assert np.all(gc[len(touched):] == 0.0)
    # sum over dz coefficients = sum of d chi2 / d z0 (partition of unity + invariance)
    lhs, rhs = gc[:len(touched)].sum(), gp[:, 1].sum()
    assert abs(lhs - rhs) <= 1e-6 * max(1.0, np.abs(gc).sum()), (lhs, rhs)
    assert np.abs(gc[:len(touched)]).max() > 1e-3


def test_fd_gradient_taylor_remainder_is_second_order(c1_inputs):
    _, _, inp = c1_inputs
    sub = _subset(inp, [3, 11])
    rng = np.random.default_rng(5)
    idx = _touched_coefs(sub, 0)[::7]
    coef0 = np.zeros(oracle.MAP_SIZE)
    coef0[_touched_coefs(sub, 2)] = 0.02 * rng.standard_normal(len(_touched_coefs(sub, 2)))
    ok, gp, gc = oracle.frozen_chi2_grad_fd(sub, coef=coef0, coef_index=idx)
    assert ok.all()
    d_st = np.zeros_like(sub["st0"])
    d_st[:, :5] = rng.standard_normal((len(sub["row0"]), 5)) * [1e-2, 1e-2, 1e-4, 1e-4, 1e-3]
    d_c = np.zeros(oracle.MAP_SIZE)
    d_c[idx] = rng.standard_normal(len(idx)) * 1e-2
    f0 = _f(sub, coef=coef0)[1].sum()
    lin = (gp * d_st[:, :5]).sum() + (gc * d_c[idx]).sum()
    rem = []
    for h in (1.0, 0.5, 0.25):
        fh = _f(sub, st0=sub["st0"] + h * d_st, coef=coef0 + h * d_c)[1].sum()
        rem.append(abs(fh - f0 - h * lin))
    assert abs(lin) > 10 * rem[0]
    for a, b in zip(rem, rem[1:]):
        assert 3.0 < a / b < 5.0, rem
