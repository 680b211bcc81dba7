"""Pins of the oracle's frame rotation (the state carried into a neighbouring
sector's frame; Section 2's merge of sector segments and Section 4's arbitrary
rotations). Independent reference: the closed-form helix (tests/helix_truth.py)
built from the state and intersected with the new frame's plane, and a
numeric Jacobian of that exact map for the covariance."""
import math

import numpy as np
import pytest

import oracle
from helix_truth import LocalHelix

C_LIGHT = 0.00299792458


def _helix_from_state(st, x0, alpha, bz=0.5):
    """Exact helix through the local state (y, z, sin phi, tan lambda, q/pT) at x0."""
    y, z, sp, tl, qpt = st[:5]
    ca, sa = math.cos(alpha), math.sin(alpha)
    gx, gy = x0 * ca - y * sa, x0 * sa + y * ca
    phi = math.asin(sp) + alpha
    return LocalHelix(1.0 / abs(qpt), 1 if qpt > 0 else -1, tl, phi, 0.0, vx=gx, vy=gy, vz=z), (gx, gy)


def _exact_new_state(st, x0, alpha, d, xnew):
    h, _ = _helix_from_state(st, x0, alpha)
    h2 = LocalHelix(h.pt, h.q, h.tanl, h.phi, alpha + d, vx=h.xv, vy=h.yv, vz=h.zv)
    return h2.at(xnew)


@pytest.mark.parametrize("q", [1.0, -1.0])
@pytest.mark.parametrize("d", [0.349066, -0.349066, 0.05])
def test_rotation_then_step_follows_the_exact_helix(q, d):
    rng = np.random.default_rng(int(1000 * abs(d)) + (q > 0))
    for _ in range(5):
        x0 = rng.uniform(100, 230)
        st = np.zeros(20)
        st[:5] = [rng.uniform(-0.15, 0.15) * x0, rng.uniform(-100, 100), rng.uniform(-0.5, 0.5),
                  rng.uniform(-1, 1), q * rng.uniform(0.2, 3.0)]
        A = rng.normal(size=(5, 5)) * np.array([0.1, 0.1, 0.01, 0.01, 0.05])
        C = A @ A.T + np.diag([1e-3, 1e-3, 1e-6, 1e-6, 1e-4])
        st[5:] = C[np.tril_indices(5)]
        ok, rs, xr = oracle.rotate(st, x0, d)
        assert ok
        xnew = xr + 2.0
        ok, got = oracle.propagate(rs, xr, xnew)
        assert ok
        ex = _exact_new_state(st, x0, 0.0, d, xnew)
        assert np.allclose(got[:5], ex, rtol=1e-10, atol=1e-10), (got[:5], ex)
        # covariance: J C J^T with the numeric Jacobian of the exact map
        J = np.zeros((5, 5))
        for k in range(5):
            hk = [1e-4, 1e-4, 1e-5, 1e-5, 1e-5][k]
            sp_, sm_ = st.copy(), st.copy()
            sp_[k] += hk
            sm_[k] -= hk
            J[:, k] = (_exact_new_state(sp_, x0, 0.0, d, xnew) - _exact_new_state(sm_, x0, 0.0, d, xnew)) / (2 * hk)
        Cn = J @ C @ J.T
        Cg = np.zeros((5, 5))
        Cg[np.tril_indices(5)] = got[5:]
        Cg = Cg + np.tril(Cg, -1).T
        scale = np.sqrt(np.outer(np.diag(Cn), np.diag(Cn)))
        assert np.abs(Cg - Cn).max() / scale.max() < 1e-6, np.abs(Cg - Cn) / scale


def test_rotation_refuses_a_track_moving_inward_in_the_new_frame():
    st = np.zeros(20)
    st[:5] = [10.0, 0.0, 0.9, 0.1, 1.0]
    st[5:] = np.eye(5)[np.tril_indices(5)]
    ok, _, _ = oracle.rotate(st, 150.0, -1.6)
    assert not ok


def test_binary32_rotation_agrees_with_fp64():
    st = np.zeros(20)
    st[:5] = [12.3, -40.0, 0.31, 0.7, -1.3]
    st[5:] = (np.eye(5) * [0.01, 0.02, 1e-4, 2e-4, 1e-3])[np.tril_indices(5)]
    ok64, s64, x64 = oracle.rotate(st, 180.0, 0.349066, precision=64)
    ok32, s32, x32 = oracle.rotate(st, 180.0, 0.349066, precision=32)
    assert ok64 and ok32
    assert abs(x32 - x64) < 1e-4 and np.allclose(s32[:5], s64[:5], rtol=1e-5, atol=1e-5)
