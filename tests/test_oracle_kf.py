"""Pins of the oracle's Kalman-filter pieces against closed forms, textbook
linear algebra, a global least-squares fit and Gaussian statistics.

The paper (Sections 2 and 3) fixes a Kalman filter over a helix in a solenoidal
field with a 5-parameter state; every check below uses mathematics that does
not depend on the oracle's own step formulas.
"""
import math

import numpy as np
import pytest
from scipy.optimize import least_squares

import oracle
from helix_truth import LocalHelix, clusters_on_rows, plane_x

RNG_SEED = 12345


def diffuse_params(**kw):
    # a weak initial prior; the per-pass reset keeps its default (x100): a
    # fully diffuse reset would make every pass re-linearise from scratch
    base = dict(c0=[1e6, 1e6, 1e2, 1e2, 1e6])
    base.update(kw)
    return oracle.default_params(**base)


def rows_inside(h, rows, smax=0.85):
    """Rows crossed before |sin phi| reaches smax (looping ends aside)."""
    out = []
    for r in rows:
        v = h.at(plane_x(r))
        if v is None or abs(v[2]) >= smax:
            break
        out.append(r)
    return np.array(out)


# ------------------------------------------------------------ asin(u)/u
def test_asin_over_matches_library():
    for u in np.linspace(-0.25, 0.25, 1001):
        ref = 1.0 if u == 0 else math.asin(u) / u
        assert oracle.asin_over(u, 64) == pytest.approx(ref, rel=1e-15, abs=1e-15)
        # binary32 series: within a few float32 ulps of the exact value
        assert abs(oracle.asin_over(u, 32) - ref) <= 3 * 2.0 ** -23 * ref


# ------------------------------------------------------------ propagation
@pytest.mark.parametrize("q", [1, -1])
@pytest.mark.parametrize("pt", [0.15, 0.3, 1.0, 10.0])
def test_propagation_follows_exact_helix(q, pt):
    # start direction tilted against the bending so the helix stays in the sector
    h = LocalHelix(pt, q, tanl=0.7, phi0=0.3 * q, alpha=0.0)
    rows = list(range(0, 151))
    truth = clusters_on_rows(h, rows)
    n = min(len(truth), 60)
    st = np.zeros(20)
    st[:5] = truth[0]
    st32 = st.copy()
    for i in range(1, n):
        ok, st = oracle.propagate(st, plane_x(i - 1), plane_x(i), 64)
        if not ok:
            break
        ok32, st32 = oracle.propagate(st32, plane_x(i - 1), plane_x(i), 32)
        assert ok32
        # FP64 step is exact to rounding; FP32 accumulates float rounding only
        assert np.allclose(st[:5], truth[i], rtol=1e-11, atol=1e-10)
        assert np.allclose(st32[:5], truth[i], rtol=2e-5, atol=2e-4)
    assert i >= 10


def test_propagation_backward_is_inverse():
    h = LocalHelix(0.4, -1, tanl=-0.3, phi0=-0.1, alpha=0.0)
    st = np.zeros(20)
    st[:5] = h.at(plane_x(40))
    ok, fwd = oracle.propagate(st, plane_x(40), plane_x(41), 64)
    ok2, back = oracle.propagate(fwd, plane_x(41), plane_x(40), 64)
    assert ok and ok2
    assert np.allclose(back[:5], st[:5], rtol=1e-13, atol=1e-12)


def test_propagation_guard():
    st = np.zeros(20)
    st[:5] = [0, 0, 0.949, 0.1, 20.0]
    # q/pT = 20 bends sin(phi) by kB*q*dx ~ -0.032 per row: moving away is fine ...
    ok, _ = oracle.propagate(st, plane_x(10), plane_x(9), 64)
    assert not ok  # ... but going the other way crosses |sin phi| = 0.95


def _jacobian_numeric(st, x1, x2, eps):
    J = np.zeros((5, 5))
    st = np.concatenate([st[:5], np.zeros(15)])
    for j in range(5):
        a, b = st.copy(), st.copy()
        a[j] += eps[j]
        b[j] -= eps[j]
        _, pa = oracle.propagate(a, x1, x2, 64)
        _, pb = oracle.propagate(b, x1, x2, 64)
        J[:, j] = (pa[:5] - pb[:5]) / (2 * eps[j])
    return J


def _unpack(c15):
    C = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            C[i, j] = C[j, i] = c15[k]
            k += 1
    return C


def _pack(C):
    return np.array([C[i, j] for i in range(5) for j in range(i + 1)])


@pytest.mark.parametrize("s", [-0.6, 0.0, 0.35, 0.8])
@pytest.mark.parametrize("q", [-8.0, 0.5, 4.0])
def test_covariance_transport_matches_numeric_jacobian(s, q):
    rng = np.random.default_rng(RNG_SEED)
    A = rng.normal(size=(5, 5))
    C = A @ A.T * 0.01 + np.eye(5) * 1e-3
    st = np.zeros(20)
    st[:5] = [1.0, 20.0, s, 0.8, q]
    st[5:] = _pack(C)
    x1, x2 = plane_x(30), plane_x(31)
    J = _jacobian_numeric(st[:5].copy(), x1, x2, [1e-4, 1e-4, 1e-6, 1e-6, 1e-5])
    ok, out = oracle.propagate(st, x1, x2, 64)
    assert ok
    ref = J @ C @ J.T
    got = _unpack(out[5:])
    # the analytic F is the exact derivative of the step
    scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    assert np.all(np.abs(got - ref) <= 2e-8 * scale + 1e-12)


# ------------------------------------------------------------ update
def test_update_is_textbook_kalman_gain():
    rng = np.random.default_rng(RNG_SEED + 1)
    p = oracle.default_params()
    for _ in range(20):
        A = rng.normal(size=(5, 5))
        C = A @ A.T * 0.05 + np.eye(5) * 0.01
        x = rng.normal(size=5)
        m = x[:2] + rng.normal(size=2) * 0.3
        st = np.concatenate([x, _pack(C)])
        chi2, out = oracle.update(st, m[0], m[1], 64, p)
        H = np.zeros((2, 5))
        H[0, 0] = H[1, 1] = 1
        V = np.diag([p.sigma_y ** 2, p.sigma_z ** 2])
        S = H @ C @ H.T + V
        K = C @ H.T @ np.linalg.inv(S)
        r = m - H @ x
        assert chi2 == pytest.approx(r @ np.linalg.solve(S, r), rel=1e-12)
        assert np.allclose(out[:5], x + K @ r, rtol=1e-12, atol=1e-13)
        assert np.allclose(_unpack(out[5:]), (np.eye(5) - K @ H) @ C, rtol=1e-10, atol=1e-13)


# ------------------------------------------------------------ seeding
@pytest.mark.parametrize("q", [1, -1])
@pytest.mark.parametrize("pt", [0.2, 1.5])
def test_seed_from_three_points_on_a_helix(q, pt):
    h = LocalHelix(pt, q, tanl=0.4, phi0=0.03, alpha=0.0)
    rows = [20, 25, 30]
    pts = clusters_on_rows(h, rows)
    ok, st = oracle.seed([plane_x(20), pts[0][0], pts[0][1], plane_x(25), pts[1][0], plane_x(30), pts[2][0],
                          pts[2][1]], 64)
    assert ok
    assert st[0] == pts[0][0] and st[1] == pts[0][1]
    assert st[2] == pytest.approx(pts[0][2], abs=1e-12)  # sin(phi) at the first point
    assert st[3] == pytest.approx(pts[0][3], rel=1e-10)  # tan(lambda)
    assert st[4] == pytest.approx(pts[0][4], rel=1e-9)  # q/pT from the curvature


# ------------------------------------------------------------ refit
def _refit_on(h, rows, ys, zs, precision=64, params=None, start=None):
    if start is None:
        ok, start = oracle.seed([plane_x(rows[0]), ys[0], zs[0], plane_x(rows[len(rows) // 2]),
                                 ys[len(rows) // 2], plane_x(rows[-1]), ys[-1], zs[-1]], precision, params)
        assert ok
    return oracle.refit(start, rows[0], rows, ys, zs, precision, params)


@pytest.mark.parametrize("q", [1, -1])
@pytest.mark.parametrize("pt", [0.15, 0.5, 3.0, 10.0])
def test_refit_recovers_noiseless_helix(q, pt):
    h = LocalHelix(pt, q, tanl=-0.6, phi0=0.3 * q, alpha=0.0)
    rows = rows_inside(h, np.arange(0, 120))
    truth = clusters_on_rows(h, rows)
    assert len(rows) >= 20
    ok, st, chi2, nacc, row, masks = _refit_on(h, rows, truth[:, 0], truth[:, 1])
    assert ok and nacc == len(rows) and row == rows[0]
    assert np.allclose(st[:5], truth[0], rtol=1e-9, atol=1e-9)
    assert chi2 < 1e-12
    # binary32 with float32 inputs: float rounding only
    t32 = truth.astype(np.float32).astype(np.float64)
    ok, st, chi2, nacc, row, masks = _refit_on(h, rows, t32[:, 0], t32[:, 1], precision=32)
    assert ok and nacc == len(rows)
    assert np.allclose(st[:5], truth[0], rtol=1e-4, atol=2e-4)


def test_refit_b0_equals_weighted_least_squares_lines():
    """At Bz = 0 the helix is a line: y = a + b x and z = c + d x. The three-pass
    filter with a diffuse prior reaches the least-squares solution."""
    p = diffuse_params(bz=0.0)  # prior x100 reset; q/pT unobservable at Bz = 0
    rng = np.random.default_rng(RNG_SEED + 2)
    for _ in range(10):
        phi, tanl = rng.uniform(-0.5, 0.5), rng.uniform(-1, 1)
        h = LocalHelix(1.0, 1, tanl, phi, 0.0, bz=0.0)
        rows = np.arange(5, 150)
        truth = clusters_on_rows(h, rows)
        ys = truth[:, 0] + rng.normal(size=len(rows)) * 0.1
        zs = truth[:, 1] + rng.normal(size=len(rows)) * 0.1
        x = plane_x(rows)
        start = np.zeros(20)
        start[:5] = [ys[0], zs[0], math.sin(phi), tanl, 0.0]
        start[5:] = _pack(np.diag([1e6, 1e6, 1e2, 1e2, 1e6]))
        ok, st, chi2, nacc, row, _ = oracle.refit(start, rows[0], rows, ys, zs, 64, p)
        assert ok and nacc == len(rows)
        X = np.stack([np.ones_like(x), x - x[0]], axis=1)
        ay, ry = np.linalg.lstsq(X, ys, rcond=None)[:2]
        az, rz = np.linalg.lstsq(X, zs, rcond=None)[:2]
        cov = np.linalg.inv(X.T @ X) * 0.01  # least-squares covariance of (a, b)
        slope = ay[1]
        s_ref = slope / math.sqrt(1 + slope * slope)
        t_ref = az[1] * math.sqrt(1 - s_ref * s_ref)
        # agreement to a small fraction of the fit's own statistical error
        sa, sb = math.sqrt(cov[0, 0]), math.sqrt(cov[1, 1])
        assert abs(st[0] - ay[0]) < 0.01 * sa
        assert abs(st[1] - az[0]) < 0.01 * sa
        assert abs(st[2] - s_ref) < 0.01 * sb
        assert abs(st[3] - t_ref) < 0.02 * sb
        chi2_ls = (ry[0] + rz[0]) / 0.01
        assert chi2 == pytest.approx(chi2_ls, rel=2e-4)


def _helix_model_residuals(par, rows, ys, zs, x0):
    """Exact helix through (x0, y0, z0) with (sin phi0, tan lambda, q/pT)."""
    y0, z0, s0, t, qpt = par
    kB = -0.00299792458 * 0.5
    k = kB * qpt
    X = plane_x(rows)
    s = s0 + k * (X - x0)
    if np.any(np.abs(s) >= 1):
        return np.full(2 * len(rows), 1e3)
    c0, c = math.sqrt(1 - s0 * s0), np.sqrt(1 - s * s)
    if abs(k) < 1e-12:
        y = y0 + (X - x0) * s0 / c0
        arc = (X - x0) / c0
    else:
        y = y0 + (c0 - c) / k
        arc = (np.arcsin(s) - math.asin(s0)) / k
    z = z0 + t * arc
    return np.concatenate([(y - ys) / 0.1, (z - zs) / 0.1])


@pytest.mark.parametrize("seed", range(6))
def test_refit_chi2_is_global_least_squares_minimum(seed):
    rng = np.random.default_rng(RNG_SEED + 10 + seed)
    pt = rng.uniform(0.25, 5.0)
    q = rng.choice([-1, 1])
    h = LocalHelix(pt, q, rng.uniform(-0.8, 0.8), 0.25 * q, 0.0)
    rows = rows_inside(h, np.arange(0, 140))
    truth = clusters_on_rows(h, rows)
    ys = truth[:, 0] + rng.normal(size=len(rows)) * 0.1
    zs = truth[:, 1] + rng.normal(size=len(rows)) * 0.1
    p = diffuse_params()
    ok, st, chi2, nacc, row, _ = _refit_on(h, rows, ys, zs, 64, p, start=np.concatenate([truth[0], _pack(
        np.diag([1e6, 1e6, 1e2, 1e2, 1e6]))]))
    assert ok and nacc == len(rows)
    x0 = plane_x(rows[0])
    sol = least_squares(_helix_model_residuals, truth[0], args=(rows, ys, zs, x0), xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, method="lm")
    chi2_min = float(np.sum(sol.fun ** 2))
    # predicted-residual chi2 of the filter == chi2 at the least-squares optimum
    assert chi2 == pytest.approx(chi2_min, rel=1e-3)
    assert np.allclose(st[:5], sol.x, rtol=1e-3, atol=1e-4)


def test_output_covariances_are_spd_and_pulls_are_normal():
    """chi2/ndf ~ 1 and unit pulls over many smeared helices (diffuse prior)."""
    rng = np.random.default_rng(RNG_SEED + 100)
    p = diffuse_params()
    pulls, chi2n = [], []
    for _ in range(800):
        pt = rng.uniform(0.3, 5.0)
        q = rng.choice([-1, 1])
        h = LocalHelix(pt, q, rng.uniform(-0.8, 0.8), 0.2 * q + rng.uniform(-0.05, 0.05), 0.0)
        rows = rows_inside(h, np.arange(0, 150), smax=0.7)
        truth = clusters_on_rows(h, rows)
        ys = truth[:, 0] + rng.normal(size=len(rows)) * 0.1
        zs = truth[:, 1] + rng.normal(size=len(rows)) * 0.1
        # start: truth smeared well inside the prior widths
        c0 = np.array([1.0, 1.0, 1e-2, 1e-2, 1.0])
        start = np.concatenate([truth[0] + rng.normal(size=5) * 0.2 * np.sqrt(c0), _pack(np.diag(c0))])
        ok, st, chi2, nacc, row, _ = oracle.refit(start, rows[0], rows, ys, zs, 64, p)
        assert ok
        C = _unpack(st[5:])
        np.linalg.cholesky(C)  # SPD
        pulls.append((st[:5] - truth[0]) / np.sqrt(np.diag(C)))
        chi2n.append(chi2 / (2 * nacc - 5))
    pulls = np.array(pulls)
    assert abs(np.mean(chi2n) - 1.0) < 0.02
    assert np.all(np.abs(pulls.mean(axis=0)) < 0.12)
    assert np.all(np.abs(pulls.std(axis=0) - 1.0) < 0.08)


def test_outlier_is_rejected_in_refit():
    h = LocalHelix(1.0, 1, 0.2, 0.0, 0.0)
    rows = np.arange(10, 100)
    truth = clusters_on_rows(h, rows)
    ys, zs = truth[:, 0].copy(), truth[:, 1].copy()
    ys[40] += 2.0  # far outside 5 sigma
    ok, st, chi2, nacc, row, masks = _refit_on(h, rows, ys, zs)
    assert ok and nacc == len(rows) - 1
    assert masks[40] & 4 == 0 and np.all(np.delete(masks, 40) & 4)


def test_replay_reproduces_decisions():
    rng = np.random.default_rng(7)
    h = LocalHelix(0.8, -1, 0.1, 0.01, 0.0)
    rows = np.arange(0, 130)
    truth = clusters_on_rows(h, rows)
    ys = truth[:, 0] + rng.normal(size=len(rows)) * 0.1
    zs = truth[:, 1] + rng.normal(size=len(rows)) * 0.1
    ok, st, chi2, nacc, row, masks = _refit_on(h, rows, ys, zs, 64)
    start = oracle.seed([plane_x(rows[0]), ys[0], zs[0], plane_x(rows[65]), ys[65], plane_x(rows[-1]), ys[-1],
                         zs[-1]], 64)[1]
    ok2, st2, chi22, nacc2, _, masks2 = oracle.refit(start, rows[0], rows, ys, zs, 64, replay=masks)
    assert ok2 and np.array_equal(masks, masks2) and np.array_equal(st, st2) and chi2 == chi22


def test_replay_uses_the_binary32_pad_row_planes():
    """The FP64 replay of a binary32 result evaluates the detector the tracker
    was given: pad-row planes at their binary32 positions. A noiseless helix
    sampled on those planes is recovered to FP64 accuracy by the replay, and
    not by the exact-plane FP64 refit, whose planes differ by up to 7.6e-6 cm."""
    h = LocalHelix(2.0, 1, tanl=0.4, phi0=0.2, alpha=0.0)
    rows = np.arange(0, 100)
    xs32 = np.array([float(np.float32(plane_x(r))) for r in rows])
    assert np.abs(xs32 - np.array([plane_x(r) for r in rows])).max() > 1e-6
    truth = np.array([h.at(x) for x in xs32])
    st0 = np.concatenate([truth[0], np.diag([1.0, 1.0, 0.25, 0.25, 400.0])[np.tril_indices(5)]])
    hs = np.array([0, len(rows)])
    masks = np.full(len(rows), 7, np.uint8)
    ok, out, chi2 = oracle.replay_f64(st0[None], [rows[0]], hs, rows, truth[:, 0], truth[:, 1], masks)
    assert ok.all() and chi2[0] < 1e-12
    assert np.allclose(out[0, :5], truth[0], rtol=1e-9, atol=1e-9)
    ok, out, chi2 = oracle.replay_f64(st0[None], [rows[0]], hs, rows, truth[:, 0], truth[:, 1], masks,
                                      planes_f32=False)
    assert ok.all() and chi2[0] > 1e-9
