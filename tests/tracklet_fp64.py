"""A second, independent FP64 derivation of one tracklet (test infrastructure).

It follows the track-following steps of arXiv:1811.11481 Section 2 (seed fit
over the CA chain, row-by-row extrapolation with pickup of the best hit, no
multiple hypotheses) and Section 3 (inward pass through the seed with outlier
rejection), with the readings of this project (windows, cuts, covariance
reset, miss counter), but shares no formula with the oracle:

* the helix step is the exact circle in the local frame: sin(phi) moves
  linearly in x (d sin(phi)/dx = curvature), y by the integral of tan(phi),
  z by tan(lambda) times the arc (asin(s2) - asin(s1)) / curvature;
* the covariance is carried by a numeric Jacobian (central differences of
  that step), not an analytic one;
* the update is the textbook matrix form K = C H^T S^-1, C <- C - K H C;
* the seed circle is found from its centre (perpendicular bisectors) and the
  tangent at the first point, not from the chord formulas.

Every decision (window, chi2 cut, best candidate, guards) also records how far
it was from flipping, so that a comparison can skip tracklets that sit on a
knife edge between two correct FP64 evaluations.
"""
from __future__ import annotations

import math

import numpy as np

KB_PER_T = -0.00299792458


class Params:
    def __init__(self, bz=0.5, sigma=0.1, nsig=3.0, chi2_pick=16.0, sinphi_max=0.95, cov_reset=100.0,
                 q_max=20.0, u_max=0.25, c0=(1.0, 1.0, 0.25, 0.25, 400.0), max_miss=8, n_rows=152):
        self.kB = KB_PER_T * bz
        self.v = sigma * sigma
        self.nsig, self.chi2_pick, self.sinphi_max = nsig, chi2_pick, sinphi_max
        self.cov_reset, self.q_max, self.u_max = cov_reset, q_max, u_max
        self.c0 = np.array(c0, float)
        self.max_miss, self.n_rows = max_miss, n_rows
        self.X = np.array([85.0 + i * 162.0 / 151.0 for i in range(n_rows)])


class Margins:
    """Smallest relative distance of any decision from its threshold."""

    def __init__(self):
        self.m = math.inf

    def note(self, value, threshold):
        scale = max(abs(threshold), 1e-12)
        self.m = min(self.m, abs(value - threshold) / scale)


def step(p, x1, x2, P: Params, marg: Margins | None = None):
    """Exact helix step of the state p = (y, z, sin phi, tan lambda, q/pT) from
    the plane x1 to x2; None where the reading's guards stop the step
    (|sin phi| >= SINPHI_MAX, or curvature * chord / 2 beyond U_MAX)."""
    d = increment(p, x1, x2, P, marg)
    return None if d is None else p + d


def increment(p, x1, x2, P: Params, marg: Margins | None = None):
    """Change of the state over the step (see step())."""
    y, z, s1, t, q = p
    dx = x2 - x1
    k = P.kB * q
    s2 = s1 + k * dx
    if marg is not None:
        marg.note(abs(s2), P.sinphi_max)
    if not abs(s2) < P.sinphi_max:
        return None
    c1, c2 = math.sqrt(1.0 - s1 * s1), math.sqrt(1.0 - s2 * s2)
    # y: integral of tan(phi) dx = (cos phi1 - cos phi2) / curvature, written
    # without the cancellation at small curvature
    dy = dx * (s1 + s2) / (c1 + c2)
    chord = math.copysign(math.hypot(dx, dy), dx)
    u = k * chord * 0.5
    if marg is not None:
        marg.note(u * u, P.u_max * P.u_max)
    if not u * u <= P.u_max * P.u_max:
        return None
    # turning angle phi2 - phi1 = asin(sin(phi2 - phi1)), with
    # sin(phi2 - phi1) = s2 c1 - s1 c2 = k dx (c1 + s1 (s1 + s2) / (c1 + c2)); arc = angle / curvature
    a = c1 + s1 * (s1 + s2) / (c1 + c2)
    w = k * dx * a
    arc = dx * a * (math.asin(w) / w if w != 0.0 else 1.0)
    return np.array([dy, t * arc, s2 - s1, 0.0, 0.0])


def jacobian(p, x1, x2, P: Params):
    scale = np.array([1e-4, 1e-4, 1e-6, 1e-6, 1e-6])
    F = np.zeros((5, 5))
    for j in range(5):
        a, b = p.copy(), p.copy()
        a[j] += scale[j]
        b[j] -= scale[j]
        fa, fb = increment(a, x1, x2, P), increment(b, x1, x2, P)
        if fa is None or fb is None:
            return None
        F[:, j] = (fa - fb) / (2 * scale[j])
    return F + np.eye(5)


def propagate(p, C, x1, x2, P, marg):
    q = step(p, x1, x2, P, marg)
    if q is None:
        return None
    F = jacobian(p, x1, x2, P)
    if F is None:
        return None
    return q, F @ C @ F.T


H = np.zeros((2, 5))
H[0, 0] = H[1, 1] = 1.0


def innovation(p, C, m, P):
    S = H @ C @ H.T + P.v * np.eye(2)
    r = np.asarray(m, float) - p[:2]
    Si = np.linalg.inv(S)
    return r, S, Si, float(r @ Si @ r)


def kf_update(p, C, m, P):
    r, S, Si, chi2 = innovation(p, C, m, P)
    K = C @ H.T @ Si
    return p + K @ r, C - K @ H @ C, chi2


def pick(p, C, ys, zs, P, marg):
    """Index of the picked candidate among (ys, zs) or -1."""
    if len(ys) == 0:
        return -1
    S = H @ C @ H.T + P.v * np.eye(2)
    wy, wz = P.nsig * math.sqrt(S[0, 0]), P.nsig * math.sqrt(S[1, 1])
    ry, rz = ys - p[0], zs - p[1]
    Si = np.linalg.inv(S)
    chi2 = Si[0, 0] * ry * ry + 2 * Si[0, 1] * ry * rz + Si[1, 1] * rz * rz
    for i in range(len(ys)):
        marg.note(abs(ry[i]), wy)
        marg.note(abs(rz[i]), wz)
        marg.note(chi2[i], P.chi2_pick)
    ok = (np.abs(ry) <= wy) & (np.abs(rz) <= wz) & (chi2 <= P.chi2_pick)
    if not ok.any():
        return -1
    idx = np.nonzero(ok)[0]
    order = idx[np.argsort(chi2[idx], kind="stable")]
    if len(order) > 1:
        marg.note(chi2[order[1]], chi2[order[0]])
    return int(order[0])


def seed(x, y, z, P):
    """Circle through three (x, y) points; tangent at the first one."""
    (x0, xm, xe), (y0, ym, ye) = x, y
    ax, ay, bx, by = xm - x0, ym - y0, xe - x0, ye - y0
    den = 2.0 * (ax * by - ay * bx)
    d02 = math.hypot(bx, by)
    if den == 0.0:
        kap, s0, arc = 0.0, by / d02, d02
    else:
        # centre relative to the first point from the two bisector equations
        a2, b2 = ax * ax + ay * ay, bx * bx + by * by
        cx = (by * a2 - ay * b2) / den
        cy = (ax * b2 - bx * a2) / den
        R = math.hypot(cx, cy)
        # tangent at the first point: perpendicular to the radius, pointing
        # towards the last point
        tx, ty = cy / R, -cx / R
        if tx * bx + ty * by < 0:
            tx, ty = -tx, -ty
        s0 = ty
        sign = 1.0 if den > 0 else -1.0  # counter-clockwise turn: positive curvature
        kap = sign / R
        half = min(1.0, d02 / (2.0 * R))
        arc = 2.0 * R * math.asin(half)
    t0 = (z[2] - z[0]) / arc
    q0 = kap / P.kB if P.kB != 0 else 0.0
    q0 = max(-P.q_max, min(P.q_max, q0))
    if not abs(s0) < P.sinphi_max:
        return None
    return np.array([y0, z[0], s0, t0, q0]), np.diag(P.c0)


def tracklet(chain_rows, chain_y, chain_z, row_y, row_z, P: Params):
    """One tracklet from its chain (rows consecutive, ascending) and the
    clusters of every row of its instance (row_y[r], row_z[r]: arrays in input
    order). Returns dict(rowpick {row: index within the row}, nhits, state,
    state_row, margin) or None if the seed or the chain fit fails."""
    marg = Margins()
    L = len(chain_rows)
    r0 = chain_rows[0]
    m, e = (L - 1) // 2, L - 1
    X = P.X
    sd = seed((X[r0], X[r0 + m], X[r0 + e]), (chain_y[0], chain_y[m], chain_y[e]),
              (chain_z[0], chain_z[m], chain_z[e]), P)
    if sd is None:
        return None
    p, C = sd
    # chain fit, every chain cluster, no gate
    for i in range(L):
        if i > 0:
            pr = propagate(p, C, X[r0 + i - 1], X[r0 + i], P, marg)
            if pr is None:
                return None
            p, C = pr
        p, C, _ = kf_update(p, C, (chain_y[i], chain_z[i]), P)
    # outward following from the row after the chain
    cur = last = r0 + e
    miss = 0
    r = cur + 1
    while r < P.n_rows and miss < P.max_miss:
        pr = propagate(p, C, X[r - 1], X[r], P, marg)
        if pr is None:
            break
        p, C = pr
        cur = r
        c = pick(p, C, row_y[r], row_z[r], P, marg)
        if c >= 0:
            p, C, _ = kf_update(p, C, (row_y[r][c], row_z[r][c]), P)
            last, miss = r, 0
        else:
            miss += 1
        r += 1
    state, state_row = np.concatenate([p, C[np.tril_indices(5)]]), cur
    # turn: drop correlations, inflate variances; back to the last picked row
    C = np.diag(np.diag(C) * P.cov_reset)
    picks = {}
    for r in range(cur - 1, last - 1, -1):
        pr = propagate(p, C, X[r + 1], X[r], P, marg)
        if pr is None:
            return dict(rowpick={}, nhits=0, state=state, state_row=state_row, margin=marg.m)
        p, C = pr
        cur = r
    miss = 0
    for r in range(last, -1, -1):
        if r != cur:
            pr = propagate(p, C, X[cur], X[r], P, marg)
            if pr is None:
                break
            p, C = pr
            cur = r
        c = pick(p, C, row_y[r], row_z[r], P, marg)
        if c >= 0:
            p, C, _ = kf_update(p, C, (row_y[r][c], row_z[r][c]), P)
            picks[r] = c
            miss = 0
        else:
            miss += 1
            if miss >= P.max_miss:
                break
    return dict(rowpick=picks, nhits=len(picks), state=state, state_row=state_row, margin=marg.m)
