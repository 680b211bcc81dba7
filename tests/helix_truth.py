"""Closed-form helix truth for pinning the oracle (FP64, independent of it).

A charge q with transverse momentum pT [GeV] in a uniform Bz [T] moves on a
circle of radius R = pT / (0.00299792458 Bz) cm; the Lorentz force q v x B
turns a positive charge clockwise seen from +z (d phi / ds = -q / R). The
crossing with a pad-row plane x_local = X is the circle/line intersection met
first along the direction of motion; z advances by tan(lambda) times the
transverse arc length. Nothing here uses the tracker's step formulas.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 0.00299792458


def plane_x(i):
    return 85.0 + i * 162.0 / 151.0


class LocalHelix:
    """Helix expressed in the frame of a sector with centre angle ``alpha``."""

    def __init__(self, pt, q, tanl, phi0, alpha, bz=0.5, vx=0.0, vy=0.0, vz=0.0):
        self.pt, self.q, self.tanl, self.bz = pt, q, tanl, bz
        ca, sa = math.cos(alpha), math.sin(alpha)
        # vertex and direction in the local frame
        self.xv = vx * ca + vy * sa
        self.yv = -vx * sa + vy * ca
        self.zv = vz
        self.phi = phi0 - alpha
        if bz == 0.0:
            self.R = math.inf
        else:
            self.R = pt / (C_LIGHT * bz)
            self.sigma = -q if bz > 0 else q  # sign of d(phi)/ds
            rho = self.sigma * self.R
            self.xc = self.xv - rho * math.sin(self.phi)
            self.yc = self.yv + rho * math.cos(self.phi)

    def at(self, X):
        """(y, z, sin phi, tan lambda, q/pT) at the first crossing of x = X."""
        if math.isinf(self.R):
            c, s = math.cos(self.phi), math.sin(self.phi)
            t = (X - self.xv) / c
            return np.array([self.yv + t * s, self.zv + self.tanl * t, s, self.tanl, 0.0])
        dx = X - self.xc
        h2 = self.R * self.R - dx * dx
        if h2 < 0:
            return None
        h = math.sqrt(h2)
        best = None
        rho = self.sigma * self.R
        for yy in (self.yc + h, self.yc - h):
            # position angle on the circle: P = C + rho (sin th, -cos th)
            th = math.atan2((X - self.xc) / rho, -(yy - self.yc) / rho)
            tau = ((th - self.phi) * self.sigma) % (2 * math.pi)
            if best is None or tau < best[0]:
                best = (tau, yy, th)
        tau, yy, th = best
        z = self.zv + self.tanl * self.R * tau
        return np.array([yy, z, math.sin(th), self.tanl, self.q / self.pt])


def clusters_on_rows(helix: LocalHelix, rows):
    out = []
    for r in rows:
        v = helix.at(plane_x(r))
        if v is None:
            break
        out.append(v)
    return np.array(out)
