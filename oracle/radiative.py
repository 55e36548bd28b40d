"""Outgoing (radiative) outer boundary for the Z4c variables (reference).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper applies outgoing boundary conditions to the dynamical variables
(Sec. III.A, through the cited radiative condition).  Near the outer boundary
each variable f is taken to behave as an outgoing spherical wave about its
asymptotic value, f = f0 + u(r - v t) / r, which is equivalent to
    d_t f = -(v / r) (x^i d_i f + (f - f0)),
r the distance from the coordinate origin.  This right-hand side replaces the
evolution equations at the physical-boundary ghost points of level 0, which
are then integrated by the same RK4 stages as the owned points (no
dissipation there).  Derivatives at a ghost point: along a direction in which
the point lies outside the domain, the second-order one-sided difference
pointing inwards, (-3 f_0 + 4 f_1 - f_2) / (2h) (mirrored on the upper side);
along the other directions the centred (f_+1 - f_-1) / (2h).  The sum is
x d_x f + y d_y f + z d_z f, left to right.

Asymptotic values and speeds (readings): f0 = 1 for W, the diagonal of the
conformal metric and the lapse, 0 for everything else; v = sqrt(2) for the
lapse (the 1+log gauge speed far away) and 1 for every other variable.
"""
from __future__ import annotations

import math

import numpy as np

NV = 22
F0 = np.zeros(NV)
F0[[0, 1, 4, 6, 18]] = 1.0          # W, gt_xx, gt_yy, gt_zz, alpha
SPEED = np.ones(NV)
SPEED[18] = math.sqrt(2.0)          # alpha


def radiative_rhs(Ypad: np.ndarray, G: int, n: tuple, h: float, origin, pts: np.ndarray,
                  f0=F0, speed=SPEED) -> np.ndarray:
    """Right-hand side at ghost points.

    Ypad: (nvars, nz + 2G, ny + 2G, nx + 2G), global index i at position i + G;
    n: owned points per dimension (x, y, z); pts: (k, 3) global indices of
    points outside [0, n-1] in at least one dimension.  Returns (nvars, k)."""
    pts = np.asarray(pts, dtype=np.int64)
    P = pts + G
    f = Ypad[:, P[:, 2], P[:, 1], P[:, 0]]
    d = []
    for dim in range(3):
        e = np.zeros(3, dtype=np.int64)
        e[dim] = 1

        def at(off, m):
            Q = P[m] + off * e
            return Ypad[:, Q[:, 2], Q[:, 1], Q[:, 0]]
        lo = pts[:, dim] < 0
        hi = pts[:, dim] > n[dim] - 1
        cen = ~(lo | hi)
        dd = np.empty_like(f)
        dd[:, cen] = (at(1, cen) - at(-1, cen)) / (2.0 * h)
        dd[:, lo] = ((-3.0 * f[:, lo] + 4.0 * at(1, lo)) - at(2, lo)) / (2.0 * h)
        dd[:, hi] = ((3.0 * f[:, hi] - 4.0 * at(-1, hi)) + at(-2, hi)) / (2.0 * h)
        d.append(dd)
    x = np.asarray(origin, dtype=np.float64)[None, :] + pts * h
    r = np.sqrt((x[:, 0] * x[:, 0] + x[:, 1] * x[:, 1]) + x[:, 2] * x[:, 2])
    adv = (x[None, :, 0] * d[0] + x[None, :, 1] * d[1]) + x[None, :, 2] * d[2]
    return -(np.asarray(speed)[:, None] / r[None, :]) * (adv + (f - np.asarray(f0)[:, None]))
