"""Seeded initial data on the canonical point order.

Canonical order of a level: its boxes in the given order, each box z-major,
then y, with x fastest.  It does not depend on how a level is split into
blocks, so the same arrays feed every implementation.

Random draws use SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014); a uniform deviate is the top
53 bits of a draw times 2**-53.
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence, Tuple

import numpy as np

from .geometry import HierarchySpec

_M64 = (1 << 64) - 1


class SplitMix64Stream:
    def __init__(self, seed: int):
        self.state = seed & _M64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * (2.0 ** -53)


def _axes(spec: HierarchySpec, level: int, box):
    lo, hi = box
    dx = spec.dx(level)
    ax = []
    for d in range(3):
        idx = np.arange(lo[d], hi[d] + 1, dtype=np.float64)
        ax.append(spec.origin[d] + idx * dx)
    return ax  # x, y, z coordinate vectors


def canonical_coords(spec: HierarchySpec, level: int):
    """x, y, z of every point of a level in canonical order."""
    xs, ys, zs = [], [], []
    for box in spec.boxes(level):
        x, y, z = _axes(spec, level, box)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        xs.append(X.ravel()); ys.append(Y.ravel()); zs.append(Z.ravel())
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)


def separable_on_spec(spec: HierarchySpec, level: int,
                      factors: Callable[[int, np.ndarray], np.ndarray],
                      terms: int = 1) -> np.ndarray:
    """Sum over t < terms of prod_d factors(t, d, coord_d), canonical order."""
    out = []
    for box in spec.boxes(level):
        x, y, z = _axes(spec, level, box)
        acc = np.zeros((z.size, y.size, x.size))
        for t in range(terms):
            fx = factors(t, 0, x); fy = factors(t, 1, y); fz = factors(t, 2, z)
            acc += fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        out.append(acc.ravel())
    return np.concatenate(out)


# ---------------------------------------------------------------------------
# Field definitions.

def standing_wave(modes=(1, 1, 1), amp: float = 1.0):
    """u = amp * prod_d sin(m_d pi x_d), Pi = 0 (a standing wave on [-1,1]^3)."""
    def fac(t, d, x):
        f = np.sin(modes[d] * math.pi * x)
        return amp * f if d == 0 else f
    return fac


def periodic_gaussian(amp: float, centre: Sequence[float], width: float, period: float = 2.0):
    """amp * exp(-|x-c|^2/w^2) summed over the 27 nearest periodic images.

    The image sum of a Gaussian factorises over dimensions, so the field is
    evaluated as a product of three periodised one-dimensional Gaussians.
    """
    def fac(t, d, x):
        g = np.zeros_like(x)
        for k in (-1, 0, 1):
            g += np.exp(-((x - centre[d] - k * period) ** 2) / (width * width))
        return amp * g if d == 0 else g
    return fac


def pulse_params(seed: int = 2, npulses: int = 8):
    """Amplitudes U(0.1,1), widths U(0.05,0.2), centres at the towers +- U(-0.1,0.1)^3."""
    rng = SplitMix64Stream(seed)
    out = []
    for p in range(npulses):
        A = 0.1 + 0.9 * rng.uniform()
        w = 0.05 + 0.15 * rng.uniform()
        ox = -0.1 + 0.2 * rng.uniform()
        oy = -0.1 + 0.2 * rng.uniform()
        oz = -0.1 + 0.2 * rng.uniform()
        cx = (-0.3 if p % 2 == 0 else 0.3) + ox
        out.append((A, w, (cx, oy, oz)))
    return out


def ensemble_params(nmembers: int, seed: int = 2):
    """Per member: modes m_d in {1,2,3} and amplitude U(0.5,1.5)."""
    rng = SplitMix64Stream(seed)
    out = []
    for _ in range(nmembers):
        m = tuple(1 + rng.next() % 3 for _ in range(3))
        a0 = 0.5 + rng.uniform()
        out.append((m, a0))
    return out


def standing_wave_on_spec(spec: HierarchySpec, level: int, modes=(1, 1, 1), amp=1.0):
    u = separable_on_spec(spec, level, standing_wave(modes, amp))
    return [u, np.zeros_like(u)]


def gaussian_on_spec(spec: HierarchySpec, level: int, amp=1.0, centre=(0.0, 0.0, 0.0),
                     width=0.2):
    u = separable_on_spec(spec, level, periodic_gaussian(amp, centre, width))
    return [u, np.zeros_like(u)]


def pulses_on_spec(spec: HierarchySpec, level: int, seed: int = 2):
    params = pulse_params(seed)
    facs = [periodic_gaussian(A, c, w) for A, w, c in params]
    u = separable_on_spec(spec, level, lambda t, d, x: facs[t](0, d, x), terms=len(facs))
    return [u, np.zeros_like(u)]


def ensemble_on_spec(spec: HierarchySpec, nmembers: int, seed: int = 2):
    """Initial data of each member of a one-level ensemble: list of [u, Pi]."""
    out = []
    for m, a0 in ensemble_params(nmembers, seed):
        out.append(standing_wave_on_spec(spec, 0, m, a0))
    return out


# ---------------------------------------------------------------------------
# Z4c initial data (22 variables in the library's slot order: W, gt_xx,xy,xz,
# yy,yz,zz, Khat, At_xx..zz, Theta, Gt^x,y,z, alpha, beta^x,y,z).

def brill_lindquist(x, y, z, m: float = 0.5, c: float = 3.0):
    """Two Brill-Lindquist punctures of bare mass m at (+-c, 0, 0), time symmetric:
    psi = 1 + m/(2 r+) + m/(2 r-), W = psi^-2, conformally flat, K = 0, zero
    shift, and the initial lapse 1/2 (1 + (1 - m/2r+ - m/2r-)/(1 + m/2r+ + m/2r-)),
    which equals 1/psi."""
    rp = np.sqrt((x - c) ** 2 + y ** 2 + z ** 2)
    rm = np.sqrt((x + c) ** 2 + y ** 2 + z ** 2)
    a = m / (2 * rp) + m / (2 * rm)
    psi = 1.0 + a
    zero = np.zeros_like(x)
    one = np.ones_like(x)
    alpha = 0.5 * (1.0 + (1.0 - a) / (1.0 + a))
    return ([psi ** -2, one, zero.copy(), zero.copy(), one.copy(), zero.copy(), one.copy(),
             zero.copy()] + [zero.copy() for _ in range(6)] + [zero.copy()] +
            [zero.copy() for _ in range(3)] + [alpha] + [zero.copy() for _ in range(3)])


def brill_lindquist_on_spec(spec: HierarchySpec, level: int, m: float = 0.5, c: float = 3.0):
    x, y, z = canonical_coords(spec, level)
    return brill_lindquist(x, y, z, m, c)


# ---------------------------------------------------------------------------
# The paper's scalar-wave test (Sec. IV.A): an outgoing spherical Gaussian.

E1_AMPLITUDE = 1.0
E1_SIGMA = 0.25 / math.sqrt(2.0)


def spherical_gaussian(t: float, x, y, z, A: float = E1_AMPLITUDE, sigma: float = E1_SIGMA):
    """Exact solution u = (f(t-r) - f(t+r))/r, Pi = du/dt of the scalar wave,
    f(v) = A exp(-v^2 / (2 sigma^2)); at r = 0 the limits -2 f'(t) and
    -2 (t f(t))' / sigma^2 are used."""
    r = np.sqrt(x * x + y * y + z * z)
    s2 = sigma * sigma
    f = lambda v: A * np.exp(-v * v / (2.0 * s2))
    small = r < 1e-9
    rs = np.where(small, 1.0, r)
    u = (f(t - rs) - f(t + rs)) / rs
    p = -(f(t - rs) * (t - rs) - f(t + rs) * (t + rs)) / (s2 * rs)
    ft = A * math.exp(-t * t / (2.0 * s2))
    u = np.where(small, 2.0 * t / s2 * ft, u)
    p = np.where(small, 2.0 * ft * (1.0 - t * t / s2) / s2, p)
    return u, p


def spherical_gaussian_on_spec(spec: HierarchySpec, level: int, t: float = 0.0):
    x, y, z = canonical_coords(spec, level)
    return list(spherical_gaussian(t, x, y, z))
