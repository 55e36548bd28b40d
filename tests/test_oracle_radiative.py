"""Pins of the reference radiative outer boundary (oracle/radiative.py).

* The ghost-point derivatives (one-sided second order across the boundary,
  centred along it) are exact on quadratics, so the right-hand side equals
  -(v/r) (x.grad f + f - f0) of the polynomial exactly; a cubic breaks it.
* On an outgoing spherical wave f = f0 + g(r - v t)/r the condition is exact
  in the continuum; the discrete right-hand side converges to d_t f at second
  order under refinement.
* Flat space is a fixed point of Z4c with this boundary, bit for bit.
* Locality: one coarse step with the radiative boundary differs from the
  frozen-ghost step only within the four stages' reach of the outer boundary.
"""
import math

import numpy as np
import pytest

from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from oracle.radiative import F0, SPEED, radiative_rhs
from workloads import HierarchySpec, brill_lindquist, brill_lindquist_on_spec, config_z4c_small

G = 3


def _shell(n):
    z, y, x = np.meshgrid(*[np.arange(-G, n[d] + G) for d in (2, 1, 0)], indexing="ij")
    p = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    inside = np.all((p >= 0) & (p < np.array(n)), axis=1)
    return p[~inside]


def _pad(fun, n, h, origin, nv=2):
    z, y, x = np.meshgrid(*[origin[d] + np.arange(-G, n[d] + G) * h for d in (2, 1, 0)],
                          indexing="ij")
    return np.stack([fun(v, x, y, z) for v in range(nv)])


def test_exact_on_quadratics_not_on_cubics():
    n, h, origin = (7, 6, 5), 0.3, (-1.1, -0.7, -0.4)
    pts = _shell(n)
    x = np.asarray(origin)[None, :] + pts * h
    r = np.linalg.norm(x, axis=1)
    f0, v = np.array([1.0, 0.0]), np.array([math.sqrt(2.0), 1.0])
    quad = lambda k, X, Y, Z: (0.5 + k) + 0.3 * X - 0.2 * Y + 0.7 * Z + X * X - 0.5 * Y * Z + 0.25 * Z * Z
    grad = lambda X, Y, Z: (0.3 + 2 * X, -0.2 - 0.5 * Z, 0.7 - 0.5 * Y + 0.5 * Z)
    got = radiative_rhs(_pad(quad, n, h, origin), G, n, h, origin, pts, f0, v)
    gx, gy, gz = grad(x[:, 0], x[:, 1], x[:, 2])
    for k in range(2):
        f = quad(k, x[:, 0], x[:, 1], x[:, 2])
        want = -(v[k] / r) * ((x[:, 0] * gx + x[:, 1] * gy + x[:, 2] * gz) + (f - f0[k]))
        assert np.abs(got[k] - want).max() < 1e-11
    cub = lambda k, X, Y, Z: X ** 3 + Y ** 3 + Z ** 3
    got = radiative_rhs(_pad(cub, n, h, origin), G, n, h, origin, pts, f0, v)
    want = -(v[0] / r) * ((3 * x[:, 0] ** 3 + 3 * x[:, 1] ** 3 + 3 * x[:, 2] ** 3) +
                          (x[:, 0] ** 3 + x[:, 1] ** 3 + x[:, 2] ** 3 - f0[0]))
    assert np.abs(got[0] - want).max() > 1e-3


def test_outgoing_wave_second_order():
    g = lambda s: np.exp(-((s - 6.0) ** 2) / 4.0)
    dg = lambda s: -(s - 6.0) / 2.0 * g(s)
    errs = []
    for m in (16, 32, 64):
        h = 16.0 / m
        n = (m + 1,) * 3
        origin = (-8.0, -8.0 + 0.37 * h, -8.0 + 0.21 * h)
        f0, v = F0[18:19], SPEED[18:19]        # the lapse: f0 = 1, v = sqrt(2)
        fun = lambda k, X, Y, Z: f0[0] + g(np.sqrt(X * X + Y * Y + Z * Z)) / np.sqrt(X * X + Y * Y + Z * Z)
        pts = _shell(n)
        got = radiative_rhs(_pad(fun, n, h, origin, 1), G, n, h, origin, pts, f0, v)
        x = np.asarray(origin)[None, :] + pts * h
        r = np.linalg.norm(x, axis=1)
        want = -v[0] * dg(r) / r          # d_t of f0 + g(r - v t)/r at t = 0
        errs.append(np.abs(got[0] - want).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def _z4c_run(spec, outer_bc, data_fn=brill_lindquist_on_spec, phys_fn=brill_lindquist):
    run = OracleRun(Hierarchy(spec, min_block=8, max_block=16), rhs="z4c", outer_bc=outer_bc)
    for l in range(spec.nlevels):
        for v, f in enumerate(data_fn(spec, l)):
            run.set_data(l, v, f)
        pr = run.phys_coords(l)
        if len(pr):
            run.set_phys(l, np.array(phys_fn(pr[:, 0], pr[:, 1], pr[:, 2])))
    return run


def _flat(x, y, z):
    one, zero = np.ones_like(x), np.zeros_like(x)
    return [one, one, zero, zero, one, zero, one] + [zero] * 11 + [one] + [zero] * 3


def test_flat_space_is_a_fixed_point():
    spec = config_z4c_small()
    run = _z4c_run(spec, "radiative", lambda s, l: _flat(*_coords(s, l)), _flat)
    before = [[run.get(l, v).copy() for v in range(22)] for l in range(spec.nlevels)]
    run.advance(2)
    for l in range(spec.nlevels):
        for v in range(22):
            assert np.array_equal(run.get(l, v), before[l][v])
    assert np.array_equal(run.rad_y, np.array(_flat(*run.rad_pts.T.astype(float)))[:, :])


def _coords(spec, l):
    from workloads import canonical_coords
    return canonical_coords(spec, l)


def test_radiative_boundary_is_local():
    spec = config_z4c_small()
    a = _z4c_run(spec, "frozen")
    b = _z4c_run(spec, "radiative")
    a.advance(1)
    b.advance(1)
    n0 = spec.ncells0[0]
    x, y, z = _coords(spec, 0)
    idx = np.rint((np.stack([x, y, z], axis=1) - np.asarray(spec.origin)) / spec.dx0).astype(int)
    dist = np.minimum(idx, n0 - idx).min(axis=1)        # points from the outer boundary
    near = dist < 4 * G
    for v in (0, 18):
        da = a.get(0, v)
        db = b.get(0, v)
        assert np.array_equal(da[~near], db[~near])
        assert not np.array_equal(da[near], db[near])
    assert np.all(np.isfinite(b.rad_y))
    assert not np.array_equal(b.rad_y, a.st[0].phys_vals[:, b.rad_first])
