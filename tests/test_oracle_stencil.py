"""Pins of the reference wave right-hand side and prolongation.

* The fourth-order centred second derivative is exact on polynomials of
  degree <= 5 and not on degree 6; the r = 4 Kreiss-Oliger operator
  (Sec. III.C) annihilates polynomials of degree <= 5.
* On a Fourier mode the discrete operators act by their closed-form symbols:
  Laplacian sum_d (-2cos 2t_d + 32cos t_d - 30)/(12h^2) and dissipation
  -(sigma/h) sum_d sin^6(t_d/2), t_d = m_d pi h.
* Degree-5 Lagrange midpoint prolongation reproduces tensor polynomials of
  degree <= 5 exactly and fails on degree 6.
"""
import math

import numpy as np
import pytest

from oracle import cbuild
from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from workloads import HierarchySpec

G = 3


def _block_rhs(ufun, pfun, n=(7, 6, 5), h=0.1, sigma=0.32, origin=(0.3, -0.2, 0.1)):
    nx, ny, nz = n
    px, py, pz = nx + 2 * G, ny + 2 * G, nz + 2 * G
    x = origin[0] + (np.arange(px) - G) * h
    y = origin[1] + (np.arange(py) - G) * h
    z = origin[2] + (np.arange(pz) - G) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    tot = px * py * pz
    Yarr = np.zeros((2, tot))
    Yarr[0] = ufun(X, Y, Z).ravel()
    Yarr[1] = pfun(X, Y, Z).ravel()
    k = np.zeros((2, tot))
    desc = np.array([[0, nx, ny, nz]], dtype=np.int64)
    cbuild.lib().orc_wave_rhs(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k),
                              h, sigma)
    sl = (slice(G, G + nz), slice(G, G + ny), slice(G, G + nx))
    own = lambda a: a.reshape(pz, py, px)[sl]
    return own(k[0]), own(k[1]), (own(X), own(Y), own(Z)), own(Yarr[0]), own(Yarr[1])


def test_laplacian_exact_degree5_and_ko_annihilates():
    u = lambda x, y, z: x ** 5 - 2 * x ** 3 * y ** 2 + y ** 4 * z + 3 * z ** 5 + x * y * z - 1
    lap = lambda x, y, z: (20 * x ** 3 - 12 * x * y ** 2) + (-4 * x ** 3 + 12 * y ** 2 * z) + \
        60 * z ** 3
    pi = lambda x, y, z: x ** 4 * y - z ** 5 + 2.0
    ku, kp, (X, Y, Z), U, P = _block_rhs(u, pi)
    # KO annihilates degree <= 5, so k_u == Pi and k_Pi == Laplacian(u)
    assert np.allclose(ku, P, rtol=0, atol=1e-10)
    assert np.allclose(kp, lap(X, Y, Z), rtol=0, atol=1e-8)


def test_laplacian_not_exact_degree6():
    u = lambda x, y, z: x ** 6
    ku, kp, (X, Y, Z), U, P = _block_rhs(u, lambda x, y, z: 0 * x, sigma=0.0)
    # D2 x^6 = 30 x^4 - 8 h^4 (exact truncation term of the 4th-order stencil)
    h = 0.1
    assert np.allclose(kp, 30 * X ** 4 - 8 * h ** 4, rtol=0, atol=1e-9)
    assert np.abs(kp - 30 * X ** 4).max() > 1e-5


def test_ko_degree6_value():
    # delta^6 x^6 = 720 h^6, so Q x^6 = sigma/(64h) * 720 h^6 per dimension
    h, sigma = 0.1, 0.32
    ku, kp, *_ = _block_rhs(lambda x, y, z: x ** 6, lambda x, y, z: 0 * x, sigma=sigma)
    assert np.allclose(ku, sigma / (64 * h) * 720 * h ** 6, rtol=1e-9, atol=0)


@pytest.mark.parametrize("m", [(1, 1, 1), (2, 1, 3), (3, 3, 2)])
def test_fourier_symbols(m):
    h, sigma = 2.0 / 32, 0.32
    w = [mi * math.pi for mi in m]
    u = lambda x, y, z: np.sin(w[0] * x) * np.sin(w[1] * y) * np.sin(w[2] * z)
    pi = lambda x, y, z: 0.5 * u(x, y, z)
    ku, kp, _, U, P = _block_rhs(u, pi, n=(9, 8, 7), h=h, sigma=sigma)
    th = [wi * h for wi in w]
    lam = sum((-2 * math.cos(2 * t) + 32 * math.cos(t) - 30) / (12 * h * h) for t in th)
    q = -(sigma / h) * sum(math.sin(t / 2) ** 6 for t in th)
    assert np.allclose(kp, lam * U + q * P, rtol=0, atol=1e-11)
    assert np.allclose(ku, P + q * U, rtol=0, atol=1e-12)


def _two_level(nonperiodic=False):
    # level 0: 24^3 cells on [-1,1]^3, level 1 box [16,32]^3 (fine indices)
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 24, (24,) * 3, (not nonperiodic,) * 3,
                         [[((16, 16, 16), (32, 32, 32))]])
    return spec


@pytest.mark.parametrize("deg,exact", [(5, True), (6, False)])
def test_prolongation_polynomial_exactness(deg, exact):
    spec = _two_level()
    hier = Hierarchy(spec, min_block=4, max_block=9)
    run = OracleRun(hier)
    parent = run.st[0]
    lev0 = hier.levels[0]
    rng = np.random.default_rng(5)
    cx, cy, cz = rng.normal(size=(3, deg + 1))

    def poly(x, y, z):
        px = sum(cx[i] * x ** i for i in range(deg + 1))
        py = sum(cy[i] * y ** i for i in range(deg + 1))
        pz = sum(cz[i] * z ** i for i in range(deg + 1))
        return px * py * pz + 0.3 * x ** deg - 0.7 * y * z ** (deg - 1)

    # write the polynomial into every parent-owned point of y_n
    for lo, hi in lev0.boxes:
        zz, yy, xx = np.meshgrid(*[np.arange(lo[d], hi[d] + 1) for d in (2, 1, 0)],
                                 indexing="ij")
        q = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
        blk, off = lev0.owner(q)
        flat = parent.flat_offset(blk, off)
        xyz = -1.0 + q * spec.dx(0)
        parent.yn[0, flat] = poly(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    P = run.pro[1].apply(parent.yn)
    rb = hier.rb[1]
    xyz = -1.0 + rb * spec.dx(1)
    want = poly(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    err = np.abs(P[0] - want).max() / np.abs(want).max()
    if exact:
        assert err < 1e-13
    else:
        assert err > 1e-9
    # even-index points are copies, bitwise
    even = np.all(rb % 2 == 0, axis=1)
    if even.any():
        blk, off = lev0.owner(rb[even] // 2)
        assert np.array_equal(P[0][even], parent.yn[0, parent.flat_offset(blk, off)])
