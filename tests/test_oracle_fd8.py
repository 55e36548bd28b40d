"""Pins of the reference eighth-order wave right-hand side (the production
stencil, Sec. III.C) and of the schedule with four ghost layers.

* The nine-point centred second derivative is exact on polynomials of degree
  <= 9; on x^10 it returns 90 x^8 - 1152 h^8, the textbook truncation term
  -2 (4!)^2 / 10! h^8 f^(10) of the order-8 stencil.  These two facts fix its
  five symmetric weights uniquely.
* The dissipation is the fifth-order operator of the fourth-order scheme.
* Single level: the fully discrete standing wave is the 2x2 matrix power of
  the RK4 stability polynomial at the discrete symbol, to rounding.
* G = 4 hierarchies: a fine level covering the periodic domain equals a
  unigrid fine run bitwise; two levels agree with a unigrid fine run to
  truncation error, shrinking at least at fourth order.
* Ninth-order dissipation (r = 8 in Sec. III.C's Q u, G = 5): zero on
  polynomials of degree <= 9 and sigma/(1024 h) 10! h^10 on x^10 (the tenth
  difference, which fixes its eleven weights); the fully discrete standing
  wave with its symbol -(sigma/h) sum sin^10(m pi h/2); a G = 5 fine level
  covering the periodic domain equals the unigrid fine run bitwise.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import cbuild
from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from workloads import (HierarchySpec, config_c1, config_c2, gaussian_on_spec, single_level,
                       standing_wave_on_spec)

G = 4


def _block_rhs8(ufun, pfun, n=(7, 6, 5), h=0.1, sigma=0.32, origin=(0.3, -0.2, 0.1), ko=5):
    G = 5 if ko == 9 else 4
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
    f = cbuild.lib().orc_wave_rhs8_ko9 if ko == 9 else cbuild.lib().orc_wave_rhs8
    f(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k), h, sigma)
    sl = (slice(G, G + nz), slice(G, G + ny), slice(G, G + nx))
    own = lambda a: a.reshape(pz, py, px)[sl]
    return own(k[0]), own(k[1]), (own(X), own(Y), own(Z)), own(Yarr[0]), own(Yarr[1])


def test_fd8_laplacian_exact_degree9():
    u = lambda x, y, z: x ** 9 - 2 * x ** 7 * y ** 2 + y ** 8 * z + 3 * z ** 9 + x * y * z - 1
    lap = lambda x, y, z: (72 * x ** 7 - 84 * x ** 5 * y ** 2) + \
        (-4 * x ** 7 + 56 * y ** 6 * z) + 216 * z ** 7
    ku, kp, (X, Y, Z), U, P = _block_rhs8(u, lambda x, y, z: 0 * x, sigma=0.0)
    want = lap(X, Y, Z)
    assert np.abs(kp - want).max() <= 1e-9 * np.abs(want).max()


def test_fd8_truncation_term_on_x10():
    h = 0.1
    ku, kp, (X, Y, Z), U, P = _block_rhs8(lambda x, y, z: x ** 10, lambda x, y, z: 0 * x,
                                          h=h, sigma=0.0)
    assert math.isclose(2 * math.factorial(4) ** 2 / math.factorial(10) * math.factorial(10),
                        1152.0)
    assert np.allclose(kp, 90 * X ** 8 - 1152 * h ** 8, rtol=0, atol=1e-9)
    assert np.abs(kp - 90 * X ** 8).max() > 1e-6


def test_fd8_dissipation_is_fifth_order():
    h, sigma = 0.1, 0.32
    ku, kp, *_ = _block_rhs8(lambda x, y, z: x ** 6, lambda x, y, z: 0 * x, sigma=sigma)
    assert np.allclose(ku, sigma / (64 * h) * 720 * h ** 6, rtol=1e-9, atol=0)
    ku, kp, (X, Y, Z), U, P = _block_rhs8(lambda x, y, z: x ** 5 - y ** 3 * z ** 2,
                                          lambda x, y, z: 0 * x, sigma=sigma)
    assert np.abs(ku).max() < 1e-11


def test_ko9_dissipation_is_ninth_order():
    h, sigma = 0.1, 0.32
    ku, kp, *_ = _block_rhs8(lambda x, y, z: x ** 10, lambda x, y, z: 0 * x, sigma=sigma, ko=9)
    assert np.allclose(ku, sigma / (1024 * h) * math.factorial(10) * h ** 10, rtol=1e-8, atol=0)
    ku, kp, *_ = _block_rhs8(lambda x, y, z: y ** 10, lambda x, y, z: 0 * x, sigma=sigma, ko=9)
    assert np.allclose(ku, sigma / (1024 * h) * math.factorial(10) * h ** 10, rtol=1e-8, atol=0)
    ku, kp, (X, Y, Z), U, P = _block_rhs8(lambda x, y, z: x ** 9 - y ** 7 * z ** 2 + z ** 6,
                                          lambda x, y, z: 0 * x, sigma=sigma, ko=9)
    assert np.abs(ku).max() < 1e-10
    # the fifth-order operator is not zero on degree 6: the two are different
    ku5, *_ = _block_rhs8(lambda x, y, z: z ** 6, lambda x, y, z: 0 * x, sigma=sigma)
    ku9, *_ = _block_rhs8(lambda x, y, z: z ** 6, lambda x, y, z: 0 * x, sigma=sigma, ko=9)
    assert np.allclose(ku5, sigma / (64 * h) * 720 * h ** 6, rtol=1e-9, atol=0)
    assert np.abs(ku9).max() < 1e-10
    # same Laplacian as the fifth-order variant (the dissipation only acts on k_u
    # through Q u and on k_Pi through Q Pi)
    g = lambda x, y, z: np.sin(x + 2 * y) * np.cos(z)
    _, kp5, *_ = _block_rhs8(g, lambda x, y, z: 0 * x, sigma=0.0)
    _, kp9, *_ = _block_rhs8(g, lambda x, y, z: 0 * x, sigma=0.0, ko=9)
    assert np.array_equal(kp5, kp9)


def _discrete_amplitude8(n, m, sigma, nsteps, cfl=0.25, L=2.0, ko=5):
    mp.mp.dps = 40
    h = mp.mpf(L) / n
    dt = cfl * h
    lam = 0
    for mi in m:
        t = mi * mp.pi * h
        lam += (2 * (8064 * mp.cos(t) - 1008 * mp.cos(2 * t) + 128 * mp.cos(3 * t)
                     - 9 * mp.cos(4 * t)) - 14350) / (5040 * h * h)
    # symbol of sigma/2^(r+2) h^(r+1) (D+ D-)^(r/2+1) on a mode: -(sigma/h) sin^(r+2)
    q = -(mp.mpf(sigma) / h) * sum(mp.sin(mi * mp.pi * h / 2) ** (ko + 1) for mi in m)
    A = mp.matrix([[q, 1], [lam, q]]) * dt
    M = mp.eye(2)
    term = mp.eye(2)
    for j in range(1, 5):
        term = term * A / j
        M = M + term
    v = mp.matrix([1, 0])
    for _ in range(nsteps):
        v = M * v
    return float(v[0]), float(v[1])


@pytest.mark.parametrize("m", [(1, 1, 1), (3, 2, 4)])
def test_fd8_fully_discrete_closed_form(m):
    n, nsteps, sigma = 24, 48, 0.32
    spec = config_c1(n)
    run = OracleRun(Hierarchy(spec, min_block=12, max_block=24, G=4), sigma=sigma, fd_order=8)
    u, p = standing_wave_on_spec(spec, 0, m, 1.0)
    run.set_data(0, 0, u)
    run.set_data(0, 1, p)
    run.advance(nsteps)
    au, ap = _discrete_amplitude8(n, m, sigma, nsteps)
    scale = np.abs(u).max()
    assert np.abs(run.get(0, 0) - au * u).max() / scale < 1e-13
    assert np.abs(run.get(0, 1) - ap * u).max() / (scale * max(1.0, abs(ap))) < 1e-13


@pytest.mark.parametrize("m", [(1, 1, 1), (3, 2, 4)])
def test_fd8_ko9_fully_discrete_closed_form(m):
    n, nsteps, sigma = 24, 48, 0.32
    spec = config_c1(n)
    run = OracleRun(Hierarchy(spec, min_block=12, max_block=24, G=5), sigma=sigma, fd_order=8,
                    ko_order=9)
    u, p = standing_wave_on_spec(spec, 0, m, 1.0)
    run.set_data(0, 0, u)
    run.set_data(0, 1, p)
    run.advance(nsteps)
    au, ap = _discrete_amplitude8(n, m, sigma, nsteps, ko=9)
    a5, _ = _discrete_amplitude8(n, m, sigma, nsteps)
    scale = np.abs(u).max()
    assert np.abs(run.get(0, 0) - au * u).max() / scale < 1e-13
    assert np.abs(run.get(0, 1) - ap * u).max() / (scale * max(1.0, abs(ap))) < 1e-13
    if m == (3, 2, 4):   # the mode where the two dissipations differ visibly
        assert abs(au - a5) > 1e-6


def test_ko9_full_cover_equals_single_level_fine():
    n = 12
    spec = HierarchySpec((-1.0,) * 3, 2.0 / n, (n,) * 3, (True,) * 3,
                         [[((0, 0, 0), (2 * n - 1,) * 3)]])
    two = _gauss_run(spec, 3, G=5, ko_order=9, min_block=5, max_block=12)
    one = _gauss_run(single_level(2 * n), 6, G=5, ko_order=9, min_block=6, max_block=12)
    ref = _gauss_run(single_level(2 * n), 6, min_block=6, max_block=12)
    for v in range(2):
        assert np.array_equal(two.get(1, v), one.get(0, v))
        assert not np.array_equal(one.get(0, v), ref.get(0, v))   # the r = 8 dissipation acted


def test_ko9_rejected_where_not_built():
    spec = config_c1(16)
    with pytest.raises(ValueError):
        OracleRun(Hierarchy(spec, G=4), fd_order=8, ko_order=9)
    with pytest.raises(ValueError):
        OracleRun(Hierarchy(spec, G=5), fd_order=4, ko_order=9)


def _gauss_run(spec, nsteps, G=4, ko_order=5, **hk):
    run = OracleRun(Hierarchy(spec, G=G, **hk), sigma=0.32, fd_order=8, ko_order=ko_order)
    for l in range(spec.nlevels):
        u, p = gaussian_on_spec(spec, l)
        run.set_data(l, 0, u)
        run.set_data(l, 1, p)
    run.advance(nsteps)
    return run


def test_fd8_full_cover_equals_single_level_fine():
    n = 12
    spec = HierarchySpec((-1.0,) * 3, 2.0 / n, (n,) * 3, (True,) * 3,
                         [[((0, 0, 0), (2 * n - 1,) * 3)]])
    two = _gauss_run(spec, 3, min_block=4, max_block=12)
    one = _gauss_run(single_level(2 * n), 6, min_block=6, max_block=12)
    for v in range(2):
        assert np.array_equal(two.get(1, v), one.get(0, v))


def test_fd8_two_level_agrees_with_unigrid_fine_to_truncation():
    diffs = []
    for nc in (16, 32):
        ncoarse = nc // 4
        two = _gauss_run(config_c2(nc), ncoarse, max_block=256)
        uni = _gauss_run(single_level(2 * nc), 2 * ncoarse, max_block=256)
        full = uni.get(0, 0).reshape((2 * nc,) * 3)
        s = slice(nc // 2, 3 * nc // 2 + 1)
        d = two.get(1, 0).reshape((nc + 1,) * 3) - full[s, s, s]
        diffs.append(np.abs(d[::2, ::2, ::2]).max() if nc == 16 else np.abs(d[::4, ::4, ::4]).max())
    assert diffs[1] > 0
    assert 8.0 < diffs[0] / diffs[1] < 40.0, diffs   # 14.3 measured: the RK4 and dense-output errors dominate
