"""Pins of the reference Z4c right-hand side with eighth-order derivatives and
the r = 8 (ninth-order) Kreiss-Oliger dissipation of Sec. III.C, five ghost
layers (oracle/z4c.c, orc_z4c_rhs8_ko9).

The dissipation is linear and added to every variable's right-hand side after
the rest, so the difference of two calls with sigma and with sigma = 0 is the
dissipation term alone, sigma / (1024 h) sum_d delta_d^10 Y.  Closed forms:

* constants and every polynomial of degree at most 9 per coordinate: zero;
* x^10: delta^10 x^10 = 10! h^10, so the term is sigma 10! h^9 / 1024
  (a wrong tap weight, a wrong normalisation or the r = 4 operator fails);
* a Fourier mode sin(k x): the term is -sigma / (1024 h) (4 sin^2(k h / 2))^5
  sin(k x), negative (dissipative) for every k;
* with sigma = 0 the result equals the fifth-order-dissipation variant's
  (orc_z4c_rhs8) bit for bit: only the dissipation differs.
"""
import math

import numpy as np

from oracle import cbuild

G = 5
PAR = np.array([0.02, 0.0, 2.0, 0.25, 40.0, 0.0])   # kappa1, kappa2, eta_c, eta_o, eta_s, sigma


def _flat(x):
    one, zero = np.ones_like(x), np.zeros_like(x)
    return [one, one, zero, zero, one, zero, one] + [zero] * 11 + [one] + [zero] * 3


def _rhs(fields_fn, n, h, sigma, fn="orc_z4c_rhs8_ko9", centre=(0.3, -0.2, 0.5)):
    px = n + 2 * G
    ax = [centre[d] + (np.arange(px) - G - (n - 1) / 2) * h for d in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    tot = px ** 3
    Yarr = np.zeros((22, tot))
    for i, v in enumerate(fields_fn(X, Y, Z)):
        Yarr[i] = np.broadcast_to(v, X.shape).ravel()
    k = np.zeros((22, tot))
    par = PAR.copy()
    par[5] = sigma
    desc = np.array([[0, n, n, n]], dtype=np.int64)
    origin = np.array([ax[0][G], ax[1][G], ax[2][G]])
    getattr(cbuild.lib(), fn)(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k), h,
                              cbuild.ptr(par), cbuild.ptr(origin), None, None)
    sl = (slice(G, G + n),) * 3
    own = lambda a: a.reshape(px, px, px)[sl]
    return np.array([own(k[i]) for i in range(22)]), (own(X), own(Y), own(Z))


def _dissipation(fields_fn, n, h, sigma):
    a, xyz = _rhs(fields_fn, n, h, sigma)
    b, _ = _rhs(fields_fn, n, h, 0.0)
    return a - b, xyz


def test_flat_space_rhs_is_exactly_zero():
    k, _ = _rhs(lambda x, y, z: _flat(x), 6, 0.1, 0.32)
    assert np.all(k == 0.0)


def test_degree_nine_polynomials_are_not_dissipated():
    # flat background plus a degree-9-per-coordinate perturbation in every variable
    def f(x, y, z):
        p = 1e-3 * (x ** 9 - 0.5 * y ** 7 * z ** 2 + 0.25 * z ** 9 * x ** 3 - y ** 4)
        return [b + (i + 1) * p for i, b in enumerate(_flat(x))]
    d, _ = _dissipation(f, 5, 0.3, 0.32)
    assert np.abs(d).max() < 1e-11, np.abs(d).max()


def test_tenth_power_gives_the_closed_form():
    h, sigma = 0.4, 0.32
    c = 1e-3
    exact = sigma * math.factorial(10) * h ** 9 / 1024.0
    for axis in range(3):
        def f(x, y, z, axis=axis):
            q = (x, y, z)[axis]
            return [b + c * (i + 1) * q ** 10 for i, b in enumerate(_flat(x))]
        d, _ = _dissipation(f, 4, h, sigma)
        for i in range(22):
            np.testing.assert_allclose(d[i], c * (i + 1) * exact, rtol=1e-9, atol=0)


def test_fourier_mode_is_damped_at_the_symbol_rate():
    h, sigma, kw = 0.1, 0.32, 7.0
    def f(x, y, z):
        return [b + 1e-4 * (i + 1) * np.sin(kw * x) for i, b in enumerate(_flat(x))]
    d, (X, _, _) = _dissipation(f, 6, h, sigma)
    sym = -sigma / (1024.0 * h) * (4.0 * math.sin(kw * h / 2.0) ** 2) ** 5
    for i in range(22):
        np.testing.assert_allclose(d[i], sym * 1e-4 * (i + 1) * np.sin(kw * X), rtol=1e-7,
                                   atol=1e-15)
    assert sym < 0.0


def test_without_dissipation_it_is_the_fifth_order_variant():
    def f(x, y, z):
        p = 1e-2 * np.sin(1.3 * x + 0.4) * np.cos(0.7 * y - 0.2 * z)
        return [b + (i % 5 + 1) * p for i, b in enumerate(_flat(x))]
    a, _ = _rhs(f, 6, 0.2, 0.0)
    b, _ = _rhs(f, 6, 0.2, 0.0, fn="orc_z4c_rhs8")
    assert np.array_equal(a, b)
