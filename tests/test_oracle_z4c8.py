"""Pins of the reference Z4c right-hand side with eighth-order derivatives
(the paper's production stencil, Sec. III.C), four ghost layers.

* Flat space: right-hand side exactly 0.
* Minkowski in a wavy slicing (tests/z4c_exact.py), an exact static vacuum
  solution: the 18 non-gauge right-hand sides and the Hamiltonian constraint
  converge to zero, and the gauge right-hand sides to their exact values, at
  eighth order (error ratio near 2^8 = 256 under halving h; a fourth-order
  weight anywhere would give 16, a wrong weight O(1)).
"""
import numpy as np
import pytest

from oracle import cbuild
from tests import z4c_exact as ze

G = 4
PAR = np.array([0.02, 0.0, 2.0, 0.25, 40.0, 0.0])   # kappa1, kappa2, eta_c, eta_o, eta_s, sigma


def _block(fields_fn, centre, n, h, par=PAR):
    px = n + 2 * G
    ax = [centre[d] + (np.arange(px) - G - (n - 1) / 2) * h for d in range(3)]
    Z, Y, Xg = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    vals = fields_fn(Xg, Y, Z)
    tot = px ** 3
    Yarr = np.zeros((22, tot))
    for i, v in enumerate(vals):
        Yarr[i] = v.ravel()
    k = np.zeros((22, tot))
    ric = np.zeros((6, tot))
    ham = np.zeros(tot)
    desc = np.array([[0, n, n, n]], dtype=np.int64)
    origin = np.array([ax[0][G], ax[1][G], ax[2][G]])
    cbuild.lib().orc_z4c_rhs8(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k), h,
                              cbuild.ptr(np.ascontiguousarray(par)), cbuild.ptr(origin),
                              cbuild.ptr(ric), cbuild.ptr(ham))
    sl = (slice(G, G + n),) * 3
    own = lambda a: a.reshape(px, px, px)[sl]
    return [own(k[i]) for i in range(22)], own(ham), (own(Xg), own(Y), own(Z))


def _ratio(quantity, h=0.16, centre=(0.4, -0.3, 0.2), n=5):
    a = quantity(n, h, centre)
    b = quantity(2 * n - 1, h / 2, centre)[::2, ::2, ::2]
    return np.abs(a).max() / np.abs(b).max()


def test_flat_space_rhs_is_exactly_zero():
    def flat(x, y, z):
        one, zero = np.ones_like(x), np.zeros_like(x)
        return [one, one, zero, zero, one, zero, one] + [zero] * 11 + [one] + [zero] * 3
    par = PAR.copy()
    par[5] = 0.32
    k, ham, _ = _block(flat, (0.3, -0.2, 0.5), 8, 0.1, par)
    assert all(np.all(a == 0.0) for a in k)
    assert np.all(ham == 0.0)


@pytest.fixture(scope="module")
def wavy():
    d = ze.wavy_z4c()
    return ze.lambdify(d["fields"]), ze.lambdify(ze.wavy_gauge_rhs())


@pytest.mark.parametrize("var", range(18))
def test_wavy_slicing_static_variables_eighth_order(wavy, var):
    fields, _ = wavy
    q = _ratio(lambda n, h, c: _block(fields, c, n, h)[0][var])
    assert 150.0 < q < 400.0, (var, q)


def test_wavy_slicing_hamiltonian_eighth_order(wavy):
    fields, _ = wavy
    q = _ratio(lambda n, h, c: _block(fields, c, n, h)[1])
    assert 150.0 < q < 400.0, q


@pytest.mark.parametrize("g", range(4))
def test_wavy_slicing_gauge_rhs_eighth_order(wavy, g):
    fields, gauge = wavy
    par = PAR.copy()
    par[2] = par[3] = 0.25

    def err(n, h, c):
        k, _, (x, y, z) = _block(fields, c, n, h, par)
        return k[18 + g] - gauge(x, y, z)[g]
    q = _ratio(err)
    assert 150.0 < q < 400.0, (g, q)
