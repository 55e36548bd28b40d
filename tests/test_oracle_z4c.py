"""Pins of the reference Z4c right-hand side (Sec. III.A).

* Flat space (W = alpha = 1, gt = delta, everything else zero): RHS exactly 0.
* Minkowski in a wavy slicing (tests/z4c_exact.py): an exact static vacuum
  solution with nontrivial shift, lapse, extrinsic curvature and conformal
  metric; the 18 non-gauge variables have zero time derivative and the
  Hamiltonian constraint vanishes, so the discrete values must converge to
  zero at fourth order; the gauge right-hand sides converge to their exact
  values.  Any dropped term, wrong sign or index leaves an O(1) residual.
* The Ricci tensor of the Ricci split equals the textbook Ricci tensor of the
  physical metric to fourth order.
* Brill-Lindquist data: Hamiltonian constraint converges to zero at fourth
  order away from the punctures.
"""
import numpy as np
import pytest

from oracle import cbuild
from tests import z4c_exact as ze

G = 3
PAR = np.array([0.02, 0.0, 2.0, 0.25, 40.0, 0.0])   # kappa1, kappa2, eta_c, eta_o, eta_s, sigma


def _block(fields_fn, centre, n, h, par=PAR):
    """Evaluate fields on one padded block of n^3 owned points and run the RHS."""
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
    cbuild.lib().orc_z4c_rhs(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k), h,
                             cbuild.ptr(np.ascontiguousarray(par)), cbuild.ptr(origin),
                             cbuild.ptr(ric), cbuild.ptr(ham))
    sl = (slice(G, G + n),) * 3
    own = lambda a: a.reshape(px, px, px)[sl]
    coords = (own(Xg), own(Y), own(Z))
    return ([own(k[i]) for i in range(22)], [own(ric[i]) for i in range(6)], own(ham), coords)


def test_flat_space_rhs_is_exactly_zero():
    def flat(x, y, z):
        one, zero = np.ones_like(x), np.zeros_like(x)
        return [one, one, zero, zero, one, zero, one] + [zero] * 11 + [one] + [zero] * 3
    par = PAR.copy()
    par[5] = 0.32
    k, ric, ham, _ = _block(flat, (0.3, -0.2, 0.5), 8, 0.1, par)
    assert all(np.all(a == 0.0) for a in k)
    assert np.all(ham == 0.0)


def _convergence(quantity, n_coarse=9, h=0.08, centre=(0.4, -0.3, 0.2)):
    """max |quantity| at common points for spacing h and h/2 over the same region."""
    a = quantity(n_coarse, h, centre)
    b = quantity(2 * n_coarse - 1, h / 2, centre)
    b = b[::2, ::2, ::2]
    return np.abs(a).max(), np.abs(b).max()


@pytest.fixture(scope="module")
def wavy():
    d = ze.wavy_z4c()
    return ze.lambdify(d["fields"]), ze.lambdify(ze.wavy_gauge_rhs())


NONGAUGE = list(range(18))


@pytest.mark.parametrize("var", NONGAUGE)
def test_wavy_slicing_static_variables_converge_to_zero(wavy, var):
    fields, _ = wavy
    e1, e2 = _convergence(lambda n, h, c: _block(fields, c, n, h)[0][var])
    if var == 14:      # Theta: its RHS is 1/2 alpha H, also zero in the continuum
        pass
    assert e2 < 1e-4, (var, e1, e2)
    assert 11.0 < e1 / e2 < 22.0, (var, e1, e2)


def test_wavy_slicing_hamiltonian_constraint(wavy):
    fields, _ = wavy
    e1, e2 = _convergence(lambda n, h, c: _block(fields, c, n, h)[2])
    assert 11.0 < e1 / e2 < 22.0, (e1, e2)


@pytest.mark.parametrize("g", range(4))
def test_wavy_slicing_gauge_rhs(wavy, g):
    fields, gauge = wavy
    par = PAR.copy()
    par[2] = par[3] = 0.25      # constant eta = 0.25, matching the exact expression

    def err(n, h, c):
        k, _, _, (x, y, z) = _block(fields, c, n, h, par)
        return k[18 + g] - gauge(x, y, z)[g]
    e1, e2 = _convergence(err)
    assert 11.0 < e1 / e2 < 22.0, (g, e1, e2)


def test_ricci_matches_textbook(wavy):
    fields, _ = wavy
    d = ze.wavy_z4c()
    R = ze.ricci(d["gamma"], d["gamma_inv"])
    sym = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Rf = ze.lambdify([R[i, j] for i, j in sym])
    for c in range(6):
        def err(n, h, cen, c=c):
            _, ric, _, (x, y, z) = _block(fields, cen, n, h)
            return ric[c] - Rf(x, y, z)[c]
        e1, e2 = _convergence(err)
        assert 11.0 < e1 / e2 < 22.0, (c, e1, e2)


def test_brill_lindquist_hamiltonian_constraint():
    bl = ze.lambdify(ze.brill_lindquist())
    e1, e2 = _convergence(lambda n, h, c: _block(bl, c, n, h)[2], h=0.1, centre=(1.2, 0.9, 0.7))
    assert 11.0 < e1 / e2 < 22.0, (e1, e2)


def test_kreiss_oliger_on_every_variable():
    # a single high-frequency bump in one variable at a time: the RHS change
    # between sigma and 0 is sigma/(64h) * (sum of sixth differences)
    h = 0.1
    def flat_bump(var):
        def f(x, y, z):
            one, zero = np.ones_like(x), np.zeros_like(x)
            out = [one, one, zero, zero, one, zero, one] + [zero] * 11 + [one] + [zero] * 3
            out[var] = out[var] + 1e-3 * x ** 6
            return out
        return f
    par = PAR.copy()
    for var in range(22):
        par[5] = 0.32
        k1, *_ = _block(flat_bump(var), (0.1, 0.2, 0.3), 6, h, par)
        par[5] = 0.0
        k0, *_ = _block(flat_bump(var), (0.1, 0.2, 0.3), 6, h, par)
        dq = k1[var] - k0[var]
        assert np.allclose(dq, 0.32 / (64 * h) * 1e-3 * 720 * h ** 6, rtol=1e-6), var
