"""Pins of the reference dense-output and ghost-stage weights (Sec. II).

Nothing here re-types the weight formulas: the checks are the continuous
Runge-Kutta order conditions, the theta = 0 / theta = 1 identities, and
brute-force symbolic runs of the fine RK4 that the ghost values stand in for.
"""
import os
from fractions import Fraction as F

import pytest
import sympy as sp

from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dense_output.txt")

# Classical RK4 tableau (textbook): nodes, coupling a_ij, weights.
C = [F(0), F(1, 2), F(1, 2), F(1)]
A = [[], [F(1, 2)], [F(0), F(1, 2)], [F(0), F(0), F(1)]]
THETAS = [F(0), F(1, 7), F(1, 4), F(1, 3), F(1, 2), F(5, 8), F(1)]


def _golden():
    b_rows, y_rows = {}, {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        t = line.split()
        if t[0].startswith("Y"):
            y_rows[int(t[0][1])] = [F(x) for x in t[1:]]
        else:
            b_rows[int(t[0])] = [F(x) for x in t[1:]]
    return b_rows, y_rows


def test_b_matches_paper_print():
    b_rows, _ = _golden()
    for th in THETAS:
        got = dense.b(th)
        for i in range(4):
            c1, c2, c3 = b_rows[i + 1]
            assert got[i] == c1 * th + c2 * th ** 2 + c3 * th ** 3


@pytest.mark.parametrize("th", THETAS)
def test_continuous_order_conditions(th):
    # Order-3 conditions of a continuous RK extension; for RK4 they determine
    # b(theta) uniquely, so a wrong coefficient anywhere fails one of them.
    bb = dense.b(th)
    assert sum(bb) == th
    assert sum(bb[i] * C[i] for i in range(4)) == th ** 2 / 2
    assert sum(bb[i] * C[i] ** 2 for i in range(4)) == th ** 3 / 3
    assert sum(bb[i] * sum(A[i][j] * C[j] for j in range(i)) for i in range(4)) == th ** 3 / 6


def test_theta_endpoints():
    assert dense.b(0) == (0, 0, 0, 0)
    assert dense.b(1) == (F(1, 6), F(1, 3), F(1, 3), F(1, 6))


def test_derivatives_are_derivatives():
    t = sp.Symbol("t")
    b_rows, _ = _golden()
    polys = [c1 * t + c2 * t ** 2 + c3 * t ** 3 for c1, c2, c3 in
             (tuple(sp.Rational(x.numerator, x.denominator) for x in b_rows[i]) for i in
              range(1, 5))]
    for m in range(1, 4):
        for th in THETAS:
            got = dense.db(th, m)
            for i in range(4):
                want = sp.diff(polys[i], t, m).subs(t, sp.Rational(th.numerator, th.denominator))
                assert sp.Rational(got[i].numerator, got[i].denominator) == want


def _sym_rk4(f, y0, h):
    k1 = f(y0)
    k2 = f(y0 + h / 2 * k1)
    k3 = f(y0 + h / 2 * k2)
    k4 = f(y0 + h * k3)
    return k1, k2, k3, k4


def _fine_stages(f, ys, h):
    Y1 = ys
    Y2 = ys + h / 2 * f(Y1)
    Y3 = ys + h / 2 * f(Y2)
    Y4 = ys + h * f(Y3)
    return [Y1, Y2, Y3, Y4]


def _ghost(y0, H, ks, stage, th0):
    w = dense.ghost_weights(stage, th0)
    return y0 + H * sum(sp.Rational(w[i].numerator, w[i].denominator) * ks[i] for i in range(4))


def _rat(x):
    return sp.Rational(x.numerator, x.denominator)


@pytest.mark.parametrize("th0", [F(0), F(1, 2)])
def test_cubic_in_time_exact(th0):
    # y' = f(t) with deg f <= 2: the solution is cubic, the dense output is exact,
    # and every ghost value must equal the fine RK4 stage value exactly.
    t, H, y0, a0, a1, a2 = sp.symbols("t H y0 a0 a1 a2")
    f = lambda tt: a0 + a1 * tt + a2 * tt ** 2
    ks = [f(0), f(H / 2), f(H / 2), f(H)]
    ys = y0 + H * sum(_rat(dense.b(th0)[i]) * ks[i] for i in range(4))
    exact_ys = y0 + sp.integrate(f(t), (t, 0, _rat(th0) * H))
    assert sp.simplify(ys - exact_ys) == 0
    h = H / 2
    t0 = _rat(th0) * H
    Y1 = ys
    Y2 = ys + h / 2 * f(t0)
    Y3 = ys + h / 2 * f(t0 + h / 2)
    Y4 = ys + h * f(t0 + h / 2)
    for s, Y in zip((1, 2, 3, 4), (Y1, Y2, Y3, Y4)):
        assert sp.expand(_ghost(y0, H, ks, s, th0) - Y) == 0
    end = y0 + sp.integrate(f(t), (t, 0, t0 + h))
    assert sp.expand(_ghost(y0, H, ks, 5, th0) - end) == 0


def _fine_trajectory_stages(f, y0, H, th0):
    """Stage vectors of the fine level's own RK4 substep starting at theta0.

    The fine level starts from y_n and takes RK4 steps of h = H/2; its second
    substep starts from the result of the first.  Returns (stages, end)."""
    h = H / 2
    ys = y0
    if th0 == F(1, 2):
        k = _sym_rk4(f, y0, h)
        ys = y0 + h / 6 * (k[0] + 2 * k[1] + 2 * k[2] + k[3])
    st = _fine_stages(f, ys, h)
    k = _sym_rk4(f, ys, h)
    return st, ys + h / 6 * (k[0] + 2 * k[1] + 2 * k[2] + k[3])


# Leading ghost-minus-fine-stage errors on y' = lambda y, z = lambda H, in units
# of y_n (a symbolic brute-force run of the fine level's own RK4 substeps).
LINEAR_LEADING = {
    (0, 1): (4, 0), (0, 2): (4, 0), (0, 3): (4, sp.Rational(-1, 128)),
    (0, 4): (4, sp.Rational(-1, 64)), (0, 5): (4, sp.Rational(-5, 384)),
    (F(1, 2), 1): (4, sp.Rational(-5, 384)), (F(1, 2), 2): (4, sp.Rational(-7, 384)),
    (F(1, 2), 3): (4, sp.Rational(-1, 384)), (F(1, 2), 4): (4, sp.Rational(-1, 128)),
    (F(1, 2), 5): (5, sp.Rational(-1, 128)),
}


@pytest.mark.parametrize("th0", [F(0), F(1, 2)])
def test_linear_problem_leading_error(th0):
    z = sp.Symbol("z")
    one = sp.Integer(1)
    f = lambda y: z * y            # lambda = z with H = 1
    ks = _sym_rk4(f, one, one)
    stages, end = _fine_trajectory_stages(f, one, one, th0)
    for s in range(1, 6):
        ref = stages[s - 1] if s < 5 else end
        diff = sp.expand(_ghost(one, one, ks, s, th0) - ref)
        poly = sp.Poly(diff, z)
        p0, lead = LINEAR_LEADING[(th0, s)]
        for p in range(p0):
            assert poly.coeff_monomial(z ** p) == 0, (s, p)
        assert poly.coeff_monomial(z ** p0) == lead, (s, diff)


class _Series:
    """Exact power series in H truncated after H^6 (coefficients are Fractions)."""
    N = 7

    def __init__(self, c):
        c = [F(x) for x in c][: self.N]
        self.c = c + [F(0)] * (self.N - len(c))

    def __add__(self, o):
        o = o if isinstance(o, _Series) else _Series([o])
        return _Series([a + b for a, b in zip(self.c, o.c)])

    __radd__ = __add__

    def __sub__(self, o):
        o = o if isinstance(o, _Series) else _Series([o])
        return _Series([a - b for a, b in zip(self.c, o.c)])

    def __mul__(self, o):
        if not isinstance(o, _Series):
            return _Series([a * F(o) for a in self.c])
        out = [F(0)] * self.N
        for i, a in enumerate(self.c):
            if a:
                for j in range(self.N - i):
                    out[i + j] += a * o.c[j]
        return _Series(out)

    __rmul__ = __mul__

    def low(self):
        return next((i for i, a in enumerate(self.c) if a), 99)


@pytest.mark.parametrize("th0", [F(0), F(1, 2)])
def test_nonlinear_problem_fourth_order(th0):
    # y' = y^2 exercises f_y y'' (k3 != k2) and f_yy: every ghost value must agree
    # with the fine level's own RK4 stage value to O(H^4); a wrong Taylor
    # coefficient, sign or step (H for h) leaves an O(H^2) or O(H^3) term.
    Hs = _Series([0, 1])
    one = _Series([1])
    f = lambda y: y * y

    def rk4(y0, h):
        k1 = f(y0)
        k2 = f(y0 + h * F(1, 2) * k1)
        k3 = f(y0 + h * F(1, 2) * k2)
        k4 = f(y0 + h * k3)
        return [k1, k2, k3, k4]

    def step(y0, h):
        k = rk4(y0, h)
        return y0 + h * F(1, 6) * (k[0] + 2 * k[1] + 2 * k[2] + k[3])

    def stages(ys, h):
        Y1 = ys
        Y2 = ys + h * F(1, 2) * f(Y1)
        Y3 = ys + h * F(1, 2) * f(Y2)
        Y4 = ys + h * f(Y3)
        return [Y1, Y2, Y3, Y4]

    ks = rk4(one, Hs)
    h = Hs * F(1, 2)
    ys = one if th0 == 0 else step(one, h)
    ref = stages(ys, h) + [step(ys, h)]
    lows = {}
    for s in range(1, 6):
        w = dense.ghost_weights(s, th0)
        ghost = one + Hs * (w[0] * ks[0] + w[1] * ks[1] + w[2] * ks[2] + w[3] * ks[3])
        lows[s] = (ghost - ref[s - 1]).low()
    for s in range(1, 6):
        assert lows[s] >= 4, (s, lows)


def test_taylor_forms_match_paper_print():
    # The ghost weights at theta0 = 0 follow from the printed Taylor forms:
    # y = y_n, y' = k1, y'' = (-3k1+2k2+2k3-k4)/H, y''' = 4(k1-k2-k3+k4)/H^2
    # (derivatives of b at 0), f_y y'' = 4(k3-k2)/H^2, h = H/2.
    _, rows = _golden()
    yd = [(1, 0, 0, 0), (-3, 2, 2, -1), (4, -4, -4, 4)]
    fyy = (0, -4, 4, 0)
    for s in range(1, 5):
        a1, a2, a3, af = rows[s]
        want = tuple(a1 * F(1, 2) * yd[0][i] + a2 * F(1, 4) * yd[1][i] + a3 * F(1, 8) * yd[2][i]
                     + af * F(1, 8) * fyy[i] for i in range(4))
        assert dense.ghost_weights(s, 0) == want


def test_second_substep_start_is_first_substep_end():
    assert dense.ghost_weights(1, F(1, 2)) == dense.ghost_weights(5, 0)
    assert dense.ghost_weights(5, F(1, 2)) == dense.b(1)


def test_f64_conversion():
    for th in (0, F(1, 2)):
        for s in range(1, 6):
            w = dense.ghost_weights(s, th)
            wf = dense.ghost_weights_f64(s, th)
            for a, b in zip(w, wf):
                assert b == float(a)


def test_aligned_weights_are_the_rk4_stages_on_a_linear_problem():
    """Uniform time steps: on y' = z y (H = 1, y_n = 1) the weights must give
    the classical RK4 stage vectors Y_s = 1 + c_s z Y_{s-1}, and stage 5 the
    RK4 amplification 1 + z + z^2/2 + z^3/6 + z^4/24, for any z."""
    from oracle.dense import aligned_weights
    for z in (F(1, 3), F(-2, 7), F(5, 2)):
        # brute force: the four stage slopes of RK4 on y' = z y
        Y = [F(1)]
        k = [z * Y[0]]
        for c in (F(1, 2), F(1, 2), F(1)):
            Y.append(1 + c * k[-1])
            k.append(z * Y[-1])
        for s in range(1, 5):
            w = aligned_weights(s)
            assert 1 + sum(wi * ki for wi, ki in zip(w, k)) == Y[s - 1]
        w = aligned_weights(5)
        assert 1 + sum(wi * ki for wi, ki in zip(w, k)) == 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
