"""Pin of every term of the reference Z4c right-hand side by manufactured fields.

All 22 variables are generic cubic polynomials (seeded dyadic coefficients):
the fourth-order D1, D2 and mixed D1 D1 are exact on them and the sixth
difference of the Kreiss-Oliger term vanishes, so at every owned point the
reference must reproduce the continuum right-hand sides of Sec. III.A up to
rounding.  The fields are chosen so that no term drops out:

* Theta != 0, so the Theta terms of Khat, At_ij (through Khat + 2 Theta),
  Gt^i (through d(2 Khat + Theta)) and Theta itself are all exercised;
* det gt != 1 and the evolved Gt^i differs from (Gt_d)^i = gt^jk Gt^i_jk,
  so the kappa1 damping of Gt^i and the evolved/computed split of the Ricci
  tensor matter;
* kappa2 != 0, and eta(r) varies across the block (eta_s = 1.25 near r = 1.3),
  so the kappa1 (1 - kappa2), kappa1 (2 + kappa2) factors and the r^4
  exponent of eta are pinned.

The continuum values come from tests/z4c_printed.py: exact SymPy arithmetic on
the printed equations, with the physical Ricci tensor and D_i D_j alpha from
the textbook definitions.  Planted mistakes (a flipped sign, a wrong factor,
a wrong exponent) in copies of the reference source must fail the comparison.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest
import sympy as sp

from oracle import cbuild
from tests import z4c_printed as zp

G = 3
N = 5
H = sp.Rational(1, 8)
CENTRE = (sp.Rational(1), sp.Rational(3, 4), sp.Rational(-1, 2))
KAPPA1, KAPPA2 = sp.Rational(5, 16), sp.Rational(3, 4)
ETA_C, ETA_O, ETA_S = sp.Rational(2), sp.Rational(1, 4), sp.Rational(5, 4)
SIGMA = 0.32
TOL = 1e-12

# owned points (i, j, k) of the 5^3 block compared with the exact values
POINTS = [(0, 0, 0), (4, 4, 4), (2, 2, 2), (4, 0, 2), (1, 3, 0), (0, 4, 3), (3, 1, 4)]


def _monomials():
    return [(a, b, c) for a in range(4) for b in range(4) for c in range(4) if a + b + c <= 3]


def _cubic(rng, scale, const):
    xi = [zp.X[d] - CENTRE[d] for d in range(3)]
    e = sp.Rational(const)
    for (a, b, c) in _monomials():
        coef = sp.Rational(int(rng.integers(-16, 17)), 16) * scale
        e += coef * xi[0] ** a * xi[1] ** b * xi[2] ** c
    return sp.expand(e)


def manufactured_fields(seed=7):
    rng = np.random.default_rng(seed)
    s = sp.Rational
    f = [None] * 22
    f[0] = _cubic(rng, s(1, 10), 1)                                  # W
    for n, (i, j) in enumerate(zp.SYM):                              # gt_ij, det != 1
        f[1 + n] = _cubic(rng, s(1, 10), s(9, 8) if i == j else 0)
    f[7] = _cubic(rng, s(1, 4), s(1, 3))                             # Khat
    for n in range(6):                                               # At_ij (not trace-free)
        f[8 + n] = _cubic(rng, s(1, 5), 0)
    f[14] = _cubic(rng, s(1, 4), s(1, 5))                            # Theta != 0
    for i in range(3):                                               # Gt^i, unrelated to gt
        f[15 + i] = _cubic(rng, s(1, 3), 0)
    f[18] = _cubic(rng, s(1, 10), s(9, 10))                          # alpha
    for i in range(3):                                               # beta^i
        f[19 + i] = _cubic(rng, s(1, 4), 0)
    return f


@pytest.fixture(scope="module")
def exact():
    F = zp.Fields(manufactured_fields())
    out = {}
    for (i, j, k) in POINTS:
        p = tuple(CENTRE[d] + (q - (N - 1) // 2) * H for d, q in enumerate((i, j, k)))
        rhs, extra = zp.evaluate(F, p, KAPPA1, KAPPA2, ETA_C, ETA_O, ETA_S)
        out[(i, j, k)] = ([float(sp.N(v, 30)) for v in rhs], extra)
    return F, out


def _oracle_block(lib, F):
    px = N + 2 * G
    ax = [float(CENTRE[d]) + (np.arange(px) - G - (N - 1) // 2) * float(H) for d in range(3)]
    Z, Y, Xg = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    tot = px ** 3
    Yarr = np.zeros((22, tot))
    for n, e in enumerate(F.f):
        fn = sp.lambdify(zp.X, e, modules="numpy")
        Yarr[n] = np.broadcast_to(np.asarray(fn(Xg, Y, Z), dtype=np.float64), Xg.shape).ravel()
    k = np.zeros((22, tot))
    ric = np.zeros((6, tot))
    ham = np.zeros(tot)
    desc = np.array([[0, N, N, N]], dtype=np.int64)
    origin = np.array([ax[0][G], ax[1][G], ax[2][G]])
    par = np.array([float(KAPPA1), float(KAPPA2), float(ETA_C), float(ETA_O), float(ETA_S), SIGMA])
    lib.orc_z4c_rhs(1, cbuild.ptr(desc), G, tot, cbuild.ptr(Yarr), cbuild.ptr(k), float(H),
                    cbuild.ptr(par), cbuild.ptr(origin), cbuild.ptr(ric), cbuild.ptr(ham))
    sl = (slice(G, G + N),) * 3
    own = lambda a: a.reshape(px, px, px)[sl]
    return [own(k[n]) for n in range(22)], [own(ric[n]) for n in range(6)], own(ham)


def _worst(lib, F, ex):
    """Largest relative deviation per variable, over the compared points."""
    k, _, _ = _oracle_block(lib, F)
    worst = np.zeros(22)
    for (i, j, kk), (vals, _) in ex.items():
        for n in range(22):
            got = k[n][kk, j, i]
            worst[n] = max(worst[n], abs(got - vals[n]) / max(1.0, abs(vals[n])))
    return worst


def test_fields_exercise_every_term(exact):
    F, ex = exact
    for (i, j, k), (vals, extra) in ex.items():
        p = tuple(CENTRE[d] + (q - (N - 1) // 2) * H for d, q in enumerate((i, j, k)))
        at = lambda n: float(zp._at(F.f[n], p))
        assert abs(at(14)) > 0.05                                   # Theta
        gt = sp.Matrix(3, 3, lambda a, b: zp._at(F.f[1 + zp._slot(a, b)], p))
        assert abs(float(gt.det()) - 1.0) > 0.05                    # det gt != 1
        assert max(abs(at(15 + a) - float(extra["Gd"][a])) for a in range(3)) > 0.05
    etas = [float(extra["eta"]) for (_, extra) in ex.values()]
    assert max(etas) - min(etas) > 0.2, etas


def test_ricci_split_equals_textbook_plus_gamma_term(exact):
    # the paper's split with the evolved Gt^i equals the textbook Ricci
    # tensor of gamma_ij = gt_ij / W^2 plus gt_k(i d_j)(Gt^k - Gt_d^k), for a
    # conformal metric with det != 1
    _, ex = exact
    for (_, extra) in ex.values():
        a, b = extra["ricci_textbook_plus_gamma_term"], extra["ricci_split"]
        for i in range(3):
            for j in range(3):
                assert sp.simplify(a[i][j] - b[i][j]) == 0


def test_reference_rhs_equals_exact_printed_equations(exact):
    F, ex = exact
    worst = _worst(cbuild.lib(), F, ex)
    assert np.all(worst <= TOL), dict(enumerate(worst))


def test_reference_ricci_and_constraint_equal_exact(exact):
    F, ex = exact
    _, ric, ham = _oracle_block(cbuild.lib(), F)
    for (i, j, k), (_, extra) in ex.items():
        R = extra["ricci_split"]
        for n, (a, b) in enumerate(zp.SYM):
            ref = float(sp.N(R[a][b], 30))
            assert abs(ric[n][k, j, i] - ref) <= TOL * max(1.0, abs(ref)), (n, ric[n][k, j, i], ref)
        href = float(sp.N(extra["ham"], 30))
        assert abs(ham[k, j, i] - href) <= TOL * max(1.0, abs(href))


# planted mistakes: (pattern in oracle/z4c.c, replacement, variables that must fail)
MUTANTS = [
    ("alp * kappa1 * (1.0 - kappa2) * Th", "alp * kappa1 * (1.0 + kappa2) * Th", [7]),
    ("alp * kappa1 * (1.0 - kappa2) * Th", "alp * kappa1 * (1.0 - kappa2) * Kh", [7]),
    ("2.0 * alp * kappa1 * (Gt[i] - Gd[i]);", "-2.0 * alp * kappa1 * (Gt[i] - Gd[i]);", [15, 16, 17]),
    ("2.0 * alp * kappa1 * (Gt[i] - Gd[i]);", "2.0 * alp * kappa1 * (Gt[i]);", [15, 16, 17]),
    ("alp * kappa1 * (2.0 + kappa2) * Th", "alp * kappa1 * (2.0 - kappa2) * Th", [14]),
    ("const double Kt = Kh + 2.0 * Th;", "const double Kt = Kh + Th;", [0, 7, 8, 14]),
    ("const double Kt = Kh + 2.0 * Th;", "const double Kt = Kh - 2.0 * Th;", [0, 7, 8, 14]),
    ("(2.0 * dKh[j] + dTh[j])", "(2.0 * dKh[j] - dTh[j])", [15, 16, 17]),
    ("(2.0 * dKh[j] + dTh[j])", "(dKh[j] + dTh[j])", [15, 16, 17]),
    ("exp(-(rq * rq) * (rq * rq))", "exp(-(rq * rq))", [19, 20, 21]),
    ("(eta_c - eta_o) * exp", "(eta_c + eta_o) * exp", [19, 20, 21]),
    ("0.75 * Gt[i] - eta * beta[i]", "0.75 * Gd[i] - eta * beta[i]", [19, 20, 21]),
    ("rt += Gd[k] * 0.5 *", "rt += Gt[k] * 0.5 *", [8, 14]),
    ("rt += 0.5 * (gt[k][i] * dGt[j][k]", "rt += 0.5 * (gt[k][j] * dGt[j][k]", [8, 14]),
    ("+ (2.0 / 3.0) * Gd[i] * divb", "+ (2.0 / 3.0) * Gt[i] * divb", [15, 16, 17]),
    ("t7 += Gd[j] * db[j][i];", "t7 += Gt[j] * db[j][i];", [15, 16, 17]),
    ("rhs[VW] = adv[VW] + (1.0 / 3.0) * W * (alp * Kt - divb);",
     "rhs[VW] = adv[VW] + (1.0 / 3.0) * W * (alp * Kt + divb);", [0]),
]


def _build_mutant(tmp_path, idx, pat, rep):
    src = open(os.path.join(os.path.dirname(cbuild.__file__), "z4c.c")).read()
    assert src.count(pat) == 1, pat
    mut = src.replace(pat, rep)
    cpath = tmp_path / f"z4c_mut{idx}.c"
    cpath.write_text(mut)
    so = tmp_path / f"libz4c_mut{idx}.so"
    flags = [f for f in cbuild.CFLAGS if f != "-fopenmp"]
    subprocess.run(["gcc", *flags, "-o", str(so), str(cpath), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    lib.orc_z4c_rhs.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_z4c_rhs.restype = None
    return lib


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_planted_mistake_fails(exact, tmp_path, idx):
    F, ex = exact
    pat, rep, vars_ = MUTANTS[idx]
    lib = _build_mutant(tmp_path, idx, pat, rep)
    worst = _worst(lib, F, ex)
    # the mutant is caught (by a margin far above rounding) on the variables it touches
    assert max(worst[v] for v in vars_) > 1e-4, (pat, rep, dict(enumerate(worst)))


def test_mutant_patterns_match_unique_lines():
    src = open(os.path.join(os.path.dirname(cbuild.__file__), "z4c.c")).read()
    for pat, _, _ in MUTANTS:
        assert len(re.findall(re.escape(pat), src)) == 1, pat
