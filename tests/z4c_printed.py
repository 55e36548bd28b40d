"""Exact evaluation of the printed Z4c equations at a point (test helper).

Sec. III.A gives the right-hand sides of W, gt_ij, Khat, At_ij, Gt^i, Theta
and the puncture gauge (lapse and shift equations, eta(r)).  This module
evaluates them in exact rational arithmetic (SymPy) for fields given as
SymPy expressions in x, y, z, at a point with rational coordinates, without
any finite differencing: every derivative is the exact symbolic one.

It is written from the equations and the standard geometric definitions,
independently of the reference C code:

* the physical metric is gamma_ij = gt_ij / W^2 (from W = gamma^(-1/6) and
  gt_ij = W^2 gamma_ij); its Christoffel symbols and Ricci tensor are the
  textbook ones, R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kl G^l_ij - G^k_jl G^l_ik,
  computed from exact first and second derivatives of gamma_ij;
* D_i D_j alpha uses the physical Christoffel symbols directly;
* the Ricci split of the paper, R^W_ij + Rt_ij with the evolved Gt^i in
  gt_k(i d_j) Gt^k and the computed (Gt_d)^k elsewhere, equals the textbook
  Ricci tensor plus gt_k(i d_j) (Gt^k - Gt_d^k); both forms are evaluated and
  returned so a test can check one against the other.

Slot order of the 22 variables: W, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz,
Khat, At_xx..At_zz, Theta, Gt^x, Gt^y, Gt^z, alpha, beta^x, beta^y, beta^z.
"""
from __future__ import annotations

import sympy as sp

X = sp.symbols("x y z", real=True)
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
R3 = range(3)


def _slot(i, j):
    return SYM.index((min(i, j), max(i, j)))


class Fields:
    """Symbolic fields with their first and second derivatives precomputed."""

    def __init__(self, exprs):
        assert len(exprs) == 22
        self.f = [sp.sympify(e) for e in exprs]
        self.d = [[sp.diff(e, X[k]) for k in R3] for e in self.f]
        self.dd = [[[sp.diff(e, X[k], X[l]) for l in R3] for k in R3] for e in self.f]
        W = self.f[0]
        # physical metric and its exact derivatives (rational functions)
        self.gam = [[self.f[1 + _slot(i, j)] / W ** 2 for j in R3] for i in R3]
        self.dgam = [[[sp.diff(self.gam[i][j], X[k]) for k in R3] for j in R3] for i in R3]
        self.ddgam = [[[[sp.diff(self.gam[i][j], X[k], X[l]) for l in R3] for k in R3]
                       for j in R3] for i in R3]


def _at(e, p):
    return e.xreplace({X[0]: p[0], X[1]: p[1], X[2]: p[2]})


def _inv(m):
    return [[v for v in row] for row in (sp.Matrix(m).inv().tolist())]


def evaluate(F: Fields, p, kappa1, kappa2, eta_c, eta_o, eta_s):
    """Exact right-hand sides (22 values) and diagnostics at point p.

    Returns (rhs, extra) with extra holding the Ricci tensor in both forms,
    the Hamiltonian constraint R + 2/3 (Khat + 2 Theta)^2 - At_ij At^ij."""
    p = [sp.Rational(c) for c in p]
    v = [_at(e, p) for e in F.f]
    d = [[_at(e, p) for e in row] for row in F.d]
    dd = [[[_at(e, p) for e in r2] for r2 in r1] for r1 in F.dd]
    W, Kh, Th, alp = v[0], v[7], v[14], v[18]
    gt = [[v[1 + _slot(i, j)] for j in R3] for i in R3]
    At = [[v[8 + _slot(i, j)] for j in R3] for i in R3]
    Gt = [v[15 + i] for i in R3]
    beta = [v[19 + i] for i in R3]
    dW = d[0]
    dgt = [[[d[1 + _slot(i, j)][k] for k in R3] for j in R3] for i in R3]      # d_k gt_ij
    ddgt = [[[[dd[1 + _slot(i, j)][k][l] for l in R3] for k in R3] for j in R3] for i in R3]
    dGt = [[d[15 + i][j] for j in R3] for i in R3]                             # d_j Gt^i
    da = d[18]
    dda = dd[18]
    db = [[d[19 + i][j] for j in R3] for i in R3]                              # d_j beta^i
    ddb = [[[dd[19 + i][j][k] for k in R3] for j in R3] for i in R3]           # d_j d_k beta^i
    dKh, dTh = d[7], d[14]
    gtu = _inv(gt)

    # ---- physical metric, textbook Christoffels and Ricci tensor ----
    g = [[_at(F.gam[i][j], p) for j in R3] for i in R3]
    dg = [[[_at(F.dgam[i][j][k], p) for k in R3] for j in R3] for i in R3]
    ddg = [[[[_at(F.ddgam[i][j][k][l], p) for l in R3] for k in R3] for j in R3] for i in R3]
    gu = _inv(g)
    Cl = [[[(dg[l][j][i] + dg[l][i][j] - dg[i][j][l]) / 2 for j in R3] for i in R3] for l in R3]
    C = [[[sum(gu[k][l] * Cl[l][i][j] for l in R3) for j in R3] for i in R3] for k in R3]
    dCl = [[[[(ddg[l][j][i][m] + ddg[l][i][j][m] - ddg[i][j][l][m]) / 2 for m in R3]
             for j in R3] for i in R3] for l in R3]                            # d_m Cl_lij
    dgu = [[[-sum(gu[k][a] * dg[a][b][m] * gu[b][l] for a in R3 for b in R3) for m in R3]
            for l in R3] for k in R3]                                          # d_m gu^kl
    dC = [[[[sum(dgu[k][l][m] * Cl[l][i][j] + gu[k][l] * dCl[l][i][j][m] for l in R3)
             for m in R3] for j in R3] for i in R3] for k in R3]               # d_m C^k_ij
    Rtext = [[sum(dC[k][i][j][k] - dC[k][i][k][j] for k in R3) +
              sum(C[k][k][l] * C[l][i][j] - C[k][j][l] * C[l][i][k] for k in R3 for l in R3)
              for j in R3] for i in R3]
    DDa = [[dda[i][j] - sum(C[k][i][j] * da[k] for k in R3) for j in R3] for i in R3]
    lapa = sum(gu[i][j] * DDa[i][j] for i in R3 for j in R3)

    # ---- conformal Christoffels, (Gt_d)^i and its derivative ----
    Ctl = [[[(dgt[l][j][i] + dgt[l][i][j] - dgt[i][j][l]) / 2 for j in R3] for i in R3]
           for l in R3]                                                        # Gt_lij
    Ct = [[[sum(gtu[k][l] * Ctl[l][i][j] for l in R3) for j in R3] for i in R3] for k in R3]
    Gd = [sum(gtu[j][k] * Ct[i][j][k] for j in R3 for k in R3) for i in R3]
    dgtu = [[[-sum(gtu[k][a] * dgt[a][b][m] * gtu[b][l] for a in R3 for b in R3) for m in R3]
             for l in R3] for k in R3]
    dCtl = [[[[(ddgt[l][j][i][m] + ddgt[l][i][j][m] - ddgt[i][j][l][m]) / 2 for m in R3]
              for j in R3] for i in R3] for l in R3]
    dCt = [[[[sum(dgtu[k][l][m] * Ctl[l][i][j] + gtu[k][l] * dCtl[l][i][j][m] for l in R3)
              for m in R3] for j in R3] for i in R3] for k in R3]
    dGd = [[sum(dgtu[j][k][m] * Ct[i][j][k] + gtu[j][k] * dCt[i][j][k][m]
                for j in R3 for k in R3) for m in R3] for i in R3]             # d_m Gd^i
    # textbook + the constraint term that the evolved Gt^i adds
    Rsplit_a = [[Rtext[i][j] + sum((gt[k][i] * (dGt[k][j] - dGd[k][j]) +
                                    gt[k][j] * (dGt[k][i] - dGd[k][i])) / 2 for k in R3)
                 for j in R3] for i in R3]

    # ---- the printed split, term by term ----
    DtDtW = [[dd[0][i][j] - sum(Ct[k][i][j] * dW[k] for k in R3) for j in R3] for i in R3]
    lapWt = sum(gtu[l][m] * DtDtW[l][m] for l in R3 for m in R3)
    dlnW2 = sum(gtu[l][m] * dW[l] * dW[m] for l in R3 for m in R3) / W ** 2
    RW = [[DtDtW[i][j] / W + gt[i][j] * lapWt / W - 2 * gt[i][j] * dlnW2 for j in R3]
          for i in R3]
    Rt = [[-sum(gtu[l][m] * ddgt[i][j][l][m] for l in R3 for m in R3) / 2
           + sum(gt[k][i] * dGt[k][j] + gt[k][j] * dGt[k][i] for k in R3) / 2
           + sum(Gd[k] * (Ctl[i][j][k] + Ctl[j][i][k]) / 2 for k in R3)
           + sum(gtu[l][m] * (Ct[k][l][i] * Ctl[j][k][m] + Ct[k][l][j] * Ctl[i][k][m]
                               + Ct[k][i][m] * Ctl[k][l][j])
                 for l in R3 for m in R3 for k in R3)
           for j in R3] for i in R3]
    Rsplit_b = [[RW[i][j] + Rt[i][j] for j in R3] for i in R3]
    Rs = sum(gu[i][j] * Rsplit_a[i][j] for i in R3 for j in R3)

    # ---- right-hand sides ----
    Ktot = Kh + 2 * Th
    adv = [sum(beta[k] * d[n][k] for k in R3) for n in range(22)]
    divb = sum(db[k][k] for k in R3)
    Atu = [[sum(gtu[i][a] * gtu[j][b] * At[a][b] for a in R3 for b in R3) for j in R3] for i in R3]
    Atmix = [[sum(gtu[k][l] * At[l][i] for l in R3) for i in R3] for k in R3]  # At^k_i
    AtAt = sum(At[i][j] * Atu[i][j] for i in R3 for j in R3)
    rhs = [None] * 22
    rhs[0] = adv[0] + W * (alp * Ktot - divb) / 3
    Xt = [[-DDa[i][j] + alp * Rsplit_a[i][j] for j in R3] for i in R3]
    trX = sum(gtu[k][l] * Xt[k][l] for k in R3 for l in R3)
    for (i, j) in SYM:
        s = _slot(i, j)
        rhs[1 + s] = (adv[1 + s] - 2 * alp * At[i][j]
                      + sum(gt[k][i] * db[k][j] + gt[k][j] * db[k][i] for k in R3)
                      - sp.Rational(2, 3) * gt[i][j] * divb)
        tf = Xt[i][j] - gt[i][j] * trX / 3
        rhs[8 + s] = (adv[8 + s] + W ** 2 * tf
                      + alp * (Ktot * At[i][j] - 2 * sum(Atmix[k][i] * At[k][j] for k in R3))
                      + sum(At[k][i] * db[k][j] + At[k][j] * db[k][i] for k in R3)
                      - sp.Rational(2, 3) * At[i][j] * divb)
    rhs[7] = adv[7] - lapa + alp * (AtAt + Ktot ** 2 / 3) + alp * kappa1 * (1 - kappa2) * Th
    for i in R3:
        rhs[15 + i] = (adv[15 + i] - 2 * sum(Atu[i][j] * da[j] for j in R3)
                       + 2 * alp * (sum(Ct[i][j][k] * Atu[j][k] for j in R3 for k in R3)
                                    - 3 * sum(Atu[i][j] * dW[j] / W for j in R3)
                                    - sum(gtu[i][j] * (2 * dKh[j] + dTh[j]) for j in R3) / 3)
                       + sum(gtu[j][k] * ddb[i][j][k] for j in R3 for k in R3)
                       + sum(gtu[i][j] * ddb[k][j][k] for j in R3 for k in R3) / 3
                       - sum(Gd[j] * db[i][j] for j in R3)
                       + sp.Rational(2, 3) * Gd[i] * divb
                       - 2 * alp * kappa1 * (Gt[i] - Gd[i]))
    rhs[14] = (adv[14] + alp * (Rs - AtAt + sp.Rational(2, 3) * Ktot ** 2) / 2
               - alp * kappa1 * (2 + kappa2) * Th)
    rhs[18] = adv[18] - 2 * alp * Kh
    r = sp.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2)
    eta = (eta_c - eta_o) * sp.exp(-(r / eta_s) ** 4) + eta_o
    for i in R3:
        rhs[19 + i] = adv[19 + i] + sp.Rational(3, 4) * Gt[i] - eta * beta[i]
    ham = Rs + sp.Rational(2, 3) * Ktot ** 2 - AtAt
    extra = {"ricci_textbook_plus_gamma_term": Rsplit_a, "ricci_split": Rsplit_b, "ham": ham,
             "Gd": Gd, "eta": eta}
    return rhs, extra
