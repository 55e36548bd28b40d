"""Exact vacuum data for pinning the Z4c right-hand side (test helper).

Minkowski space written in a wavy slicing t = T - hs(x): with x = X,
    ds^2 = -dt^2 - 2 d_i hs dt dx^i + (delta_ij - d_i hs d_j hs) dx^i dx^j,
so the 3+1 data are
    gamma_ij = delta_ij - h_i h_j,  beta_i = -h_i,  alpha = 1/sqrt(1 - |dh|^2),
    K_ij = (D_i beta_j + D_j beta_i) / (2 alpha)   (the metric is t-independent),
with h_i = d_i hs.  The spacetime is flat and static in these coordinates, so
with this lapse and shift every non-gauge variable has zero time derivative,
while the shift, lapse, extrinsic curvature and the conformal metric are all
nontrivial.  The Z4c variables follow from their definitions (Sec. III.A):
W = det(gamma)^(-1/6), gt = W^2 gamma, Khat = K (Theta = 0),
At = W^2 (K - gamma K / 3), Gt^i = -d_j gt^ij.

Also: Brill-Lindquist two-puncture data (psi = 1 + m/(2 r+) + m/(2 r-),
W = psi^-2, alpha = 1/psi, all else flat/zero), whose Hamiltonian constraint
vanishes away from the punctures; and the textbook Ricci tensor of a metric,
R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kl G^l_ij - G^k_jl G^l_ik.
"""
from __future__ import annotations

import functools

import numpy as np
import sympy as sp

X = sp.symbols("x y z", real=True)


def _wavy_height(eps=0.15):
    x, y, z = X
    return eps * (sp.sin(1.3 * x + 0.2) * sp.cos(0.9 * y - 0.4) + 0.6 * sp.sin(1.1 * z + 0.7 * x)
                  + 0.3 * sp.cos(0.8 * y + 1.2 * z))


def christoffel(g, ginv):
    n = 3
    return [[[sum(ginv[k, l] * (sp.diff(g[l, i], X[j]) + sp.diff(g[l, j], X[i])
                                - sp.diff(g[i, j], X[l])) / 2 for l in range(n))
              for j in range(n)] for i in range(n)] for k in range(n)]


def ricci(g, ginv):
    G = christoffel(g, ginv)
    R = sp.zeros(3, 3)
    for i in range(3):
        for j in range(3):
            R[i, j] = sum(sp.diff(G[k][i][j], X[k]) - sp.diff(G[k][i][k], X[j]) for k in range(3)) + \
                sum(G[k][k][l] * G[l][i][j] - G[k][j][l] * G[l][i][k]
                    for k in range(3) for l in range(3))
    return R


@functools.lru_cache(maxsize=None)
def wavy_z4c(eps=0.15):
    """22 Z4c fields (sympy expressions, slot order of the library) plus extras."""
    hs = _wavy_height(eps)
    hd = [sp.diff(hs, xi) for xi in X]
    q = sum(a * a for a in hd)
    gam = sp.Matrix(3, 3, lambda i, j: (1 if i == j else 0) - hd[i] * hd[j])
    gamu = sp.Matrix(3, 3, lambda i, j: (1 if i == j else 0) + hd[i] * hd[j] / (1 - q))
    beta_l = [-a for a in hd]
    beta_u = [sum(gamu[i, j] * beta_l[j] for j in range(3)) for i in range(3)]
    alpha = 1 / sp.sqrt(1 - q)
    G = christoffel(gam, gamu)
    Dbeta = [[sp.diff(beta_l[j], X[i]) - sum(G[k][i][j] * beta_l[k] for k in range(3))
              for j in range(3)] for i in range(3)]
    K = sp.Matrix(3, 3, lambda i, j: (Dbeta[i][j] + Dbeta[j][i]) / (2 * alpha))
    trK = sum(gamu[i, j] * K[i, j] for i in range(3) for j in range(3))
    W = (1 - q) ** sp.Rational(-1, 6)          # det(gamma) = 1 - |dh|^2
    gt = W ** 2 * gam
    gtu = gamu / W ** 2
    At = W ** 2 * (K - gam * trK / 3)
    Gt = [-sum(sp.diff(gtu[i, j], X[j]) for j in range(3)) for i in range(3)]
    sym = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    fields = ([W] + [gt[i, j] for i, j in sym] + [trK] + [At[i, j] for i, j in sym] +
              [sp.Integer(0)] + Gt + [alpha] + beta_u)
    return {"fields": fields, "gamma": gam, "gamma_inv": gamu, "trK": trK, "alpha": alpha,
            "beta": beta_u, "Gt": Gt}


def wavy_gauge_rhs(eps=0.15, eta=0.25):
    """Exact d_t alpha and d_t beta^i from the gauge equations on the wavy data."""
    d = wavy_z4c(eps)
    f = d["fields"]
    alpha, Kh, beta, Gt = f[18], f[7], f[19:22], f[15:18]
    adv = lambda u: sum(beta[k] * sp.diff(u, X[k]) for k in range(3))
    dalpha = adv(alpha) - 2 * alpha * Kh
    dbeta = [adv(beta[i]) + sp.Rational(3, 4) * Gt[i] - eta * beta[i] for i in range(3)]
    return [dalpha] + dbeta


def lambdify(exprs):
    fns = [sp.lambdify(X, e, modules="numpy") for e in exprs]

    def ev(x, y, z):
        out = []
        for fn in fns:
            v = fn(x, y, z)
            out.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.broadcast(x, y, z).shape)
                       .copy())
        return out
    return ev


def brill_lindquist(m=0.5, c=3.0):
    x, y, z = X
    rp = sp.sqrt((x - c) ** 2 + y ** 2 + z ** 2)
    rm = sp.sqrt((x + c) ** 2 + y ** 2 + z ** 2)
    psi = 1 + m / (2 * rp) + m / (2 * rm)
    zero = sp.Integer(0)
    one = sp.Integer(1)
    fields = ([psi ** -2, one, zero, zero, one, zero, one, zero] + [zero] * 6 + [zero] +
              [zero] * 3 + [1 / psi] + [zero] * 3)
    return fields
