"""RK4, dense output and fine-stage ghost weights (reference).

TEST INFRASTRUCTURE ONLY (see the package header).

Everything here is exact rational arithmetic on the formulas of Sec. II:

* classical RK4 (Eqs. rk1-rk5): nodes c = (0, 1/2, 1/2, 1), weights
  (1, 2, 2, 1)/6, stage vectors Y2 = y + h/2 k1, Y3 = y + h/2 k2,
  Y4 = y + h k3;
* dense output (Eq. denseoutput1): y(t_n + theta H) = y_n + H sum_i b_i(theta) k_i
  with b_1 = theta - 3/2 theta^2 + 2/3 theta^3, b_2 = b_3 = theta^2 - 2/3 theta^3,
  b_4 = -1/2 theta^2 + 2/3 theta^3;
* time derivatives (Eq. denseoutput2): y^(m) = H^(1-m) sum_i b_i^(m)(theta) k_i;
* Taylor forms of the fine stage vectors (Eqs. Y1-Y4) with the fine step
  h = H/2 and f_y y'' = 4 (k3 - k2) / H^2 built from the coarse slopes.

The fine ghost value of stage s of the fine substep that starts at theta0
(0 for the first substep, 1/2 for the second) is
    y_n + H * (w1 k1 + w2 k2 + w3 k3 + w4 k4)
with (y_n, k_i) the coarse vectors prolonged in space; `ghost_weights`
returns (w1..w4).  Stage 5 ("end") is the dense-output solution at
theta0 + 1/2, used for the ghosts of the state after the substep.

Pinned by tests/test_oracle_dense.py: continuous-RK order conditions,
theta = 0/1 identities, exactness on cubic-in-time solutions against a
brute-force fine RK4 run, and the O(z^4) leading errors on y' = lambda y
against a symbolic fine RK4 run.
"""
from __future__ import annotations

from fractions import Fraction as F

RK4_C = (F(0), F(1, 2), F(1, 2), F(1))
RK4_B = (F(1, 6), F(1, 3), F(1, 3), F(1, 6))
STAGES = ("Y1", "Y2", "Y3", "Y4", "end")


def b(theta):
    """Dense-output weights b_i(theta), i = 1..4."""
    t = F(theta)
    b1 = t - F(3, 2) * t ** 2 + F(2, 3) * t ** 3
    b23 = t ** 2 - F(2, 3) * t ** 3
    b4 = -F(1, 2) * t ** 2 + F(2, 3) * t ** 3
    return (b1, b23, b23, b4)


def db(theta, m):
    """m-th theta-derivative of b_i(theta)."""
    t = F(theta)
    if m == 0:
        return b(t)
    if m == 1:
        return (1 - 3 * t + 2 * t ** 2, 2 * t - 2 * t ** 2, 2 * t - 2 * t ** 2, -t + 2 * t ** 2)
    if m == 2:
        return (-3 + 4 * t, 2 - 4 * t, 2 - 4 * t, -1 + 4 * t)
    if m == 3:
        return (F(4), F(-4), F(-4), F(4))
    return (F(0),) * 4


def ghost_weights(stage: int, theta0):
    """(w1..w4) such that the ghost value is y_n + H * sum_i w_i k_i.

    stage 1..4 are the fine stage vectors Y1..Y4 of the substep starting at
    theta0; stage 5 is the solution at theta0 + 1/2.  All in units of the
    coarse step H, with the fine step h = H/2.
    """
    th = F(theta0)
    if stage == 5:
        return b(th + F(1, 2))
    # coefficients multiplying H*k_i of y, y', y'', y''' (derivative m carries
    # H^(1-m), so H^m y^(m) = H * sum b_i^(m) k_i) and of H^2 f_y y'' = 4(k3-k2)
    y0, y1, y2, y3 = db(th, 0), db(th, 1), db(th, 2), db(th, 3)
    fyy = (F(0), F(-4), F(4), F(0))
    h = F(1, 2)  # fine step in units of H

    def comb(cy1, cy2, cy3, cf):
        # y + cy1 h y' + cy2 h^2 y'' + cy3 h^3 y''' + cf h^3 f_y y''
        return tuple(y0[i] + cy1 * h * y1[i] + cy2 * h ** 2 * y2[i] + cy3 * h ** 3 * y3[i]
                     + cf * h ** 3 * fyy[i] for i in range(4))

    if stage == 1:
        return comb(0, 0, 0, 0)
    if stage == 2:
        return comb(F(1, 2), 0, 0, 0)
    if stage == 3:
        return comb(F(1, 2), F(1, 4), F(1, 16), -F(1, 16))
    if stage == 4:
        return comb(F(1), F(1, 2), F(1, 8), F(1, 8))
    raise ValueError(stage)


def ghost_weights_f64(stage: int, theta0):
    return tuple(float(w.numerator) / float(w.denominator) for w in ghost_weights(stage, theta0))


def aligned_weights(stage: int):
    """Uniform time steps (the comparison runs of Sec. IV.A): parent and child
    take the same step H, so the ghost of fine stage s is the parent's own stage
    vector at the same time, Y_s = y_n + c_s H k_{s-1} (Eqs. rk2-rk4), and the
    ghost after the step is y_{n+1} (Eq. rk5); returned as (w1..w4) of H k_i."""
    w = [F(0)] * 4
    if stage == 5:
        return RK4_B
    if stage >= 2:
        w[stage - 2] = RK4_C[stage - 1]
    return tuple(w)
