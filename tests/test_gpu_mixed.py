"""Mixed precision against the FP64 GPU path, which is itself bitwise equal
to the CPU reference.

The mixed wave path evaluates k1 = f(y_n) in FP64 and, since the wave
right-hand side f is linear, k_s = k1 + f(e_s) for s = 2..4 with the stage
increment e_s = c_s dt k_{s-1} in FP32; slopes are stored in FP32 and the
RK4 combination, dense output, prolongation and restriction stay FP64.

Error model.  Rounding e_s to FP32 perturbs it by at most eps32 c_s dt |Pi|
(e_u = c_s dt k_u with k_u ~ Pi); the fourth-order Laplacian amplifies a
perturbation by at most 16/h^2 (three dimensions, sum of |coefficients| over
12 h^2), and the FP32 stencil sums add at most as much again, so stage s
changes k_Pi by at most 32 eps32 c_s dt max|Pi| / h^2.  RK4 weights these
slopes by dt/6 (2, 2, 1) with c = (1/2, 1/2, 1), so one step changes Pi by at
most 16 (dt/h)^2 eps32 max|Pi| = eps32 max|Pi| (dt = h/4): the injection per
step does not depend on h.  Over N steps this gives the strict bound
N eps32 max|Pi|.  The roundings are independent from step to step and the
dissipation removes the grid-scale part, so the accumulated error grows like
a random walk instead; the tests check the model
    B_Pi = sqrt(N) eps32 max|Pi| / 2,   B_u = t B_Pi
with N the steps of the finest level (restriction carries its error to every
coarser level), t the elapsed time, and u the time integral of Pi's error.
The measured errors sit within about 2-15x (Pi) and 8-40x (u) of it at every
size tested, so an FP32 path that regressed to rounding y_n itself (an
error 1/h times larger) fails it.
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from workloads import config_c2, config_c3, gaussian_on_spec, pulses_on_spec

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


def mixed_bounds(spec, ncoarse, t, pi_max):
    """(B_u, B_Pi) of the error model above."""
    n = ncoarse * (1 << (spec.nlevels - 1))
    b_pi = 0.5 * np.sqrt(n) * EPS32 * pi_max
    return t * b_pi, b_pi


def _run(spec, precision, ncoarse, data_fn, **kw):
    ctx = sc.Context(device="cuda:0", precision=precision)
    ctx.build_spec(spec, **kw)
    ctx.bind()
    for l in range(spec.nlevels):
        for v, f in enumerate(data_fn(spec, l)):
            ctx.set_initial_data(0, l, v, f)
    ctx.advance(ncoarse)
    out = [[ctx.read_back(0, l, v) for v in range(2)] for l in range(spec.nlevels)]
    t = ctx.level_time(0)
    ctx.close()
    return out, t


@pytest.mark.parametrize("spec,ncoarse", [(config_c2(32), 8), (config_c3(64, nlev=4), 2),
                                          (config_c3(64, nlev=4), 8)])
def test_mixed_error_within_bound(spec, ncoarse):
    data = pulses_on_spec if spec.nlevels > 2 else gaussian_on_spec
    a, t = _run(spec, sc.SC_FP64, ncoarse, data)
    b, _ = _run(spec, sc.SC_MIXED, ncoarse, data)
    pi_max = max(np.abs(a[l][1]).max() for l in range(spec.nlevels))
    bounds = mixed_bounds(spec, ncoarse, t, pi_max)
    for l in range(spec.nlevels):
        for v in range(2):
            err = np.abs(a[l][v] - b[l][v]).max()
            print(f"level {l} var {v}: |mixed - fp64| = {err:.3e}, bound {bounds[v]:.3e} "
                  f"(ratio {err / bounds[v]:.3f})")
            assert err <= bounds[v], (l, v, err, bounds[v])
            assert err > 0  # the FP32 path really ran


def test_mixed_keeps_fourth_order():
    fine = {}
    for nc in (16, 32, 64):
        out, _ = _run(config_c2(nc), sc.SC_MIXED, int(round(0.5 / (0.25 * 2.0 / nc))),
                      gaussian_on_spec, max_block=256)
        fine[nc] = out[1][0].reshape((nc + 1,) * 3)
    e1 = fine[16][::2, ::2, ::2] - fine[32][::4, ::4, ::4]
    e2 = fine[32][::4, ::4, ::4] - fine[64][::8, ::8, ::8]
    Q = np.abs(e1).max() / np.abs(e2).max()
    print("mixed self-convergence ratio", Q)
    assert 12.0 < Q < 20.0


def test_mixed_exec_modes_bitwise_equal():
    spec = config_c3(64, nlev=3)
    outs = []
    for mode in (sc.SC_EXEC_BATCHED, sc.SC_EXEC_PER_BLOCK, sc.SC_EXEC_GRAPH):
        ctx = sc.Context(device="cuda:0", precision=sc.SC_MIXED, exec=mode)
        ctx.build_spec(spec)
        ctx.bind()
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        ctx.advance(3)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(2)])
        outs[-1] += [ctx.read_back(0, l, v, sc.SC_ARR_K2) for l in range(3) for v in range(2)]
        ctx.close()
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)
