"""Mixed precision (FP32-shadow stencil, FP64 state/RK4/dense output/prolongation/
restriction) against the FP64 GPU path, which is itself bitwise equal to the
CPU reference.

Parity is bounded, not exact.  Rounding a stage vector to FP32 perturbs it by
at most eps32 |u| (eps32 = 2^-24); the fourth-order Laplacian amplifies a
perturbation by at most 64/(12 h^2) per dimension (sum of |coefficients| over
12 h^2), i.e. 16 eps32 |u| / h^2 for three dimensions, and the FP32 rounding
of the stencil sums adds at most as much again, so the slope of Pi carries an
error below 32 eps32 max|u| / h^2 per evaluation (the dissipation terms are
O(1/h) and smaller).  RK4 integrates it over time t with weights summing to
one per step, giving the per-level model bound
    |Pi_mixed - Pi_fp64| <= t * 32 eps32 max|u| / h^2
(u picks up at most t times that).  Restriction copies finer-level values
into the coarser levels, so a level's error is bounded by the finest spacing
in the hierarchy, h = dx of the finest level.  The tests check the measured
error against that bound and that fourth-order convergence is kept.
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from workloads import config_c2, config_c3, gaussian_on_spec, pulses_on_spec

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


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


@pytest.mark.parametrize("spec,ncoarse", [(config_c2(32), 8), (config_c3(64, nlev=4), 2)])
def test_mixed_error_within_bound(spec, ncoarse):
    data = pulses_on_spec if spec.nlevels > 2 else gaussian_on_spec
    a, t = _run(spec, sc.SC_FP64, ncoarse, data)
    b, _ = _run(spec, sc.SC_MIXED, ncoarse, data)
    for l in range(spec.nlevels):
        umax = np.abs(a[l][0]).max()
        h = spec.dx(spec.nlevels - 1)
        bound = t * 32 * EPS32 * umax / (h * h)
        for v in range(2):
            err = np.abs(a[l][v] - b[l][v]).max()
            print(f"level {l} var {v}: |mixed - fp64| = {err:.3e}, bound {bound:.3e}")
            assert err <= bound, (l, v, err, bound)
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
