"""Pins of the reference subcycled evolution.

* One periodic level with a standing wave: the fully discrete solution is a
  2x2 matrix power acting on the mode amplitude (the RK4 stability
  polynomial of the discrete operator's Fourier symbol); the run must match
  it to rounding, and the exact continuum solution cos(sqrt(3) pi t) to
  truncation error.
* Partition invariance: blocks are bookkeeping, so results are bitwise
  independent of the block seed and block sizes.
* Full cover: a fine level covering the whole periodic domain has no
  refinement boundary and must reproduce a single-level fine run bitwise
  (checks the substep count, the fine time step and restriction).
* Two-level Gaussian: cube symmetries hold to rounding, self-convergence is
  fourth order (ratio near 16 under doubling), and the difference from a
  single-level fine run shrinks at fourth order.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from workloads import (HierarchySpec, config_c1, config_c2, gaussian_on_spec, single_level,
                       standing_wave_on_spec)


def discrete_amplitude(n, m, sigma, nsteps, cfl=0.25, L=2.0):
    """u-amplitude of the fully discrete standing wave after nsteps RK4 steps."""
    mp.mp.dps = 40
    h = mp.mpf(L) / n
    dt = cfl * h
    lam = sum((-2 * mp.cos(2 * mi * mp.pi * h) + 32 * mp.cos(mi * mp.pi * h) - 30) / (12 * h * h)
              for mi in m)
    q = -(mp.mpf(sigma) / h) * sum(mp.sin(mi * mp.pi * h / 2) ** 6 for mi in m)
    A = mp.matrix([[q, 1], [lam, q]]) * dt
    M = mp.eye(2)
    term = mp.eye(2)
    for j in range(1, 5):
        term = term * A / j
        M = M + term
    v = mp.matrix([1, 0])
    for _ in range(nsteps):
        v = M * v
    return float(v[0]), float(v[1])


def _run_c1(n, m, sigma, nsteps, max_block=48, amp=1.0):
    spec = config_c1(n)
    run = OracleRun(Hierarchy(spec, max_block=max_block, min_block=min(16, n // 2)), sigma=sigma)
    u, p = standing_wave_on_spec(spec, 0, m, amp)
    run.set_data(0, 0, u)
    run.set_data(0, 1, p)
    run.advance(nsteps)
    return run, u


@pytest.mark.parametrize("sigma", [0.32, 0.0])
@pytest.mark.parametrize("m", [(1, 1, 1), (2, 1, 3)])
def test_c1_fully_discrete_closed_form(sigma, m):
    n, nsteps = 32, 64
    run, u0 = _run_c1(n, m, sigma, nsteps)
    au, ap = discrete_amplitude(n, m, sigma, nsteps)
    u = run.get(0, 0)
    p = run.get(0, 1)
    scale = np.abs(u0).max()
    assert np.abs(u - au * u0).max() / scale < 1e-13
    assert np.abs(p - ap * u0).max() / (scale * max(1.0, abs(ap))) < 1e-13
    assert abs(run.t[0] - 1.0) < 1e-15


def test_c1_matches_continuum_to_truncation():
    run, u0 = _run_c1(32, (1, 1, 1), 0.32, 64)
    i = np.argmax(np.abs(u0))
    a = run.get(0, 0)[i] / u0[i]
    err = abs(a - math.cos(math.sqrt(3) * math.pi))
    assert 3.5e-5 < err < 5.5e-5


def test_c1_continuum_convergence_order():
    errs = []
    for n in (16, 32):
        run, u0 = _run_c1(n, (1, 1, 1), 0.0, 2 * n)
        i = np.argmax(np.abs(u0))
        errs.append(abs(run.get(0, 0)[i] / u0[i] - math.cos(math.sqrt(3) * math.pi)))
    assert 13 < errs[0] / errs[1] < 19


def _two_level_run(spec, ncoarse, sigma=0.32, **hk):
    run = OracleRun(Hierarchy(spec, **hk), sigma=sigma)
    for l in range(spec.nlevels):
        u, p = gaussian_on_spec(spec, l)
        run.set_data(l, 0, u)
        run.set_data(l, 1, p)
    run.advance(ncoarse)
    return run


def test_partition_invariance():
    spec = config_c2(16)
    outs = []
    for seed, mn, mx in ((1, 4, 17), (2, 4, 8), (3, 5, 9), (1, 4, 12)):
        run = _two_level_run(spec, 3, block_seed=seed, min_block=mn, max_block=mx)
        outs.append([run.get(l, v) for l in range(2) for v in range(2)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_full_cover_equals_single_level_fine():
    n = 12
    spec = HierarchySpec((-1.0,) * 3, 2.0 / n, (n,) * 3, (True,) * 3,
                         [[((0, 0, 0), (2 * n - 1,) * 3)]])
    two = _two_level_run(spec, 3, min_block=4, max_block=12)
    fine_spec = single_level(2 * n)
    one = OracleRun(Hierarchy(fine_spec, min_block=6, max_block=12), sigma=0.32)
    u, p = gaussian_on_spec(fine_spec, 0)
    one.set_data(0, 0, u)
    one.set_data(0, 1, p)
    one.advance(6)
    for v in range(2):
        assert np.array_equal(two.get(1, v), one.get(0, v))
        # the coarse level holds the injected fine solution
        assert np.array_equal(two.get(0, v), one.get(0, v).reshape((2 * n,) * 3)[::2, ::2, ::2]
                              .ravel())


def test_two_level_cube_symmetries():
    nc = 16
    spec = config_c2(nc)
    run = _two_level_run(spec, 8, min_block=4, max_block=9)
    u0 = run.get(0, 0).reshape((nc,) * 3)
    n1 = nc + 1
    u1 = run.get(1, 0).reshape((n1,) * 3)
    scale = np.abs(u1).max()
    # x -> -x: level 0 index i -> (N - i) mod N; level 1 box is symmetric about its centre
    refl0 = np.roll(u0[:, :, ::-1], 1, axis=2)
    assert np.abs(u0 - refl0).max() / scale < 1e-13
    assert np.abs(u1 - u1[:, :, ::-1]).max() / scale < 1e-13
    # axis permutations
    for axes in ((0, 2, 1), (1, 0, 2), (2, 1, 0)):
        assert np.abs(u1 - u1.transpose(axes)).max() / scale < 1e-13
    assert np.abs(u1).max() > 0.1


def _fine_level_common(nc, sigma, tfin):
    spec = config_c2(nc)
    run = _two_level_run(spec, int(round(tfin / (0.25 * 2.0 / nc))), sigma=sigma,
                         max_block=256)
    n1 = nc + 1
    return run.get(1, 0).reshape((n1,) * 3)


def test_two_level_self_convergence_fourth_order():
    f16 = _fine_level_common(16, 0.32, 0.5)
    f32 = _fine_level_common(32, 0.32, 0.5)
    f64 = _fine_level_common(64, 0.32, 0.5)
    e1 = f16[::2, ::2, ::2] - f32[::4, ::4, ::4]
    e2 = f32[::4, ::4, ::4] - f64[::8, ::8, ::8]
    Q = np.abs(e1).max() / np.abs(e2).max()
    assert 12.0 < Q < 20.0, Q


def _unigrid_fine(nc, ncoarse):
    spec = single_level(2 * nc)
    run = OracleRun(Hierarchy(spec, max_block=256, min_block=16), sigma=0.32)
    u, p = gaussian_on_spec(spec, 0)
    run.set_data(0, 0, u)
    run.set_data(0, 1, p)
    run.advance(2 * ncoarse)
    full = run.get(0, 0).reshape((2 * nc,) * 3)
    s = slice(nc // 2, 3 * nc // 2 + 1)
    return full[s, s, s]


def test_two_level_agrees_with_unigrid_fine_to_truncation():
    diffs = []
    for nc in (16, 32):
        ncoarse = nc // 4     # t = 0.125
        two = _two_level_run(config_c2(nc), ncoarse, max_block=256)
        n1 = nc + 1
        d = two.get(1, 0).reshape((n1,) * 3) - _unigrid_fine(nc, ncoarse)
        diffs.append(np.abs(d[::2, ::2, ::2]).max() if nc == 16 else
                     np.abs(d[::4, ::4, ::4]).max())
    assert diffs[1] > 0
    assert 8.0 < diffs[0] / diffs[1] < 40.0, diffs


# --- uniform time steps (the paper's comparison mode, Sec. IV.A) ------------

def _uniform_run(spec, nsteps, sigma=0.32, **hk):
    run = OracleRun(Hierarchy(spec, **hk), sigma=sigma, subcycling=False)
    for l in range(spec.nlevels):
        u, p = gaussian_on_spec(spec, l)
        run.set_data(l, 0, u)
        run.set_data(l, 1, p)
    run.advance(nsteps)
    return run


def test_uniform_dt_full_cover_equals_single_level_fine():
    """Every level takes the finest step once per parent step: with the fine
    level covering the periodic domain, the fine level is a unigrid run with
    one step per coarse step and the coarse level its injection."""
    n = 12
    spec = HierarchySpec((-1.0,) * 3, 2.0 / n, (n,) * 3, (True,) * 3,
                         [[((0, 0, 0), (2 * n - 1,) * 3)]])
    two = _uniform_run(spec, 5, min_block=4, max_block=12)
    assert two.dt[0] == two.dt[1] == 0.25 * 2.0 / (2 * n)
    fine_spec = single_level(2 * n)
    one = OracleRun(Hierarchy(fine_spec, min_block=6, max_block=12), sigma=0.32)
    u, p = gaussian_on_spec(fine_spec, 0)
    one.set_data(0, 0, u)
    one.set_data(0, 1, p)
    one.advance(5)
    for v in range(2):
        assert np.array_equal(two.get(1, v), one.get(0, v))
        assert np.array_equal(two.get(0, v), one.get(0, v).reshape((2 * n,) * 3)[::2, ::2, ::2]
                              .ravel())


def test_uniform_dt_agrees_with_unigrid_fine_to_truncation():
    """The fine level of a two-level uniform-step run differs from a unigrid
    fine run only through the coarse solution behind its refinement boundary:
    the difference falls by about 2^4 under refinement."""
    diffs = []
    for nc in (16, 32):
        ncoarse = nc // 4     # t = 0.125 on the fine step
        two = _uniform_run(config_c2(nc), 2 * ncoarse, max_block=256)
        n1 = nc + 1
        d = two.get(1, 0).reshape((n1,) * 3) - _unigrid_fine(nc, ncoarse)
        diffs.append(np.abs(d[::2, ::2, ::2]).max() if nc == 16 else
                     np.abs(d[::4, ::4, ::4]).max())
    assert diffs[1] > 0
    assert 8.0 < diffs[0] / diffs[1] < 40.0, diffs


def test_uniform_dt_and_subcycling_agree_to_truncation():
    """Both schedules converge to the same solution: their difference on the
    fine level falls by about 2^4 under refinement."""
    diffs = []
    for nc in (16, 32):
        ncoarse = nc // 4
        sub = _two_level_run(config_c2(nc), ncoarse, max_block=256)
        uni = _uniform_run(config_c2(nc), 2 * ncoarse, max_block=256)
        assert abs(sub.t[1] - uni.t[1]) < 1e-15 and abs(sub.t[0] - uni.t[0]) < 1e-15
        n1 = nc + 1
        d = (sub.get(1, 0) - uni.get(1, 0)).reshape((n1,) * 3)
        diffs.append(np.abs(d[::2, ::2, ::2]).max() if nc == 16 else
                     np.abs(d[::4, ::4, ::4]).max())
    assert diffs[1] > 0
    assert 8.0 < diffs[0] / diffs[1] < 40.0, diffs
