"""Closed-form initial data evaluated by the library (sc_set_initial_data_analytic)
against the same fields from the shared input generator (workloads/), which
the other tests upload with sc_set_initial_data.

The two sides evaluate the same formulas with their own sin, exp and sqrt, so
they agree to a few ulps, not bitwise: the bound is 1e-13 relative to the
field's max norm.  Seeded kinds must draw the same parameters (SplitMix64) as
the generator, which a wrong draw order or mapping would break by O(1).  For
Brill-Lindquist data the frozen physical-boundary ghosts are set too: one
coarse step from the analytic data equals, to the same bound, one from host
data with the ghosts set through sc_set_phys_data.
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from workloads import (brill_lindquist, brill_lindquist_on_spec, config_c1, config_c2, config_c3,
                       config_e1, config_z4c_small, ensemble_c1, ensemble_on_spec, gaussian_on_spec,
                       pulses_on_spec, spherical_gaussian_on_spec, standing_wave_on_spec)

pytestmark = pytest.mark.gpu
TOL = 1e-13


def _ctx(spec, **kw):
    ctx = sc.Context(device="cuda:0", **kw)
    ctx.build_spec(spec, min_block=8, max_block=24)
    ctx.bind()
    return ctx


def _check(ctx, spec, want, member=0, nvars=2):
    for l in range(spec.nlevels):
        for v in range(nvars):
            got = ctx.read_back(member, l, v)
            w = want(l)[v]
            scale = max(np.abs(w).max(), 1e-300)
            e = np.abs(got - w).max() / scale if np.abs(w).max() > 0 else np.abs(got).max()
            assert e <= TOL, (l, v, e)


def test_standing_wave():
    spec = config_c1(32)
    ctx = _ctx(spec)
    ctx.set_initial_data_analytic(sc.SC_ID_STANDING_WAVE, (1.25, 1, 2, 3))
    _check(ctx, spec, lambda l: standing_wave_on_spec(spec, l, (1, 2, 3), 1.25))
    ctx.close()


def test_seeded_ensemble_standing_waves():
    nm = 6
    spec = ensemble_c1(nm, 16)
    ctx = _ctx(spec)
    ctx.set_initial_data_analytic(sc.SC_ID_STANDING_WAVE, (), seed=2)
    data = ensemble_on_spec(spec, nm, seed=2)
    for m in range(nm):
        _check(ctx, spec, lambda l, m=m: data[m], member=m)
    ctx.close()


def test_gaussian_explicit_parameters():
    spec = config_c2(16)
    ctx = _ctx(spec)
    ctx.set_initial_data_analytic(sc.SC_ID_GAUSSIAN_PULSES, (1, 2.0, 1.0, 0.2, 0.0, 0.0, 0.0))
    _check(ctx, spec, lambda l: gaussian_on_spec(spec, l))
    ctx.close()


@pytest.mark.parametrize("precision", [sc.SC_FP64, sc.SC_MIXED])
def test_seeded_pulses_on_the_towers(precision):
    spec = config_c3(64, nlev=4)
    ctx = _ctx(spec, precision=precision)
    ctx.set_initial_data_analytic(sc.SC_ID_GAUSSIAN_PULSES, (8, 2.0, 0.3), seed=2)
    _check(ctx, spec, lambda l: pulses_on_spec(spec, l, seed=2))
    ctx.close()


def test_spherical_gaussian():
    spec = config_e1(60, half=6.0)
    ctx = _ctx(spec)
    ctx.set_initial_data_analytic(sc.SC_ID_SPHERICAL_GAUSSIAN, (1.0, 0.25 / np.sqrt(2.0), 0.3))
    _check(ctx, spec, lambda l: spherical_gaussian_on_spec(spec, l, 0.3))
    ctx.close()


def test_brill_lindquist_fields_and_frozen_ghosts():
    spec = config_z4c_small()
    a = _ctx(spec, rhs=sc.SC_RHS_Z4C)
    a.set_initial_data_analytic(sc.SC_ID_BRILL_LINDQUIST, (0.5, 0.5, 3.0, -3.0))
    _check(a, spec, lambda l: brill_lindquist_on_spec(spec, l), nvars=22)
    b = _ctx(spec, rhs=sc.SC_RHS_Z4C)
    for l in range(spec.nlevels):
        for v, f in enumerate(brill_lindquist_on_spec(spec, l)):
            b.set_initial_data(0, l, v, f)
        p = b.phys_points(l)
        if len(p):
            vals = brill_lindquist(p[:, 0], p[:, 1], p[:, 2])
            for v in range(22):
                b.set_phys_data(0, l, v, vals[v])
    a.advance(1)
    b.advance(1)
    for l in range(spec.nlevels):
        for v in range(22):
            x, y = a.read_back(0, l, v), b.read_back(0, l, v)
            scale = max(np.abs(y).max(), 1.0)
            assert np.abs(x - y).max() / scale <= 1e-12, (l, v)
    a.close()
    b.close()


def test_rejects_bad_kinds_and_parameters():
    spec = config_c1(16)
    ctx = _ctx(spec)
    for kind, params in ((99, ()), (sc.SC_ID_BRILL_LINDQUIST, (0.5, 0.5, 3.0, -3.0)),
                         (sc.SC_ID_STANDING_WAVE, (1.0, 2.0)),
                         (sc.SC_ID_GAUSSIAN_PULSES, (40, 2.0, 0.3)),
                         (sc.SC_ID_SPHERICAL_GAUSSIAN, (1.0, 0.0, 0.0))):
        with pytest.raises(sc.ScError) as e:
            ctx.set_initial_data_analytic(kind, params)
        assert e.value.code == sc.SC_E_ARG
    ctx.close()
