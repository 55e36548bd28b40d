"""GPU parity: libsubcyc (HIP, gfx950) against the CPU reference.

FP64 fields must agree within 1e-12 relative max-norm per variable per level
(normalised by the reference's max |value|); the kernels evaluate every
expression in the same order as the reference without FP contraction, so the
observed difference is expected to be exactly zero, and the tests report it.
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from workloads import (HierarchySpec, config_c1, config_c2, config_c3, ensemble_c1,
                       ensemble_on_spec, gaussian_on_spec, pulses_on_spec, standing_wave_on_spec, config_e1, spherical_gaussian_on_spec,
                       grown_for_buffer_zones)

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _gpu(spec, exec=sc.SC_EXEC_BATCHED, sigma=0.32, precision=sc.SC_FP64,
         time_stepping=sc.SC_SUBCYCLED, **kw):
    ctx = sc.Context(device="cuda:0", exec=exec, sigma=sigma, precision=precision,
                     time_stepping=time_stepping)
    ctx.build_spec(spec, **kw)
    ctx.bind()
    return ctx


def _pair(spec, data_fn, sigma=0.32, exec=sc.SC_EXEC_BATCHED, **kw):
    ctx = _gpu(spec, exec=exec, sigma=sigma, **kw)
    ref = OracleRun(Hierarchy(spec, **kw), sigma=sigma)
    for l in range(spec.nlevels):
        for v, f in enumerate(data_fn(spec, l)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
    return ctx, ref


def _rel(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def _compare_all(ctx, ref, arrays=("y",)):
    worst = 0.0
    amap = {"y": sc.SC_ARR_Y, "yn": sc.SC_ARR_YN, "k1": sc.SC_ARR_K1, "k2": sc.SC_ARR_K2,
            "k3": sc.SC_ARR_K3, "k4": sc.SC_ARR_K4}
    for l in range(ref.L):
        for v in range(2):
            for arr in arrays:
                if arr == "k4" and l == ref.L - 1:
                    continue      # the finest level does not keep k4
                e = _rel(ctx.read_back(0, l, v, amap[arr]), ref.get(l, v, arr))
                assert e <= TOL, (l, v, arr, e)
                worst = max(worst, e)
    return worst


@pytest.mark.parametrize("max_block", [48, 16])
def test_c1_single_level(max_block):
    spec = config_c1(32)
    ctx, ref = _pair(spec, lambda s, l: standing_wave_on_spec(s, l), min_block=8,
                     max_block=max_block)
    ctx.advance(16)
    ref.advance(16)
    w = _compare_all(ctx, ref, arrays=("y", "yn", "k1", "k2", "k3", "k4"))
    print("c1 worst rel diff", w)
    assert abs(ctx.level_time(0) - ref.t[0]) < 1e-15


def test_c2_two_level_fields_and_slopes():
    spec = config_c2(16)
    ctx, ref = _pair(spec, gaussian_on_spec, min_block=4, max_block=9)
    ctx.advance(3)
    ref.advance(3)
    w = _compare_all(ctx, ref, arrays=("y", "yn", "k1", "k2", "k3", "k4"))
    print("c2 worst rel diff", w)


def test_rb_ghost_values_match_reference():
    spec = config_c2(16)
    ctx, ref = _pair(spec, gaussian_on_spec, min_block=4, max_block=9)
    ctx.advance(1)
    ref.advance(1)
    # one more parent step plus its prolongation, driven piece by piece
    ctx.step_level(0)
    ctx.prolongate(1)
    ref.rk4_step(0)
    ref.prolongate(1)
    for sub, th in ((0, 0.0), (1, 0.5)):
        ref.theta0[1] = th
        for which in (1, 2, 3, 4, 5):
            want = ref.rb_values(1, which)
            for v in range(2):
                got = ctx.read_rb(0, 1, which, sub, v)
                e = _rel(got, want[v])
                assert e <= TOL, (sub, which, v, e)


def test_three_level_two_boxes():
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                         [[((4, 4, 4), (22, 22, 22))],
                          [((16, 16, 16), (24, 26, 24)), ((28, 16, 18), (36, 24, 26))]])
    ctx, ref = _pair(spec, lambda s, l: gaussian_on_spec(s, l, centre=(0.1, -0.05, 0.0),
                                                         width=0.3),
                     min_block=4, max_block=8, block_seed=9)
    ctx.advance(2)
    ref.advance(2)
    _compare_all(ctx, ref, arrays=("y", "k2"))


def test_c3_family_small():
    spec = config_c3(64, nlev=4)
    ctx, ref = _pair(spec, lambda s, l: pulses_on_spec(s, l))
    ctx.advance(1)
    ref.advance(1)
    w = _compare_all(ctx, ref, arrays=("y", "k4"))
    print("c3(64, 4 levels) worst rel diff", w)


def test_exec_modes_bitwise_equal():
    spec = config_c3(64, nlev=3)
    outs = []
    for mode in (sc.SC_EXEC_BATCHED, sc.SC_EXEC_PER_BLOCK, sc.SC_EXEC_GRAPH):
        ctx = _gpu(spec, exec=mode)
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        ctx.advance(3)     # graph mode: captures both buffer parities and replays
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(2)])
        assert abs(ctx.level_time(2) - 3 * 4 * 0.25 * spec.dx(2)) < 1e-12
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_nan_poisoned_halos_are_never_read():
    spec = config_c2(16)
    clean = _gpu(spec, min_block=4, max_block=9)
    dirty = _gpu(spec, min_block=4, max_block=9)
    dirty.poison_halos()
    for ctx in (clean, dirty):
        for l in range(2):
            for v, f in enumerate(gaussian_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        ctx.advance(2)
    assert dirty.check_finite() == sc.SC_OK
    for l in range(2):
        for v in range(2):
            assert np.array_equal(clean.read_back(0, l, v), dirty.read_back(0, l, v))


def test_ensemble_members_match_their_own_reference():
    nm = 6
    spec = ensemble_c1(nm, 16)
    ctx = _gpu(spec, min_block=8, max_block=16)
    data = ensemble_on_spec(spec, nm)
    for m in range(nm):
        for v in range(2):
            ctx.set_initial_data(m, 0, v, data[m][v])
    ctx.advance(8)
    single = config_c1(16)
    for m in (0, 3, nm - 1):
        ref = OracleRun(Hierarchy(single, min_block=8, max_block=16))
        for v in range(2):
            ref.set_data(0, v, data[m][v])
        ref.advance(8)
        for v in range(2):
            assert _rel(ctx.read_back(m, 0, v), ref.get(0, v)) <= TOL


def test_norms_and_nonfinite_flag():
    spec = config_c2(16)
    ctx, ref = _pair(spec, gaussian_on_spec, min_block=4, max_block=9)
    ctx.advance(1)
    ref.advance(1)
    for l in range(2):
        u = ref.get(l, 0)
        n = ctx.norms(0, l, 0)
        assert abs(n[0] - np.abs(u).max()) <= 1e-15 * np.abs(u).max()
        assert abs(n[1] - np.sqrt(np.mean(u * u))) <= 1e-13 * n[1]
        assert n[2] == 0
    assert ctx.check_finite() == sc.SC_OK
    bad = gaussian_on_spec(spec, 1)[0]
    bad[17] = np.nan
    ctx.set_initial_data(0, 1, 0, bad)
    assert ctx.check_finite() == sc.SC_E_NONFINITE
    assert ctx.norms(0, 1, 0)[2] == 1


def test_autotuned_tiles_bitwise_equal():
    spec = config_c3(64, nlev=4)
    outs = []
    for tune in (False, True):
        ctx = _gpu(spec)
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        if tune:
            ctx.autotune(1)
            print([ctx.tile_shape(l) for l in range(spec.nlevels)])
        ctx.advance(2)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(2)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("mixed", [False, True])
def test_pinned_tile_shapes_bitwise_equal(mixed):
    """Every stencil-kernel variant (one or two points per thread, one or two
    planes of loads in flight, z-chunks that split boxes into upward and
    downward marching pieces, odd and ragged chunks) gives the same bits."""
    spec = config_c3(64, nlev=4)
    prec = sc.SC_MIXED if mixed else sc.SC_FP64
    shapes = [None, (4, 0, 2, 1), (7, 0, 2, 2), (12, 64, 1, 2), (1 << 20, 0, 2, 1), (5, 16, 2, 1),
              (9, 0, 2, 2), (6, 24, 1, 2), (8, 0, 2, 2, 512), (13, 16, 1, 2, 512), (5, 0, 1, 2, 512),
              (7, 0, 2, 2, 256, 128), (9, 0, 1, 2, 512, 40), (6, 0, 2, 1, 256, 17)]
    outs = []
    for sh in shapes:
        ctx = _gpu(spec, precision=prec)
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        if sh is not None:
            for l in range(spec.nlevels):
                ctx.set_tile_shape(l, *sh)
                got = ctx.tile_shape(l)
                assert (got["tz"], got["depth"], got["slots"]) == (sh[0], sh[2], sh[3])
                assert got["threads"] == (sh[4] if len(sh) > 4 else 256)
                assert got["tx"] <= (min(sh[5], 78) if len(sh) > 5 else 64)
        ctx.advance(2)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(2)])
        ctx.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_autotuned_shapes_set_back_cut_the_same_tiles():
    """The shape sc_tile_shape reports after autotuning (widths included),
    passed to sc_set_tile_shape in a fresh context, cuts the same tiles."""
    spec = config_c3(64, nlev=4)
    shapes = []
    for k in range(2):
        ctx = _gpu(spec)
        for l in range(spec.nlevels):
            for v, f in enumerate(pulses_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        if k == 0:
            ctx.autotune(1)
        else:
            for l, sh in enumerate(shapes[0]):
                ctx.set_tile_shape(l, sh["tz"], sh["grid"], sh["depth"], sh["slots"],
                                   sh["threads"], sh["tx"])
        shapes.append([ctx.tile_shape(l) for l in range(spec.nlevels)])
        ctx.close()
    assert shapes[0] == shapes[1]


def test_set_tile_shape_rejects_bad_arguments():
    spec = config_c3(64, nlev=2)
    ctx = _gpu(spec)
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
    for args in ((0, 3, 0, 1, 2), (0, 8, -1, 1, 2), (0, 8, 0, 3, 2), (0, 8, 0, 1, 4), (5, 8, 0, 1, 2),
                 (0, 8, 0, 1, 1), (0, 8, 0, 4, 2), (0, 8, 0, 4, 1), (0, 8, 0, 2, 1, 512),
                 (0, 8, 0, 2, 2, 384), (0, 8, 0, 2, 2, 256, -1), (0, 8, 0, 2, 2, 256, 129)):
        with pytest.raises(sc.ScError):
            ctx.set_tile_shape(*args)
    ctx.set_tile_shape(0, 8, 0, 2, 1)
    assert ctx.tile_shape(0)["slots"] == 1 and ctx.tile_shape(0)["depth"] == 2


def test_k4_not_kept_on_finest_level():
    spec = config_c2(16)
    ctx, ref = _pair(spec, gaussian_on_spec, min_block=4, max_block=9)
    ctx.advance(1)
    ctx.read_back(0, 0, 0, sc.SC_ARR_K4)
    with pytest.raises(sc.ScError) as e:
        ctx.read_back(0, 1, 0, sc.SC_ARR_K4)
    assert e.value.code == sc.SC_E_STATE


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH, sc.SC_EXEC_PER_BLOCK])
def test_uniform_time_steps_match_reference(exec):
    """Every level on the finest step, ghosts from the parent's stage values at
    the same time (the paper's non-subcycled comparison mode)."""
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                         [[((4, 4, 4), (22, 22, 22))],
                          [((16, 16, 16), (24, 26, 24)), ((28, 16, 18), (36, 24, 26))]])
    kw = dict(min_block=4, max_block=8, block_seed=9)
    ctx = _gpu(spec, exec=exec, time_stepping=sc.SC_UNIFORM_DT, **kw)
    ref = OracleRun(Hierarchy(spec, **kw), sigma=0.32, subcycling=False)
    for l in range(spec.nlevels):
        for v, f in enumerate(gaussian_on_spec(spec, l, centre=(0.1, -0.05, 0.0), width=0.3)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
    ctx.advance(5)
    ref.advance(5)
    for l in range(spec.nlevels):
        assert abs(ctx.level_time(l) - ref.t[l]) < 1e-15
    w = _compare_all(ctx, ref, arrays=("y", "k3"))
    print("uniform time steps worst rel diff", w)


@pytest.mark.parametrize("ts", [sc.SC_SUBCYCLED, sc.SC_UNIFORM_DT])
def test_e1_layout_matches_reference(ts):
    """The scalar-wave test layout of Sec. IV.A at a coarse resolution (periodic
    [-6,6]^3 of 24 cells, refined boxes over [-4,4]^3 and [-1,1]^3) with the
    spherical Gaussian, both time-stepping modes."""
    spec = config_e1(24)
    kw = dict(min_block=8, max_block=16)
    ctx = _gpu(spec, time_stepping=ts, **kw)
    ref = OracleRun(Hierarchy(spec, **kw), sigma=0.32, subcycling=ts == sc.SC_SUBCYCLED)
    for l in range(spec.nlevels):
        for v, f in enumerate(spherical_gaussian_on_spec(spec, l, 0.0)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
    n = 2 if ts == sc.SC_SUBCYCLED else 8
    ctx.advance(n)
    ref.advance(n)
    print("e1 layout worst rel diff", _compare_all(ctx, ref, arrays=("y", "k1")))


# --- buffer zones (the Carpet scheme the paper compares against, Sec. II) ---

def _bz_spec():
    return grown_for_buffer_zones(
        HierarchySpec((-1.0,) * 3, 2.0 / 32, (32,) * 3, (True,) * 3,
                      [[((16,) * 3, (48,) * 3)], [((48,) * 3, (78,) * 3)]]), 10)


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH, sc.SC_EXEC_PER_BLOCK])
def test_buffer_zones_match_reference(exec):
    """Five coarse steps: the first with linear time interpolation at each
    level's first step, then quadratic; in graph mode the first runs eagerly
    and the next four capture and replay the three buffer rotations."""
    spec = _bz_spec()
    kw = dict(min_block=16, max_block=48, block_seed=5)
    ctx = _gpu(spec, exec=exec, time_stepping=sc.SC_BUFFER_ZONES, **kw)
    ref = OracleRun(Hierarchy(spec, buffer=9, **kw), sigma=0.32, buffer_zones=True)
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
    ctx.advance(2)
    ctx.advance(3)
    ref.advance(5)
    w = _compare_all(ctx, ref, arrays=("y", "yn", "k1", "k2", "k3", "k4"))
    print("buffer zones exec", exec, "worst rel diff", w)
    for l in range(spec.nlevels):
        assert abs(ctx.level_time(l) - ref.t[l]) < 1e-15
    with pytest.raises(sc.ScError) as e:
        ctx.step_level(1, 0)
    assert e.value.code == sc.SC_E_STATE


def test_graph_recaptured_after_single_level_steps():
    """A graph bakes in every level's state buffer; a level stepped on its own
    (sc_step_level) in between must not replay a stale graph.  The same call
    sequence in graph and batched mode gives the same bits."""
    spec = config_c2(16)
    outs = []
    for mode in (sc.SC_EXEC_GRAPH, sc.SC_EXEC_BATCHED):
        ctx = _gpu(spec, exec=mode, min_block=4, max_block=9)
        for l in range(spec.nlevels):
            for v, f in enumerate(gaussian_on_spec(spec, l)):
                ctx.set_initial_data(0, l, v, f)
        ctx.advance(2)
        ctx.prolongate(1)
        ctx.step_level(1, 0)     # one step: level 1's state buffer index flips
        ctx.advance(3)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(2)])
        ctx.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_close_right_after_advance_waits_for_the_stream():
    """close() returns only when the context's queued kernels are done, so the
    arena can go back to the allocator at once."""
    spec = config_c3(64, nlev=3)
    ctx = _gpu(spec, exec=sc.SC_EXEC_BATCHED)
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
    stream = ctx.stream
    ctx.advance(20)
    ctx.close()
    assert stream.query()


@pytest.mark.parametrize("mode", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH])
def test_restart_from_read_back_state_is_bitwise(mode):
    """Checkpoint and resume at a coarse-step boundary: every level's state read
    back after two coarse steps and loaded into a new context, then two more
    coarse steps, equals four uninterrupted coarse steps bit for bit (at a
    coarse-step boundary every level sits at the same time, and the schedule
    reads nothing from before it but the state)."""
    spec = config_c3(64, nlev=3)
    data = [pulses_on_spec(spec, l) for l in range(spec.nlevels)]

    def fresh():
        ctx = _gpu(spec, exec=mode)
        return ctx

    a = fresh()
    for l in range(spec.nlevels):
        for v in range(2):
            a.set_initial_data(0, l, v, data[l][v])
    a.advance(2)
    saved = [[a.read_back(0, l, v) for v in range(2)] for l in range(spec.nlevels)]
    a.advance(2)
    want = [[a.read_back(0, l, v) for v in range(2)] for l in range(spec.nlevels)]
    a.close()
    b = fresh()
    for l in range(spec.nlevels):
        for v in range(2):
            b.set_initial_data(0, l, v, saved[l][v])
    b.advance(2)
    for l in range(spec.nlevels):
        for v in range(2):
            assert np.array_equal(b.read_back(0, l, v), want[l][v]), (l, v)
    b.close()


def test_stage_kernel_timing_counts_every_launch_and_its_bytes():
    """sc_profile_read after eager coarse steps: one record per batched stage
    launch (levels without ghost sync share one event pair per level step),
    positive time, and the algorithmic bytes of every launch: per owned point
    and variable 16, 24, 24, 48 B for stages 1-4, 8 B less at stage 4 of the
    finest level (no k4 stored); graph mode refuses timing."""
    spec = config_c3(64, nlev=4)
    ctx = _gpu(spec, exec=sc.SC_EXEC_BATCHED)
    for l in range(spec.nlevels):
        for v, f in enumerate(pulses_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
    ctx.profile_enable(True)
    ctx.advance(2)
    n, ms, b = ctx.profile_read()
    steps = [2 * (1 << l) for l in range(spec.nlevels)]
    assert n == 4 * sum(steps)
    assert ms > 0.0
    want = 0.0
    for l in range(spec.nlevels):
        per = 16 + 24 + 24 + (48 if l + 1 < spec.nlevels else 40)
        want += steps[l] * per * 2 * spec.npoints(l)
    assert b == want
    ctx.profile_enable(False)
    ctx.close()
    g = _gpu(spec, exec=sc.SC_EXEC_GRAPH)
    with pytest.raises(sc.ScError) as e:
        g.profile_enable(True)
    assert e.value.code == sc.SC_E_STATE
    g.close()
