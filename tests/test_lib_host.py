"""Host-side checks of libsubcyc.so (no GPU needed).

* every function declared in include/subcyc.h is exported;
* the library's block, ghost, RB and restriction maps are bit-identical to
  the reference builder's (canonical word stream);
* argument, nesting and state-machine errors come back as status codes;
* with buffer zones (B = 3G) the buffer lists, the restriction pairs without
  buffer points and the nesting rule against parent buffer points match too.
"""
import ctypes
import hashlib
import os
import re

import numpy as np
import pytest

import paper_2503_09629_amd as sc
from oracle.hierarchy import Hierarchy, NestingError
from workloads import HierarchySpec, config_c2, config_c3, config_c5, grown_for_buffer_zones

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "subcyc.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(sc_\w+)\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    L = sc.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(sc.binding.EXPORTED)


def _ctx_maps(spec, **kw):
    ctx = sc.Context()
    ctx.build_spec(spec, **kw)
    return ctx


SPECS = {
    "two-level-tiny": (HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                                     [[((6, 4, 8), (18, 14, 16))]]), dict(min_block=4, max_block=8)),
    "three-level-two-boxes": (HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                                            [[((4, 4, 4), (22, 22, 22))],
                                             [((16, 16, 16), (24, 26, 24)),
                                              ((28, 16, 18), (36, 24, 26))]]),
                              dict(min_block=4, max_block=8, block_seed=9)),
    "non-periodic": (HierarchySpec((0.0,) * 3, 0.1, (10, 10, 10), (False, True, False),
                                   [[((8, 4, 8), (12, 12, 12))]]), dict(min_block=4, max_block=8)),
    "full-cover": (HierarchySpec((-1.0,) * 3, 2.0 / 8, (8,) * 3, (True,) * 3,
                                 [[((0, 0, 0), (15, 15, 15))]]), dict(min_block=4, max_block=8)),
    "c2-16": (config_c2(16), dict(min_block=4, max_block=9)),
    "c2-32": (config_c2(32), dict()),
    "c3-64": (config_c3(64), dict()),
    "c3-64-seed2": (config_c3(64), dict(block_seed=2, min_block=16, max_block=32)),
    "c5-96": (config_c5(96), dict()),
}


@pytest.mark.parametrize("name", sorted(SPECS))
def test_maps_bit_identical_to_reference(name):
    spec, kw = SPECS[name]
    ref = Hierarchy(spec, **kw).export()
    got = _ctx_maps(spec, **kw).export_maps()
    assert got.shape == ref.shape
    assert hashlib.sha256(got.tobytes()).hexdigest() == hashlib.sha256(ref.tobytes()).hexdigest()


def test_counts_match_reference():
    spec, kw = SPECS["c3-64"]
    ref = Hierarchy(spec, **kw)
    ctx = _ctx_maps(spec, **kw)
    for l in range(spec.nlevels):
        assert ctx.counts(l) == ref.counts(l)


def test_nesting_errors_are_status_codes():
    base = dict(origin=(-1.0,) * 3, dx0=2.0 / 16, ncells0=(16,) * 3, periodic=(True,) * 3)
    bad = [
        [[((8, 8, 8), (17, 24, 24))]],
        [[((8, 8, 8), (34, 24, 24))]],
        [[((8, 8, 8), (16, 16, 16)), ((14, 14, 14), (24, 24, 24))]],
        [[((8, 8, 8), (24, 24, 24))], [((16, 18, 18), (30, 30, 30))]],
    ]
    for fb in bad:
        spec = HierarchySpec(fine_boxes=fb, **base)
        with pytest.raises(NestingError):
            Hierarchy(spec, min_block=4)
        with pytest.raises(sc.ScError) as e:
            _ctx_maps(spec, min_block=4)
        assert e.value.code == sc.SC_E_NEST


def test_argument_and_state_errors():
    with pytest.raises(sc.ScError) as e:
        sc.Context(cfl=0.75)
    assert e.value.code == sc.SC_E_ARG
    ctx = sc.Context()
    with pytest.raises(sc.ScError) as e:
        ctx.advance(1)
    assert e.value.code == sc.SC_E_STATE
    with pytest.raises(sc.ScError) as e:
        ctx.device_bytes()
    assert e.value.code == sc.SC_E_STATE
    spec, kw = SPECS["c2-16"]
    ctx.build_spec(spec, **kw)
    with pytest.raises(sc.ScError) as e:
        ctx.build_spec(spec, **kw)
    assert e.value.code == sc.SC_E_STATE
    with pytest.raises(sc.ScError) as e:
        ctx.advance(1)            # not bound yet
    assert e.value.code == sc.SC_E_STATE
    assert ctx.device_bytes() > 0
    with pytest.raises(sc.ScError) as e:
        ctx.counts(5)
    assert e.value.code == sc.SC_E_ARG


def test_arena_size_scales_with_members():
    spec, kw = SPECS["c2-16"]
    a = _ctx_maps(spec, **kw).device_bytes()
    spec2 = HierarchySpec(spec.origin, spec.dx0, spec.ncells0, spec.periodic, spec.fine_boxes,
                          nmembers=4)
    b = _ctx_maps(spec2, **kw).device_bytes()
    assert 3.5 * a < b < 4.5 * a


BZ_SPECS = {
    "c2-24-grown": (grown_for_buffer_zones(config_c2(24), 10), dict(min_block=16, max_block=48)),
    "three-level-grown": (grown_for_buffer_zones(
        HierarchySpec((-1.0,) * 3, 2.0 / 32, (32,) * 3, (True,) * 3,
                      [[((16,) * 3, (48,) * 3)], [((48,) * 3, (78,) * 3)]]), 10),
        dict(min_block=16, max_block=48, block_seed=5)),
}


@pytest.mark.parametrize("name", sorted(BZ_SPECS))
def test_buffer_zone_maps_bit_identical_to_reference(name):
    spec, kw = BZ_SPECS[name]
    ref = Hierarchy(spec, buffer=9, **kw)
    assert all(len(b) > 0 for b in ref.buffer[1:])
    ctx = sc.Context(time_stepping=sc.SC_BUFFER_ZONES)
    ctx.build_spec(spec, **kw)
    got = ctx.export_maps()
    want = ref.export()
    assert [ctx.buffer_count(l) for l in range(spec.nlevels)] == [len(b) for b in ref.buffer]
    assert got[1] == 2
    assert got.shape == want.shape
    assert hashlib.sha256(got.tobytes()).hexdigest() == hashlib.sha256(want.tobytes()).hexdigest()


def test_buffer_zone_nesting_error():
    # level 2's stencils stay in level 1 but reach its buffer points
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 32, (32,) * 3, (True,) * 3,
                         [[((16,) * 3, (48,) * 3)], [((40,) * 3, (86,) * 3)]])
    Hierarchy(spec, min_block=8, max_block=24)
    _ctx_maps(spec, min_block=8, max_block=24)
    with pytest.raises(NestingError):
        Hierarchy(spec, min_block=8, max_block=24, buffer=9)
    ctx = sc.Context(time_stepping=sc.SC_BUFFER_ZONES)
    with pytest.raises(sc.ScError) as e:
        ctx.build_spec(spec, min_block=8, max_block=24)
    assert e.value.code == sc.SC_E_NEST


def test_buffer_zones_need_wave_fp64():
    for kw in (dict(precision=sc.SC_MIXED), dict(rhs=sc.SC_RHS_Z4C)):
        with pytest.raises(sc.ScError) as e:
            sc.Context(time_stepping=sc.SC_BUFFER_ZONES, **kw)
        assert e.value.code == sc.SC_E_ARG


@pytest.mark.parametrize("name", ["two-level-tiny", "three-level-two-boxes", "c2-16"])
def test_four_ghost_layer_maps_bit_identical_to_reference(name):
    spec, kw = SPECS[name]
    ref = Hierarchy(spec, G=4, **kw).export()
    ctx = sc.Context(fd_order=8)
    ctx.build_spec(spec, **kw)
    got = ctx.export_maps()
    assert got.shape == ref.shape
    assert hashlib.sha256(got.tobytes()).hexdigest() == hashlib.sha256(ref.tobytes()).hexdigest()


def test_eighth_order_configuration_rules():
    sc.Context(fd_order=8)
    sc.Context(fd_order=8, time_stepping=sc.SC_UNIFORM_DT)
    sc.Context(fd_order=8, rhs=sc.SC_RHS_Z4C)
    for kw in (dict(precision=sc.SC_MIXED), dict(rhs=sc.SC_RHS_Z4C, precision=sc.SC_MIXED),
               dict(time_stepping=sc.SC_BUFFER_ZONES), dict(fd_order=6)):
        with pytest.raises(sc.ScError) as e:
            sc.Context(**dict(dict(fd_order=8), **kw))
        assert e.value.code == sc.SC_E_ARG


@pytest.mark.parametrize("name", ["two-level-tiny", "c2-16"])
def test_five_ghost_layer_maps_bit_identical_to_reference(name):
    spec, kw = SPECS[name]
    ref = Hierarchy(spec, G=5, **kw).export()
    ctx = sc.Context(fd_order=8, ko_order=9)
    ctx.build_spec(spec, **kw)
    got = ctx.export_maps()
    assert got.shape == ref.shape
    assert hashlib.sha256(got.tobytes()).hexdigest() == hashlib.sha256(ref.tobytes()).hexdigest()


def test_ninth_order_dissipation_configuration_rules():
    """Five ghost layers (the r = 8 dissipation) with eighth-order derivatives,
    wave or Z4c (either outer boundary), FP64; not with mixed precision or
    buffer zones; a hierarchy whose five-layer RB stencils leave the parent
    level is a nesting error."""
    sc.Context(fd_order=8, ko_order=9)
    sc.Context(fd_order=8, ko_order=9, time_stepping=sc.SC_UNIFORM_DT)
    sc.Context(fd_order=8, ko_order=9, rhs=sc.SC_RHS_Z4C)
    sc.Context(fd_order=8, ko_order=9, rhs=sc.SC_RHS_Z4C, outer_bc=sc.SC_BC_RADIATIVE)
    for kw in (dict(precision=sc.SC_MIXED), dict(rhs=sc.SC_RHS_Z4C, precision=sc.SC_MIXED),
               dict(time_stepping=sc.SC_BUFFER_ZONES)):
        with pytest.raises(sc.ScError) as e:
            sc.Context(**dict(dict(fd_order=8, ko_order=9), **kw))
        assert e.value.code == sc.SC_E_ARG
    spec, kw = SPECS["three-level-two-boxes"]
    ctx = sc.Context(fd_order=8, ko_order=9)
    with pytest.raises(sc.ScError) as e:
        ctx.build_spec(spec, **kw)
    assert e.value.code == sc.SC_E_NEST


def test_radiative_boundary_configuration_rules():
    sc.Context(rhs=sc.SC_RHS_Z4C, outer_bc=sc.SC_BC_RADIATIVE)
    for kw in (dict(rhs=sc.SC_RHS_WAVE), dict(rhs=sc.SC_RHS_Z4C, precision=sc.SC_MIXED),
               dict(rhs=sc.SC_RHS_Z4C, outer_bc=2)):
        with pytest.raises(sc.ScError) as e:
            sc.Context(**dict(dict(outer_bc=sc.SC_BC_RADIATIVE), **kw))
        assert e.value.code == sc.SC_E_ARG
    ctx = sc.Context(rhs=sc.SC_RHS_Z4C, outer_bc=sc.SC_BC_RADIATIVE)
    with pytest.raises(sc.ScError) as e:     # periodic domain
        ctx.build_spec(config_c2(16), min_block=4, max_block=9)
    assert e.value.code == sc.SC_E_ARG


def test_z4c_contexts_cut_short_tiles():
    """The Z4c kernels run one wave per SIMD, so Z4c contexts cut two-plane
    tiles of at most 256 points per plane (several per resident workgroup
    slot); wave contexts keep the stencil kernel's default cut."""
    spec = config_c5(96)
    z = sc.Context(rhs=sc.SC_RHS_Z4C)
    z.build_spec(spec)
    w = sc.Context()
    w.build_spec(spec)
    for l in range(spec.nlevels):
        zs, ws = z.tile_shape(l), w.tile_shape(l)
        assert zs["tz"] == 2 and zs["slots"] == 1, zs
        assert zs["tx"] * zs["ty"] <= 256, zs
        assert zs["tiles"] >= 10 * ws["tiles"], (zs, ws)
        assert ws["tz"] == 16 and ws["slots"] == 2, ws


def test_z4c_contexts_launch_one_workgroup_per_tile():
    """Z4c launches: one workgroup per tile, rounded up to whole rounds of the
    eight XCDs."""
    spec = config_c5(96)
    z = sc.Context(rhs=sc.SC_RHS_Z4C)
    z.build_spec(spec)
    for l in range(spec.nlevels):
        s = z.tile_shape(l)
        assert s["grid"] % 8 == 0 and s["tiles"] <= s["grid"] < s["tiles"] + 8, s
