"""Z4c on the GPU against the CPU reference (Sec. III.A), on a small
three-level two-puncture hierarchy with frozen physical-boundary ghosts.

FP64 parity bar: 1e-12 relative max-norm per variable per level (normalised
by the reference's max |value|; variables that are still identically zero in
the reference are compared in absolute terms against 1e-12).
"""
import numpy as np
import pytest

import paper_2503_09629_amd as sc
from oracle.evolve import OracleRun
from oracle.hierarchy import Hierarchy
from workloads import brill_lindquist, brill_lindquist_on_spec, config_z4c_small

pytestmark = pytest.mark.gpu
TOL = 1e-12
KW = dict(min_block=8, max_block=16)


def _pair(spec, exec=sc.SC_EXEC_BATCHED, precision=sc.SC_FP64, outer_bc=sc.SC_BC_FROZEN,
          fd_order=4, ko_order=5):
    ctx = sc.Context(device="cuda:0", rhs=sc.SC_RHS_Z4C, exec=exec, precision=precision,
                     outer_bc=outer_bc, fd_order=fd_order, ko_order=ko_order)
    ctx.build_spec(spec, **KW)
    ctx.bind()
    G = (5 if ko_order == 9 else 4) if fd_order == 8 else 3
    ref = OracleRun(Hierarchy(spec, G=G, **KW), rhs="z4c",
                    outer_bc="radiative" if outer_bc == sc.SC_BC_RADIATIVE else "frozen",
                    fd_order=fd_order, ko_order=ko_order)
    for l in range(spec.nlevels):
        for v, f in enumerate(brill_lindquist_on_spec(spec, l)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
        p = ctx.phys_points(l)
        if len(p):
            vals = brill_lindquist(p[:, 0], p[:, 1], p[:, 2])
            for v in range(22):
                ctx.set_phys_data(0, l, v, vals[v])
        pr = ref.phys_coords(l)
        if len(pr):
            ref.set_phys(l, np.array(brill_lindquist(pr[:, 0], pr[:, 1], pr[:, 2])))
    return ctx, ref


def _compare(ctx, ref, arrays=(sc.SC_ARR_Y,)):
    names = {sc.SC_ARR_Y: "y", sc.SC_ARR_K1: "k1", sc.SC_ARR_K4: "k4"}
    worst = 0.0
    for l in range(ref.L):
        for v in range(22):
            for arr in arrays:
                a = ctx.read_back(0, l, v, arr)
                b = ref.get(l, v, names[arr])
                s = np.abs(b).max()
                e = np.abs(a - b).max() / (s if s > 1e-300 else 1.0)
                assert e <= TOL, (l, v, arr, e)
                worst = max(worst, e)
    return worst


def test_z4c_parity_two_coarse_steps():
    spec = config_z4c_small()
    ctx, ref = _pair(spec)
    ctx.advance(2)
    ref.advance(2)
    w = _compare(ctx, ref, arrays=(sc.SC_ARR_Y, sc.SC_ARR_K1, sc.SC_ARR_K4))
    print("z4c worst rel diff", w)


def test_z4c_exec_modes_agree():
    spec = config_z4c_small()
    outs = []
    for mode in (sc.SC_EXEC_BATCHED, sc.SC_EXEC_PER_BLOCK, sc.SC_EXEC_GRAPH):
        ctx, _ = _pair(spec, exec=mode)
        ctx.advance(2)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(22)])
        ctx.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)



@pytest.mark.parametrize("precision", [sc.SC_FP64, sc.SC_MIXED])
def test_z4c_tile_cuts_bitwise_equal(precision):
    """Every point of every tile is computed once, whatever the cut: the
    default Z4c tiles (two planes, threads packed over the tile's x-y points)
    and two other cuts give the same bits."""
    spec = config_z4c_small()
    outs = []
    for shape in (None, (16, 0, 2, 2, 256), (5, 0, 1, 2, 512)):
        ctx, _ = _pair(spec, precision=precision)
        if shape is not None:
            for l in range(spec.nlevels):
                ctx.set_tile_shape(l, *shape)
        ctx.advance(2)
        outs.append([ctx.read_back(0, l, v) for l in range(spec.nlevels) for v in range(22)])
        ctx.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)

def test_z4c_hamiltonian_constraint_matches_reference():
    spec = config_z4c_small()
    ctx, ref = _pair(spec)
    ctx.advance(1)
    ref.advance(1)
    for l in range(spec.nlevels):
        a = ctx.hamiltonian(0, l)
        b = ref.hamiltonian(l)
        e = np.abs(a - b).max() / np.abs(b).max()
        print("level", l, "H max", np.abs(b).max(), "rel diff", e)
        assert e <= TOL


def test_z4c_fp32_rhs_variant_within_bound():
    """FP32 stage vectors, slopes and right-hand side, FP64 state update: after
    two coarse steps every variable on every level is within
    t * 32 eps32 * max|y| / h_finest^2 of the FP64 run (the FP32 rounding of
    the stage values, amplified by the second differences, accumulated over
    the run; the same form as the wave system's bound)."""
    spec = config_z4c_small()
    out = {}
    for prec in (sc.SC_FP64, sc.SC_MIXED):
        ctx, _ = _pair(spec, precision=prec)
        ctx.advance(2)
        out[prec] = [[ctx.read_back(0, l, v) for v in range(22)] for l in range(spec.nlevels)]
        t = ctx.level_time(0)
        ctx.close()
    eps32 = float(np.finfo(np.float32).eps)
    hf = spec.dx(spec.nlevels - 1)
    ymax = max(np.abs(a).max() for lev in out[sc.SC_FP64] for a in lev)
    bound = t * 32.0 * eps32 * ymax / hf ** 2
    worst = 0.0
    for l in range(spec.nlevels):
        for v in range(22):
            d = np.abs(out[sc.SC_MIXED][l][v] - out[sc.SC_FP64][l][v]).max()
            worst = max(worst, d)
            assert np.isfinite(d) and d <= bound, (l, v, d, bound)
    print("z4c fp32-rhs worst |mixed - fp64|", worst, "bound", bound)
    assert worst > 0.0   # the variant really ran in FP32


def test_z4c_fp32_rhs_variant_hamiltonian():
    spec = config_z4c_small()
    hs = {}
    for prec in (sc.SC_FP64, sc.SC_MIXED):
        ctx, _ = _pair(spec, precision=prec)
        ctx.advance(1)
        hs[prec] = [ctx.hamiltonian(0, l) for l in range(spec.nlevels)]
        ctx.close()
    for l in range(spec.nlevels):
        a, b = hs[sc.SC_MIXED][l], hs[sc.SC_FP64][l]
        e = np.abs(a - b).max() / np.abs(b).max()
        print("level", l, "H rel diff fp32-rhs vs fp64", e)
        assert e < 1e-3


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH, sc.SC_EXEC_PER_BLOCK])
def test_z4c_radiative_boundary_matches_reference(exec):
    """Evolved outer ghosts (radiative condition) on level 0: fields and slopes
    on every level after two coarse steps, and the Hamiltonian constraint."""
    spec = config_z4c_small()
    ctx, ref = _pair(spec, exec=exec, outer_bc=sc.SC_BC_RADIATIVE)
    ctx.advance(2)
    ref.advance(2)
    w = _compare(ctx, ref, arrays=(sc.SC_ARR_Y, sc.SC_ARR_K1, sc.SC_ARR_K4))
    print("z4c radiative exec", exec, "worst rel diff", w)
    if exec == sc.SC_EXEC_BATCHED:
        for l in range(spec.nlevels):
            a, b = ctx.hamiltonian(0, l), ref.hamiltonian(l)
            e = np.abs(a - b).max() / np.abs(b).max()
            print("level", l, "H rel diff", e)
            assert e <= TOL


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH])
@pytest.mark.parametrize("bc", [sc.SC_BC_FROZEN, sc.SC_BC_RADIATIVE])
def test_z4c_eighth_order_matches_reference(exec, bc):
    """Eighth-order derivatives with four ghost layers (the production stencil
    of Sec. III.C), with both outer boundaries."""
    spec = config_z4c_small()
    ctx, ref = _pair(spec, exec=exec, outer_bc=bc, fd_order=8)
    ctx.advance(2)
    ref.advance(2)
    w = _compare(ctx, ref, arrays=(sc.SC_ARR_Y, sc.SC_ARR_K1, sc.SC_ARR_K4))
    print("z4c eighth order exec", exec, "bc", bc, "worst rel diff", w)
    if exec == sc.SC_EXEC_BATCHED:
        for l in range(spec.nlevels):
            a, b = ctx.hamiltonian(0, l), ref.hamiltonian(l)
            e = np.abs(a - b).max() / np.abs(b).max()
            print("level", l, "H rel diff", e)
            assert e <= TOL


@pytest.mark.parametrize("exec", [sc.SC_EXEC_BATCHED, sc.SC_EXEC_GRAPH, sc.SC_EXEC_PER_BLOCK])
@pytest.mark.parametrize("bc", [sc.SC_BC_FROZEN, sc.SC_BC_RADIATIVE])
def test_z4c_ninth_order_dissipation_matches_reference(exec, bc):
    """Eighth-order derivatives with the r = 8 dissipation (Sec. III.C's
    ninth-order option), five ghost layers, both outer boundaries (towers of
    20 cells: the five-layer refinement-boundary stencils stay inside one
    parent box)."""
    spec = config_z4c_small(nt=20)
    ctx, ref = _pair(spec, exec=exec, outer_bc=bc, fd_order=8, ko_order=9)
    ctx.advance(2)
    ref.advance(2)
    w = _compare(ctx, ref, arrays=(sc.SC_ARR_Y, sc.SC_ARR_K1, sc.SC_ARR_K4))
    print("z4c ninth-order dissipation exec", exec, "bc", bc, "worst rel diff", w)


def test_z4c_tile_shape_can_be_set_back():
    """The shape sc_tile_shape reports for a Z4c level can be pinned again with
    sc_set_tile_shape (two-plane z-chunks), and a pinned cut gives the same bits."""
    spec = config_z4c_small()
    a, _ = _pair(spec)
    b, _ = _pair(spec)
    for l in range(spec.nlevels):
        sh = b.tile_shape(l)
        b.set_tile_shape(l, sh["tz"], sh["grid"], sh["depth"], sh["slots"], sh["threads"])
        assert b.tile_shape(l) == sh
    b.set_tile_shape(1, 3)
    assert b.tile_shape(1)["tz"] == 3
    a.advance(1)
    b.advance(1)
    for l in range(spec.nlevels):
        for v in range(22):
            assert np.array_equal(a.read_back(0, l, v), b.read_back(0, l, v)), (l, v)
    a.close()
    b.close()
