"""GPU parity at the benchmark configurations' full sizes: the 7-level towers
at N0 = 128 (27,424,754 owned points) in the launch configuration the
benchmark times (autotuned tile shapes; graph mode for whole coarse steps),
its FP32-shadow variant, the single-level and two-level wave runs, and the
7-level Z4c puncture hierarchy (8,581,008 points, 22 variables).

The reference evolves this hierarchy in about a minute per coarse step, so:
* level 0's RK4 step (y_{n+1} and k1..k4) is checked at sampled points, each
  against a reference run on a 31^3 patch around the point: the step reads
  at most 4 * 3 points away, so the patch's frozen edge values (exact at
  stage 1) cannot reach its centre;
* the refinement-boundary ghost values of level 1 (the eight stage tables and
  both end values) are checked at sampled RB points against the reference
  prolongation and dense-output combination of level 0's y_n and k1..k4;
* a whole coarse step in the benchmark configuration is compared with the
  reference evolving the whole hierarchy (every owned point of every level),
  and bitwise with per-block launches (the tiling must not change a bit);
* after the coarse step every restricted parent point equals its child value;
* the mixed-precision run stays within the stated bound of the FP64 run;
* the single-level run to t = 1 and the two-level run at coarse 64^3 are
  small enough for the reference to evolve whole;
* Z4c: level 0's step at sampled interior points against reference patch
  runs, and the FP32 right-hand side within its bound after a coarse step.
"""
from fractions import Fraction

import numpy as np
import pytest

import paper_2503_09629_amd as sc
from oracle.dense import ghost_weights_f64
from oracle.evolve import OracleRun, Prolongation, dense_ghost_value
from oracle.hierarchy import Hierarchy
from workloads import (HierarchySpec, brill_lindquist, brill_lindquist_on_spec, config_c1,
                       config_c2, config_c3, config_c5, gaussian_on_spec, pulses_on_spec,
                       standing_wave_on_spec)

pytestmark = pytest.mark.gpu
TOL = 1e-12
N0 = 128
KARR = (sc.SC_ARR_K1, sc.SC_ARR_K2, sc.SC_ARR_K3, sc.SC_ARR_K4)


@pytest.fixture(scope="module")
def towers():
    spec = config_c3(N0)
    print("full-size towers:", spec.total_points(), "points", flush=True)
    return spec, [pulses_on_spec(spec, l) for l in range(spec.nlevels)]


def _ctx(spec, data, exec, tune=False):
    ctx = sc.Context(device="cuda:0", exec=exec)
    ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
    ctx.bind()
    for l in range(spec.nlevels):
        for v in range(2):
            ctx.set_initial_data(0, l, v, data[l][v])
    if tune:
        ctx.autotune(3)
    return ctx


def _patch_step(u0, p, R=15):
    """Reference RK4 step of level 0 on the (2R+1)^3 patch centred on p;
    returns y_{n+1}, k1..k4 at the centre, per variable."""
    n = u0[0].shape[0]
    pspec = HierarchySpec((0.0,) * 3, 2.0 / n, (2 * R,) * 3, (False,) * 3, [])
    run = OracleRun(Hierarchy(pspec, min_block=16, max_block=48), sigma=0.32)
    ix = [(p[d] - R + np.arange(2 * R + 1)) % n for d in range(3)]
    for v in range(2):
        run.set_data(0, v, u0[v][np.ix_(ix[2], ix[1], ix[0])].ravel())
    q = np.rint(run.phys_coords(0) / pspec.dx0).astype(np.int64)     # patch indices
    g = (q + (np.asarray(p) - R)[None, :]) % n
    run.set_phys(0, np.stack([u0[v][g[:, 2], g[:, 1], g[:, 0]] for v in range(2)]))
    run.advance(1)
    c = (R * (2 * R + 1) + R) * (2 * R + 1) + R
    return {a: [run.get(0, v, a)[c] for v in range(2)] for a in ("y", "k1", "k2", "k3", "k4")}


def test_level0_step_and_level1_ghosts_sampled(towers):
    spec, data = towers
    ctx = _ctx(spec, data, sc.SC_EXEC_GRAPH, tune=True)
    print("tile shapes:", [ctx.tile_shape(l) for l in range(spec.nlevels)], flush=True)
    n = spec.ncells0[0]
    u0 = [data[0][v].reshape(n, n, n) for v in range(2)]
    scale = max(np.abs(u0[0]).max(), np.abs(u0[1]).max(), 1.0)
    ctx.step_level(0, 0)
    got = {"y": [ctx.read_back(0, 0, v).reshape(n, n, n) for v in range(2)]}
    for i, a in enumerate(KARR):
        got[f"k{i + 1}"] = [ctx.read_back(0, 0, v, a).reshape(n, n, n) for v in range(2)]
    rng = np.random.default_rng(11)
    worst = 0.0
    for p in rng.integers(0, n, size=(24, 3)):
        ref = _patch_step(u0, p)
        for a, vals in ref.items():
            for v in range(2):
                sc_ = scale if a == "y" else max(np.abs(got[a][v]).max(), 1.0)
                e = abs(got[a][v][p[2], p[1], p[0]] - vals[v]) / sc_
                assert e <= TOL, (tuple(p), a, v, e)
                worst = max(worst, e)
    print("level-0 step at 24 sampled points: worst rel diff", worst, flush=True)

    # level 1's refinement-boundary ghosts from level 0's last step
    ctx.prolongate(1)
    (lo, hi), = spec.fine_boxes[0]
    zz, yy, xx = np.meshgrid(*[np.arange(lo[d] - 3, hi[d] + 4) for d in (2, 1, 0)], indexing="ij")
    halo = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    inside = np.all((halo >= np.array(lo)) & (halo <= np.array(hi)), axis=1)
    rb = halo[~inside]                              # sorted by (z, y, x), as the RB list
    assert len(rb) == ctx.counts(1)[2]
    sel = np.sort(rng.choice(len(rb), size=512, replace=False))
    pro = Prolongation(None, 1, None, pts=rb[sel],
                       index_of=lambda q: ((q[:, 2] % n) * n + (q[:, 1] % n)) * n + (q[:, 0] % n),
                       vstride=n ** 3)
    Py = pro.apply(np.stack([ctx.read_back(0, 0, v, sc.SC_ARR_YN) for v in range(2)]))
    Pk = [pro.apply(np.stack([ctx.read_back(0, 0, v, a) for v in range(2)])) for a in KARR]
    H = 0.25 * spec.dx0
    worst = 0.0
    for sub in (0, 1):
        for fill in range(1, 6):
            want = dense_ghost_value(Py, Pk, ghost_weights_f64(fill, Fraction(sub, 2)), H)
            for v in range(2):
                got_rb = ctx.read_rb(0, 1, fill, sub, v)[sel]
                e = np.abs(got_rb - want[v]).max() / scale
                assert e <= TOL, (sub, fill, v, e)
                worst = max(worst, e)
    print("level-1 RB ghosts at 512 sampled points, 10 fills: worst rel diff", worst, flush=True)
    ctx.close()


def _canon_index(spec, l, pts):
    """Canonical position of level-l points (each inside one of the level's boxes)."""
    out = np.full(len(pts), -1, dtype=np.int64)
    off = 0
    for lo, hi in spec.boxes(l):
        lo, hi = np.array(lo), np.array(hi)
        nb = hi - lo + 1
        m = np.all((pts >= lo) & (pts <= hi), axis=1)
        r = pts[m] - lo
        out[m] = off + (r[:, 2] * nb[1] + r[:, 1]) * nb[0] + r[:, 0]
        off += int(np.prod(nb))
    assert (out >= 0).all()
    return out


@pytest.fixture(scope="module")
def towers_step(towers):
    """One coarse step of the towers in the benchmark configuration (FP64)."""
    spec, data = towers
    g = _ctx(spec, data, sc.SC_EXEC_GRAPH, tune=True)
    g.advance(1)
    yg = [[g.read_back(0, l, v) for v in range(2)] for l in range(spec.nlevels)]
    tg = [g.level_time(l) for l in range(spec.nlevels)]
    g.close()
    return yg, tg


def test_coarse_step_every_level_against_reference(towers, towers_step):
    """One whole coarse step of the benchmark hierarchy (all 7 levels, 127
    level steps, every prolongation and restriction) against the reference
    evolving the same hierarchy: every owned point of every level, 1e-12
    relative to the reference's max norm per variable and level."""
    import time
    spec, data = towers
    yg, tg = towers_step
    t0 = time.perf_counter()
    ref = OracleRun(Hierarchy(spec, block_seed=1, min_block=16, max_block=48))
    for l in range(spec.nlevels):
        for v in range(2):
            ref.set_data(l, v, data[l][v])
    print(f"reference set up in {time.perf_counter() - t0:.0f} s", flush=True)
    t0 = time.perf_counter()
    ref.advance(1)
    print(f"reference coarse step in {time.perf_counter() - t0:.0f} s", flush=True)
    bitwise = True
    for l in range(spec.nlevels):
        assert ref.t[l] == tg[l]
        for v in range(2):
            want = ref.get(l, v)
            e = np.abs(yg[l][v] - want).max() / max(np.abs(want).max(), 1e-300)
            bitwise = bitwise and np.array_equal(yg[l][v], want)
            print(f"level {l} var {v}: {len(want)} points, rel max diff {e:.3e}", flush=True)
            assert e <= TOL, (l, v, e)
    print("tuned graph run vs reference after one coarse step, all levels; bitwise:", bitwise,
          flush=True)
    del ref


def test_coarse_step_graph_equals_per_block_and_restriction(towers, towers_step):
    spec, data = towers
    yg, tg = towers_step
    p = _ctx(spec, data, sc.SC_EXEC_PER_BLOCK)
    p.advance(1)
    for l in range(spec.nlevels):
        assert p.level_time(l) == tg[l]
        for v in range(2):
            assert np.array_equal(p.read_back(0, l, v), yg[l][v]), (l, v)
    p.close()
    print("graph (tuned) == per block after one coarse step, all 7 levels", flush=True)
    # restriction: y_{l-1}(I) == y_l(2I) wherever 2I is a level-l point
    for l in range(1, spec.nlevels):
        for lo, hi in spec.boxes(l):
            ev = [np.arange(lo[d] + lo[d] % 2, hi[d] + 1, 2) for d in range(3)]
            zz, yy, xx = np.meshgrid(ev[2], ev[1], ev[0], indexing="ij")
            fine = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
            fi = _canon_index(spec, l, fine)
            ci = _canon_index(spec, l - 1, fine // 2)
            for v in range(2):
                assert np.array_equal(yg[l - 1][v][ci], yg[l][v][fi]), (l, v)
    print("restriction holds on every level pair", flush=True)


def test_mixed_full_size_within_bound(towers, towers_step):
    """The mixed-precision towers (the benchmark's mixed line) after one
    coarse step: |Pi_mixed - Pi_fp64| <= sqrt(N) eps32 max|Pi| / 2 and
    |u_mixed - u_fp64| <= t times that, N = 64 steps of the finest level (the
    error model derived in test_gpu_mixed)."""
    from tests.test_gpu_mixed import mixed_bounds
    spec, data = towers
    yg, tg = towers_step
    ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_GRAPH, precision=sc.SC_MIXED)
    ctx.build_spec(spec, block_seed=1, min_block=16, max_block=48)
    ctx.bind()
    for l in range(spec.nlevels):
        for v in range(2):
            ctx.set_initial_data(0, l, v, data[l][v])
    ctx.autotune(3)
    ctx.advance(1)
    pi_max = max(np.abs(yg[l][1]).max() for l in range(spec.nlevels))
    bounds = mixed_bounds(spec, 1, tg[0], pi_max)
    for l in range(spec.nlevels):
        for v in range(2):
            err = np.abs(ctx.read_back(0, l, v) - yg[l][v]).max()
            print(f"mixed level {l} var {v}: {err:.3e} (bound {bounds[v]:.3e}, "
                  f"ratio {err / bounds[v]:.3f})", flush=True)
            assert 0 < err <= bounds[v], (l, v, err, bounds[v])
    ctx.close()
def _whole(spec, data_fn, ncoarse, **kw):
    ctx = sc.Context(device="cuda:0", exec=sc.SC_EXEC_GRAPH)
    ctx.build_spec(spec, **kw)
    ctx.bind()
    ref = OracleRun(Hierarchy(spec, **kw), sigma=0.32)
    for l in range(spec.nlevels):
        for v, f in enumerate(data_fn(spec, l)):
            ctx.set_initial_data(0, l, v, f)
            ref.set_data(l, v, f)
    ctx.autotune(3)
    ctx.advance(ncoarse)
    ref.advance(ncoarse)
    worst = 0.0
    for l in range(spec.nlevels):
        assert ctx.level_time(l) == ref.t[l]
        for v in range(2):
            b = ref.get(l, v)
            e = np.abs(ctx.read_back(0, l, v) - b).max() / np.abs(b).max()
            assert e <= TOL, (l, v, e)
            worst = max(worst, e)
    ctx.close()
    return worst


def test_single_level_to_t1_matches_reference():
    """32^3 periodic standing wave, dt = 0.25 dx, 64 steps to t = 1."""
    w = _whole(config_c1(32), standing_wave_on_spec, 64, min_block=16, max_block=48)
    print("single level to t = 1: worst rel diff", w)


def test_two_level_coarse64_matches_reference():
    """Coarse 64^3 with the fine box [-1/2, 1/2]^3 (65^3 fine points), Gaussian
    pulse, 4 coarse steps."""
    w = _whole(config_c2(64), gaussian_on_spec, 4, min_block=16, max_block=48)
    print("two levels, coarse 64^3: worst rel diff", w)


@pytest.fixture(scope="module")
def punctures():
    spec = config_c5(96)
    print("full-size Z4c:", spec.total_points(), "points", flush=True)
    return spec, [brill_lindquist_on_spec(spec, l) for l in range(spec.nlevels)]


def _z4c_ctx(spec, data, precision=sc.SC_FP64, fd_order=4, ko_order=5):
    ctx = sc.Context(device="cuda:0", rhs=sc.SC_RHS_Z4C, exec=sc.SC_EXEC_GRAPH,
                     precision=precision, fd_order=fd_order, ko_order=ko_order)
    ctx.build_spec(spec)
    ctx.bind()
    for l in range(spec.nlevels):
        for v in range(22):
            ctx.set_initial_data(0, l, v, data[l][v])
        p = ctx.phys_points(l)
        if len(p):
            vals = brill_lindquist(p[:, 0], p[:, 1], p[:, 2])
            for v in range(22):
                ctx.set_phys_data(0, l, v, vals[v])
    return ctx


def test_z4c_level0_step_sampled(punctures):
    """Level 0 of the puncture hierarchy (97^3 points, frozen outer ghosts):
    one RK4 step at 6 sampled interior points against reference runs on 31^3
    patches whose edges are exact at stage 1 and 15 points from the centre."""
    spec, data = punctures
    ctx = _z4c_ctx(spec, data)
    ctx.step_level(0, 0)
    n = spec.ncells0[0] + 1
    got = [ctx.read_back(0, 0, v).reshape(n, n, n) for v in range(22)]
    gk1 = [ctx.read_back(0, 0, v, sc.SC_ARR_K1).reshape(n, n, n) for v in range(22)]
    u0 = [data[0][v].reshape(n, n, n) for v in range(22)]
    R = 15
    rng = np.random.default_rng(5)
    worst = 0.0
    for p in rng.integers(R + 3, n - R - 3, size=(6, 3)):
        corner = np.asarray(spec.origin) + (p - R) * spec.dx0
        pspec = HierarchySpec(tuple(corner), spec.dx0, (2 * R,) * 3, (False,) * 3, [])
        run = OracleRun(Hierarchy(pspec, min_block=16, max_block=48), rhs="z4c")
        sl = tuple(slice(p[d] - R, p[d] + R + 1) for d in (2, 1, 0))
        for v in range(22):
            run.set_data(0, v, u0[v][sl].ravel())
        q = np.rint((run.phys_coords(0) - corner[None, :]) / spec.dx0).astype(np.int64)
        g = q + (p - R)[None, :]
        run.set_phys(0, np.stack([u0[v][g[:, 2], g[:, 1], g[:, 0]] for v in range(22)]))
        run.advance(1)
        c = (R * (2 * R + 1) + R) * (2 * R + 1) + R
        for v in range(22):
            for arr, a, ref in ((got, "y", run.get(0, v)[c]), (gk1, "k1", run.get(0, v, "k1")[c])):
                s_ = max(np.abs(arr[v]).max(), 1e-300)
                e = abs(arr[v][p[2], p[1], p[0]] - ref) / s_
                assert e <= TOL, (tuple(p), v, a, e)
                worst = max(worst, e)
    print("z4c level-0 step at 6 sampled points: worst rel diff", worst, flush=True)
    ctx.close()


@pytest.mark.parametrize("orders", [(4, 5), (8, 5), (8, 9)], ids=["fd4-ko5", "fd8-ko5", "fd8-ko9"])
def test_z4c_first_descent_every_level_against_reference(punctures, orders):
    """The puncture hierarchy at full size: one RK4 step of every level, coarse
    to fine, each level's RB ghosts prolonged from its parent's step (the
    recursion's first descent), against the reference doing the same; every
    owned point of every level and variable, 1e-12 relative to the reference's
    max norm.  Fourth order, and eighth-order derivatives with the r = 4 and the
    r = 8 dissipation (four and five ghost layers: the derivative pass's
    32-plane columns, the nine- and eleven-tap advection/dissipation pass on the
    full-size boxes)."""
    import time
    fd, ko = orders
    spec, data = punctures
    ctx = _z4c_ctx(spec, data, fd_order=fd, ko_order=ko)
    G = (5 if ko == 9 else 4) if fd == 8 else 3
    ref = OracleRun(Hierarchy(spec, G=G, min_block=16, max_block=48), rhs="z4c", fd_order=fd,
                    ko_order=ko)
    for l in range(spec.nlevels):
        for v in range(22):
            ref.set_data(l, v, data[l][v])
        pr = ref.phys_coords(l)
        if len(pr):
            ref.set_phys(l, np.array(brill_lindquist(pr[:, 0], pr[:, 1], pr[:, 2])))
    t0 = time.perf_counter()
    for l in range(spec.nlevels):
        ctx.step_level(l, 0)
        ref.rk4_step(l)
        if l + 1 < spec.nlevels:
            ctx.prolongate(l + 1)
            ref.prolongate(l + 1)
            ref.theta0[l + 1] = 0.0
    print(f"reference descent in {time.perf_counter() - t0:.0f} s", flush=True)
    worst = 0.0
    for l in range(spec.nlevels):
        for v in range(22):
            want = ref.get(l, v)
            e = np.abs(ctx.read_back(0, l, v) - want).max() / max(np.abs(want).max(), 1e-300)
            assert e <= TOL, (l, v, e)
            worst = max(worst, e)
        print(f"level {l}: {len(want)} points, worst rel diff so far {worst:.3e}", flush=True)
    ctx.close()


def test_z4c_fp32_rhs_full_size_within_bound(punctures):
    """After one coarse step of the 7-level puncture hierarchy the FP32
    right-hand side stays within t * 32 eps32 max|y| / h_finest^2 of FP64."""
    spec, data = punctures
    out, t = {}, None
    for prec in (sc.SC_FP64, sc.SC_MIXED):
        ctx = _z4c_ctx(spec, data, prec)
        ctx.advance(1)
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
            assert np.isfinite(d) and d <= bound, (l, v, d, bound)
            worst = max(worst, d)
    print("z4c full size fp32-rhs worst |mixed - fp64|", worst, "bound", bound, flush=True)
    assert worst > 0.0
