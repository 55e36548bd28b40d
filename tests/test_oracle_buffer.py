"""Pins of the reference buffer-zone scheme (the Carpet baseline of Sec. II,
Fig. 1).

* Buffer points: a naive loop over every owned point and every RB point with
  the Chebyshev distance (across periodic wraps) gives the same list.
* Restriction skips exactly the buffer points.
* Time interpolation: the weights reproduce polynomials in time of degree 2
  (three states) and 1 (two states) exactly.
* An exact solution linear in time and quadratic (harmonic) in space,
  u = t + x^2 - y^2, Pi = 1, is reproduced to rounding on every valid point of
  a three-level run (prolongation, time interpolation of both kinds,
  restriction and the frozen stage ghosts all take part).
* Buffer width: with B = 3G the valid points do not depend on what the RB
  ghosts hold at stages 2-4 (garbage planted there changes only buffer points).
* Against a unigrid run at the fine resolution, the fine level's difference
  shrinks under refinement.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle.evolve import OracleRun, time_interp_weights
from oracle.hierarchy import Hierarchy, NestingError
from workloads import (HierarchySpec, canonical_coords, config_c2, gaussian_on_spec,
                       grown_for_buffer_zones, single_level)


def _tiny_specs():
    return [
        # periodic two-level, fine box away from the domain edge
        HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                      [[((6, 4, 8), (18, 14, 16))]]),
        # fine box whose halo wraps across the periodic boundary in x
        HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                      [[((2, 6, 6), (20, 16, 16))]]),
        # two boxes on level 1 three points apart, non-periodic in x and z
        HierarchySpec((0.0,) * 3, 0.1, (14, 14, 14), (False, True, False),
                      [[((6, 4, 6), (12, 12, 12)), ((16, 4, 14), (22, 12, 20))]]),
    ]


def _brute_buffer(spec, hier, l, B):
    N = [n << l for n in spec.ncells0]
    rb = [tuple(q) for q in hier.rb[l].tolist()]
    out = []
    for lo, hi in spec.boxes(l):
        for z in range(lo[2], hi[2] + 1):
            for y in range(lo[1], hi[1] + 1):
                for x in range(lo[0], hi[0] + 1):
                    p = (x, y, z)
                    hit = False
                    for q in rb:
                        ok = True
                        for d in range(3):
                            dd = abs(p[d] - q[d])
                            if spec.periodic[d]:
                                dd = min(dd % N[d], N[d] - dd % N[d])
                            if dd > B:
                                ok = False
                                break
                        if ok:
                            hit = True
                            break
                    if hit:
                        out.append(p)
    out.sort(key=lambda p: (p[2], p[1], p[0]))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


@pytest.mark.parametrize("which", range(3))
@pytest.mark.parametrize("B", [1, 3])
def test_buffer_points_match_brute_force(which, B):
    spec = _tiny_specs()[which]
    hier = Hierarchy(spec, min_block=3, max_block=6, G=1, buffer=B)
    for l in range(1, spec.nlevels):
        assert np.array_equal(hier.buffer[l], _brute_buffer(spec, hier, l, B))


@pytest.mark.parametrize("which", range(3))
def test_restriction_skips_exactly_the_buffer(which):
    spec = _tiny_specs()[which]
    plain = Hierarchy(spec, min_block=3, max_block=6, G=1)
    hier = Hierarchy(spec, min_block=3, max_block=6, G=1, buffer=2)
    for l in range(1, spec.nlevels):
        lev = hier.levels[l]
        buf = set(map(tuple, hier.buffer[l].tolist()))

        def fine_points(pairs):
            b, off = pairs[:, 2], pairs[:, 3]
            n = lev.bdims[b]
            r = np.stack([off % n[:, 0], (off // n[:, 0]) % n[:, 1],
                          off // (n[:, 0] * n[:, 1])], axis=1)
            return [tuple(p) for p in (lev.blocks[b, 0, :] + r).tolist()]

        got = fine_points(hier.restrict[l])
        want = [p for p in fine_points(plain.restrict[l]) if p not in buf]
        assert sorted(got) == sorted(want)
        assert not any(p in buf for p in got)
        assert len(got) < len(fine_points(plain.restrict[l]))


def test_stencil_into_parent_buffer_is_a_nesting_error():
    # level 2 sits close to level 1's edge: its stencils reach level-1 buffer points
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 16, (16,) * 3, (True,) * 3,
                         [[((8,) * 3, (24,) * 3)], [((22,) * 3, (42,) * 3)]])
    Hierarchy(spec, min_block=3, max_block=8, G=1)          # fine without buffers
    with pytest.raises(NestingError):
        Hierarchy(spec, min_block=3, max_block=8, G=1, buffer=3)


def test_time_interpolation_weights_are_exact_on_polynomials():
    for th in (Fraction(0), Fraction(1, 2), Fraction(1, 3), Fraction(1)):
        w = time_interp_weights(th, True)
        for deg in range(3):
            assert sum(wi * Fraction(t) ** deg for wi, t in zip(w, (-1, 0, 1))) == th ** deg
        w = time_interp_weights(th, False)
        assert w[0] == 0
        for deg in range(2):
            assert sum(wi * Fraction(t) ** deg for wi, t in zip(w, (-1, 0, 1))) == th ** deg
    assert time_interp_weights(Fraction(1, 2), True) == (Fraction(-1, 8), Fraction(3, 4),
                                                           Fraction(3, 8))


def _exact_linear_spec():
    # non-periodic [-1,1]^3; level 1 from coarse index 20 to 44, level 2 inside
    # level 1's valid region with room for its stencils
    return HierarchySpec((-1.0,) * 3, 2.0 / 64, (64,) * 3, (False,) * 3,
                         [[((40,) * 3, (88,) * 3)], [((106,) * 3, (148,) * 3)]])


def _is_buffer(spec, hier, l):
    x, y, z = canonical_coords(spec, l)
    idx = np.round((np.stack([x, y, z], axis=1) - np.array(spec.origin)) /
                   spec.dx(l)).astype(np.int64)
    key = lambda q: (q[:, 2] << 42) | (q[:, 1] << 21) | q[:, 0]
    return np.isin(key(idx), key(hier.buffer[l])), (x, y, z)


def test_linear_in_time_solution_is_exact_on_valid_points():
    spec = _exact_linear_spec()
    hier = Hierarchy(spec, min_block=16, max_block=48, buffer=9)
    run = OracleRun(hier, sigma=0.32, buffer_zones=True)
    for l in range(spec.nlevels):
        x, y, z = canonical_coords(spec, l)
        run.set_data(l, 0, x * x - y * y)
        run.set_data(l, 1, np.ones_like(x))
        if len(run.st[l].phys_dst):
            X = run.phys_coords(l)
            run.set_phys(l, np.stack([X[:, 0] ** 2 - X[:, 1] ** 2, np.ones(len(X))]))
    run.advance(1)
    T = run.t[0]
    assert T == run.t[1] == run.t[2] > 0
    for l in range(spec.nlevels):
        buf, (x, y, z) = _is_buffer(spec, hier, l)
        # level 0's frozen outer ghosts spoil 4 G points per coarse step
        far = np.all(np.abs(np.stack([x, y, z], axis=1)) < 1 - 14 * spec.dx(0), axis=1)
        m = ~buf & far
        assert m.sum() > 1000
        assert np.abs(run.get(l, 0)[m] - (T + (x * x - y * y)[m])).max() < 1e-14
        assert np.abs(run.get(l, 1)[m] - 1.0).max() < 1e-14
        if l > 0:   # buffer points end the step invalid (their stage ghosts were frozen)
            assert np.abs(run.get(l, 0)[buf] - (T + (x * x - y * y)[buf])).max() > 1e-6


def _gaussian_buffer_run(spec, hier, ncoarse, plant=False):
    run = OracleRun(hier, sigma=0.32, buffer_zones=True)
    for l in range(spec.nlevels):
        u, p = gaussian_on_spec(spec, l)
        run.set_data(l, 0, u)
        run.set_data(l, 1, p)
    if plant:
        rng = np.random.default_rng(7)
        orig = run.rb_values

        def garbage(l, stage):
            v = orig(l, stage)
            return v if stage == 1 else v + 1e3 * rng.standard_normal(v.shape)
        run.rb_values = garbage
    run.advance(ncoarse)
    return run


def test_valid_points_ignore_stage_ghosts():
    spec = grown_for_buffer_zones(
        HierarchySpec((-1.0,) * 3, 2.0 / 32, (32,) * 3, (True,) * 3,
                      [[((16,) * 3, (48,) * 3)], [((48,) * 3, (78,) * 3)]]), 10)
    hier = Hierarchy(spec, min_block=16, max_block=48, buffer=9)
    a = _gaussian_buffer_run(spec, hier, 1)
    b = _gaussian_buffer_run(spec, hier, 1, plant=True)
    for l in range(spec.nlevels):
        buf, _ = _is_buffer(spec, hier, l)
        for v in range(2):
            assert np.array_equal(a.get(l, v)[~buf], b.get(l, v)[~buf])
            if l > 0:
                assert not np.array_equal(a.get(l, v)[buf], b.get(l, v)[buf])


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


def test_second_order_at_the_buffer_boundary():
    """The buffer refill interpolates the parent in time with a quadratic
    (local error O(H^3) per fine step), so the fine level's difference from a
    unigrid fine run falls by about 2^2 under refinement: second order, where
    the dense-output fill keeps fourth order (a linear interpolant would
    give first order)."""
    diffs = []
    for nc in (24, 48):
        spec = grown_for_buffer_zones(config_c2(nc), 10)
        hier = Hierarchy(spec, max_block=256, min_block=16, buffer=9)
        run = _gaussian_buffer_run(spec, hier, nc // 4)
        lo, hi = spec.fine_boxes[0][0]
        n = hi[0] - lo[0] + 1
        o = nc // 2 - lo[0]
        s = slice(o, o + nc + 1)
        d = run.get(1, 0).reshape((n,) * 3)[s, s, s] - _unigrid_fine(nc, nc // 4)
        diffs.append(np.abs(d[::2, ::2, ::2]).max() if nc == 24 else
                     np.abs(d[::4, ::4, ::4]).max())
    assert diffs[1] > 0
    assert 3.0 < diffs[0] / diffs[1] < 6.0, diffs
