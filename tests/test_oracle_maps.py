"""Pins of the reference block split and index maps.

The vectorised builder is compared with a deliberately naive pure-Python
classification (loops over every ghost point and every block) on tiny
hierarchies, and with structural invariants on the benchmark geometries.
"""
import os

import numpy as np
import pytest

from oracle.hierarchy import MAGIC, PHYS, RB, SYNC, Hierarchy, NestingError
from oracle.splitmix import SplitMix64
from workloads import HierarchySpec, config_c2, config_c3, config_c5

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_published_outputs():
    seeds = {}
    cur = None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("seed"):
            cur = int(line.split()[1]); seeds[cur] = []
        else:
            seeds[cur].append(int(line, 0))
    for seed, outs in seeds.items():
        r = SplitMix64(seed)
        assert [r.next() for _ in outs] == outs


def _tiny_specs():
    return [
        # periodic two-level, fine box away from the domain edge
        HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                      [[((6, 4, 8), (18, 14, 16))]]),
        # periodic three-level with two fine boxes on level 2
        HierarchySpec((-1.0,) * 3, 2.0 / 12, (12, 12, 12), (True,) * 3,
                      [[((4, 4, 4), (22, 22, 22))],
                       [((16, 16, 16), (24, 26, 24)), ((28, 16, 18), (36, 24, 26))]]),
        # non-periodic in x and z: level-0 blocks at the domain edge get PHYS ghosts
        HierarchySpec((0.0,) * 3, 0.1, (10, 10, 10), (False, True, False),
                      [[((8, 4, 8), (12, 12, 12))]]),
    ]


def _brute_force(spec, hier):
    """Naive classification straight from the definitions."""
    G = hier.G
    out = []
    for l in range(spec.nlevels):
        lev = hier.levels[l]
        N = [n << l for n in spec.ncells0]
        blocks = [tuple(map(tuple, b)) for b in lev.blocks]

        def owner(q):
            for i, (lo, hi) in enumerate(blocks):
                if all(lo[d] <= q[d] <= hi[d] for d in range(3)):
                    n = [hi[d] - lo[d] + 1 for d in range(3)]
                    r = [q[d] - lo[d] for d in range(3)]
                    return i, (r[2] * n[1] + r[1]) * n[0] + r[0]
            return None

        slots = []
        rbset = set()
        for b, (lo, hi) in enumerate(blocks):
            per = []
            for z in range(lo[2] - G, hi[2] + G + 1):
                for y in range(lo[1] - G, hi[1] + G + 1):
                    for x in range(lo[0] - G, hi[0] + G + 1):
                        p = (x, y, z)
                        if all(lo[d] <= p[d] <= hi[d] for d in range(3)):
                            continue
                        q = list(p)
                        phys = False
                        for d in range(3):
                            if spec.periodic[d]:
                                q[d] %= N[d]
                            elif not 0 <= q[d] <= N[d]:
                                phys = True
                        if phys:
                            per.append((PHYS, -1, 0))
                            continue
                        o = owner(q)
                        if o is not None:
                            per.append((SYNC, o[0], o[1]))
                        else:
                            per.append((RB, tuple(q), 0))
                            rbset.add((q[2], q[1], q[0]))
            slots.append(per)
        rblist = sorted(rbset)
        idx = {k: i for i, k in enumerate(rblist)}
        for per in slots:
            for j, (k, a, c) in enumerate(per):
                if k == RB:
                    per[j] = (RB, idx[(a[2], a[1], a[0])], 0)
        pairs = []
        if l > 0:
            plev = hier.levels[l - 1]
            pblocks = [tuple(map(tuple, b)) for b in plev.blocks]
            for fb, (lo, hi) in enumerate(blocks):
                n = [hi[d] - lo[d] + 1 for d in range(3)]
                for z in range(lo[2], hi[2] + 1):
                    for y in range(lo[1], hi[1] + 1):
                        for x in range(lo[0], hi[0] + 1):
                            if x % 2 or y % 2 or z % 2:
                                continue
                            I = (x // 2, y // 2, z // 2)
                            for cb, (clo, chi) in enumerate(pblocks):
                                if all(clo[d] <= I[d] <= chi[d] for d in range(3)):
                                    cn = [chi[d] - clo[d] + 1 for d in range(3)]
                                    co = ((I[2] - clo[2]) * cn[1] + I[1] - clo[1]) * cn[0] + \
                                        I[0] - clo[0]
                                    fo = ((z - lo[2]) * n[1] + y - lo[1]) * n[0] + x - lo[0]
                                    pairs.append((cb, co, fb, fo))
            pairs.sort()
        out.append((slots, [(q[2], q[1], q[0]) for q in rblist], pairs))
    return out


@pytest.mark.parametrize("which", range(3))
def test_maps_match_brute_force(which):
    spec = _tiny_specs()[which]
    hier = Hierarchy(spec, block_seed=7, min_block=4, max_block=8)
    ref = _brute_force(spec, hier)
    for l, (slots, rblist, pairs) in enumerate(ref):
        for b, per in enumerate(slots):
            kind, a, c = hier.ghosts[l][b]
            got = [(int(k), int(x), int(y) if k == SYNC else 0) for k, x, y in zip(kind, a, c)]
            assert got == per
        assert [tuple(map(int, q)) for q in hier.rb[l]] == rblist
        assert [tuple(map(int, p)) for p in hier.restrict[l]] == pairs


def test_kd_split_invariants():
    spec = config_c3(64)
    for seed in (1, 2):
        h = Hierarchy(spec, block_seed=seed)
        for l, lev in enumerate(h.levels):
            assert (lev.bdims >= 16).all() and (lev.bdims <= 48).all()
            assert lev.nowned == spec.npoints(l)   # blocks tile the boxes exactly
    a = Hierarchy(spec, block_seed=1).export()
    b = Hierarchy(spec, block_seed=1).export()
    c = Hierarchy(spec, block_seed=2).export()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_ghost_classes_partition_and_rb_sorted():
    h = Hierarchy(config_c2(16), min_block=4, max_block=12)
    for l in range(h.nlevels):
        lev = h.levels[l]
        for b in range(lev.nblocks):
            kind, a, c = h.ghosts[l][b]
            n = lev.bdims[b]
            assert len(kind) == np.prod(n + 6) - np.prod(n)
            assert set(np.unique(kind)) <= {SYNC, RB}
        rb = h.rb[l]
        key = (rb[:, 2] << 42) | (rb[:, 1] << 21) | rb[:, 0]
        assert (np.diff(key) > 0).all()
    assert len(h.rb[0]) == 0 and len(h.rb[1]) > 0


def test_export_layout():
    h = Hierarchy(config_c2(16), min_block=4, max_block=12)
    e = h.export()
    assert e.dtype == np.dtype("<i8")
    assert list(e[:4]) == [MAGIC, 1, 2, 1]
    nb, no, nrb = h.counts(0)
    assert list(e[4:9]) == [0, nb, no, nrb, 0]


def test_nesting_errors():
    base = dict(origin=(-1.0,) * 3, dx0=2.0 / 16, ncells0=(16,) * 3, periodic=(True,) * 3)
    with pytest.raises(NestingError):   # odd bound
        Hierarchy(HierarchySpec(fine_boxes=[[((8, 8, 8), (17, 24, 24))]], **base), min_block=4)
    with pytest.raises(NestingError):   # outside the domain
        Hierarchy(HierarchySpec(fine_boxes=[[((8, 8, 8), (34, 24, 24))]], **base), min_block=4)
    with pytest.raises(NestingError):   # overlapping boxes
        Hierarchy(HierarchySpec(fine_boxes=[[((8, 8, 8), (16, 16, 16)),
                                             ((14, 14, 14), (24, 24, 24))]], **base),
                  min_block=4)
    with pytest.raises(NestingError):   # level-2 stencil leaves level 1
        Hierarchy(HierarchySpec(fine_boxes=[[((8, 8, 8), (24, 24, 24))],
                                            [((16, 18, 18), (30, 30, 30))]], **base),
                  min_block=4)
    # a level-2 box with enough margin is accepted
    Hierarchy(HierarchySpec(fine_boxes=[[((8, 8, 8), (24, 24, 24))],
                                        [((24, 24, 24), (30, 30, 30))]], **base), min_block=4)


def test_full_cover_box_allowed():
    spec = HierarchySpec((-1.0,) * 3, 2.0 / 8, (8,) * 3, (True,) * 3,
                         [[((0, 0, 0), (15, 15, 15))]])
    h = Hierarchy(spec, min_block=4, max_block=8)
    assert len(h.rb[1]) == 0
    assert len(h.restrict[1]) == 8 ** 3


def test_benchmark_geometry_counts():
    s3 = config_c3(128)
    assert s3.total_points() == 27424754
    assert s3.updates_per_coarse_step() == 542962934
    s5 = config_c5(96)
    assert s5.total_points() == 8581008
    assert [len(s5.boxes(l)) for l in range(7)] == [1, 1, 1, 1, 1, 1, 2]
    b6 = s5.boxes(6)
    assert b6[1][0][0] - b6[0][1][0] == 48
