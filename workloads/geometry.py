"""Refinement geometry of the benchmark configurations.

A hierarchy is described by its coarse grid and by the boxes of every finer
level.  Grids are vertex centred: on level l the index i sits at
x = origin + i * dx0 / 2**l, and level l-1 index I coincides with level l
index 2I (the refinement ratio is 2 in space, as in the paper's algorithm
summary in Sec. II).  Boxes are inclusive index ranges on their own level.

Level 0 is always the whole domain: [0, N0-1] in a periodic dimension (N0
distinct vertices) and [0, N0] in a non-periodic one.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]


@dataclass
class HierarchySpec:
    origin: Tuple[float, float, float]
    dx0: float
    ncells0: Tuple[int, int, int]
    periodic: Tuple[bool, bool, bool]
    fine_boxes: List[List[Box]] = field(default_factory=list)  # levels 1..L-1
    nmembers: int = 1
    name: str = ""

    @property
    def nlevels(self) -> int:
        return 1 + len(self.fine_boxes)

    def level0_box(self) -> Box:
        hi = tuple(n - 1 if p else n for n, p in zip(self.ncells0, self.periodic))
        return ((0, 0, 0), hi)

    def boxes(self, level: int) -> List[Box]:
        return [self.level0_box()] if level == 0 else list(self.fine_boxes[level - 1])

    def dx(self, level: int) -> float:
        return self.dx0 / (1 << level)

    def npoints(self, level: int) -> int:
        tot = 0
        for lo, hi in self.boxes(level):
            n = 1
            for d in range(3):
                n *= hi[d] - lo[d] + 1
            tot += n
        return tot

    def total_points(self) -> int:
        return sum(self.npoints(l) for l in range(self.nlevels))

    def updates_per_coarse_step(self) -> int:
        """Owned points times level steps in one coarse step (one member)."""
        return sum(self.npoints(l) << l for l in range(self.nlevels))

    def flat_boxes(self):
        """(nboxes_per_level for levels 1.., concatenated boxes) as plain lists."""
        counts = [len(b) for b in self.fine_boxes]
        flat = [bx for lev in self.fine_boxes for bx in lev]
        return counts, flat


def single_level(n: int, lo: float = -1.0, hi: float = 1.0, periodic: bool = True,
                 nmembers: int = 1, name: str = "") -> HierarchySpec:
    dx0 = (hi - lo) / n
    return HierarchySpec((lo, lo, lo), dx0, (n, n, n), (periodic,) * 3, [], nmembers, name)


def two_level_cube(nc: int, flo: int, fhi: int, name: str = "") -> HierarchySpec:
    """Periodic [-1,1]^3 with nc cells and one fine cube [flo, fhi]^3 (fine indices)."""
    spec = single_level(nc, name=name)
    spec.fine_boxes = [[((flo,) * 3, (fhi,) * 3)]]
    return spec


def _round_half_even(x: float) -> int:
    return int(round(x))  # Python's round() is round-half-to-even


def tower_family(n0: int, nb: int, L: float, nt: int, c: float, nlev: int,
                 origin: Sequence[float], periodic: bool, name: str = "") -> HierarchySpec:
    """Two nested towers of refinement centred at (-c,0,0) and (+c,0,0).

    The family is laid out at the base resolution nb and then scaled by
    f = n0/nb, so refinement boundaries sit at the same physical places for
    every member.  On each level a tower is a cube of nt cells (at the base
    resolution) centred on the even vertex nearest the centre; the two towers
    merge into their bounding box when the gap between them is below
    48*nb/128 cells, which reproduces a puncture-like layout merged on the
    coarse levels and split on the fine ones.
    """
    assert n0 % nb == 0
    f = n0 // nb
    dx0b = 2.0 * L / nb
    levels: List[List[Box]] = []
    for l in range(1, nlev):
        dxl = dx0b / (1 << l)
        towers = []
        for sgn in (-1.0, 1.0):
            xc = (sgn * c, 0.0, 0.0)
            C = [2 * _round_half_even((xc[d] - origin[d]) / (2.0 * dxl)) for d in range(3)]
            lo = tuple(C[d] - nt // 2 for d in range(3))
            hi = tuple(C[d] + nt // 2 for d in range(3))
            towers.append((lo, hi))
        (lom, him), (lop, hip) = towers
        if lop[0] - him[0] < 48 * nb // 128:
            lo = tuple(min(lom[d], lop[d]) for d in range(3))
            hi = tuple(max(him[d], hip[d]) for d in range(3))
            boxes = [(lo, hi)]
        else:
            boxes = towers
        boxes = [(tuple(f * v for v in lo), tuple(f * v for v in hi)) for lo, hi in boxes]
        levels.append(boxes)
    return HierarchySpec(tuple(origin), 2.0 * L / n0, (n0,) * 3, (periodic,) * 3, levels, 1, name)


# ---------------------------------------------------------------------------
# The benchmark configurations.

def config_c1(n: int = 32) -> HierarchySpec:
    """Scalar wave, one periodic level of n^3 cells on [-1,1]^3."""
    return single_level(n, name=f"wave-1level-{n}^3-periodic")


def ensemble_c1(nmembers: int, n: int = 32) -> HierarchySpec:
    return single_level(n, nmembers=nmembers, name=f"wave-1level-{n}^3-x{nmembers}")


def config_c2(nc: int = 64) -> HierarchySpec:
    """Scalar wave, coarse nc^3 periodic on [-1,1]^3 plus fine box [-1/2,1/2]^3."""
    return two_level_cube(nc, nc // 2, 3 * nc // 2, name=f"wave-2level-{nc}^3")


def config_c3(n0: int = 128, nlev: int = 7) -> HierarchySpec:
    """Scalar wave, 7 levels, two towers at x = -0.3, +0.3 merging on coarse levels."""
    return tower_family(n0, 64, 1.0, 64, 0.3, nlev, (-1.0, -1.0, -1.0), True,
                        name=f"wave-{nlev}level-towers-{n0}^3")


def config_c5(n0: int = 96, nlev: int = 7) -> HierarchySpec:
    """Z4c puncture layout: [-128,128]^3, towers of 96 cells at x = -3, +3.

    The y and z origins are shifted by half a finest-level spacing so that no
    vertex of any level falls on a puncture.
    """
    dfine = (256.0 / n0) / (1 << (nlev - 1))
    origin = (-128.0, -128.0 + dfine / 2, -128.0 + dfine / 2)
    return tower_family(n0, 96, 128.0, 96, 3.0, nlev, origin, False,
                        name=f"z4c-{nlev}level-towers-{n0}^3")


def config_z4c_small(n0: int = 24, nlev: int = 3, half: float = 16.0, nt: int = 16) -> HierarchySpec:
    """A small puncture layout for tests: [-half, half]^3, towers at x = -3, +3."""
    dfine = (2.0 * half / n0) / (1 << (nlev - 1))
    origin = (-half, -half + dfine / 2, -half + dfine / 2)
    return tower_family(n0, n0, half, nt, 3.0, nlev, origin, False,
                        name=f"z4c-{nlev}level-towers-{n0}^3")


def config_e1(n0: int = 375, half: float = 6.0, radii=(4.0, 1.0)) -> HierarchySpec:
    """The paper's scalar-wave test layout (Sec. IV.A): a periodic cube
    [-half, half]^3 of n0 cells and two refined levels whose boxes cover
    [-r, r]^3 for r = 4 and 1, each snapped outward to even indices of its
    parent.  n0 = 375, 450, 540 give the coarse spacings 0.032, 0.032/1.2 and
    0.032/1.44 on [-6, 6]^3."""
    dx0 = 2.0 * half / n0
    levels: List[List[Box]] = []
    for l, r in enumerate(radii, start=1):
        dxl = dx0 / (1 << l)
        a = (half - r) / dxl            # index of x = -r on level l
        b = (half + r) / dxl            # index of x = +r
        lo = 2 * math.floor(round(a, 9) / 2)
        hi = 2 * math.ceil(round(b, 9) / 2)
        levels.append([((lo,) * 3, (hi,) * 3)])
    return HierarchySpec((-half,) * 3, dx0, (n0,) * 3, (True,) * 3, levels, 1,
                         name=f"wave-e1-{n0}^3")


def grown_for_buffer_zones(spec: HierarchySpec, grow: int) -> HierarchySpec:
    """The same layout with every fine box grown by `grow` points (even) of its
    own level on each side, clipped to the domain, so that a buffer-zone run
    whose buffers are at most `grow` wide keeps at least the original boxes as
    its valid region."""
    if grow % 2:
        raise ValueError("grow must be even (box bounds stay even)")
    levels: List[List[Box]] = []
    for l, boxes in enumerate(spec.fine_boxes, start=1):
        N = [n << l for n in spec.ncells0]
        out = []
        for lo, hi in boxes:
            nlo, nhi = [], []
            for d in range(3):
                top = N[d] - 1 if spec.periodic[d] else N[d]
                if spec.periodic[d] and lo[d] == 0 and hi[d] == N[d] - 1:
                    nlo.append(lo[d]); nhi.append(hi[d])
                    continue
                nlo.append(max(lo[d] - grow, 0))
                h = min(hi[d] + grow, top)
                nhi.append(h - (h % 2))
            out.append((tuple(nlo), tuple(nhi)))
        levels.append(out)
    return HierarchySpec(spec.origin, spec.dx0, spec.ncells0, spec.periodic, levels,
                         spec.nmembers, spec.name + f"-grown{grow}")
