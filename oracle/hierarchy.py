"""Block hierarchy and index maps (reference).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper evolves each refinement level on blocks ("inter-process
boundaries", Sec. I and Sec. V) and fills the ghost zones of a block either
from a neighbouring block of the same level or, at a refinement boundary,
from the coarser level (Sec. II).  The ghost width at refinement boundaries
equals the width at block boundaries.  This module states every map that
follows from that structure:

* block split: each level box is cut recursively along its longest side
  (ties: x, then y, then z) at a split point drawn from one SplitMix64 stream
  per level (seed = block_seed + level); the left part gets between
  min_block and n - min_block points and is split first.
* ghost classes of block b: the points of [lo-G, hi+G]^3 minus [lo, hi]^3,
  visited z-major, then y, x fastest; periodic dimensions wrap; a point
  outside a non-periodic domain is PHYS; a point owned by a block of the same
  level is SYNC(owner, owner-local offset); otherwise it is RB, a
  refinement-boundary point filled from the parent level.
* RB list: the distinct RB points of a level sorted by (z, y, x), each with
  its parent base index floor(q/2) and odd-index parity bits.
* restriction pairs: every parent-owned point I whose image 2I is owned on
  the level, sorted by (parent block, parent offset).
* nesting: fine boxes have even bounds (or span a whole periodic dimension),
  lie in the domain, and every parent point of every RB point's
  prolongation stencil is parent-owned.
* canonical export: one int64 word stream holding all of the above.

Buffer zones (the Carpet scheme the paper compares against, Sec. II and
Fig. 1), when `buffer` = B > 0: the buffer points of a fine level are its
owned points within Chebyshev distance B of one of its RB points (periodic
dimensions measured across the wrap).  They are evolved like any owned point
but refilled from the parent with the RB points before every fine step, and
they are not restricted.  Every parent point of the prolongation stencil of
an RB or buffer point must be parent-owned and, on a parent that has buffer
points itself, not one of them.

Pinned by tests/test_oracle_maps.py: brute-force pure-Python classification
on tiny hierarchies, tiling and size invariants, sortedness/uniqueness, and
the SplitMix64 published outputs.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .splitmix import SplitMix64

SYNC, RB, PHYS = 0, 1, 2
MAGIC = 0x53554243  # "SUBC"


class NestingError(ValueError):
    pass


def kd_split(lo, hi, rng, min_block, max_block, out):
    n = [hi[d] - lo[d] + 1 for d in range(3)]
    if max(n) <= max_block:
        out.append((tuple(lo), tuple(hi)))
        return
    d = max(range(3), key=lambda i: (n[i], -i))  # longest, ties -> lowest axis
    s = min_block + rng.next() % (n[d] - 2 * min_block + 1)
    lhi = list(hi); lhi[d] = lo[d] + s - 1
    rlo = list(lo); rlo[d] = lo[d] + s
    kd_split(lo, lhi, rng, min_block, max_block, out)
    kd_split(rlo, hi, rng, min_block, max_block, out)


class Level:
    def __init__(self, spec, level: int, block_seed: int, min_block: int, max_block: int,
                 G: int):
        self.level = level
        self.G = G
        self.boxes = spec.boxes(level)
        self.periodic = tuple(bool(p) for p in spec.periodic)
        self.N = tuple(n << level for n in spec.ncells0)
        rng = SplitMix64(block_seed + level)
        blocks = []
        self.block_box = []
        for ib, (lo, hi) in enumerate(self.boxes):
            for d in range(3):
                if hi[d] - lo[d] + 1 < min_block:
                    raise NestingError(f"level {level} box side shorter than min_block")
            sub = []
            kd_split(list(lo), list(hi), rng, min_block, max_block, sub)
            blocks += sub
            self.block_box += [ib] * len(sub)
        self.blocks = np.array(blocks, dtype=np.int64).reshape(-1, 2, 3)
        self.nblocks = len(blocks)
        self.bdims = self.blocks[:, 1, :] - self.blocks[:, 0, :] + 1  # (nb,3) x,y,z
        self.nowned = int(np.prod(self.bdims, axis=1).sum())
        # per-box dense block-id lookup
        self._boxlut = []
        for ib, (lo, hi) in enumerate(self.boxes):
            n = [hi[d] - lo[d] + 1 for d in range(3)]
            lut = np.full((n[2], n[1], n[0]), -1, dtype=np.int32)
            for b in range(self.nblocks):
                if self.block_box[b] != ib:
                    continue
                blo, bhi = self.blocks[b]
                lut[blo[2] - lo[2]:bhi[2] - lo[2] + 1, blo[1] - lo[1]:bhi[1] - lo[1] + 1,
                    blo[0] - lo[0]:bhi[0] - lo[0] + 1] = b
            if (lut < 0).any():
                raise AssertionError("blocks do not tile the level box")
            self._boxlut.append(lut)

    # -- point queries -----------------------------------------------------
    def wrap(self, p: np.ndarray) -> np.ndarray:
        q = p.copy()
        for d in range(3):
            if self.periodic[d]:
                q[:, d] = np.mod(q[:, d], self.N[d])
        return q

    def outside_domain(self, q: np.ndarray) -> np.ndarray:
        m = np.zeros(len(q), dtype=bool)
        for d in range(3):
            if not self.periodic[d]:
                m |= (q[:, d] < 0) | (q[:, d] > self.N[d])
        return m

    def owner(self, q: np.ndarray):
        """Owner block and owner-local offset of (wrapped) points; -1 if not owned."""
        blk = np.full(len(q), -1, dtype=np.int64)
        for ib, (lo, hi) in enumerate(self.boxes):
            inside = np.ones(len(q), dtype=bool)
            for d in range(3):
                inside &= (q[:, d] >= lo[d]) & (q[:, d] <= hi[d])
            if inside.any():
                l = q[inside] - np.array(lo)
                blk[inside] = self._boxlut[ib][l[:, 2], l[:, 1], l[:, 0]]
        off = np.full(len(q), -1, dtype=np.int64)
        ok = blk >= 0
        if ok.any():
            b = blk[ok]
            lo = self.blocks[b, 0, :]
            n = self.bdims[b]
            r = q[ok] - lo
            off[ok] = (r[:, 2] * n[:, 1] + r[:, 1]) * n[:, 0] + r[:, 0]
        return blk, off

    def ghost_points(self, b: int) -> np.ndarray:
        """Ghost points of block b in visiting order (z-major, y, x fastest)."""
        G = self.G
        lo, hi = self.blocks[b]
        z, y, x = np.meshgrid(np.arange(lo[2] - G, hi[2] + G + 1),
                              np.arange(lo[1] - G, hi[1] + G + 1),
                              np.arange(lo[0] - G, hi[0] + G + 1), indexing="ij")
        p = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.int64)
        interior = np.ones(len(p), dtype=bool)
        for d in range(3):
            interior &= (p[:, d] >= lo[d]) & (p[:, d] <= hi[d])
        return p[~interior]


class Hierarchy:
    """All levels with their maps.  `spec` is a workloads.HierarchySpec."""

    def __init__(self, spec, block_seed: int = 1, min_block: int = 16, max_block: int = 48,
                 G: int = 3, buffer: int = 0):
        if max_block < 2 * min_block - 1:
            raise ValueError("max_block must be at least 2*min_block-1")
        if buffer < 0:
            raise ValueError("buffer must be >= 0")
        self.spec = spec
        self.G = G
        self.B = buffer
        self.nlevels = spec.nlevels
        self.levels: List[Level] = []
        self._check_boxes()
        for l in range(self.nlevels):
            self.levels.append(Level(spec, l, block_seed, min_block, max_block, G))
        self.ghosts = []      # per level: list per block of (kind, a, b) arrays
        self.rb = []          # per level: (nrb,3) int64 sorted by (z,y,x)
        self.restrict = []    # per level: (npairs,4) int64 (empty for level 0)
        for l in range(self.nlevels):
            self._classify(l)
        empty = np.zeros((0, 3), dtype=np.int64)
        self.buffer = [empty] + [self._buffer_points(l) if buffer else empty
                                 for l in range(1, self.nlevels)]
        for l in range(1, self.nlevels):
            self._check_stencils(l)
        self.restrict.append(np.zeros((0, 4), dtype=np.int64))
        for l in range(1, self.nlevels):
            self.restrict.append(self._restriction_pairs(l))

    # -- nesting ----------------------------------------------------------
    def _check_boxes(self):
        spec = self.spec
        for l in range(1, spec.nlevels):
            N = [n << l for n in spec.ncells0]
            boxes = spec.boxes(l)
            for lo, hi in boxes:
                for d in range(3):
                    full = spec.periodic[d] and lo[d] == 0 and hi[d] == N[d] - 1
                    if not full and (lo[d] % 2 or hi[d] % 2):
                        raise NestingError(f"level {l}: box bounds must be even")
                    top = N[d] - 1 if spec.periodic[d] else N[d]
                    if lo[d] < 0 or hi[d] > top or lo[d] > hi[d]:
                        raise NestingError(f"level {l}: box outside the domain")
            for i in range(len(boxes)):
                for j in range(i + 1, len(boxes)):
                    a, b = boxes[i], boxes[j]
                    if all(a[0][d] <= b[1][d] and b[0][d] <= a[1][d] for d in range(3)):
                        raise NestingError(f"level {l}: boxes overlap")

    def _classify(self, l: int):
        lev = self.levels[l]
        per_block = []
        rbpts = []
        for b in range(lev.nblocks):
            p = lev.ghost_points(b)
            q = lev.wrap(p)
            kind = np.full(len(q), RB, dtype=np.int64)
            a = np.zeros(len(q), dtype=np.int64)
            c = np.zeros(len(q), dtype=np.int64)
            phys = lev.outside_domain(q)
            kind[phys] = PHYS
            a[phys] = -1
            blk, off = lev.owner(np.where(phys[:, None], 0, q))
            sync = (~phys) & (blk >= 0)
            kind[sync] = SYNC
            a[sync] = blk[sync]
            c[sync] = off[sync]
            rbm = kind == RB
            if l == 0 and rbm.any():
                raise NestingError("level 0 has refinement-boundary ghosts")
            per_block.append([kind, a, c, q])
            rbpts.append(q[rbm])
        allrb = np.concatenate(rbpts) if rbpts else np.zeros((0, 3), dtype=np.int64)
        key = self._key(allrb)
        ukey, first = np.unique(key, return_index=True)
        rb = allrb[first]
        for kind, a, c, q in per_block:
            rbm = kind == RB
            a[rbm] = np.searchsorted(ukey, self._key(q[rbm]))
        self.ghosts.append([(k, a, c) for k, a, c, _ in per_block])
        self.rb.append(rb)

    @staticmethod
    def _key(q):
        q = np.asarray(q, dtype=np.int64)
        return (q[:, 2] << 42) | (q[:, 1] << 21) | q[:, 0]

    @staticmethod
    def stencil_1d(qd: int):
        """Parent indices of the prolongation stencil along one dimension."""
        if qd % 2 == 0:
            return [qd // 2]
        base = qd // 2
        return list(range(base - 2, base + 4))

    def _buffer_points(self, l: int) -> np.ndarray:
        """Owned points within Chebyshev distance B of an RB point, sorted by (z, y, x)."""
        lev = self.levels[l]
        B = self.B
        rbkeys = self._key(self.rb[l])
        out = []
        for lo, hi in lev.boxes:
            lo = np.array(lo, dtype=np.int64)
            hi = np.array(hi, dtype=np.int64)
            n = hi - lo + 1 + 2 * B
            zz, yy, xx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]),
                                     indexing="ij")
            w = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1) + (lo - B)
            q = lev.wrap(w)
            isrb = np.isin(self._key(q), rbkeys) & ~lev.outside_domain(q)
            m = isrb.reshape(n[2], n[1], n[0])
            # Chebyshev dilation by B: one pass of shifted ORs per axis
            for ax in range(3):
                acc = m.copy()
                for sft in range(1, B + 1):
                    lo_sl = [slice(None)] * 3
                    hi_sl = [slice(None)] * 3
                    lo_sl[ax] = slice(sft, None)
                    hi_sl[ax] = slice(None, -sft)
                    acc[tuple(lo_sl)] |= m[tuple(hi_sl)]
                    acc[tuple(hi_sl)] |= m[tuple(lo_sl)]
                m = acc
            inner = m[B:n[2] - B, B:n[1] - B, B:n[0] - B]
            z, y, x = np.nonzero(inner)
            out.append(np.stack([x, y, z], axis=1) + lo)
        pts = np.concatenate(out).astype(np.int64) if out else np.zeros((0, 3), dtype=np.int64)
        order = np.argsort(self._key(pts), kind="stable")
        return pts[order]

    def _check_stencils(self, l: int):
        if self.B:
            self._check_stencils_buffer(l)
            return
        parent = self.levels[l - 1]
        rb = self.rb[l]
        if len(rb) == 0:
            return
        base = rb // 2
        odd = (rb % 2) == 1
        smin = np.where(odd, base - 2, base)
        smax = np.where(odd, base + 3, base)
        # fast path: the stencil's bounding box lies in one parent box
        covered = np.zeros(len(rb), dtype=bool)
        for lo, hi in parent.boxes:
            ok = np.ones(len(rb), dtype=bool)
            for d in range(3):
                full = parent.periodic[d] and lo[d] == 0 and hi[d] == parent.N[d] - 1
                if not full:
                    ok &= (smin[:, d] >= lo[d]) & (smax[:, d] <= hi[d])
            covered |= ok
        rest = np.nonzero(~covered)[0]
        if len(rest) == 0:
            return
        # general path: every stencil point must be owned by some parent block
        for ox in range(-2, 4):
            for oy in range(-2, 4):
                for oz in range(-2, 4):
                    off = np.array([ox, oy, oz])
                    r = rest[np.all(odd[rest] | (off == 0), axis=1)]
                    if len(r) == 0:
                        continue
                    pts = parent.wrap(base[r] + np.where(odd[r], off, 0))
                    if parent.outside_domain(pts).any():
                        raise NestingError(
                            f"level {l}: prolongation stencil leaves the domain")
                    blk, _ = parent.owner(pts)
                    if (blk < 0).any():
                        raise NestingError(
                            f"level {l}: prolongation stencil leaves the parent level")

    def _check_stencils_buffer(self, l: int):
        """Every stencil point of every RB and buffer point is parent-owned and
        not a parent buffer point."""
        parent = self.levels[l - 1]
        pts = np.concatenate([self.rb[l], self.buffer[l]])
        if len(pts) == 0:
            return
        pbuf = self._key(self.buffer[l - 1])
        base = pts // 2
        odd = (pts % 2) == 1
        for ox in range(-2, 4):
            for oy in range(-2, 4):
                for oz in range(-2, 4):
                    off = np.array([ox, oy, oz])
                    r = np.nonzero(np.all(odd | (off == 0), axis=1))[0]
                    if len(r) == 0:
                        continue
                    q = parent.wrap(base[r] + np.where(odd[r], off, 0))
                    if parent.outside_domain(q).any():
                        raise NestingError(f"level {l}: prolongation stencil leaves the domain")
                    blk, _ = parent.owner(q)
                    if (blk < 0).any():
                        raise NestingError(
                            f"level {l}: prolongation stencil leaves the parent level")
                    if len(pbuf) and np.isin(self._key(q), pbuf).any():
                        raise NestingError(
                            f"level {l}: prolongation stencil reads parent buffer points")

    def _restriction_pairs(self, l: int):
        fine = self.levels[l]
        parent = self.levels[l - 1]
        out = []
        for b in range(fine.nblocks):
            lo, hi = fine.blocks[b]
            ev = [np.arange(lo[d] + (lo[d] % 2), hi[d] + 1, 2) for d in range(3)]
            if any(len(e) == 0 for e in ev):
                continue
            z, y, x = np.meshgrid(ev[2], ev[1], ev[0], indexing="ij")
            q = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
            if len(self.buffer[l]):
                q = q[~np.isin(self._key(q), self._key(self.buffer[l]))]
                if len(q) == 0:
                    continue
            r = q - lo
            n = fine.bdims[b]
            foff = (r[:, 2] * n[1] + r[:, 1]) * n[0] + r[:, 0]
            cb, coff = parent.owner(parent.wrap(q // 2))
            if (cb < 0).any():
                raise NestingError(f"level {l}: restriction target not parent-owned")
            out.append(np.stack([cb, coff, np.full(len(q), b), foff], axis=1))
        if not out:
            return np.zeros((0, 4), dtype=np.int64)
        pairs = np.concatenate(out).astype(np.int64)
        order = np.lexsort((pairs[:, 1], pairs[:, 0]))
        return pairs[order]

    # -- queries -------------------------------------------------------------
    def counts(self, l: int):
        lev = self.levels[l]
        return lev.nblocks, lev.nowned, len(self.rb[l])

    def export(self) -> np.ndarray:
        """Canonical little-endian int64 word stream of all maps."""
        version = 2 if self.B else 1
        words = [np.array([MAGIC, version, self.nlevels, self.spec.nmembers], dtype=np.int64)]
        for l in range(self.nlevels):
            lev = self.levels[l]
            rb = self.rb[l]
            rs = self.restrict[l]
            words.append(np.array([l, lev.nblocks, lev.nowned, len(rb), len(rs)],
                                  dtype=np.int64))
            words.append(lev.blocks.reshape(-1, 6).astype(np.int64))
            for kind, a, c in self.ghosts[l]:
                w = np.stack([kind, a, np.where(kind == SYNC, c, 0)], axis=1)
                words.append(w.astype(np.int64))
            if len(rb):
                par = (rb[:, 0] % 2) | ((rb[:, 1] % 2) << 1) | ((rb[:, 2] % 2) << 2)
                words.append(np.concatenate([rb, rb // 2, par[:, None]], axis=1))
            if len(rs):
                words.append(rs)
            if self.B:
                bz = self.buffer[l]
                words.append(np.array([len(bz)], dtype=np.int64))
                if len(bz):
                    par = (bz[:, 0] % 2) | ((bz[:, 1] % 2) << 1) | ((bz[:, 2] % 2) << 2)
                    words.append(np.concatenate([bz, bz // 2, par[:, None]], axis=1))
        return np.concatenate([w.ravel() for w in words]).astype("<i8")
