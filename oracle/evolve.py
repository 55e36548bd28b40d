"""Subcycled RK4 on a block hierarchy (reference driver).

TEST INFRASTRUCTURE ONLY (see the package header).

Implements the algorithm summary of Sec. II step by step:

  advance_level(l):
      rk4_step(l)                       # steps 1/3/5: full RK4 update, keep k1..k4
      if l has a child:
          prolongate(l+1)               # step 2: y_n, k1..k4 of l to l+1's RB points
          advance_level(l+1) at theta0 = 0    # step 3 (+ recursion, step 4)
          advance_level(l+1) at theta0 = 1/2  # step 5 (+ recursion, step 6)
          restrict(l+1 -> l)            # step 7
      fill(l, y, end)                   # RB ghosts of y from dense output at theta0+1/2
      t_l += dt_l

  rk4_step(l):
      y_n <- y; Y <- y_n
      for s = 1..4:
          fill(l, Y, s)                 # SYNC copy, RB ghost = stage value, PHYS frozen
          k_s <- f(Y)  on owned points
          if s < 4: Y <- y_n + c_{s+1} dt_l k_s  on owned points
      y <- y_n + dt_l/6 (((k1 + 2k2) + 2k3) + k4)  on owned points

Prolongation (once per parent step, for five vectors, Sec. II and Fig. 1):
for each RB point q, P[V](q) is the tensor product over dimensions of a copy
(even q_d) or the degree-5 Lagrange midpoint weights (3,-25,150,150,-25,3)/256
on parent points floor(q_d/2)-2 .. floor(q_d/2)+3 (odd q_d), applied along x
first, then y, then z, each sum left to right.  Only parent-owned points are
read.  The RB ghost of stage s at substep theta0 is
    P[y_n] + H * (((w1 P[k1] + w2 P[k2]) + w3 P[k3]) + w4 P[k4])
with H = dt_{l-1} and w from oracle.dense.ghost_weights.

Restriction is injection: y_{l-1}(I) <- y_l(2I) for every restriction pair.

Time steps: dt_l = cfl * dx_l.

Buffer zones (buffer_zones=True; the Carpet scheme of Sec. II and Fig. 1,
the baseline of the paper's cost comparison; the hierarchy carries buffer
points, oracle.hierarchy):

  advance_level(l, theta0):
      if l > 0: prolong the parent's state at t_parent + theta0 H into the
                RB points and the buffer points (one vector)
      rk4_step(l)                       # RB ghosts keep that value at every stage
      if l has a child: advance_level(l+1, 0); advance_level(l+1, 1/2); restrict
      t_l += dt_l

The parent state at t_n + theta0 H is the Lagrange interpolant in time over
the parent's last three states y_{n-1}, y_n, y_{n+1} (nodes -H, 0, H), each
prolonged in space first: theta0 = 0 gives P[y_n]; theta0 = 1/2 gives
((-1/8 P[y_{n-1}] + 3/4 P[y_n]) + 3/8 P[y_{n+1}]).  Before the parent has a
y_{n-1} (its first step) the interpolant is linear over y_n, y_{n+1}:
((0 P[y_n] + 1/2 P[y_n]) + 1/2 P[y_{n+1}]).  Restriction skips buffer points.

Radiative outer boundary (outer_bc="radiative", Z4c on a non-periodic
domain): the physical-boundary ghosts of level 0 are evolved, not frozen.
Each RK4 stage gives them the stage value y_n + c_s dt k_{s-1} like an owned
point and the right-hand side of oracle.radiative; the step ends with
y_{n+1} = y_n + dt/6 (((k1 + 2k2) + 2k3) + k4) there as well.

Uniform time steps (subcycling=False; the comparison runs of Sec. IV.A):
every level steps with the finest level's dt, advance_level takes one child
step per parent step, and the RB ghost of stage s is the parent's stage vector
at the same time, P[y_n] + dt * c_s P[k_{s-1}] (oracle.dense.aligned_weights),
with the parent's step already complete.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import cbuild
from .dense import aligned_weights, ghost_weights_f64
from .hierarchy import PHYS, RB, SYNC, Hierarchy
from .radiative import radiative_rhs

PROLONG_W = tuple(w / 256.0 for w in (3.0, -25.0, 150.0, 150.0, -25.0, 3.0))
RK_C_NEXT = (0.5, 0.5, 1.0)


class _LevelState:
    def __init__(self, hier: Hierarchy, l: int, nvars: int):
        lev = hier.levels[l]
        G = hier.G
        self.G = G
        nb = lev.nblocks
        dims = lev.bdims
        pdims = dims + 2 * G
        psize = np.prod(pdims, axis=1)
        base = np.zeros(nb, dtype=np.int64)
        base[1:] = np.cumsum(psize)[:-1]
        self.base = base
        self.pdims = pdims
        self.total = int(psize.sum())
        self.desc = np.ascontiguousarray(
            np.concatenate([base[:, None], dims], axis=1).astype(np.int64))
        self.nvars = nvars
        z = lambda: np.zeros((nvars, self.total))
        self.y, self.yn, self.Y = z(), z(), z()
        self.k = [z(), z(), z(), z()]
        self.lev = lev
        # ghost slot destinations and sources
        sd, ss, rd, ri, pd = [], [], [], [], []
        for b in range(nb):
            kind, a, c = hier.ghosts[l][b]
            p = lev.ghost_points(b)
            dst = self.flat_local(b, p - lev.blocks[b, 0, :])
            m = kind == SYNC
            sd.append(dst[m]); ss.append(self.flat_offset(a[m], c[m]))
            m = kind == RB
            rd.append(dst[m]); ri.append(a[m])
            m = kind == PHYS
            pd.append(dst[m])
        cat = lambda v: np.ascontiguousarray(np.concatenate(v).astype(np.int64)) if v else \
            np.zeros(0, dtype=np.int64)
        self.sync_dst, self.sync_src = cat(sd), cat(ss)
        self.rb_dst, self.rb_idx = cat(rd), cat(ri)
        self.phys_dst = cat(pd)
        self.phys_vals = np.zeros((nvars, len(self.phys_dst)))
        # canonical order of owned points
        canon = []
        for lo, hi in lev.boxes:
            zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2] + 1), np.arange(lo[1], hi[1] + 1),
                                     np.arange(lo[0], hi[0] + 1), indexing="ij")
            q = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.int64)
            blk, off = lev.owner(q)
            canon.append(self.flat_offset(blk, off))
        self.canon = np.concatenate(canon)
        self.owned_mask = np.zeros(self.total, dtype=bool)
        self.owned_mask[self.canon] = True

    def flat_local(self, b, r):
        """Flat index of block-local coordinates r (owned origin at 0, ghosts negative)."""
        G = self.G
        px, py = self.pdims[b, 0], self.pdims[b, 1]
        return self.base[b] + ((r[:, 2] + G) * py + (r[:, 1] + G)) * px + (r[:, 0] + G)

    def flat_offset(self, blk, off):
        """Flat index of owned points given (owner block, owner-local offset)."""
        blk = np.asarray(blk, dtype=np.int64)
        off = np.asarray(off, dtype=np.int64)
        n = self.lev.bdims[blk]
        x = off % n[:, 0]
        y = (off // n[:, 0]) % n[:, 1]
        z = off // (n[:, 0] * n[:, 1])
        G = self.G
        px, py = self.pdims[blk, 0], self.pdims[blk, 1]
        return self.base[blk] + ((z + G) * py + (y + G)) * px + (x + G)


def time_interp_weights(theta: Fraction, history: bool):
    """Lagrange weights in time at t_n + theta H over the nodes -H, 0, H (three
    states) or 0, H (two states; the first weight is then 0)."""
    th = Fraction(theta)
    if history:
        return (th * (th - 1) / 2, (1 - th) * (1 + th), th * (th + 1) / 2)
    return (Fraction(0), 1 - th, th)


def dense_ghost_value(Py, Pk, w, H):
    """Ghost stage value from the prolonged parent data (Sec. II dense output):
    P[y_n] + H * (((w1 P[k1] + w2 P[k2]) + w3 P[k3]) + w4 P[k4])."""
    return Py + H * (((w[0] * Pk[0] + w[1] * Pk[1]) + w[2] * Pk[2]) + w[3] * Pk[3])


class Prolongation:
    """Gather plan of the prolongation into a list of fine points (default:
    the level's RB list).  index_of, if given, maps parent global indices
    (k, 3) to positions in the arrays passed to apply() (default: the parent
    level's per-block storage)."""

    def __init__(self, hier: Hierarchy, l: int, parent: _LevelState, pts=None,
                 index_of=None, vstride=None):
        rb = hier.rb[l] if pts is None else pts
        plev = hier.levels[l - 1] if hier is not None else None
        self.n = len(rb)
        self.par = np.ascontiguousarray(
            ((rb[:, 0] % 2) | ((rb[:, 1] % 2) << 1) | ((rb[:, 2] % 2) << 2)).astype(np.int64))
        counts = np.ones(self.n, dtype=np.int64)
        for d in range(3):
            counts *= np.where((self.par >> d) & 1, 6, 1)
        self.start = np.zeros(self.n + 1, dtype=np.int64)
        self.start[1:] = np.cumsum(counts)
        self.idx = np.zeros(int(self.start[-1]), dtype=np.int64)
        for cls in range(8):
            sel = np.nonzero(self.par == cls)[0]
            if len(sel) == 0:
                continue
            odd = [(cls >> d) & 1 for d in range(3)]
            offs = [np.arange(-2, 4) if odd[d] else np.arange(0, 1) for d in range(3)]
            base = rb[sel] // 2
            X = base[:, 0][:, None, None, None] + offs[0][None, None, None, :]
            Y = base[:, 1][:, None, None, None] + offs[1][None, None, :, None]
            Z = base[:, 2][:, None, None, None] + offs[2][None, :, None, None]
            X, Y, Z = np.broadcast_arrays(X, Y, Z)       # (n, sz, sy, sx): z-major order
            pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
            if index_of is not None:
                flat = np.asarray(index_of(pts), dtype=np.int64).reshape(len(sel), -1)
            else:
                blk, off = plev.owner(plev.wrap(pts))
                assert (blk >= 0).all()
                flat = parent.flat_offset(blk, off).reshape(len(sel), -1)
            m = flat.shape[1]
            pos = self.start[sel][:, None] + np.arange(m)[None, :]
            self.idx[pos.ravel()] = flat.ravel()
        self.vstride = parent.total if vstride is None else vstride

    def apply(self, V: np.ndarray) -> np.ndarray:
        out = np.empty((V.shape[0], self.n))
        if self.n:
            cbuild.lib().orc_prolong(self.n, cbuild.ptr(self.start), cbuild.ptr(self.par),
                                     cbuild.ptr(self.idx), V.shape[0], self.vstride,
                                     cbuild.ptr(V), cbuild.ptr(out))
        return out


Z4C_DEFAULTS = dict(kappa1=0.02, kappa2=0.0, eta_c=2.0, eta_o=0.25, eta_s=40.0)


class OracleRun:
    """Reference evolution of one member of a hierarchy.

    rhs: "wave" (variables u, Pi) or "z4c" (22 variables, Sec. III.A; see
    oracle/z4c.c).  fd_order: 4, or 8 for eighth-order derivatives
    (oracle/stencil.c, oracle/z4c.c; needs a hierarchy with G >= 4).  ko_order:
    5 (the r = 4 dissipation of Sec. III.C), or 9 (r = 8, with fd_order 8 on
    a hierarchy with G >= 5).  sigma: Kreiss-Oliger strength.  cfl: dt_l = cfl * dx_l.
    z4c: kappa1, kappa2, eta_c, eta_o, eta_s.
    """

    def __init__(self, hier: Hierarchy, rhs: str = "wave", sigma: float = 0.32,
                 cfl: float = 0.25, z4c: dict = None, subcycling: bool = True,
                 buffer_zones: bool = False, fd_order: int = 4, outer_bc: str = "frozen",
                 ko_order: int = 5):
        if rhs not in ("wave", "z4c"):
            raise ValueError(rhs)
        if fd_order not in (4, 8) or (fd_order == 8 and hier.G < 4):
            raise ValueError("fd_order 8 needs G >= 4")
        if ko_order not in (5, 9) or (ko_order == 9 and (fd_order != 8 or hier.G < 5)):
            raise ValueError("ko_order 9 needs fd_order 8 and G >= 5")
        self.fd_order = fd_order
        self.ko_order = ko_order
        if outer_bc not in ("frozen", "radiative"):
            raise ValueError(outer_bc)
        if outer_bc == "radiative" and (rhs != "z4c" or any(hier.spec.periodic)):
            raise ValueError("the radiative boundary needs Z4c on a non-periodic domain")
        self.radiative = outer_bc == "radiative"
        if buffer_zones and (not subcycling or hier.B <= 0):
            raise ValueError("buffer zones need subcycling and a hierarchy with buffer points")
        self.rhs_kind = rhs
        self.hier = hier
        self.spec = hier.spec
        self.nvars = 2 if rhs == "wave" else 22
        z = dict(Z4C_DEFAULTS, **(z4c or {}))
        self.z4c_par = np.array([z["kappa1"], z["kappa2"], z["eta_c"], z["eta_o"], z["eta_s"],
                                 sigma])
        self.sigma = sigma
        self.cfl = cfl
        self.lib = cbuild.lib()
        self.L = hier.nlevels
        self.st = [_LevelState(hier, l, self.nvars) for l in range(self.L)]
        # coordinates of every block's owned point (0,0,0), for position-dependent terms
        self.block_origin = []
        for l in range(self.L):
            lo = hier.levels[l].blocks[:, 0, :].astype(np.float64)
            o = np.array(self.spec.origin)[None, :] + lo * self.spec.dx(l)
            self.block_origin.append(np.ascontiguousarray(o.ravel()))
        self.pro = [None] + [Prolongation(hier, l, self.st[l - 1]) for l in range(1, self.L)]
        self.P = [None] * self.L           # prolonged (y_n, k1..k4) per level
        self.theta0 = [0.0] * self.L
        self.t = [0.0] * self.L
        self.dx = [self.spec.dx(l) for l in range(self.L)]
        self.subcycling = subcycling
        self.buffer_zones = buffer_zones
        if buffer_zones:
            self.bz_pro = [None]
            self.bz_dst = [None]
            for l in range(1, self.L):
                pts = np.concatenate([hier.rb[l], hier.buffer[l]])
                self.bz_pro.append(Prolongation(hier, l, self.st[l - 1], pts))
                blk, off = hier.levels[l].owner(hier.buffer[l])
                self.bz_dst.append(self.st[l].flat_offset(blk, off))
            for st in self.st:
                st.yprev = np.zeros_like(st.y)
                st.nsteps = 0
                st.history = False
        if self.radiative:
            self._init_radiative()
        if subcycling:
            self.dt = [cfl * self.dx[l] for l in range(self.L)]
            self.weights = {(s, th): ghost_weights_f64(s, Fraction(th))
                            for s in range(1, 6) for th in (0.0, 0.5)}
        else:
            self.dt = [cfl * self.dx[self.L - 1]] * self.L
            self.weights = {(s, th): tuple(float(w) for w in aligned_weights(s))
                            for s in range(1, 6) for th in (0.0, 0.5)}

    def _init_radiative(self) -> None:
        """Distinct physical-boundary points of level 0 (the whole ghost shell
        of its box) and the map from the blocks' ghost slots to them."""
        for l in range(1, self.L):
            if len(self.st[l].phys_dst):
                raise ValueError("the radiative boundary applies to level 0 only")
        lev = self.hier.levels[0]
        pts = [lev.ghost_points(b)[self.hier.ghosts[0][b][0] == PHYS] for b in range(lev.nblocks)]
        pts = np.concatenate(pts)
        q = pts + self.hier.G                      # non-negative for the key
        key = (q[:, 2] << 42) | (q[:, 1] << 21) | q[:, 0]
        _, first, inv = np.unique(key, return_index=True, return_inverse=True)
        self.rad_pts = pts[first]
        self.rad_first = first
        self.rad_inv = inv
        self.rad_n = tuple(int(v) + 1 for v in self.spec.ncells0)   # owned points per dimension
        G = self.hier.G
        shell = np.prod([v + 2 * G for v in self.rad_n]) - np.prod(self.rad_n)
        assert len(self.rad_pts) == shell
        self.rad_y = np.zeros((self.nvars, len(self.rad_pts)))
        self.rad_k = [np.zeros_like(self.rad_y) for _ in range(4)]

    def _padded_level0(self, A: np.ndarray, ghosts: np.ndarray) -> np.ndarray:
        G = self.hier.G
        nx, ny, nz = self.rad_n
        out = np.zeros((self.nvars, nz + 2 * G, ny + 2 * G, nx + 2 * G))
        out[:, G:G + nz, G:G + ny, G:G + nx] = A[:, self.st[0].canon].reshape(self.nvars, nz, ny, nx)
        P = self.rad_pts + G
        out[:, P[:, 2], P[:, 1], P[:, 0]] = ghosts
        return out

    def _radiative_step(self) -> None:
        """One RK4 step of level 0 with evolved outer ghosts."""
        st = self.st[0]
        dt = self.dt[0]
        yn = self.rad_y.copy()
        st.yn[:] = st.y
        st.Y[:] = st.yn
        for s in range(1, 5):
            g = yn if s == 1 else yn + (RK_C_NEXT[s - 2] * dt) * self.rad_k[s - 2]
            st.phys_vals = g[:, self.rad_inv]
            self.fill(0, st.Y, s)
            self.rhs(0, st.Y, st.k[s - 1])
            self.rad_k[s - 1] = radiative_rhs(self._padded_level0(st.Y, g), self.hier.G,
                                              self.rad_n, self.dx[0], self.spec.origin,
                                              self.rad_pts)
            if s < 4:
                self.lib.orc_stage(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total,
                                   self.nvars, cbuild.ptr(st.yn), cbuild.ptr(st.k[s - 1]),
                                   cbuild.ptr(st.Y), RK_C_NEXT[s - 1] * dt)
        k1, k2, k3, k4 = st.k
        self.lib.orc_final(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total, self.nvars,
                           cbuild.ptr(st.yn), cbuild.ptr(k1), cbuild.ptr(k2), cbuild.ptr(k3),
                           cbuild.ptr(k4), cbuild.ptr(st.y), dt)
        r1, r2, r3, r4 = self.rad_k
        self.rad_y = yn + (dt / 6.0) * (((r1 + 2.0 * r2) + 2.0 * r3) + r4)
        st.phys_vals = self.rad_y[:, self.rad_inv]

    # -- data ----------------------------------------------------------------
    def set_data(self, l: int, var: int, values) -> None:
        st = self.st[l]
        st.y[var, st.canon] = np.asarray(values, dtype=np.float64)

    def get(self, l: int, var: int, which: str = "y") -> np.ndarray:
        st = self.st[l]
        arr = {"y": st.y, "yn": st.yn, "k1": st.k[0], "k2": st.k[1], "k3": st.k[2],
               "k4": st.k[3]}[which]
        return arr[var, st.canon].copy()

    def set_phys(self, l: int, values: np.ndarray) -> None:
        self.st[l].phys_vals[:] = values
        if self.radiative and l == 0:
            self.rad_y = np.array(values, dtype=np.float64)[:, self.rad_first]

    def phys_coords(self, l: int) -> np.ndarray:
        """x, y, z of the level's PHYS ghost slots, in fill order."""
        lev = self.hier.levels[l]
        pts = []
        for b in range(lev.nblocks):
            kind = self.hier.ghosts[l][b][0]
            p = lev.ghost_points(b)
            pts.append(p[kind == PHYS])
        p = np.concatenate(pts) if pts else np.zeros((0, 3), dtype=np.int64)
        return np.array(self.spec.origin)[None, :] + p * self.spec.dx(l)

    # -- pieces of the algorithm ---------------------------------------------
    def rb_values(self, l: int, stage: int) -> np.ndarray:
        if self.buffer_zones:
            return self.P[l]              # the step's prolonged state, every stage
        Py, Pk1, Pk2, Pk3, Pk4 = self.P[l]
        return dense_ghost_value(Py, (Pk1, Pk2, Pk3, Pk4), self.weights[(stage, self.theta0[l])],
                                 self.dt[l - 1])

    def fill(self, l: int, A: np.ndarray, stage: int) -> None:
        st = self.st[l]
        if len(st.sync_dst):
            self.lib.orc_copy_points(len(st.sync_dst), cbuild.ptr(st.sync_dst),
                                     cbuild.ptr(st.sync_src), self.nvars, st.total,
                                     cbuild.ptr(A))
        if l > 0 and len(st.rb_dst):
            A[:, st.rb_dst] = self.rb_values(l, stage)[:, st.rb_idx]
        if len(st.phys_dst):
            A[:, st.phys_dst] = st.phys_vals

    def rhs(self, l: int, Y: np.ndarray, k: np.ndarray) -> None:
        st = self.st[l]
        if self.rhs_kind == "wave":
            f = (self.lib.orc_wave_rhs8_ko9 if self.ko_order == 9 else
                 self.lib.orc_wave_rhs8 if self.fd_order == 8 else self.lib.orc_wave_rhs)
            f(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total, cbuild.ptr(Y), cbuild.ptr(k),
              self.dx[l], self.sigma)
        else:
            f = (self.lib.orc_z4c_rhs8_ko9 if self.ko_order == 9 else
                 self.lib.orc_z4c_rhs8 if self.fd_order == 8 else self.lib.orc_z4c_rhs)
            f(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total, cbuild.ptr(Y), cbuild.ptr(k),
              self.dx[l], cbuild.ptr(self.z4c_par), cbuild.ptr(self.block_origin[l]), None, None)

    def hamiltonian(self, l: int) -> np.ndarray:
        """Hamiltonian constraint of the current state on owned points (canonical order)."""
        st = self.st[l]
        A = st.y.copy()
        saved = self.P[l]
        if l > 0 and saved is None:
            # before the first step: ghosts from the parent's current state
            z = np.zeros((self.nvars, self.pro[l].n))
            self.P[l] = [self.pro[l].apply(self.st[l - 1].y), z, z, z, z]
        self.fill(l, A, 5)
        self.P[l] = saved
        k = np.zeros_like(A)
        ham = np.zeros(st.total)
        f = self.lib.orc_z4c_rhs8 if self.fd_order == 8 else self.lib.orc_z4c_rhs
        f(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total,
                             cbuild.ptr(A), cbuild.ptr(k), self.dx[l], cbuild.ptr(self.z4c_par),
                             cbuild.ptr(self.block_origin[l]), None, cbuild.ptr(ham))
        return ham[st.canon]

    def rk4_step(self, l: int) -> None:
        if self.radiative and l == 0:
            self._radiative_step()
            return
        st = self.st[l]
        dt = self.dt[l]
        if self.buffer_zones:
            st.yprev[:] = st.yn
            st.history = st.nsteps > 0
            st.nsteps += 1
        st.yn[:] = st.y
        st.Y[:] = st.yn
        for s in range(1, 5):
            self.fill(l, st.Y, s)
            self.rhs(l, st.Y, st.k[s - 1])
            if s < 4:
                self.lib.orc_stage(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total,
                                   self.nvars, cbuild.ptr(st.yn), cbuild.ptr(st.k[s - 1]),
                                   cbuild.ptr(st.Y), RK_C_NEXT[s - 1] * dt)
        k1, k2, k3, k4 = st.k
        self.lib.orc_final(st.lev.nblocks, cbuild.ptr(st.desc), st.G, st.total, self.nvars,
                           cbuild.ptr(st.yn), cbuild.ptr(k1), cbuild.ptr(k2), cbuild.ptr(k3),
                           cbuild.ptr(k4), cbuild.ptr(st.y), dt)

    def prolongate(self, l: int) -> None:
        par = self.st[l - 1]
        pro = self.pro[l]
        self.P[l] = [pro.apply(par.yn)] + [pro.apply(k) for k in par.k]

    def prolongate_buffer(self, l: int, theta0: float) -> None:
        """Buffer-zone scheme: the parent's state at t + theta0 H into the RB
        slots (kept for every stage of the step) and the buffer points."""
        par = self.st[l - 1]
        pro = self.bz_pro[l]
        nrb = len(self.hier.rb[l])
        if theta0 == 0.0:
            V = pro.apply(par.yn)
        else:
            a, b, c = (float(w) for w in time_interp_weights(Fraction(theta0), par.history))
            older = par.yprev if par.history else par.yn
            V = (a * pro.apply(older) + b * pro.apply(par.yn)) + c * pro.apply(par.y)
        self.P[l] = V[:, :nrb]
        st = self.st[l]
        st.y[:, self.bz_dst[l]] = V[:, nrb:]

    def restrict(self, l: int) -> None:
        pairs = self.hier.restrict[l]
        if len(pairs) == 0:
            return
        fine, coarse = self.st[l], self.st[l - 1]
        src = fine.flat_offset(pairs[:, 2], pairs[:, 3])
        dst = coarse.flat_offset(pairs[:, 0], pairs[:, 1])
        coarse.y[:, dst] = fine.y[:, src]

    def advance_level_buffer(self, l: int, theta0: float) -> None:
        if l > 0:
            self.prolongate_buffer(l, theta0)
        self.rk4_step(l)
        if l + 1 < self.L:
            self.advance_level_buffer(l + 1, 0.0)
            self.advance_level_buffer(l + 1, 0.5)
            self.restrict(l + 1)
        self.fill(l, self.st[l].y, 5)
        self.t[l] += self.dt[l]

    def advance_level(self, l: int) -> None:
        if self.buffer_zones:
            self.advance_level_buffer(l, 0.0)
            return
        self.rk4_step(l)
        if l + 1 < self.L:
            self.prolongate(l + 1)
            self.theta0[l + 1] = 0.0
            self.advance_level(l + 1)
            if self.subcycling:
                self.theta0[l + 1] = 0.5
                self.advance_level(l + 1)
            self.restrict(l + 1)
        self.fill(l, self.st[l].y, 5)
        self.t[l] += self.dt[l]

    def advance(self, ncoarse: int = 1) -> None:
        for _ in range(ncoarse):
            self.advance_level(0)
