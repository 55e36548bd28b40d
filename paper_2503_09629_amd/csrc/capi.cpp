// C-ABI of libsubcyc: context, hierarchy, arena, scheduler, readers.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "runtime.hpp"
#include "z4c.hpp"

using namespace sc;

namespace {
// A roctx range over a host scope (a level step, a stage, a prolongation),
// visible in rocprofv3 --marker-trace; without a profiler the calls do nothing.
// In graph mode the ranges mark the capture, not the replays.
struct Range {
  template <typename... A>
  explicit Range(const char* fmt, A... args) {
    char buf[96];
    std::snprintf(buf, sizeof buf, fmt, args...);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
}  // namespace

namespace {

thread_local std::string g_create_error;

int fail(sc_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, SC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// ---------------------------------------------------------------------------
// Dense-output weights (Sec. II) in exact rational arithmetic.
struct Rat {
  int64_t n, d;
  Rat(int64_t a = 0, int64_t b = 1) : n(a), d(b) { norm(); }
  void norm() {
    if (d < 0) n = -n, d = -d;
    int64_t g = std::gcd(n < 0 ? -n : n, d);
    if (g > 1) n /= g, d /= g;
  }
  Rat operator+(Rat o) const { return Rat(n * o.d + o.n * d, d * o.d); }
  Rat operator-(Rat o) const { return Rat(n * o.d - o.n * d, d * o.d); }
  Rat operator*(Rat o) const { return Rat(n * o.n, d * o.d); }
  double f() const { return (double)n / (double)d; }
};

// b_i(theta) of the RK4 dense output and its theta-derivatives (order m).
void dense_b(Rat th, int m, Rat out[4]) {
  Rat t2 = th * th, t3 = t2 * th;
  switch (m) {
    case 0:
      out[0] = th - Rat(3, 2) * t2 + Rat(2, 3) * t3;
      out[1] = out[2] = t2 - Rat(2, 3) * t3;
      out[3] = Rat(-1, 2) * t2 + Rat(2, 3) * t3;
      break;
    case 1:
      out[0] = Rat(1) - Rat(3) * th + Rat(2) * t2;
      out[1] = out[2] = Rat(2) * th - Rat(2) * t2;
      out[3] = Rat(-1) * th + Rat(2) * t2;
      break;
    case 2:
      out[0] = Rat(-3) + Rat(4) * th;
      out[1] = out[2] = Rat(2) - Rat(4) * th;
      out[3] = Rat(-1) + Rat(4) * th;
      break;
    default:
      out[0] = Rat(4);
      out[1] = out[2] = Rat(-4);
      out[3] = Rat(4);
  }
}

// Ghost value = y_n + H * sum_i w_i k_i for fine stage `fill` (1..4, Taylor
// forms of Y1..Y4 with fine step h = H/2 and f_y y'' = 4 (k3 - k2) / H^2)
// or the end value (5, dense output at theta0 + 1/2).
// Uniform time steps: the stage value of the parent at the fine stage's own
// time, y_n + c_s H k_{s-1} (fills 1-4), and y_{n+1} (fill 5), as weights of
// H k_i.
void aligned_weights(int fill, Rat r[4]) {
  static const Rat c[4] = {Rat(0), Rat(1, 2), Rat(1, 2), Rat(1)};
  for (int i = 0; i < 4; ++i) r[i] = Rat(0);
  if (fill == 5) {
    r[0] = Rat(1, 6), r[1] = Rat(1, 3), r[2] = Rat(1, 3), r[3] = Rat(1, 6);
  } else if (fill >= 2) {
    r[fill - 2] = c[fill - 1];
  }
}

void ghost_weights(int fill, Rat th0, Rat r[4]) {
  if (fill == 5) {
    dense_b(th0 + Rat(1, 2), 0, r);
  } else {
    Rat b0[4], b1[4], b2[4], b3[4];
    dense_b(th0, 0, b0);
    dense_b(th0, 1, b1);
    dense_b(th0, 2, b2);
    dense_b(th0, 3, b3);
    const Rat fyy[4] = {Rat(0), Rat(-4), Rat(4), Rat(0)};
    // coefficients of h y', h^2 y'', h^3 y''', h^3 f_y y'' in Eqs. Y1-Y4
    Rat c1, c2, c3, cf;
    if (fill == 2) c1 = Rat(1, 2);
    if (fill == 3) c1 = Rat(1, 2), c2 = Rat(1, 4), c3 = Rat(1, 16), cf = Rat(-1, 16);
    if (fill == 4) c1 = Rat(1), c2 = Rat(1, 2), c3 = Rat(1, 8), cf = Rat(1, 8);
    const Rat h(1, 2), h2 = h * h, h3 = h2 * h;
    for (int i = 0; i < 4; ++i)
      r[i] = b0[i] + c1 * h * b1[i] + c2 * h2 * b2[i] + c3 * h3 * b3[i] + cf * h3 * fyy[i];
  }
}

// ---------------------------------------------------------------------------
// Device layout.

inline int64_t floordiv2(int64_t a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

void split_even(int64_t n, int64_t maxlen, std::vector<std::pair<int, int>>* out) {
  out->clear();
  const int64_t parts = (n + maxlen - 1) / maxlen;
  int64_t start = 0;
  for (int64_t p = 0; p < parts; ++p) {
    const int64_t len = n / parts + (p < n % parts ? 1 : 0);
    out->push_back({(int)start, (int)len});
    start += len;
  }
}

// Largest tile height for tiles at most nxm points wide: at most
// kStageSlots owned points per thread, an LDS window of at most kWinCap points
// and at most kRingSlots ring points per thread.
int tile_ty_cap(int nxm, int slots, int threads, int R) {
  int t = threads * slots / nxm;
  t = std::min(t, stage_win_cap(threads) / (nxm + 2 * R) - 2 * R);
  t = std::min(t, (threads * stage_ring_slots(threads) - 2 * R * (nxm + 2 * R)) / (2 * R));
  return std::max(t, 1);
}

// Widest tile whose one-row window and ring fit the family's LDS window and
// ring slots (78 for radius 3; 55 for radius 4; 40 for radius 5).
int tile_tx_cap(int threads, int R) {
  const int by_ring = threads * stage_ring_slots(threads) / (2 * R) - 2 * R - 1;
  const int by_win = stage_win_cap(threads) / (1 + 2 * R) - 2 * R;
  return std::max(1, std::min(kTileMaxX, std::min(by_ring, by_win)));
}

// stencil kernel variants: (threads, points per thread, planes of loads in flight)
bool stage_variant_ok(int slots, int depth, int threads = 256) {
  if (threads == 512) return slots == 2 && (depth == 1 || depth == 2);
  if (threads != 256) return false;
  return (slots == 2 && (depth == 1 || depth == 2)) || (slots == 1 && depth == 2);
}

bool tile_fits(int nx, int ny, int slots, int threads, int R) {
  return nx >= 1 && ny >= 1 && nx <= kTileMaxX && nx * ny <= threads * slots &&
         (nx + 2 * R) * (ny + 2 * R) <= stage_win_cap(threads) &&
         2 * R * (nx + 2 * R) + 2 * R * ny <= threads * stage_ring_slots(threads);
}

// Grid of the batched Z4c launches: one workgroup per tile, rounded up to
// whole rounds of the 8 XCDs (the kernels give each XCD a contiguous run of
// the tile list; the spare workgroups exit at once).  No persistent second
// pass: its tiles would all fall to the first XCDs' workgroups.
int z4c_grid(int ntiles) { return (ntiles + 7) / 8 * 8; }

void tile_region(int box, const int64_t o[3], const int64_t n[3], const TileShape& s,
                 std::vector<TileDev>* out) {
  std::vector<std::pair<int, int>> sx, sy, sz;
  split_even(n[0], std::min(s.tx, tile_tx_cap(s.threads, s.radius)), &sx);
  int nxm = 1;
  for (auto& x : sx) nxm = std::max(nxm, x.second);
  split_even(n[1], std::min(s.ty, tile_ty_cap(nxm, s.slots, s.threads, s.radius)), &sy);
  split_even(n[2], s.tz, &sz);
  // order: y rows of tiles, then z chunks, then x, so that a contiguous run of
  // the table (one XCD's share) is a slab holding whole z stacks: the halo
  // planes shared by neighbouring chunks are then read from one L2
  for (auto& y : sy)
    for (size_t iz = 0; iz < sz.size(); ++iz)
      for (auto& x : sx) {
        TileDev t;
        t.box = box;
        t.x0 = (int)o[0] + x.first;
        t.y0 = (int)o[1] + y.first;
        t.z0 = (int)o[2] + sz[iz].first;
        t.nx = x.second;
        t.ny = y.second;
        t.nz = sz[iz].second;
        // neighbouring z chunks march towards (and away from) their common
        // face at the same time, so its halo planes are read while cached
        t.dir = (int32_t)(iz & 1);
        out->push_back(t);
      }
}

// Columns of the Z4c derivative pass over a region of box `box`: x-y tiles
// of at most kDerTx x kDerTy points, z chunks of at most tz planes.
void der_region(int box, const int64_t o[3], const int64_t n[3], int tz,
                std::vector<TileDev>* out) {
  std::vector<std::pair<int, int>> sx, sy, sz;
  split_even(n[0], kDerTx, &sx);
  split_even(n[1], kDerTy, &sy);
  split_even(n[2], tz, &sz);
  for (auto& y : sy)
    for (auto& x : sx)
      for (auto& z : sz) {
        TileDev t;
        t.box = box;
        t.x0 = (int)o[0] + x.first;
        t.y0 = (int)o[1] + y.first;
        t.z0 = (int)o[2] + z.first;
        t.nx = x.second;
        t.ny = y.second;
        t.nz = z.second;
        t.dir = 0;
        out->push_back(t);
      }
}

// parent box of level l-1 holding the whole prolongation stencil of q
int stencil_parent(const LevelMaps& P, const int64_t q[3]) {
  int64_t smin[3], smax[3];
  for (int d = 0; d < 3; ++d) {
    int64_t base = floordiv2(q[d]);
    smin[d] = (q[d] & 1) ? base - 2 : base;
    smax[d] = (q[d] & 1) ? base + 3 : base;
  }
  for (size_t i = 0; i < P.boxes.size(); ++i) {
    const IBox& b = P.boxes[i];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      bool full = P.periodic[d] && b.lo[d] == 0 && b.hi[d] == P.N[d] - 1;
      if (!full) in = in && smin[d] >= b.lo[d] && smax[d] <= b.hi[d];
    }
    if (in) return (int)i;
  }
  return -1;
}

std::string build_layout(sc_ctx* c) {
  const Hierarchy& H = c->hier;
  const int G = c->G;   // ghost layers = padding of every box array
  const int nm = H.geo.nmembers;
  const int nl = H.geo.nlevels;
  c->lev.assign(nl, LevelDev());
  for (int l = 0; l < nl; ++l) {
    const LevelMaps& M = H.levels[l];
    LevelDev& L = c->lev[l];
    L.dx = H.geo.dx0 / (double)(int64_t(1) << l);
    // subcycled: dt_l = cfl dx_l; uniform: the finest level's step everywhere
    L.dt = c->cfg.cfl * (c->cfg.time_stepping == SC_UNIFORM_DT
                             ? H.geo.dx0 / (double)(int64_t(1) << (nl - 1))
                             : L.dx);
    L.nb_member = (int)M.boxes.size();
    L.has_child = l + 1 < nl;
    L.nbuf = c->cfg.time_stepping == SC_BUFFER_ZONES ? 3 : 2;
    L.shape.radius = c->fd_order == 8 ? (c->G == 5 ? 5 : 4) : 3;
    if (c->cfg.rhs == SC_RHS_Z4C) {
      // the Z4c kernels run one wave per SIMD (two 128-thread workgroups per
      // CU): short, half-height tiles (two planes, at most 256 points per
      // plane) give each CU several to interleave instead of leaving it idle
      // after the box's few tall tiles are handed out (the tile table is
      // sized for at least this many)
      L.shape.tz = 2;
      L.shape.slots = 1;
    }
    L.nyh = l == 0 ? 1 : 8;
    // boxes of member 0
    std::vector<BoxDev> b0(L.nb_member);
    int64_t base = 0;
    L.prefix.assign(L.nb_member + 1, 0);
    for (int ib = 0; ib < L.nb_member; ++ib) {
      const IBox& bx = M.boxes[ib];
      BoxDev& B = b0[ib];
      B.base = base;
      B.nx = (int)bx.n(0);
      B.ny = (int)bx.n(1);
      B.nz = (int)bx.n(2);
      B.px = B.nx + 2 * G;
      B.py = B.ny + 2 * G;
      for (int d = 0; d < 3; ++d) {
        B.lo[d] = (int)bx.lo[d];
        B.wrapN[d] = (M.periodic[d] && bx.lo[d] == 0 && bx.hi[d] == M.N[d] - 1) ? (int)M.N[d] : 0;
      }
      B.pad = G;
      base += (int64_t)B.px * B.py * (B.nz + 2 * G);
      L.prefix[ib + 1] = L.prefix[ib] + bx.volume();
    }
    L.member_total = base;
    L.total = base * nm;
    L.owned_member = L.prefix[L.nb_member];
    for (int m = 0; m < nm; ++m)
      for (int ib = 0; ib < L.nb_member; ++ib) {
        BoxDev B = b0[ib];
        B.base += m * L.member_total;
        L.boxes.push_back(B);
      }
    // halo classification of every box (member 0), replicated per member
    std::vector<SyncEntry> sync0;
    std::vector<ProlongEntry> pro0;
    std::vector<int64_t> phys0;
    std::map<int64_t, int64_t> first;  // RB key -> first halo offset
    for (int ib = 0; ib < L.nb_member; ++ib) {
      const BoxDev& B = b0[ib];
      for (int z = -G; z < B.nz + G; ++z)
        for (int y = -G; y < B.ny + G; ++y)
          for (int x = -G; x < B.nx + G; ++x) {
            if (x >= 0 && x < B.nx && y >= 0 && y < B.ny && z >= 0 && z < B.nz) continue;
            const int64_t dst = B.base + ((int64_t)(z + G) * B.py + (y + G)) * B.px + (x + G);
            int64_t p[3] = {B.lo[0] + x, B.lo[1] + y, B.lo[2] + z}, q[3];
            M.wrap(p, q);
            if (M.outside(q)) {
              phys0.push_back(dst);
              L.phys_q.insert(L.phys_q.end(), {p[0], p[1], p[2]});
              continue;
            }
            int ob = M.box_of(q);
            if (ob >= 0) {
              const BoxDev& O = b0[ob];
              const int64_t src = O.base +
                                  ((q[2] - O.lo[2] + G) * O.py + (q[1] - O.lo[1] + G)) * O.px +
                                  (q[0] - O.lo[0] + G);
              sync0.push_back({dst, src});
              continue;
            }
            if (l == 0) return "level 0 has unowned halo points";
            const int pb = stencil_parent(H.levels[l - 1], q);
            if (pb < 0) return "prolongation stencil not inside one parent box";
            ProlongEntry e;
            e.dst = dst;
            for (int d = 0; d < 3; ++d) e.q[d] = (int32_t)q[d];
            e.pbox = pb;
            pro0.push_back(e);
            const int64_t key = (q[2] << 42) | (q[1] << 21) | q[0];
            first.emplace(key, dst);
          }
    }
    // buffer zones: the buffer points (owned) take the same prolonged value as
    // the RB slots before every fine step, so they join the prolongation list
    for (const auto& q : M.buffer) {
      const int ib = M.box_of(q.data());
      if (ib < 0) return "buffer point outside the level's boxes";
      const BoxDev& B = b0[ib];
      ProlongEntry e;
      e.dst = B.base + ((q[2] - B.lo[2] + G) * B.py + (q[1] - B.lo[1] + G)) * B.px +
              (q[0] - B.lo[0] + G);
      for (int d = 0; d < 3; ++d) e.q[d] = (int32_t)q[d];
      e.pbox = stencil_parent(H.levels[l - 1], q.data());
      if (e.pbox < 0) return "prolongation stencil not inside one parent box";
      pro0.push_back(e);
    }
    const int npb = l > 0 ? c->lev[l - 1].nb_member : 0;
    // group RB halo slots (and buffer points) into bricks: the slots of each
    // face of a fine box form slabs of the shell's full thickness (with buffer
    // zones the buffer points under the face too) by up to 17 points along the
    // face (the face cut into chunks of even start), edge pieces and corners
    // likewise; any other point goes into a cell of a box-local 8-point
    // lattice.  A group too large for one brick is cut into 8-point cells.
    // Slots that wrap periodically or whose stencils span two parent boxes
    // stay per point.
    std::vector<ProlongEntry> rest0;
    std::vector<ProlongBrick> bricks0;
    {
      // shell depth: the ghost layers, and with buffer zones the buffer points
      // inside the box (at most 3G deep); the chunk width along a face is the
      // largest of 16, 14, ... whose slabs (the last chunk one wider) fit a brick
      const int depth = G + (c->cfg.time_stepping == SC_BUFFER_ZONES ? 3 * G : 0);
      int cw = 16;
      for (; cw > 4; cw -= 2) {
        bool ok = true;
        for (int dn = 0; dn < 3 && ok; ++dn)
          for (int al = 0; al < 2 && ok; ++al) {
            int a[3], n[3];
            for (int d = 0; d < 3; ++d) {
              a[d] = 2 + al;   // both parities of the first index
              n[d] = d == dn ? depth : cw + 1;
            }
            ok = sc::brick_fits(a, n);
          }
        if (ok) break;
      }
      auto chunk = [cw](int p, int n) {   // face chunks of cw points, the last up to cw + 1
        const int nc = std::max(1, (n - 1 + cw - 1) / cw);
        return std::min(p / cw, nc - 1);
      };
      const int bdepth = depth - G;   // buffer points this deep inside count as the shell
      // key: box, kind (0 shell, 1 inside), side code, then per-dimension chunk or cell
      std::map<std::array<int64_t, 6>, std::vector<size_t>> groups;
      std::vector<std::array<int, 4>> where(pro0.size());   // box and box-local point
      for (size_t i = 0; i < pro0.size(); ++i) {
        const ProlongEntry& e = pro0[i];
        int ib = -1;
        for (int b = 0; b < L.nb_member; ++b)
          if (e.dst >= b0[b].base &&
              e.dst < b0[b].base + (int64_t)b0[b].px * b0[b].py * (b0[b].nz + 2 * G))
            ib = b;
        const BoxDev& B = b0[ib];
        const int64_t r = e.dst - B.base;
        const int hx = (int)(r % B.px) - G, hy = (int)((r / B.px) % B.py) - G,
                  hz = (int)(r / ((int64_t)B.px * B.py)) - G;
        if (B.lo[0] + hx != e.q[0] || B.lo[1] + hy != e.q[1] || B.lo[2] + hz != e.q[2]) {
          rest0.push_back(e);
          continue;
        }
        where[i] = {ib, hx, hy, hz};
        const int h[3] = {hx, hy, hz}, bn[3] = {B.nx, B.ny, B.nz};
        int side = 0, outside = 0;
        int64_t c[3];
        for (int d = 2; d >= 0; --d) {
          const int sd = h[d] < bdepth ? 1 : (h[d] >= bn[d] - bdepth ? 2 : 0);
          side = side * 3 + sd;
          outside |= sd;
          c[d] = sd ? 0 : chunk(h[d], bn[d]);
        }
        if (!outside)
          groups[{(int64_t)ib, 1, 0, h[2] >> 3, h[1] >> 3, h[0] >> 3}].push_back(i);
        else
          groups[{(int64_t)ib, 0, side, c[2], c[1], c[0]}].push_back(i);
      }
      auto emit = [&](const std::vector<size_t>& idx) -> bool {
        const int pb = pro0[idx[0]].pbox;
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        for (size_t i : idx) {
          if (pro0[i].pbox != pb) return false;
          for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], pro0[i].q[d]);
            hi[d] = std::max(hi[d], pro0[i].q[d]);
          }
        }
        int n[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
        if (!sc::brick_fits(lo, n)) return false;
        ProlongBrick bk{};
        bk.fbox = where[idx[0]][0];
        bk.pbox = pb;
        for (int d = 0; d < 3; ++d) {
          bk.a[d] = lo[d];
          bk.n[d] = n[d];
        }
        for (size_t i : idx) {
          const int fx = pro0[i].q[0] - lo[0], fy = pro0[i].q[1] - lo[1], fz = pro0[i].q[2] - lo[2];
          const int bit = (fz * bk.n[1] + fy) * bk.n[0] + fx;
          bk.mask[bit >> 6] |= uint64_t(1) << (bit & 63);
        }
        bricks0.push_back(bk);
        return true;
      };
      for (auto& kv : groups) {
        if (emit(kv.second)) continue;
        std::map<std::array<int, 3>, std::vector<size_t>> cells;   // box-local 8-point cells
        for (size_t i : kv.second)
          cells[{where[i][3] >> 3, where[i][2] >> 3, where[i][1] >> 3}].push_back(i);
        for (auto& ck : cells)
          if (!emit(ck.second))
            for (size_t i : ck.second) rest0.push_back(pro0[i]);
      }
    }
    for (int m = 0; m < nm; ++m) {
      const int64_t off = m * L.member_total;
      for (auto e : sync0) L.sync.push_back({e.dst + off, e.src + off});
      for (auto e : rest0) {
        e.dst += off;
        e.pbox += m * npb;
        L.prolong.push_back(e);
      }
      for (auto bk : bricks0) {
        L.brick_max_pts = std::max(L.brick_max_pts, bk.n[0] * bk.n[1] * bk.n[2]);
        bk.fbox += m * L.nb_member;
        bk.pbox += m * npb;
        L.bricks.push_back(bk);
      }
      for (auto d : phys0) L.phys.push_back(d + off);
    }
    // prolongation entries grouped by parity class (stable: halo order kept
    // within a class), so a workgroup runs one stencil shape
    {
      auto cls = [](const ProlongEntry& e) { return (e.q[0] & 1) | ((e.q[1] & 1) << 1) | ((e.q[2] & 1) << 2); };
      std::stable_sort(L.prolong.begin(), L.prolong.end(),
                       [&](const ProlongEntry& x, const ProlongEntry& y) { return cls(x) < cls(y); });
      for (int k = 0; k < 9; ++k) L.prolong_cls[k] = 0;
      for (const auto& e : L.prolong) ++L.prolong_cls[cls(e) + 1];
      for (int k = 0; k < 8; ++k) L.prolong_cls[k + 1] += L.prolong_cls[k];
    }
    // RB list (sorted) entries for readers
    L.nrb = (int64_t)M.rb.size();
    for (int m = 0; m < nm; ++m)
      for (int64_t j = 0; j < L.nrb; ++j) {
        const auto& q = M.rb[j];
        ProlongEntry e;
        e.dst = j;
        for (int d = 0; d < 3; ++d) e.q[d] = (int32_t)q[d];
        e.pbox = stencil_parent(H.levels[l - 1], q.data()) + m * npb;
        L.rblist.push_back(e);
        const int64_t key = (q[2] << 42) | (q[1] << 21) | q[0];
        auto it = first.find(key);
        if (it == first.end()) return "RB list entry without a halo slot";
        L.rbfirst.push_back(it->second + m * L.member_total);
      }
    {
      auto cls = [](const ProlongEntry& e) { return (e.q[0] & 1) | ((e.q[1] & 1) << 1) | ((e.q[2] & 1) << 2); };
      for (int m = 0; m < nm; ++m)
        std::stable_sort(L.rblist.begin() + m * L.nrb, L.rblist.begin() + (m + 1) * L.nrb,
                         [&](const ProlongEntry& x, const ProlongEntry& y) { return cls(x) < cls(y); });
      for (int k = 0; k < 9; ++k) L.rblist_cls[k] = 0;
      for (int64_t j = 0; j < L.nrb; ++j) ++L.rblist_cls[cls(L.rblist[j]) + 1];
      for (int k = 0; k < 8; ++k) L.rblist_cls[k + 1] += L.rblist_cls[k];
    }
    // restriction regions (this level as the fine level)
    if (l > 0) {
      const LevelMaps& P = H.levels[l - 1];
      const int npbm = c->lev[l - 1].nb_member;
      std::vector<RestrictRegion> r0;
      for (int fb = 0; fb < L.nb_member; ++fb) {
        const IBox& f = M.boxes[fb];
        for (int pb = 0; pb < npbm; ++pb) {
          const IBox& pbx = P.boxes[pb];
          RestrictRegion R;
          R.fbox = fb;
          R.pbox = pb;
          int64_t cnt = 1;
          for (int d = 0; d < 3; ++d) {
            int64_t a = std::max((f.lo[d] + 1) / 2, pbx.lo[d]);
            int64_t b = std::min(f.hi[d] / 2, pbx.hi[d]);
            R.c0[d] = (int)a;
            R.n[d] = (int)std::max<int64_t>(0, b - a + 1);
            cnt *= R.n[d];
          }
          if (cnt <= 0) continue;
          if (M.buffer.empty()) {
            R.start = cnt;  // temporarily the count
            r0.push_back(R);
            continue;
          }
          // buffer zones: only parent points whose image is not a buffer
          // point; one region if they form a box, else one per x run
          std::vector<uint8_t> ok((size_t)cnt);
          int64_t nok = 0, vlo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, vhi[3] = {-1, -1, -1};
          size_t i = 0;
          for (int z = 0; z < R.n[2]; ++z)
            for (int y = 0; y < R.n[1]; ++y)
              for (int x = 0; x < R.n[0]; ++x, ++i) {
                const int64_t q[3] = {2 * (int64_t)(R.c0[0] + x), 2 * (int64_t)(R.c0[1] + y),
                                      2 * (int64_t)(R.c0[2] + z)};
                ok[i] = !M.is_buffer(q);
                if (!ok[i]) continue;
                ++nok;
                const int64_t v[3] = {x, y, z};
                for (int d = 0; d < 3; ++d) {
                  vlo[d] = std::min(vlo[d], v[d]);
                  vhi[d] = std::max(vhi[d], v[d]);
                }
              }
          if (nok == 0) continue;
          const int64_t bvol = (vhi[0] - vlo[0] + 1) * (vhi[1] - vlo[1] + 1) * (vhi[2] - vlo[2] + 1);
          if (bvol == nok) {
            RestrictRegion Q = R;
            for (int d = 0; d < 3; ++d) {
              Q.c0[d] = R.c0[d] + (int)vlo[d];
              Q.n[d] = (int)(vhi[d] - vlo[d] + 1);
            }
            Q.start = nok;
            r0.push_back(Q);
            continue;
          }
          for (int z = 0; z < R.n[2]; ++z)
            for (int y = 0; y < R.n[1]; ++y) {
              const size_t row = ((size_t)z * R.n[1] + y) * R.n[0];
              for (int x = 0; x < R.n[0];) {
                if (!ok[row + x]) {
                  ++x;
                  continue;
                }
                int e = x;
                while (e < R.n[0] && ok[row + e]) ++e;
                RestrictRegion Q = R;
                Q.c0[0] = R.c0[0] + x;
                Q.c0[1] = R.c0[1] + y;
                Q.c0[2] = R.c0[2] + z;
                Q.n[0] = e - x;
                Q.n[1] = Q.n[2] = 1;
                Q.start = e - x;
                r0.push_back(Q);
                x = e;
              }
            }
        }
      }
      int64_t start = 0;
      for (int m = 0; m < nm; ++m)
        for (auto R : r0) {
          const int64_t cnt = R.start;
          R.fbox += m * L.nb_member;
          R.pbox += m * npbm;
          R.start = start;
          start += cnt;
          L.restr.push_back(R);
        }
      L.restr_total = start;
    }
    // tiles: batched over boxes, and per block
    for (int ib = 0; ib < (int)L.boxes.size(); ++ib) {
      const BoxDev& B = L.boxes[ib];
      const int64_t o[3] = {0, 0, 0}, n[3] = {B.nx, B.ny, B.nz};
      tile_region(ib, o, n, L.shape, &L.tiles);
    }
    L.btile_start.push_back(0);
    for (int m = 0; m < nm; ++m)
      for (size_t b = 0; b < M.blocks.size(); ++b) {
        const IBox& bl = M.blocks[b];
        const int ib = M.block_box[b];
        const IBox& bx = M.boxes[ib];
        const int64_t o[3] = {bl.lo[0] - bx.lo[0], bl.lo[1] - bx.lo[1], bl.lo[2] - bx.lo[2]};
        const int64_t n[3] = {bl.n(0), bl.n(1), bl.n(2)};
        tile_region(m * L.nb_member + ib, o, n, L.shape, &L.btiles);
        L.btile_start.push_back((int32_t)L.btiles.size());
      }
    if (c->cfg.rhs == SC_RHS_Z4C) {
      for (int ib = 0; ib < (int)L.boxes.size(); ++ib) {
        const BoxDev& B = L.boxes[ib];
        const int64_t o[3] = {0, 0, 0}, n[3] = {B.nx, B.ny, B.nz};
        der_region(ib, o, n, der_tz(c->fd_order), &L.dtiles);
      }
      L.bdtile_start.push_back(0);
      for (int m = 0; m < nm; ++m)
        for (size_t b = 0; b < M.blocks.size(); ++b) {
          const IBox& bl = M.blocks[b];
          const int ib = M.block_box[b];
          const IBox& bx = M.boxes[ib];
          const int64_t o[3] = {bl.lo[0] - bx.lo[0], bl.lo[1] - bx.lo[1], bl.lo[2] - bx.lo[2]};
          const int64_t n[3] = {bl.n(0), bl.n(1), bl.n(2)};
          der_region(m * L.nb_member + ib, o, n, der_tz(c->fd_order), &L.bdtiles);
          L.bdtile_start.push_back((int32_t)L.bdtiles.size());
        }
    }
  }
  return "";
}

// Host-side bounds check of every device table before anything is uploaded:
// each kernel index derived from these tables stays inside its buffers.
std::string validate_layout(const sc_ctx* c) {
  const int G = c->G;
  for (size_t l = 0; l < c->lev.size(); ++l) {
    const LevelDev& L = c->lev[l];
    auto in_level = [&](int64_t o) { return o >= 0 && o < L.total; };
    auto tile_ok = [&](const TileDev& t, int slots, int threads) {
      if (t.box < 0 || t.box >= (int)L.boxes.size()) return false;
      const BoxDev& B = L.boxes[t.box];
      return tile_fits(t.nx, t.ny, slots, threads, L.shape.radius) && t.nz >= 1 &&
             (t.dir == 0 || t.dir == 1) &&
             t.x0 >= 0 && t.y0 >= 0 && t.z0 >= 0 && t.x0 + t.nx <= B.nx &&
             t.y0 + t.ny <= B.ny && t.z0 + t.nz <= B.nz;
    };
    for (const TileDev& t : L.tiles)
      if (!tile_ok(t, L.shape.slots, L.shape.threads)) return "tile outside its box";
    for (const TileDev& t : L.btiles)
      if (!tile_ok(t, kStageSlotsMax, kStageThreads)) return "block tile outside its box";
    for (const std::vector<TileDev>* v : {&L.dtiles, &L.bdtiles})
      for (const TileDev& t : *v) {
        if (t.box < 0 || t.box >= (int)L.boxes.size()) return "derivative column outside its box";
        const BoxDev& B = L.boxes[t.box];
        if (t.nx < 1 || t.ny < 1 || t.nz < 1 || t.nx > kDerTx || t.ny > kDerTy ||
            t.nz > der_tz(c->fd_order) || t.x0 < 0 || t.y0 < 0 || t.z0 < 0 || t.x0 + t.nx > B.nx ||
            t.y0 + t.ny > B.ny || t.z0 + t.nz > B.nz)
          return "derivative column outside its box";
      }
    for (const BoxDev& B : L.boxes)
      if (!in_level(B.base) ||
          B.base + (int64_t)B.px * B.py * (B.nz + 2 * G) > L.total)
        return "box array outside the level arrays";
    for (const SyncEntry& e : L.sync)
      if (!in_level(e.dst) || !in_level(e.src)) return "halo copy entry out of range";
    for (int64_t d : L.phys)
      if (!in_level(d)) return "physical ghost entry out of range";
    for (int64_t d : L.rbfirst)
      if (!in_level(d)) return "RB reader entry out of range";
    if (l == 0 && (!L.prolong.empty() || !L.restr.empty())) return "level 0 has parent data";
    if (l > 0) {
      const LevelDev& P = c->lev[l - 1];
      auto pro_ok = [&](const ProlongEntry& e) {
        if (e.pbox < 0 || e.pbox >= (int)P.boxes.size()) return false;
        const BoxDev& B = P.boxes[e.pbox];
        const int n[3] = {B.nx, B.ny, B.nz};
        for (int d = 0; d < 3; ++d) {
          const int base = e.q[d] >> 1, odd = e.q[d] & 1;
          if (e.q[d] < 0) return false;
          if (B.wrapN[d] > 0) continue;
          const int a = odd ? base - 2 : base, b = odd ? base + 3 : base;
          if (a - B.lo[d] < 0 || b - B.lo[d] >= n[d]) return false;
        }
        return true;
      };
      for (const ProlongEntry& e : L.prolong)
        if (!pro_ok(e) || !in_level(e.dst)) return "prolongation entry out of range";
      for (const ProlongBrick& bk : L.bricks) {
        if (bk.fbox < 0 || bk.fbox >= (int)L.boxes.size() || bk.pbox < 0 ||
            bk.pbox >= (int)P.boxes.size())
          return "brick box out of range";
        const BoxDev& F = L.boxes[bk.fbox];
        const int fn[3] = {F.nx, F.ny, F.nz};
        if (!sc::brick_fits(bk.a, bk.n)) return "brick exceeds the kernel's limits";
        const BoxDev& Pb = P.boxes[bk.pbox];
        if ((int64_t)F.px * F.py * (F.nz + 2 * G) >= (int64_t(1) << 32) ||
            (int64_t)Pb.px * Pb.py * (Pb.nz + 2 * G) >= (int64_t(1) << 32))
          return "box too large for the bricks' 32-bit offsets";
        for (int d = 0; d < 3; ++d)
          if (bk.a[d] < 0 || bk.a[d] - F.lo[d] < -G || bk.a[d] + bk.n[d] - 1 - F.lo[d] >= fn[d] + G)
            return "brick outside its fine box halo";
        for (int z = 0; z < bk.n[2]; ++z)
          for (int y = 0; y < bk.n[1]; ++y)
            for (int x = 0; x < bk.n[0]; ++x) {
              const int bit = (z * bk.n[1] + y) * bk.n[0] + x;
              if (!((bk.mask[bit >> 6] >> (bit & 63)) & 1)) continue;
              ProlongEntry e;
              e.dst = 0;
              e.q[0] = bk.a[0] + x;
              e.q[1] = bk.a[1] + y;
              e.q[2] = bk.a[2] + z;
              e.pbox = bk.pbox;
              if (!pro_ok(e)) return "brick point stencil outside its parent box";
            }
      }
      for (const ProlongEntry& e : L.rblist)
        if (!pro_ok(e) || e.dst < 0 || e.dst >= L.nrb) return "RB list entry out of range";
      int64_t expect = 0;
      for (const RestrictRegion& R : L.restr) {
        if (R.fbox < 0 || R.fbox >= (int)L.boxes.size() || R.pbox < 0 ||
            R.pbox >= (int)P.boxes.size() || R.start != expect)
          return "restriction region malformed";
        const BoxDev &F = L.boxes[R.fbox], &Pb = P.boxes[R.pbox];
        const int fn[3] = {F.nx, F.ny, F.nz}, pn[3] = {Pb.nx, Pb.ny, Pb.nz};
        for (int d = 0; d < 3; ++d) {
          const int a = R.c0[d], b = R.c0[d] + R.n[d] - 1;
          if (R.n[d] < 1 || 2 * a - F.lo[d] < 0 || 2 * b - F.lo[d] >= fn[d] ||
              a - Pb.lo[d] < 0 || b - Pb.lo[d] >= pn[d])
            return "restriction region outside its boxes";
        }
        expect += (int64_t)R.n[0] * R.n[1] * R.n[2];
      }
      if (expect != L.restr_total) return "restriction count mismatch";
    }
    if ((int64_t)L.prefix.back() != L.owned_member) return "canonical prefix mismatch";
  }
  return "";
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void plan_arena(sc_ctx* c) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  int64_t maxowned = 0;
  for (LevelDev& L : c->lev) {
    const size_t arr = sizeof(double) * (size_t)c->nvars * (size_t)L.total;
    const size_t arrs = c->esz * (size_t)c->nvars * (size_t)L.total;
    for (int i = 0; i < L.nbuf; ++i) L.o_y[i] = take(arr);
    for (int i = 0; i < 2; ++i) L.o_y32[i] = (c->mixed && !c->wave_mixed) ? take(arr / 2) : 0;
    for (int i = 0; i < 4; ++i) L.o_k[i] = take(arrs);
    for (int i = 0; i < L.nyh; ++i) L.o_yh[i] = take(arrs);
    L.nyd = c->wave_mixed ? (L.nyh == 1 ? 1 : 2) : 0;
    for (int i = 0; i < L.nyd; ++i) L.o_yd[i] = take(arr);
    L.o_ys = c->cfg.rhs == SC_RHS_Z4C ? take(sizeof(double) * (size_t)kZ4cScratch * (size_t)L.total) : 0;
    L.o_boxes = take(sizeof(BoxDev) * L.boxes.size());
    L.o_prefix = take(sizeof(int64_t) * L.prefix.size());
    L.o_sync = take(sizeof(SyncEntry) * L.sync.size());
    L.o_prolong = take(sizeof(ProlongEntry) * L.prolong.size());
    L.o_bricks = take(sizeof(ProlongBrick) * L.bricks.size());
    L.o_rblist = take(sizeof(ProlongEntry) * L.rblist.size());
    L.o_rbfirst = take(sizeof(int64_t) * L.rbfirst.size());
    L.o_phys = take(sizeof(int64_t) * L.phys.size());
    L.o_restr = take(sizeof(RestrictRegion) * L.restr.size());
    {
      // the most tiles any shape the autotuner tries can make
      L.tiles_capacity = L.tiles.size();
      for (int tx : {kTileMaxX, 32}) {
        std::vector<TileDev> most;
        TileShape sh = L.shape;
        sh.tx = tx;
        sh.tz = kTuneTzMin;
        sh.slots = 1;
        for (int ib = 0; ib < (int)L.boxes.size(); ++ib) {
          const BoxDev& B = L.boxes[ib];
          const int64_t o[3] = {0, 0, 0}, n[3] = {B.nx, B.ny, B.nz};
          tile_region(ib, o, n, sh, &most);
        }
        L.tiles_capacity = std::max(L.tiles_capacity, most.size());
      }
    }
    L.o_tiles = take(sizeof(TileDev) * L.tiles_capacity);
    L.o_btiles = take(sizeof(TileDev) * L.btiles.size());
    L.o_dtiles = take(sizeof(TileDev) * L.dtiles.size());
    L.o_bdtiles = take(sizeof(TileDev) * L.bdtiles.size());
    maxowned = std::max(maxowned, std::max(L.owned_member, L.nrb * (int64_t)c->hier.geo.nmembers));
    maxowned = std::max(maxowned, (int64_t)L.phys_q.size() / 3);
  }
  // Z4c: one FP64 derivative scratch (the FP64 right-hand side and the
  // constraint), sized for the largest level (levels run one after another)
  int64_t maxtotal = 0;
  for (const LevelDev& L : c->lev) maxtotal = std::max(maxtotal, L.total);
  c->o_der = c->cfg.rhs == SC_RHS_Z4C
                 ? take(sizeof(double) * (size_t)kZ4cDer * (size_t)maxtotal) : 0;
  c->stage_elems = std::max<int64_t>(maxowned, 1);
  c->o_stage = take(sizeof(double) * (size_t)c->stage_elems);
  c->norm_parts_max = norm_parts(maxowned);
  c->o_partials = take(sizeof(double) * 4 * (size_t)c->norm_parts_max);
  c->o_norm_out = take(sizeof(double) * 4);
  c->o_flag = take(sizeof(unsigned int));
  c->arena_bytes = off;
}

template <class T>
T* at(sc_ctx* c, size_t o) {
  return reinterpret_cast<T*>(c->arena + o);
}

template <class T>
hipError_t upload(sc_ctx* c, T* dst, const std::vector<T>& v) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, c->stream);
}

// ---------------------------------------------------------------------------
// Scheduler.

int yh_index(int level, int substep, int stage) { return level == 0 ? 0 : substep * 4 + stage - 1; }

// State buffers rotate: y[cur] is the current state, y[nxt] receives the next
// one, y[prv] holds the state the last step started from (two buffers: nxt ==
// prv; three with buffer zones, where y[nxt] still holds y_{n-1} until the
// level's next step overwrites it).
inline int nxt(const LevelDev& L) { return (L.cur + 1) % L.nbuf; }
inline int prv(const LevelDev& L) { return (L.cur + L.nbuf - 1) % L.nbuf; }
inline bool buffer_zones(const sc_ctx* c) { return c->cfg.time_stepping == SC_BUFFER_ZONES; }

int take_events(sc_ctx* c, hipEvent_t* e0, hipEvent_t* e1) {
  while (c->ev_pool.size() < c->ev_used + 2) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  *e0 = c->ev_pool[c->ev_used];
  *e1 = c->ev_pool[c->ev_used + 1];
  c->ev_used += 2;
  return SC_OK;
}

// Element offset helper for the typed level arrays (k, Yh).
inline void* elem(void* base, int64_t i, size_t esz) { return static_cast<char*>(base) + i * esz; }

int enqueue_stage_launches(sc_ctx* c, int l, int stage, bool per_block, const void* yn,
                           const void* kprev, const void* yh) {
  LevelDev& L = c->lev[l];
  StageArgs a{};
  a.stage = stage;
  a.boxes = L.d_boxes;
  a.yn = yn;
  a.kprev = kprev;
  a.Yh = yh;
  a.k1 = L.k[0];
  a.k2 = L.k[1];
  a.k3 = L.k[2];
  a.kout = L.k[stage - 1];
  a.yn64 = L.y[L.cur];
  a.ynew = L.y[nxt(L)];
  a.vstride = L.total;
  static const double cnext[5] = {0.0, 0.0, 0.5, 0.5, 1.0};
  a.cdt = cnext[stage] * L.dt;
  a.dt6 = L.dt / 6.0;
  a.radius = L.shape.radius;
  a.clap = a.radius >= 4 ? 1.0 / (5040.0 * L.dx * L.dx) : 1.0 / (12.0 * L.dx * L.dx);
  a.cko = c->cfg.ko_sigma / ((a.radius == 5 ? 1024.0 : 64.0) * L.dx);
  a.nonfinite = c->d_nonfinite;
  // k4 is read only by the prolongation into a finer level
  a.write_k = (stage < 4 || L.has_child) ? 1 : 0;
  if (!per_block) {
    a.tiles = L.d_tiles;
    a.ntiles = (int32_t)L.tiles.size();
    int grid = std::min<int>(a.ntiles, L.shape.grid > 0 ? L.shape.grid : c->grid_cap);
    grid = (grid + 7) / 8 * 8;  // a multiple of the XCD count (the kernel's tile remap)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool own_events = c->profiling && !c->ev_grouped;   // else the level step's pair
    if (own_events) {
      int rc = take_events(c, &e0, &e1);
      if (rc) return rc;
      HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    HIPCHK(c, launch_stage(a, grid, c->mixed, L.shape.depth, L.shape.slots, L.shape.threads,
                           c->stream));
    if (own_events) HIPCHK(c, hipEventRecord(e1, c->stream));
    if (c->profiling) {
      ++c->ev_launches;
      // algorithmic bytes per owned point and variable: the stencil operands
      // y_n and k_{s-1}, the new slope, and for stage 4 also k1, k2, the FP64
      // y_n and y_{n+1}; mixed: stage 1 reads the FP64 y_n and writes an FP32
      // k1, stages 2-4 read the FP32 k_{s-1} (and k1 at stages 3, 4), stage 4
      // also k2, the FP64 y_n and y_{n+1}
      static const double fp64[5] = {0, 16, 24, 24, 48};
      static const double mixed[5] = {0, 12, 8, 12, 32};
      double per_var = c->mixed ? mixed[stage] : fp64[stage];
      if (!a.write_k) per_var -= c->esz;  // k4 not stored on the finest level
      c->ev_bytes.push_back(per_var * c->nvars * (double)(L.owned_member * c->hier.geo.nmembers));
    }
    ++c->launches;
  } else {
    const int nblk = (int)L.btile_start.size() - 1;
    for (int b = 0; b < nblk; ++b) {
      a.tiles = L.d_btiles + L.btile_start[b];
      a.ntiles = L.btile_start[b + 1] - L.btile_start[b];
      HIPCHK(c, launch_stage(a, a.ntiles, c->mixed, 1, kStageSlotsMax, kStageThreads, c->stream));
      ++c->launches;
    }
  }
  return SC_OK;
}

Z4cArgs z4c_args(sc_ctx* c, int l) {
  LevelDev& L = c->lev[l];
  Z4cArgs a{};
  a.boxes = L.d_boxes;
  a.vstride = L.total;
  a.h = L.dx;
  a.dt6 = L.dt / 6.0;
  a.sigma = c->cfg.ko_sigma;
  a.kappa1 = c->cfg.z4c_kappa1;
  a.kappa2 = c->cfg.z4c_kappa2;
  a.eta_c = c->cfg.z4c_eta_c;
  a.eta_o = c->cfg.z4c_eta_o;
  a.eta_s = c->cfg.z4c_eta_s;
  for (int d = 0; d < 3; ++d) a.origin[d] = c->hier.geo.origin[d];
  a.ord = c->fd_order;
  a.ko_r = c->G == 5 ? 8 : 4;
  a.nonfinite = c->d_nonfinite;
  a.der = c->d_der;
  a.dtiles = L.d_dtiles;   // the whole level; per-block launches narrow it
  a.ndtiles = (int32_t)L.dtiles.size();
  return a;
}

// Z4c stage: write Y_s = y_n + c_s dt k_{s-1} (y_n for s = 1) on the owned
// points into the stage's halo table, whose halo the fills have written, then
// the RHS reads the table alone.
int enqueue_z4c_launches(sc_ctx* c, int l, int stage, bool per_block, const void* kprev,
                         const void* yh) {
  LevelDev& L = c->lev[l];
  static const double cnext[5] = {0.0, 0.0, 0.5, 0.5, 1.0};
  Z4cArgs a = z4c_args(c, l);
  a.stage = stage;
  void* table = const_cast<void*>(yh);
  a.Y = table;
  a.yn = L.y[L.cur];
  a.k1 = L.k[0];
  a.k2 = L.k[1];
  a.k3 = L.k[2];
  a.kout = L.k[stage - 1];
  a.ynew = L.y[nxt(L)];
  a.ynew32 = c->mixed ? L.y32[1 - L.cur] : nullptr;
  a.geo = L.Ys;   // kZ4cScratch arrays of double: room for the curvature arrays in either precision
  // radiative outer boundary: level 0's ghost stage values go into the table
  // before any stencil reads them; their right-hand side follows the interior's
  const bool rad = c->cfg.outer_bc == SC_BC_RADIATIVE && l == 0 && !L.phys.empty();
  Z4cRadArgs ra{};
  if (rad) {
    ra.idx = L.d_phys;
    ra.n = (int64_t)L.phys.size();
    ra.per_member = ra.n / c->hier.geo.nmembers;
    ra.boxes = L.d_boxes;
    ra.Y = static_cast<const double*>(yh);
    ra.yn = L.y[L.cur];
    ra.kprev = stage >= 2 ? static_cast<const double*>(kprev) : nullptr;
    ra.k1 = static_cast<const double*>(L.k[0]);
    ra.k2 = static_cast<const double*>(L.k[1]);
    ra.k3 = static_cast<const double*>(L.k[2]);
    ra.kout = static_cast<double*>(L.k[stage - 1]);
    ra.ynew = L.y[nxt(L)];
    ra.table = static_cast<double*>(table);
    ra.vstride = L.total;
    ra.stage = stage;
    ra.cdt = cnext[stage] * L.dt;
    ra.dt6 = L.dt / 6.0;
    ra.h = L.dx;
    for (int d = 0; d < 3; ++d) ra.origin[d] = c->hier.geo.origin[d];
    HIPCHK(c, launch_z4c_rad_fill(ra, c->stream));
    ++c->launches;
  }
  Z4cCombineArgs cb{};
  cb.nvars = c->nvars;
  cb.boxes = L.d_boxes;
  cb.yn = c->mixed ? static_cast<const void*>(L.y32[L.cur]) : L.y[L.cur];
  cb.kprev = stage >= 2 ? kprev : nullptr;
  cb.Y = table;
  cb.vstride = L.total;
  cb.cdt = cnext[stage] * L.dt;
  auto run = [&](const TileDev* tiles, int ntiles, int grid) -> int {
    cb.tiles = tiles;
    cb.ntiles = ntiles;
    HIPCHK(c, launch_z4c_combine(cb, grid, c->mixed, c->stream));
    ++c->launches;
    a.tiles = tiles;
    a.ntiles = ntiles;
    HIPCHK(c, launch_z4c_stage(a, grid, c->mixed, c->stream));
    ++c->launches;
    return SC_OK;
  };
  if (!per_block) {
    const int rc = run(L.d_tiles, (int)L.tiles.size(), z4c_grid((int)L.tiles.size()));
    if (rc) return rc;
  } else {
    // per block: every block's stage vector must be complete before any
    // block's stencil reads its neighbours, so all combines go first
    const int nblk = (int)L.btile_start.size() - 1;
    for (int b = 0; b < nblk; ++b) {
      const int n = L.btile_start[b + 1] - L.btile_start[b];
      cb.tiles = L.d_btiles + L.btile_start[b];
      cb.ntiles = n;
      HIPCHK(c, launch_z4c_combine(cb, n, c->mixed, c->stream));
      ++c->launches;
    }
    for (int b = 0; b < nblk; ++b) {
      const int n = L.btile_start[b + 1] - L.btile_start[b];
      a.tiles = L.d_btiles + L.btile_start[b];
      a.ntiles = n;
      a.dtiles = L.d_bdtiles + L.bdtile_start[b];
      a.ndtiles = L.bdtile_start[b + 1] - L.bdtile_start[b];
      HIPCHK(c, launch_z4c_stage(a, n, c->mixed, c->stream));
      ++c->launches;
    }
  }
  if (rad) {
    HIPCHK(c, launch_z4c_radiative(ra, c->stream));
    ++c->launches;
  }
  return SC_OK;
}

int rk4_step(sc_ctx* c, int l, int substep, bool per_block) {
  LevelDev& L = c->lev[l];
  // the Z4c FP32 right-hand side reads the FP32 shadow of y_n; the wave
  // reads the FP64 y_n (mixed: at stage 1 only)
  const bool shadow = c->mixed && !c->wave_mixed;
  const void* yn = shadow ? static_cast<const void*>(L.y32[L.cur]) : L.y[L.cur];
  // kernel timing: when nothing but the four batched stage launches runs on
  // the stream during the step (no ghost sync), one event pair spans all four
  hipEvent_t g0 = nullptr, g1 = nullptr;
  c->ev_grouped = false;
  if (c->profiling && !per_block && L.sync.empty() && c->cfg.rhs == SC_RHS_WAVE) {
    int rc = take_events(c, &g0, &g1);
    if (rc) return rc;
    HIPCHK(c, hipEventRecord(g0, c->stream));
    c->ev_grouped = true;
  }
  for (int s = 1; s <= 4; ++s) {
    // buffer zones: the RB ghosts keep the step's prolonged value at every stage
    void* yh = L.Yh[buffer_zones(c) ? (l == 0 ? 0 : substep * 4) : yh_index(l, substep, s)];
    if (c->wave_mixed && s == 1) yh = L.Yd[l == 0 ? 0 : substep];
    const void* kprev = s == 1 ? nullptr : L.k[s - 2];
    if (!L.sync.empty()) {
      SyncArgs sa{};
      sa.e = L.d_sync;
      sa.n = (int64_t)L.sync.size();
      sa.yn = yn;
      sa.kprev = kprev;
      sa.out = yh;
      sa.vstride = L.total;
      static const double cnext[5] = {0.0, 0.0, 0.5, 0.5, 1.0};
      sa.cdt = cnext[s] * L.dt;
      sa.nvars = c->nvars;
      sa.inc = c->wave_mixed && s > 1;
      const bool f32 = c->wave_mixed ? s > 1 : c->mixed;
      HIPCHK(c, launch_sync(sa, f32, c->stream));
      ++c->launches;
    }
    int rc = c->cfg.rhs == SC_RHS_Z4C ? enqueue_z4c_launches(c, l, s, per_block, kprev, yh)
                                      : enqueue_stage_launches(c, l, s, per_block, yn, kprev, yh);
    if (rc) {
      c->ev_grouped = false;
      return rc;
    }
  }
  if (c->ev_grouped) {
    c->ev_grouped = false;
    HIPCHK(c, hipEventRecord(g1, c->stream));
  }
  L.cur = nxt(L);
  ++L.steps_done;
  return SC_OK;
}

// Prolongation from the parent's last step (y_n = the buffer it stepped from,
// k1..k4) into the fine level: outputs[i] with weights[i].
// Output o is FP32 if bit o of f32_mask is set, and a stage increment
// (weights minus the substep's Y1 weights, no P[y_n] term) if bit o of inc_mask is.
int prolong_into(sc_ctx* c, int fl, const ProlongEntry* entries, const int64_t* cls, int nout,
                 void* const* outs, const int* fills, const int* subs, int64_t ovstride,
                 uint32_t f32_mask, uint32_t inc_mask, int var_only, bool with_bricks) {
  auto wsel = [&](int o) -> const double* {
    return ((inc_mask >> o) & 1) ? c->weights_inc[subs[o]][fills[o] - 1]
                                 : c->weights[subs[o]][fills[o] - 1];
  };
  LevelDev& P = c->lev[fl - 1];
  LevelDev& F = c->lev[fl];
  if (with_bricks && !F.bricks.empty()) {
    BrickArgs b{};
    b.b = F.d_bricks;
    b.nbricks = (int32_t)F.bricks.size();
    b.max_pts = F.brick_max_pts;
    b.nout = nout;
    b.nvars = c->nvars;
    b.fboxes = F.d_boxes;
    b.pboxes = P.d_boxes;
    b.py = P.y[prv(P)];
    for (int i = 0; i < 4; ++i) b.pk[i] = P.k[i];
    b.pvstride = P.total;
    b.ovstride = ovstride;
    b.H = P.dt;
    b.f32_mask = f32_mask;
    b.inc_mask = inc_mask;
    for (int o = 0; o < nout; ++o) {
      b.out[o] = outs[o];
      for (int i = 0; i < 4; ++i) b.w[o][i] = wsel(o)[i];
    }
    HIPCHK(c, launch_prolong_bricks(b, c->mixed, c->stream));
    ++c->launches;
  }
  const int64_t n = cls[8];
  if (n <= 0) return SC_OK;
  ProlongArgs a{};
  a.e = entries;
  a.n = n;
  a.blk_start[0] = 0;
  for (int k = 0; k < 9; ++k) a.cls_start[k] = cls[k];
  for (int k = 0; k < 8; ++k)
    a.blk_start[k + 1] = a.blk_start[k] + (int32_t)((cls[k + 1] - cls[k] + 255) / 256);
  a.pboxes = P.d_boxes;
  a.py = P.y[prv(P)];
  for (int i = 0; i < 4; ++i) a.pk[i] = P.k[i];
  a.pvstride = P.total;
  a.ovstride = ovstride;
  a.H = P.dt;
  a.nout = nout;
  a.nvars = c->nvars;
  if (var_only >= 0) {  // a single variable, outputs unstrided
    a.nvars = 1;
    a.py += var_only * P.total;
    for (int i = 0; i < 4; ++i) a.pk[i] = elem(P.k[i], var_only * P.total, c->esz);
  }
  a.f32_mask = f32_mask;
  a.inc_mask = inc_mask;
  for (int o = 0; o < nout; ++o) {
    a.out[o] = outs[o];
    for (int i = 0; i < 4; ++i) a.w[o][i] = wsel(o)[i];
  }
  HIPCHK(c, launch_prolong(a, c->mixed, c->stream));
  ++c->launches;
  return SC_OK;
}

int prolongate(sc_ctx* c, int fl) {
  LevelDev& F = c->lev[fl];
  void* outs[8];
  int fills[8], subs[8];
  uint32_t f32_mask = 0, inc_mask = 0;
  const int nsub = c->cfg.time_stepping == SC_UNIFORM_DT ? 1 : 2;   // fine steps per parent step
  for (int sub = 0; sub < nsub; ++sub)
    for (int s = 1; s <= 4; ++s) {
      const int o = sub * 4 + s - 1;
      outs[o] = F.Yh[o];
      fills[o] = s;
      subs[o] = sub;
      if (c->wave_mixed) {   // FP64 Y1, FP32 increments Y_s - Y1
        if (s == 1) outs[o] = F.Yd[sub];
        else f32_mask |= 1u << o, inc_mask |= 1u << o;
      } else if (c->mixed) {
        f32_mask |= 1u << o;
      }
    }
  return prolong_into(c, fl, F.d_prolong, F.prolong_cls, 4 * nsub, outs, fills, subs, F.total,
                      f32_mask, inc_mask, -1, true);
}

// Buffer zones: the parent's state at the start of fine substep `sub`
// (theta0 = sub / 2), interpolated in time over its last three states
// (two while it has made one step), prolonged into the RB slots of the
// substep's ghost table and into the buffer points of the fine state.  The
// parent has completed its step: y_{n+1} = y[cur], y_n = y[prv], y_{n-1} =
// y[nxt].
int prolongate_buffer(sc_ctx* c, int fl, int sub) {
  LevelDev& P = c->lev[fl - 1];
  LevelDev& F = c->lev[fl];
  const double* yn = P.y[prv(P)];
  const double* ynew = P.y[P.cur];
  const bool history = P.steps_done >= 2;
  const double* yold = history ? P.y[nxt(P)] : yn;   // weight 0 without history
  const int nin = sub == 0 ? 1 : 3;
  double w[3] = {0.0, 0.5, 0.5};
  if (history) w[0] = -0.125, w[1] = 0.75, w[2] = 0.375;
  void* outs[2] = {F.y[F.cur], F.Yh[sub * 4]};
  if (!F.bricks.empty()) {
    BrickArgs b{};
    b.b = F.d_bricks;
    b.nbricks = (int32_t)F.bricks.size();
    b.max_pts = F.brick_max_pts;
    b.nout = 2;
    b.nvars = c->nvars;
    b.fboxes = F.d_boxes;
    b.pboxes = P.d_boxes;
    b.py = yn;
    b.pk[0] = yold;
    b.pk[1] = ynew;
    b.pvstride = P.total;
    b.ovstride = F.total;
    b.H = P.dt;
    for (int o = 0; o < 2; ++o) {
      b.out[o] = outs[o];
      for (int i = 0; i < 3; ++i) b.w[o][i] = w[i];
    }
    HIPCHK(c, launch_prolong_bricks(b, false, c->stream, nin));
    ++c->launches;
  }
  const int64_t n = F.prolong_cls[8];
  if (n <= 0) return SC_OK;
  ProlongArgs a{};
  a.e = F.d_prolong;
  a.n = n;
  a.blk_start[0] = 0;
  for (int k = 0; k < 9; ++k) a.cls_start[k] = F.prolong_cls[k];
  for (int k = 0; k < 8; ++k)
    a.blk_start[k + 1] =
        a.blk_start[k] + (int32_t)((F.prolong_cls[k + 1] - F.prolong_cls[k] + 255) / 256);
  a.pboxes = P.d_boxes;
  a.py = yn;
  a.pk[0] = yold;
  a.pk[1] = ynew;
  a.pvstride = P.total;
  a.ovstride = F.total;
  a.H = P.dt;
  a.nout = 2;
  a.nvars = c->nvars;
  for (int o = 0; o < 2; ++o) {
    a.out[o] = outs[o];
    for (int i = 0; i < 3; ++i) a.w[o][i] = w[i];
  }
  HIPCHK(c, launch_prolong(a, false, c->stream, nin));
  ++c->launches;
  return SC_OK;
}

int restrict_level(sc_ctx* c, int fl) {
  LevelDev& F = c->lev[fl];
  LevelDev& P = c->lev[fl - 1];
  if (F.restr_total == 0) return SC_OK;
  RestrictArgs a{};
  a.r = F.d_restr;
  a.nregions = (int)F.restr.size();
  a.ntotal = F.restr_total;
  a.fboxes = F.d_boxes;
  a.pboxes = P.d_boxes;
  a.fy = F.y[F.cur];
  a.py = P.y[P.cur];
  a.py32 = (c->mixed && !c->wave_mixed) ? P.y32[P.cur] : nullptr;
  a.fvstride = F.total;
  a.pvstride = P.total;
  a.nvars = c->nvars;
  HIPCHK(c, launch_restrict(a, c->stream));
  ++c->launches;
  return SC_OK;
}

// Buffer zones (Carpet): refill from the parent, step, recurse, restrict.
int advance_level_buffer(sc_ctx* c, int l, int substep, bool per_block) {
  Range r("level %d step %lld (substep %d, buffer zones)", l, (long long)c->lev[l].steps_done,
          substep);
  int rc;
  if (l > 0 && (rc = prolongate_buffer(c, l, substep))) return rc;
  if ((rc = rk4_step(c, l, substep, per_block))) return rc;
  if (l + 1 < (int)c->lev.size()) {
    if ((rc = advance_level_buffer(c, l + 1, 0, per_block))) return rc;
    if ((rc = advance_level_buffer(c, l + 1, 1, per_block))) return rc;
    if ((rc = restrict_level(c, l + 1))) return rc;
  }
  c->lev[l].t += c->lev[l].dt;
  return SC_OK;
}

int advance_level(sc_ctx* c, int l, int substep, bool per_block) {
  if (buffer_zones(c)) return advance_level_buffer(c, l, substep, per_block);
  Range r("level %d step %lld (substep %d)", l, (long long)c->lev[l].steps_done, substep);
  int rc;
  {
    Range r4("rk4 level %d", l);
    if ((rc = rk4_step(c, l, substep, per_block))) return rc;
  }
  if (l + 1 < (int)c->lev.size()) {
    {
      Range rp("prolongate level %d", l + 1);
      if ((rc = prolongate(c, l + 1))) return rc;
    }
    if ((rc = advance_level(c, l + 1, 0, per_block))) return rc;
    if (c->cfg.time_stepping != SC_UNIFORM_DT &&
        (rc = advance_level(c, l + 1, 1, per_block)))
      return rc;
    if ((rc = restrict_level(c, l + 1))) return rc;
  }
  c->lev[l].t += c->lev[l].dt;
  return SC_OK;
}

int check_ready(const sc_ctx* c, int need) {
  if (!c) return SC_E_ARG;
  if (c->state < need) {
    const_cast<sc_ctx*>(c)->err = "call out of order (state machine)";
    return SC_E_STATE;
  }
  return SC_OK;
}

// Array of one variable: FP64 state buffers, or the typed slope arrays.
void* array_ptr(sc_ctx* c, int l, int array, int var, bool* f32) {
  LevelDev& L = c->lev[l];
  *f32 = false;
  switch (array) {
    case SC_ARR_Y: return L.y[L.cur] + var * L.total;
    case SC_ARR_YN: return L.y[prv(L)] + var * L.total;
    default:
      *f32 = c->mixed;
      return elem(L.k[array - 1], var * L.total, c->esz);
  }
}

int scatter_phys(sc_ctx* c, int member, int level, int var);

// One deterministic reduction (NormArgs) with the given partials and output
// buffers; r = {max, sum, weight sum, non-finite count}.  Synchronises.
int reduce(sc_ctx* c, const NormArgs& a, bool f32, double* partials, double* dout, double r[4]) {
  HIPCHK(c, launch_norms(a, f32, partials, dout, c->stream));
  HIPCHK(c, hipMemcpyAsync(r, dout, sizeof(double) * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

int hamiltonian_into_scratch(sc_ctx* c, int level);

// New data: clear the device flag of non-finite state values and its host copy
// (a fill kernel, not a memset, so the call may sit in captured work).
int reset_nonfinite(sc_ctx* c) {
  HIPCHK(c, launch_fill_u32(c->d_nonfinite, 1, 0u, c->stream));
  if (c->flag_pending) HIPCHK(c, hipEventSynchronize(c->flag_ev));
  c->flag_pending = false;
  *c->h_flag = 0;
  return SC_OK;
}

PackArgs member_pack(sc_ctx* c, int member, int l, void* arr) {
  LevelDev& L = c->lev[l];
  PackArgs a{};
  a.boxes = L.d_boxes + member * L.nb_member;
  a.prefix = L.d_prefix;
  a.nboxes = L.nb_member;
  a.n = L.owned_member;
  a.arr = arr;
  a.buf = c->d_stage;
  return a;
}

}  // namespace

// ===========================================================================
extern "C" {

int sc_config_default(sc_config* cfg) {
  if (!cfg) return SC_E_ARG;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->abi_version = SC_ABI_VERSION;
  cfg->rhs = SC_RHS_WAVE;
  cfg->precision = SC_FP64;
  cfg->exec = SC_EXEC_BATCHED;
  cfg->nghost = 3;
  cfg->fd_order = 4;
  cfg->ko_sigma = 0.32;
  cfg->cfl = 0.25;
  cfg->z4c_kappa1 = 0.02;
  cfg->z4c_kappa2 = 0.0;
  cfg->z4c_eta_c = 2.0;
  cfg->z4c_eta_o = 0.25;
  cfg->z4c_eta_s = 40.0;
  return SC_OK;
}

int sc_create(const sc_config* cfg, void* hip_stream, sc_ctx** out) {
  if (!cfg || !out) {
    g_create_error = "null argument";
    return SC_E_ARG;
  }
  *out = nullptr;
  if (cfg->abi_version != SC_ABI_VERSION) {
    g_create_error = "abi_version mismatch";
    return SC_E_ARG;
  }
  const bool rhs_ok = (cfg->rhs == SC_RHS_WAVE || cfg->rhs == SC_RHS_Z4C) &&
                     (cfg->time_stepping == SC_SUBCYCLED || cfg->time_stepping == SC_UNIFORM_DT ||
                      (cfg->time_stepping == SC_BUFFER_ZONES && cfg->rhs == SC_RHS_WAVE &&
                       cfg->precision == SC_FP64));
  // eighth order: FP64, four ghost layers (five: the r = 8 dissipation),
  // subcycled or uniform steps
  const bool order_ok =
      (cfg->fd_order == 4 && cfg->nghost == 3) ||
      (cfg->fd_order == 8 && (cfg->nghost == 4 || cfg->nghost == 5) &&
       cfg->precision == SC_FP64 &&
       cfg->time_stepping != SC_BUFFER_ZONES);
  // radiative outer boundary: Z4c, FP64
  const bool bc_ok = cfg->outer_bc == SC_BC_FROZEN ||
                     (cfg->outer_bc == SC_BC_RADIATIVE && cfg->rhs == SC_RHS_Z4C &&
                      cfg->precision == SC_FP64);
  if (!rhs_ok || !order_ok || !bc_ok || !(cfg->z4c_eta_s > 0.0) ||
      !(cfg->cfl > 0.0 && cfg->cfl <= 0.5) ||
      cfg->ko_sigma < 0.0 || (cfg->precision != SC_FP64 && cfg->precision != SC_MIXED) ||
      cfg->exec < 0 || cfg->exec > 2) {
    g_create_error = "unsupported configuration (rhs, time stepping (buffer zones: wave, FP64), "
                     "fd_order 4 with nghost 3 or 8 with nghost 4 (FP64, no buffer zones) or "
                     "nghost 5 (r = 8 dissipation, FP64, no buffer zones), "
                     "outer_bc (radiative: Z4c, FP64), "
                     "0 < cfl <= 0.5, sigma >= 0, precision, exec)";
    return SC_E_ARG;
  }
  sc_ctx* c = new sc_ctx();
  c->cfg = *cfg;
  c->mixed = cfg->precision == SC_MIXED;
  c->nvars = cfg->rhs == SC_RHS_Z4C ? 22 : 2;
  c->G = cfg->nghost;
  c->fd_order = cfg->fd_order;
  c->esz = c->mixed ? sizeof(float) : sizeof(double);
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->wave_mixed = c->mixed && cfg->rhs == SC_RHS_WAVE;
  for (int sub = 0; sub < 2; ++sub) {
    Rat r1[4];
    for (int f = 1; f <= 5; ++f) {
      Rat r[4];
      if (cfg->time_stepping == SC_UNIFORM_DT) aligned_weights(f, r);
      else ghost_weights(f, sub ? Rat(1, 2) : Rat(0), r);
      if (f == 1)
        for (int i = 0; i < 4; ++i) r1[i] = r[i];
      // stage increment Y_f - Y_1 of the substep, exact before rounding
      for (int i = 0; i < 4; ++i) {
        c->weights[sub][f - 1][i] = r[i].f();
        c->weights_inc[sub][f - 1][i] = (r[i] - r1[i]).f();
      }
    }
  }
  *out = c;
  return SC_OK;
}

int sc_destroy(sc_ctx* c) {
  if (!c) return SC_OK;
  // kernels still queued on the caller's stream write into the arena, which
  // the caller may free (or hand to another tensor) as soon as this returns
  if (c->state >= 2 && c->stream) (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < 3; ++i)
    if (c->graph[i]) (void)hipGraphExecDestroy(c->graph[i]);
  delete c;
  return SC_OK;
}

const char* sc_last_error(const sc_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int sc_build_hierarchy(sc_ctx* c, int32_t nmembers, const double origin[3], double dx0,
                       const int64_t ncells0[3], const int32_t periodic[3], int32_t nlevels,
                       const int32_t* nboxes_per_level, const sc_box* boxes, uint64_t block_seed,
                       int32_t min_block, int32_t max_block) {
  if (!c) return SC_E_ARG;
  if (c->state != 0) return fail(c, SC_E_STATE, "hierarchy already built");
  if (!origin || !ncells0 || !periodic || nlevels < 1 || nmembers < 1 || !(dx0 > 0.0) ||
      (nlevels > 1 && (!nboxes_per_level || !boxes)))
    return fail(c, SC_E_ARG, "bad hierarchy arguments");
  Geometry g;
  g.nmembers = nmembers;
  g.dx0 = dx0;
  g.nlevels = nlevels;
  for (int d = 0; d < 3; ++d) {
    g.origin[d] = origin[d];
    g.ncells0[d] = ncells0[d];
    g.periodic[d] = periodic[d] != 0;
    if (ncells0[d] < 1 || ncells0[d] > (int64_t(1) << 20) >> (nlevels - 1))
      return fail(c, SC_E_ARG, "ncells0 out of range");
  }
  int64_t k = 0;
  for (int l = 1; l < nlevels; ++l) {
    if (nboxes_per_level[l - 1] < 1) return fail(c, SC_E_ARG, "a fine level needs a box");
    std::vector<IBox> lv;
    for (int i = 0; i < nboxes_per_level[l - 1]; ++i, ++k) {
      IBox b;
      for (int d = 0; d < 3; ++d) {
        b.lo[d] = boxes[k].lo[d];
        b.hi[d] = boxes[k].hi[d];
      }
      lv.push_back(b);
    }
    g.fine_boxes.push_back(lv);
  }
  bool nest = false;
  // buffer zones: three ghost widths of buffer points (the RK4 stages after
  // the first each spoil one ghost width of the fine level's edge)
  const int bz = c->cfg.time_stepping == SC_BUFFER_ZONES ? 3 * c->cfg.nghost : 0;
  std::string e = c->hier.build(g, c->cfg.nghost, block_seed, min_block, max_block, &nest, bz);
  if (!e.empty()) return fail(c, nest ? SC_E_NEST : SC_E_ARG, e);
  e = build_layout(c);
  if (!e.empty()) return fail(c, SC_E_NEST, e);
  e = validate_layout(c);
  if (!e.empty()) return fail(c, SC_E_ARG, "internal layout check: " + e);
  if (c->cfg.outer_bc == SC_BC_RADIATIVE) {
    for (size_t l = 1; l < c->lev.size(); ++l)
      if (!c->lev[l].phys.empty())
        return fail(c, SC_E_ARG, "radiative boundary: only level 0 may touch the outer boundary");
    for (int d = 0; d < 3; ++d)
      if (g.periodic[d]) return fail(c, SC_E_ARG, "radiative boundary: the domain must not be periodic");
  }
  plan_arena(c);
  c->state = 1;
  return SC_OK;
}

int sc_get_counts(const sc_ctx* c, int32_t level, int32_t* nblocks, int64_t* nowned,
                  int64_t* nrb) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->hier.levels.size()) return SC_E_ARG;
  const LevelMaps& M = c->hier.levels[level];
  if (nblocks) *nblocks = (int32_t)M.blocks.size();
  if (nowned) *nowned = M.nowned;
  if (nrb) *nrb = (int64_t)M.rb.size();
  return SC_OK;
}

int sc_buffer_count(const sc_ctx* c, int32_t level, int64_t* nbuffer) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->hier.levels.size() || !nbuffer) return SC_E_ARG;
  *nbuffer = (int64_t)c->hier.levels[level].buffer.size();
  return SC_OK;
}

int sc_export_maps(const sc_ctx* c, int64_t* words, int64_t* nwords) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (!nwords) return SC_E_ARG;
  std::vector<int64_t> w;
  c->hier.export_words(&w);
  if (!words) {
    *nwords = (int64_t)w.size();
    return SC_OK;
  }
  if (*nwords < (int64_t)w.size()) {
    const_cast<sc_ctx*>(c)->err = "export buffer too small";
    return SC_E_ARG;
  }
  std::memcpy(words, w.data(), sizeof(int64_t) * w.size());
  *nwords = (int64_t)w.size();
  return SC_OK;
}

int sc_device_bytes(const sc_ctx* c, size_t* nbytes) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (!nbytes) return SC_E_ARG;
  *nbytes = c->arena_bytes;
  return SC_OK;
}

int sc_bind_device_memory(sc_ctx* c, void* dptr, size_t nbytes) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (!dptr) return fail(c, SC_E_ARG, "null arena");
  if (nbytes < c->arena_bytes) return fail(c, SC_E_MEM, "arena smaller than sc_device_bytes");
  if (reinterpret_cast<uintptr_t>(dptr) & 255) return fail(c, SC_E_MEM, "arena not 256-byte aligned");
  c->arena = static_cast<char*>(dptr);
  int dev = 0, ncu = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  c->grid_cap = std::max(ncu, 1) * 8;
  HIPCHK(c, hipMemsetAsync(c->arena, 0, c->arena_bytes, c->stream));
  for (LevelDev& L : c->lev) {
    for (int i = 0; i < L.nbuf; ++i) L.y[i] = at<double>(c, L.o_y[i]);
    for (int i = 0; i < 2; ++i)
      L.y32[i] = (c->mixed && !c->wave_mixed) ? at<float>(c, L.o_y32[i]) : nullptr;
    for (int i = 0; i < 4; ++i) L.k[i] = at<char>(c, L.o_k[i]);
    for (int i = 0; i < L.nyh; ++i) L.Yh[i] = at<char>(c, L.o_yh[i]);
    for (int i = 0; i < L.nyd; ++i) L.Yd[i] = at<double>(c, L.o_yd[i]);
    L.Ys = c->cfg.rhs == SC_RHS_Z4C ? at<double>(c, L.o_ys) : nullptr;
    L.d_boxes = at<BoxDev>(c, L.o_boxes);
    L.d_prefix = at<int64_t>(c, L.o_prefix);
    L.d_sync = at<SyncEntry>(c, L.o_sync);
    L.d_prolong = at<ProlongEntry>(c, L.o_prolong);
    L.d_bricks = at<ProlongBrick>(c, L.o_bricks);
    L.d_rblist = at<ProlongEntry>(c, L.o_rblist);
    L.d_rbfirst = at<int64_t>(c, L.o_rbfirst);
    L.d_phys = at<int64_t>(c, L.o_phys);
    L.d_restr = at<RestrictRegion>(c, L.o_restr);
    L.d_tiles = at<TileDev>(c, L.o_tiles);
    L.d_btiles = at<TileDev>(c, L.o_btiles);
    L.d_dtiles = at<TileDev>(c, L.o_dtiles);
    L.d_bdtiles = at<TileDev>(c, L.o_bdtiles);
    HIPCHK(c, upload(c, L.d_boxes, L.boxes));
    HIPCHK(c, upload(c, L.d_prefix, L.prefix));
    HIPCHK(c, upload(c, L.d_sync, L.sync));
    HIPCHK(c, upload(c, L.d_prolong, L.prolong));
    HIPCHK(c, upload(c, L.d_bricks, L.bricks));
    HIPCHK(c, upload(c, L.d_rblist, L.rblist));
    HIPCHK(c, upload(c, L.d_rbfirst, L.rbfirst));
    HIPCHK(c, upload(c, L.d_phys, L.phys));
    HIPCHK(c, upload(c, L.d_restr, L.restr));
    HIPCHK(c, upload(c, L.d_tiles, L.tiles));
    HIPCHK(c, upload(c, L.d_btiles, L.btiles));
    HIPCHK(c, upload(c, L.d_dtiles, L.dtiles));
    HIPCHK(c, upload(c, L.d_bdtiles, L.bdtiles));
  }
  c->d_stage = at<double>(c, c->o_stage);
  c->d_der = c->cfg.rhs == SC_RHS_Z4C ? at<double>(c, c->o_der) : nullptr;
  c->d_partials = at<double>(c, c->o_partials);
  c->d_norm_out = at<double>(c, c->o_norm_out);
  c->d_nonfinite = at<unsigned int>(c, c->o_flag);   // zeroed with the arena
  if (!c->h_flag) HIPCHK(c, hipHostMalloc((void**)&c->h_flag, sizeof(unsigned int)));
  *c->h_flag = 0;
  if (!c->flag_ev) HIPCHK(c, hipEventCreateWithFlags(&c->flag_ev, hipEventDisableTiming));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->state = 2;
  return SC_OK;
}

int sc_set_initial_data(sc_ctx* c, int32_t member, int32_t level, int32_t var,
                        const double* host, int64_t n) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || !host)
    return fail(c, SC_E_ARG, "bad initial-data arguments");
  LevelDev& L = c->lev[level];
  if (n != L.owned_member) return fail(c, SC_E_ARG, "n must equal the level's owned points");
  HIPCHK(c, hipMemcpyAsync(c->d_stage, host, sizeof(double) * n, hipMemcpyHostToDevice,
                           c->stream));
  PackArgs a = member_pack(c, member, level, L.y[L.cur] + var * L.total);
  HIPCHK(c, launch_pack(a, true, false, c->stream));
  if (c->mixed && !c->wave_mixed)
    HIPCHK(c, launch_to_f32(L.y[L.cur] + var * L.total, L.y32[L.cur] + var * L.total, L.total,
                            c->stream));
  rc = reset_nonfinite(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->state = 3;
  return SC_OK;
}

int sc_set_initial_data_analytic(sc_ctx* c, int32_t kind, const double* params, int32_t nparams,
                                 uint64_t seed) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (nparams < 0 || (nparams > 0 && !params)) return fail(c, SC_E_ARG, "bad parameter list");
  const bool wave = c->cfg.rhs == SC_RHS_WAVE;
  const int nm = c->hier.geo.nmembers;
  // per-member parameter sets
  std::vector<std::vector<double>> P(nm);
  switch (kind) {
    case SC_ID_STANDING_WAVE:
      if (!wave) return fail(c, SC_E_ARG, "a standing wave is wave-equation data");
      if (nparams == 4 || nparams == 5) {
        for (auto& p : P) {
          p.assign(params, params + nparams);
          p.resize(5, 0.0);
        }
      } else if (nparams == 0) {   // ensemble: modes {1,2,3}^3 and amplitude U(0.5, 1.5)
        SplitMix64 rng(seed);
        for (auto& p : P) {
          double m[3];
          for (int d = 0; d < 3; ++d) m[d] = (double)(1 + rng.next() % 3);
          const double amp = 0.5 + rng.uniform();
          p = {amp, m[0], m[1], m[2], 0.0};
        }
      } else {
        return fail(c, SC_E_ARG, "standing wave: 4 or 5 parameters (A, m_x, m_y, m_z[, t]) or 0 "
                                 "(seeded)");
      }
      break;
    case SC_ID_GAUSSIAN_PULSES: {
      if (!wave) return fail(c, SC_E_ARG, "Gaussian pulses are wave-equation data");
      if (nparams < 2) return fail(c, SC_E_ARG, "Gaussian pulses: npulses, period, ...");
      const int np = (int)params[0];
      if (np < 1 || np > 32 || params[0] != (double)np || !(params[1] >= 0.0))
        return fail(c, SC_E_ARG, "Gaussian pulses: 1 <= npulses <= 32, period >= 0");
      std::vector<double> p = {(double)np, params[1]};
      if (nparams == 3) {   // seeded: A U(0.1,1), w U(0.05,0.2), centre (-+x_t, 0, 0) + U(-0.1,0.1)^3
        SplitMix64 rng(seed);
        for (int q = 0; q < np; ++q) {
          const double A = 0.1 + 0.9 * rng.uniform();
          const double w = 0.05 + 0.15 * rng.uniform();
          const double ox = -0.1 + 0.2 * rng.uniform();
          const double oy = -0.1 + 0.2 * rng.uniform();
          const double oz = -0.1 + 0.2 * rng.uniform();
          const double cx = (q % 2 == 0 ? -params[2] : params[2]) + ox;
          p.insert(p.end(), {A, w, cx, oy, oz});
        }
      } else if (nparams == 2 + 5 * np) {
        p.insert(p.end(), params + 2, params + nparams);
        for (int q = 0; q < np; ++q)
          if (!(p[2 + 5 * q + 1] > 0.0)) return fail(c, SC_E_ARG, "Gaussian pulses: widths > 0");
      } else {
        return fail(c, SC_E_ARG, "Gaussian pulses: 3 parameters (npulses, period, x_tower; "
                                 "seeded) or 2 + 5 npulses (A, w, c_x, c_y, c_z per pulse)");
      }
      for (auto& q : P) q = p;
      break;
    }
    case SC_ID_BRILL_LINDQUIST:
      if (wave) return fail(c, SC_E_ARG, "Brill-Lindquist data need the Z4c right-hand side");
      if (nparams != 4) return fail(c, SC_E_ARG, "Brill-Lindquist: (m_+, m_-, x_+, x_-)");
      for (auto& p : P) p.assign(params, params + 4);
      break;
    case SC_ID_SPHERICAL_GAUSSIAN:
      if (!wave) return fail(c, SC_E_ARG, "the spherical Gaussian is wave-equation data");
      if (nparams != 3 || !(params[1] > 0.0))
        return fail(c, SC_E_ARG, "spherical Gaussian: (A, sigma > 0, t)");
      for (auto& p : P) p.assign(params, params + 3);
      break;
    default:
      return fail(c, SC_E_ARG, "unknown initial-data kind");
  }
  for (int l = 0; l < (int)c->lev.size(); ++l) {
    LevelDev& L = c->lev[l];
    for (int m = 0; m < nm; ++m) {
      InitArgs a{};
      a.kind = kind;
      a.nvars = c->nvars;
      a.boxes = L.d_boxes + m * L.nb_member;
      a.prefix = L.d_prefix;
      a.nboxes = L.nb_member;
      for (int d = 0; d < 3; ++d) a.origin[d] = c->hier.geo.origin[d];
      a.dx = L.dx;
      a.vstride = L.total;
      std::copy(P[m].begin(), P[m].end(), a.p);
      // owned points of the current state (and its FP32 shadow)
      a.n = L.owned_member;
      a.out = L.y[L.cur];
      a.out32 = (c->mixed && !c->wave_mixed) ? L.y32[L.cur] : nullptr;
      HIPCHK(c, launch_init(a, c->stream));
      // frozen physical-boundary ghosts take the same closed form
      const int64_t per = (int64_t)L.phys_q.size() / 3;
      if (per == 0) continue;
      a.n = per;
      a.idx = L.d_phys + m * per;
      a.out = c->d_stage;
      a.out32 = nullptr;
      for (int v = 0; v < c->nvars; ++v) {
        a.var = v;
        HIPCHK(c, launch_init(a, c->stream));
        rc = scatter_phys(c, m, l, v);
        if (rc) return rc;
      }
    }
  }
  rc = reset_nonfinite(c);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->state = 3;
  return SC_OK;
}

int sc_phys_count(const sc_ctx* c, int32_t level, int64_t* n) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || !n) return SC_E_ARG;
  *n = (int64_t)c->lev[level].phys_q.size() / 3;
  return SC_OK;
}

int sc_phys_points(const sc_ctx* c, int32_t level, double* xyz, int64_t n) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || !xyz) return SC_E_ARG;
  const LevelDev& L = c->lev[level];
  if (n != (int64_t)L.phys_q.size() / 3) return SC_E_ARG;
  const double dx = L.dx;
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) xyz[3 * i + d] = c->hier.geo.origin[d] + L.phys_q[3 * i + d] * dx;
  return SC_OK;
}

int sc_set_phys_data(sc_ctx* c, int32_t member, int32_t level, int32_t var, const double* host,
                     int64_t n) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || !host)
    return fail(c, SC_E_ARG, "bad physical-ghost arguments");
  LevelDev& L = c->lev[level];
  const int64_t per = (int64_t)L.phys_q.size() / 3;
  if (n != per) return fail(c, SC_E_ARG, "n must equal sc_phys_count");
  if (per == 0) return SC_OK;
  HIPCHK(c, hipMemcpyAsync(c->d_stage, host, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  rc = scatter_phys(c, member, level, var);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

}  // extern "C"

namespace {

// The values of one variable at the physical-boundary ghosts of one member
// of a level, in the library's order in d_stage, into every array that holds
// those ghosts: the halo tables and the state buffers.
int scatter_phys(sc_ctx* c, int member, int level, int var) {
  LevelDev& L = c->lev[level];
  const int64_t per = (int64_t)L.phys_q.size() / 3, n = per;
  const int64_t* idx = L.d_phys + member * per;
  for (int i = 0; i < L.nyh; ++i) {
    void* dst = elem(L.Yh[i], var * L.total, c->esz);
    // mixed wave: frozen ghosts have zero stage increments; their value
    // lives in the FP64 stage-1 tables
    if (c->wave_mixed) HIPCHK(c, launch_scatter_value(idx, n, 0.0, dst, true, c->stream));
    else HIPCHK(c, launch_scatter(idx, n, c->d_stage, dst, c->mixed, c->stream));
  }
  for (int i = 0; i < L.nyd; ++i)
    HIPCHK(c, launch_scatter(idx, n, c->d_stage, L.Yd[i] + var * L.total, false, c->stream));
  for (int i = 0; i < L.nbuf; ++i)
    HIPCHK(c, launch_scatter(idx, n, c->d_stage, L.y[i] + var * L.total, false, c->stream));
  return SC_OK;
}

}  // namespace

extern "C" {

int sc_hamiltonian(sc_ctx* c, int32_t member, int32_t level, double* host, int64_t n) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (c->cfg.rhs != SC_RHS_Z4C) return fail(c, SC_E_STATE, "the Hamiltonian constraint needs Z4c");
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || !host)
    return fail(c, SC_E_ARG, "bad constraint arguments");
  LevelDev& L = c->lev[level];
  if (n != L.owned_member) return fail(c, SC_E_ARG, "n must equal the level's owned points");
  if (level > 0 && c->lev[level - 1].t == 0.0)
    return fail(c, SC_E_STATE, "refinement-boundary ghosts need one parent step first");
  rc = hamiltonian_into_scratch(c, level);
  if (rc) return rc;
  PackArgs pa = member_pack(c, member, level, L.Ys);
  HIPCHK(c, launch_pack(pa, false, false, c->stream));
  HIPCHK(c, hipMemcpyAsync(host, c->d_stage, sizeof(double) * n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

}  // extern "C"

namespace {

// Hamiltonian constraint of the current state of a level (all members) into
// the level's scratch array, after filling the state's ghosts (SYNC,
// physical, and the dense-output end value on refinement boundaries).
int hamiltonian_into_scratch(sc_ctx* c, int level) {
  LevelDev& L = c->lev[level];
  int rc = sc_fill_ghosts(c, level, SC_FILL_END, 1);
  if (rc) return rc;
  Z4cArgs a = z4c_args(c, level);
  a.Y = L.y[L.cur];   // the END fill wrote the state's own halo
  a.ham = L.Ys;       // scratch: one variable's worth of the curvature array
  a.tiles = L.d_tiles;
  a.ntiles = (int32_t)L.tiles.size();
  HIPCHK(c, launch_z4c_stage(a, z4c_grid(a.ntiles), false, c->stream));
  return SC_OK;
}

}  // namespace

extern "C" {

int sc_advance(sc_ctx* c, int32_t ncoarse) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (ncoarse < 0) return fail(c, SC_E_ARG, "ncoarse < 0");
  // the flag copied after the previous call's steps, if it has arrived (no wait)
  if (c->flag_pending && hipEventQuery(c->flag_ev) == hipSuccess) c->flag_pending = false;
  if (!c->flag_pending && *c->h_flag)
    return fail(c, SC_E_NONFINITE, "an earlier coarse step produced a non-finite state value "
                                   "(sc_check_finite locates it; new initial data clear it)");
  c->launches = 0;
  for (int i = 0; i < ncoarse; ++i) {
    Range r("coarse step %lld", (long long)c->lev[0].steps_done);
    // buffer zones: the first coarse step interpolates linearly in time at
    // each level's first step, later ones quadratically; only the latter
    // repeat, so the first runs eagerly
    if (c->cfg.exec == SC_EXEC_GRAPH && !(buffer_zones(c) && c->lev[0].steps_done == 0)) {
      const int parity = c->lev[0].cur;
      // a graph bakes in every level's buffer indices at capture; a level
      // stepped on its own since then (sc_step_level) needs a new capture
      if (c->graph_ready[parity]) {
        bool same = c->graph_cur[parity].size() == c->lev.size();
        for (size_t l = 0; same && l < c->lev.size(); ++l)
          same = c->graph_cur[parity][l] == c->lev[l].cur;
        if (!same) {
          (void)hipGraphExecDestroy(c->graph[parity]);
          c->graph[parity] = nullptr;
          c->graph_ready[parity] = false;
        }
      }
      if (!c->graph_ready[parity]) {
        // capture one coarse step starting from this buffer parity
        std::vector<int> cur0(c->lev.size());
        std::vector<double> t0(c->lev.size());
        std::vector<int64_t> n0(c->lev.size());
        for (size_t l = 0; l < c->lev.size(); ++l)
          cur0[l] = c->lev[l].cur, t0[l] = c->lev[l].t, n0[l] = c->lev[l].steps_done;
        Range rc_("graph capture (level-0 buffer %d)", parity);
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        rc = advance_level(c, 0, 0, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        for (size_t l = 0; l < c->lev.size(); ++l)
          c->lev[l].cur = cur0[l], c->lev[l].t = t0[l], c->lev[l].steps_done = n0[l];
        if (rc) return rc;
        if (e != hipSuccess) return fail(c, SC_E_HIP, std::string("capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
          return fail(c, SC_E_HIP, std::string("instantiate: ") + hipGetErrorString(e));
        c->graph_ready[parity] = true;
        c->graph_cur[parity] = cur0;
      }
      c->launches = 0;
      HIPCHK(c, hipGraphLaunch(c->graph[parity], c->stream));
      // replay the host bookkeeping of one coarse step
      for (size_t l = 0; l < c->lev.size(); ++l) {
        const int64_t steps = c->cfg.time_stepping == SC_UNIFORM_DT ? 1 : int64_t(1) << l;
        LevelDev& L = c->lev[l];
        L.cur = (int)((L.cur + steps) % L.nbuf);
        L.steps_done += steps;
        for (int64_t s = 0; s < steps; ++s) L.t += L.dt;
      }
      ++c->launches;
    } else {
      rc = advance_level(c, 0, 0, c->cfg.exec == SC_EXEC_PER_BLOCK);
      if (rc) return rc;
    }
  }
  if (ncoarse > 0 && !c->flag_pending) {
    HIPCHK(c, hipMemcpyAsync(c->h_flag, c->d_nonfinite, sizeof(unsigned int),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->flag_ev, c->stream));
    c->flag_pending = true;
  }
  return SC_OK;
}

int sc_step_level(sc_ctx* c, int32_t level, int32_t substep) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (buffer_zones(c)) return fail(c, SC_E_STATE, "buffer zones: use sc_advance");
  if (level < 0 || level >= (int)c->lev.size() || substep < 0 || substep > 1)
    return fail(c, SC_E_ARG, "bad level or substep");
  rc = rk4_step(c, level, level == 0 ? 0 : substep, c->cfg.exec == SC_EXEC_PER_BLOCK);
  if (!rc) c->lev[level].t += c->lev[level].dt;
  return rc;
}

int sc_prolongate(sc_ctx* c, int32_t fine_level) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (buffer_zones(c)) return fail(c, SC_E_STATE, "buffer zones: use sc_advance");
  if (fine_level < 1 || fine_level >= (int)c->lev.size()) return fail(c, SC_E_ARG, "bad level");
  return prolongate(c, fine_level);
}

int sc_restrict(sc_ctx* c, int32_t fine_level) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (fine_level < 1 || fine_level >= (int)c->lev.size()) return fail(c, SC_E_ARG, "bad level");
  return restrict_level(c, fine_level);
}

int sc_fill_ghosts(sc_ctx* c, int32_t level, int32_t which, int32_t substep) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (buffer_zones(c)) return fail(c, SC_E_STATE, "buffer zones: use sc_advance");
  if (level < 0 || level >= (int)c->lev.size() || which < 1 || which > 5 || substep < 0 ||
      substep > 1)
    return fail(c, SC_E_ARG, "bad fill arguments");
  LevelDev& L = c->lev[level];
  double* y = L.y[L.cur];
  if (!L.sync.empty()) {
    SyncArgs sa{};
    sa.e = L.d_sync;
    sa.n = (int64_t)L.sync.size();
    sa.yn = y;
    sa.kprev = nullptr;
    sa.out = y;
    sa.vstride = L.total;
    sa.nvars = c->nvars;
    HIPCHK(c, launch_sync(sa, false, c->stream));
  }
  if (level > 0) {
    void* outs[1] = {y};
    const int fills[1] = {which}, subs[1] = {substep};
    rc = prolong_into(c, level, L.d_prolong, L.prolong_cls, 1, outs, fills, subs, L.total,
                      0u, 0u, -1, true);
    if (rc) return rc;
  }
  return SC_OK;
}

int sc_read_back(sc_ctx* c, int32_t member, int32_t level, int32_t var, int32_t array,
                 double* host, int64_t n) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || array < 0 || array > 5 ||
      !host)
    return fail(c, SC_E_ARG, "bad read-back arguments");
  LevelDev& L = c->lev[level];
  if (n != L.owned_member) return fail(c, SC_E_ARG, "n must equal the level's owned points");
  if (array == SC_ARR_K4 && !L.has_child && c->cfg.rhs == SC_RHS_WAVE)
    return fail(c, SC_E_STATE, "k4 is kept only on levels that have a finer level");
  bool f32 = false;
  PackArgs a = member_pack(c, member, level, array_ptr(c, level, array, var, &f32));
  HIPCHK(c, launch_pack(a, false, f32, c->stream));
  HIPCHK(c, hipMemcpyAsync(host, c->d_stage, sizeof(double) * n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

int sc_read_rb(sc_ctx* c, int32_t member, int32_t level, int32_t which, int32_t substep,
               int32_t var, double* host, int64_t n) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (level < 1 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || which < 1 || which > 5 || substep < 0 || substep > 1 ||
      var < 0 || var >= c->nvars || !host)
    return fail(c, SC_E_ARG, "bad RB read arguments");
  if (buffer_zones(c)) return fail(c, SC_E_STATE, "buffer zones: no dense-output RB values");
  LevelDev& L = c->lev[level];
  if (n != L.nrb) return fail(c, SC_E_ARG, "n must equal the level's RB points");
  const int64_t* idx = L.d_rbfirst + member * L.nrb;
  if (which <= 4 && c->wave_mixed) {   // FP64 Y1 plus the FP32 increment
    const double* base = L.Yd[substep] + var * L.total;
    if (which == 1)
      HIPCHK(c, launch_gather(idx, L.nrb, base, false, c->d_stage, c->stream));
    else
      HIPCHK(c, launch_gather_sum(idx, L.nrb, base,
                                  static_cast<const float*>(elem(L.Yh[substep * 4 + which - 1],
                                                                 var * L.total, c->esz)),
                                  c->d_stage, c->stream));
  } else if (which <= 4) {
    const void* src = elem(L.Yh[substep * 4 + which - 1], var * L.total, c->esz);
    HIPCHK(c, launch_gather(idx, L.nrb, src, c->mixed, c->d_stage, c->stream));
  } else {
    void* outs[1] = {c->d_stage};
    const int fills[1] = {5}, subs[1] = {substep};
    rc = prolong_into(c, level, L.d_rblist + member * L.nrb, L.rblist_cls, 1, outs, fills, subs,
                      0, 0u, 0u, var, false);
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpyAsync(host, c->d_stage, sizeof(double) * n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

int sc_norms(sc_ctx* c, int32_t member, int32_t level, int32_t var, int32_t array,
             double out[3]) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || array < 0 || array > 5 ||
      !out)
    return fail(c, SC_E_ARG, "bad norm arguments");
  bool f32 = false;
  NormArgs a{};
  a.p = member_pack(c, member, level, array_ptr(c, level, array, var, &f32));
  a.mode = 0;
  double r[4];
  rc = reduce(c, a, f32, c->d_partials, c->d_norm_out, r);
  if (rc) return rc;
  out[0] = r[0];
  out[1] = r[2] > 0 ? std::sqrt(r[1] / r[2]) : 0.0;
  out[2] = r[3];
  return SC_OK;
}

int sc_norms_noalloc(sc_ctx* c, int32_t member, int32_t level, int32_t var, int32_t array,
                     double out[3]) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || array < 0 || array > 5 ||
      !out)
    return fail(c, SC_E_ARG, "bad norm arguments");
  const int64_t n = c->lev[level].owned_member;
  if (norm_parts(n) > kNoAllocParts) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "level %d has %lld owned points; the static reduction workspace holds at most "
             "%lld (use sc_norms)", level, (long long)n,
             (long long)kNoAllocParts * (long long)kNormPointsPerPart);
    return fail(c, SC_E_ARG, msg);
  }
  double* ws = nullptr;
  HIPCHK(c, noalloc_scratch(&ws));
  bool f32 = false;
  NormArgs a{};
  a.p = member_pack(c, member, level, array_ptr(c, level, array, var, &f32));
  a.mode = 0;
  double r[4];
  rc = reduce(c, a, f32, ws, ws + 4 * kNoAllocParts, r);
  if (rc) return rc;
  out[0] = r[0];
  out[1] = r[2] > 0 ? std::sqrt(r[1] / r[2]) : 0.0;
  out[2] = r[3];
  return SC_OK;
}

int sc_error_norms(sc_ctx* c, int32_t member, int32_t level, int32_t var, int32_t kind,
                   const double* params, int32_t nparams, double out[3]) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || member < 0 ||
      member >= c->hier.geo.nmembers || var < 0 || var >= c->nvars || !out)
    return fail(c, SC_E_ARG, "bad error-norm arguments");
  if (kind != SC_ID_STANDING_WAVE && kind != SC_ID_SPHERICAL_GAUSSIAN)
    return fail(c, SC_E_ARG, "error norms need a closed-form solution at time t: "
                             "SC_ID_STANDING_WAVE or SC_ID_SPHERICAL_GAUSSIAN");
  if (c->cfg.rhs != SC_RHS_WAVE) return fail(c, SC_E_ARG, "closed forms are wave solutions");
  if (kind == SC_ID_STANDING_WAVE && nparams != 5)
    return fail(c, SC_E_ARG, "standing wave: (A, m_x, m_y, m_z, t)");
  if (kind == SC_ID_SPHERICAL_GAUSSIAN && (nparams != 3 || !(params && params[1] > 0.0)))
    return fail(c, SC_E_ARG, "spherical Gaussian: (A, sigma > 0, t)");
  if (!params) return fail(c, SC_E_ARG, "null parameters");
  LevelDev& L = c->lev[level];
  NormArgs a{};
  bool f32 = false;
  a.p = member_pack(c, member, level, array_ptr(c, level, SC_ARR_Y, var, &f32));
  a.mode = 1;
  a.exact.kind = kind;
  a.exact.var = var;
  a.exact.dx = L.dx;
  for (int d = 0; d < 3; ++d) a.exact.origin[d] = c->hier.geo.origin[d];
  std::copy(params, params + nparams, a.exact.p);
  double r[4];
  rc = reduce(c, a, false, c->d_partials, c->d_norm_out, r);
  if (rc) return rc;
  out[0] = r[0];
  out[1] = r[2] > 0 ? std::sqrt(r[1] / r[2]) : 0.0;
  out[2] = r[3];
  return SC_OK;
}

int sc_constraint_norm(sc_ctx* c, int32_t member, double rmax, double alpha_min, double out[3]) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (c->cfg.rhs != SC_RHS_Z4C) return fail(c, SC_E_STATE, "the Hamiltonian constraint needs Z4c");
  if (member < 0 || member >= c->hier.geo.nmembers || !out || !(rmax > 0.0))
    return fail(c, SC_E_ARG, "bad constraint-norm arguments");
  const int nl = (int)c->lev.size();
  for (int l = 1; l < nl; ++l)
    if (c->lev[l - 1].t == 0.0)
      return fail(c, SC_E_STATE, "refinement-boundary ghosts need one parent step first");
  double num = 0.0, den = 0.0, hmax = 0.0, bad = 0.0;
  for (int l = 0; l < nl; ++l) {   // levels in order: a fixed summation order
    LevelDev& L = c->lev[l];
    rc = hamiltonian_into_scratch(c, l);
    if (rc) return rc;
    NormArgs a{};
    a.p = member_pack(c, member, l, L.Ys);
    a.mode = 2;
    a.exact.dx = L.dx;
    for (int d = 0; d < 3; ++d) a.exact.origin[d] = c->hier.geo.origin[d];
    a.alpha = L.y[L.cur] + 18 * L.total;
    if (l + 1 < nl) {
      const LevelDev& F = c->lev[l + 1];
      a.child = F.d_boxes + member * F.nb_member;
      a.nchild = F.nb_member;
    }
    a.rmax = rmax;
    a.amin = alpha_min;
    a.cell = L.dx * L.dx * L.dx;
    double r[4];
    rc = reduce(c, a, false, c->d_partials, c->d_norm_out, r);
    if (rc) return rc;
    hmax = std::max(hmax, r[0]);
    num += r[1];
    den += r[2];
    bad += r[3];
  }
  out[0] = den > 0 ? std::sqrt(num / den) : 0.0;
  out[1] = hmax;
  out[2] = bad;
  return SC_OK;
}

int sc_check_finite(sc_ctx* c) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (c->flag_pending) {
    HIPCHK(c, hipEventSynchronize(c->flag_ev));
    c->flag_pending = false;
  }
  for (int l = 0; l < (int)c->lev.size(); ++l)
    for (int m = 0; m < c->hier.geo.nmembers; ++m)
      for (int v = 0; v < c->nvars; ++v) {
        double o[3];
        if ((rc = sc_norms(c, m, l, v, SC_ARR_Y, o))) return rc;
        if (o[2] > 0) {
          char msg[128];
          snprintf(msg, sizeof msg, "non-finite values on level %d member %d var %d", l, m, v);
          return fail(c, SC_E_NONFINITE, msg);
        }
      }
  return SC_OK;
}

int sc_level_time(const sc_ctx* c, int32_t level, double* t) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || !t) return SC_E_ARG;
  *t = c->lev[level].t;
  return SC_OK;
}

int sc_set_exec(sc_ctx* c, int32_t exec) {
  if (!c) return SC_E_ARG;
  if (exec < 0 || exec > 2) return fail(c, SC_E_ARG, "bad exec mode");
  c->cfg.exec = exec;
  return SC_OK;
}

int sc_poison_halos(sc_ctx* c) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  const double nan = std::nan("");
  for (LevelDev& L : c->lev) {
    if (!L.phys.empty()) return fail(c, SC_E_STATE, "poisoning would erase physical ghosts");
    for (int i = 0; i < L.nyh; ++i)
      HIPCHK(c, launch_fill(L.Yh[i], c->nvars * L.total, nan, c->mixed, c->stream));
    for (int i = 0; i < L.nyd; ++i)
      HIPCHK(c, launch_fill(L.Yd[i], c->nvars * L.total, nan, false, c->stream));
    for (int i = 0; i < 4; ++i)
      HIPCHK(c, launch_fill(L.k[i], c->nvars * L.total, nan, c->mixed, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SC_OK;
}

static void drop_graphs(sc_ctx* c) {
  for (int i = 0; i < 3; ++i) {
    if (c->graph[i]) (void)hipGraphExecDestroy(c->graph[i]);
    c->graph[i] = nullptr;
    c->graph_ready[i] = false;
  }
}

int sc_set_tile_shape(sc_ctx* c, int32_t level, int32_t tz, int32_t grid, int32_t depth,
                      int32_t slots, int32_t threads, int32_t tx) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size()) return fail(c, SC_E_ARG, "level out of range");
  const bool z4c = c->cfg.rhs == SC_RHS_Z4C;
  if (tz < (z4c ? kZ4cTzMin : kTuneTzMin) || tz > (1 << 20))
    return fail(c, SC_E_ARG, "z-chunk out of range");
  if (grid < 0) return fail(c, SC_E_ARG, "grid must be >= 0");
  if (tx < 0 || tx > kTileMaxX) return fail(c, SC_E_ARG, "tile width out of range");
  if (!z4c && !stage_variant_ok(slots, depth, threads))
    return fail(c, SC_E_ARG, "(threads, points per thread, planes in flight) must be (256, 2, 1), "
                             "(256, 2, 2), (256, 1, 2), (512, 2, 1) or (512, 2, 2)");
  LevelDev& L = c->lev[level];
  TileShape sh = L.shape;
  sh.tz = tz;
  if (!z4c) {   // the Z4c kernels keep their own workgroup shape and grid
    sh.depth = depth;
    sh.slots = slots;
    sh.threads = threads;
    sh.tx = tx > 0 ? tx : kTileDefaultX;
  }
  std::vector<TileDev> tl;
  for (int ib = 0; ib < (int)L.boxes.size(); ++ib) {
    const BoxDev& B = L.boxes[ib];
    const int64_t o[3] = {0, 0, 0}, n[3] = {B.nx, B.ny, B.nz};
    tile_region(ib, o, n, sh, &tl);
  }
  if (tl.size() > L.tiles_capacity)
    return fail(c, SC_E_ARG, "z-chunk gives more tiles than the tile table holds");
  sh.grid = (grid == 0 || z4c) ? 0 : std::min<int>(grid, (int)tl.size());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, upload(c, L.d_tiles, tl));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  L.tiles = tl;
  L.shape = sh;
  drop_graphs(c);
  return SC_OK;
}

int sc_autotune(sc_ctx* c, int32_t reps) {
  int rc = check_ready(c, 3);
  if (rc) return rc;
  if (reps < 1 || reps > 1000) return fail(c, SC_E_ARG, "reps must be in [1, 1000]");
  if (c->cfg.rhs != SC_RHS_WAVE) return fail(c, SC_E_STATE, "autotuning covers the wave stencil");
  int dev = 0, ncu = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const bool prof = c->profiling;
  c->profiling = false;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  for (size_t l = 0; l < c->lev.size(); ++l) {
    LevelDev& L = c->lev[l];
    // every candidate's time, in search order; the first one within
    // kTuneSlack of the fastest wins, so that shapes whose times differ by
    // less than the timing noise do not trade places from run to run
    struct Cand {
      float ms;
      TileShape shape;
      size_t tiles;   // index into tables
    };
    std::vector<Cand> cands;
    std::vector<std::vector<TileDev>> tables;
    const TileShape shape0 = L.shape;
    const std::vector<TileDev> tiles0 = L.tiles;
    for (int tx : {kTileMaxX, kTileDefaultX, 32})
    for (int threads : {256, 512})
    for (int slots : {2, 1})
    for (int tz : kTuneTz) {
      if (!stage_variant_ok(slots, 2, threads)) continue;
      TileShape sh = L.shape;
      sh.tx = tx;
      sh.tz = tz;
      sh.slots = slots;
      sh.threads = threads;
      std::vector<TileDev> tl;
      for (int ib = 0; ib < (int)L.boxes.size(); ++ib) {
        const BoxDev& B = L.boxes[ib];
        const int64_t o[3] = {0, 0, 0}, n[3] = {B.nx, B.ny, B.nz};
        tile_region(ib, o, n, sh, &tl);
      }
      if (tl.size() > L.tiles_capacity) continue;
      HIPCHK(c, upload(c, L.d_tiles, tl));
      L.tiles = tl;
      tables.push_back(tl);
      for (int depth : {1, 2})
      for (int g : {2 * ncu, 3 * ncu, 4 * ncu, 8 * ncu, 1 << 30}) {
        if (!stage_variant_ok(slots, depth, threads)) break;
        sh.grid = std::min<int>(g, (int)tl.size());
        sh.depth = depth;
        L.shape = sh;
        // one RK4 step's four stage launches on the bound data (stage s reads
        // y_n, k_{s-1} and a halo table, writes k_s; stage 4 writes the
        // state buffer the next step writes anyway)
        const void* yn = L.y[L.cur];
        auto rk_stages = [&]() -> int {
          for (int st = 1; st <= 4; ++st) {
            const void* table = (c->wave_mixed && st == 1) ? (const void*)L.Yd[0] : L.Yh[0];
            const int r2 = enqueue_stage_launches(c, (int)l, st, false, yn,
                                                  st == 1 ? nullptr : L.k[st - 2], table);
            if (r2) return r2;
          }
          return SC_OK;
        };
        if ((rc = rk_stages())) return rc;
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r)
          if ((rc = rk_stages())) return rc;
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        cands.push_back({ms, sh, tables.size() - 1});
        if (g >= (int)tl.size()) break;
      }
    }
    L.shape = shape0;
    L.tiles = tiles0;
    if (!cands.empty()) {
      float best = cands[0].ms;
      for (const Cand& k : cands) best = std::min(best, k.ms);
      for (const Cand& k : cands)
        if (k.ms <= best * (1.0f + kTuneSlack)) {
          L.shape = k.shape;
          L.tiles = tables[k.tiles];
          break;
        }
    }
    HIPCHK(c, upload(c, L.d_tiles, L.tiles));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->profiling = prof;
  drop_graphs(c);
  return SC_OK;
}

int sc_tile_shape(const sc_ctx* c, int32_t level, int32_t out[8]) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (level < 0 || level >= (int)c->lev.size() || !out) return SC_E_ARG;
  const LevelDev& L = c->lev[level];
  out[0] = 0;
  out[1] = 0;
  for (const TileDev& t : L.tiles) {
    out[0] = std::max<int32_t>(out[0], t.nx);
    out[1] = std::max<int32_t>(out[1], t.ny);
  }
  out[2] = L.shape.tz;
  // the launched grid: Z4c one workgroup per tile; the stencil kernel its
  // persistent grid, both rounded up to a multiple of the XCD count
  out[3] = c->cfg.rhs == SC_RHS_Z4C
               ? z4c_grid((int)L.tiles.size())
               : (std::min<int>((int)L.tiles.size(), L.shape.grid > 0 ? L.shape.grid : c->grid_cap) +
                  7) / 8 * 8;
  out[4] = (int32_t)L.tiles.size();
  out[5] = L.shape.depth;
  out[6] = L.shape.slots;
  out[7] = L.shape.threads;
  return SC_OK;
}

int sc_profile_enable(sc_ctx* c, int32_t on) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (on && c->cfg.exec == SC_EXEC_GRAPH)
    return fail(c, SC_E_STATE, "kernel timing needs an eager execution mode");
  c->profiling = on != 0;
  c->ev_used = 0;
  c->ev_launches = 0;
  c->ev_bytes.clear();
  return SC_OK;
}

int sc_profile_read(sc_ctx* c, int64_t* nlaunches, double* total_ms, double* alg_bytes) {
  int rc = check_ready(c, 2);
  if (rc) return rc;
  if (!nlaunches || !total_ms || !alg_bytes) return fail(c, SC_E_ARG, "null output");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ms = 0.0, bytes = 0.0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[i], c->ev_pool[i + 1]));
    ms += t;
  }
  for (double b : c->ev_bytes) bytes += b;
  *nlaunches = c->ev_launches;
  *total_ms = ms;
  *alg_bytes = bytes;
  c->ev_used = 0;
  c->ev_launches = 0;
  c->ev_bytes.clear();
  return SC_OK;
}

int sc_stats(const sc_ctx* c, int64_t* updates_per_coarse_step, int64_t* launches) {
  int rc = check_ready(c, 1);
  if (rc) return rc;
  if (updates_per_coarse_step) {
    int64_t u = 0;
    if (c->cfg.time_stepping == SC_UNIFORM_DT)
      for (const LevelDev& L : c->lev) u += L.owned_member;
    else
      u = c->hier.updates_per_coarse_step();
    *updates_per_coarse_step = u * c->hier.geo.nmembers;
  }
  if (launches) *launches = c->launches;
  return SC_OK;
}

}  // extern "C"
