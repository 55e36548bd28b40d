// Block split, ghost classification, refinement-boundary lists, restriction
// pairs, nesting checks and the canonical map export.
#include "hierarchy.hpp"

#include <algorithm>
#include <cstdio>

namespace sc {

namespace {

// Recursive cut along the longest side (ties: lowest axis), left part first.
void split_box(const IBox& b, SplitMix64& rng, int64_t min_block, int64_t max_block,
               std::vector<IBox>* out) {
  int64_t n[3] = {b.n(0), b.n(1), b.n(2)};
  int64_t m = std::max(n[0], std::max(n[1], n[2]));
  if (m <= max_block) {
    out->push_back(b);
    return;
  }
  int d = (n[0] == m) ? 0 : (n[1] == m ? 1 : 2);
  uint64_t span = (uint64_t)(n[d] - 2 * min_block + 1);
  int64_t s = min_block + (int64_t)(rng.next() % span);
  IBox left = b, right = b;
  left.hi[d] = b.lo[d] + s - 1;
  right.lo[d] = b.lo[d] + s;
  split_box(left, rng, min_block, max_block, out);
  split_box(right, rng, min_block, max_block, out);
}

inline int64_t rb_key(const int64_t q[3]) { return (q[2] << 42) | (q[1] << 21) | q[0]; }

inline int64_t floordiv2(int64_t a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

}  // namespace

void LevelMaps::wrap(const int64_t p[3], int64_t q[3]) const {
  for (int d = 0; d < 3; ++d) {
    q[d] = p[d];
    if (periodic[d]) q[d] = ((p[d] % N[d]) + N[d]) % N[d];
  }
}

bool LevelMaps::outside(const int64_t q[3]) const {
  for (int d = 0; d < 3; ++d)
    if (!periodic[d] && (q[d] < 0 || q[d] > N[d])) return true;
  return false;
}

int LevelMaps::box_of(const int64_t q[3]) const {
  for (size_t i = 0; i < boxes.size(); ++i)
    if (boxes[i].contains(q)) return (int)i;
  return -1;
}

bool LevelMaps::is_buffer(const int64_t q[3]) const {
  return std::binary_search(buffer_keys.begin(), buffer_keys.end(), rb_key(q));
}

bool LevelMaps::owner(const int64_t q[3], int32_t* block, int64_t* offset) const {
  int ib = box_of(q);
  if (ib < 0) return false;
  const IBox& bx = boxes[ib];
  int64_t l = ((q[2] - bx.lo[2]) * bx.n(1) + (q[1] - bx.lo[1])) * bx.n(0) + (q[0] - bx.lo[0]);
  int32_t b = lut[ib][l];
  const IBox& bl = blocks[b];
  *block = b;
  *offset = ((q[2] - bl.lo[2]) * bl.n(1) + (q[1] - bl.lo[1])) * bl.n(0) + (q[0] - bl.lo[0]);
  return true;
}

// Buffer points of one level: per box, mark the RB points that fall in the
// window [lo - B, hi + B] (each RB point at every periodic image), dilate the
// marks by B along x, y and z in turn with running counts, and keep the
// marked box points.
static void find_buffer(LevelMaps& L, int B) {
  std::vector<std::array<int64_t, 3>> pts;
  for (const IBox& bx : L.boxes) {
    int64_t n[3], lo[3];
    for (int d = 0; d < 3; ++d) {
      n[d] = bx.n(d) + 2 * B;
      lo[d] = bx.lo[d] - B;
    }
    std::vector<uint8_t> m((size_t)(n[0] * n[1] * n[2]), 0), t(m.size());
    for (const auto& q : L.rb) {
      // window coordinates of q and of its periodic images
      int64_t c[3][3];
      int nc[3];
      for (int d = 0; d < 3; ++d) {
        nc[d] = 0;
        const int nk = L.periodic[d] ? 1 : 0;
        for (int k = -nk; k <= nk; ++k) {
          const int64_t v = q[d] + k * L.N[d] - lo[d];
          if (v >= 0 && v < n[d]) c[d][nc[d]++] = v;
        }
      }
      for (int a = 0; a < nc[2]; ++a)
        for (int b = 0; b < nc[1]; ++b)
          for (int e = 0; e < nc[0]; ++e) m[(size_t)((c[2][a] * n[1] + c[1][b]) * n[0] + c[0][e])] = 1;
    }
    const int64_t stride[3] = {1, n[0], n[0] * n[1]};
    for (int d = 0; d < 3; ++d) {
      // t = 1 where some mark lies within B along axis d
      const int64_t nd = n[d], sd = stride[d];
      const int64_t nlines = (int64_t)m.size() / nd;
      for (int64_t line = 0; line < nlines; ++line) {
        // base of the line: decompose the line index over the other two axes
        int64_t base;
        if (d == 0) base = line * n[0];
        else if (d == 1) base = (line / n[0]) * n[0] * n[1] + line % n[0];
        else base = line;
        int cnt = 0;
        for (int64_t k = 0; k < std::min<int64_t>(B, nd); ++k) cnt += m[base + k * sd];
        for (int64_t k = 0; k < nd; ++k) {
          if (k + B < nd) cnt += m[base + (k + B) * sd];
          if (k - B - 1 >= 0) cnt -= m[base + (k - B - 1) * sd];
          t[base + k * sd] = cnt > 0;
        }
      }
      m.swap(t);
    }
    for (int64_t z = 0; z < bx.n(2); ++z)
      for (int64_t y = 0; y < bx.n(1); ++y)
        for (int64_t x = 0; x < bx.n(0); ++x)
          if (m[(size_t)(((z + B) * n[1] + (y + B)) * n[0] + (x + B))])
            pts.push_back({bx.lo[0] + x, bx.lo[1] + y, bx.lo[2] + z});
  }
  std::sort(pts.begin(), pts.end(), [](const std::array<int64_t, 3>& a, const std::array<int64_t, 3>& b) {
    return rb_key(a.data()) < rb_key(b.data());
  });
  L.buffer = pts;
  L.buffer_keys.resize(pts.size());
  for (size_t k = 0; k < pts.size(); ++k) L.buffer_keys[k] = rb_key(pts[k].data());
}

std::string Hierarchy::build(const Geometry& g, int G_, uint64_t block_seed, int min_block,
                             int max_block, bool* nest_error, int buffer) {
  geo = g;
  G = G_;
  B = buffer;
  *nest_error = false;
  char msg[256];
  if (max_block < 2 * min_block - 1 || min_block < 1)
    return "max_block must be at least 2*min_block-1 and min_block >= 1";
  if (buffer < 0) return "buffer width must be >= 0";
  levels.assign(g.nlevels, LevelMaps());
  // ---- boxes, alignment, containment, overlap
  for (int l = 0; l < g.nlevels; ++l) {
    LevelMaps& L = levels[l];
    L.level = l;
    for (int d = 0; d < 3; ++d) {
      L.N[d] = g.ncells0[d] << l;
      L.periodic[d] = g.periodic[d];
    }
    if (l == 0) {
      IBox b;
      for (int d = 0; d < 3; ++d) {
        b.lo[d] = 0;
        b.hi[d] = g.periodic[d] ? g.ncells0[d] - 1 : g.ncells0[d];
      }
      L.boxes.push_back(b);
    } else {
      L.boxes = g.fine_boxes[l - 1];
      for (const IBox& b : L.boxes) {
        for (int d = 0; d < 3; ++d) {
          bool full = g.periodic[d] && b.lo[d] == 0 && b.hi[d] == L.N[d] - 1;
          if (!full && ((b.lo[d] & 1) || (b.hi[d] & 1))) {
            *nest_error = true;
            snprintf(msg, sizeof msg, "level %d: box bounds must be even", l);
            return msg;
          }
          int64_t top = g.periodic[d] ? L.N[d] - 1 : L.N[d];
          if (b.lo[d] < 0 || b.hi[d] > top || b.lo[d] > b.hi[d]) {
            *nest_error = true;
            snprintf(msg, sizeof msg, "level %d: box outside the domain", l);
            return msg;
          }
        }
      }
      for (size_t i = 0; i < L.boxes.size(); ++i)
        for (size_t j = i + 1; j < L.boxes.size(); ++j) {
          const IBox &a = L.boxes[i], &b = L.boxes[j];
          bool ov = true;
          for (int d = 0; d < 3; ++d) ov = ov && a.lo[d] <= b.hi[d] && b.lo[d] <= a.hi[d];
          if (ov) {
            *nest_error = true;
            snprintf(msg, sizeof msg, "level %d: boxes overlap", l);
            return msg;
          }
        }
    }
    for (const IBox& b : L.boxes)
      for (int d = 0; d < 3; ++d)
        if (b.n(d) < min_block) {
          *nest_error = true;
          snprintf(msg, sizeof msg, "level %d: box side shorter than min_block", l);
          return msg;
        }
  }
  // ---- block split and owner lookup tables
  for (int l = 0; l < g.nlevels; ++l) {
    LevelMaps& L = levels[l];
    SplitMix64 rng(block_seed + (uint64_t)l);
    for (size_t ib = 0; ib < L.boxes.size(); ++ib) {
      std::vector<IBox> sub;
      split_box(L.boxes[ib], rng, min_block, max_block, &sub);
      for (const IBox& b : sub) {
        L.blocks.push_back(b);
        L.block_box.push_back((int32_t)ib);
        L.nowned += b.volume();
      }
    }
    L.lut.resize(L.boxes.size());
    for (size_t ib = 0; ib < L.boxes.size(); ++ib) {
      const IBox& bx = L.boxes[ib];
      L.lut[ib].assign((size_t)bx.volume(), -1);
    }
    for (size_t b = 0; b < L.blocks.size(); ++b) {
      const IBox& bl = L.blocks[b];
      const IBox& bx = L.boxes[L.block_box[b]];
      for (int64_t z = bl.lo[2]; z <= bl.hi[2]; ++z)
        for (int64_t y = bl.lo[1]; y <= bl.hi[1]; ++y)
          for (int64_t x = bl.lo[0]; x <= bl.hi[0]; ++x)
            L.lut[L.block_box[b]][((z - bx.lo[2]) * bx.n(1) + (y - bx.lo[1])) * bx.n(0) +
                                  (x - bx.lo[0])] = (int32_t)b;
    }
  }
  // ---- ghost classification and RB lists
  for (int l = 0; l < g.nlevels; ++l) {
    LevelMaps& L = levels[l];
    L.ghost_start.assign(L.blocks.size() + 1, 0);
    std::vector<int64_t> rbkeys;
    std::vector<size_t> rbslot;
    for (size_t b = 0; b < L.blocks.size(); ++b) {
      const IBox& bl = L.blocks[b];
      L.ghost_start[b] = (int64_t)L.gkind.size();
      int64_t p[3], q[3];
      for (p[2] = bl.lo[2] - G; p[2] <= bl.hi[2] + G; ++p[2])
        for (p[1] = bl.lo[1] - G; p[1] <= bl.hi[1] + G; ++p[1])
          for (p[0] = bl.lo[0] - G; p[0] <= bl.hi[0] + G; ++p[0]) {
            if (bl.contains(p)) continue;
            L.wrap(p, q);
            int32_t ob;
            int64_t off;
            if (L.outside(q)) {
              L.gkind.push_back(kPhys);
              L.ga.push_back(-1);
              L.gc.push_back(0);
            } else if (L.owner(q, &ob, &off)) {
              L.gkind.push_back(kSync);
              L.ga.push_back(ob);
              L.gc.push_back(off);
            } else {
              if (l == 0) {
                *nest_error = true;
                return "level 0 has unowned ghost points";
              }
              rbslot.push_back(L.gkind.size());
              rbkeys.push_back(rb_key(q));
              L.gkind.push_back(kRb);
              L.ga.push_back(0);
              L.gc.push_back(0);
            }
          }
    }
    L.ghost_start[L.blocks.size()] = (int64_t)L.gkind.size();
    std::vector<int64_t> uk = rbkeys;
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    for (size_t i = 0; i < rbslot.size(); ++i)
      L.ga[rbslot[i]] = std::lower_bound(uk.begin(), uk.end(), rbkeys[i]) - uk.begin();
    L.rb.resize(uk.size());
    const int64_t m21 = (int64_t(1) << 21) - 1;
    for (size_t i = 0; i < uk.size(); ++i)
      L.rb[i] = {uk[i] & m21, (uk[i] >> 21) & m21, uk[i] >> 42};
  }
  if (B > 0)
    for (int l = 1; l < g.nlevels; ++l) find_buffer(levels[l], B);
  // ---- nesting of prolongation stencils: each RB (and buffer) point's
  //      stencil must lie in one parent box (periodic dimensions spanned by
  //      that box wrap) and, with buffer zones, avoid the parent's buffer points
  for (int l = 1; l < g.nlevels; ++l) {
    const LevelMaps& P = levels[l - 1];
    std::vector<std::array<int64_t, 3>> pts = levels[l].rb;
    pts.insert(pts.end(), levels[l].buffer.begin(), levels[l].buffer.end());
    // parent buffer points per parent box as summed-volume tables, so that a
    // stencil's box is tested in O(1)
    std::vector<std::vector<int32_t>> sat(P.buffer.empty() ? 0 : P.boxes.size());
    for (size_t ib = 0; ib < sat.size(); ++ib) {
      const IBox& b = P.boxes[ib];
      const int64_t n0 = b.n(0) + 1, n1 = b.n(1) + 1, n2 = b.n(2) + 1;
      std::vector<int32_t>& S = sat[ib];
      S.assign((size_t)(n0 * n1 * n2), 0);
      for (const auto& c : P.buffer) {
        if (!b.contains(c.data())) continue;
        S[(size_t)(((c[2] - b.lo[2] + 1) * n1 + (c[1] - b.lo[1] + 1)) * n0 + (c[0] - b.lo[0] + 1))] = 1;
      }
      for (int64_t z = 1; z < n2; ++z)
        for (int64_t y = 1; y < n1; ++y)
          for (int64_t x = 1; x < n0; ++x) {
            auto at = [&](int64_t zz, int64_t yy, int64_t xx) -> int32_t& {
              return S[(size_t)((zz * n1 + yy) * n0 + xx)];
            };
            at(z, y, x) += at(z - 1, y, x) + at(z, y - 1, x) + at(z, y, x - 1) - at(z - 1, y - 1, x) -
                           at(z - 1, y, x - 1) - at(z, y - 1, x - 1) + at(z - 1, y - 1, x - 1);
          }
    }
    // buffer points of parent box ib in the box-local ranges [a, b] (inclusive)
    auto count = [&](size_t ib, const int64_t a[3], const int64_t b[3]) -> int64_t {
      const IBox& bx = P.boxes[ib];
      const int64_t n0 = bx.n(0) + 1, n1 = bx.n(1) + 1;
      const std::vector<int32_t>& S = sat[ib];
      auto at = [&](int64_t z, int64_t y, int64_t x) -> int64_t { return S[(size_t)((z * n1 + y) * n0 + x)]; };
      const int64_t x0 = a[0], x1 = b[0] + 1, y0 = a[1], y1 = b[1] + 1, z0 = a[2], z1 = b[2] + 1;
      return at(z1, y1, x1) - at(z0, y1, x1) - at(z1, y0, x1) - at(z1, y1, x0) + at(z0, y0, x1) +
             at(z0, y1, x0) + at(z1, y0, x0) - at(z0, y0, x0);
    };
    for (const auto& q : pts) {
      int64_t smin[3], smax[3];
      for (int d = 0; d < 3; ++d) {
        int64_t base = floordiv2(q[d]);
        smin[d] = (q[d] & 1) ? base - 2 : base;
        smax[d] = (q[d] & 1) ? base + 3 : base;
      }
      bool ok = false;
      size_t pbox = 0;
      for (size_t ib = 0; ib < P.boxes.size(); ++ib) {
        const IBox& b = P.boxes[ib];
        bool in = true;
        for (int d = 0; d < 3; ++d) {
          bool full = P.periodic[d] && b.lo[d] == 0 && b.hi[d] == P.N[d] - 1;
          if (!full) in = in && smin[d] >= b.lo[d] && smax[d] <= b.hi[d];
        }
        if (in) {
          ok = true;
          pbox = ib;
          break;
        }
      }
      if (!ok) {
        *nest_error = true;
        snprintf(msg, sizeof msg,
                 "level %d: prolongation stencil of RB point (%lld,%lld,%lld) is not inside one "
                 "parent box",
                 l, (long long)q[0], (long long)q[1], (long long)q[2]);
        return msg;
      }
      if (!P.buffer.empty()) {
        // the stencil range in box-local coordinates, split where a
        // box-spanning periodic dimension wraps
        const IBox& b = P.boxes[pbox];
        int64_t ra[3][2], rb[3][2];
        int nr[3];
        for (int d = 0; d < 3; ++d) {
          const int64_t a = smin[d] - b.lo[d], e = smax[d] - b.lo[d], n = b.n(d);
          if (a >= 0 && e < n) {
            nr[d] = 1, ra[d][0] = a, rb[d][0] = e;
          } else if (a < 0) {   // wraps below: [a + n, n - 1] and [0, e]
            nr[d] = 2, ra[d][0] = a + n, rb[d][0] = n - 1, ra[d][1] = 0, rb[d][1] = e;
          } else {              // wraps above: [a, n - 1] and [0, e - n]
            nr[d] = 2, ra[d][0] = a, rb[d][0] = n - 1, ra[d][1] = 0, rb[d][1] = e - n;
          }
        }
        int64_t hits = 0;
        for (int i = 0; i < nr[0]; ++i)
          for (int j = 0; j < nr[1]; ++j)
            for (int k = 0; k < nr[2]; ++k) {
              const int64_t a[3] = {ra[0][i], ra[1][j], ra[2][k]};
              const int64_t e[3] = {rb[0][i], rb[1][j], rb[2][k]};
              hits += count(pbox, a, e);
            }
        if (hits > 0) {
          *nest_error = true;
          snprintf(msg, sizeof msg,
                   "level %d: prolongation stencil of (%lld,%lld,%lld) reads parent buffer points",
                   l, (long long)q[0], (long long)q[1], (long long)q[2]);
          return msg;
        }
      }
    }
  }
  // ---- restriction pairs
  for (int l = 1; l < g.nlevels; ++l) {
    LevelMaps& F = levels[l];
    const LevelMaps& P = levels[l - 1];
    for (size_t b = 0; b < F.blocks.size(); ++b) {
      const IBox& bl = F.blocks[b];
      int64_t q[3], c[3];
      for (q[2] = bl.lo[2] + (bl.lo[2] & 1); q[2] <= bl.hi[2]; q[2] += 2)
        for (q[1] = bl.lo[1] + (bl.lo[1] & 1); q[1] <= bl.hi[1]; q[1] += 2)
          for (q[0] = bl.lo[0] + (bl.lo[0] & 1); q[0] <= bl.hi[0]; q[0] += 2) {
            if (!F.buffer.empty() && F.is_buffer(q)) continue;
            int64_t h[3] = {q[0] / 2, q[1] / 2, q[2] / 2};
            P.wrap(h, c);
            int32_t cb;
            int64_t coff;
            if (!P.owner(c, &cb, &coff)) {
              *nest_error = true;
              snprintf(msg, sizeof msg, "level %d: restriction target not parent-owned", l);
              return msg;
            }
            int64_t foff =
                ((q[2] - bl.lo[2]) * bl.n(1) + (q[1] - bl.lo[1])) * bl.n(0) + (q[0] - bl.lo[0]);
            F.restrict_pairs.push_back({cb, coff, (int64_t)b, foff});
          }
    }
    std::sort(F.restrict_pairs.begin(), F.restrict_pairs.end(),
              [](const std::array<int64_t, 4>& a, const std::array<int64_t, 4>& b) {
                return a[0] != b[0] ? a[0] < b[0] : a[1] < b[1];
              });
  }
  return "";
}

void Hierarchy::export_words(std::vector<int64_t>* out) const {
  std::vector<int64_t>& w = *out;
  w.clear();
  w.insert(w.end(), {0x53554243, B > 0 ? 2 : 1, geo.nlevels, geo.nmembers});
  for (const LevelMaps& L : levels) {
    w.insert(w.end(), {L.level, (int64_t)L.blocks.size(), L.nowned, (int64_t)L.rb.size(),
                       (int64_t)L.restrict_pairs.size()});
    for (const IBox& b : L.blocks)
      w.insert(w.end(), {b.lo[0], b.lo[1], b.lo[2], b.hi[0], b.hi[1], b.hi[2]});
    for (size_t i = 0; i < L.gkind.size(); ++i)
      w.insert(w.end(), {(int64_t)L.gkind[i], L.ga[i], L.gkind[i] == kSync ? L.gc[i] : 0});
    for (const auto& q : L.rb)
      w.insert(w.end(), {q[0], q[1], q[2], q[0] / 2, q[1] / 2, q[2] / 2,
                         (q[0] & 1) | ((q[1] & 1) << 1) | ((q[2] & 1) << 2)});
    for (const auto& r : L.restrict_pairs) w.insert(w.end(), {r[0], r[1], r[2], r[3]});
    if (B > 0) {
      w.push_back((int64_t)L.buffer.size());
      for (const auto& q : L.buffer)
        w.insert(w.end(), {q[0], q[1], q[2], q[0] / 2, q[1] / 2, q[2] / 2,
                           (q[0] & 1) | ((q[1] & 1) << 1) | ((q[2] & 1) << 2)});
    }
  }
}

int64_t Hierarchy::updates_per_coarse_step() const {
  int64_t u = 0;
  for (const LevelMaps& L : levels) u += L.nowned << L.level;
  return u;
}

}  // namespace sc
