// Block hierarchy and index maps (host side, built once per context).
//
// Levels are nested vertex-centred grids with refinement ratio 2 (the
// paper's algorithm summary in Sec. II).  Each level box is cut into blocks,
// the unit at which the paper's driver exchanges ghost zones between
// processes; a block's ghost zone is filled from another block of the same
// level (SYNC), from the parent level at a refinement boundary (RB), or by
// the physical boundary (PHYS).  The refinement-boundary ghost width equals
// the block-boundary ghost width, which is the point of the method.
//
// Buffer zones (the Carpet scheme the paper compares against, Sec. II and
// Fig. 1): with a buffer width B > 0 the buffer points of a fine level are its
// owned points within Chebyshev distance B of one of its RB points; they are
// refilled from the parent before every fine step and never restricted, and
// the parent points that prolongation reads must not be buffer points.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace sc {

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the block split draws one
// stream per level; seeded initial data draw their parameters from it.
struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }   // top 53 bits
};

enum GhostKind : int8_t { kSync = 0, kRb = 1, kPhys = 2 };

struct IBox {
  int64_t lo[3], hi[3];
  int64_t n(int d) const { return hi[d] - lo[d] + 1; }
  int64_t volume() const { return n(0) * n(1) * n(2); }
  bool contains(const int64_t q[3]) const {
    return q[0] >= lo[0] && q[0] <= hi[0] && q[1] >= lo[1] && q[1] <= hi[1] && q[2] >= lo[2] &&
           q[2] <= hi[2];
  }
};

struct LevelMaps {
  int level = 0;
  int64_t N[3] = {0, 0, 0};   // domain extent in cells at this level
  bool periodic[3] = {false, false, false};
  std::vector<IBox> boxes;    // the level's boxes (level 0: the whole domain)
  std::vector<IBox> blocks;   // block id order
  std::vector<int32_t> block_box;
  std::vector<std::vector<int32_t>> lut;  // per box: block id of every owned point
  int64_t nowned = 0;
  // ghost slots of every block in visiting order, concatenated
  std::vector<int64_t> ghost_start;  // nblocks + 1
  std::vector<int8_t> gkind;
  std::vector<int64_t> ga, gc;       // SYNC: owner, offset; RB: rb index, 0; PHYS: -1, 0
  std::vector<std::array<int64_t, 3>> rb;  // distinct RB points sorted by (z, y, x)
  std::vector<std::array<int64_t, 4>> restrict_pairs;  // [pblock, poffset, block, offset]
  std::vector<std::array<int64_t, 3>> buffer;  // buffer points sorted by (z, y, x)
  std::vector<int64_t> buffer_keys;            // their keys, ascending
  bool is_buffer(const int64_t q[3]) const;

  void wrap(const int64_t p[3], int64_t q[3]) const;
  bool outside(const int64_t q[3]) const;
  // owner block of a wrapped point and the offset within it; false if unowned
  bool owner(const int64_t q[3], int32_t* block, int64_t* offset) const;
  // index of the box holding a wrapped point, -1 if none
  int box_of(const int64_t q[3]) const;
};

struct Geometry {
  int32_t nmembers = 1;
  double origin[3] = {0, 0, 0};
  double dx0 = 1.0;
  int64_t ncells0[3] = {0, 0, 0};
  bool periodic[3] = {false, false, false};
  int32_t nlevels = 1;
  std::vector<std::vector<IBox>> fine_boxes;  // levels 1..
};

struct Hierarchy {
  Geometry geo;
  int G = 3;
  int B = 0;   // buffer width (0: no buffer zones)
  std::vector<LevelMaps> levels;

  // Returns an empty string on success, else the reason; *nest_error tells a
  // nesting/alignment violation from a plain argument error.
  std::string build(const Geometry& g, int G, uint64_t block_seed, int min_block,
                    int max_block, bool* nest_error, int buffer = 0);
  void export_words(std::vector<int64_t>* out) const;
  int64_t updates_per_coarse_step() const;
};

}  // namespace sc
