// Device-side tables and kernel entry points.
//
// Storage on the GPU: every box of a level (for every ensemble member) is
// one padded array per variable, owned points plus G halo layers per side
// (BoxDev::pad; 3 for the fourth-order stencils, 4 for the eighth-order
// wave), x fastest, row pitch px = nx + 2G, plane pitch px * (ny + 2G).  The
// blocks of a box are index ranges of that array, so a ghost point shared
// between two blocks of the same box is simply the neighbour's owned point:
// on one GPU the block-boundary exchange costs nothing.  Only the box halo
// is ever written by a ghost fill.
//
// Per level and variable the arrays are: the state y (two buffers, swapped
// every step), the slopes k1..k4, and the halo tables Yh: one per (substep,
// stage) on refinement levels (8), holding the stage ghost values produced
// by prolongation, and one on level 0 for the periodic/intra-level copies.
// Wave right-hand side in mixed precision: the stage-1 tables are FP64 (Yd,
// one per substep) and the tables of stages 2-4 hold the FP32 stage
// increments Y_s - Y_1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sc {

constexpr int kG = 3;   // stencil radius of the fourth-order kernels (their ghost width)

struct BoxDev {
  int64_t base;         // offset of the padded array within the level arrays
  int32_t nx, ny, nz;   // owned extents
  int32_t px, py;       // padded row and plane pitches (nx + 2 pad, ny + 2 pad)
  int32_t lo[3];        // global index of owned point (0,0,0)
  int32_t wrapN[3];     // >0: this box spans a periodic dimension of N points
  int32_t pad;          // ghost layers around the owned points (the context's G)
};

struct TileDev {
  int32_t box;
  int32_t x0, y0, z0;   // box-local owned coordinates of the tile origin
  int32_t nx, ny, nz;
  int32_t dir;          // stage kernel z marching direction: 0 upward, 1 downward
};

struct SyncEntry {      // halo point <- owned point of the same level
  int64_t dst, src;     // offsets within the level arrays
};

struct ProlongEntry {   // refinement-boundary halo point
  int64_t dst;          // offset within the fine level arrays (or output index)
  int32_t q[3];         // global fine index (wrapped)
  int32_t pbox;         // parent box holding the whole prolongation stencil
};

// A brick of refinement-boundary halo points of one fine box: the fine
// index range [a, a + n), the parent box holding every stencil of its RB
// points, and a bitmask of which points are RB slots (bit (z * n_y + y) *
// n_x + x).  Bricks are face slabs of the RB shell (its full thickness by at
// most kBrickDim points along the face), edge pieces and corners; the parent
// region under a brick, its x-interpolated and its xy-interpolated planes
// must fit the LDS and per-thread limits below (brick_fits).
constexpr int kBrickThreads = 512;
constexpr int kBrickDim = 17;                      // fine points per dimension
constexpr int kBrickPts = 3 * kBrickThreads;       // fine points per brick
constexpr int kBrickV = 4 * kBrickThreads;         // parent points under a brick
constexpr int kBrickPX = 4 * kBrickThreads;        // after the x pass
constexpr int kBrickPY = 5 * kBrickThreads;        // after the y pass
constexpr int kBrickLds = 6144;                    // V + PX + PY doubles
struct ProlongBrick {
  int32_t fbox, pbox;
  int32_t a[3];
  int32_t n[3];
  uint64_t mask[kBrickPts / 64];
};

// Parent points per dimension under the fine range [a, a + n) (a >= 0): from
// the first stencil start to the last stencil end of the degree-5 operator.
inline __host__ __device__ int brick_parent_first(int a) { return (a >> 1) - 2; }
inline __host__ __device__ int brick_parent_count(int a, int n) {
  return ((a + n - 1) >> 1) + 3 - brick_parent_first(a) + 1;
}
inline bool brick_fits(const int a[3], const int n[3]) {
  int cn[3];
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 1 || n[d] > kBrickDim) return false;
    cn[d] = brick_parent_count(a[d], n[d]);
  }
  const int nv = cn[0] * cn[1] * cn[2], npx = cn[2] * cn[1] * n[0], npy = cn[2] * n[1] * n[0];
  return n[0] * n[1] * n[2] <= kBrickPts && nv <= kBrickV && npx <= kBrickPX &&
         npy <= kBrickPY && nv + npx + npy <= kBrickLds;
}

struct RestrictRegion {
  int32_t fbox, pbox;
  int32_t c0[3];        // first parent index (global)
  int32_t n[3];         // parent points per dimension
  int64_t start;        // prefix count of parent points before this region
};

constexpr int kMaxOut = 8;

// Stencil operands are FP64 in SC_FP64 mode.  In SC_MIXED mode stage 1
// reads the FP64 y_n and an FP64 halo table and stores an FP32 k1; stages
// 2-4 read the FP32 k_{s-1} and FP32 increment tables (the `void` pointers
// below hold those types); the state, the RK4 combination and everything on
// the refinement boundary stay FP64.
struct StageArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t stage;
  const BoxDev* boxes;
  const void* yn;      // stencil operand: y_n (unused by the increment form)
  const void* kprev;   // stencil operand: k_{s-1}
  const void* Yh;      // halo table of this (substep, stage)
  const void* k1;
  const void* k2;
  const void* k3;
  void* kout;          // k_s
  const double* yn64;  // FP64 y_n for the final combination (stage 4)
  double* ynew;        // FP64 y_{n+1} (stage 4)
  int64_t vstride;
  double cdt;    // c_s * dt: interior stage vector Y = y_n + cdt * k_{s-1}
  double dt6;    // dt / 6
  double clap;   // 1 / (12 h^2) (radius 3) or 1 / (5040 h^2) (radius 4)
  double cko;    // sigma / (64 h)
  int32_t write_k;
  int32_t radius;  // stencil radius: 3 (fourth order) or 4 (eighth order, FP64); the
                   // boxes must be padded by at least this much
  unsigned int* nonfinite;   // set to 1 when stage 4 writes a non-finite y_{n+1}
};

struct SyncArgs {
  const SyncEntry* e;
  int64_t n;
  const void* yn;
  const void* kprev;   // null: copy y_n
  void* out;
  int64_t vstride;
  double cdt;
  int32_t nvars;
  int32_t inc;         // 1: copy the stage increment cdt * k_{s-1} (mixed wave)
};

struct ProlongArgs {
  const ProlongEntry* e;
  int64_t n;
  // entries are sorted by parity class (odd x = 1, odd y = 2, odd z = 4):
  // class c occupies [cls_start[c], cls_start[c+1]) and workgroups
  // [blk_start[c], blk_start[c+1])
  int64_t cls_start[9];
  int32_t blk_start[9];
  const BoxDev* pboxes;          // parent level boxes
  const double* py;              // parent y_n (FP64)
  const void* pk[4];             // parent k1..k4 (FP64, or FP32 in mixed mode); see nin
  int64_t pvstride;
  void* out[kMaxOut];            // outputs, one per combination
  int64_t ovstride;
  double w[kMaxOut][4];          // dense-output weights per combination
  double H;                      // parent time step
  int32_t nout;
  int32_t nvars;
  uint32_t f32_mask;             // bit o: output o is FP32 (else FP64)
  uint32_t inc_mask;             // bit o: output o omits P[y_n] (a stage increment)
};

struct BrickArgs {
  const ProlongBrick* b;
  int32_t nbricks;
  int32_t max_pts;     // largest n_x n_y n_z over the bricks (picks the kernel variant)
  int32_t nout;
  int32_t nvars;
  const BoxDev* fboxes;
  const BoxDev* pboxes;
  const double* py;
  const void* pk[4];
  int64_t pvstride;
  void* out[kMaxOut];
  int64_t ovstride;
  double w[kMaxOut][4];
  double H;
  uint32_t f32_mask;   // as in ProlongArgs
  uint32_t inc_mask;
};

struct RestrictArgs {
  const RestrictRegion* r;
  int32_t nregions;
  int64_t ntotal;
  const BoxDev* fboxes;
  const BoxDev* pboxes;
  const double* fy;
  double* py;
  float* py32;            // parent FP32 shadow (mixed) or null
  int64_t fvstride, pvstride;
  int32_t nvars;
};

struct PackArgs {
  const BoxDev* boxes;    // boxes of one member of one level
  const int64_t* prefix;  // nboxes + 1 canonical prefix counts (device)
  int32_t nboxes;
  int64_t n;
  void* arr;              // level array of the variable (already offset by var)
  double* buf;            // canonical buffer
};

// Closed-form initial data evaluated on the device (sc_set_initial_data_analytic).
constexpr int kInitParams = 6 + 5 * 32;
struct InitArgs {
  int32_t kind;           // SC_ID_*
  int32_t nvars;
  const BoxDev* boxes;    // boxes of one member of one level
  const int64_t* prefix;  // canonical prefix counts (device)
  int32_t nboxes;
  int64_t n;              // points to evaluate
  const int64_t* idx;     // null: the member's owned points in canonical order;
                          // else level-array offsets of halo points
  double origin[3];
  double dx;
  int32_t var;            // halo points: the variable evaluated
  double* out;            // owned points: the level array of variable 0 (variables
                          // vstride apart); halo points: n values of variable var
  float* out32;           // FP32 shadow of the owned points (Z4c mixed) or null
  int64_t vstride;
  double p[kInitParams];  // the kind's parameters (see sc_set_initial_data_analytic)
};

// Deterministic reductions over the owned points of one member of a level
// (see k_norms_partial): per point a value v and a weight w (1 unless mode 2);
// the result is {max |v|, sum w v^2, sum w, non-finite count}.
//   mode 0: v = the array's value
//   mode 1: v = the array's value minus the closed form `exact` (variable exact.var)
//   mode 2: v = the array's value (a constraint), w = cell at points that no child box
//           covers, with r < rmax and the lapse alpha > amin, else the point is skipped
constexpr int64_t kNormPointsPerPart = 8192;   // points per partial workgroup
struct NormArgs {
  PackArgs p;             // the points (p.arr: the level array of the variable)
  int32_t mode;
  InitArgs exact;         // modes 1, 2: origin and dx (mode 1: the closed form)
  const double* alpha;    // mode 2: the lapse (level array)
  const BoxDev* child;    // mode 2: boxes of the finer level (same member)
  int32_t nchild;
  double rmax, amin, cell;
};
// partial workgroups of a reduction over n points (the partials array holds 4 per part)
int norm_parts(int64_t n);
// Static reduction workspace (no allocation): partials of at most
// kNoAllocParts workgroups, then the 4-double result.  noalloc_scratch gives
// the current device's address of it (looked up once per device).
constexpr int kNoAllocParts = 4096;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(double** out);

// launchers (kernels.hip); `f32` selects FP32 arrays
// mixed: the mixed-precision stage kernels (see StageArgs)
// depth: planes of loads in flight (1 or 2); slots: owned points per thread (1 or 2);
// threads: 256 or 512 per workgroup; the tiles must have been cut for slots and threads
hipError_t launch_stage(const StageArgs& a, int grid, bool mixed, int depth, int slots, int threads,
                        hipStream_t s);
hipError_t launch_sync(const SyncArgs& a, bool f32, hipStream_t s);
// k_f32: parent slopes are FP32; output types and forms in the args' masks
// nin: 5 = (y_n, k1..k4) with dense-output weights; 3 = (y_n, y_{n-1}, y_{n+1})
// with time-interpolation weights w[o][0..2] on (y_{n-1}, y_n, y_{n+1}) (pk[0] =
// y_{n-1}, pk[1] = y_{n+1}, FP64); 1 = y_n alone
hipError_t launch_prolong(const ProlongArgs& a, bool k_f32, hipStream_t s, int nin = 5);
hipError_t launch_prolong_bricks(const BrickArgs& a, bool k_f32, hipStream_t s, int nin = 5);
// dst[i] = base[idx[i]] + inc[idx[i]] (stage value from stage-1 and increment tables)
hipError_t launch_gather_sum(const int64_t* idx, int64_t n, const double* base, const float* inc,
                             double* dst, hipStream_t s);
// dst[idx[i]] = v
hipError_t launch_scatter_value(const int64_t* idx, int64_t n, double v, void* dst, bool f32,
                                hipStream_t s);
hipError_t launch_restrict(const RestrictArgs& a, hipStream_t s);
hipError_t launch_pack(const PackArgs& a, bool unpack, bool f32, hipStream_t s);
// out: 4 doubles {max, sum, weight sum, non-finite count}
hipError_t launch_norms(const NormArgs& a, bool f32, double* partials, double* out, hipStream_t s);
hipError_t launch_gather(const int64_t* idx, int64_t n, const void* src, bool f32, double* dst,
                         hipStream_t s);
hipError_t launch_fill(void* p, int64_t n, double v, bool f32, hipStream_t s);
hipError_t launch_scatter(const int64_t* idx, int64_t n, const double* src, void* dst, bool f32,
                          hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s);
hipError_t launch_init(const InitArgs& a, hipStream_t s);

// Stencil-kernel workgroup families: threads, ring points per thread and plane,
// and LDS window capacity per variable and plane ((nx+6)(ny+6) points).  The
// wide family runs one larger tile per CU: a smaller ring per owned point and
// fewer tiles sharing each XCD's L2.
template <int NT> struct StageFamily;
template <> struct StageFamily<256> { static constexpr int ring = 2, wincap = 1024; };
template <> struct StageFamily<512> { static constexpr int ring = 1, wincap = 1600; };
constexpr int kStageThreads = 256;   // the default family (per-block mode uses it)
constexpr int kStageSlotsMax = 2;    // owned points per thread and plane of a stencil tile (1 or 2)
inline int stage_ring_slots(int threads) { return threads == 512 ? 1 : 2; }
inline int stage_win_cap(int threads) { return threads == 512 ? 1600 : 1024; }
constexpr int kTileMaxX = 128;    // widest stencil tile (points in x; the LDS window and ring
                                  // slots cap it lower, at 78 for radius 3)
constexpr int kTileDefaultX = 64; // widest tile of a context's untuned shape

}  // namespace sc
