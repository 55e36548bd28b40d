// Context state: device layout of the hierarchy, arena plan and scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/subcyc.h"
#include "device.hpp"
#include "hierarchy.hpp"

namespace sc {

struct TileShape {
  int tx = kTileDefaultX, ty = 1 << 20, tz = 16;   // tx, ty: caps on the tile width and height
  int grid = 0;   // persistent workgroups for the batched stage kernel (0: context default)
  int depth = 1;  // stage kernel: planes of loads in flight ahead of the computed plane
  int slots = 2;  // owned points per stage-kernel thread (tiles of at most threads * slots points)
  int threads = 256;  // stage-kernel workgroup size (256 or 512)
  int radius = 3;     // stencil radius (3: fourth order, 4: eighth order); sizes the LDS frame
};

// z-chunk depths the autotuner tries; the tile table region is sized for the
// shallowest (most tiles).  Consecutive depths up to 16 let the tile count land
// just under a whole number of rounds of resident workgroups: a tile takes a
// sizeable part of a launch, so a last round that fills few CUs costs much.
constexpr int kTuneTz[] = {4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 18, 20,
                           24, 28, 32, 40, 48, 64, 1 << 20};
constexpr int kTuneTzMin = 4;
constexpr float kTuneSlack = 0.015f;   // autotuner: candidates this close to the fastest tie
constexpr int kZ4cTzMin = 2;   // Z4c contexts cut two-plane tiles by default

struct LevelDev {
  int nb_member = 0;                 // boxes per member
  int64_t member_total = 0;          // padded points per member
  int64_t total = 0;                 // padded points, all members (variable stride)
  int64_t owned_member = 0;          // owned points per member
  int64_t nrb = 0;                   // distinct RB points per member
  std::vector<BoxDev> boxes;         // all members
  std::vector<int64_t> prefix;       // canonical prefix per member box (nb_member + 1)
  std::vector<SyncEntry> sync;
  std::vector<ProlongBrick> bricks;   // RB halo slots grouped in bricks (all members)
  int brick_max_pts = 0;              // largest brick (fine points of its index box)
  std::vector<ProlongEntry> prolong; // remaining RB halo slots, sorted by parity class
  int64_t prolong_cls[9] = {0};      // class prefix of `prolong`
  int64_t rblist_cls[9] = {0};       // class prefix of one member's `rblist`
  std::vector<ProlongEntry> rblist;  // RB list entries of every member, dst = list index j
  std::vector<int64_t> rbfirst;      // halo offset of the first slot of each RB list entry
  std::vector<int64_t> phys;         // physical-boundary halo offsets, all members
  std::vector<int64_t> phys_q;       // their global indices (member 0), xyz triples
  std::vector<RestrictRegion> restr;
  int64_t restr_total = 0;
  std::vector<TileDev> tiles;        // batched: tiles over the boxes
  size_t tiles_capacity = 0;         // tile slots reserved in the arena
  std::vector<TileDev> btiles;       // per block: tiles clipped to blocks
  std::vector<int32_t> btile_start;  // nblocks (all members) + 1
  // Z4c FP64: the derivative pass's columns over the boxes, and per block
  std::vector<TileDev> dtiles;
  std::vector<TileDev> bdtiles;
  std::vector<int32_t> bdtile_start;  // nblocks (all members) + 1
  TileShape shape;
  int nyh = 1;
  bool has_child = false;
  // arena offsets (bytes)
  size_t o_y[3], o_y32[2], o_k[4], o_yh[8], o_yd[2], o_boxes, o_prefix, o_sync, o_prolong,
      o_rblist, o_rbfirst, o_phys, o_restr, o_tiles, o_btiles, o_ys, o_bricks, o_dtiles,
      o_bdtiles;
  // device pointers after binding.  y: FP64 state; y32: its FP32 shadow
  // (Z4c mixed mode only); k and Yh hold the slope type (FP64, or FP32 in
  // mixed mode); Yd: FP64 stage-1 halo tables of the mixed wave (one per
  // substep; its Yh tables of stages 2-4 hold FP32 stage increments).
  double* y[3] = {nullptr, nullptr, nullptr};
  float* y32[2] = {nullptr, nullptr};
  void* k[4] = {nullptr, nullptr, nullptr, nullptr};
  void* Yh[8] = {nullptr};
  double* Yd[2] = {nullptr, nullptr};
  int nyd = 0;
  double* Ys = nullptr;              // Z4c: materialised stage vector
  BoxDev* d_boxes = nullptr;
  int64_t* d_prefix = nullptr;
  SyncEntry* d_sync = nullptr;
  ProlongEntry* d_prolong = nullptr;
  ProlongBrick* d_bricks = nullptr;
  ProlongEntry* d_rblist = nullptr;
  int64_t* d_rbfirst = nullptr;
  int64_t* d_phys = nullptr;
  RestrictRegion* d_restr = nullptr;
  TileDev* d_tiles = nullptr;
  TileDev* d_btiles = nullptr;
  TileDev* d_dtiles = nullptr;
  TileDev* d_bdtiles = nullptr;
  int cur = 0;
  int nbuf = 2;                      // state buffers in rotation (3 with buffer zones)
  int64_t steps_done = 0;            // RK4 steps taken (buffer zones: time-interpolation history)
  double t = 0.0;
  double dx = 0.0, dt = 0.0;
};

}  // namespace sc

struct sc_ctx {
  sc_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;  // 0 created, 1 built, 2 bound, 3 ready
  sc::Hierarchy hier;
  std::vector<sc::LevelDev> lev;
  int nvars = 2;
  int G = 3;            // ghost layers (3: fourth-order stencils; 4: eighth-order wave)
  int fd_order = 4;     // wave Laplacian order (4 or 8)
  bool mixed = false;   // SC_MIXED: FP32 stencil operands
  bool wave_mixed = false;   // SC_MIXED with the wave: FP64 k1, FP32 stage increments
  size_t esz = 8;       // bytes per element of k and Yh arrays
  size_t arena_bytes = 0;
  size_t o_stage = 0, o_partials = 0, o_norm_out = 0, o_flag = 0, o_der = 0;
  double* d_der = nullptr;       // Z4c FP64: derivative scratch of the largest level
  int norm_parts_max = 1;        // partial workgroups of the largest reduction
  unsigned int* d_nonfinite = nullptr;   // set by stage 4 on a non-finite y_{n+1}
  unsigned int* h_flag = nullptr;        // pinned host copy, read after flag_ev
  hipEvent_t flag_ev = nullptr;
  bool flag_pending = false;
  int64_t stage_elems = 0;
  char* arena = nullptr;
  double* d_stage = nullptr;
  double* d_partials = nullptr;
  double* d_norm_out = nullptr;
  int grid_cap = 0;  // persistent grid size cap for stage kernels
  int64_t launches = 0;
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};   // one per level-0 buffer index
  bool graph_ready[3] = {false, false, false};
  std::vector<int> graph_cur[3];   // every level's buffer index when each graph was captured
  double weights[2][5][4];      // [substep][fill-1][i]
  double weights_inc[2][5][4];  // the same minus the substep's Y1 weights (stage increments)
  // stage-kernel timing with HIP events (eager modes)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;                  // events handed out (pairs use 2)
  int64_t ev_launches = 0;             // stage launches the recorded pairs span
  bool ev_grouped = false;             // a level step's pair spans its stage launches
  std::vector<double> ev_bytes;        // algorithmic bytes per recorded launch
  ~sc_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (flag_ev) (void)hipEventDestroy(flag_ev);
    if (h_flag) (void)hipHostFree(h_flag);
  }
};
