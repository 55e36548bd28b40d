// Z4c stage kernels (z4c.hip).
#pragma once

#include "device.hpp"

namespace sc {

constexpr int kZ4cThreads = 128;
// Curvature values per point that the curvature pass hands to the evolution
// pass; the level's scratch array holds this many arrays of double.
constexpr int kZ4cGeo = 24;
constexpr int kZ4cScratch = kZ4cGeo;
// Derivative pass (FP64): the first derivatives of W, gt_ij, Khat, Theta,
// Gt^i, alpha, beta^i (16 variables x 3) and the second derivatives of gt_ij,
// W, alpha, beta^i (11 variables x 6 pairs) that the curvature and evolution
// passes use, stored per point in the level's padded layout.
constexpr int kZ4cDer1 = 16 * 3;
constexpr int kZ4cDer = kZ4cDer1 + 11 * 6;
// The derivative pass's own columns: at most kDerTx x kDerTy points in x-y
// (one per thread of a 256-thread workgroup; wide rows, so that the stores of
// neighbouring columns complete whole memory lines) and der_tz(order) planes
// in z (deeper at eighth order, whose four-plane reach costs more per column;
// sizes chosen by timing C5).
constexpr int kDerTx = 64;
constexpr int kDerTy = 4;
constexpr int der_tz(int ord) { return ord == 8 ? 32 : 16; }

struct Z4cArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t stage;
  const TileDev* dtiles;   // the derivative pass's columns over the same region (FP64)
  int32_t ndtiles;
  const BoxDev* boxes;
  const void* Y;      // stage vector on the padded boxes (owned points and halo), TS
  const double* yn;   // FP64 y_n (stage 4)
  const void* k1;     // slopes, TS
  const void* k2;
  const void* k3;
  void* kout;         // k_s, TS (null in constraint mode)
  double* ynew;       // FP64 y_{n+1} (stage 4)
  float* ynew32;      // its FP32 shadow (FP32 variant, stage 4)
  double* ham;        // constraint mode (FP64 only): Hamiltonian constraint out, else null
  void* geo;          // curvature scratch: 24 arrays of TS in the level's padded layout
  double* der;        // FP64: derivative scratch, kZ4cDer arrays in the level's padded layout
  int64_t vstride;
  double h, dt6, sigma, kappa1, kappa2, eta_c, eta_o, eta_s;
  double origin[3];   // coordinates of global index (0,0,0) of the level
  int32_t ord;        // derivative order: 4, or 8 (FP64, boxes padded by 4)
  int32_t ko_r;       // dissipation operator r: 4, or 8 (eighth order, FP64, boxes padded by 5)
  unsigned int* nonfinite;   // set to 1 when stage 4 writes a non-finite y_{n+1}
};

struct Z4cCombineArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t nvars;
  const BoxDev* boxes;
  const void* yn;     // y_n, TS (the FP32 shadow in the FP32 variant)
  const void* kprev;  // k_{s-1}, TS, or null at stage 1
  void* Y;            // stage vector out, TS
  int64_t vstride;
  double cdt;
};

// Radiative outer boundary (level 0, FP64): the physical-boundary ghost slots
// of the level's single box, all members.
struct Z4cRadArgs {
  const int64_t* idx;    // halo offsets of the ghost slots (member-major)
  int64_t n;             // slots, all members
  int64_t per_member;    // slots per member
  const BoxDev* boxes;   // level-0 boxes, one per member
  const double* Y;       // stage vector table (owned and halo)
  const double* yn;      // y_n (ghost values live in the halo of the state arrays)
  const double* kprev;   // k_{s-1} (stage fill), null at stage 1
  const double* k1;      // stage 4
  const double* k2;
  const double* k3;
  double* kout;          // k_s at the ghosts
  double* ynew;          // y_{n+1} at the ghosts (stage 4)
  double* table;         // stage fill output: the stage vector table
  int64_t vstride;
  int32_t stage;
  double cdt;            // c_s dt (stage fill)
  double dt6;
  double h;
  double origin[3];
};
// the ghosts' stage values y_n + c_s dt k_{s-1} into the table (before the
// interior stencils), and their right-hand side (after)
hipError_t launch_z4c_rad_fill(const Z4cRadArgs& a, hipStream_t s);
hipError_t launch_z4c_radiative(const Z4cRadArgs& a, hipStream_t s);

// f32: FP32-RHS variant (TS = float)
hipError_t launch_z4c_stage(const Z4cArgs& a, int grid, bool f32, hipStream_t s);
hipError_t launch_z4c_combine(const Z4cCombineArgs& a, int grid, bool f32, hipStream_t s);

}  // namespace sc
