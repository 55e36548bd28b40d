// Z4c stage kernels (z4c.hip).
#pragma once

#include "device.hpp"

namespace sc {

constexpr int kZ4cThreads = 128;
// Curvature values per point that the curvature pass hands to the evolution
// pass; the level's scratch array holds this many arrays of double.
constexpr int kZ4cGeo = 24;
constexpr int kZ4cScratch = kZ4cGeo;

struct Z4cArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t stage;
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
  int64_t vstride;
  double h, dt6, sigma, kappa1, kappa2, eta_c, eta_o, eta_s;
  double origin[3];   // coordinates of global index (0,0,0) of the level
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

// f32: FP32-RHS variant (TS = float)
hipError_t launch_z4c_stage(const Z4cArgs& a, int grid, bool f32, hipStream_t s);
hipError_t launch_z4c_combine(const Z4cCombineArgs& a, int grid, bool f32, hipStream_t s);

}  // namespace sc
