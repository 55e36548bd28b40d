// Z4c stage kernels (z4c.hip).
#pragma once

#include "device.hpp"

namespace sc {

constexpr int kZ4cThreads = 128;

struct Z4cArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t stage;
  const BoxDev* boxes;
  const double* Y;    // stage vector on the padded boxes (owned points and halo)
  const double* yn;   // y_n (stage 4)
  const double* k1;
  const double* k2;
  const double* k3;
  double* kout;       // k_s (null in constraint mode)
  double* ynew;       // y_{n+1} (stage 4)
  double* ham;        // constraint mode: Hamiltonian constraint out, else null
  int64_t vstride;
  double h, dt6, sigma, kappa1, kappa2, eta_c, eta_o, eta_s;
  double origin[3];   // coordinates of global index (0,0,0) of the level
};

struct Z4cCombineArgs {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t nvars;
  const BoxDev* boxes;
  const double* yn;
  const double* kprev;
  double* Y;
  int64_t vstride;
  double cdt;
};

hipError_t launch_z4c_stage(const Z4cArgs& a, int grid, hipStream_t s);
hipError_t launch_z4c_combine(const Z4cCombineArgs& a, int grid, hipStream_t s);

}  // namespace sc
