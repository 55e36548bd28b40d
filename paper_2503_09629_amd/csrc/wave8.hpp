// Eighth-order wave right-hand side (wave8.hip).
#pragma once

#include "device.hpp"

namespace sc {

struct Wave8Args {
  const TileDev* tiles;
  int32_t ntiles;
  int32_t stage;
  const BoxDev* boxes;   // padded with at least 4 ghost layers
  const double* Y;       // stage vector Y_s, owned points and halo, variables u, Pi
  const double* yn;      // y_n (stage 4)
  const double* k1;      // slopes of the earlier stages (stage 4)
  const double* k2;
  const double* k3;
  double* kout;          // k_s, or null (stage 4 on a level without a finer one)
  double* ynew;          // y_{n+1} (stage 4)
  int64_t vstride;
  double clap;           // 1 / (5040 h^2)
  double cko;            // sigma / (64 h)
  double dt6;            // dt / 6
};

// grid: workgroups (persistent over the tile table); 0: one per tile
hipError_t launch_wave8_stage(const Wave8Args& a, int grid, hipStream_t s);

}  // namespace sc
