// Eighth-order right-hand side of the wave system (the production stencil of
// Sec. III.C): per dimension the centred nine-point second difference with
// weights (-9, 128, -1008, 8064, -14350, 8064, -1008, 128, -9) / 5040 h^2,
// and the fifth-order Kreiss-Oliger term sigma / (64 h) * (sixth difference)
// on both variables:
//   k_u = Pi + Q u,   k_Pi = (D2x + D2y + D2z) u + Q Pi.
// The stage vector is materialised in the stage's halo table (owned points
// by the combine kernel, halo by the ghost fills), so one thread computes one
// point from taps of one padded array; at stage 4 it also forms
// y_{n+1} = y_n + (dt/6) (((k1 + 2 k2) + 2 k3) + k4).  Sums run in the order
// written, without contraction.
#include "wave8.hpp"

namespace sc {
namespace {

__device__ __forceinline__ double d8(const double* u, int64_t s) {
  return (((((((-9.0 * u[-4 * s] + 128.0 * u[-3 * s]) - 1008.0 * u[-2 * s]) + 8064.0 * u[-s]) -
             14350.0 * u[0]) + 8064.0 * u[s]) - 1008.0 * u[2 * s]) + 128.0 * u[3 * s]) -
         9.0 * u[4 * s];
}

__device__ __forceinline__ double ko6(const double* u, int64_t s) {
  return (((((u[-3 * s] - 6.0 * u[-2 * s]) + 15.0 * u[-s]) - 20.0 * u[0]) + 15.0 * u[s]) -
          6.0 * u[2 * s]) + u[3 * s];
}

template <int STAGE>
__global__ __launch_bounds__(256) void k_wave8_stage(Wave8Args a) {
  const int tx = threadIdx.x % kTileMaxX, ty = threadIdx.x / kTileMaxX;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const TileDev T = a.tiles[t];
    const BoxDev B = a.boxes[T.box];
    const int64_t sy = B.px, sz = (int64_t)B.px * B.py;
    for (int ry = ty; ry < T.ny; ry += 256 / kTileMaxX) {
      if (tx >= T.nx) continue;
      for (int iz = 0; iz < T.nz; ++iz) {
        const int64_t o = B.base + ((int64_t)(T.z0 + iz + B.pad) * B.py + (T.y0 + ry + B.pad)) *
                                       (int64_t)B.px + (T.x0 + tx + B.pad);
        const double* U = a.Y + o;
        const double* P = a.Y + a.vstride + o;
        const double lap = ((d8(U, 1) + d8(U, sy)) + d8(U, sz)) * a.clap;
        const double qu = a.cko * ((ko6(U, 1) + ko6(U, sy)) + ko6(U, sz));
        const double qp = a.cko * ((ko6(P, 1) + ko6(P, sy)) + ko6(P, sz));
        const double ku = P[0] + qu;
        const double kp = lap + qp;
        if (a.kout) {
          a.kout[o] = ku;
          a.kout[o + a.vstride] = kp;
        }
        if constexpr (STAGE == 4) {
          const double k[2] = {ku, kp};
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int64_t ov = o + v * a.vstride;
            const double s = ((a.k1[ov] + 2.0 * a.k2[ov]) + 2.0 * a.k3[ov]) + k[v];
            a.ynew[ov] = a.yn[ov] + a.dt6 * s;
          }
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_wave8_stage(const Wave8Args& a, int grid, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 g(grid > 0 ? grid : a.ntiles), b(256);
  if (a.stage == 4) hipLaunchKernelGGL(k_wave8_stage<4>, g, b, 0, s, a);
  else hipLaunchKernelGGL(k_wave8_stage<1>, g, b, 0, s, a);
  return hipGetLastError();
}

}  // namespace sc
