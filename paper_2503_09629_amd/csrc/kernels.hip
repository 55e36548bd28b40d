// HIP kernels for gfx950: wave RHS + RK4 stage update, halo copies,
// five-vector prolongation with dense-output stage values, restriction,
// canonical pack/unpack and deterministic norms.
//
// Every floating-point expression is written in one fixed evaluation order
// and the file is compiled without FP contraction, so each value is the
// correctly rounded result of the stated sequence of operations.  The
// stencil type TS is double (FP64 mode, and the first stage of mixed mode)
// or float (stages 2-4 of mixed mode, which evaluate the right-hand side of
// the stage increment Y_s - y_n in FP32); the slope type TK is double or
// float; the state update stays FP64.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "device.hpp"

namespace sc {
namespace {

template <typename T>
__device__ __forceinline__ T d2(T m2, T m1, T c, T p1, T p2) {
  // fourth-order centred second difference, without the 1/(12 h^2) factor
  return (((-m2 + T(16) * m1) - T(30) * c) + T(16) * p1) - p2;
}

template <typename T>
__device__ __forceinline__ T ko7(T m3, T m2, T m1, T c, T p1, T p2, T p3) {
  // sixth difference: h^6 D+^3 D-^3 u, the r = 4 Kreiss-Oliger stencil (Sec. III.C)
  return (((((m3 - T(6) * m2) + T(15) * m1) - T(20) * c) + T(15) * p1) - T(6) * p2) + p3;
}

__device__ __forceinline__ int64_t padded_offset(const BoxDev& B, int x, int y, int z) {
  return B.base + ((int64_t)(z + B.pad) * B.py + (y + B.pad)) * (int64_t)B.px + (x + B.pad);
}

// Ring of the LDS window of a tile (the R-point frame around nx x ny owned
// points): index i in [0, 2R(nx+2R) + 2R ny) -> window coordinates (lx, ly).
template <int R>
__device__ __forceinline__ void ring_coord(int i, int nx, int ny, int* lx, int* ly) {
  const int W = nx + 2 * R;
  if (i < R * W) {
    *ly = i / W;
    *lx = i - *ly * W;
  } else if (i < 2 * R * W) {
    const int j = i - R * W;
    *ly = ny + R + j / W;
    *lx = j % W;
  } else {
    const int j = i - 2 * R * W;
    const int c = j % (2 * R);
    *ly = R + j / (2 * R);
    *lx = c < R ? c : nx + c;
  }
}

// tenth difference: h^10 D+^5 D-^5 u, the r = 8 Kreiss-Oliger stencil
// (Sec. III.C's ninth-order option), taps t(-5..5)
template <typename T, typename Tap>
__device__ __forceinline__ T ko11(const Tap& t) {
  return (((((((((t(-5) - T(10) * t(-4)) + T(45) * t(-3)) - T(120) * t(-2)) + T(210) * t(-1)) -
              T(252) * t(0)) + T(210) * t(1)) - T(120) * t(2)) + T(45) * t(3)) - T(10) * t(4)) +
         t(5);
}

template <typename T>
__device__ __forceinline__ T d8(T m4, T m3, T m2, T m1, T c, T p1, T p2, T p3, T p4) {
  // eighth-order centred second difference times 5040 h^2 (Sec. III.C's production stencil)
  return (((((((T(-9) * m4 + T(128) * m3) - T(1008) * m2) + T(8064) * m1) - T(14350) * c) +
            T(8064) * p1) - T(1008) * p2) + T(128) * p3) - T(9) * p4;
}

template <typename TS>
__device__ __forceinline__ TS load_at(const char* base, uint32_t byte_off) {
  return *reinterpret_cast<const TS*>(base + byte_off);
}

// Stencil operand from its raw loads: owned points (in) are the stage vector
// y_n + (c_s dt) k_{s-1} (Y1 = y_n), or in increment form (INC) the stage
// increment (c_s dt) k_{s-1} alone; halo points are the halo-table value,
// loaded into ra.
template <int STAGE, bool INC, typename TS>
__device__ __forceinline__ TS stage_form(TS ra, TS rk, TS cdt, bool in) {
  if constexpr (STAGE == 1) {
    return ra;
  } else if constexpr (INC) {
    const TS e = cdt * rk;
    return in ? e : ra;
  } else {
    const TS y = ra + cdt * rk;
    return in ? y : ra;
  }
}

// One RK4 stage of the scalar wave on one tile of nx x ny points in x-y (at
// most S per thread, threads mapped row by row) and nz planes, marched in z
// direction DZ (+1 upward, -1 downward) one plane per step.  R is the stencil
// radius: 3 for the fourth-order Laplacian, 4 for the eighth-order one, 5 for
// the eighth-order one with the r = 8 dissipation.  The
// x-y plane of stage values (tile plus the R-point ring) is staged in LDS
// (double buffered, row pitch nx + 2R): the tile's own points come from the
// (2R+1)-plane z column each thread keeps in registers, only the ring is read
// from memory.
// Every load has a valid address (lanes without a point read a clamped one
// and drop the value), so no load sits behind a branch.  The loads of plane
// z + D (ring) and z + D + 3 (column) are issued while plane z is computed,
// D = DEPTH planes ahead (two register sets alternate when D = 2); the stage
// value Y = y_n + c dt k is formed when a set is consumed.  One barrier per
// plane.
//   k_u  = Pi + Q u,   k_Pi = Lap u + Q Pi
//   Lap  = ((d2_x + d2_y) + d2_z) / (12 h^2)        (R = 3)
//        = ((d8_x + d8_y) + d8_z) / (5040 h^2)      (R = 4)
//   Q    = sigma/(64 h) ((ko_x + ko_y) + ko_z)       (R = 3, 4: sixth differences)
//        = sigma/(1024 h) ((ko_x + ko_y) + ko_z)     (R = 5: tenth differences)
// Stage 4 also forms y_{n+1} = y_n + (dt/6) (((k1 + 2 k2) + 2 k3) + k4) in FP64.
// The z stencils take their taps in increasing z whatever the direction, so
// both directions give the same bits.
// Increment form (mixed mode, TS = float, stages 2-4): the wave right-hand
// side f is linear, so k_s = f(y_n + e_s) = k1 + f(e_s) with the stage
// increment e_s = c_s dt k_{s-1} (halo: the table holds Y_s - Y_1).  Only e_s,
// of size O(dt |k|), passes through FP32 arithmetic, so the FP32 rounding that
// the stencil amplifies by 1/h^2 is that of e_s, not of y_n; k1 = f(y_n) is
// evaluated in FP64 (TS = double, TK = float).
template <typename TS, int S, int RM>
struct StageRaw {   // raw loads of one ring plane and one column plane
  TS ra[2][RM], rk[2][RM];
  TS ca[2][S], ck[2][S];
};

template <int STAGE, typename TS, typename TK, int DEPTH, int S, bool WK, int NT, int R>
__device__ __forceinline__ void stage_tile(const StageArgs& a, const TileDev& T, const BoxDev& B,
                                           TS* lds) {
  constexpr bool INC = sizeof(TS) == 4;   // FP32 stencils evaluate the stage increment
  static_assert(!INC || (STAGE > 1 && sizeof(TK) == 4), "increment form: stages 2-4, FP32 slopes");
  static_assert(STAGE == 1 || sizeof(TK) == sizeof(TS), "stencil operand k_{s-1} has the slope type");
  constexpr int RM = StageFamily<NT>::ring;
  constexpr int kWinCap = StageFamily<NT>::wincap;
  constexpr int kWinStride = kWinCap + 8;   // per-variable LDS stride: window plus a spare slot
  constexpr int QN = 2 * R + 1;   // z column: planes z-R .. z+R along DZ
  const TS clap = TS(a.clap), cko = TS(a.cko), cdt = TS(a.cdt);
  const char* yn = static_cast<const char*>(a.yn);
  const char* kp = static_cast<const char*>(a.kprev);
  const char* yh = static_cast<const char*>(a.Yh);
  const int W = T.nx + 2 * R;
  const int64_t ps = (int64_t)B.px * B.py;     // points per z plane
  // planes the tile reads and computes, and the first computed plane
  const int zlo = T.z0 - R, zhi = T.z0 + T.nz + R - 1;
  const bool up = T.dir == 0;
  const int DZ = up ? 1 : -1;
  const int z0 = up ? T.z0 : T.z0 + T.nz - 1;
  auto clampz = [&](int z, int lo, int hi) { return z < lo ? lo : (z > hi ? hi : z); };
  auto zin = [&](int z) { return (unsigned)z < (unsigned)B.nz; };
  // byte offset of plane z of variable v within the level arrays
  auto plane = [&](int z, int v) -> int64_t {
    return (int64_t)sizeof(TS) * (B.base + (int64_t)(z + B.pad) * ps + (int64_t)v * a.vstride);
  };
  bool act[S];
  int li[S];
  uint32_t cb[S];  // byte offset of the point within its plane
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = threadIdx.x + s * NT;
    act[s] = i < T.nx * T.ny;
    const int ic = act[s] ? i : 0;
    const int px = ic % T.nx, py = ic / T.nx;
    li[s] = (py + R) * W + px + R;
    cb[s] = (uint32_t)sizeof(TS) * (uint32_t)((T.y0 + py + B.pad) * B.px + (T.x0 + px + B.pad));
  }
  const int nring = 2 * R * W + 2 * R * T.ny;
  bool ract[RM], rin[RM];
  int rli[RM];
  uint32_t rb[RM];
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    const int i = threadIdx.x + k * NT;
    ract[k] = i < nring;
    int lx = 0, ly = 0;
    ring_coord<R>(ract[k] ? i : 0, T.nx, T.ny, &lx, &ly);
    rli[k] = ly * W + lx;
    const int x = T.x0 - R + lx, y = T.y0 - R + ly;
    rin[k] = (unsigned)x < (unsigned)B.nx && (unsigned)y < (unsigned)B.ny;
    rb[k] = (uint32_t)sizeof(TS) * (uint32_t)((y + B.pad) * B.px + (x + B.pad));
  }
  // raw loads of ring plane z0 + DZ j and column plane z0 + DZ (j + R)
  auto issue = [&](StageRaw<TS, S, RM>& X, int j) {
    const int zr = clampz(z0 + DZ * j, T.z0, T.z0 + T.nz - 1);
    const int zq = clampz(z0 + DZ * (j + R), zlo, zhi);
    const bool qin = zin(zq);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int64_t pr = plane(zr, v);
#pragma unroll
      for (int k = 0; k < RM; ++k) {
        if constexpr (INC) {   // owned points need only the slope
          X.ra[v][k] = TS(0);
          if (!rin[k]) X.ra[v][k] = load_at<TS>(yh + pr, rb[k]);
        } else {
          X.ra[v][k] = load_at<TS>((rin[k] ? yn : yh) + pr, rb[k]);
        }
        X.rk[v][k] = STAGE > 1 ? load_at<TS>(kp + pr, rb[k]) : TS(0);
      }
      const int64_t pq = plane(zq, v);
      const char* src = (qin ? yn : yh) + pq;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if constexpr (INC) X.ca[v][s] = qin ? TS(0) : load_at<TS>(src, cb[s]);
        else X.ca[v][s] = load_at<TS>(src, cb[s]);
        X.ck[v][s] = STAGE > 1 ? load_at<TS>(kp + pq, cb[s]) : TS(0);
      }
    }
  };
  TS q[2][S][QN];   // stage values of the z column, in marching order
  bool bad = false;  // stage 4: a non-finite y_{n+1} was written (reported once per tile)
  // prologue: column planes z0 - R DZ .. z0 + (R - 1) DZ into q[1..2R]
#pragma unroll
  for (int j = 1; j < QN; ++j) {
    const int z = clampz(z0 + DZ * (j - 1 - R), zlo, zhi);
    const bool in = zin(z);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int64_t pb = plane(z, v);
      const char* src = (in ? yn : yh) + pb;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const TS va = (INC && in) ? TS(0) : load_at<TS>(src, cb[s]);
        const TS vk = STAGE > 1 ? load_at<TS>(kp + pb, cb[s]) : TS(0);
        q[v][s][j] = stage_form<STAGE, INC, TS>(va, vk, cdt, in);
      }
    }
  }
  StageRaw<TS, S, RM> regs[DEPTH];
#pragma unroll
  for (int j = 0; j < DEPTH; ++j) issue(regs[j], j);
  // one plane: consume a register set (ring plane iz, column plane iz + R), refill it
  // with the planes DEPTH further on, compute plane iz
  auto step = [&](int iz, StageRaw<TS, S, RM>& P, TS* L) {
    const int z = z0 + DZ * iz;
    const bool zc = zin(z0 + DZ * (iz + R));
#pragma unroll
    for (int j = 0; j < QN - 1; ++j)
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int v = 0; v < 2; ++v) q[v][s][j] = q[v][s][j + 1];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        q[v][s][QN - 1] = stage_form<STAGE, INC, TS>(P.ca[v][s], P.ck[v][s], cdt, zc);
    const bool zr = zin(z);
    // lanes without a point write the spare slot past the window: no branch
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      TS* Lv = L + v * kWinStride;
#pragma unroll
      for (int s = 0; s < S; ++s) Lv[act[s] ? li[s] : kWinCap] = q[v][s][R];
#pragma unroll
      for (int k = 0; k < RM; ++k)
        Lv[ract[k] ? rli[k] : kWinCap] =
            stage_form<STAGE, INC, TS>(P.ra[v][k], P.rk[v][k], cdt, rin[k] && zr);
    }
    __syncthreads();
    issue(P, iz + DEPTH);   // in flight during this plane's arithmetic
    const TS* Lu = L;
    const TS* Lp = L + kWinStride;
    // column taps in increasing z: zt[m] is plane z + m - R
    auto zt = [&](int v, int s, int m) -> TS { return up ? q[v][s][m] : q[v][s][2 * R - m]; };
    // stage 4 reads the slopes and y_n at the point, the increment form k1:
    // issue those loads first
    TK c1[2][S], c2[2][S], c3[2][S];
    double c0[2][S];
    const int64_t pe = B.base + (int64_t)(z + B.pad) * ps;   // element offset of the plane
    if constexpr (STAGE == 4 || INC) {
      const TK* k1 = static_cast<const TK*>(a.k1);
      const TK* k2 = static_cast<const TK*>(a.k2);
      const TK* k3 = static_cast<const TK*>(a.k3);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int64_t o = pe + cb[s] / (uint32_t)sizeof(TS) + v * a.vstride;
          c1[v][s] = k1[o];
          if constexpr (STAGE == 4) {
            c2[v][s] = k2[o];
            c3[v][s] = k3[o];
            c0[v][s] = a.yn64[o];
          }
        }
    }
    // lanes without a point compute and store the tile's first point again
    // (same inputs, same bits), so the stores need no branch either
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int c = li[s];
      const TS cu = q[0][s][R], cp = q[1][s][R];
      TS lapx, lapy, lapz;
      if constexpr (R == 3) {
        lapx = d2<TS>(Lu[c - 2], Lu[c - 1], cu, Lu[c + 1], Lu[c + 2]);
        lapy = d2<TS>(Lu[c - 2 * W], Lu[c - W], cu, Lu[c + W], Lu[c + 2 * W]);
        lapz = d2<TS>(zt(0, s, 1), zt(0, s, 2), cu, zt(0, s, 4), zt(0, s, 5));
      } else {
        lapx = d8<TS>(Lu[c - 4], Lu[c - 3], Lu[c - 2], Lu[c - 1], cu, Lu[c + 1], Lu[c + 2],
                      Lu[c + 3], Lu[c + 4]);
        lapy = d8<TS>(Lu[c - 4 * W], Lu[c - 3 * W], Lu[c - 2 * W], Lu[c - W], cu, Lu[c + W],
                      Lu[c + 2 * W], Lu[c + 3 * W], Lu[c + 4 * W]);
        lapz = d8<TS>(zt(0, s, R - 4), zt(0, s, R - 3), zt(0, s, R - 2), zt(0, s, R - 1), cu,
                      zt(0, s, R + 1), zt(0, s, R + 2), zt(0, s, R + 3), zt(0, s, R + 4));
      }
      const TS lap = ((lapx + lapy) + lapz) * clap;
      TS Q[2];
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const TS* Lv = v == 0 ? Lu : Lp;
        const TS cc = q[v][s][R];
        if constexpr (R == 5) {   // r = 8 dissipation
          const TS kx = ko11<TS>([&](int j) { return j == 0 ? cc : Lv[c + j]; });
          const TS ky = ko11<TS>([&](int j) { return j == 0 ? cc : Lv[c + j * W]; });
          const TS kz = ko11<TS>([&](int j) { return j == 0 ? cc : zt(v, s, R + j); });
          Q[v] = cko * ((kx + ky) + kz);
        } else {
          const TS kx = ko7<TS>(Lv[c - 3], Lv[c - 2], Lv[c - 1], cc, Lv[c + 1], Lv[c + 2], Lv[c + 3]);
          const TS ky = ko7<TS>(Lv[c - 3 * W], Lv[c - 2 * W], Lv[c - W], cc, Lv[c + W],
                                Lv[c + 2 * W], Lv[c + 3 * W]);
          const TS kz = ko7<TS>(zt(v, s, R - 3), zt(v, s, R - 2), zt(v, s, R - 1), cc,
                                zt(v, s, R + 1), zt(v, s, R + 2), zt(v, s, R + 3));
          Q[v] = cko * ((kx + ky) + kz);
        }
      }
      TK kv[2];
      if constexpr (INC) {   // k_s = k1 + f(e_s)
        kv[0] = c1[0][s] + (cp + Q[0]);
        kv[1] = c1[1][s] + (lap + Q[1]);
      } else {
        kv[0] = (TK)(cp + Q[0]);
        kv[1] = (TK)(lap + Q[1]);
      }
      const int64_t o = pe + cb[s] / (uint32_t)sizeof(TS);
      if constexpr (WK) {
        TK* ko = static_cast<TK*>(a.kout);
        ko[o] = kv[0];
        ko[o + a.vstride] = kv[1];
      }
      if constexpr (STAGE == 4) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int64_t ov = o + v * a.vstride;
          const double sm = (((double)c1[v][s] + 2.0 * (double)c2[v][s]) + 2.0 * (double)c3[v][s]) +
                            (double)kv[v];
          const double yv = c0[v][s] + a.dt6 * sm;
          a.ynew[ov] = yv;
          bad = bad || !isfinite(yv);
        }
      }
    }
  };
  // DEPTH planes per trip, each with its own register set (static names);
  // the last partial trip is guarded
  int iz = 0;
  for (; iz + DEPTH <= T.nz; iz += DEPTH) {
#pragma unroll
    for (int j = 0; j < DEPTH; ++j) step(iz + j, regs[j], lds + ((iz + j) & 1) * 2 * kWinStride);
  }
#pragma unroll
  for (int j = 0; j < DEPTH - 1; ++j)
    if (iz + j < T.nz) step(iz + j, regs[j], lds + ((iz + j) & 1) * 2 * kWinStride);
  if (STAGE == 4 && bad) atomicOr(a.nonfinite, 1u);
  __syncthreads();
}

// Persistent stage kernel: workgroups stride over the tile list; a tile's
// dir field picks its z marching direction.
template <int STAGE, typename TS, typename TK, int DEPTH, int S, bool WK, int NT, int R>
__global__ __launch_bounds__(NT) void k_wave_stage(StageArgs a) {
  __shared__ TS lds[2 * 2 * (StageFamily<NT>::wincap + 8)];
  // consecutive workgroups land on different XCDs (round robin over 8); give
  // each XCD a contiguous run of tiles so neighbouring tiles share its L2
  const int g = (gridDim.x % 8 == 0)
                    ? (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8)
                    : (int)blockIdx.x;
  for (int t = g; t < a.ntiles; t += gridDim.x) {
    const TileDev T = a.tiles[t];
    const BoxDev B = a.boxes[T.box];
    stage_tile<STAGE, TS, TK, DEPTH, S, WK, NT, R>(a, T, B, lds);
  }
}

// Halo copy from an owned point of the same level: the stage vector there
// (y_n + cdt k_{s-1}, evaluated exactly as the stencil kernel does), y_n,
// or in increment form the stage increment cdt k_{s-1}.
template <typename TS>
__global__ __launch_bounds__(256) void k_sync(SyncArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const SyncEntry e = a.e[i];
  const TS* yn = static_cast<const TS*>(a.yn);
  const TS* kp = static_cast<const TS*>(a.kprev);
  TS* out = static_cast<TS*>(a.out);
  for (int v = 0; v < a.nvars; ++v) {
    const int64_t s = e.src + v * a.vstride;
    out[e.dst + v * a.vstride] =
        a.inc ? TS(a.cdt) * kp[s] : (kp ? yn[s] + TS(a.cdt) * kp[s] : yn[s]);
  }
}

// Combination of the prolonged input vectors v[0..NIN-1] for output o.
// NIN = 5 (dense output): v = (y_n, k1..k4),
//   P[y_n] + H (((w1 P[k1] + w2 P[k2]) + w3 P[k3]) + w4 P[k4]);
// NIN = 3 (buffer zones, time interpolation): v = (y_n, y_{n-1}, y_{n+1}),
//   ((w1 P[y_{n-1}] + w2 P[y_n]) + w3 P[y_{n+1}]);
// NIN = 1 (buffer zones at the parent's own time): P[y_n].
// An increment output (inc) omits P[y_n]: H (((w1 P[k1] + ...) + w4 P[k4]).
template <int NIN>
__device__ __forceinline__ double prolong_combine(const double (&v)[NIN], const double* w,
                                                  double H, bool inc) {
  if constexpr (NIN == 5) {
    const double s = ((w[0] * v[1] + w[1] * v[2]) + w[2] * v[3]) + w[3] * v[4];
    return inc ? H * s : v[0] + H * s;
  } else if constexpr (NIN == 3) {
    return (w[0] * v[1] + w[1] * v[0]) + w[2] * v[2];
  } else {
    return v[0];
  }
}

// Output o of a prolongation is FP32 when bit o of f32_mask is set.
__device__ __forceinline__ void store_out(void* out, int64_t i, bool f32, double v) {
  if (f32) static_cast<float*>(out)[i] = (float)v;
  else static_cast<double*>(out)[i] = v;
}

// Prolongation of NIN parent vectors (y_n first, then the pk[]) to one fine
// point, x first, then y, then z, with the degree-5 Lagrange midpoint weights
// at odd fine indices and a copy at even ones; then each requested
// combination (prolong_combine), all in FP64.  The parity class is a
// template parameter, so every loop has a compile-time trip count, and each
// stencil tap gathers all NIN vectors.
template <int NIN, int OX, int OY, int OZ, typename TK>
__device__ __forceinline__ void prolong_one(const ProlongArgs& a, int64_t i) {
  constexpr int NX = OX ? 6 : 1, NY = OY ? 6 : 1, NZ = OZ ? 6 : 1;
  constexpr double W[6] = {3.0 / 256.0, -25.0 / 256.0, 150.0 / 256.0,
                           150.0 / 256.0, -25.0 / 256.0, 3.0 / 256.0};
  const ProlongEntry e = a.e[i];
  const BoxDev P = a.pboxes[e.pbox];
  const int64_t pitch[3] = {1, (int64_t)P.px, (int64_t)P.px * P.py};
  int64_t ox[NX], oy[NY], oz[NZ];
  auto offs = [&](int d, int odd, int j) -> int64_t {
    const int base = e.q[d] >> 1;
    int I = odd ? base - 2 + j : base;
    if (P.wrapN[d] > 0) I = ((I % P.wrapN[d]) + P.wrapN[d]) % P.wrapN[d];
    return (int64_t)(I - P.lo[d] + P.pad) * pitch[d];
  };
#pragma unroll
  for (int j = 0; j < NX; ++j) ox[j] = offs(0, OX, j);
#pragma unroll
  for (int j = 0; j < NY; ++j) oy[j] = offs(1, OY, j);
#pragma unroll
  for (int j = 0; j < NZ; ++j) oz[j] = offs(2, OZ, j);
  for (int v = 0; v < a.nvars; ++v) {
    const int64_t vb = P.base + v * a.pvstride;
    double pz[NIN];
#pragma unroll
    for (int jz = 0; jz < NZ; ++jz) {
      double py[NIN];
#pragma unroll
      for (int jy = 0; jy < NY; ++jy) {
        double px[NIN];
#pragma unroll
        for (int jx = 0; jx < NX; ++jx) {
          const int64_t o = vb + oz[jz] + oy[jy] + ox[jx];
          double t[NIN];
          t[0] = a.py[o];
#pragma unroll
          for (int m = 1; m < NIN; ++m) t[m] = (double)static_cast<const TK*>(a.pk[m - 1])[o];
#pragma unroll
          for (int m = 0; m < NIN; ++m) {
            if constexpr (NX == 1) px[m] = t[m];
            else px[m] = jx == 0 ? W[0] * t[m] : px[m] + W[jx] * t[m];
          }
        }
#pragma unroll
        for (int m = 0; m < NIN; ++m) {
          if constexpr (NY == 1) py[m] = px[m];
          else py[m] = jy == 0 ? W[0] * px[m] : py[m] + W[jy] * px[m];
        }
      }
#pragma unroll
      for (int m = 0; m < NIN; ++m) {
        if constexpr (NZ == 1) pz[m] = py[m];
        else pz[m] = jz == 0 ? W[0] * py[m] : pz[m] + W[jz] * py[m];
      }
    }
    for (int o = 0; o < a.nout; ++o)
      store_out(a.out[o], e.dst + v * a.ovstride, (a.f32_mask >> o) & 1,
                prolong_combine<NIN>(pz, a.w[o], a.H, (a.inc_mask >> o) & 1));
  }
}

template <int NIN, typename TK>
__global__ __launch_bounds__(256) void k_prolong(ProlongArgs a) {
  const int b = blockIdx.x;
  int cls = 0;
  while (cls < 7 && b >= a.blk_start[cls + 1]) ++cls;
  const int64_t i = a.cls_start[cls] + (int64_t)(b - a.blk_start[cls]) * 256 + threadIdx.x;
  if (i >= a.cls_start[cls + 1]) return;
  switch (cls) {
    case 0: prolong_one<NIN, 0, 0, 0, TK>(a, i); break;
    case 1: prolong_one<NIN, 1, 0, 0, TK>(a, i); break;
    case 2: prolong_one<NIN, 0, 1, 0, TK>(a, i); break;
    case 3: prolong_one<NIN, 1, 1, 0, TK>(a, i); break;
    case 4: prolong_one<NIN, 0, 0, 1, TK>(a, i); break;
    case 5: prolong_one<NIN, 1, 0, 1, TK>(a, i); break;
    case 6: prolong_one<NIN, 0, 1, 1, TK>(a, i); break;
    default: prolong_one<NIN, 1, 1, 1, TK>(a, i); break;
  }
}

// Brick prolongation: one workgroup per brick (a face slab, edge piece or
// corner of a fine box's RB shell).  For each variable and each of the input
// vectors, the parent region under the brick is staged in LDS, interpolated
// along x for every fine x of the brick, then along y, then along z (the same
// left-to-right sums as the per-point form, so the values are identical), and
// the dense-output combinations are written for the brick's RB points.  Each
// vector's parent values for the next variable are loaded as soon as the
// current ones are in LDS, so they have the rest of the variable's passes to
// arrive.  Each thread's share of the three passes is worked out once per
// brick and packed as (source place, destination place, odd, in range); in
// the z pass the destination of entry i is fine point i.  ZE: fine points per
// thread (2 covers the three-layer shell's slabs, 3 the four-layer one's).
__device__ __forceinline__ double brick_tap(const double* src, int st, bool odd) {
  constexpr double W[6] = {3.0 / 256.0, -25.0 / 256.0, 150.0 / 256.0,
                           150.0 / 256.0, -25.0 / 256.0, 3.0 / 256.0};
  if (!odd) return src[0];
  double r = W[0] * src[0];
#pragma unroll
  for (int j = 1; j < 6; ++j) r = r + W[j] * src[j * st];
  return r;
}

// i / d for i * d < 2^20, with m = brick_magic(d): i m / 2^20 exceeds i / d
// by less than i / 2^20 < 1 / d, which cannot carry it past the next integer.
__device__ __forceinline__ unsigned brick_magic(unsigned d) { return (1u << 20) / d + 1u; }
__device__ __forceinline__ unsigned brick_div(unsigned i, unsigned m) { return (i * m) >> 20; }

constexpr unsigned kTapOdd = 1u << 12, kTapOn = 1u << 13, kTapWrite = 1u << 14;
constexpr unsigned kPassOdd = 1u << 24, kPassOn = 1u << 25;
constexpr unsigned kNoPoint = 0xffffffffu;

template <int NIN, typename TK, int ZE>
__global__ __launch_bounds__(kBrickThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_prolong_bricks(BrickArgs a) {
  constexpr int NT = kBrickThreads;
  constexpr int NL = kBrickV / NT, XE = kBrickPX / NT, YE = kBrickPY / NT;
  static_assert(kBrickV % NT == 0 && kBrickPX % NT == 0 && kBrickPY % NT == 0 &&
                ZE * NT <= kBrickPts && kBrickPY < 4096, "brick limits");
  __shared__ double S[kBrickLds];
  // consecutive workgroups land on different XCDs; give each XCD a
  // contiguous run of bricks so overlapping parent regions share its L2
  const int g = (gridDim.x % 8 == 0)
                    ? (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8)
                    : (int)blockIdx.x;
  if (g >= a.nbricks) return;
  const ProlongBrick& Bk = a.b[g];
  const int ba[3] = {Bk.a[0], Bk.a[1], Bk.a[2]};
  const int n0 = Bk.n[0], n1 = Bk.n[1], n2 = Bk.n[2];
  const BoxDev F = a.fboxes[Bk.fbox];
  const BoxDev P = a.pboxes[Bk.pbox];
  int C0[3], cn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    C0[d] = brick_parent_first(ba[d]);
    cn[d] = brick_parent_count(ba[d], Bk.n[d]);
  }
  const int nv = cn[0] * cn[1] * cn[2], npx = cn[2] * cn[1] * n0, npy = cn[2] * n1 * n0;
  const int n01 = n0 * n1, npts = n01 * n2;
  double* V = S;                 // [cz][cy][cx]
  double* PX = S + nv;           // [cz][cy][fx]
  double* PY = PX + npx;         // [cz][fy][fx]
  const int pn[3] = {P.nx, P.ny, P.nz};
  const unsigned pitch[3] = {1u, (unsigned)P.px, (unsigned)P.px * (unsigned)P.py};
  const int tid = threadIdx.x;
  // parent points of this thread (place tid + j NT of V): offset from the
  // parent box's base (periodic wrap, then clamped into the padded box)
  unsigned co[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int i = tid + j * NT;
    const int c[3] = {i % cn[0], (i / cn[0]) % cn[1], i / (cn[0] * cn[1])};
    unsigned o = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int I = C0[d] + c[d];
      if (P.wrapN[d] > 0) I = ((I % P.wrapN[d]) + P.wrapN[d]) % P.wrapN[d];
      int loc = I - P.lo[d];
      loc = loc < -P.pad ? -P.pad : (loc > pn[d] + P.pad - 1 ? pn[d] + P.pad - 1 : loc);
      o += (unsigned)(loc + P.pad) * pitch[d];
    }
    co[j] = i < nv ? o : kNoPoint;
  }
  const unsigned m0 = brick_magic(n0), m01 = brick_magic(n01);
  // x and y passes: the entries whose fine index is even (copies) come first,
  // then the odd ones (six-point sums), so that a wave's lanes take one branch
  const int ex = ba[0] & 1, nex = (n0 - ex + 1) >> 1, nox = n0 - nex;   // first even fx, counts
  const int ey = ba[1] & 1, ney = (n1 - ey + 1) >> 1, noy = n1 - ney;
  const int rows = cn[2] * cn[1];
  const unsigned mex = brick_magic(nex > 0 ? nex : 1), mox = brick_magic(nox > 0 ? nox : 1);
  const unsigned mey = brick_magic(ney > 0 ? ney : 1), moy = brick_magic(noy > 0 ? noy : 1);
  unsigned xa[XE], ya[YE], za[ZE], dst[ZE];
#pragma unroll
  for (int e = 0; e < XE; ++e) {            // PX place r n0 + fx, r = cz cn1 + cy
    const int i = tid + e * NT;
    const bool odd = i >= rows * nex;
    const unsigned ii = odd ? i - rows * nex : i;
    const unsigned r = brick_div(ii, odd ? mox : mex), k = ii - r * (odd ? nox : nex);
    const unsigned fx = (odd ? 1 - ex : ex) + 2 * k;
    const int q = ba[0] + (int)fx, b = (q >> 1) - C0[0] - (odd ? 2 : 0);
    xa[e] = i < npx ? (r * cn[0] + b) | ((r * n0 + fx) << 12) | (odd ? kPassOdd : 0u) | kPassOn : 0u;
  }
#pragma unroll
  for (int e = 0; e < YE; ++e) {            // PY place (cz n1 + fy) n0 + fx
    const int i = tid + e * NT;
    const bool odd = i >= cn[2] * ney * n0;
    const unsigned ii = odd ? i - cn[2] * ney * n0 : i;
    const unsigned t = brick_div(ii, m0), fx = ii - t * n0;
    const unsigned cz = brick_div(t, odd ? moy : mey), k = t - cz * (odd ? noy : ney);
    const unsigned fy = (odd ? 1 - ey : ey) + 2 * k;
    const int q = ba[1] + (int)fy, b = (q >> 1) - C0[1] - (odd ? 2 : 0);
    ya[e] = i < npy ? ((cz * cn[1] + b) * n0 + fx) | (((cz * n1 + fy) * n0 + fx) << 12) |
                          (odd ? kPassOdd : 0u) | kPassOn
                    : 0u;
  }
#pragma unroll
  for (int e = 0; e < ZE; ++e) {            // fine point i = fz n01 + (fy n0 + fx)
    const unsigned i = tid + e * NT, fz = brick_div(i, m01), j = i - fz * n01;
    const unsigned fy = brick_div(j, m0), fx = j - fy * n0;
    const int q = ba[2] + (int)fz, b = (q >> 1) - C0[2] - ((q & 1) ? 2 : 0);
    const bool on = (int)i < npts;
    const bool w = on && ((Bk.mask[i >> 6] >> (i & 63)) & 1);
    za[e] = on ? (b * n01 + j) | ((q & 1) ? kTapOdd : 0u) | kTapOn | (w ? kTapWrite : 0u) : 0u;
    dst[e] = ((unsigned)(ba[2] + (int)fz - F.lo[2] + F.pad) * (unsigned)F.py +
              (unsigned)(ba[1] + (int)fy - F.lo[1] + F.pad)) * (unsigned)F.px +
             (unsigned)(ba[0] + (int)fx - F.lo[0] + F.pad);
  }
  const int sty = n0, stz = n01;
  auto load = [&](int v, int m, double (&R)[NL]) {
    const int64_t vo = P.base + (int64_t)v * a.pvstride;
    if (m == 0) {
      const double* src = a.py + vo;
#pragma unroll
      for (int j = 0; j < NL; ++j)
        if (co[j] != kNoPoint) R[j] = src[co[j]];
    } else {
      const TK* src = static_cast<const TK*>(a.pk[m - 1]) + vo;
#pragma unroll
      for (int j = 0; j < NL; ++j)
        if (co[j] != kNoPoint) R[j] = (double)src[co[j]];
    }
  };
  double R[NIN][NL];
#pragma unroll
  for (int m = 0; m < NIN; ++m) load(0, m, R[m]);
  for (int v = 0; v < a.nvars; ++v) {
    double Pv[ZE][NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) {
#pragma unroll
      for (int j = 0; j < NL; ++j)
        if (co[j] != kNoPoint) V[tid + j * NT] = R[m][j];
      __syncthreads();
      if (v + 1 < a.nvars) load(v + 1, m, R[m]);   // in flight for the rest of this variable
#pragma unroll
      for (int e = 0; e < XE; ++e)
        if (xa[e] & kPassOn)
          PX[(xa[e] >> 12) & 4095u] = brick_tap(V + (xa[e] & 4095u), 1, xa[e] & kPassOdd);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < YE; ++e)
        if (ya[e] & kPassOn)
          PY[(ya[e] >> 12) & 4095u] = brick_tap(PX + (ya[e] & 4095u), sty, ya[e] & kPassOdd);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < ZE; ++e)
        Pv[e][m] = (za[e] & kTapOn) ? brick_tap(PY + (za[e] & 4095u), stz, za[e] & kTapOdd) : 0.0;
    }
    const int64_t ob = F.base + (int64_t)v * a.ovstride;
#pragma unroll
    for (int e = 0; e < ZE; ++e) {
      if (!(za[e] & kTapWrite)) continue;
      const int64_t d = ob + dst[e];
      for (int o = 0; o < a.nout; ++o)
        store_out(a.out[o], d, (a.f32_mask >> o) & 1,
                  prolong_combine<NIN>(Pv[e], a.w[o], a.H, (a.inc_mask >> o) & 1));
    }
  }
}

// Injection y_parent(I) <- y_fine(2I) over (fine box, parent box) regions.
__global__ __launch_bounds__(256) void k_restrict(RestrictArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ntotal) return;
  int r = 0;
  while (r + 1 < a.nregions && a.r[r + 1].start <= i) ++r;
  const RestrictRegion R = a.r[r];
  const int64_t l = i - R.start;
  const int cx = R.c0[0] + (int)(l % R.n[0]);
  const int cy = R.c0[1] + (int)((l / R.n[0]) % R.n[1]);
  const int cz = R.c0[2] + (int)(l / ((int64_t)R.n[0] * R.n[1]));
  const BoxDev F = a.fboxes[R.fbox];
  const BoxDev P = a.pboxes[R.pbox];
  const int64_t fo = padded_offset(F, 2 * cx - F.lo[0], 2 * cy - F.lo[1], 2 * cz - F.lo[2]);
  const int64_t po = padded_offset(P, cx - P.lo[0], cy - P.lo[1], cz - P.lo[2]);
  for (int v = 0; v < a.nvars; ++v) {
    const double y = a.fy[fo + v * a.fvstride];
    a.py[po + v * a.pvstride] = y;
    if (a.py32) a.py32[po + v * a.pvstride] = (float)y;
  }
}

__device__ __forceinline__ int64_t canonical_to_offset(const PackArgs& a, int64_t i) {
  int b = 0;
  while (b + 1 < a.nboxes && a.prefix[b + 1] <= i) ++b;
  const BoxDev B = a.boxes[b];
  const int64_t l = i - a.prefix[b];
  const int x = (int)(l % B.nx);
  const int y = (int)((l / B.nx) % B.ny);
  const int z = (int)(l / ((int64_t)B.nx * B.ny));
  return padded_offset(B, x, y, z);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack(PackArgs a, int unpack) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t o = canonical_to_offset(a, i);
  T* arr = static_cast<T*>(a.arr);
  if (unpack) arr[o] = (T)a.buf[i];
  else a.buf[i] = (double)arr[o];
}

// Closed-form initial data.  Kinds (parameters in InitArgs::p):
//  1 standing wave  u = A cos(w t) S, Pi = -A w sin(w t) S with
//    S = sin(m_x pi x) sin(m_y pi y) sin(m_z pi z), w = pi |m|; p = (A, m_x, m_y, m_z, t)
//    (at t = 0: u = A S, Pi = 0)
//  2 Gaussian pulses u = sum_p A_p g_p(x) g_p(y) g_p(z), Pi = 0, with
//    g_p(x) = sum_{k=-K..K} exp(-(x - c_{p,x} - k L)^2 / w_p^2) (K = 1 if the
//    period L > 0, else 0); p = (npulses, L, then A, w, c_x, c_y, c_z per pulse)
//  3 Brill-Lindquist punctures (22 Z4c variables): psi = 1 + a,
//    a = m_+ / (2 r_+) + m_- / (2 r_-), W = psi^-2, gt = delta, lapse
//    (1 + (1 - a) / (1 + a)) / 2, the rest 0; p = (m_+, m_-, x_+, x_-) with the
//    punctures at (x_+, 0, 0) and (x_-, 0, 0)
//  4 outgoing spherical Gaussian u = (f(t - r) - f(t + r)) / r, Pi = du/dt,
//    f(v) = A exp(-v^2 / (2 sigma^2)), limits at r = 0; p = (A, sigma, t)
__device__ __forceinline__ double periodised_gauss(double x, double c, double w, double L) {
  if (L <= 0.0) {
    const double d = x - c;
    return exp(-(d * d) / (w * w));
  }
  double g = 0.0;
  for (int k = -1; k <= 1; ++k) {
    const double d = (x - c) - k * L;
    g += exp(-(d * d) / (w * w));
  }
  return g;
}

__device__ double init_value(const InitArgs& a, double x, double y, double z, int v) {
  const double* p = a.p;
  switch (a.kind) {
    case 1: {
      const double t = p[4];
      if (t == 0.0) {
        if (v != 0) return 0.0;
        const double fx = p[0] * sin(p[1] * M_PI * x);
        return (sin(p[3] * M_PI * z) * sin(p[2] * M_PI * y)) * fx;
      }
      const double w = M_PI * sqrt((p[1] * p[1] + p[2] * p[2]) + p[3] * p[3]);
      const double S = (sin(p[3] * M_PI * z) * sin(p[2] * M_PI * y)) * sin(p[1] * M_PI * x);
      return v == 0 ? (p[0] * cos(w * t)) * S : (-p[0] * w * sin(w * t)) * S;
    }
    case 2: {
      if (v != 0) return 0.0;
      const int np = (int)p[0];
      double u = 0.0;
      for (int q = 0; q < np; ++q) {
        const double* c = p + 2 + 5 * q;
        const double gx = c[0] * periodised_gauss(x, c[2], c[1], p[1]);
        u += (periodised_gauss(z, c[4], c[1], p[1]) * periodised_gauss(y, c[3], c[1], p[1])) * gx;
      }
      return u;
    }
    case 3: {
      const double dp = x - p[2], dm = x - p[3];
      const double rp = sqrt(dp * dp + y * y + z * z), rm = sqrt(dm * dm + y * y + z * z);
      const double s = p[0] / (2.0 * rp) + p[1] / (2.0 * rm);
      const double psi = 1.0 + s;
      if (v == 0) return 1.0 / (psi * psi);
      if (v == 1 || v == 4 || v == 6) return 1.0;
      if (v == 18) return 0.5 * (1.0 + (1.0 - s) / (1.0 + s));
      return 0.0;
    }
    case 4: {
      const double A = p[0], s2 = p[1] * p[1], t = p[2];
      const double r = sqrt(x * x + y * y + z * z);
      auto f = [&](double q) { return A * exp(-q * q / (2.0 * s2)); };
      if (r < 1e-9) {
        const double ft = f(t);
        return v == 0 ? 2.0 * t / s2 * ft : 2.0 * ft * (1.0 - t * t / s2) / s2;
      }
      if (v == 0) return (f(t - r) - f(t + r)) / r;
      return -(f(t - r) * (t - r) - f(t + r) * (t + r)) / (s2 * r);
    }
    default:
      return 0.0;
  }
}

// Deterministic reductions: a grid of ceil(n / kNormPointsPerPart)
// workgroups (the count depends only on n), each thread accumulating a fixed
// strided subset, then a fixed butterfly over the 64 lanes of each wave
// (cross-lane shuffles), the four waves combined in order, and one final
// workgroup combining the partials the same way.  Every call on the same data
// gives the same bits.  Accumulated per point: a max term, a sum term, a
// weight term and a count of non-finite values.
struct Acc {
  double m, s, w, bad;
};

__device__ __forceinline__ Acc acc_combine(Acc a, Acc b) {
  return {fmax(a.m, b.m), a.s + b.s, a.w + b.w, a.bad + b.bad};
}

__device__ __forceinline__ Acc acc_block(Acc a, Acc* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Acc o;
    o.m = __shfl_xor(a.m, off, 64);
    o.s = __shfl_xor(a.s, off, 64);
    o.w = __shfl_xor(a.w, off, 64);
    o.bad = __shfl_xor(a.bad, off, 64);
    a = acc_combine(a, o);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) lds[wave] = a;
  __syncthreads();
  Acc r = lds[0];
  for (int w = 1; w < (int)(blockDim.x / 64); ++w) r = acc_combine(r, lds[w]);
  return r;
}

// Point i of a reduction: its canonical offset and global index.
__device__ __forceinline__ int64_t canonical_point(const PackArgs& a, int64_t i, int gi[3]) {
  int b = 0;
  while (b + 1 < a.nboxes && a.prefix[b + 1] <= i) ++b;
  const BoxDev B = a.boxes[b];
  const int64_t l = i - a.prefix[b];
  const int x = (int)(l % B.nx), y = (int)((l / B.nx) % B.ny), z = (int)(l / ((int64_t)B.nx * B.ny));
  gi[0] = B.lo[0] + x, gi[1] = B.lo[1] + y, gi[2] = B.lo[2] + z;
  return padded_offset(B, x, y, z);
}

template <typename T>
__global__ __launch_bounds__(256) void k_norms_partial(NormArgs a, double* partials) {
  __shared__ Acc lds[4];
  Acc r{0.0, 0.0, 0.0, 0.0};
  const T* arr = static_cast<const T*>(a.p.arr);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.p.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int gi[3];
    const int64_t o = canonical_point(a.p, i, gi);
    double v = (double)arr[o], w = 1.0;
    if (a.mode == 1) {            // difference to the closed form
      const double x = a.exact.origin[0] + gi[0] * a.exact.dx;
      const double y = a.exact.origin[1] + gi[1] * a.exact.dx;
      const double z = a.exact.origin[2] + gi[2] * a.exact.dx;
      v = v - init_value(a.exact, x, y, z, a.exact.var);
    } else if (a.mode == 2) {     // composite-grid weight of a constraint value
      bool covered = false;
      for (int c = 0; c < a.nchild; ++c) {
        const BoxDev& C = a.child[c];
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int n = d == 0 ? C.nx : (d == 1 ? C.ny : C.nz);
          in = in && 2 * gi[d] >= C.lo[d] && 2 * gi[d] < C.lo[d] + n;
        }
        covered = covered || in;
      }
      const double x = a.exact.origin[0] + gi[0] * a.exact.dx;
      const double y = a.exact.origin[1] + gi[1] * a.exact.dx;
      const double z = a.exact.origin[2] + gi[2] * a.exact.dx;
      const double rr = sqrt((x * x + y * y) + z * z);
      w = (!covered && rr < a.rmax && a.alpha[o] > a.amin) ? a.cell : 0.0;
      if (w == 0.0) continue;
    }
    if (!isfinite(v)) {
      r.bad += 1.0;
    } else {
      r.m = fmax(r.m, fabs(v));
      r.s += w * (v * v);
      r.w += w;
    }
  }
  r = acc_block(r, lds);
  if (threadIdx.x == 0) {
    partials[4 * blockIdx.x + 0] = r.m;
    partials[4 * blockIdx.x + 1] = r.s;
    partials[4 * blockIdx.x + 2] = r.w;
    partials[4 * blockIdx.x + 3] = r.bad;
  }
}

__global__ __launch_bounds__(256) void k_norms_final(const double* partials, int nparts,
                                                     double* out) {
  __shared__ Acc lds[4];
  Acc r{0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += blockDim.x)
    r = acc_combine(r, Acc{partials[4 * i], partials[4 * i + 1], partials[4 * i + 2],
                           partials[4 * i + 3]});
  r = acc_block(r, lds);
  if (threadIdx.x == 0) {
    out[0] = r.m;
    out[1] = r.s;
    out[2] = r.w;
    out[3] = r.bad;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const int64_t* idx, int64_t n, const T* src,
                                                double* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[idx[i]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const int64_t* idx, int64_t n, const double* src,
                                                 T* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = (T)src[i];
}

// Stage value from a stage-1 table (FP64) and an increment table (FP32).
__global__ __launch_bounds__(256) void k_gather_sum(const int64_t* idx, int64_t n, const double* base,
                                                    const float* inc, double* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = base[idx[i]] + (double)inc[idx[i]];
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_value(const int64_t* idx, int64_t n, T v, T* dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = v;
}

__global__ __launch_bounds__(256) void k_to_f32(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

__global__ __launch_bounds__(256) void k_init(InitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int64_t off;
  int gi[3];
  if (!a.idx) {   // owned point i of the member, canonical order
    int b = 0;
    while (b + 1 < a.nboxes && a.prefix[b + 1] <= i) ++b;
    const BoxDev B = a.boxes[b];
    const int64_t l = i - a.prefix[b];
    const int lx = (int)(l % B.nx), ly = (int)((l / B.nx) % B.ny);
    const int lz = (int)(l / ((int64_t)B.nx * B.ny));
    off = padded_offset(B, lx, ly, lz);
    gi[0] = B.lo[0] + lx, gi[1] = B.lo[1] + ly, gi[2] = B.lo[2] + lz;
  } else {        // a halo point given by its level-array offset
    off = a.idx[i];
    int b = 0;
    while (b + 1 < a.nboxes && a.boxes[b + 1].base <= off) ++b;
    const BoxDev B = a.boxes[b];
    const int64_t r = off - B.base;
    gi[0] = B.lo[0] + (int)(r % B.px) - B.pad;
    gi[1] = B.lo[1] + (int)((r / B.px) % B.py) - B.pad;
    gi[2] = B.lo[2] + (int)(r / ((int64_t)B.px * B.py)) - B.pad;
  }
  const double x = a.origin[0] + gi[0] * a.dx, y = a.origin[1] + gi[1] * a.dx,
               z = a.origin[2] + gi[2] * a.dx;
  if (a.idx) {
    a.out[i] = init_value(a, x, y, z, a.var);
    return;
  }
  for (int v = 0; v < a.nvars; ++v) {
    const double val = init_value(a, x, y, z, v);
    a.out[off + v * a.vstride] = val;
    if (a.out32) a.out32[off + v * a.vstride] = (float)val;
  }
}

inline unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// FP64: every stage <double, double>.  Mixed: stage 1 <double, float> (k1 =
// f(y_n) in FP64, stored FP32), stages 2-4 <float, float> (increment form).
template <bool MIXED, int DEPTH, int S, int NT, int R>
void stage_dispatch(const StageArgs& a, dim3 g, hipStream_t s) {
  using TS = typename std::conditional<MIXED, float, double>::type;
  using TK = TS;
  const dim3 b(NT);
  switch (a.stage) {
    case 1:
      if constexpr (MIXED)
        hipLaunchKernelGGL((k_wave_stage<1, double, float, DEPTH, S, true, NT, R>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_wave_stage<1, double, double, DEPTH, S, true, NT, R>), g, b, 0, s, a);
      break;
    case 2: hipLaunchKernelGGL((k_wave_stage<2, TS, TK, DEPTH, S, true, NT, R>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_wave_stage<3, TS, TK, DEPTH, S, true, NT, R>), g, b, 0, s, a); break;
    default:
      if (a.write_k) hipLaunchKernelGGL((k_wave_stage<4, TS, TK, DEPTH, S, true, NT, R>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_wave_stage<4, TS, TK, DEPTH, S, false, NT, R>), g, b, 0, s, a);
      break;
  }
}

// (threads, points per thread, planes in flight): (256, 2, 1), (256, 2, 2),
// (256, 1, 2), (512, 2, 1), (512, 2, 2)
template <bool MIXED, int R>
void stage_variant(const StageArgs& a, dim3 g, int depth, int slots, int threads, hipStream_t s) {
  if (threads == 512) {
    if (depth == 2) stage_dispatch<MIXED, 2, 2, 512, R>(a, g, s);
    else stage_dispatch<MIXED, 1, 2, 512, R>(a, g, s);
  } else if (slots == 1) {
    stage_dispatch<MIXED, 2, 1, 256, R>(a, g, s);
  } else {
    if (depth == 2) stage_dispatch<MIXED, 2, 2, 256, R>(a, g, s);
    else stage_dispatch<MIXED, 1, 2, 256, R>(a, g, s);
  }
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, int grid, bool mixed, int depth, int slots, int threads,
                        hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 g(grid > 0 ? grid : a.ntiles);
  if (a.radius == 4 || a.radius == 5) {   // eighth order (r = 4 or r = 8 dissipation): FP64 only
    if (mixed) return hipErrorInvalidValue;
    if (a.radius == 4) stage_variant<false, 4>(a, g, depth, slots, threads, s);
    else stage_variant<false, 5>(a, g, depth, slots, threads, s);
  } else if (a.radius == 3) {
    if (mixed) stage_variant<true, 3>(a, g, depth, slots, threads, s);
    else stage_variant<false, 3>(a, g, depth, slots, threads, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sync(const SyncArgs& a, bool f32, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (f32) hipLaunchKernelGGL(k_sync<float>, dim3(blocks_for(a.n)), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_sync<double>, dim3(blocks_for(a.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prolong(const ProlongArgs& a, bool k_f32, hipStream_t s, int nin) {
  if (a.n <= 0) return hipSuccess;
  const dim3 g(a.blk_start[8]), b(256);
  if (nin != 5) {   // buffer zones: FP64 state vectors only
    if (k_f32 || a.f32_mask || a.inc_mask || (nin != 1 && nin != 3)) return hipErrorInvalidValue;
    if (nin == 1) hipLaunchKernelGGL((k_prolong<1, double>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_prolong<3, double>), g, b, 0, s, a);
    return hipGetLastError();
  }
  if (k_f32) hipLaunchKernelGGL((k_prolong<5, float>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_prolong<5, double>), g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prolong_bricks(const BrickArgs& a, bool k_f32, hipStream_t s, int nin) {
  if (a.nbricks <= 0) return hipSuccess;
  if (a.max_pts > 3 * kBrickThreads) return hipErrorInvalidValue;
  const dim3 g((unsigned)((a.nbricks + 7) / 8 * 8)), b(kBrickThreads);   // whole XCD rounds; extra groups exit
  const bool ze2 = a.max_pts <= 2 * kBrickThreads;
  if (nin != 5) {   // buffer zones: FP64 state vectors only
    if (k_f32 || a.f32_mask || a.inc_mask || (nin != 1 && nin != 3)) return hipErrorInvalidValue;
    if (nin == 1) {
      if (ze2) hipLaunchKernelGGL((k_prolong_bricks<1, double, 2>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_prolong_bricks<1, double, 3>), g, b, 0, s, a);
    } else {
      if (ze2) hipLaunchKernelGGL((k_prolong_bricks<3, double, 2>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_prolong_bricks<3, double, 3>), g, b, 0, s, a);
    }
    return hipGetLastError();
  }
  if (k_f32) {
    if (ze2) hipLaunchKernelGGL((k_prolong_bricks<5, float, 2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_prolong_bricks<5, float, 3>), g, b, 0, s, a);
  } else {
    if (ze2) hipLaunchKernelGGL((k_prolong_bricks<5, double, 2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_prolong_bricks<5, double, 3>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_restrict(const RestrictArgs& a, hipStream_t s) {
  if (a.ntotal <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3(blocks_for(a.ntotal)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, bool unpack, bool f32, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_pack<float>, dim3(blocks_for(a.n)), dim3(256), 0, s, a, unpack ? 1 : 0);
  else
    hipLaunchKernelGGL(k_pack<double>, dim3(blocks_for(a.n)), dim3(256), 0, s, a, unpack ? 1 : 0);
  return hipGetLastError();
}

// Library-held reduction workspace for callers that cannot allocate (the
// partials of at most kNoAllocParts workgroups and the 4-double result).
// One copy per GPU, at its own address; host code must use the address from
// hipGetSymbolAddress, never the name.
static __device__ __align__(256) double scratch[4 * kNoAllocParts + 4];

hipError_t noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {   // once per device, with that device current
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr[dev]), HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      ptr[dev] = nullptr;
      return e;
    }
  }
  *out = ptr[dev];
  return hipSuccess;
}

int norm_parts(int64_t n) {
  return (int)std::max<int64_t>(1, (n + kNormPointsPerPart - 1) / kNormPointsPerPart);
}

hipError_t launch_norms(const NormArgs& a, bool f32, double* partials, double* out,
                        hipStream_t s) {
  const int nparts = norm_parts(a.p.n);
  if (f32) hipLaunchKernelGGL(k_norms_partial<float>, dim3(nparts), dim3(256), 0, s, a, partials);
  else hipLaunchKernelGGL(k_norms_partial<double>, dim3(nparts), dim3(256), 0, s, a, partials);
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(256), 0, s, partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_gather(const int64_t* idx, int64_t n, const void* src, bool f32, double* dst,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_gather<float>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n,
                       static_cast<const float*>(src), dst);
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n,
                       static_cast<const double*>(src), dst);
  return hipGetLastError();
}

hipError_t launch_fill(void* p, int64_t n, double v, bool f32, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(n)), dim3(256), 0, s,
                       static_cast<float*>(p), n, (float)v);
  else
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(n)), dim3(256), 0, s,
                       static_cast<double*>(p), n, v);
  return hipGetLastError();
}

hipError_t launch_scatter(const int64_t* idx, int64_t n, const double* src, void* dst, bool f32,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_scatter<float>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, src,
                       static_cast<float*>(dst));
  else
    hipLaunchKernelGGL(k_scatter<double>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, src,
                       static_cast<double*>(dst));
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<unsigned int>, dim3(blocks_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_gather_sum(const int64_t* idx, int64_t n, const double* base, const float* inc,
                             double* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_sum, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, base, inc, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_value(const int64_t* idx, int64_t n, double v, void* dst, bool f32,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_scatter_value<float>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n,
                       (float)v, static_cast<float*>(dst));
  else
    hipLaunchKernelGGL(k_scatter_value<double>, dim3(blocks_for(n)), dim3(256), 0, s, idx, n, v,
                       static_cast<double*>(dst));
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init, dim3(blocks_for(a.n)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace sc
