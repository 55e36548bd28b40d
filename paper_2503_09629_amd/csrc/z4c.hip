// Z4c right-hand side (Sec. III.A) with the puncture gauge and Kreiss-Oliger
// dissipation (Sec. III.C), fused with the RK4 stage update, for gfx950.
//
// Variables (slot order): W, gt_xx,xy,xz,yy,yz,zz, Khat, At_xx..zz, Theta,
// Gt^x,y,z, alpha, beta^x,y,z.  Vacuum.  Derivatives: fourth-order (or,
// with four ghost layers, eighth-order) centred first and second differences,
// mixed second derivatives as D1_a(D1_b); advection beta^k d_k with the
// centred first difference; dissipation with r = 4 (or, with five ghost
// layers, r = 8).  The relations the
// paper's equations use without printing them are the standard conformal
// ones: Gt_kij = (d_i gt_jk + d_j gt_ik - d_k gt_ij)/2, Gt^k_ij = gt^kl Gt_lij,
// Gd^i = gt^jk Gt^i_jk, physical Christoffels
// G^k_ij = Gt^k_ij - (delta^k_i d_j W + delta^k_j d_i W - gt_ij gt^kl d_l W)/W,
// D^i D_i alpha = W^2 gt^ij D_i D_j alpha, R = W^2 gt^ij R_ij,
// [X]^TF = X - gt gt^kl X_kl / 3.
//
// The arithmetic type TS is double, or float for the FP32-RHS variant (FP32
// stage vector and slopes, FP32 right-hand side; y_{n+1} is formed in FP64
// from FP64 y_n and the stored slopes, with its FP32 shadow beside it).
//
// The stage vector is materialised once per stage (k_z4c_combine writes the
// owned points into the stage's halo table, whose halo the ghost fills have
// written), because every one of its 22 components is read about 40 times by
// the stencils; a stencil tap is then one load from one padded array.
//
// FP64 right-hand side, in passes over the level: k_z4c_derivs stores the 114
// first and second derivatives the later passes use in a per-point scratch;
// k_z4c_geom (two launches) forms the curvature terms into a second scratch;
// k_z4c_evol the evolution, gauge and damping terms; k_z4c_advko adds the
// advection and the dissipation and completes the stage.  The FP32 variant
// runs the curvature and evolution terms in one pass, one thread per point,
// with the first derivatives in registers and every second derivative
// contracted as soon as it is formed.
#include "device.hpp"
#include "z4c.hpp"

namespace sc {
namespace {

constexpr int VW = 0, VG = 1, VKH = 7, VA = 8, VTH = 14, VGAM = 15, VALP = 18, VB = 19, NV = 22;

__device__ __forceinline__ int sym(int i, int j) {
  // (0,0)->0 (0,1)->1 (0,2)->2 (1,1)->3 (1,2)->4 (2,2)->5
  const int a = i < j ? i : j, b = i < j ? j : i;
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

// Scratch slot of the first derivative d_k of variable v, and of the second
// derivative d_k d_l (k <= l), in the derivative pass's arrays (-1: not stored).
__host__ __device__ constexpr int der1_slot(int v, int k) {
  const int s = v == VW ? 0 : (v >= VG && v < VG + 6) ? v : v == VKH ? 7 : v == VTH ? 8
              : (v >= VGAM && v < VGAM + 3) ? 9 + (v - VGAM) : v == VALP ? 12
              : (v >= VB && v < VB + 3) ? 13 + (v - VB) : -1;
  return s < 0 ? -1 : 3 * s + k;
}
__host__ __device__ constexpr int der2_slot(int v, int k, int l) {
  const int s = (v >= VG && v < VG + 6) ? v - VG : v == VW ? 6 : v == VALP ? 7
              : (v >= VB && v < VB + 3) ? 8 + (v - VB) : -1;
  const int a = k < l ? k : l, b = k < l ? l : k;
  const int pr = a == 0 ? b : (a == 1 ? 2 + b : 5);
  return s < 0 ? -1 : kZ4cDer1 + 6 * s + pr;
}

// ORD: 4 (five-point centred derivatives) or 8 (nine-point, four ghost layers)
// SCR: take first derivatives and second derivatives from the derivative
// pass's scratch (FP64) instead of forming them from stencil taps
// LDS: the taps come from one variable's planes staged in LDS (plane z + dz
// at lds + zb[dz + reach], the point at offset lo, row pitch lpx) instead of
// the stage vector
template <typename TS, int ORD, bool SCR = false, bool LDS = false>
struct Pt {
  const Z4cArgs* a;
  BoxDev B;
  int x, y, z;
  int64_t o;
  int64_t px, pxy;
  const TS* lds;
  int lo, lpx;
  int zb[ORD == 8 ? 9 : 5];
  // the stage vector on the whole padded box (owned points and halo) is one
  // array, so a tap is one unconditional load
  __device__ TS at(int v, int dx, int dy, int dz) const {
    if constexpr (LDS) return lds[zb[dz + (ORD == 8 ? 4 : 2)] + lo + dx + dy * lpx];
    else return static_cast<const TS*>(a->Y)[o + dx + dy * px + dz * pxy + v * a->vstride];
  }
  __device__ TS tap(int v, int d, int j) const {
    return at(v, d == 0 ? j : 0, d == 1 ? j : 0, d == 2 ? j : 0);
  }
  // first difference from the taps t(-R..R) (c1 = 1/(12h) or 1/(840h))
  template <typename Tap>
  __device__ static TS diff1(const Tap& t, TS c1) {
    if constexpr (ORD == 8)
      return (((((((TS(3.0) * t(-4) - TS(32.0) * t(-3)) + TS(168.0) * t(-2)) - TS(672.0) * t(-1)) +
                 TS(672.0) * t(1)) - TS(168.0) * t(2)) + TS(32.0) * t(3)) - TS(3.0) * t(4)) * c1;
    else
      return (((t(-2) - TS(8.0) * t(-1)) + TS(8.0) * t(1)) - t(2)) * c1;
  }
  __device__ TS d1(int v, int d, TS c1) const {
    if constexpr (SCR)   // the passes never use the derivatives that are not stored
      return der1_slot(v, d) < 0 ? TS(0.0) : a->der[o + der1_slot(v, d) * a->vstride];
    else if constexpr (ORD == 8)
      return diff1([&](int j) { return tap(v, d, j); }, c1);
    else   // written out: this form keeps the fourth-order kernels' register allocation
      return (((tap(v, d, -2) - TS(8.0) * tap(v, d, -1)) + TS(8.0) * tap(v, d, 1)) - tap(v, d, 2)) * c1;
  }
  __device__ TS d2(int v, int d, TS c2) const {
    if constexpr (ORD == 8)
      return ((((((((-TS(9.0) * tap(v, d, -4) + TS(128.0) * tap(v, d, -3)) - TS(1008.0) * tap(v, d, -2)) +
                   TS(8064.0) * tap(v, d, -1)) - TS(14350.0) * tap(v, d, 0)) + TS(8064.0) * tap(v, d, 1)) -
                TS(1008.0) * tap(v, d, 2)) + TS(128.0) * tap(v, d, 3)) - TS(9.0) * tap(v, d, 4)) * c2;
    else
      return ((((-tap(v, d, -2) + TS(16.0) * tap(v, d, -1)) - TS(30.0) * tap(v, d, 0)) + TS(16.0) * tap(v, d, 1)) -
              tap(v, d, 2)) * c2;
  }
  // D1 along d of D1 along e
  __device__ TS dm(int v, int d, int e, TS c1) const {
    auto inner = [&](int j) {
      const int sx = (d == 0 ? j : 0), sy = (d == 1 ? j : 0), sz = (d == 2 ? j : 0);
      auto t = [&](int i) {
        return at(v, sx + (e == 0 ? i : 0), sy + (e == 1 ? i : 0), sz + (e == 2 ? i : 0));
      };
      if constexpr (ORD == 8) return diff1(t, c1);
      else return (((t(-2) - TS(8.0) * t(-1)) + TS(8.0) * t(1)) - t(2)) * c1;
    };
    if constexpr (ORD == 8) return diff1(inner, c1);
    else return (((inner(-2) - TS(8.0) * inner(-1)) + TS(8.0) * inner(1)) - inner(2)) * c1;
  }
  __device__ TS ko(int v, int d) const {
    return (((((tap(v, d, -3) - TS(6.0) * tap(v, d, -2)) + TS(15.0) * tap(v, d, -1)) - TS(20.0) * tap(v, d, 0)) +
             TS(15.0) * tap(v, d, 1)) - TS(6.0) * tap(v, d, 2)) + tap(v, d, 3);
  }
  // second derivative (k, l) with k <= l
  __device__ TS dd(int v, int k, int l, TS c1, TS c2) const {
    if constexpr (SCR)
      return der2_slot(v, k, l) < 0 ? TS(0.0) : a->der[o + der2_slot(v, k, l) * a->vstride];
    else return k == l ? d2(v, k, c2) : dm(v, k, l, c1);
  }
};

// Curvature pass (one point): the Ricci tensor R_ij, D_i D_j alpha, the
// contracted conformal Christoffels Gt^i, Gt^i_jk At^jk and the shift's
// gt^jk d_j d_k beta^i and d_i (d_k beta^k), written to the per-point scratch
// (24 values: R and D_i D_j alpha in symmetric order, then Gt^i,
// Gt^i_jk At^jk, gt^jk d_j d_k beta^i, d_i d_k beta^k), or the Hamiltonian
// constraint.
// PART 0: all 24 values (or the constraint); 1: R_ij and Gt^i (or the
// constraint); 2: D_i D_j alpha, Gt^i_jk At^jk and the shift terms.  Each
// value is computed the same way in every part.
template <typename TS, int ORD, bool SCR, int PART = 0>
__device__ void z4c_geom(const Pt<TS, ORD, SCR>& p, const Z4cArgs& a, TS* out, double* ham_out) {
  const TS h = TS(a.h);
  const TS c1 = TS(1.0) / (TS(ORD == 8 ? 840.0 : 12.0) * h);
  const TS c2 = TS(1.0) / (TS(ORD == 8 ? 5040.0 : 12.0) * h * h);
  TS v[NV], d[NV][3];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i] = p.at(i, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) d[i][k] = p.d1(i, k, c1);
  }
  [[maybe_unused]] const TS W = v[VW], Kh = v[VKH], Th = v[VTH], alp = v[VALP];
  TS gt[3][3], At[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gt[i][j] = v[VG + sym(i, j)];
      At[i][j] = v[VA + sym(i, j)];
    }
  const TS det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                     gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                     gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  TS gu[3][3];
  gu[0][0] = (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) / det;
  gu[0][1] = (gt[0][2] * gt[2][1] - gt[0][1] * gt[2][2]) / det;
  gu[0][2] = (gt[0][1] * gt[1][2] - gt[0][2] * gt[1][1]) / det;
  gu[1][1] = (gt[0][0] * gt[2][2] - gt[0][2] * gt[2][0]) / det;
  gu[1][2] = (gt[0][2] * gt[1][0] - gt[0][0] * gt[1][2]) / det;
  gu[2][2] = (gt[0][0] * gt[1][1] - gt[0][1] * gt[1][0]) / det;
  gu[1][0] = gu[0][1];
  gu[2][0] = gu[0][2];
  gu[2][1] = gu[1][2];
  // Christoffel symbols of the conformal metric: Gl[k][i][j] = Gt_kij, G = Gt^k_ij
  TS Gl[3][3][3], G[3][3][3], Gd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Gl[k][i][j] = TS(0.5) * ((d[VG + sym(j, k)][i] + d[VG + sym(i, k)][j]) - d[VG + sym(i, j)][k]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        TS s = TS(0.0);
#pragma unroll
        for (int l = 0; l < 3; ++l) s += gu[k][l] * Gl[l][i][j];
        G[k][i][j] = s;
      }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    TS s = TS(0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) s += gu[j][k] * G[i][j][k];
    Gd[i] = s;
  }
  const TS dW[3] = {d[VW][0], d[VW][1], d[VW][2]};
  TS R[3][3], Rs = TS(0.0);
  if constexpr (PART != 2) {
  // -1/2 gt^lm d_l d_m gt_ij, contracted as each second derivative is formed
  TS Rlap[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    TS dd[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = k; l < 3; ++l) {
        dd[k][l] = p.dd(VG + c, k, l, c1, c2);
        dd[l][k] = dd[k][l];
      }
    TS s = TS(0.0);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) s -= TS(0.5) * gu[l][m] * dd[l][m];
    Rlap[c] = s;
  }
  TS ddW[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = k; l < 3; ++l) {
      ddW[k][l] = p.dd(VW, k, l, c1, c2);
      ddW[l][k] = ddW[k][l];
    }
  // Ricci tensor R_ij = R^W_ij + Rt_ij
  TS DDW[3][3], lapW = TS(0.0), dWsq = TS(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      TS s = ddW[i][j];
#pragma unroll
      for (int k = 0; k < 3; ++k) s -= G[k][i][j] * dW[k];
      DDW[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      lapW += gu[i][j] * DDW[i][j];
      dWsq += gu[i][j] * dW[i] * dW[j];
    }
  dWsq /= W * W;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      TS rt = Rlap[sym(i, j)];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        rt += TS(0.5) * (gt[k][i] * d[VGAM + k][j] + gt[k][j] * d[VGAM + k][i]);
        rt += Gd[k] * TS(0.5) * (Gl[i][j][k] + Gl[j][i][k]);
      }
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          TS s = TS(0.0);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            s += (G[k][l][i] * Gl[j][k][m] + G[k][l][j] * Gl[i][k][m]) + G[k][i][m] * Gl[k][l][j];
          rt += gu[l][m] * s;
        }
      const TS rw = DDW[i][j] / W + gt[i][j] * lapW / W - TS(2.0) * gt[i][j] * dWsq;
      R[i][j] = rw + rt;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Rs += gu[i][j] * R[i][j];
  Rs *= W * W;
  }   // PART != 2
  // raised At
  TS Atu[3][3], Atm[3][3], AtA = TS(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      TS s = TS(0.0), m = TS(0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        m += gu[i][k] * At[k][j];
#pragma unroll
        for (int l = 0; l < 3; ++l) s += gu[i][k] * gu[j][l] * At[k][l];
      }
      Atu[i][j] = s;
      Atm[i][j] = m;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AtA += At[i][j] * Atu[i][j];
  const TS Kt = Kh + TS(2.0) * Th;
  if constexpr (PART != 2) {
    if (ham_out) {
      *ham_out = (double)(Rs + (TS(2.0) / TS(3.0)) * Kt * Kt - AtA);
      return;
    }
  }
  if constexpr (PART != 2) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) out[sym(i, j)] = R[i][j];
#pragma unroll
    for (int i = 0; i < 3; ++i) out[12 + i] = Gd[i];
  }
  if constexpr (PART == 1) return;
  else {
  TS dda[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = k; l < 3; ++l) {
      dda[k][l] = p.dd(VALP, k, l, c1, c2);
      dda[l][k] = dda[k][l];
    }
  // lapse: D_i D_j alpha with the physical Christoffels
  const TS da[3] = {d[VALP][0], d[VALP][1], d[VALP][2]};
  TS gudW[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    TS s = TS(0.0);
#pragma unroll
    for (int l = 0; l < 3; ++l) s += gu[k][l] * dW[l];
    gudW[k] = s;
  }
  TS DDa[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      TS s = dda[i][j];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const TS Gp = G[k][i][j] - (((k == i ? dW[j] : TS(0.0)) + (k == j ? dW[i] : TS(0.0))) -
                                         gt[i][j] * gudW[k]) / W;
        s -= Gp * da[k];
      }
      DDa[i][j] = s;
    }
  TS t2[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    TS s = TS(0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) s += G[i][j][k] * Atu[j][k];
    t2[i] = s;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) out[6 + sym(i, j)] = DDa[i][j];
  // shift: gt^jk d_j d_k beta^i and d_j (d_k beta^k)
  TS lapb[3], gdivb[3] = {TS(0.0), TS(0.0), TS(0.0)};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    TS dd[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = k; l < 3; ++l) {
        dd[k][l] = p.dd(VB + i, k, l, c1, c2);
        dd[l][k] = dd[k][l];
      }
    TS s = TS(0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) s += gu[j][k] * dd[j][k];
    lapb[i] = s;
#pragma unroll
    for (int j = 0; j < 3; ++j) gdivb[j] += dd[j][i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    out[15 + i] = t2[i];
    out[18 + i] = lapb[i];
    out[21 + i] = gdivb[i];
  }
  }   // PART != 1
}

// Evolution pass (one point): every right-hand side except advection and
// dissipation, from the curvature scratch of the same point.
// geo(c) returns curvature value c of the point (the order z4c_geom writes).
template <typename TS, int ORD, bool SCR, typename Geo>
__device__ void z4c_evol(const Pt<TS, ORD, SCR>& p, const Z4cArgs& a, const Geo& geo, TS* rhs) {
  const TS h = TS(a.h);
  const TS c1 = TS(1.0) / (TS(ORD == 8 ? 840.0 : 12.0) * h);
  TS v[NV], d[NV][3];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    v[i] = p.at(i, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) d[i][k] = p.d1(i, k, c1);
  }
  [[maybe_unused]] const TS W = v[VW], Kh = v[VKH], Th = v[VTH], alp = v[VALP];
  TS gt[3][3], At[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gt[i][j] = v[VG + sym(i, j)];
      At[i][j] = v[VA + sym(i, j)];
    }
  const TS det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                     gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                     gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  TS gu[3][3];
  gu[0][0] = (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) / det;
  gu[0][1] = (gt[0][2] * gt[2][1] - gt[0][1] * gt[2][2]) / det;
  gu[0][2] = (gt[0][1] * gt[1][2] - gt[0][2] * gt[1][1]) / det;
  gu[1][1] = (gt[0][0] * gt[2][2] - gt[0][2] * gt[2][0]) / det;
  gu[1][2] = (gt[0][2] * gt[1][0] - gt[0][0] * gt[1][2]) / det;
  gu[2][2] = (gt[0][0] * gt[1][1] - gt[0][1] * gt[1][0]) / det;
  gu[1][0] = gu[0][1];
  gu[2][0] = gu[0][2];
  gu[2][1] = gu[1][2];
  TS R[3][3], DDa[3][3], Gd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      R[i][j] = geo(sym(i, j));
      DDa[i][j] = geo(6 + sym(i, j));
    }
#pragma unroll
  for (int i = 0; i < 3; ++i) Gd[i] = geo(12 + i);
  TS lapb[3], gdivb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lapb[i] = geo(18 + i);
    gdivb[i] = geo(21 + i);
  }
  const TS dW[3] = {d[VW][0], d[VW][1], d[VW][2]};
  const TS da[3] = {d[VALP][0], d[VALP][1], d[VALP][2]};
  TS Rs = TS(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Rs += gu[i][j] * R[i][j];
  Rs *= W * W;
  TS lapa = TS(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) lapa += gu[i][j] * DDa[i][j];
  lapa *= W * W;
  // raised At
  TS Atu[3][3], Atm[3][3], AtA = TS(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      TS s = TS(0.0), m = TS(0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        m += gu[i][k] * At[k][j];
#pragma unroll
        for (int l = 0; l < 3; ++l) s += gu[i][k] * gu[j][l] * At[k][l];
      }
      Atu[i][j] = s;
      Atm[i][j] = m;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AtA += At[i][j] * Atu[i][j];
  const TS Kt = Kh + TS(2.0) * Th;
  const TS beta[3] = {v[VB], v[VB + 1], v[VB + 2]};
  TS divb = TS(0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) divb += d[VB + k][k];
  rhs[VW] = (TS(1.0) / TS(3.0)) * W * (alp * Kt - divb);
  TS trX = TS(0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) trX += gu[k][l] * (-DDa[k][l] + alp * R[k][l]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      TS lg = TS(0.0), la = TS(0.0), aa = TS(0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lg += gt[k][i] * d[VB + k][j] + gt[k][j] * d[VB + k][i];
        la += At[k][i] * d[VB + k][j] + At[k][j] * d[VB + k][i];
        aa += Atm[k][i] * At[k][j];
      }
      const int s = sym(i, j);
      rhs[VG + s] = -TS(2.0) * alp * At[i][j] + lg - (TS(2.0) / TS(3.0)) * gt[i][j] * divb;
      const TS tf = (-DDa[i][j] + alp * R[i][j]) - (TS(1.0) / TS(3.0)) * gt[i][j] * trX;
      rhs[VA + s] = W * W * tf + alp * (Kt * At[i][j] - TS(2.0) * aa) + la -
                    (TS(2.0) / TS(3.0)) * At[i][j] * divb;
    }
  rhs[VKH] = -lapa + alp * (AtA + (TS(1.0) / TS(3.0)) * Kt * Kt) +
             alp * TS(a.kappa1) * (TS(1.0) - TS(a.kappa2)) * Th;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    TS t1 = TS(0.0), t3 = TS(0.0), t4 = TS(0.0), t6 = TS(0.0), t7 = TS(0.0);
    const TS t2 = geo(15 + i);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      t1 += Atu[i][j] * da[j];
      t3 += Atu[i][j] * dW[j] / W;
      t4 += gu[i][j] * (TS(2.0) * d[VKH][j] + d[VTH][j]);
      t6 += gu[i][j] * gdivb[j];
      t7 += Gd[j] * d[VB + i][j];
    }
    rhs[VGAM + i] = -TS(2.0) * t1 + TS(2.0) * alp * (t2 - TS(3.0) * t3 - (TS(1.0) / TS(3.0)) * t4) +
                    lapb[i] + (TS(1.0) / TS(3.0)) * t6 - t7 + (TS(2.0) / TS(3.0)) * Gd[i] * divb -
                    TS(2.0) * alp * TS(a.kappa1) * (v[VGAM + i] - Gd[i]);
  }
  rhs[VTH] = TS(0.5) * alp * (Rs - AtA + (TS(2.0) / TS(3.0)) * Kt * Kt) -
             alp * TS(a.kappa1) * (TS(2.0) + TS(a.kappa2)) * Th;
  rhs[VALP] = -TS(2.0) * alp * Kh;
  // damping eta(r) from the point's coordinates, in FP64
  const double xc = a.origin[0] + (p.B.lo[0] + p.x) * a.h;
  const double yc = a.origin[1] + (p.B.lo[1] + p.y) * a.h;
  const double zc = a.origin[2] + (p.B.lo[2] + p.z) * a.h;
  const double r = sqrt(xc * xc + yc * yc + zc * zc);
  const double rq = r / a.eta_s;
  const TS eta = TS((a.eta_c - a.eta_o) * exp(-(rq * rq) * (rq * rq)) + a.eta_o);
#pragma unroll
  for (int i = 0; i < 3; ++i) rhs[VB + i] = TS(0.75) * v[VGAM + i] - eta * beta[i];
  // the advection terms beta^k d_k and the dissipation are added by k_z4c_advko
}

// First tile of a persistent workgroup.  Consecutive workgroups land on
// different XCDs (round robin over 8); giving each XCD a contiguous run of the
// tile list lets neighbouring tiles, whose stencil halos overlap, share its L2.
__device__ __forceinline__ int xcd_first_tile() {
  return gridDim.x % 8 == 0 ? (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8)
                            : (int)blockIdx.x;
}

// One thread per owned point of the tiles: calls point(p) for each.
template <typename TS, int ORD, bool SCR, typename F>
__device__ __forceinline__ void z4c_points(const Z4cArgs& a, F point) {
  for (int t = xcd_first_tile(); t < a.ntiles; t += gridDim.x) {
    const TileDev T = a.tiles[t];
    const BoxDev B = a.boxes[T.box];
    // threads packed over the tile's x-y points row by row: no lane idles on
    // a tile narrower than a wavefront
    for (int ixy = threadIdx.x; ixy < T.nx * T.ny; ixy += kZ4cThreads) {
      const int rx = ixy % T.nx, ry = ixy / T.nx;
      for (int iz = 0; iz < T.nz; ++iz) {
        Pt<TS, ORD, SCR> p;
        p.a = &a;
        p.B = B;
        p.x = T.x0 + rx;
        p.y = T.y0 + ry;
        p.z = T.z0 + iz;
        p.px = B.px;
        p.pxy = (int64_t)B.px * B.py;
        p.o = B.base + ((int64_t)(p.z + B.pad) * B.py + (p.y + B.pad)) * (int64_t)B.px + (p.x + B.pad);
        point(p);
      }
    }
  }
}

// Curvature pass into the per-point scratch, or the Hamiltonian constraint.
// (One kernel for both modes: on C5, measured with 16-plane tiles, this
// allocation ran faster than a constraint-free variant without spills, 3.7
// against 4.2 s per coarse step, or a split of the pass by output, 4.3 s.)
// Two launches share the work (PART 1: R_ij, Gt^i or the constraint; PART 2:
// the rest), so each holds about half of the curvature algebra's live values.
template <typename TS, int ORD, int PART>
__global__ __launch_bounds__(kZ4cThreads) void k_z4c_geom(Z4cArgs a) {
  TS* geo = static_cast<TS*>(a.geo);
  z4c_points<TS, ORD, true>(a, [&](const Pt<TS, ORD, true>& p) {
    if constexpr (sizeof(TS) == 8 && PART == 1) {
      if (a.ham) {
        double hm;
        z4c_geom<TS, ORD, true, PART>(p, a, nullptr, &hm);
        a.ham[p.o] = hm;
        return;
      }
    }
    TS g[kZ4cGeo];
    z4c_geom<TS, ORD, true, PART>(p, a, g, nullptr);
    if constexpr (PART == 1) {
#pragma unroll
      for (int c = 0; c < 6; ++c) geo[p.o + c * a.vstride] = g[c];
#pragma unroll
      for (int c = 12; c < 15; ++c) geo[p.o + c * a.vstride] = g[c];
    } else {
#pragma unroll
      for (int c = 6; c < 12; ++c) geo[p.o + c * a.vstride] = g[c];
#pragma unroll
      for (int c = 15; c < kZ4cGeo; ++c) geo[p.o + c * a.vstride] = g[c];
    }
  });
}

// Derivative pass (FP64): every first and second derivative the curvature
// and evolution passes read, formed with the same stencils as the tap form
// (so the same bits) and stored at once.  Work item: one variable on one
// derivative column (a tile of at most kDerTx x kDerTy points in x-y, a
// chunk of at most der_tz(ORD) planes in z).  The workgroup marches the
// column in z with a ring of 2H + 2 planes of the variable's block (the
// column's x-y extent plus the stencil reach H on every side) in LDS: the
// taps of a point come from the planes z - H .. z + H, and the plane H + 1
// ahead is read from memory while the current plane's derivatives are formed,
// so each stage-vector value of the block is read once per column.  At fourth order the work items run
// variable by variable over the column list, so neighbouring columns, whose
// blocks overlap, are read together from one XCD's L2; at eighth order
// (two workgroups per CU) column by column, all 16 variables of a column
// together (the faster order there, measured on C5).
template <int ORD> constexpr int kDerPlane = (kDerTx + 2 * (ORD == 8 ? 4 : 2)) *
                                             (kDerTy + 2 * (ORD == 8 ? 4 : 2));
template <int ORD>
__global__ __launch_bounds__(256, ORD == 4 ? 4 : 2) void k_z4c_derivs(Z4cArgs a) {
  constexpr int H = ORD == 8 ? 4 : 2;   // reach of the first and mixed differences
  constexpr int NP = 2 * H + 2;         // ring slots
  constexpr int P = kDerPlane<ORD>;     // slot size in doubles
  constexpr int KL = (P + 255) / 256;   // block values per thread and plane
  static_assert(kDerTx * kDerTy <= 256, "one point per thread and plane");
  __shared__ double ring[NP * P];
  const double h = a.h;
  const double c1 = 1.0 / ((ORD == 8 ? 840.0 : 12.0) * h);
  const double c2 = 1.0 / ((ORD == 8 ? 5040.0 : 12.0) * h * h);
  // the 16 variables with stored first derivatives; the first 11 of them in
  // V2 order have stored second derivatives too
  constexpr int VS[16] = {VG, VG + 1, VG + 2, VG + 3, VG + 4, VG + 5, VW, VALP, VB, VB + 1, VB + 2,
                          VKH, VTH, VGAM, VGAM + 1, VGAM + 2};
  const int nwork = a.ndtiles * 16;
  const int tid = threadIdx.x;
  for (int w = xcd_first_tile(); w < nwork; w += gridDim.x) {
    const int n = ORD == 8 ? w % 16 : w / a.ndtiles;
    const TileDev T = a.dtiles[ORD == 8 ? w / 16 : w - n * a.ndtiles];
    const BoxDev B = a.boxes[T.box];
    const int v = VS[n];
    const int bx = T.nx + 2 * H, nxy = bx * (T.ny + 2 * H);
    const int64_t pxy = (int64_t)B.px * B.py;
    // this thread's places of the block plane (tid + 256 k), as offsets
    // within a plane of the box
    int32_t oxy[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int e = tid + k * 256;
      const int ly = e / bx, lx = e - ly * bx;
      oxy[k] = (T.y0 + ly - H + B.pad) * B.px + (T.x0 + lx - H + B.pad);
    }
    // block plane j (z = z0 - H + j) of the variable
    const double* src = static_cast<const double*>(a.Y) + B.base + v * a.vstride +
                        (int64_t)(T.z0 - H + B.pad) * pxy;
    for (int j = 0; j <= 2 * H; ++j)
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = tid + k * 256;
        if (e < nxy) ring[j * P + e] = src[j * pxy + oxy[k]];
      }
    __syncthreads();
    const bool own = tid < T.nx * T.ny;
    const int rx = own ? tid % T.nx : 0, ry = own ? tid / T.nx : 0;
    int64_t o = B.base + ((int64_t)(T.z0 + B.pad) * B.py + (T.y0 + ry + B.pad)) * (int64_t)B.px +
                (T.x0 + rx + B.pad);
    int s0 = 0;   // ring slot of block plane iz (z - H)
    for (int iz = 0; iz < T.nz; ++iz) {
      // block plane iz + 2H + 1, needed from the next plane on
      const bool more = iz + 1 < T.nz;
      double pre[KL];
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = tid + k * 256;
        pre[k] = (more && e < nxy) ? src[(int64_t)(iz + 2 * H + 1) * pxy + oxy[k]] : 0.0;
      }
      if (own) {
        Pt<double, ORD, false, true> p;
        p.lds = ring;
        p.lpx = bx;
        p.lo = (ry + H) * bx + (rx + H);
#pragma unroll
        for (int m = 0; m <= 2 * H; ++m) p.zb[m] = (s0 + m < NP ? s0 + m : s0 + m - NP) * P;
#pragma unroll
        for (int k = 0; k < 3; ++k) a.der[o + der1_slot(v, k) * a.vstride] = p.d1(v, k, c1);
        if (n < 11)
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = k; l < 3; ++l)
              a.der[o + der2_slot(v, k, l) * a.vstride] = p.dd(v, k, l, c1, c2);
      }
      // the slot of block plane iz - 1, which no thread reads any more
      const int sw = s0 == 0 ? NP - 1 : s0 - 1;
      if (more)
#pragma unroll
        for (int k = 0; k < KL; ++k) {
          const int e = tid + k * 256;
          if (e < nxy) ring[sw * P + e] = pre[k];
        }
      __syncthreads();
      s0 = s0 + 1 == NP ? 0 : s0 + 1;
      o += pxy;
    }
  }
}

// Gauge, constraint-damping and source terms of the right-hand side (no
// advection, no dissipation) from the curvature scratch.
// FUSED: the curvature pass runs in the same thread and hands its values over
// in registers (no scratch traffic, more registers live).
template <typename TS, bool FUSED, int ORD>
__global__ __launch_bounds__(kZ4cThreads) void k_z4c_stage(Z4cArgs a) {
  TS* kout = static_cast<TS*>(a.kout);
  // FP32 (fused): taps; FP64: derivatives from the derivative pass
  constexpr bool SCR = !FUSED;
  z4c_points<TS, ORD, SCR>(a, [&](const Pt<TS, ORD, SCR>& p) {
    TS rhs[NV];
    if constexpr (FUSED) {
      TS g[kZ4cGeo];
      z4c_geom<TS, ORD, SCR>(p, a, g, nullptr);
      z4c_evol<TS, ORD, SCR>(p, a, [&](int c) -> TS { return g[c]; }, rhs);
    } else {
      const TS* geo = static_cast<const TS*>(a.geo);
      z4c_evol<TS, ORD, SCR>(p, a, [&](int c) -> TS { return geo[p.o + c * a.vstride]; }, rhs);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) kout[p.o + i * a.vstride] = rhs[i];
  });
}

// Evolution pass, FP64: k_z4c_stage without the fused curvature, held to two
// waves per SIMD (it needs a few registers more than half the file).
template <int ORD>
__global__ __launch_bounds__(kZ4cThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_z4c_evol(Z4cArgs a) {
  double* kout = static_cast<double*>(a.kout);
  const double* geo = static_cast<const double*>(a.geo);
  z4c_points<double, ORD, true>(a, [&](const Pt<double, ORD, true>& p) {
    double rhs[NV];
    z4c_evol<double, ORD, true>(p, a, [&](int c) -> double { return geo[p.o + c * a.vstride]; },
                                rhs);
#pragma unroll
    for (int i = 0; i < NV; ++i) kout[p.o + i * a.vstride] = rhs[i];
  });
}

// Completes k_s: adds the advection terms beta^k d_k Y (centred first
// differences of the derivative order) and the Kreiss-Oliger dissipation of
// every variable; at stage 4 also forms
// y_{n+1} = y_n + (dt/6) (((k1 + 2 k2) + 2 k3) + k4) in FP64.  Both stencils
// read taps along the axes only.  KR: the dissipation's reach, 3 (r = 4,
// sigma/(64 h) delta^6) or 5 (r = 8, sigma/(1024 h) delta^10, Sec. III.C's
// ninth-order option).
template <int STAGE, typename TS, int ORD, int KR = 3>
__global__ __launch_bounds__(256) void k_z4c_advko(Z4cArgs a) {
  static_assert(KR == 3 || (KR == 5 && ORD == 8), "r = 8 dissipation: eighth order only");
  const TS* Y = static_cast<const TS*>(a.Y);
  TS* kout = static_cast<TS*>(a.kout);
  const TS* k1 = static_cast<const TS*>(a.k1);
  const TS* k2 = static_cast<const TS*>(a.k2);
  const TS* k3 = static_cast<const TS*>(a.k3);
  const TS h = TS(a.h);
  const TS c1 = TS(1.0) / (TS(ORD == 8 ? 840.0 : 12.0) * h);
  const TS cko = TS(a.sigma) / (TS(KR == 5 ? 1024.0 : 64.0) * h);
  // taps per side: the first difference's (2 or 4) or the dissipation's
  constexpr int R = KR == 5 ? 5 : (ORD == 8 ? 4 : 3);
  bool bad = false;   // stage 4: a non-finite y_{n+1} was written (reported once per thread)
  for (int t = xcd_first_tile(); t < a.ntiles; t += gridDim.x) {
    const TileDev T = a.tiles[t];
    const BoxDev B = a.boxes[T.box];
    const int64_t st[3] = {1, (int64_t)B.px, (int64_t)B.px * B.py};
    for (int ixy = threadIdx.x; ixy < T.nx * T.ny; ixy += 256) {   // packed, as in z4c_points
      const int rx = ixy % T.nx, ry = ixy / T.nx;
      for (int iz = 0; iz < T.nz; ++iz) {
        const int64_t o = B.base + ((int64_t)(T.z0 + iz + B.pad) * B.py + (T.y0 + ry + B.pad)) *
                                       (int64_t)B.px + (T.x0 + rx + B.pad);
        TS beta[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) beta[k] = Y[o + (VB + k) * a.vstride];
        for (int i = 0; i < NV; ++i) {
          const int64_t oi = o + i * a.vstride;
          TS adv = TS(0.0), ko[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            TS tp[2 * R + 1];
#pragma unroll
            for (int j = 0; j < 2 * R + 1; ++j) tp[j] = Y[oi + (j - R) * st[d]];
            const TS d1 = Pt<TS, ORD>::diff1([&](int j) { return tp[R + j]; }, c1);
            adv += beta[d] * d1;
            if constexpr (KR == 5)
              ko[d] = (((((((((tp[R - 5] - TS(10.0) * tp[R - 4]) + TS(45.0) * tp[R - 3]) -
                             TS(120.0) * tp[R - 2]) + TS(210.0) * tp[R - 1]) - TS(252.0) * tp[R]) +
                          TS(210.0) * tp[R + 1]) - TS(120.0) * tp[R + 2]) + TS(45.0) * tp[R + 3]) -
                       TS(10.0) * tp[R + 4]) + tp[R + 5];
            else
              ko[d] = (((((tp[R - 3] - TS(6.0) * tp[R - 2]) + TS(15.0) * tp[R - 1]) - TS(20.0) * tp[R]) +
                        TS(15.0) * tp[R + 1]) - TS(6.0) * tp[R + 2]) + tp[R + 3];
          }
          const TS k = (kout[oi] + adv) + cko * ((ko[0] + ko[1]) + ko[2]);
          kout[oi] = k;
          if constexpr (STAGE == 4) {
            const double s = (((double)k1[oi] + 2.0 * (double)k2[oi]) + 2.0 * (double)k3[oi]) +
                             (double)k;
            const double yv = a.yn[oi] + a.dt6 * s;
            a.ynew[oi] = yv;
            if constexpr (sizeof(TS) == 4) a.ynew32[oi] = (float)yv;
            bad = bad || !isfinite(yv);
          }
        }
      }
    }
  }
  if (STAGE == 4 && bad) atomicOr(a.nonfinite, 1u);
}

// Y = y_n + cdt k_{s-1} on the owned points of the tiles (all variables);
// Y = y_n when kprev is null (stage 1).
template <typename TS>
__global__ __launch_bounds__(256) void k_z4c_combine(Z4cCombineArgs a) {
  const TS* yn = static_cast<const TS*>(a.yn);
  const TS* kprev = static_cast<const TS*>(a.kprev);
  TS* Y = static_cast<TS*>(a.Y);
  const TS cdt = TS(a.cdt);
  for (int t = xcd_first_tile(); t < a.ntiles; t += gridDim.x) {
    const TileDev T = a.tiles[t];
    const BoxDev B = a.boxes[T.box];
    for (int ixy = threadIdx.x; ixy < T.nx * T.ny; ixy += 256) {   // packed, as in z4c_points
      const int rx = ixy % T.nx, ry = ixy / T.nx;
      for (int iz = 0; iz < T.nz; ++iz) {
        const int64_t o = B.base + ((int64_t)(T.z0 + iz + B.pad) * B.py + (T.y0 + ry + B.pad)) *
                                       (int64_t)B.px + (T.x0 + rx + B.pad);
        for (int i = 0; i < a.nvars; ++i) {
          const int64_t oi = o + i * a.vstride;
          Y[oi] = kprev ? yn[oi] + cdt * kprev[oi] : yn[oi];
        }
      }
    }
  }
}

// Stage values of the radiative ghosts: Y = y_n + c_s dt k_{s-1} (y_n at
// stage 1), evaluated as for an owned point.
__global__ __launch_bounds__(256) void k_z4c_rad_fill(Z4cRadArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t o = a.idx[i];
  for (int v = 0; v < NV; ++v) {
    const int64_t ov = o + v * a.vstride;
    a.table[ov] = a.kprev ? a.yn[ov] + a.cdt * a.kprev[ov] : a.yn[ov];
  }
}

// Outgoing (radiative) condition at a ghost point outside the domain:
// d_t f = -(v / r) (x^i d_i f + (f - f0)), r from the coordinate origin, with
// second-order one-sided differences pointing inwards along directions in
// which the point lies outside the box and centred ones along the others.
// f0 = 1 for W, the conformal metric's diagonal and the lapse, 0 otherwise;
// v = sqrt(2) for the lapse, 1 otherwise.  Stage 4 also forms y_{n+1}.
__global__ __launch_bounds__(256) void k_z4c_radiative(Z4cRadArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const BoxDev B = a.boxes[i / a.per_member];
  const int64_t o = a.idx[i];
  const int64_t r = o - B.base, pxy = (int64_t)B.px * B.py;
  const int c[3] = {(int)(r % B.px) - B.pad, (int)((r / B.px) % B.py) - B.pad,
                    (int)(r / pxy) - B.pad};
  const int n[3] = {B.nx, B.ny, B.nz};
  const int64_t st[3] = {1, B.px, pxy};
  double x[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) x[d] = a.origin[d] + (double)(B.lo[d] + c[d]) * a.h;
  const double rad = sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
  for (int v = 0; v < NV; ++v) {
    const double* F = a.Y + o + v * a.vstride;
    const double f = F[0];
    double dv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t s = st[d];
      if (c[d] < 0) dv[d] = ((-3.0 * f + 4.0 * F[s]) - F[2 * s]) / (2.0 * a.h);
      else if (c[d] >= n[d]) dv[d] = ((3.0 * f - 4.0 * F[-s]) + F[-2 * s]) / (2.0 * a.h);
      else dv[d] = (F[s] - F[-s]) / (2.0 * a.h);
    }
    const double adv = (x[0] * dv[0] + x[1] * dv[1]) + x[2] * dv[2];
    const bool one = v == VW || v == VG || v == VG + 3 || v == VG + 5 || v == VALP;
    const double f0 = one ? 1.0 : 0.0;
    const double sp = v == VALP ? sqrt(2.0) : 1.0;
    const double k = -(sp / rad) * (adv + (f - f0));
    const int64_t ov = o + v * a.vstride;
    a.kout[ov] = k;
    if (a.stage == 4) {
      const double sm = ((a.k1[ov] + 2.0 * a.k2[ov]) + 2.0 * a.k3[ov]) + k;
      a.ynew[ov] = a.yn[ov] + a.dt6 * sm;
    }
  }
}

}  // namespace

hipError_t launch_z4c_rad_fill(const Z4cRadArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_z4c_rad_fill, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_z4c_radiative(const Z4cRadArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_z4c_radiative, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int ORD>
void z4c_stage_f64(const Z4cArgs& a, dim3 g, dim3 b, dim3 b2, hipStream_t s) {
  // one workgroup per variable and derivative column, in whole rounds of the
  // 8 XCDs (the spare workgroups exit at once)
  const dim3 gd((unsigned)((a.ndtiles * 16 + 7) / 8 * 8));
  hipLaunchKernelGGL((k_z4c_derivs<ORD>), gd, b2, 0, s, a);
  hipLaunchKernelGGL((k_z4c_geom<double, ORD, 1>), g, b, 0, s, a);
  if (!a.ham) {
    hipLaunchKernelGGL((k_z4c_geom<double, ORD, 2>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_z4c_evol<ORD>), g, b, 0, s, a);
    if constexpr (ORD == 8) {
      if (a.ko_r == 8) {
        if (a.stage == 4) hipLaunchKernelGGL((k_z4c_advko<4, double, 8, 5>), g, b2, 0, s, a);
        else hipLaunchKernelGGL((k_z4c_advko<1, double, 8, 5>), g, b2, 0, s, a);
        return;
      }
    }
    if (a.stage == 4) hipLaunchKernelGGL((k_z4c_advko<4, double, ORD>), g, b2, 0, s, a);
    else hipLaunchKernelGGL((k_z4c_advko<1, double, ORD>), g, b2, 0, s, a);
  }
}

hipError_t launch_z4c_stage(const Z4cArgs& a, int grid, bool f32, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 g(grid > 0 ? grid : a.ntiles), b(kZ4cThreads), b2(256);
  if (a.ord != 4 && a.ord != 8) return hipErrorInvalidValue;
  if (a.ko_r != 4 && !(a.ko_r == 8 && a.ord == 8 && !f32)) return hipErrorInvalidValue;
  // FP64 needs the derivative scratch and the derivative columns
  if (!f32 && (!a.der || !a.dtiles || a.ndtiles <= 0)) return hipErrorInvalidValue;
  if (f32) {
    if (a.ord != 4) return hipErrorInvalidValue;   // the FP32 variant is fourth order
    // FP32: the fused kernel fits the register file; FP64: two passes, since
    // one would spill
    hipLaunchKernelGGL((k_z4c_stage<float, true, 4>), g, b, 0, s, a);
    if (a.stage == 4) hipLaunchKernelGGL((k_z4c_advko<4, float, 4>), g, b2, 0, s, a);
    else hipLaunchKernelGGL((k_z4c_advko<1, float, 4>), g, b2, 0, s, a);
  } else if (a.ord == 8) {
    z4c_stage_f64<8>(a, g, b, b2, s);
  } else {
    z4c_stage_f64<4>(a, g, b, b2, s);
  }
  return hipGetLastError();
}

hipError_t launch_z4c_combine(const Z4cCombineArgs& a, int grid, bool f32, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 g(grid > 0 ? grid : a.ntiles), b(256);
  if (f32) hipLaunchKernelGGL(k_z4c_combine<float>, g, b, 0, s, a);
  else hipLaunchKernelGGL(k_z4c_combine<double>, g, b, 0, s, a);
  return hipGetLastError();
}

}  // namespace sc
