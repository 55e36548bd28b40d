/* Reference Z4c right-hand side (TEST INFRASTRUCTURE ONLY).
 *
 * Sec. III.A: evolution of W, conformal metric gt_ij, Khat, At_ij, Theta,
 * Gt^i with the Ricci split R_ij = R^W_ij + Rt_ij, the puncture gauge
 * (1+log lapse  d_t alpha = beta.d alpha - 2 alpha Khat,  Gamma-driver shift
 * d_t beta^i = beta.d beta^i + 3/4 Gt^i - eta(r) beta^i,
 * eta(r) = (eta_c - eta_o) exp(-(r/eta_s)^4) + eta_o), vacuum, and r = 4
 * Kreiss-Oliger dissipation (Sec. III.C) on all 22 variables.  Standard
 * conformal relations the equations use without printing them:
 *   Gt_kij = (d_i gt_jk + d_j gt_ik - d_k gt_ij)/2,  Gt^k_ij = gtu^kl Gt_lij,
 *   Gd^i = gtu^jk Gt^i_jk,
 *   physical Christoffels G^k_ij = Gt^k_ij - (delta^k_i d_j W + delta^k_j d_i W
 *                                  - gt_ij gtu^kl d_l W)/W,
 *   D_i D_j alpha = d_i d_j alpha - G^k_ij d_k alpha,  D^i D_i = W^2 gtu^ij D_i D_j,
 *   Dt_i Dt_j W = d_i d_j W - Gt^k_ij d_k W,  R = W^2 gtu^ij R_ij,
 *   [X]^TF_ij = X_ij - gt_ij gtu^kl X_kl / 3,  indices raised with gtu.
 * Derivatives: fourth-order centred D1, D2, and D1_x(D1_y) for mixed second
 * derivatives; advection beta^k d_k uses the centred D1.  With order 8 (the
 * paper's production stencil, Sec. III.C; G >= 4) the same with the
 * eighth-order centred weights: D1 = (3, -32, 168, -672, 0, 672, -168, 32, -3)
 * / (840 h), D2 = (-9, 128, -1008, 8064, -14350, 8064, -1008, 128, -9)
 * / (5040 h^2); the dissipation stays the r = 4 operator, or (Sec. III.C's
 * ninth-order option, G >= 5) is the r = 8 operator
 *   Q u = sigma / (1024 h) sum_d delta_d^10 u,
 *   delta^10 = (1, -10, 45, -120, 210, -252, 210, -120, 45, -10, 1).
 * Variables (slot order): W, gt_xx,xy,xz,yy,yz,zz, Khat, At_xx..zz, Theta,
 * Gt^x,y,z, alpha, beta^x,y,z.
 * Storage as in stencil.c: padded blocks {base, nx, ny, nz}, variable v at
 * offset v * vstride.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

enum { VW = 0, VG = 1, VKH = 7, VA = 8, VTH = 14, VGAM = 15, VALP = 18, VB = 19, NV = 22 };

static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static int ORDER = 4;   /* set per call of the right-hand side */
static int KORD = 4;    /* dissipation operator r: 4, or 8 */

static double D1(const double* a, int64_t o, int64_t s, double c1) {
  if (ORDER == 8)
    return (((((((3.0 * a[o - 4 * s] - 32.0 * a[o - 3 * s]) + 168.0 * a[o - 2 * s]) -
                672.0 * a[o - s]) + 672.0 * a[o + s]) - 168.0 * a[o + 2 * s]) +
             32.0 * a[o + 3 * s]) - 3.0 * a[o + 4 * s]) * c1;
  return (((a[o - 2 * s] - 8.0 * a[o - s]) + 8.0 * a[o + s]) - a[o + 2 * s]) * c1;
}

static double D2(const double* a, int64_t o, int64_t s, double c2) {
  if (ORDER == 8)
    return ((((((((-9.0 * a[o - 4 * s] + 128.0 * a[o - 3 * s]) - 1008.0 * a[o - 2 * s]) +
                 8064.0 * a[o - s]) - 14350.0 * a[o]) + 8064.0 * a[o + s]) -
              1008.0 * a[o + 2 * s]) + 128.0 * a[o + 3 * s]) - 9.0 * a[o + 4 * s]) * c2;
  return ((((-a[o - 2 * s] + 16.0 * a[o - s]) - 30.0 * a[o]) + 16.0 * a[o + s]) - a[o + 2 * s]) *
         c2;
}

static double DM(const double* a, int64_t o, int64_t s, int64_t t, double c1) {
  /* D1 along s of D1 along t */
  if (ORDER == 8)
    return (((((((3.0 * D1(a, o - 4 * s, t, c1) - 32.0 * D1(a, o - 3 * s, t, c1)) +
                 168.0 * D1(a, o - 2 * s, t, c1)) - 672.0 * D1(a, o - s, t, c1)) +
               672.0 * D1(a, o + s, t, c1)) - 168.0 * D1(a, o + 2 * s, t, c1)) +
             32.0 * D1(a, o + 3 * s, t, c1)) - 3.0 * D1(a, o + 4 * s, t, c1)) * c1;
  return (((D1(a, o - 2 * s, t, c1) - 8.0 * D1(a, o - s, t, c1)) + 8.0 * D1(a, o + s, t, c1)) -
          D1(a, o + 2 * s, t, c1)) *
         c1;
}

static double KO(const double* a, int64_t o, int64_t s) {
  if (KORD == 8)
    return (((((((((a[o - 5 * s] - 10.0 * a[o - 4 * s]) + 45.0 * a[o - 3 * s]) -
                  120.0 * a[o - 2 * s]) + 210.0 * a[o - s]) - 252.0 * a[o]) +
               210.0 * a[o + s]) - 120.0 * a[o + 2 * s]) + 45.0 * a[o + 3 * s]) -
             10.0 * a[o + 4 * s]) + a[o + 5 * s];
  return (((((a[o - 3 * s] - 6.0 * a[o - 2 * s]) + 15.0 * a[o - s]) - 20.0 * a[o]) +
           15.0 * a[o + s]) - 6.0 * a[o + 2 * s]) + a[o + 3 * s];
}

/* par: kappa1, kappa2, eta_c, eta_o, eta_s, sigma */
static void z4c_point(const double* Y, int64_t o, int64_t vs, const int64_t st[3], double h,
                      const double* par, const double xyz[3], double* rhs, double* ricci,
                      double* ham) {
  const double c1 = ORDER == 8 ? 1.0 / (840.0 * h) : 1.0 / (12.0 * h);
  const double c2 = ORDER == 8 ? 1.0 / (5040.0 * h * h) : 1.0 / (12.0 * h * h);
  const double kappa1 = par[0], kappa2 = par[1], eta_c = par[2], eta_o = par[3],
               eta_s = par[4], sigma = par[5];
  double v[NV], d[NV][3];
  for (int i = 0; i < NV; ++i) {
    v[i] = Y[i * vs + o];
    for (int k = 0; k < 3; ++k) d[i][k] = D1(Y + i * vs, o, st[k], c1);
  }
  /* second derivatives of W, gt_ij, alpha, beta^i */
  static const int need2[11] = {VW, VG, VG + 1, VG + 2, VG + 3, VG + 4, VG + 5, VALP, VB, VB + 1, VB + 2};
  double dd[NV][3][3];
  memset(dd, 0, sizeof dd);
  for (int n = 0; n < 11; ++n) {
    const int i = need2[n];
    for (int k = 0; k < 3; ++k)
      for (int l = k; l < 3; ++l) {
        const double x = (k == l) ? D2(Y + i * vs, o, st[k], c2) : DM(Y + i * vs, o, st[k], st[l], c1);
        dd[i][k][l] = x;
        dd[i][l][k] = x;
      }
  }
  const double W = v[VW], Kh = v[VKH], Th = v[VTH], alp = v[VALP];
  double gt[3][3], At[3][3], Gt[3], beta[3], dW[3], da[3], dKh[3], dTh[3];
  double dgt[3][3][3], ddgt[3][3][3][3], dAt[3][3][3], dGt[3][3], db[3][3], ddb[3][3][3];
  double ddW[3][3], dda[3][3];
  for (int i = 0; i < 3; ++i) {
    Gt[i] = v[VGAM + i];
    beta[i] = v[VB + i];
    dW[i] = d[VW][i];
    da[i] = d[VALP][i];
    dKh[i] = d[VKH][i];
    dTh[i] = d[VTH][i];
    for (int j = 0; j < 3; ++j) {
      gt[i][j] = v[VG + SYM[i][j]];
      At[i][j] = v[VA + SYM[i][j]];
      dGt[i][j] = d[VGAM + j][i];    /* d_i Gt^j */
      db[i][j] = d[VB + j][i];       /* d_i beta^j */
      ddW[i][j] = dd[VW][i][j];
      dda[i][j] = dd[VALP][i][j];
      for (int k = 0; k < 3; ++k) {
        dgt[k][i][j] = d[VG + SYM[i][j]][k];    /* d_k gt_ij */
        dAt[k][i][j] = d[VA + SYM[i][j]][k];
        ddb[i][j][k] = dd[VB + k][i][j];         /* d_i d_j beta^k */
        for (int l = 0; l < 3; ++l) ddgt[k][l][i][j] = dd[VG + SYM[i][j]][k][l];
      }
    }
  }
  (void)dAt;
  /* inverse conformal metric */
  const double det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                     gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                     gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  double gu[3][3];
  gu[0][0] = (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) / det;
  gu[0][1] = (gt[0][2] * gt[2][1] - gt[0][1] * gt[2][2]) / det;
  gu[0][2] = (gt[0][1] * gt[1][2] - gt[0][2] * gt[1][1]) / det;
  gu[1][0] = gu[0][1];
  gu[1][1] = (gt[0][0] * gt[2][2] - gt[0][2] * gt[2][0]) / det;
  gu[1][2] = (gt[0][2] * gt[1][0] - gt[0][0] * gt[1][2]) / det;
  gu[2][0] = gu[0][2];
  gu[2][1] = gu[1][2];
  gu[2][2] = (gt[0][0] * gt[1][1] - gt[0][1] * gt[1][0]) / det;
  /* Christoffels of gt */
  double Gl[3][3][3], G[3][3][3], Gd[3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Gl[k][i][j] = 0.5 * ((dgt[i][j][k] + dgt[j][i][k]) - dgt[k][i][j]);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += gu[k][l] * Gl[l][i][j];
        G[k][i][j] = s;
      }
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s += gu[j][k] * G[i][j][k];
    Gd[i] = s;
  }
  /* Ricci tensor R_ij = R^W_ij + Rt_ij */
  double DDW[3][3], lapW = 0.0, dWsq = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = ddW[i][j];
      for (int k = 0; k < 3; ++k) s -= G[k][i][j] * dW[k];
      DDW[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      lapW += gu[i][j] * DDW[i][j];
      dWsq += gu[i][j] * dW[i] * dW[j];
    }
  dWsq /= W * W;
  double R[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double rt = 0.0;
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) rt -= 0.5 * gu[l][m] * ddgt[l][m][i][j];
      for (int k = 0; k < 3; ++k) {
        rt += 0.5 * (gt[k][i] * dGt[j][k] + gt[k][j] * dGt[i][k]);
        rt += Gd[k] * 0.5 * (Gl[i][j][k] + Gl[j][i][k]);
      }
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) {
          double s = 0.0;
          for (int k = 0; k < 3; ++k)
            s += (G[k][l][i] * Gl[j][k][m] + G[k][l][j] * Gl[i][k][m]) + G[k][i][m] * Gl[k][l][j];
          rt += gu[l][m] * s;
        }
      const double rw = DDW[i][j] / W + gt[i][j] * lapW / W - 2.0 * gt[i][j] * dWsq;
      R[i][j] = rw + rt;
    }
  double Rs = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Rs += gu[i][j] * R[i][j];
  Rs *= W * W;
  /* lapse second covariant derivatives with the physical Christoffels */
  double gudW[3];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int l = 0; l < 3; ++l) s += gu[k][l] * dW[l];
    gudW[k] = s;
  }
  double DDa[3][3], lapa = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = dda[i][j];
      for (int k = 0; k < 3; ++k) {
        const double Gp = G[k][i][j] - (((k == i ? dW[j] : 0.0) + (k == j ? dW[i] : 0.0)) -
                                         gt[i][j] * gudW[k]) / W;
        s -= Gp * da[k];
      }
      DDa[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) lapa += gu[i][j] * DDa[i][j];
  lapa *= W * W;
  /* raised At */
  double Atu[3][3], Atm[3][3], AtA = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0, m = 0.0;
      for (int k = 0; k < 3; ++k) {
        m += gu[i][k] * At[k][j];
        for (int l = 0; l < 3; ++l) s += gu[i][k] * gu[j][l] * At[k][l];
      }
      Atu[i][j] = s;
      Atm[i][j] = m; /* At^i_j */
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AtA += At[i][j] * Atu[i][j];
  double divb = 0.0;
  for (int k = 0; k < 3; ++k) divb += db[k][k];
  const double Kt = Kh + 2.0 * Th;
  double adv[NV];
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += beta[k] * d[i][k];
    adv[i] = s;
  }
  /* W */
  rhs[VW] = adv[VW] + (1.0 / 3.0) * W * (alp * Kt - divb);
  /* gt_ij and At_ij */
  double X[3][3], trX = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) X[i][j] = -DDa[i][j] + alp * R[i][j];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) trX += gu[k][l] * X[k][l];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      double lg = 0.0, la = 0.0, aa = 0.0;
      for (int k = 0; k < 3; ++k) {
        lg += gt[k][i] * db[j][k] + gt[k][j] * db[i][k];
        la += At[k][i] * db[j][k] + At[k][j] * db[i][k];
        aa += Atm[k][i] * At[k][j];
      }
      const int s = SYM[i][j];
      rhs[VG + s] = adv[VG + s] - 2.0 * alp * At[i][j] + lg - (2.0 / 3.0) * gt[i][j] * divb;
      const double tf = X[i][j] - (1.0 / 3.0) * gt[i][j] * trX;
      rhs[VA + s] = adv[VA + s] + W * W * tf + alp * (Kt * At[i][j] - 2.0 * aa) + la -
                    (2.0 / 3.0) * At[i][j] * divb;
    }
  /* Khat */
  rhs[VKH] = adv[VKH] - lapa + alp * (AtA + (1.0 / 3.0) * Kt * Kt) +
             alp * kappa1 * (1.0 - kappa2) * Th;
  /* Gt^i */
  for (int i = 0; i < 3; ++i) {
    double t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0, t5 = 0.0, t6 = 0.0, t7 = 0.0;
    for (int j = 0; j < 3; ++j) {
      t1 += Atu[i][j] * da[j];
      t3 += Atu[i][j] * dW[j] / W;
      t4 += gu[i][j] * (2.0 * dKh[j] + dTh[j]);
      t7 += Gd[j] * db[j][i];
      for (int k = 0; k < 3; ++k) {
        t2 += G[i][j][k] * Atu[j][k];
        t5 += gu[j][k] * ddb[j][k][i];
        t6 += gu[i][j] * ddb[j][k][k];
      }
    }
    rhs[VGAM + i] = adv[VGAM + i] - 2.0 * t1 + 2.0 * alp * (t2 - 3.0 * t3 - (1.0 / 3.0) * t4) + t5 +
                    (1.0 / 3.0) * t6 - t7 + (2.0 / 3.0) * Gd[i] * divb -
                    2.0 * alp * kappa1 * (Gt[i] - Gd[i]);
  }
  /* Theta */
  rhs[VTH] = adv[VTH] + 0.5 * alp * (Rs - AtA + (2.0 / 3.0) * Kt * Kt) -
             alp * kappa1 * (2.0 + kappa2) * Th;
  /* gauge */
  rhs[VALP] = adv[VALP] - 2.0 * alp * Kh;
  const double r = sqrt(xyz[0] * xyz[0] + xyz[1] * xyz[1] + xyz[2] * xyz[2]);
  const double rq = r / eta_s;
  const double eta = (eta_c - eta_o) * exp(-(rq * rq) * (rq * rq)) + eta_o;
  for (int i = 0; i < 3; ++i) rhs[VB + i] = adv[VB + i] + 0.75 * Gt[i] - eta * beta[i];
  /* Kreiss-Oliger dissipation on every variable */
  const double cko = sigma / ((KORD == 8 ? 1024.0 : 64.0) * h);
  for (int i = 0; i < NV; ++i) {
    const double* a = Y + i * vs;
    rhs[i] += cko * ((KO(a, o, st[0]) + KO(a, o, st[1])) + KO(a, o, st[2]));
  }
  if (ricci)
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) ricci[SYM[i][j]] = R[i][j];
  if (ham) *ham = Rs + (2.0 / 3.0) * Kt * Kt - AtA;
}

/* k = Z4c RHS of Y on owned points.  origin[3*b..] = coordinates of block b's
 * owned point (0,0,0).  ricci (6 slots) and ham (1 slot) are optional outputs
 * in the same padded layout. */
static void z4c_rhs(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                    double* k, double h, const double* par, const double* origin, double* ricci,
                    double* ham) {
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t st[3] = {1, nx + 2 * G, (int64_t)(nx + 2 * G) * (ny + 2 * G)};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t o = base + (z + G) * st[2] + (y + G) * st[1] + (x + G);
          const double xyz[3] = {origin[3 * b] + x * h, origin[3 * b + 1] + y * h,
                                 origin[3 * b + 2] + z * h};
          double r[NV], ric[6], hm;
          z4c_point(Y, o, vstride, st, h, par, xyz, r, ric, &hm);
          for (int i = 0; i < NV; ++i) k[i * vstride + o] = r[i];
          if (ricci)
            for (int i = 0; i < 6; ++i) ricci[i * vstride + o] = ric[i];
          if (ham) ham[o] = hm;
        }
  }
}

void orc_z4c_rhs(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y, double* k,
                 double h, const double* par, const double* origin, double* ricci, double* ham) {
  ORDER = 4;
  KORD = 4;
  z4c_rhs(nb, desc, G, vstride, Y, k, h, par, origin, ricci, ham);
}

/* The same with the eighth-order derivatives (G >= 4). */
void orc_z4c_rhs8(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                  double* k, double h, const double* par, const double* origin, double* ricci,
                  double* ham) {
  ORDER = 8;
  KORD = 4;
  z4c_rhs(nb, desc, G, vstride, Y, k, h, par, origin, ricci, ham);
}

/* Eighth-order derivatives with the r = 8 dissipation (G >= 5). */
void orc_z4c_rhs8_ko9(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                      double* k, double h, const double* par, const double* origin,
                      double* ricci, double* ham) {
  ORDER = 8;
  KORD = 8;
  z4c_rhs(nb, desc, G, vstride, Y, k, h, par, origin, ricci, ham);
}
