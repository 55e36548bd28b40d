/* Reference scalar loops for the wave system (TEST INFRASTRUCTURE ONLY).
 *
 * Plain FP64, one point at a time, built with -O2 -ffp-contract=off so every
 * sum is evaluated in the order written here.  OpenMP splits the
 * z-planes of a block over threads; every point is computed by one thread
 * from inputs no thread writes, so results do not depend on the thread
 * count.
 *
 * Storage: every block holds its owned points plus G ghost layers per side,
 * x fastest; a block descriptor is {base, nx, ny, nz} with base the flat
 * offset of the padded block and n* the owned extents.  Variable v of a
 * level lives at offset v * vstride.
 *
 * Right-hand side (Sec. IV.A and Sec. III.C):
 *   du/dt  = Pi + Q u,     dPi/dt = Laplacian(u) + Q Pi
 * Laplacian: per dimension (-u[-2] + 16u[-1] - 30u[0] + 16u[+1] - u[+2]),
 *   summed x + y + z and multiplied by 1/(12 h^2)   (fourth order, centred).
 * Kreiss-Oliger dissipation with r = 4:
 *   Q u = (-1)^(r/2) sigma / 2^(r+2) * sum_i h^(r+1) D+^3 D-^3 u
 *       = sigma/(64 h) * sum_i (u[-3] - 6u[-2] + 15u[-1] - 20u[0] + 15u[+1] - 6u[+2] + u[+3])
 * Eighth order (the production stencil, Sec. III.C; orc_wave_rhs8): per dimension
 *   (-9u[-4] + 128u[-3] - 1008u[-2] + 8064u[-1] - 14350u[0] + 8064u[+1]
 *    - 1008u[+2] + 128u[+3] - 9u[+4]), summed x + y + z, times 1/(5040 h^2)
 *   (the centred weights -1/560, 8/315, -1/5, 8/5, -205/72 over 5040), with the
 *   same fifth-order (r = 4) dissipation; needs G >= 4.
 * Ninth-order dissipation (r = 8, the option Sec. III.C adds beside the
 * eighth-order derivatives; orc_wave_rhs8_ko9): the same Qu with r = 8,
 *   Q u = sigma/2^10 * sum_i h^9 D+^5 D-^5 u
 *       = sigma/(1024 h) * sum_i (u[-5] - 10u[-4] + 45u[-3] - 120u[-2] + 210u[-1] - 252u[0]
 *                                 + 210u[+1] - 120u[+2] + 45u[+3] - 10u[+4] + u[+5])
 *   (the tenth difference: binomial weights of (D+ D-)^5 h^10); needs G >= 5.
 * RK4 (Eqs. rk1-rk5): Y_{s+1} = y_n + (c_{s+1} dt) k_s with c = 1/2, 1/2, 1;
 *   y_{n+1} = y_n + (dt/6) * (((k1 + 2 k2) + 2 k3) + k4).
 */
#include <stdint.h>

#define P(a, o) ((a)[(o)])

static inline double d2(double m2, double m1, double c, double p1, double p2) {
  return (((-m2 + 16.0 * m1) - 30.0 * c) + 16.0 * p1) - p2;
}

static inline double ko(double m3, double m2, double m1, double c, double p1, double p2,
                        double p3) {
  return (((((m3 - 6.0 * m2) + 15.0 * m1) - 20.0 * c) + 15.0 * p1) - 6.0 * p2) + p3;
}

void orc_wave_rhs(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                  double* k, double h, double sigma) {
  const double clap = 1.0 / (12.0 * h * h);
  const double cko = sigma / (64.0 * h);
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t sx = 1, sy = nx + 2 * G, sz = (int64_t)(nx + 2 * G) * (ny + 2 * G);
    const double* U = Y + base;
    const double* PI = Y + vstride + base;
    double* KU = k + base;
    double* KP = k + vstride + base;
#pragma omp parallel for schedule(static)
    for (int z = G; z < G + nz; ++z)
      for (int y = G; y < G + ny; ++y)
        for (int x = G; x < G + nx; ++x) {
          const int64_t o = z * sz + y * sy + x * sx;
          const double lx = d2(P(U, o - 2 * sx), P(U, o - sx), P(U, o), P(U, o + sx), P(U, o + 2 * sx));
          const double ly = d2(P(U, o - 2 * sy), P(U, o - sy), P(U, o), P(U, o + sy), P(U, o + 2 * sy));
          const double lz = d2(P(U, o - 2 * sz), P(U, o - sz), P(U, o), P(U, o + sz), P(U, o + 2 * sz));
          const double lap = ((lx + ly) + lz) * clap;
          double q[2];
          for (int v = 0; v < 2; ++v) {
            const double* A = v == 0 ? U : PI;
            const double kx = ko(P(A, o - 3 * sx), P(A, o - 2 * sx), P(A, o - sx), P(A, o),
                                 P(A, o + sx), P(A, o + 2 * sx), P(A, o + 3 * sx));
            const double ky = ko(P(A, o - 3 * sy), P(A, o - 2 * sy), P(A, o - sy), P(A, o),
                                 P(A, o + sy), P(A, o + 2 * sy), P(A, o + 3 * sy));
            const double kz = ko(P(A, o - 3 * sz), P(A, o - 2 * sz), P(A, o - sz), P(A, o),
                                 P(A, o + sz), P(A, o + 2 * sz), P(A, o + 3 * sz));
            q[v] = cko * ((kx + ky) + kz);
          }
          KU[o] = P(PI, o) + q[0];
          KP[o] = lap + q[1];
        }
  }
}

static inline double d8(double m4, double m3, double m2, double m1, double c, double p1,
                        double p2, double p3, double p4) {
  return (((((((-9.0 * m4 + 128.0 * m3) - 1008.0 * m2) + 8064.0 * m1) - 14350.0 * c) +
            8064.0 * p1) - 1008.0 * p2) + 128.0 * p3) - 9.0 * p4;
}

static inline double ko11(const double* A, int64_t o, int64_t s) {
  return (((((((((P(A, o - 5 * s) - 10.0 * P(A, o - 4 * s)) + 45.0 * P(A, o - 3 * s)) -
               120.0 * P(A, o - 2 * s)) + 210.0 * P(A, o - s)) - 252.0 * P(A, o)) +
            210.0 * P(A, o + s)) - 120.0 * P(A, o + 2 * s)) + 45.0 * P(A, o + 3 * s)) -
          10.0 * P(A, o + 4 * s)) + P(A, o + 5 * s);
}

/* Eighth-order Laplacian with the r = 8 dissipation (G >= 5). */
void orc_wave_rhs8_ko9(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                       double* k, double h, double sigma) {
  const double clap = 1.0 / (5040.0 * h * h);
  const double cko = sigma / (1024.0 * h);
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t sx = 1, sy = nx + 2 * G, sz = (int64_t)(nx + 2 * G) * (ny + 2 * G);
    const double* U = Y + base;
    const double* PI = Y + vstride + base;
    double* KU = k + base;
    double* KP = k + vstride + base;
#pragma omp parallel for schedule(static)
    for (int z = G; z < G + nz; ++z)
      for (int y = G; y < G + ny; ++y)
        for (int x = G; x < G + nx; ++x) {
          const int64_t o = z * sz + y * sy + x * sx;
          double l[3];
          const int64_t st[3] = {sx, sy, sz};
          for (int d = 0; d < 3; ++d) {
            const int64_t s = st[d];
            l[d] = d8(P(U, o - 4 * s), P(U, o - 3 * s), P(U, o - 2 * s), P(U, o - s), P(U, o),
                      P(U, o + s), P(U, o + 2 * s), P(U, o + 3 * s), P(U, o + 4 * s));
          }
          const double lap = ((l[0] + l[1]) + l[2]) * clap;
          double q[2];
          for (int v = 0; v < 2; ++v) {
            const double* A = v == 0 ? U : PI;
            q[v] = cko * ((ko11(A, o, sx) + ko11(A, o, sy)) + ko11(A, o, sz));
          }
          KU[o] = P(PI, o) + q[0];
          KP[o] = lap + q[1];
        }
  }
}

void orc_wave_rhs8(int nb, const int64_t* desc, int G, int64_t vstride, const double* Y,
                   double* k, double h, double sigma) {
  const double clap = 1.0 / (5040.0 * h * h);
  const double cko = sigma / (64.0 * h);
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t sx = 1, sy = nx + 2 * G, sz = (int64_t)(nx + 2 * G) * (ny + 2 * G);
    const double* U = Y + base;
    const double* PI = Y + vstride + base;
    double* KU = k + base;
    double* KP = k + vstride + base;
#pragma omp parallel for schedule(static)
    for (int z = G; z < G + nz; ++z)
      for (int y = G; y < G + ny; ++y)
        for (int x = G; x < G + nx; ++x) {
          const int64_t o = z * sz + y * sy + x * sx;
          double l[3];
          const int64_t st[3] = {sx, sy, sz};
          for (int d = 0; d < 3; ++d) {
            const int64_t s = st[d];
            l[d] = d8(P(U, o - 4 * s), P(U, o - 3 * s), P(U, o - 2 * s), P(U, o - s), P(U, o),
                      P(U, o + s), P(U, o + 2 * s), P(U, o + 3 * s), P(U, o + 4 * s));
          }
          const double lap = ((l[0] + l[1]) + l[2]) * clap;
          double q[2];
          for (int v = 0; v < 2; ++v) {
            const double* A = v == 0 ? U : PI;
            const double kx = ko(P(A, o - 3 * sx), P(A, o - 2 * sx), P(A, o - sx), P(A, o),
                                 P(A, o + sx), P(A, o + 2 * sx), P(A, o + 3 * sx));
            const double ky = ko(P(A, o - 3 * sy), P(A, o - 2 * sy), P(A, o - sy), P(A, o),
                                 P(A, o + sy), P(A, o + 2 * sy), P(A, o + 3 * sy));
            const double kz = ko(P(A, o - 3 * sz), P(A, o - 2 * sz), P(A, o - sz), P(A, o),
                                 P(A, o + sz), P(A, o + 2 * sz), P(A, o + 3 * sz));
            q[v] = cko * ((kx + ky) + kz);
          }
          KU[o] = P(PI, o) + q[0];
          KP[o] = lap + q[1];
        }
  }
}

/* Y = y_n + cdt * k on owned points. */
void orc_stage(int nb, const int64_t* desc, int G, int64_t vstride, int nvars,
               const double* yn, const double* k, double* Y, double cdt) {
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t sy = nx + 2 * G, sz = (int64_t)(nx + 2 * G) * (ny + 2 * G);
    for (int v = 0; v < nvars; ++v)
#pragma omp parallel for schedule(static)
      for (int z = G; z < G + nz; ++z)
        for (int y = G; y < G + ny; ++y)
          for (int x = G; x < G + nx; ++x) {
            const int64_t o = v * vstride + base + z * sz + y * sy + x;
            Y[o] = yn[o] + cdt * k[o];
          }
  }
}

/* y = y_n + (dt/6) * (((k1 + 2 k2) + 2 k3) + k4) on owned points. */
void orc_final(int nb, const int64_t* desc, int G, int64_t vstride, int nvars,
               const double* yn, const double* k1, const double* k2, const double* k3,
               const double* k4, double* ynew, double dt) {
  const double dt6 = dt / 6.0;
  for (int b = 0; b < nb; ++b) {
    const int64_t base = desc[4 * b];
    const int nx = (int)desc[4 * b + 1], ny = (int)desc[4 * b + 2], nz = (int)desc[4 * b + 3];
    const int64_t sy = nx + 2 * G, sz = (int64_t)(nx + 2 * G) * (ny + 2 * G);
    for (int v = 0; v < nvars; ++v)
#pragma omp parallel for schedule(static)
      for (int z = G; z < G + nz; ++z)
        for (int y = G; y < G + ny; ++y)
          for (int x = G; x < G + nx; ++x) {
            const int64_t o = v * vstride + base + z * sz + y * sy + x;
            const double s = ((k1[o] + 2.0 * k2[o]) + 2.0 * k3[o]) + k4[o];
            ynew[o] = yn[o] + dt6 * s;
          }
  }
}

/* A[dst[i]] = A[src[i]] for every variable (ghost copy from an owner). */
void orc_copy_points(int64_t n, const int64_t* dst, const int64_t* src, int nvars,
                     int64_t vstride, double* A) {
  for (int v = 0; v < nvars; ++v) {
    double* a = A + v * vstride;
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) a[dst[i]] = a[src[i]];
  }
}

/* Five-vector prolongation to refinement-boundary points, one vector at a time.
 * Point i has parity bits par[i] (bit d set: odd index along d) and its
 * parent stencil points at idx[start[i] .. start[i+1]) in z-major, y, x
 * order (6 points along an odd dimension, 1 along an even one).  Along an
 * odd dimension the degree-5 Lagrange midpoint weights
 * (3, -25, 150, 150, -25, 3)/256 are applied left to right; along an even
 * one the value is copied.  x is interpolated first, then y, then z. */
void orc_prolong(int64_t n, const int64_t* start, const int64_t* par, const int64_t* idx,
                 int nvars, int64_t vstride, const double* V, double* out) {
  static const double w[6] = {3.0 / 256.0, -25.0 / 256.0, 150.0 / 256.0,
                              150.0 / 256.0, -25.0 / 256.0, 3.0 / 256.0};
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const int ox = (int)(par[i] & 1), oy = (int)((par[i] >> 1) & 1), oz = (int)((par[i] >> 2) & 1);
    const int nx = ox ? 6 : 1, ny = oy ? 6 : 1, nz = oz ? 6 : 1;
    const int64_t* ix = idx + start[i];
    for (int v = 0; v < nvars; ++v) {
      const double* a = V + v * vstride;
      double pz = 0.0;
      for (int jz = 0; jz < nz; ++jz) {
        double py = 0.0;
        for (int jy = 0; jy < ny; ++jy) {
          const int64_t* row = ix + (jz * ny + jy) * nx;
          double px;
          if (ox) {
            px = w[0] * a[row[0]];
            for (int jx = 1; jx < 6; ++jx) px = px + w[jx] * a[row[jx]];
          } else {
            px = a[row[0]];
          }
          if (oy) py = (jy == 0) ? w[0] * px : py + w[jy] * px;
          else py = px;
        }
        if (oz) pz = (jz == 0) ? w[0] * py : pz + w[jz] * py;
        else pz = py;
      }
      out[v * n + i] = pz;
    }
  }
}
