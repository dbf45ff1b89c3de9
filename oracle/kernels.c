/*
 * Oracle (test infrastructure only): the regularized Stokes kernels.
 *
 * The five MRS functions are eq. MRS_kernels of Section 7, written exactly as
 * printed there (each carries its 1/(8 pi) factor):
 *   H1 = (2 eps^2 + r^2) / (8 pi (r^2+eps^2)^(3/2))
 *   H2 = 1 / (8 pi (r^2+eps^2)^(3/2))
 *   Q  = (5 eps^2 + 2 r^2) / (8 pi (r^2+eps^2)^(5/2))
 *   D1 = (10 eps^4 - 7 eps^2 r^2 - 2 r^4) / (8 pi (r^2+eps^2)^(7/2))
 *   D2 = (21 eps^2 + 6 r^2) / (8 pi (r^2+eps^2)^(7/2))
 * with r = |x - y|, x the target and y the source.
 *
 * Pair interactions, d = x - y:
 *   Stokeslet (eq. Velocity_1):      u += f H1 + (f.d) d H2
 *   rotlet (torque terms of eq. MRS_2 with zero force):
 *                                   u += 1/2 (n x d) Q
 *                                   w += 1/4 n D1 + 1/4 (n.d) d D2
 *   Stokeslet + rotlet (eq. MRS_2, weights (f, n), outputs (u, w)):
 *                                   u += f H1 + (f.d) d H2 + 1/2 (n x d) Q
 *                                   w += 1/2 (f x d) Q + 1/4 n D1
 *                                        + 1/4 (n.d) d D2
 *   polynomial test kernel:          u_c += (poly_c + x.y)^poly_p f_c
 * When eps = 0 and r = 0 the singular self term is omitted (Section 1: the
 * i = j term is dropped only for a singular kernel).
 */
#include <math.h>
#include "oracle.h"

static const double PI = 3.14159265358979323846;

void orc_mrs_functions(double r2, double eps, double out5[5]) {
  double e2 = eps * eps;
  double e4 = e2 * e2;
  double s = r2 + e2;                       /* r^2 + eps^2 */
  double s32 = s * sqrt(s);                 /* (r^2+eps^2)^(3/2) */
  double s52 = s32 * s;                     /* (r^2+eps^2)^(5/2) */
  double s72 = s52 * s;                     /* (r^2+eps^2)^(7/2) */
  double c = 8.0 * PI;
  out5[0] = (2.0 * e2 + r2) / (c * s32);
  out5[1] = 1.0 / (c * s32);
  out5[2] = (5.0 * e2 + 2.0 * r2) / (c * s52);
  out5[3] = (10.0 * e4 - 7.0 * e2 * r2 - 2.0 * r2 * r2) / (c * s72);
  out5[4] = (21.0 * e2 + 6.0 * r2) / (c * s72);
}

int orc_kernel_dims(int kernel, int* wdim, int* odim) {
  switch (kernel) {
    case ORC_STOKESLET: *wdim = 3; *odim = 3; return 0;
    case ORC_ROTLET:    *wdim = 3; *odim = 6; return 0;
    case ORC_FULL:      *wdim = 6; *odim = 6; return 0;
    case ORC_POLY:      *wdim = 3; *odim = 3; return 0;
    default: return -1;
  }
}

void orc_pair(int kernel, double eps, int poly_p, double poly_c,
              const double x[3], const double y[3], const double* f,
              double* out) {
  if (kernel == ORC_POLY) {
    double dot = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    double base = poly_c + dot;
    double v = 1.0;
    for (int e = 0; e < poly_p; ++e) v *= base;
    out[0] += v * f[0];
    out[1] += v * f[1];
    out[2] += v * f[2];
    return;
  }
  double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (eps == 0.0 && r2 == 0.0) return;   /* singular self term omitted */
  double m[5];
  orc_mrs_functions(r2, eps, m);
  if (kernel == ORC_STOKESLET) {
    double fd = f[0] * d[0] + f[1] * d[1] + f[2] * d[2];
    for (int a = 0; a < 3; ++a) out[a] += f[a] * m[0] + fd * d[a] * m[1];
  } else if (kernel == ORC_FULL) { /* f[0:3] force, f[3:6] torque */
    const double* fo = f;
    const double* to = f + 3;
    double fd = fo[0] * d[0] + fo[1] * d[1] + fo[2] * d[2];
    double nd = to[0] * d[0] + to[1] * d[1] + to[2] * d[2];
    double nxd[3] = {to[1] * d[2] - to[2] * d[1],
                     to[2] * d[0] - to[0] * d[2],
                     to[0] * d[1] - to[1] * d[0]};
    double fxd[3] = {fo[1] * d[2] - fo[2] * d[1],
                     fo[2] * d[0] - fo[0] * d[2],
                     fo[0] * d[1] - fo[1] * d[0]};
    for (int a = 0; a < 3; ++a)
      out[a] += fo[a] * m[0] + fd * d[a] * m[1] + 0.5 * nxd[a] * m[2];
    for (int a = 0; a < 3; ++a)
      out[3 + a] += 0.5 * fxd[a] * m[2] + 0.25 * to[a] * m[3] + 0.25 * nd * d[a] * m[4];
  } else { /* ORC_ROTLET: f holds the torque n */
    double nxd[3] = {f[1] * d[2] - f[2] * d[1],
                     f[2] * d[0] - f[0] * d[2],
                     f[0] * d[1] - f[1] * d[0]};
    double nd = f[0] * d[0] + f[1] * d[1] + f[2] * d[2];
    for (int a = 0; a < 3; ++a) out[a] += 0.5 * nxd[a] * m[2];
    for (int a = 0; a < 3; ++a)
      out[3 + a] += 0.25 * f[a] * m[3] + 0.25 * nd * d[a] * m[4];
  }
}
