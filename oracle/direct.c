/*
 * Oracle (test infrastructure only): the direct sum of eq. N-body,
 *   u(x_i) = sum_j k(x_i, y_j) f_j,
 * with targets x_i that need not be the sources (Section 8 notes that
 * coinciding targets and sources is not essential).  Sources are visited in
 * input order.  OpenMP splits the targets, the paper's own parallel axis.
 *
 * The compensated variant keeps a Neumaier (improved Kahan) running sum per
 * output component; the pair term is still computed in plain FP64.
 */
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

static void direct_one(int kernel, double eps, int poly_p, double poly_c,
                       const double x[3], const double* sx, const double* sy,
                       const double* sz, int64_t n, const double* w,
                       int compensated, double* acc, int wdim, int odim) {
  double sum[6] = {0}, comp[6] = {0};
  for (int64_t j = 0; j < n; ++j) {
    double y[3] = {sx[j], sy[j], sz[j]};
    double f[6];
    for (int k = 0; k < wdim; ++k) f[k] = w[k * n + j];
    double term[6] = {0};
    orc_pair(kernel, eps, poly_p, poly_c, x, y, f, term);
    for (int c = 0; c < odim; ++c) {
      if (!compensated) {
        sum[c] += term[c];
      } else {
        double t = sum[c] + term[c];
        if (fabs(sum[c]) >= fabs(term[c]))
          comp[c] += (sum[c] - t) + term[c];
        else
          comp[c] += (term[c] - t) + sum[c];
        sum[c] = t;
      }
    }
  }
  for (int c = 0; c < odim; ++c) acc[c] = sum[c] + comp[c];
}

int orc_direct(int kernel, double eps, int poly_p, double poly_c,
               const double* tx, const double* ty, const double* tz, int64_t m,
               const double* sx, const double* sy, const double* sz, int64_t n,
               const double* w, int compensated, double* out) {
  int wdim, odim;
  if (orc_kernel_dims(kernel, &wdim, &odim)) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < m; ++i) {
    double x[3] = {tx[i], ty[i], tz[i]};
    double acc[6];
    direct_one(kernel, eps, poly_p, poly_c, x, sx, sy, sz, n, w, compensated,
               acc, wdim, odim);
    for (int c = 0; c < odim; ++c) out[c * m + i] = acc[c];
  }
  return 0;
}

int orc_direct_subset(int kernel, double eps, int poly_p, double poly_c,
                      const double* tx, const double* ty, const double* tz,
                      const int64_t* idx, int64_t k,
                      const double* sx, const double* sy, const double* sz, int64_t n,
                      const double* w, double* out) {
  int wdim, odim;
  if (orc_kernel_dims(kernel, &wdim, &odim)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < k; ++q) {
    int64_t i = idx[q];
    double x[3] = {tx[i], ty[i], tz[i]};
    double acc[6];
    direct_one(kernel, eps, poly_p, poly_c, x, sx, sy, sz, n, w, 0, acc, wdim, odim);
    for (int c = 0; c < odim; ++c) out[c * k + q] = acc[c];
  }
  return 0;
}

double orc_rel_l2(const double* ref, const double* approx, int64_t count) {
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    double e = ref[i] - approx[i];
    num += e * e;
    den += ref[i] * ref[i];
  }
  return den > 0.0 ? sqrt(num / den) : sqrt(num);
}
