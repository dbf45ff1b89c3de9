/*
 * Oracle (test infrastructure only): barycentric Lagrange interpolation and
 * the modified weights.
 *
 * Section 3: Chebyshev points of the 2nd kind s_k = cos(k pi / n), k = 0..n
 * (eq. Chebyshev_points); they are computed here as sin(pi (n - 2k) / (2n)),
 * the same numbers written so that the middle point is exactly 0 and the set
 * is exactly symmetric in floating point.  The simple weights are
 * w_k = (-1)^k delta_k with delta = 1/2 at both ends (eq.
 * barycentric_weights); by scale invariance they serve on any interval
 * [a, b] with the mapped points (a+b)/2 + t (b-a)/2.
 *
 * L_k(t) in the 2nd barycentric form (eq. Barycentric-1D): if t is within
 * DBL_MIN of some s_j the value is the Kronecker delta, otherwise
 * (w_k/(t - s_k)) / sum_j (w_j/(t - s_j)).
 *
 * Modified weights (eq. modified_weights):
 *   fhat_k = sum_{y_j in C} L_k1(y_j1) L_k2(y_j2) L_k3(y_j3) f_j,
 * computed for each cluster by the steps of Algorithm 1: per particle the
 * terms a(k, l) = w_k / (y_l - s_k) and their sums, the exact-hit flags,
 * denom = sum(1) sum(2) sum(3), then the tensor-product accumulation.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static const double PI = 3.14159265358979323846;

void orc_cheb_points(int n, double* t) {
  for (int k = 0; k <= n; ++k) t[k] = sin(PI * (double)(n - 2 * k) / (2.0 * n));
}

void orc_bary_weights(int n, double* w) {
  for (int k = 0; k <= n; ++k) {
    double delta = (k == 0 || k == n) ? 0.5 : 1.0;
    w[k] = (k % 2 == 0) ? delta : -delta;
  }
}

void orc_lagrange_bary(int n, const double* s, double t, double* L) {
  double w[64];
  orc_bary_weights(n, w);
  int flag = -1;
  double sum = 0.0;
  for (int k = 0; k <= n; ++k) {
    double diff = t - s[k];
    if (fabs(diff) <= DBL_MIN) {
      flag = k;
    } else {
      L[k] = w[k] / diff;
      sum += L[k];
    }
  }
  if (flag > -1) {
    for (int k = 0; k <= n; ++k) L[k] = 0.0;
    L[flag] = 1.0;
    return;
  }
  for (int k = 0; k <= n; ++k) L[k] = L[k] / sum;
}

void orc_lagrange_product(int n, const double* s, double t, double* L) {
  for (int k = 0; k <= n; ++k) {
    double num = 1.0, den = 1.0;
    for (int j = 0; j <= n; ++j) {
      if (j == k) continue;
      num *= t - s[j];
      den *= s[k] - s[j];
    }
    L[k] = num / den;
  }
}

void orc_cluster_grids(const orc_tree* t, int n, double* grid) {
  int64_t nn = orc_tree_nnodes(t);
  double* box = malloc(sizeof(double) * 6 * (nn > 0 ? nn : 1));
  orc_tree_export(t, NULL, box, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
  double tk[64];
  orc_cheb_points(n, tk);
  for (int64_t q = 0; q < nn; ++q)
    for (int a = 0; a < 3; ++a) {
      double lo = box[6 * q + a], hi = box[6 * q + 3 + a];
      double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
      for (int k = 0; k <= n; ++k) grid[(q * 3 + a) * (n + 1) + k] = c + h * tk[k];
    }
  free(box);
}

int orc_modified_weights(const orc_tree* t, const double* x, const double* y,
                         const double* z, const double* w, int wdim, int n,
                         int form, double* fhat) {
  if (n < 1 || n > 60) return -1;
  int64_t nn = orc_tree_nnodes(t);
  int64_t np = orc_tree_npoints(t);
  int64_t* perm = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
  int64_t* pb = malloc(sizeof(int64_t) * (nn > 0 ? nn : 1));
  int64_t* pe = malloc(sizeof(int64_t) * (nn > 0 ? nn : 1));
  orc_tree_export(t, perm, NULL, NULL, NULL, NULL, NULL, pb, pe, NULL, NULL);
  double* grid = malloc(sizeof(double) * 3 * (n + 1) * (nn > 0 ? nn : 1));
  orc_cluster_grids(t, n, grid);
  double wk[64];
  orc_bary_weights(n, wk);
  const int n1 = n + 1;
  const int64_t nk = (int64_t)n1 * n1 * n1;
  const double* xyz[3] = {x, y, z};

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nn; ++q) {
    double* fq = fhat + q * wdim * nk;
    const double* s = grid + q * 3 * n1;     /* s[a * n1 + k] */
    for (int64_t i = 0; i < wdim * nk; ++i) fq[i] = 0.0;   /* Alg. 1: init */
    double a[3][64];
    for (int64_t p = pb[q]; p < pe[q]; ++p) {             /* loop over j */
      int64_t j = perm[p];
      double denom;
      if (form == 0) {
        int flag[3] = {-1, -1, -1};
        double sum[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k <= n; ++k)
          for (int l = 0; l < 3; ++l) {
            double diff = xyz[l][j] - s[l * n1 + k];
            if (fabs(diff) <= DBL_MIN) {
              flag[l] = k;
            } else {
              a[l][k] = wk[k] / diff;
              sum[l] += a[l][k];
            }
          }
        for (int l = 0; l < 3; ++l)
          if (flag[l] > -1) {
            sum[l] = 1.0;
            for (int k = 0; k <= n; ++k) a[l][k] = 0.0;
            a[l][flag[l]] = 1.0;
          }
        denom = sum[0] * sum[1] * sum[2];
      } else {
        for (int l = 0; l < 3; ++l)
          orc_lagrange_product(n, s + l * n1, xyz[l][j], a[l]);
        denom = 1.0;
      }
      for (int k1 = 0; k1 <= n; ++k1)
        for (int k2 = 0; k2 <= n; ++k2)
          for (int k3 = 0; k3 <= n; ++k3) {
            double basis = a[0][k1] * a[1][k2] * a[2][k3] / denom;
            int64_t kk = ((int64_t)k1 * n1 + k2) * n1 + k3;
            for (int c = 0; c < wdim; ++c)
              fq[c * nk + kk] += basis * w[(int64_t)c * np + j];
          }
    }
  }
  free(perm); free(pb); free(pe); free(grid);
  return 0;
}
