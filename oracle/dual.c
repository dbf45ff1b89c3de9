/*
 * Oracle (test infrastructure only): the cluster-cluster variant of the
 * barycentric Lagrange treecode, which Section 9 names as the next step:
 * the kernel is interpolated in the target variable as well as in the
 * source variable.
 *
 * Both point sets get a tree with the Section 6 rules (source leaf size
 * leaf_max, target leaf size leaf_t).  A target cluster A has a Chebyshev
 * grid t_m on its box exactly like a source cluster, and potentials g_A[m]
 * at its grid points.  With P = (n+1)^3 grid points per cluster, the
 * traversal starts at the two roots; for a pair (A, C) with
 * R2 = |c_A - c_C|^2:
 *  - if R2 > 0 and (r_A + r_C)^2 <= theta^2 R2 (the MAC of eq. MAC with the
 *    target cluster's radius added):
 *      |A| > P and |C| > P:  g_A[m] += sum_k K(t_m, s_k) fhat_k        (CC)
 *      |C| > P only:         u(x) += sum_k K(x, s_k) fhat_k, x in A    (PC)
 *      |A| > P only:         g_A[m] += sum_{y in C} K(t_m, y) f_y      (CP)
 *      otherwise:            u(x) += sum_{y in C} K(x, y) f_y, x in A  (PP)
 *    (an approximation is used only on the side where it saves work);
 *  - else if both are leaves: PP;
 *  - else the pair is refined: A's children if C is a leaf, or if A is not a
 *    leaf and r_A >= r_C; otherwise C's children; children in stored order.
 * Finally every target collects the potentials of every cluster that holds
 * it: u(x) += sum_m L_m(x) g_A[m], with L_m(x) = L_k1(x1) L_k2(x2) L_k3(x3)
 * on A's grid, in the barycentric form with the exact-hit rule of
 * Algorithm 1 (the interpolation of eq. pc_approximation_3D applied to the
 * target variable).
 *
 * With the separation rule (p->deg_min >= 1, see treecode.c) the source
 * side of a CC or PC pair uses the degree orc_rule_degree gives the pair's
 * ratio (r_A + r_C)/R; target grids, the size tests and the downward
 * interpolation keep the degree n.
 *
 * Summation order: pairs in traversal order; grid points and proxies with k3
 * fastest; particles in tree order; then the clusters holding a target, in
 * node order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
  int64_t n, nn;
  int64_t* perm;
  double* center;
  double* radius;
  int32_t* first;
  int32_t* count;
  int64_t* pb;
  int64_t* pe;
  double* pts;    /* tree-ordered [3][n] */
  double* grid;   /* [nn][3][n1] */
} side_t;

typedef struct {
  const orc_params* p;
  int n1, wdim, odim;
  int64_t P;
  side_t s, t;
  double* ws;     /* tree-ordered source weights [wdim][n] */
  double T[ORC_MAX_DEGREE + 1];       /* separation-rule thresholds */
  double* sgrid[ORC_MAX_DEGREE + 1];  /* per degree d: source grids [nn_s][3][d+1] */
  double* fhat[ORC_MAX_DEGREE + 1];   /* per degree d: [nn_s][wdim][(d+1)^3] */
  double* g;      /* [nn_t][P][odim] */
  char* has_g;    /* [nn_t] */
  double* u;      /* [nt][odim], target tree order */
  int64_t cnt[5]; /* CC, PC, CP, PP kernel evaluations; downward (x, m) terms */
} dual_ctx;

static int side_init(side_t* s, const double* x, const double* y, const double* z, int64_t n,
                     int64_t leaf, int n1) {
  memset(s, 0, sizeof *s);
  orc_tree* t = orc_tree_new(x, y, z, n, leaf);
  if (!t) return -1;
  int64_t nn = orc_tree_nnodes(t);
  int64_t nn1 = nn > 0 ? nn : 1, n_1 = n > 0 ? n : 1;
  s->n = n;
  s->nn = nn;
  s->perm = malloc(sizeof(int64_t) * n_1);
  s->center = malloc(sizeof(double) * 3 * nn1);
  s->radius = malloc(sizeof(double) * nn1);
  s->first = malloc(sizeof(int32_t) * nn1);
  s->count = malloc(sizeof(int32_t) * nn1);
  s->pb = malloc(sizeof(int64_t) * nn1);
  s->pe = malloc(sizeof(int64_t) * nn1);
  s->pts = malloc(sizeof(double) * 3 * n_1);
  s->grid = malloc(sizeof(double) * 3 * n1 * nn1);
  orc_tree_export(t, s->perm, NULL, s->center, s->radius, s->first, s->count, s->pb, s->pe,
                  NULL, NULL);
  if (nn > 0) orc_cluster_grids(t, n1 - 1, s->grid);
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = s->perm[i];
    s->pts[i] = x[j];
    s->pts[n + i] = y[j];
    s->pts[2 * n + i] = z[j];
  }
  orc_tree_free(t);
  return 0;
}

static void side_free(side_t* s) {
  free(s->perm); free(s->center); free(s->radius); free(s->first); free(s->count);
  free(s->pb); free(s->pe); free(s->pts); free(s->grid);
}

/* grid point m = (k1, k2, k3), k3 fastest, of cluster q */
static void grid_point(const side_t* s, int n1, int64_t q, int64_t m, double out[3]) {
  const double* g = s->grid + q * 3 * n1;
  out[0] = g[m / (n1 * n1)];
  out[1] = g[n1 + (m / n1) % n1];
  out[2] = g[2 * n1 + m % n1];
}

static void source_point(const dual_ctx* c, int64_t j, double y[3], double f[6]) {
  const int64_t n = c->s.n;
  y[0] = c->s.pts[j];
  y[1] = c->s.pts[n + j];
  y[2] = c->s.pts[2 * n + j];
  for (int k = 0; k < c->wdim; ++k) f[k] = c->ws[k * n + j];
}

/* proxy k of source cluster q at degree d */
static void proxy(const dual_ctx* c, int d, int64_t q, int64_t k, double s[3], double f[6]) {
  const int n1 = d + 1;
  const int64_t nk = (int64_t)n1 * n1 * n1;
  const double* g = c->sgrid[d] + q * 3 * n1;
  s[0] = g[k / (n1 * n1)];
  s[1] = g[n1 + (k / n1) % n1];
  s[2] = g[2 * n1 + k % n1];
  for (int a = 0; a < c->wdim; ++a) f[a] = c->fhat[d][(q * c->wdim + a) * nk + k];
}

static void target_point(const dual_ctx* c, int64_t i, double x[3]) {
  const int64_t m = c->t.n;
  x[0] = c->t.pts[i];
  x[1] = c->t.pts[m + i];
  x[2] = c->t.pts[2 * m + i];
}

static void add_pair(const dual_ctx* c, const double* x, const double* y, const double* f,
                     double* acc) {
  orc_pair(c->p->kernel, c->p->eps, c->p->poly_p, c->p->poly_c, x, y, f, acc);
}

static void interact(dual_ctx* c, int64_t A, int64_t C) {
  const side_t* T = &c->t;
  const side_t* S = &c->s;
  const int64_t na = T->pe[A] - T->pb[A], nc = S->pe[C] - S->pb[C];
  const double dx = T->center[3 * A] - S->center[3 * C];
  const double dy = T->center[3 * A + 1] - S->center[3 * C + 1];
  const double dz = T->center[3 * A + 2] - S->center[3 * C + 2];
  const double R2 = dx * dx + dy * dy + dz * dz;
  const double rr = T->radius[A] + S->radius[C];
  const double th = c->p->theta;
  const int mac = R2 > 0.0 && rr * rr <= (th * th) * R2;
  const int leafA = T->count[A] == 0, leafC = S->count[C] == 0;
  /* the source side's degree under the separation rule (n when it is off) */
  const int d = mac ? orc_rule_degree(c->p, c->T, rr, R2) : c->n1 - 1;
  const int64_t Pd = (int64_t)(d + 1) * (d + 1) * (d + 1);
  double x[3], y[3], f[6];
  if (mac && na > c->P && nc > c->P) {                 /* CC */
    for (int64_t m = 0; m < c->P; ++m) {
      grid_point(T, c->n1, A, m, x);
      double* gm = c->g + (A * c->P + m) * c->odim;
      for (int64_t k = 0; k < Pd; ++k) {
        proxy(c, d, C, k, y, f);
        add_pair(c, x, y, f, gm);
      }
    }
    c->has_g[A] = 1;
    c->cnt[0] += c->P * Pd;
  } else if (mac && nc > c->P) {                       /* PC */
    for (int64_t i = T->pb[A]; i < T->pe[A]; ++i) {
      target_point(c, i, x);
      for (int64_t k = 0; k < Pd; ++k) {
        proxy(c, d, C, k, y, f);
        add_pair(c, x, y, f, c->u + i * c->odim);
      }
    }
    c->cnt[1] += na * Pd;
  } else if (mac && na > c->P) {                       /* CP */
    for (int64_t m = 0; m < c->P; ++m) {
      grid_point(T, c->n1, A, m, x);
      double* gm = c->g + (A * c->P + m) * c->odim;
      for (int64_t j = S->pb[C]; j < S->pe[C]; ++j) {
        source_point(c, j, y, f);
        add_pair(c, x, y, f, gm);
      }
    }
    c->has_g[A] = 1;
    c->cnt[2] += c->P * nc;
  } else if (mac || (leafA && leafC)) {                /* PP */
    for (int64_t i = T->pb[A]; i < T->pe[A]; ++i) {
      target_point(c, i, x);
      for (int64_t j = S->pb[C]; j < S->pe[C]; ++j) {
        source_point(c, j, y, f);
        add_pair(c, x, y, f, c->u + i * c->odim);
      }
    }
    c->cnt[3] += na * nc;
  } else if (leafC || (!leafA && T->radius[A] >= S->radius[C])) {
    for (int32_t k = 0; k < T->count[A]; ++k) interact(c, T->first[A] + k, C);
  } else {
    for (int32_t k = 0; k < S->count[C]; ++k) interact(c, A, S->first[C] + k);
  }
}

/* u(x) += sum_m L_m(x) g_A[m] for every target x of every cluster A with
 * potentials. */
static void downward(dual_ctx* c) {
  const int n1 = c->n1;
  double Lx[ORC_MAX_DEGREE + 1], Ly[ORC_MAX_DEGREE + 1], Lz[ORC_MAX_DEGREE + 1];
  for (int64_t A = 0; A < c->t.nn; ++A) {
    if (!c->has_g[A]) continue;
    const double* g = c->t.grid + A * 3 * n1;
    for (int64_t i = c->t.pb[A]; i < c->t.pe[A]; ++i) {
      double x[3];
      target_point(c, i, x);
      orc_lagrange_bary(n1 - 1, g, x[0], Lx);
      orc_lagrange_bary(n1 - 1, g + n1, x[1], Ly);
      orc_lagrange_bary(n1 - 1, g + 2 * n1, x[2], Lz);
      double* ui = c->u + i * c->odim;
      for (int64_t m = 0; m < c->P; ++m) {
        const double L = Lx[m / (n1 * n1)] * Ly[(m / n1) % n1] * Lz[m % n1];
        const double* gm = c->g + (A * c->P + m) * c->odim;
        for (int k = 0; k < c->odim; ++k) ui[k] += L * gm[k];
      }
      c->cnt[4] += c->P;
    }
  }
}

int orc_dual_treecode(const orc_params* p, int64_t leaf_t,
                      const double* tx, const double* ty, const double* tz, int64_t m,
                      const double* sx, const double* sy, const double* sz, int64_t n,
                      const double* w, double* out, int64_t counts[5]) {
  if (p->degree < 1 || p->degree > ORC_MAX_DEGREE || p->leaf_max < 1 || leaf_t < 1) return -1;
  dual_ctx c;
  memset(&c, 0, sizeof c);
  c.p = p;
  c.n1 = p->degree + 1;
  c.P = (int64_t)c.n1 * c.n1 * c.n1;
  if (orc_kernel_dims(p->kernel, &c.wdim, &c.odim)) return -1;
  orc_rule_table(p, c.T);
  int rc = side_init(&c.s, sx, sy, sz, n, p->leaf_max, c.n1);
  if (!rc) rc = side_init(&c.t, tx, ty, tz, m, leaf_t, c.n1);
  if (!rc) {
    int64_t nn_s = c.s.nn > 0 ? c.s.nn : 1, nn_t = c.t.nn > 0 ? c.t.nn : 1;
    int64_t n_1 = n > 0 ? n : 1, m_1 = m > 0 ? m : 1;
    c.ws = malloc(sizeof(double) * c.wdim * n_1);
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < c.wdim; ++k) c.ws[k * n + i] = w[k * n + c.s.perm[i]];
    c.g = calloc((size_t)(nn_t * c.P * c.odim), sizeof(double));
    c.has_g = calloc((size_t)nn_t, 1);
    c.u = calloc((size_t)(m_1 * c.odim), sizeof(double));
    /* source grids and modified weights of every degree the rule can give */
    orc_tree* st = orc_tree_new(sx, sy, sz, n, p->leaf_max);
    const int dlo = p->deg_min >= 1 && p->deg_min < p->degree ? p->deg_min : p->degree;
    for (int d = dlo; d <= p->degree && !rc; ++d) {
      const int64_t n1 = d + 1;
      c.sgrid[d] = calloc((size_t)(nn_s * 3 * n1), sizeof(double));
      c.fhat[d] = calloc((size_t)(nn_s * c.wdim * n1 * n1 * n1), sizeof(double));
      if (n > 0) {
        orc_cluster_grids(st, d, c.sgrid[d]);
        rc = orc_modified_weights(st, sx, sy, sz, w, c.wdim, d, 0, c.fhat[d]);
      }
    }
    orc_tree_free(st);
    if (!rc && n > 0 && m > 0) {
      interact(&c, 0, 0);
      downward(&c);
    }
    for (int64_t i = 0; !rc && i < m; ++i)
      for (int k = 0; k < c.odim; ++k) out[k * m + c.t.perm[i]] = c.u[i * c.odim + k];
    if (counts) memcpy(counts, c.cnt, sizeof c.cnt);
  }
  free(c.ws); free(c.g); free(c.has_g); free(c.u);
  for (int d = 0; d <= ORC_MAX_DEGREE; ++d) { free(c.sgrid[d]); free(c.fhat[d]); }
  side_free(&c.s);
  side_free(&c.t);
  return rc;
}
