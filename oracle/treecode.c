/*
 * Oracle (test infrastructure only): the treecode of Algorithm 2.
 *
 * For each target x the walk starts at the root; for a cluster C:
 *   - if the MAC holds, add the far-field approximation
 *       sum_k k(x, s_k) fhat_k            (eq. pc_approximation_3D),
 *   - else, if C is a leaf, add the direct sum over its particles
 *       sum_{y_j in C} k(x, y_j) f_j       (eq. pc_interaction_3D),
 *   - else visit the children in order.
 * The MAC is r/R <= theta (eq. MAC), tested in squared form as
 *   R2 > 0  and  r*r <= (theta*theta)*R2,  R2 = dx*dx + dy*dy + dz*dz,
 * so a cluster whose center coincides with the target is never approximated.
 *
 * mac_mode 1 replaces x by a batch of targets sharing one walk (batches as
 * built by orc_batches): the batch's
 * center c_B and radius r_B stand in for x, and the test becomes
 *   R2 > 0  and  (r_B + r)*(r_B + r) <= (theta*theta)*R2.
 * Since |x - y_c| >= R - r_B for every x in the batch, an accepted cluster
 * also satisfies the per-target MAC for theta <= 1; with one target per
 * batch (r_B = 0) the two modes agree bit for bit.
 *
 * Separation rule (deg_min >= 1; not in the paper, which uses one degree):
 * Chebyshev interpolation of a function analytic inside the Bernstein
 * ellipse of parameter 1/kappa converges like kappa^n; for the kernel seen
 * from a cluster at ratio rho = r/R the singularity at the target gives
 * kappa(rho) = rho / (1 + sqrt(1 - rho^2)).  An accepted cluster at ratio
 * rho = (r_B + r_C)/R is interpolated with the smallest degree
 * d in [deg_min, degree] with kappa(rho)^(d+1) <= kappa(theta)^(degree+1):
 * no cluster exceeds the error scale of the worst accepted cluster of the
 * fixed-degree walk (rho = theta, degree), and well-separated clusters use
 * fewer grid points.  Equivalently rho^2 <= T[d] with the thresholds
 *   T[d] = (2k / (1 + k^2))^2,  k = kappa(theta)^((degree+1)/(d+1)),
 * so the per-cluster decision needs only the MAC's rr and R2.
 *
 * Summation order: clusters in depth-first order with children in their
 * stored order, grid points with k3 fastest, leaf particles in tree order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
  int64_t nn, n;
  int64_t* perm;
  double* center;
  double* radius;
  int32_t* child_first;
  int32_t* child_count;
  int64_t* pbegin;
  int64_t* pend;
  double* ys;      /* tree-ordered sources [3][n] */
  double* ws;      /* tree-ordered weights [wdim][n] */
  double T[ORC_MAX_DEGREE + 1];       /* separation-rule thresholds */
  double* grid[ORC_MAX_DEGREE + 1];   /* per degree d: [nn][3][d+1] */
  double* fhat[ORC_MAX_DEGREE + 1];   /* per degree d: [nn][wdim][(d+1)^3] */
  int wdim, odim;
  const orc_params* p;
} walk_ctx;

void orc_rule_table(const orc_params* p, double* T) {
  for (int d = 0; d <= ORC_MAX_DEGREE; ++d) T[d] = -1.0;
  if (p->deg_min < 1 || p->deg_min >= p->degree) return;
  const double kt = p->theta / (1.0 + sqrt(1.0 - p->theta * p->theta));
  for (int d = p->deg_min; d < p->degree; ++d) {
    const double k = pow(kt, (double)(p->degree + 1) / (double)(d + 1));
    const double r = (2.0 * k) / (1.0 + k * k);
    T[d] = r * r;
  }
}

int orc_rule_degree(const orc_params* p, const double* T, double rr, double R2) {
  if (p->deg_min < 1 || p->deg_min >= p->degree) return p->degree;
  const double q = (rr * rr) / R2;
  for (int d = p->deg_min; d < p->degree; ++d)
    if (q <= T[d]) return d;
  return p->degree;
}

/* 0 if the MAC fails, else 1 + the degree the cluster is interpolated with. */
static int mac_holds(const walk_ctx* c, const double xc[3], double rB,
                     int64_t q) {
  double dx = xc[0] - c->center[3 * q + 0];
  double dy = xc[1] - c->center[3 * q + 1];
  double dz = xc[2] - c->center[3 * q + 2];
  double R2 = dx * dx + dy * dy + dz * dz;
  if (!(R2 > 0.0)) return 0;
  double rr = rB + c->radius[q];
  if (!(rr * rr <= (c->p->theta * c->p->theta) * R2)) return 0;
  return 1 + orc_rule_degree(c->p, c->T, rr, R2);
}

static void compute_velocity(const walk_ctx* c, const double x[3],
                             const double xc[3], double rB, int64_t q,
                             double* acc, int64_t* np, int64_t* nd) {
  const orc_params* p = c->p;
  const int acc_deg = mac_holds(c, xc, rB, q);
  if (acc_deg) {
    const int n1 = acc_deg;   /* degree + 1 */
    const int64_t nk = (int64_t)n1 * n1 * n1;
    const double* g = c->grid[n1 - 1] + q * 3 * n1;
    const double* fq = c->fhat[n1 - 1] + q * c->wdim * nk;
    for (int k1 = 0; k1 < n1; ++k1)
      for (int k2 = 0; k2 < n1; ++k2)
        for (int k3 = 0; k3 < n1; ++k3) {
          int64_t kk = ((int64_t)k1 * n1 + k2) * n1 + k3;
          double s[3] = {g[k1], g[n1 + k2], g[2 * n1 + k3]};
          double f[6];
          for (int k = 0; k < c->wdim; ++k) f[k] = fq[k * nk + kk];
          orc_pair(p->kernel, p->eps, p->poly_p, p->poly_c, x, s, f, acc);
        }
    *np += nk;
  } else if (c->child_count[q] == 0) {
    for (int64_t j = c->pbegin[q]; j < c->pend[q]; ++j) {
      double y[3] = {c->ys[j], c->ys[c->n + j], c->ys[2 * c->n + j]};
      double f[6];
      for (int k = 0; k < c->wdim; ++k) f[k] = c->ws[k * c->n + j];
      orc_pair(p->kernel, p->eps, p->poly_p, p->poly_c, x, y, f, acc);
    }
    *nd += c->pend[q] - c->pbegin[q];
  } else {
    for (int32_t ch = 0; ch < c->child_count[q]; ++ch)
      compute_velocity(c, x, xc, rB, c->child_first[q] + ch, acc, np, nd);
  }
}

static void ctx_free(walk_ctx* c) {
  free(c->perm); free(c->center); free(c->radius); free(c->child_first);
  free(c->child_count); free(c->pbegin); free(c->pend); free(c->ys);
  free(c->ws);
  for (int d = 0; d <= ORC_MAX_DEGREE; ++d) { free(c->grid[d]); free(c->fhat[d]); }
}

/* Tree export plus tree-ordered copies of the sources; with degree >= 1 also
 * the grids and the modified weights. */
static int ctx_init(walk_ctx* c, const orc_params* p, const double* sx,
                    const double* sy, const double* sz, int64_t n,
                    const double* w) {
  memset(c, 0, sizeof *c);
  c->p = p;
  orc_rule_table(p, c->T);
  if (orc_kernel_dims(p->kernel, &c->wdim, &c->odim)) return -1;
  orc_tree* t = orc_tree_new(sx, sy, sz, n, p->leaf_max);
  int64_t nn = orc_tree_nnodes(t);
  int64_t nn1 = nn > 0 ? nn : 1, n_1 = n > 0 ? n : 1;
  c->nn = nn;
  c->n = n;
  c->perm = malloc(sizeof(int64_t) * n_1);
  c->center = malloc(sizeof(double) * 3 * nn1);
  c->radius = malloc(sizeof(double) * nn1);
  c->child_first = malloc(sizeof(int32_t) * nn1);
  c->child_count = malloc(sizeof(int32_t) * nn1);
  c->pbegin = malloc(sizeof(int64_t) * nn1);
  c->pend = malloc(sizeof(int64_t) * nn1);
  orc_tree_export(t, c->perm, NULL, c->center, c->radius, c->child_first,
                  c->child_count, c->pbegin, c->pend, NULL, NULL);
  c->ys = malloc(sizeof(double) * 3 * n_1);
  c->ws = malloc(sizeof(double) * c->wdim * n_1);
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = c->perm[i];
    c->ys[i] = sx[j];
    c->ys[n + i] = sy[j];
    c->ys[2 * n + i] = sz[j];
    for (int k = 0; k < c->wdim; ++k) c->ws[k * n + i] = w[k * n + j];
  }
  int rc = 0;
  const int dlo = p->deg_min >= 1 && p->deg_min < p->degree ? p->deg_min : p->degree;
  for (int d = dlo; d <= p->degree && rc == 0; ++d) {
    const int64_t n1 = d + 1;
    c->grid[d] = malloc(sizeof(double) * 3 * n1 * nn1);
    c->fhat[d] = malloc(sizeof(double) * c->wdim * n1 * n1 * n1 * nn1);
    orc_cluster_grids(t, d, c->grid[d]);
    rc = orc_modified_weights(t, sx, sy, sz, w, c->wdim, d, 0, c->fhat[d]);
  }
  orc_tree_free(t);
  return rc;
}

int orc_treecode(const orc_params* p,
                 const double* tx, const double* ty, const double* tz, int64_t m,
                 const double* sx, const double* sy, const double* sz, int64_t n,
                 const double* w, const int64_t* sample, int64_t ksample,
                 double* out, int64_t* n_proxy_evals, int64_t* n_direct_evals) {
  if (p->degree < 1 || p->degree > ORC_MAX_DEGREE || p->leaf_max < 1 || p->deg_min < 0)
    return -1;
  walk_ctx c;
  if (ctx_init(&c, p, sx, sy, sz, n, w)) { ctx_free(&c); return -1; }
  int64_t nout = ksample > 0 ? ksample : m;

  /* batch geometry for every target (mode 1) */
  double* bc = NULL;
  double* br = NULL;
  int64_t* tbatch = NULL;
  if (p->mac_mode == 1 && m > 0) {
    int64_t nbmax = orc_batches(tx, ty, tz, m, p->batch_size, p->order_leaf,
                                p->group_max, NULL, NULL, NULL, NULL);
    int64_t* tperm = malloc(sizeof(int64_t) * m);
    int64_t* bptr = malloc(sizeof(int64_t) * (nbmax + 1));
    bc = malloc(sizeof(double) * 3 * nbmax);
    br = malloc(sizeof(double) * nbmax);
    tbatch = malloc(sizeof(int64_t) * m);
    int64_t nb = orc_batches(tx, ty, tz, m, p->batch_size, p->order_leaf,
                             p->group_max, tperm, bptr, bc, br);
    for (int64_t b = 0; b < nb; ++b)
      for (int64_t i = bptr[b]; i < bptr[b + 1]; ++i) tbatch[tperm[i]] = b;
    free(tperm);
    free(bptr);
  }

  int64_t tot_p = 0, tot_d = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : tot_p, tot_d)
  for (int64_t q = 0; q < nout; ++q) {
    int64_t i = ksample > 0 ? sample[q] : q;
    double x[3] = {tx[i], ty[i], tz[i]};
    double acc[6] = {0};
    int64_t np = 0, nd = 0;
    if (n > 0) {
      if (p->mac_mode == 1) {
        int64_t b = tbatch[i];
        compute_velocity(&c, x, bc + 3 * b, br[b], 0, acc, &np, &nd);
      } else {
        compute_velocity(&c, x, x, 0.0, 0, acc, &np, &nd);
      }
    }
    for (int k = 0; k < c.odim; ++k) out[k * nout + q] = acc[k];
    tot_p += np;
    tot_d += nd;
  }
  if (n_proxy_evals) *n_proxy_evals = tot_p;
  if (n_direct_evals) *n_direct_evals = tot_d;
  free(bc); free(br); free(tbatch);
  ctx_free(&c);
  return 0;
}

/* ---- interaction lists of the batch walk -------------------------------- */
struct orc_lists {
  int64_t nb, m;
  int64_t* tperm;
  int64_t* bptr;
  int64_t* prox_ptr;
  int64_t* dir_ptr;
  int32_t* prox;
  int32_t* pdeg;
  int32_t* dir;
  int64_t nprox, ndir;
};

typedef struct { int32_t* v; int64_t n, cap; } ivec;
static void ipush(ivec* a, int32_t x) {
  if (a->n == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 256;
    a->v = realloc(a->v, sizeof(int32_t) * a->cap);
  }
  a->v[a->n++] = x;
}

static void list_walk(const walk_ctx* c, const double xc[3], double rB,
                      int64_t q, ivec* prox, ivec* pdeg, ivec* dir) {
  const int acc_deg = mac_holds(c, xc, rB, q);
  if (acc_deg) {
    ipush(prox, (int32_t)q);
    ipush(pdeg, acc_deg - 1);
  } else if (c->child_count[q] == 0) {
    ipush(dir, (int32_t)q);
  } else {
    for (int32_t ch = 0; ch < c->child_count[q]; ++ch)
      list_walk(c, xc, rB, c->child_first[q] + ch, prox, pdeg, dir);
  }
}

orc_lists* orc_lists_new(const double* sx, const double* sy, const double* sz,
                         int64_t n, int64_t leaf_max,
                         const double* tx, const double* ty, const double* tz,
                         int64_t m, double theta, int64_t batch_size,
                         int64_t order_leaf, int64_t group_max, int degree,
                         int deg_min) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.kernel = ORC_STOKESLET;
  p.degree = degree >= 1 ? degree : 1;
  p.deg_min = deg_min;
  p.theta = theta;
  p.leaf_max = leaf_max;
  p.mac_mode = 1;
  /* The walk needs only the tree: build it directly, without weights. */
  walk_ctx c;
  memset(&c, 0, sizeof c);
  c.p = &p;
  orc_rule_table(&p, c.T);
  orc_tree* t = orc_tree_new(sx, sy, sz, n, leaf_max);
  int64_t nn = orc_tree_nnodes(t), nn1 = nn > 0 ? nn : 1;
  c.nn = nn;
  c.center = malloc(sizeof(double) * 3 * nn1);
  c.radius = malloc(sizeof(double) * nn1);
  c.child_first = malloc(sizeof(int32_t) * nn1);
  c.child_count = malloc(sizeof(int32_t) * nn1);
  orc_tree_export(t, NULL, NULL, c.center, c.radius, c.child_first,
                  c.child_count, NULL, NULL, NULL, NULL);
  orc_tree_free(t);

  orc_lists* L = calloc(1, sizeof(orc_lists));
  int64_t nbmax = orc_batches(tx, ty, tz, m, batch_size, order_leaf, group_max,
                              NULL, NULL, NULL, NULL);
  L->m = m;
  L->tperm = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
  L->bptr = malloc(sizeof(int64_t) * (nbmax + 1));
  double* bc = malloc(sizeof(double) * 3 * (nbmax > 0 ? nbmax : 1));
  double* br = malloc(sizeof(double) * (nbmax > 0 ? nbmax : 1));
  L->nb = orc_batches(tx, ty, tz, m, batch_size, order_leaf, group_max,
                      L->tperm, L->bptr, bc, br);
  L->prox_ptr = malloc(sizeof(int64_t) * (L->nb + 1));
  L->dir_ptr = malloc(sizeof(int64_t) * (L->nb + 1));
  ivec prox = {0}, pdeg = {0}, dir = {0};
  for (int64_t b = 0; b < L->nb; ++b) {
    L->prox_ptr[b] = prox.n;
    L->dir_ptr[b] = dir.n;
    if (nn > 0) list_walk(&c, bc + 3 * b, br[b], 0, &prox, &pdeg, &dir);
  }
  L->prox_ptr[L->nb] = prox.n;
  L->dir_ptr[L->nb] = dir.n;
  L->prox = prox.v;
  L->pdeg = pdeg.v;
  L->dir = dir.v;
  L->nprox = prox.n;
  L->ndir = dir.n;
  free(bc); free(br);
  free(c.center); free(c.radius); free(c.child_first); free(c.child_count);
  return L;
}

void orc_lists_sizes(const orc_lists* L, int64_t* nb, int64_t* nprox,
                     int64_t* ndir) {
  *nb = L->nb;
  *nprox = L->nprox;
  *ndir = L->ndir;
}

void orc_lists_export(const orc_lists* L, int64_t* tperm, int64_t* bptr,
                      int64_t* prox_ptr, int32_t* prox_ids, int64_t* dir_ptr,
                      int32_t* dir_ids) {
  if (tperm) memcpy(tperm, L->tperm, sizeof(int64_t) * L->m);
  if (bptr) memcpy(bptr, L->bptr, sizeof(int64_t) * (L->nb + 1));
  if (prox_ptr) memcpy(prox_ptr, L->prox_ptr, sizeof(int64_t) * (L->nb + 1));
  if (dir_ptr) memcpy(dir_ptr, L->dir_ptr, sizeof(int64_t) * (L->nb + 1));
  if (prox_ids && L->nprox) memcpy(prox_ids, L->prox, sizeof(int32_t) * L->nprox);
  if (dir_ids && L->ndir) memcpy(dir_ids, L->dir, sizeof(int32_t) * L->ndir);
}

void orc_lists_export_degrees(const orc_lists* L, int32_t* prox_deg) {
  if (prox_deg && L->nprox) memcpy(prox_deg, L->pdeg, sizeof(int32_t) * L->nprox);
}

void orc_lists_free(orc_lists* L) {
  if (!L) return;
  free(L->tperm); free(L->bptr); free(L->prox_ptr); free(L->dir_ptr);
  free(L->prox); free(L->pdeg); free(L->dir);
  free(L);
}
