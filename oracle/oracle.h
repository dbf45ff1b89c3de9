/*
 * CPU FP64 oracle for the barycentric Lagrange treecode (Wang, Krasny and
 * Tlupova, "A kernel-independent treecode based on barycentric Lagrange
 * interpolation", arXiv:1902.02250).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the tests, the smoke check and the CPU
 * baseline of the benchmark use it.  It shares no code with the HIP path.
 *
 * Everything here is plain, slow and written to be checked against the
 * paper by eye:
 *   kernels.c   - the MRS functions H1, H2, Q, D1, D2 (eq. MRS_kernels) and
 *                 the Stokeslet / rotlet / polynomial pair interactions
 *                 (eqs. Velocity_1, MRS_2)
 *   direct.c    - the O(N^2) direct sum (eq. N-body), plain and Neumaier-
 *                 compensated
 *   tree.c      - the cluster tree of Section 6 and the target batches
 *   bary.c      - Chebyshev points of the 2nd kind, the simple barycentric
 *                 weights, the barycentric and product forms of L_k, and
 *                 the modified weights of Algorithm 1
 *   treecode.c  - Algorithm 2 (per-target MAC, or the shared batch MAC),
 *                 interaction-list export and interaction counts
 *   dual.c      - the cluster-cluster variant (interpolation in the target
 *                 variable too), named as future work in Section 9
 * All arithmetic is FP64; the library is compiled with -ffp-contract=off so
 * that no multiply-add is fused behind the reader's back.
 */
#ifndef BLTC_ORACLE_H
#define BLTC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_STOKESLET = 0, ORC_ROTLET = 1, ORC_FULL = 2, ORC_POLY = 100 };

/* ---- kernels.c ---------------------------------------------------------- */
/* H1, H2, Q, D1, D2 at squared distance r2 (eq. MRS_kernels). */
void orc_mrs_functions(double r2, double eps, double out5[5]);
/* Weight and output dimension of a kernel: Stokeslet 3->3, rotlet 3->6
 * (u then w), polynomial test kernel 3->3 (scalar kernel per component).
 * Returns 0, or -1 for an unknown kernel. */
int orc_kernel_dims(int kernel, int* wdim, int* odim);
/* out[0:odim] += k(x, y) f, with x the target and y the source. */
void orc_pair(int kernel, double eps, int poly_p, double poly_c,
              const double x[3], const double y[3], const double* f,
              double* out);

/* ---- direct.c ----------------------------------------------------------- */
/* out[c*m + i] = sum_j k(x_i, y_j) f_j[c]  (eq. N-body), for all m targets.
 * w is [wdim][n] (component-major).  compensated = 1 uses Neumaier sums. */
int orc_direct(int kernel, double eps, int poly_p, double poly_c,
               const double* tx, const double* ty, const double* tz, int64_t m,
               const double* sx, const double* sy, const double* sz, int64_t n,
               const double* w, int compensated, double* out);
/* Same sum for the targets idx[0:k] only; out is [odim][k]. */
int orc_direct_subset(int kernel, double eps, int poly_p, double poly_c,
                      const double* tx, const double* ty, const double* tz,
                      const int64_t* idx, int64_t k,
                      const double* sx, const double* sy, const double* sz, int64_t n,
                      const double* w, double* out);

/* ---- tree.c ------------------------------------------------------------- */
typedef struct orc_tree orc_tree;
orc_tree* orc_tree_new(const double* x, const double* y, const double* z,
                       int64_t n, int64_t leaf_max);
void      orc_tree_free(orc_tree* t);
int64_t   orc_tree_nnodes(const orc_tree* t);
int32_t   orc_tree_depth(const orc_tree* t);
int64_t   orc_tree_npoints(const orc_tree* t);
/* Copies out: perm[n] (tree position -> input index), box[nn][6]
 * (lo x, lo y, lo z, hi x, hi y, hi z), center[nn][3], radius[nn],
 * child_first[nn], child_count[nn], pbegin[nn], pend[nn], level[nn],
 * parent[nn].  Any pointer may be NULL. */
void orc_tree_export(const orc_tree* t, int64_t* perm, double* box,
                     double* center, double* radius, int32_t* child_first,
                     int32_t* child_count, int64_t* pbegin, int64_t* pend,
                     int32_t* level, int32_t* parent);

/* Target batches: targets ordered by a tree of leaf size order_leaf; the
 * maximal nodes of that tree holding at most group_max targets ("groups")
 * are cut into consecutive chunks of batch_size.  order_leaf = 0 instead
 * cuts the targets into balanced k-d batches (tree.c).  Returns the number
 * of batches nb; fills tperm[m], bptr[nb+1], bcenter[nb][3], bradius[nb]
 * (pass NULL arrays first to get nb). */
int64_t orc_batches(const double* tx, const double* ty, const double* tz,
                    int64_t m, int64_t batch_size, int64_t order_leaf,
                    int64_t group_max, int64_t* tperm, int64_t* bptr,
                    double* bcenter, double* bradius);

/* ---- bary.c ------------------------------------------------------------- */
/* Chebyshev points of the 2nd kind on [-1,1], descending (eq.
 * Chebyshev_points), and the simple barycentric weights (eq.
 * barycentric_weights). */
void orc_cheb_points(int n, double* t);
void orc_bary_weights(int n, double* w);
/* L_k(t) for k = 0..n on nodes s, barycentric 2nd form with the exact-hit
 * rule (eq. Barycentric-1D, Algorithm 1). */
void orc_lagrange_bary(int n, const double* s, double t, double* L);
/* L_k(t) from the product formula (eq. Lagrange_polynomial). */
void orc_lagrange_product(int n, const double* s, double t, double* L);
/* Cluster grids: grid[node][axis][k] = mapped Chebyshev points. */
void orc_cluster_grids(const orc_tree* t, int n, double* grid);
/* Modified weights of every cluster, fhat[node][c][k1][k2][k3]
 * (eq. modified_weights).  form 0 = Algorithm 1 (barycentric), form 1 =
 * product-form Lagrange polynomials (a brute-force check for tiny cases).
 * x, y, z, w are in input order; w is [wdim][n]. */
int orc_modified_weights(const orc_tree* t, const double* x, const double* y,
                         const double* z, const double* w, int wdim, int n,
                         int form, double* fhat);

/* ---- treecode.c --------------------------------------------------------- */
#define ORC_MAX_DEGREE 16
typedef struct {
  int kernel;          /* ORC_STOKESLET, ORC_ROTLET, ORC_FULL, ORC_POLY */
  double eps;          /* MRS regularisation */
  int poly_p;          /* polynomial kernel degree */
  double poly_c;       /* polynomial kernel constant */
  int degree;          /* interpolation degree n >= 1 */
  double theta;        /* MAC parameter */
  int64_t leaf_max;    /* N0 */
  int mac_mode;        /* 0: per-target MAC r/R <= theta (paper);
                          1: shared batch MAC (r_B + r_C)/R <= theta */
  int64_t batch_size;  /* targets per batch (mode 1) */
  int64_t order_leaf;  /* leaf size of the target ordering tree (mode 1) */
  int64_t group_max;   /* batches never span two groups of this size (mode 1) */
  int deg_min;         /* 0: every accepted cluster uses `degree` (paper);
                          >= 1: separation rule, degrees in [deg_min, degree] */
} orc_params;

/* Separation rule (deg_min >= 1), see treecode.c: thresholds T[d] for
 * d in [deg_min, degree - 1] (others -1), and the degree of an accepted
 * cluster: the smallest such d with (rr*rr)/R2 <= T[d], else `degree`. */
void orc_rule_table(const orc_params* p, double* T);
int orc_rule_degree(const orc_params* p, const double* T, double rr, double R2);

/* Treecode velocities out[odim][m] in input order.  Counts of kernel
 * evaluations (proxy and direct) are returned through the two pointers
 * (either may be NULL).  If sample/ksample are given (ksample > 0), only the
 * targets sample[0:ksample] are evaluated and out is [odim][ksample]. */
int orc_treecode(const orc_params* p,
                 const double* tx, const double* ty, const double* tz, int64_t m,
                 const double* sx, const double* sy, const double* sz, int64_t n,
                 const double* w, const int64_t* sample, int64_t ksample,
                 double* out, int64_t* n_proxy_evals, int64_t* n_direct_evals);

/* Interaction lists of the batch walk (mode 1) as CSR arrays over batches.
 * Call once with NULL arrays to get the sizes, then with arrays. */
typedef struct orc_lists orc_lists;
orc_lists* orc_lists_new(const double* sx, const double* sy, const double* sz,
                         int64_t n, int64_t leaf_max,
                         const double* tx, const double* ty, const double* tz,
                         int64_t m, double theta, int64_t batch_size,
                         int64_t order_leaf, int64_t group_max, int degree,
                         int deg_min);
/* Degree of every proxy-list entry (orc_rule_degree; `degree` if deg_min = 0). */
void orc_lists_export_degrees(const orc_lists* L, int32_t* prox_deg);
void orc_lists_sizes(const orc_lists* L, int64_t* nb, int64_t* nprox,
                     int64_t* ndir);
void orc_lists_export(const orc_lists* L, int64_t* tperm, int64_t* bptr,
                      int64_t* prox_ptr, int32_t* prox_ids, int64_t* dir_ptr,
                      int32_t* dir_ids);
void orc_lists_free(orc_lists* L);

/* ---- dual.c ------------------------------------------------------------- */
/* Cluster-cluster variant (Section 9's next step; rules in dual.c): target
 * tree of leaf size leaf_t, potentials at target-cluster grid points,
 * interpolated down to the targets.  Uses p->kernel, eps, poly_p, poly_c,
 * degree, theta, leaf_max (sources).  out[odim][m] in input order;
 * counts (may be NULL): kernel evaluations of the CC, PC, CP and PP
 * interactions and the downward (target, grid point) terms. */
int orc_dual_treecode(const orc_params* p, int64_t leaf_t,
                      const double* tx, const double* ty, const double* tz, int64_t m,
                      const double* sx, const double* sy, const double* sz, int64_t n,
                      const double* w, double* out, int64_t counts[5]);

/* Relative L2 error of eq. error over all components. */
double orc_rel_l2(const double* ref, const double* approx, int64_t count);

#ifdef __cplusplus
}
#endif
#endif
