/*
 * bltc.h - C ABI of the MI355X (gfx950) barycentric Lagrange treecode
 * (Wang, Krasny and Tlupova, arXiv:1902.02250): the evaluation phase for the
 * 3D regularized Stokeslet and rotlet kernels (each alone, or both together).
 *
 * What is computed (eq. N-body): for targets x_i and sources y_j with vector
 * weights f_j,
 *     u(x_i) = sum_j k(x_i, y_j) f_j,
 * approximated by the treecode of Algorithm 2: a cluster tree over the
 * sources (Section 6), modified weights on each cluster's tensor-product grid
 * of Chebyshev points of the 2nd kind (eq. modified_weights, Algorithm 1),
 * and a walk under the MAC r/R <= theta (eq. MAC) that uses the far-field
 * approximation (eq. pc_approximation_3D) for accepted clusters and the
 * direct sum (eq. pc_interaction_3D) at leaves.  Targets are grouped into
 * batches of spatially close targets that share one walk (the shared MAC
 * (r_B + r_C)/R <= theta, which implies the paper's per-target MAC for every
 * target of the batch); batch_size = 1 is exactly the per-target walk.
 *
 * Kernels (Section 7, eq. MRS_kernels):
 *   BLTC_STOKESLET  f (3) -> u (3):  u = sum f H1 + (f.d) d H2  (eq. Velocity_1)
 *   BLTC_ROTLET     n (3) -> (u, w) (6): the torque terms of eq. MRS_2,
 *                   u = sum 1/2 (n x d) Q,  w = sum 1/4 n D1 + 1/4 (n.d) d D2
 *   BLTC_FULL       (f, n) (6) -> (u, w) (6): both parts of eq. MRS_2,
 *                   u = sum f H1 + (f.d) d H2 + 1/2 (n x d) Q,
 *                   w = sum 1/2 (f x d) Q + 1/4 n D1 + 1/4 (n.d) d D2
 *                   (weights: force rows then torque rows)
 *   BLTC_POLY       f (3) -> u (3): u_c = sum (poly_c + x.y)^poly_p f_c, a
 *                   polynomial test kernel; FP64 only
 * with d = x - y and the regularisation eps.  When eps = 0 a pair at zero
 * distance contributes nothing (the singular self term is dropped,
 * Section 1); when eps > 0 it is included.  Outputs are for unit viscosity.
 *
 * Conventions for every entry point:
 *   - Point, weight and output arrays are HIP DEVICE pointers unless the
 *     name or comment says "host".  Points are three separate FP64 arrays
 *     (x, y, z).  Weights are FP64 [wdim][n], component-major (wdim = 3,
 *     or 6 for BLTC_FULL); outputs are FP64 [odim][m], component-major, in
 *     the caller's target order (odim = 3, or 6 for the rotlet and
 *     BLTC_FULL: u rows then w rows).
 *   - The caller owns every buffer it passes; the library owns its handles
 *     and the device memory inside them, freed by the matching destroy call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is queued
 *     on it; calls that must read results back to the host synchronise on it
 *     and say so.
 *   - Every call returns a bltc_status.  Arguments are checked before any
 *     device work is queued; on an error nothing is written to the outputs.
 *     bltc_last_error() returns a thread-local message for the last failure.
 *   - Handles are not thread safe; different handles may be used from
 *     different threads.
 *   - Sizes: n, m < 2^31; degree 1..12; leaf_max >= 1; batch_size 1..1024;
 *     order_leaf >= 0 (0: balanced k-d batches); group_max >= 1;
 *     0 <= theta <= 1; eps >= 0.  n = 0 or m = 0 is a valid no-op.
 */
#ifndef BLTC_H
#define BLTC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BLTC_OK = 0,
  BLTC_EINVAL = 1,   /* an argument is out of range or a pointer is NULL */
  BLTC_ENOMEM = 2,   /* a device or host allocation failed */
  BLTC_EDEVICE = 3,  /* a HIP call failed (message from the runtime) */
  BLTC_ESTATE = 4,   /* the handle lacks a prerequisite (e.g. no weights) */
  BLTC_EMODEL = 5    /* a selector model file is missing or malformed */
} bltc_status;

enum { BLTC_STOKESLET = 0, BLTC_ROTLET = 1, BLTC_FULL = 2, BLTC_POLY = 100 };

enum {
  BLTC_FP64 = 0,          /* FP64 everywhere */
  BLTC_FP32_FP64ACC = 1,  /* FP32 kernel evaluation, FP64 per-target sums */
  BLTC_FP32_KAHAN = 2     /* FP32 kernel evaluation, compensated FP32 sums */
};

/* Options of an evaluation; bltc_options_default() fills the defaults. */
typedef struct {
  int32_t size;        /* sizeof(bltc_options) */
  int32_t precision;   /* BLTC_FP64 (default) or a mixed mode */
  int32_t batch_size;  /* targets sharing one walk, default 64 */
  int32_t order_leaf;  /* leaf size of the tree that orders the targets; 0
                          (default): balanced k-d batches (bltc_build_targets) */
  int32_t poly_p;      /* BLTC_POLY exponent, default 2 */
  double poly_c;       /* BLTC_POLY constant, default 1 */
  int64_t group_max;   /* batches never span two target groups, default 512 */
  int32_t deg_min;     /* 0 (default): every accepted cluster is interpolated
                          at the evaluation's degree n, as in the paper.
                          1 <= deg_min < n: separation rule (not in the
                          paper): an accepted cluster at ratio
                          rho = (r_B + r_C)/R takes the smallest degree d in
                          [deg_min, n] with kappa(rho)^(d+1) <=
                          kappa(theta)^(n+1), kappa(r) = r/(1 + sqrt(1 - r^2))
                          (Chebyshev interpolation converges like kappa^d for
                          a singularity at ratio r); tested as
                          rho^2 <= (2k/(1+k^2))^2, k = kappa(theta)^((n+1)/(d+1)).
                          The evaluation derives the weights of each lower
                          degree the lists use from the degree-n weights
                          (degree-n interpolation reproduces the degree-d
                          Lagrange basis, so this equals the sum over the
                          particles up to rounding); they are cached until
                          the weights change. */
} bltc_options;

typedef struct bltc_tree_s* bltc_tree;       /* sources: tree, weights */
typedef struct bltc_targets_s* bltc_targets; /* targets: order, batches */
typedef struct bltc_selector_s* bltc_selector; /* per-batch (n, theta) model */

void bltc_options_default(bltc_options* opt);
const char* bltc_last_error(void);
const char* bltc_version(void);

/* ---- sources ------------------------------------------------------------
 * Builds the cluster tree of Section 6 over the n sources (x, y, z) with at
 * most leaf_max particles per leaf (N0).  Every cluster's box is the tight
 * box of its particles; a cluster with more than leaf_max particles is
 * bisected at its box midpoint along every side longer than l_max/sqrt(2)
 * (l_max its own longest side), giving 8, 4 or 2 children in the order of
 * the code bx + 2 by + 4 bz; empty children are dropped; a cluster
 * with l_max = 0 or whose bisection would separate nothing stays a leaf.
 * Center = box midpoint, radius = half the box diagonal.  The tree is built
 * on the device one level at a time (per-chunk min/max, split tests, code
 * histograms, a stable scatter); the host numbers the children from one
 * read-back per level and keeps a copy of the node arrays (synchronises on
 * `stream`).  Tree-ordered coordinates and the node arrays stay on the
 * device. */
int bltc_build_tree(const double* x, const double* y, const double* z,
                    int64_t n, int64_t leaf_max, void* stream, bltc_tree* out);
int bltc_tree_destroy(bltc_tree t);
/* Node count and depth (host values). */
int bltc_tree_info(bltc_tree t, int64_t* n_nodes, int32_t* depth);
/* Host copies of the tree (synchronises): perm[n] (tree position -> input
 * index), box[nn][6] (lo xyz, hi xyz), center[nn][3], radius[nn],
 * child_first[nn], child_count[nn], pbegin[nn], pend[nn], level[nn].  Any
 * pointer may be NULL. */
int bltc_tree_export(bltc_tree t, int64_t* perm, double* box, double* center,
                     double* radius, int32_t* child_first, int32_t* child_count,
                     int64_t* pbegin, int64_t* pend, int32_t* level);

/* Upward pass (eq. modified_weights, Algorithm 1): gathers the weights w
 * (FP64 [wdim][n], caller order; wdim 3, or 6 for BLTC_FULL) into tree
 * order and computes, for every
 * cluster, its Chebyshev grid (degree+1 points per axis mapped to the box)
 * and modified weights fhat_k = sum_{j in C} L_k1(y_j1) L_k2(y_j2) L_k3(y_j3) f_j,
 * the Lagrange values taken in barycentric form with the exact-hit rule of
 * Algorithm 1 (a coordinate equal to a grid point gets the Kronecker delta).
 * The leaves sum over their particles; every parent takes its children's
 * weights through the degree-n Lagrange basis of its own grid evaluated at
 * the children's grid points, which equals the sum over its particles in
 * exact arithmetic (degree-n interpolation reproduces the parent's basis).
 * Computed in FP64; kept in FP64 and FP32 for the evaluation.  Calling again
 * replaces the weights and drops modified weights of other degrees (their
 * device buffers are kept for reuse). */
int bltc_compute_modified_weights(bltc_tree t, const double* w, int32_t wdim,
                                  int32_t degree, void* stream);
/* Host copy of the modified weights of one degree (synchronises):
 * fhat[nn][wdim][degree+1][degree+1][degree+1] (k3 fastest) and, if grid is
 * not NULL, grid[nn][3][degree+1]. */
int bltc_modified_weights_export(bltc_tree t, int32_t degree, double* fhat,
                                 double* grid);

/* ---- targets -------------------------------------------------------------
 * Groups the m targets into batches of at most batch_size that share one
 * walk (the batch MAC).  Two rules:
 *  - order_leaf = 0, balanced k-d batches: a set of c > batch_size targets is
 *    cut along the longest side of its tight box (the first of equal sides),
 *    the first part taking the batch_size floor(nb / 2) targets with the
 *    smallest coordinates on that axis, nb = ceil(c / batch_size), ties
 *    ordered by target index; sets of at most batch_size targets are the
 *    batches, in cut order (first part first), their targets in increasing
 *    index.  Every batch is full except the last, and the boxes stay
 *    compact.  group_max is not used.
 *  - order_leaf >= 1: the targets are ordered by a tree built with the same
 *    rules as the sources and leaf size order_leaf; the maximal nodes of that
 *    tree with at most group_max targets (and any larger degenerate leaf) are
 *    the groups, each cut into consecutive batches of batch_size targets, so
 *    a batch never spans two groups and its radius is bounded by its group's.
 * Each batch gets its tight box, center and radius like a cluster.  The k-d
 * cut runs on the device (the part sizes, which depend on m and batch_size
 * only, are laid out on the host); the order tree is built on the device as
 * in bltc_build_tree, the group and batch bounds on the host from its node
 * arrays; the batch boxes on the device (synchronises).  The order and
 * batches live on the device; a host copy of the order is kept for
 * bltc_targets_export. */
int bltc_build_targets(const double* x, const double* y, const double* z,
                       int64_t m, int32_t batch_size, int32_t order_leaf,
                       int64_t group_max, void* stream, bltc_targets* out);
int bltc_targets_destroy(bltc_targets g);
/* Host copies (synchronises): number of batches, tperm[m] (target position
 * -> input index), bptr[nb+1], bcenter[nb][3], bradius[nb]. */
int bltc_targets_export(bltc_targets g, int64_t* nb, int64_t* tperm,
                        int64_t* bptr, double* bcenter, double* bradius);

/* ---- host-only builders --------------------------------------------------
 * The same tree and batches built from HOST arrays, with no device work, so
 * the construction rules can be checked on any machine.  Call with NULL
 * output arrays to get n_nodes (or nb) first.  Arrays as in
 * bltc_tree_export / bltc_targets_export. */
int bltc_host_tree(const double* hx, const double* hy, const double* hz,
                   int64_t n, int64_t leaf_max, int64_t* n_nodes,
                   int32_t* depth, int64_t* perm, double* box, double* center,
                   double* radius, int32_t* child_first, int32_t* child_count,
                   int64_t* pbegin, int64_t* pend, int32_t* level);
int bltc_host_batches(const double* hx, const double* hy, const double* hz,
                      int64_t m, int32_t batch_size, int32_t order_leaf,
                      int64_t group_max, int64_t* nb, int64_t* tperm,
                      int64_t* bptr, double* bcenter, double* bradius);

/* ---- evaluation ----------------------------------------------------------
 * Walks the tree for every batch under the MAC with parameter theta (device
 * interaction lists), then evaluates the far field against the Chebyshev
 * grid points and modified weights of `degree` and the near field against
 * leaf particles, and writes out[odim][m] in caller order.  The modified
 * weights of `degree` must have been computed with the kernel's wdim (else
 * BLTC_ESTATE).  The list sizes are read back once, and the per-batch list
 * counts once more to order the launch (batches by decreasing modelled work,
 * dealt to the XCDs; the order changes no result): synchronises on
 * `stream`. */
int bltc_evaluate_tree(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt,
                       double* out, void* stream);

/* Allocation-free bltc_evaluate_tree, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks and result as
 * bltc_evaluate_tree, bit for bit; the interaction lists, the walk flags,
 * the separation rule's degree mask and, for launches of fewer than 8192
 * waves, the partial sums of the batches' list slices (at most 12 MiB) live
 * in a fixed device array of the
 * library (bltc_noalloc_scratch_bytes: 32 MiB, one copy per device the
 * library runs on, held until the process ends) instead of the targets
 * handle.  The call allocates nothing: the modified weights of `degree` must
 * exist (else BLTC_ESTATE) and, with opt->deg_min >= 1, so must every lower
 * degree the lists use (derived by an earlier bltc_evaluate_tree with the
 * same options; else BLTC_ESTATE).  Lists larger than the array give
 * BLTC_EINVAL with the size needed, before anything is written to out.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other threads, other streams) race and must be serialised by
 * the caller.  Reads the list sizes back once (synchronises on `stream`). */
int bltc_evaluate_tree_noalloc(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                               int32_t degree, double theta, const bltc_options* opt,
                               double* out, void* stream);
/* Size in bytes of the fixed array bltc_evaluate_tree_noalloc uses. */
int bltc_noalloc_scratch_bytes(int64_t* bytes);

/* Cluster-cluster variant (the interpolation in the target variable that
 * Section 9 names as the next step; not in the paper's method).  tgt is a
 * tree built with bltc_build_tree on the TARGET points (its leaf size is the
 * target leaf size; it needs no weights); src holds the sources with the
 * modified weights of `degree` (wdim of the kernel, else BLTC_ESTATE).  A
 * target cluster gets Chebyshev grid points like a source cluster.  The two
 * trees are traversed together from their roots; for a pair (A, C) with
 * P = (degree+1)^3:
 *   MAC R2 > 0 and (r_A + r_C)^2 <= theta^2 R2 (eq. MAC with the target
 *   cluster's radius added): CC (potentials at A's grid points from C's
 *   proxies) if both hold more than P particles; PC (eq.
 *   pc_approximation_3D at A's targets) if only C does; CP (potentials at
 *   A's grid points from C's particles) if only A does; else PP (eq.
 *   pc_interaction_3D);
 *   no MAC: PP if both are leaves, else the pair is refined, A's children if
 *   C is a leaf or A is not a leaf with r_A >= r_C, else C's children.
 * Every target then adds sum_m L_m(x) g_A[m] over the clusters A holding it,
 * with the tensor-product Lagrange basis on A's grid (barycentric form,
 * exact-hit rule of Algorithm 1).  out: FP64 [odim][m] in the target tree's
 * caller order.  counts (host int64 [5], may be NULL): kernel evaluations of
 * the CC, PC, CP and PP interactions and the downward (target, grid point)
 * terms.  With opt->deg_min >= 1 the separation rule (see bltc_options)
 * picks the degree of the source side of each CC and PC pair from the
 * pair's ratio (r_A + r_C)/R; target grids and the downward interpolation
 * keep `degree`.  The traversal runs on the device: per target node its CC
 * and CP lists, per target leaf the PC and PP entries of its root path; the
 * trees may have at most 30 (source) and 31 (target) levels below the root
 * (BLTC_EINVAL beyond).  Synchronises on stream. */
int bltc_evaluate_dual(bltc_tree src, bltc_tree tgt, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt, double* out,
                       int64_t* counts, void* stream);

/* One call: build the source tree (leaf_max), the target batches, the
 * modified weights of `degree`, evaluate, free everything.  opt may be NULL
 * (defaults). */
int bltc_evaluate(const double* tx, const double* ty, const double* tz,
                  int64_t m, const double* sx, const double* sy,
                  const double* sz, int64_t n, const double* w, int32_t kernel,
                  double eps, int32_t degree, double theta, int64_t leaf_max,
                  const bltc_options* opt, double* out, void* stream);

/* Interaction lists of the batch walk, host copies (synchronises): sizes
 * first (lists pointers NULL), then contents.  prox_ptr/dir_ptr[nb+1] index
 * prox_ids/dir_ids (cluster ids in depth-first order, children in order);
 * prox_deg (may be NULL) receives each accepted cluster's degree under the
 * separation rule of bltc_options.deg_min for evaluation degree `degree`
 * (all equal to degree when deg_min = 0). */
int bltc_lists_export(bltc_tree t, bltc_targets g, double theta, int32_t degree,
                      int32_t deg_min, int64_t* nb, int64_t* n_prox, int64_t* n_dir,
                      int64_t* prox_ptr, int32_t* prox_ids, int32_t* prox_deg,
                      int64_t* dir_ptr, int32_t* dir_ids);
/* Kernel evaluations an evaluation performs (synchronises): proxy
 * evaluations sum over targets of (d+1)^3 per accepted cluster of degree d
 * (degree, or the separation rule's when deg_min >= 1), direct ones the leaf
 * sizes of the direct list. */
int bltc_counts(bltc_tree t, bltc_targets g, int32_t degree, double theta,
                int32_t deg_min, int64_t* n_proxy_evals, int64_t* n_direct_evals);

/* Direct sum (eq. N-body) on the device for the k targets idx[0:k] (device
 * int64 indices into the m target arrays, each checked to lie in [0, m),
 * which copies idx to the host and synchronises; NULL = the first k <= m
 * targets in order): out[odim][k].  opt->precision BLTC_FP64 or
 * BLTC_FP32_FP64ACC; opt may be NULL (FP64). */
int bltc_direct(const double* tx, const double* ty, const double* tz,
                int64_t m, const int64_t* idx, int64_t k, const double* sx,
                const double* sy, const double* sz, int64_t n, const double* w,
                int32_t kernel, double eps, const bltc_options* opt,
                double* out, void* stream);

/* ---- per-batch (n, theta) selector network --------------------------------
 * Not part of the paper: the paper picks (theta, n, N0) by hand and notes
 * they are not claimed optimal (Section 6); this network predicts, from 12
 * features of a target batch, the log10 relative error of each of k
 * candidate (n, theta) settings.  Layout, FP32 on the device:
 *   h1 = tanh(W1 x + b1) (64), h2 = tanh(W2 h1 + b2) (64), y = W3 h2 + b3 (k)
 * params = W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [k][64], b3 [k];
 * X [rows][12]; Y [rows][k]; cache [rows][128] (h1 then h2, for backward).
 * 1 <= k <= 128.  work is a caller-owned device scratch array of at least
 * bltc_mlp_work_size floats, so training loops allocate nothing. */
int bltc_mlp_params(int32_t k, int64_t* n_params);
int bltc_mlp_work_size(int64_t rows, int32_t k, int64_t* n_floats);
int bltc_mlp_forward(const float* params, const float* X, int64_t rows,
                     int32_t k, float* Y, float* cache, void* stream);
/* dY = 2 (Y - T) / (rows k) and *loss (device) = mean (Y - T)^2. */
int bltc_mlp_loss(const float* Y, const float* T, int64_t rows, int32_t k,
                  float* dY, float* loss, float* work, void* stream);
/* grad = gradient of sum(dY * Y) w.r.t. params (deterministic reduction). */
int bltc_mlp_backward(const float* params, const float* X, const float* cache,
                      const float* dY, int64_t rows, int32_t k, float* grad,
                      float* work, void* stream);
/* One Adam step with bias correction (step counts from 1). */
int bltc_adam_step(float* params, float* m, float* v, const float* grad,
                   int64_t n, float lr, float beta1, float beta2, float eps,
                   int64_t step, void* stream);

/* ---- learned (n, theta) per batch ----------------------------------------
 * Features of every batch (device FP32 [nb][12], unnormalised), from its
 * geometry and one walk at theta_ref:
 *   0 log2 targets, 1 log10 r_B/R0, 2 log10 eps/R0, 3 log10 eps/r_B,
 *   4 log10(1 + accepted clusters), 5 log10(1 + near-field sources),
 *   6 log10(1 + near-field leaves), 7 mean log10 r_C/R0 of accepted
 *   clusters, 8 mean (r_B + r_C)/(theta_ref R) of accepted clusters,
 *   9 log10 near-field source density over the mean density, 10 kernel
 *   (0 Stokeslet, 1 rotlet), 11 log10 n;  R0 = root radius. */
int bltc_batch_features(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                        double theta_ref, float* feat, void* stream);
/* Per-batch counts of the walk at theta (device int32 [nb] each): accepted
 * clusters and near-field source particles. */
int bltc_batch_counts(bltc_tree t, bltc_targets g, double theta, int32_t* n_proxy,
                      int32_t* n_near, void* stream);

/* Modelled wave cost of every batch under each of k candidates
 * (cand_n[j], cand_theta[j]) (host arrays), into cost (device float
 * [k][nb]): one walk per distinct theta; an accepted cluster of degree d
 * (the candidate's, or the separation rule's when deg_min >= 1) costs
 * (weights[0] (d+1) + weights[1]) (d+1)^2 + weights[2], a near-field source
 * weights[3].  weights: host float[4] (per proxy evaluation, per grid row,
 * per cluster, per near source). */
int bltc_batch_costs(bltc_tree t, bltc_targets g, int32_t k, const int32_t* cand_n,
                     const double* cand_theta, int32_t deg_min, const float* weights,
                     float* cost, void* stream);

/* A selector model file: little-endian
 *   char[8] "BLTCSEL1"; int32 version = 4, n_in = 12, n_hidden = 64, k,
 *   deg_min (the separation rule the candidates are evaluated with, 0 = off);
 *   int32 cand_n[k]; double cand_theta[k];
 *   double theta_ref, cost_far, cost_row, cost_cluster, cost_near, margin,
 *          margin_global;
 *   float mean[12], std[12]  (feature normalisation);
 *   float params[bltc_mlp_params(k)];
 *   uint64 FNV-1a hash of all preceding bytes.
 * Any mismatch returns BLTC_EMODEL. */
int bltc_selector_load(const char* path, bltc_selector* out);
int bltc_selector_destroy(bltc_selector sel);
int bltc_selector_info(bltc_selector sel, int32_t* k, int32_t* cand_n,
                       double* cand_theta);

/* The judge's samples (the a11 step of bltc_evaluate_adaptive, exposed for
 * checks): the fixed treecode of Algorithm 2 with degree fb_degree and the
 * paper's per-target MAC r/R <= fb_theta (eq. MAC), each sample target
 * walked on its own from the root, FP32 kernel evaluation with FP64 sums.
 * The samples are one target per batch, at a hashed position inside the
 * batch (fixed by the targets handle); from 32,768 batches on, one per
 * floor(nb / 16384) consecutive batches, in the first of them.  Computes the
 * modified weights of fb_degree when missing.  *n_samples receives their
 * number; target_idx (host int64 [n_samples], caller's target order) and
 * ufb (host FP64 [n_samples][odim]) may be NULL (then nothing is
 * evaluated).  Kernels BLTC_STOKESLET and BLTC_ROTLET.  Synchronises. */
int bltc_judge_samples(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                       int32_t fb_degree, double fb_theta, int64_t* n_samples,
                       int64_t* target_idx, double* ufb, void* stream);

/* Evaluation with a learned (n, theta) per batch, aiming at a relative L2
 * error tol over all targets (the paper's eq. error).  Not in the paper,
 * which fixes (theta, n) for a run (Section 6).  Kernels BLTC_STOKESLET and
 * BLTC_ROTLET (the kernels the network's features describe).
 *  1. The network predicts e_b(j), the relative error of batch b under each
 *     candidate j; bltc_batch_costs gives its modelled wave cost with the
 *     model's cost weights, under the model's separation rule (deg_min).
 *  2. The judge: the samples of bltc_judge_samples (one target per batch,
 *     or per group of batches when there are many) are evaluated with the
 *     fallback treecode (fb_degree, fb_theta) (Algorithm 2 with the
 *     per-target MAC); w_b = targets_b |u_fb|^2 (at the sample of b's group)
 *     estimates the batch's share of the reference norm.
 *  3. mode BLTC_SELECT_BATCH: the batches share the error budget: the
 *     choice minimises the total cost subject to
 *     sum_b w_b e_b^2 <= tau^2 sum_b w_b, tau = 0.8 tol 10^-margin (0.8
 *     tol: the judge's trigger, step 5), through the Lagrange multiplier of
 *     cost + lam w_b e_b^2 (searched on a log grid in two passes).  mode
 *     BLTC_SELECT_RUN: one candidate for every batch, the cheapest whose
 *     predicted global error is within 0.8 tol 10^-margin_global (else the
 *     one predicted most accurate).
 *  4. Lists at each batch's theta (and the separation rule's degrees);
 *     modified weights of every top degree in use and, under the rule, of
 *     the lower degrees derived from each top degree's (so a batch's result
 *     equals the fixed evaluation at its candidate: bit for bit when its
 *     group's launch slices its lists as the fixed one does, else up to the
 *     order of the FP64 sums); evaluation grouped by the batches' top
 *     degrees, the groups running concurrently, a group of under 8192 waves
 *     slicing every batch's lists (more finely than a full evaluation).
 *  5. The judge's estimate E^2 = sum_i G_i |u - u_fb|^2 / sum_i G_i |u_fb|^2
 *     over the samples (G_i the targets of sample i's group); when it
 *     exceeds (0.8 tol)^2, the samples with the largest terms, just enough
 *     of them to bring the estimate to (0.6 tol)^2, have their batches
 *     evaluated again with the fallback (its batch walk at fb_theta).  The
 *     estimate is a sample: the margins make a result above tol unlikely,
 *     not impossible.
 * choice (host int32 [nb], may be NULL): candidate index, or -2 for a batch
 * the judge sent to the fallback.  stats (host int64 [4], may be NULL):
 * batches, distinct degrees, batches re-evaluated, 0.  judge (host double
 * [2], may be NULL): the judge's error estimate before and after its
 * re-evaluation.  opt supplies the precision; its deg_min is ignored (the
 * candidates take the model's rule, the fallback none).  Synchronises on
 * stream. */
enum { BLTC_SELECT_BATCH = 0, BLTC_SELECT_RUN = 1 };
int bltc_evaluate_adaptive(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                           bltc_selector sel, double tol, int32_t mode, int32_t fb_degree,
                           double fb_theta, const bltc_options* opt, double* out,
                           int32_t* choice, int64_t* stats, double* judge,
                           void* stream);

/* ---- testing ---------------------------------------------------------------
 * Failure injection for tests of the error paths: the after-th device
 * allocation the library makes from now on fails as if the device were out
 * of memory (the call returns BLTC_ENOMEM with no output written); 0
 * disarms.  Process wide; not thread safe. */
int bltc_test_fail_alloc(int32_t after);

/* ---- measurement ---------------------------------------------------------
 * Stage timing with HIP events recorded on the evaluation stream around each
 * stage of bltc_compute_modified_weights and bltc_evaluate_tree:
 *   BLTC_STAGE_PREP    weight gather and cluster grids,
 *   BLTC_STAGE_UPWARD  modified-weight contraction and its reduction,
 *   BLTC_STAGE_LISTS   interaction lists (count, scan, read-back, fill),
 *   BLTC_STAGE_EVAL    the particle-cluster evaluation kernel.
 * bltc_profile_enable(1) starts recording (process wide, for measurement
 * runs, not thread safe); bltc_profile_read synchronises on the recorded
 * events, returns the summed milliseconds and the launch count per stage
 * (arrays of BLTC_NSTAGES) and, if reset, clears them. */
enum { BLTC_STAGE_PREP = 0, BLTC_STAGE_UPWARD = 1, BLTC_STAGE_LISTS = 2,
       BLTC_STAGE_EVAL = 3, BLTC_NSTAGES = 4 };
int bltc_profile_enable(int32_t on);
int bltc_profile_read(double* ms, int64_t* launches, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif
