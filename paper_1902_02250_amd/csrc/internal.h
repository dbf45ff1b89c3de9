// Internal declarations of the treecode library: handle layouts, the host
// tree builder and the kernel launchers.  Nothing here is part of the C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace bltc {

constexpr int kMaxDegree = 12;
constexpr int kWave = 64;
constexpr int kUpwardChunk = 512;    // particles per upward-pass work group
constexpr int kMlpIn = 12;           // selector network: features
constexpr int kMlpHidden = 64;       // selector network: hidden width
constexpr int kMlpMaxOut = 128;      // selector network: most candidates
// The judge samples one target in every batch up to 2 kJudgeMinSamples
// batches, above that one in every nb / kJudgeMinSamples consecutive batches.
constexpr int64_t kJudgeMinSamples = 16384;
inline int judge_stride(int64_t nb) {
  return (int)(nb / kJudgeMinSamples > 1 ? nb / kJudgeMinSamples : 1);
}
// A proxy-list entry holds the cluster id in its low kDegShift bits and,
// under the separation rule, the cluster's degree above them (0: the
// evaluation's degree).
constexpr int kDegShift = 27;
constexpr int32_t kIdMask = (1 << kDegShift) - 1;

// ---- host tree (Section 6) ------------------------------------------------
struct HostTree {
  int64_t n = 0;
  int32_t depth = 0;
  std::vector<int32_t> perm;     // tree position -> input index
  std::vector<double> box;       // [nn][6]: lo x, lo y, lo z, hi x, hi y, hi z
  std::vector<double> ctr;       // [nn][3]
  std::vector<double> rad;       // [nn]
  std::vector<int32_t> first, count, level, begin, end;
  int64_t nnodes() const { return (int64_t)rad.size(); }
};

void build_host_tree(const double* x, const double* y, const double* z,
                     int64_t n, int64_t leaf_max, HostTree& t);

// Target batches: tree order (leaf size order_leaf); every group node (a
// maximal node with at most group_max targets) is cut into consecutive chunks
// of batch_size, so no batch spans two groups.
struct HostBatches {
  std::vector<int32_t> perm;     // target position -> input index
  std::vector<int32_t> bptr;     // [nb+1]
  std::vector<double> geo;       // [nb][4]: center xyz, radius
};
void build_host_batches(const double* x, const double* y, const double* z,
                        int64_t m, int32_t batch_size, int32_t order_leaf,
                        int64_t group_max, HostBatches& b);
// Batch starts bptr[nb+1] and ends bend[nb] over an order tree: the group
// nodes in tree order, each cut into consecutive pieces of batch_size.
void batch_bounds(const HostTree& order, int32_t batch_size, int64_t group_max,
                  std::vector<int32_t>& bptr, std::vector<int32_t>& bend);
// Balanced k-d batches (order_leaf = 0): a part of c > batch_size targets is
// cut along the longest side of its tight box (the first of equal sides),
// the first part taking the batch_size floor(nb / 2) targets with the
// smallest coordinates on that axis (ties by index), nb = ceil(c /
// batch_size); parts of at most batch_size targets are batches, in cut
// order, their targets in increasing index.  Every batch is full except at
// most one.  perm[m] (position -> index), bptr[nb + 1].
void kd_batches(const double* x, const double* y, const double* z, int64_t m, int32_t bs,
                std::vector<int32_t>& perm, std::vector<int32_t>& bptr);


// Unit Chebyshev points of the 2nd kind, descending.
void cheb_points(int degree, double* t);

// One cluster of a tree level as the device builder computes it.
struct TreeLevelNode {
  double lo[3], hi[3], ctr[3], rad;
  int32_t mask;      // axes to bisect (bit a); 0 = no split attempted
  int32_t pad;
};
constexpr int kTreeChunk = 8192;   // particles per work group in the tree build

// ---- kernel launch arguments ----------------------------------------------
// The cut of a tree for walks shared by a wave's lanes (walk.h): the
// clusters at the cut depth and the shallower leaves, in depth-first order,
// with each one's ancestors root first (at most kCutMaxDepth, -1 padded)
// and, in bit j of cut_first, whether it is the first cut node under its
// ancestor j.
constexpr int kCutMaxDepth = 8;

struct Nodes {                 // device node arrays
  const double4* geo;          // center xyz, radius
  const int2* range;           // particle range [begin, end) in tree order
  const int2* kids;            // first child, child count
  const int32_t* skip;         // next node in depth-first order after the subtree (-1: end)
  int64_t nn;
  const int32_t* cut = nullptr;        // [ncut]
  const int32_t* cut_anc = nullptr;    // [ncut][kCutMaxDepth]
  const uint32_t* cut_first = nullptr; // [ncut]
  int32_t ncut = 0;
};

// Separation rule for the degree of an accepted cluster: the smallest d in
// [deg_min, degree) with (r_B + r_C)^2 / R^2 <= T[d], else degree; off when
// deg_min = 0.
struct Rule {
  int32_t deg_min = 0, degree = 0;
  double T[kMaxDegree + 1] = {};
};

struct ListArgs {
  const double4* bgeo;         // batch center, radius
  int64_t nb;
  Nodes nodes;
  double theta;
  Rule rule;
  // separation rule per batch (learned evaluation): batch b uses candidate
  // choice[b], whose thresholds are cand_T[choice[b]][.] and degree
  // cand_deg[choice[b]]; rule_deg_min 0 turns it off
  const int32_t* choice = nullptr;
  const double* cand_T = nullptr;
  const int32_t* cand_deg = nullptr;
  int32_t rule_deg_min = 0;
  const double* theta_b = nullptr;  // [nb] per-batch theta, or NULL
  int32_t* pcnt;               // [nb] proxy count (count pass)
  int32_t* dcnt;               // [nb] direct count
  int32_t* scnt = nullptr;     // [nb] near-field source count, or NULL
  const int32_t* pptr;         // [nb+1] (fill pass)
  const int32_t* dptr;
  int32_t* pids;
  int32_t* dids;
  int32_t* err;                // error flag (unused by the stackless walk)
};

struct P2PArgs {
  const int32_t* bmap = nullptr;  // batches to evaluate (NULL: all nb)
  int64_t nmap = 0;
  const double* tx;            // tree-ordered targets [3][m]
  int64_t m;
  const int32_t* tperm;        // target position -> caller index
  const int32_t* bptr;         // [nb+1]
  const double4* bgeo;
  int64_t nb;
  int32_t wpb;                 // waves per batch
  const int32_t* pptr;
  const int32_t* pids;
  const int32_t* dptr;
  const int32_t* dids;
  const int2* range;
  const double* grid;          // [nn][3][n1]
  const void* fhat;            // [nn][n1][n1][3][n1], FP64 or FP32
  const double* grid_d[kMaxDegree + 1] = {};  // per degree (separation rule)
  const void* fhat_d[kMaxDegree + 1] = {};
  const double* ys;            // tree-ordered sources [3][n]
  const double* w64;           // tree-ordered weights [3][n]
  const float* w32;
  int64_t n;
  double eps;
  int32_t poly_p;
  double poly_c;
  double scale_u, scale_w;     // constant factors applied at the end
  double* out;                 // [odim][m] caller order
  // split mode (split != NULL): wave w evaluates batch split[w].x over the
  // entries [split[w].y, split[w].z) of its proxy list (split[w].w == 0) or
  // of its direct list (split[w].w != 0), and writes unscaled FP64 sums to
  // partial[w][odim][64]
  const int4* split = nullptr;
  int64_t nsplit = 0;
  double* partial = nullptr;
  // XCD ranges of the launch order (NULL: contiguous equal counts): XCD x
  // runs the waves [xstart[x], xstart[x + 1]); xmax the longest range (host
  // value)
  const int32_t* xstart = nullptr;
  int32_t xmax = 0;
  // slices per batch (without split): slices > 1 gives each (batch, wave of
  // targets) that many waves, slice j taking the j-th of `slices` equal parts
  // of the batch's proxy list (by entries) and of its near-field tiles (64
  // sources each, along the runs of contiguous leaves), and
  // writing unscaled FP64 sums to spart[((i wpb + wv) slices + j)][odim][64]
  // for the batch at launch position i (bmap[i], or i); launch_slice_reduce
  // then adds the slices in order and scatters
  int32_t slices = 1;
  double* spart = nullptr;
};

// Cluster-cluster variant: interpolation of the grid potentials to targets.
struct DualDownArgs {
  const int32_t* bptr;         // target batches [nb+1] in target tree order
  int64_t nb;
  int32_t wpb = 1;             // waves of 64 targets per batch
  const double* tx;            // tree-ordered targets [3][m]
  int64_t m;
  const int32_t* tperm;        // target position -> caller index
  const int32_t* dptr;         // per batch: entries (grid slot, target node)
  const int32_t* dgi;
  const int32_t* dnode;
  const double* tgrid;
  const double* g;             // grid potentials [odim][gstride], slot gi at gi (n+1)^3
  int64_t gstride;
  double* out;                 // [odim][m] caller order, added to
};

// The judge's samples: the fixed treecode of Algorithm 2 at single targets
// (one wave each), walked with the per-target MAC.
struct SampleArgs {
  const int32_t* spos;         // [ns] sampled target positions (tree order)
  int ns;
  const double* tx;            // tree-ordered targets [3][m]
  int64_t m;
  const int2* range;           // [nn] cluster source ranges
  // each sample's lists: its walk of Algorithm 2 with the per-target MAC
  const int32_t* pptr;         // [ns+1] proxy (accepted cluster) lists
  const int32_t* pids;
  const int32_t* dptr;         // [ns+1] direct (leaf) lists
  const int32_t* dids;
  const double* grid;          // [nn][3][n1] of the fallback degree
  const float* fh32;           // its modified weights, evaluation layout
  const double* ys;            // tree-ordered sources [3][n]
  const float* w32;
  int64_t n;
  double eps, scale_u, scale_w;
  double* ufb;                 // [ns][odim]
};

struct FeatArgs {
  const double4* bgeo;
  const int32_t* bptr;
  int64_t nb;
  Nodes nodes;
  const double* box;           // [nn][6]
  double theta_ref;
  double eps;
  int kernel;
  int64_t n_src;
  const float* mean;           // [12] or NULL: raw features
  const float* stdv;
  float* feat;                 // [nb][12]
};

struct Candidates {
  int32_t n[kMlpMaxOut];
  int32_t t[kMlpMaxOut];       // index of the candidate's theta
};

// Modelled cost weights of one wave: per proxy evaluation, per grid row,
// per accepted cluster and per near-field source.
struct Costs {
  float far, row, clu, nearf;
};

// Modelled wave cost of every batch under the candidates that share one
// theta: one walk per batch; an accepted cluster costs
// (far n1 + row) n1^2 + clu with n1 - 1 its degree (the candidate's, or the
// separation rule's), a near-field source costs nearf.
constexpr int kMaxPerTheta = 16;
// The candidates sharing one theta.
struct CostGroup {
  double theta;
  int32_t nc;                          // candidates with this theta
  int32_t deg[kMaxPerTheta];           // their degrees
  int32_t row[kMaxPerTheta];           // output row of each candidate
  // The rule's degree of an accepted cluster depends on its qq = (rr/R)^2
  // only through the bucket k = #{U[j] < qq} of the group's sorted distinct
  // thresholds U[0..nu); C[i][k] (i < nc, k <= nu) is the cost of a cluster
  // in bucket k for candidate i.
  int32_t nu;
  int32_t u_off, c_off;                // offsets into CostArgs::U and ::C
};
constexpr int kMaxThetaGroups = 8;     // theta groups per launch (grid y)
constexpr int kMaxBuckets = kMaxPerTheta * kMaxDegree;   // most thresholds per group

struct CostArgs {
  const double4* bgeo;
  int64_t nb;
  Nodes nodes;
  int32_t ngroups;
  CostGroup grp[kMaxThetaGroups];
  const double* U;                     // the groups' thresholds (device)
  const float* C;                      // the groups' bucket costs [nc][nu + 1] (device)
  float nearf;                         // cost of one near-field source
  float* cost;                         // [rows][nb]
  int32_t* err;
};

// The dual traversal of the cluster-cluster variant on the device: one wave
// per target node (per-node mode: that node's CC and CP lists and the
// evaluation counts) or per target leaf (per-leaf mode: the PC and PP
// entries of the leaf and of all its ancestors).  The waves walk the source
// tree over its cut (walk.h) with the target's level along its root path as
// state; the decisions are the host traversal's, FP64 without contraction.
constexpr int kDualMaxDepth = 32;      // most levels of either tree
struct DualArgs {
  Nodes src;                           // the source tree with its cut
  const int32_t* slevel;               // [snn] source node depth
  const double4* tgeo;                 // target tree: center, radius
  const int2* trange;
  const int2* tkids;
  const int32_t* tparent;              // [tnn], -1 at the root
  const int32_t* items;                // per-leaf mode: the leaves; per-node mode: NULL
  int64_t nitems;
  double th2;                          // theta theta
  int64_t P;                           // (n + 1)^3
  int32_t n1;
  Rule rule;
  int32_t* cnt0;                       // count pass: CC (per node) or PC (per leaf) entries
  int32_t* cnt1;                       // CP (per node) or PP (per leaf) entries
  unsigned long long* work;            // per-node count pass: [5] evaluations CC, PC, CP, PP, downward
  const int32_t* ptr0;                 // fill pass: offsets [nitems + 1]
  const int32_t* ptr1;
  int32_t* ids0;
  int32_t* ids1;
};
hipError_t launch_dual_walk(const DualArgs& a, bool per_leaf, bool fill, hipStream_t s);
// Grid slots of the target nodes with CC or CP work: flag[q] = 1 for them.
hipError_t launch_dual_flags(const int32_t* ncc, const int32_t* ncp, int64_t nn, int32_t* flag,
                             hipStream_t s);
// For every flagged node q: slot gi = slot[q], gnode[gi] = q, gbgeo[gi] = its
// geometry, gbptr[gi] = gi P, gpptr[gi] = ccptr[q], gdptr[gi] = cpptr[q], and
// work[4] += |q| P; entry ng of gbptr, gpptr, gdptr closes the arrays.
hipError_t launch_dual_slots(const int32_t* flag, const int32_t* slot, int64_t nn, int64_t ng,
                             int64_t P, const double4* tgeo, const int2* trange,
                             const int32_t* ccptr, const int32_t* cpptr, int32_t* gnode,
                             double4* gbgeo, int32_t* gbptr, int32_t* gpptr, int32_t* gdptr,
                             unsigned long long* work, hipStream_t s);
// Per leaf (leaves[l]): the slots of the flagged nodes on its root path, root
// first (count pass: xcnt[l]; fill pass: xgi and xnode at xptr[l]).
hipError_t launch_dual_xlists(const int32_t* leaves, int64_t nl, const int32_t* tparent,
                              const int32_t* flag, const int32_t* slot, int32_t* xcnt,
                              const int32_t* xptr, int32_t* xgi, int32_t* xnode, bool fill,
                              hipStream_t s);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
// Balanced k-d target batches on the device (k_kd.hip).  Parts above
// kKdLocal targets are cut level by level over all of them: chunks (part,
// begin, end) of at most kKdChunk positions, each part's chunks consecutive
// from cfirst[part]; keys (part, coordinate, index) in hi/lo (n2, a power of
// two >= 2048, padded with all-ones keys), lo's low 44 bits the index.
// Parts of at most kKdLocal targets finish in one work group each and write
// perm.
constexpr int kKdLocal = 4096;
constexpr int kKdChunk = 4096;
hipError_t launch_kd_init(uint64_t* hi, uint64_t* lo, int64_t m, int64_t n2, hipStream_t s);
hipError_t launch_kd_level(const int4* chunks, int32_t nchunks, const int32_t* cut,
                           const int32_t* cfirst, int32_t nseg, const double* x,
                           const double* y, const double* z, double* part, int32_t* axis,
                           uint64_t* hi, uint64_t* lo, int64_t n2, hipStream_t s);
hipError_t launch_kd_local(const int2* parts, int32_t nparts, const uint64_t* lo,
                           const double* x, const double* y, const double* z, int32_t bs,
                           int32_t* perm, hipStream_t s);

// ---- launchers (defined in the .hip files) --------------------------------
// sgeo[i] = (target spos[i], radius 0): a sample as a batch of one target,
// whose batch MAC is the per-target MAC.
hipError_t launch_sample_geo(const int32_t* spos, int ns, const double* tx, int64_t m,
                             double4* sgeo, hipStream_t s);
hipError_t launch_fallback_samples(int kernel, int degree, const SampleArgs& a,
                                   hipStream_t s);
hipError_t launch_features(const FeatArgs& a, hipStream_t s);
int64_t alloc_blocks(int64_t nb);
hipError_t launch_pred_err2(const float* Y, int k, int64_t nb, double* e2, hipStream_t s);
hipError_t launch_alloc(const double* e2, int k, int64_t nb, const float* cost,
                        const double* wt, double inv_wsum, const double* lam, int G,
                        double* partial, double* sums, hipStream_t s);
hipError_t launch_cand_totals(const double* e2, int k, int64_t nb, const float* cost,
                              const double* wt, double inv_wsum, double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_choose(const double* e2, int k, int64_t nb, const float* cost,
                         const double* wt, double inv_wsum, double lam, int32_t* choice,
                         hipStream_t s);
hipError_t launch_judge(int ns, int stride, int64_t nb, const int32_t* bptr,
                        const int32_t* spos, const int32_t* tperm, const double* out,
                        int64_t m, int od, const double* ufb, double* usq, double* contrib,
                        double* partial, double* sums, hipStream_t s);
hipError_t launch_batch_weights(int64_t nb, int stride, const int32_t* bptr,
                                const double* usq, double* wt, hipStream_t s);
hipError_t launch_flag(int ns, const double* contrib, double thr, int32_t* flag,
                       hipStream_t s);
hipError_t launch_cand_costs(const CostArgs& a, hipStream_t s);
// mask[0] = the bits 1 << d of the degrees d that the proxy lists of the
// batches bsel[0..nsel) carry (all nsel batches when bsel is NULL).
hipError_t launch_degree_mask(const int32_t* bsel, int64_t nsel, const int32_t* pptr,
                              const int32_t* pids, uint32_t* mask, hipStream_t s);
hipError_t launch_dual_points(const int32_t* gnode, int64_t ng, int n1, const double* tgrid,
                              double* pts, hipStream_t s);
hipError_t launch_dual_down(int odim, int n1, const DualDownArgs& a, hipStream_t s);
hipError_t launch_tree_init(const double* x, const double* y, const double* z, int64_t n,
                            double* c, int32_t* perm, hipStream_t s);
hipError_t launch_tree_level(const int4* chunks, int64_t nch, const int32_t* cptr,
                             const int2* range, int nl, const double* c, int64_t n,
                             int64_t leaf_max, double* cmm, TreeLevelNode* nodes,
                             int32_t* hist, hipStream_t s);
// Partitions the chunks of splitting clusters (pos[c][8] != 0) of the
// current order (c, perm) through the scratch buffers (tc, tperm); (c, perm)
// hold the new order afterwards.
hipError_t launch_tree_scatter(const int4* chunks, int64_t nch, const int32_t* pos, int64_t n,
                               const TreeLevelNode* nodes, double* c, int32_t* perm,
                               double* tc, int32_t* tperm, hipStream_t s);
hipError_t launch_batch_geo(const double* c, int64_t m, const int32_t* bptr, const int32_t* bend,
                            int64_t nb, double4* geo, hipStream_t s);
hipError_t launch_gather_points(const double* x, const double* y,
                                const double* z, const int32_t* perm,
                                int64_t n, double* out3, hipStream_t s);
hipError_t launch_gather_weights(const double* w, const int32_t* perm,
                                 int64_t n, int wd, double* w64, float* w32,
                                 hipStream_t s);
hipError_t launch_grids(const double* box, int64_t nn, int degree,
                        const double* unit_nodes, double* grid, hipStream_t s);
hipError_t launch_upward(const double* ys, const double* w64, int64_t n, int wd,
                         const int4* chunks, int64_t nchunks,
                         const double* grid, int degree, double* partial, hipStream_t s);
hipError_t launch_upward_reduce(const int32_t* chunk_ptr, int64_t nn,
                                const double* partial, int degree, int wd,
                                double* fhat64, double* p2p64, float* p2p32, hipStream_t s);
// Lower-degree weights from a higher degree's of the same clusters:
// R[k * n1 + m] = L^d_k(t^n_m) on the reference nodes, d1 = d + 1 <= n1 = n + 1.
struct RestrictArgs {
  double R[(kMaxDegree + 1) * (kMaxDegree + 1)];
  int32_t d1 = 0, n1 = 0;
};
hipError_t launch_restrict(const RestrictArgs& a, int64_t nn, int wd, const double* src,
                           double* fhat64, double* p2p64, float* p2p32, hipStream_t s);
// Parents nodes[0..count) from their children's weights (one tree level).
hipError_t launch_m2m(const int32_t* nodes, int64_t count, const int2* kids, int degree, int wd,
                      const double* grid, double* fhat64, double* p2p64, float* p2p32,
                      hipStream_t s);
hipError_t launch_lists(const ListArgs& a, bool fill, hipStream_t s);
hipError_t launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* out,
                                 int32_t* overflow, hipStream_t s);
// out[c][tperm[t]] = scale * (sum of the slices sptr[r] .. sptr[r+1] of
// partial) for every target t of batch bmap[r].
hipError_t launch_split_reduce(const int32_t* sptr, const int32_t* bmap, int64_t nr,
                               const int32_t* bptr, const int32_t* tperm, const double* partial,
                               int odim, double su, double sw, int64_t m, double* out,
                               hipStream_t s);
hipError_t launch_p2p(int kernel, int precision, int degree,
                      const P2PArgs& a, hipStream_t s);
// out[c][tperm[t]] = scale * sum over j < slices of spart[((i wpb + wv)
// slices + j)][c][t - bptr[b] - 64 wv] for every target t of the batches
// b = bmap[i], i < n (or b = i), in wave wv of 64 targets.
hipError_t launch_slice_reduce(const int32_t* bmap, int64_t n, const int32_t* bptr, int wpb,
                               int slices, const int32_t* tperm, const double* spart, int odim,
                               double su, double sw, int64_t m, double* out, hipStream_t s);
hipError_t launch_direct(int kernel, int precision, const double* tx,
                         const double* ty, const double* tz,
                         const int64_t* idx, int64_t k, const double* sx,
                         const double* sy, const double* sz, int64_t n,
                         const double* w, double eps, int32_t poly_p,
                         double poly_c, double scale_u, double scale_w,
                         double* out, hipStream_t s);

// selector network (k_mlp.hip)
int64_t mlp_params(int k);
int64_t mlp_work_floats(int64_t rows, int k);
hipError_t launch_mlp_forward(const float* p, const float* X, int64_t rows,
                              int k, float* Y, float* cache, hipStream_t s);
hipError_t launch_mlp_loss(const float* Y, const float* T, int64_t total,
                           float* dY, float* loss, float* work, hipStream_t s);
hipError_t launch_mlp_backward(const float* p, const float* X,
                               const float* cache, const float* dY,
                               int64_t rows, int k, float* grad, float* work,
                               hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n,
                       float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s);

}  // namespace bltc

// ---- handles ----------------------------------------------------------------
struct bltc_degree_data {
  double* grid = nullptr;      // [nn][3][n1]
  double* fhat64 = nullptr;    // [nn][3][nk] (k3 fastest)
  double* p2p64 = nullptr;     // [nn][n1][n1][3][n1]
  float* p2p32 = nullptr;
};

struct bltc_dual_cache;
struct bltc_split_cache;

struct bltc_tree_s {
  int device = 0;
  int64_t n = 0, leaf_max = 0;
  bltc::HostTree host;
  int32_t* d_perm = nullptr;   // [n]
  double* d_y = nullptr;       // tree-ordered [3][n]
  double* d_box = nullptr;     // [nn][6]
  double4* d_geo = nullptr;
  int2* d_range = nullptr;
  int2* d_kids = nullptr;
  int32_t* d_skip = nullptr;   // depth-first successor past each subtree
  int32_t* d_level = nullptr;  // node depth
  int32_t* d_parent = nullptr; // parent node, -1 at the root
  int32_t* d_cut = nullptr;    // the cut for lane-shared walks (see Nodes)
  int32_t* d_cut_anc = nullptr;
  uint32_t* d_cut_first = nullptr;
  int32_t ncut = 0;
  // weights
  bool has_w = false;
  int32_t wdim = 3;            // weight components: 3, or 6 for force and torque
  double* d_w64 = nullptr;     // tree-ordered [wdim][n]
  float* d_w32 = nullptr;
  std::map<int, bltc_degree_data> deg;
  std::map<int, bltc_degree_data> spare;   // buffers of stale tables, by degree
  // separation rule: degree d derived from the weights of degree n > d,
  // keyed (d, n), and the buffers of stale ones
  std::map<std::pair<int, int>, bltc_degree_data> derived, spare_derived;
  bltc_dual_cache* dual = nullptr;   // cluster-cluster buffers (as the target tree)
  // upward pass: chunks of the leaves' particle ranges, and the parents by
  // level, deepest level first
  int64_t nchunks = 0;
  int4* d_chunks = nullptr;    // node, begin, end, 0
  int32_t* d_chunk_ptr = nullptr;  // [nn+1]
  int32_t* d_parents = nullptr;    // parents, deepest level first
  std::vector<std::pair<int64_t, int64_t>> parent_levels;   // (offset, count) per level
  double* d_partial = nullptr;
  size_t partial_cap = 0;      // doubles
};

namespace bltc {
// Interaction lists of one walk over all batches (grown on demand).
struct ListSet {
  int32_t* cnt = nullptr;      // [3][nb]: proxies, leaves, near sources
  int32_t* ptr = nullptr;      // [2][nb+1]: proxy and leaf CSR pointers
  int32_t* pids = nullptr;
  int32_t* dids = nullptr;
  int64_t pcap = 0, dcap = 0;
  // Storage owned elsewhere and never grown: pids heads a region of pcap
  // int32 that holds the proxy list and then the leaf list (at pids plus
  // the proxy total rounded up to 64 entries).
  bool fixed = false;
  int32_t* flags = nullptr;    // [4] walk and scan flags, or NULL: the targets' own
};
}  // namespace bltc

struct bltc_targets_s {
  int device = 0;
  bltc_split_cache* split = nullptr;   // the judge's repair slices (grown on demand)
  uint32_t* d_dmask = nullptr;   // [kMaxDegree + 1] degrees used per evaluation group
  int64_t m = 0, nb = 0;
  int32_t batch_size = 0, order_leaf = 0;
  int64_t group_max = 0;
  bltc::HostBatches host;
  int32_t* d_tperm = nullptr;
  double* d_x = nullptr;       // tree-ordered [3][m]
  int32_t* d_bptr = nullptr;
  double4* d_bgeo = nullptr;
  int32_t* d_flags = nullptr;  // [4]: walk error, scan overflow x2, spare
  bltc::ListSet ls[2];         // [0] evaluation lists, [1] the fallback's lists (repairs)
  // per-batch selection scratch (allocated on first adaptive call)
  float* d_feat = nullptr;     // [nb][12]
  float* d_Y = nullptr;        // [nb][k]
  int64_t ycap = 0;
  int32_t* d_pc = nullptr;     // [ntheta][nb]
  int32_t* d_sc = nullptr;
  int64_t pccap = 0;
  int32_t* d_choice = nullptr; // [nb]
  int32_t* d_bmap = nullptr;   // [nb]
  int32_t* d_xmap = nullptr;   // [nb] batch order of the evaluation launches (per group)
  double* d_spart = nullptr;   // slice partial sums (small launches), grown on demand
  int64_t spart_cap = 0;       // doubles
  int32_t* d_xstart = nullptr; // [kMaxDegree + 1][9] XCD ranges in waves (per group)
  std::vector<int32_t> h_xmap, h_xstart;   // their host copies (sources of the uploads)
  std::vector<int32_t> h_cnt;  // list counts read back for the order
  double* d_theta_b = nullptr; // [nb]
  int32_t* d_spos = nullptr;   // judge samples, one per sstride batches (tree order)
  double4* d_sgeo = nullptr;   // [nsamp] the samples as batches of one target
  int32_t* d_sflags = nullptr; // [4] walk and scan flags of the samples' lists
  bltc::ListSet ls_samp;       // the samples' lists (per-target MAC, fallback theta)
  double* d_ufb = nullptr;     // [nb][6]
  int32_t nsamp = 0;           // judge samples (one per sstride batches)
  int32_t sstride = 1;         // batches per judge sample (judge_stride)
  double* d_usq = nullptr;     // [nsamp] |u_fb|^2 at the samples
  double* d_wt = nullptr;      // [nb] batch weights targets_b |u_fb|^2
  double* d_contrib = nullptr; // [nsamp] judge error contributions
  double* d_part = nullptr;    // [blocks][G][2] partial sums
  double* d_sums = nullptr;    // [G][2]
  double* d_lam = nullptr;     // [G]
  float* d_cost = nullptr;     // [k][nb] modelled costs
  double* d_e2 = nullptr;      // [k][nb] predicted squared errors
  int64_t costcap = 0;
  double* d_candT = nullptr;   // [k][kMaxDegree+1] rule thresholds
  void* d_costtab = nullptr;   // the cost groups' thresholds and bucket costs
  int64_t costtab_cap = 0;     // bytes
  int32_t* d_candn = nullptr;  // [k] candidate degrees
};

struct bltc_selector_s {
  int32_t k = 0;
  std::vector<int32_t> cand_n;
  std::vector<double> cand_theta;
  double theta_ref = 0.7, margin = 0.0;
  double margin_global = 0.0;  // margin of the whole-run choice
  int32_t deg_min = 0;         // separation rule the candidates use
  double cost_far = 1.0, cost_row = 0.0, cost_clu = 0.0, cost_near = 1.0;
  std::vector<float> mean, stdv, params;
  float* d_params = nullptr;
  float* d_mean = nullptr;
  float* d_std = nullptr;
};
