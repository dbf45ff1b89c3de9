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
constexpr int kStackMax = 512;       // depth-first stack of the list walk
constexpr int kUpwardChunk = 2048;   // particles per upward-pass work group

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

// Unit Chebyshev points of the 2nd kind, descending.
void cheb_points(int degree, double* t);

// ---- kernel launch arguments ----------------------------------------------
struct Nodes {                 // device node arrays
  const double4* geo;          // center xyz, radius
  const int2* range;           // particle range [begin, end) in tree order
  const int2* kids;            // first child, child count
  int64_t nn;
};

struct ListArgs {
  const double4* bgeo;         // batch center, radius
  int64_t nb;
  Nodes nodes;
  double theta;
  int32_t* pcnt;               // [nb] proxy count (count pass)
  int32_t* dcnt;               // [nb] direct count
  const int32_t* pptr;         // [nb+1] (fill pass)
  const int32_t* dptr;
  int32_t* pids;
  int32_t* dids;
  int32_t* err;                // set to 1 if a stack overflows
};

struct P2PArgs {
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
  const double* ys;            // tree-ordered sources [3][n]
  const double* w64;           // tree-ordered weights [3][n]
  const float* w32;
  int64_t n;
  double eps;
  int32_t poly_p;
  double poly_c;
  double scale_u, scale_w;     // constant factors applied at the end
  double* out;                 // [odim][m] caller order
};

// ---- launchers (defined in the .hip files) --------------------------------
hipError_t launch_gather_points(const double* x, const double* y,
                                const double* z, const int32_t* perm,
                                int64_t n, double* out3, hipStream_t s);
hipError_t launch_gather_weights(const double* w, const int32_t* perm,
                                 int64_t n, double* w64, float* w32,
                                 hipStream_t s);
hipError_t launch_grids(const double* box, int64_t nn, int degree,
                        const double* unit_nodes, double* grid, hipStream_t s);
hipError_t launch_upward(const double* ys, const double* w64, int64_t n,
                         const int4* chunks, int64_t nchunks,
                         const double* grid, int degree, double* partial,
                         hipStream_t s);
hipError_t launch_upward_reduce(const int32_t* chunk_ptr, int64_t nn,
                                const double* partial, int degree,
                                double* fhat64, double* p2p64, float* p2p32,
                                hipStream_t s);
hipError_t launch_lists(const ListArgs& a, bool fill, hipStream_t s);
hipError_t launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* out,
                                 int32_t* overflow, hipStream_t s);
hipError_t launch_p2p(int kernel, int precision, int degree,
                      const P2PArgs& a, hipStream_t s);
hipError_t launch_direct(int kernel, int precision, const double* tx,
                         const double* ty, const double* tz,
                         const int64_t* idx, int64_t k, const double* sx,
                         const double* sy, const double* sz, int64_t n,
                         const double* w, double eps, int32_t poly_p,
                         double poly_c, double scale_u, double scale_w,
                         double* out, hipStream_t s);

}  // namespace bltc

// ---- handles ----------------------------------------------------------------
struct bltc_degree_data {
  double* grid = nullptr;      // [nn][3][n1]
  double* fhat64 = nullptr;    // [nn][3][nk] (k3 fastest)
  double* p2p64 = nullptr;     // [nn][n1][n1][3][n1]
  float* p2p32 = nullptr;
};

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
  // weights
  bool has_w = false;
  double* d_w64 = nullptr;     // tree-ordered [3][n]
  float* d_w32 = nullptr;
  std::map<int, bltc_degree_data> deg;
  // upward-pass chunks
  int64_t nchunks = 0;
  int4* d_chunks = nullptr;    // node, begin, end, 0
  int32_t* d_chunk_ptr = nullptr;  // [nn+1]
  double* d_partial = nullptr;
  size_t partial_cap = 0;      // doubles
};

struct bltc_targets_s {
  int device = 0;
  int64_t m = 0, nb = 0;
  int32_t batch_size = 0, order_leaf = 0;
  int64_t group_max = 0;
  bltc::HostBatches host;
  int32_t* d_tperm = nullptr;
  double* d_x = nullptr;       // tree-ordered [3][m]
  int32_t* d_bptr = nullptr;
  double4* d_bgeo = nullptr;
  // interaction-list scratch, grown on demand
  int32_t* d_cnt = nullptr;    // [2][nb]
  int32_t* d_ptr = nullptr;    // [2][nb+1]
  int32_t* d_flags = nullptr;  // [4]: stack overflow, scan overflow
  int32_t* d_pids = nullptr;
  int32_t* d_dids = nullptr;
  int64_t pcap = 0, dcap = 0;
};
