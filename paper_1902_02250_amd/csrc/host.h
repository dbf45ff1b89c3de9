// Host-side internals shared by the units of the C ABI: error handling,
// device allocation and copies, library streams, argument checks, stage
// timing, and the sequencing helpers each unit offers the others.  Nothing
// here is part of the C ABI.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <exception>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "bltc.h"
#include "internal.h"

namespace bltc {
namespace api {

// ---- errors ------------------------------------------------------------------
// Records msg as the thread's last error and returns code.
int fail(int code, const std::string& msg);

// Thrown inside the library only; every entry point catches it.
struct HipError {
  int code;
  std::string msg;
};

void hipchk(hipError_t e, const char* what);

// Test hook: when positive, the n-th device allocation from now fails as if
// the device were out of memory (counted per process, then disarmed).
extern int g_fail_alloc_after;

// Runs f, turning every exception into a status and a message.
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(BLTC_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(BLTC_EDEVICE, e.what());
  } catch (...) {
    return fail(BLTC_EDEVICE, "unknown failure");
  }
}

// ---- device memory -----------------------------------------------------------
void* dalloc_bytes(size_t bytes);

template <typename T>
T* dalloc(size_t count) {
  return static_cast<T*>(dalloc_bytes(sizeof(T) * (count ? count : 1)));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Allocates p when it is still NULL.
template <typename T>
void ensure_alloc(T*& p, size_t count) {
  if (!p) p = dalloc<T>(count);
}

template <typename T>
void h2d(T* dst, const T* src, size_t count, hipStream_t s) {
  if (count)
    hipchk(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s),
           "hipMemcpyAsync H2D");
}

template <typename T>
void d2h(T* dst, const T* src, size_t count, hipStream_t s) {
  if (count)
    hipchk(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyDeviceToHost, s),
           "hipMemcpyAsync D2H");
}

void sync(hipStream_t s);

// Device buffers freed on scope exit unless released; owned by exactly one
// holder (no copies).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void reserve(size_t n) {
    if (n <= cap) return;
    dfree(p);
    cap = 0;   // a failed allocation leaves an empty buffer, never a stale capacity
    p = dalloc<T>(n);
    cap = n;
  }
  T* release() {
    T* q = p;
    p = nullptr;
    cap = 0;
    return q;
  }
  ~DevBuf() { dfree(p); }
};

// ---- streams and events ------------------------------------------------------
// Library-owned streams (default priority) for independent launches, per
// device, created on first use and kept for the life of the process.
constexpr int kSideStreams = 4;
hipStream_t side_stream(int i);

// Events without timing, destroyed with the holder.
struct Events {
  std::vector<hipEvent_t> ev;
  hipEvent_t make();
  ~Events();
};

// ---- argument checks ---------------------------------------------------------
bool device_ptr(const void* p);
inline int odim_of(int kernel) { return kernel == BLTC_ROTLET || kernel == BLTC_FULL ? 6 : 3; }
inline int wdim_of(int kernel) { return kernel == BLTC_FULL ? 6 : 3; }
bool valid_kernel(int k);
int check_points(const double* x, const double* y, const double* z, int64_t n,
                 const char* what);
int check_options(const bltc_options* o, int kernel);
int check_eval(int kernel, double eps, int degree, double theta);
// The common 1/(8 pi) and the rotlet's 1/2 (velocity) and 1/4 (angular
// velocity), applied once per target.
void kernel_scales(int kernel, double* su, double* sw);

// ---- stage timing ------------------------------------------------------------
// Records events around one stage on stream s while profiling is on.
struct StageTimer {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(int st, hipStream_t str);
  void stop();
};

// ---- sources (api_tree.cpp) --------------------------------------------------
void destroy_degree(bltc_degree_data& d);
void destroy_tree(bltc_tree t);
void destroy_targets(bltc_targets g);
// The cluster tree built on the device level by level; returns the
// tree-ordered coordinates [3][n] and the permutation in device memory.
void build_device_tree(const double* x, const double* y, const double* z, int64_t n,
                       int64_t leaf_max, hipStream_t s, bltc::HostTree& t, double** coords,
                       int32_t** perm);
void build_tree(const double* x, const double* y, const double* z, int64_t n,
                int64_t leaf_max, hipStream_t s, bltc_tree t);
void build_targets(const double* x, const double* y, const double* z, int64_t m, int32_t bs,
                   int32_t leaf, int64_t gmax, hipStream_t s, bltc_targets g);
void set_weights(bltc_tree t, const double* w, int wdim, hipStream_t s);
// The device node arrays of a tree, with its cut, for the walk kernels.
bltc::Nodes tree_nodes(bltc_tree t);
// Grid and modified weights of one degree, cached until the weights change.
void ensure_degree(bltc_tree t, int degree, hipStream_t s);
// Weights of degree d < n derived from those of degree n, cached under (d, n).
const bltc_degree_data& ensure_derived(bltc_tree t, int d, int n, hipStream_t s);

// ---- evaluation (api_eval.cpp) -----------------------------------------------
bltc::Rule make_rule(double theta, int degree, int deg_min);
bltc::ListArgs list_args(bltc_tree t, bltc_targets g, double theta, const double* theta_b,
                         bltc::ListSet& L);
// Device interaction lists of every batch (MAC theta, or theta_b[b]) into L;
// returns the list sizes (synchronises on s).
void build_lists(bltc_tree t, bltc_targets g, double theta, const double* theta_b,
                 bltc::ListSet& L, hipStream_t s, int64_t* np, int64_t* nd,
                 const bltc::Rule* rule = nullptr, const bltc::ListArgs* per_batch = nullptr);
using DegreeGroups = std::vector<std::pair<int, std::pair<const int32_t*, int64_t>>>;
void derive_used_degrees(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int rule_min,
                         const DegreeGroups& grp, hipStream_t s);
// Argument block of the particle-cluster kernel for the batches in bmap
// (all if NULL) with lists L and the modified weights of `degree`.
bltc::P2PArgs p2p_args(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int kernel,
                       double eps, int degree, const bltc_options& o, const int32_t* bmap,
                       int64_t nmap, double* out);
// slices > 1 (with spart of slices_bytes): each batch's lists in that many
// parts, summed in order by launch_slice_reduce after the launch.
void run_p2p(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int kernel, double eps,
             int degree, const bltc_options& o, const int32_t* bmap, int64_t nmap,
             double* out, hipStream_t s, const int4* split = nullptr, int64_t nsplit = 0,
             double* partial = nullptr, const int32_t* xstart = nullptr, int32_t xmax = 0,
             int slices = 1, double* spart = nullptr);
// Slices per batch of a launch over nb batches (wpb waves of 64 targets
// each, odim outputs): a launch of fewer waves than kSliceWaves (8 per SIMD)
// splits every batch's lists into that many parts, at most kMaxSlices, with
// partial sums of at most kSliceBytes.  A function of the launch's size and
// the kernel alone: the fixed and allocation-free evaluations of a targets
// handle slice alike (bit for bit equal); a degree group of the per-batch
// selection, launched alone, may take more slices than a full evaluation,
// which changes only the order of its FP64 sums.
constexpr int64_t kSliceWaves = 8192;
constexpr int kMaxSlices = 16;
constexpr int64_t kSliceBytes = int64_t(12) << 20;
inline int slices_for(int64_t nb, int wpb, int odim) {
  const int64_t w = nb * wpb;
  if (w <= 0 || w >= kSliceWaves) return 1;
  int64_t k = (kSliceWaves + w - 1) / w;
  k = std::min<int64_t>(k, kMaxSlices);
  k = std::min<int64_t>(k, kSliceBytes / (w * odim * 64 * (int64_t)sizeof(double)));
  return (int)std::max<int64_t>(k, 1);
}
inline int64_t slices_bytes(int64_t nb, int wpb, int odim, int slices) {
  return nb * wpb * slices * odim * 64 * (int64_t)sizeof(double);
}
// The slice partial-sum buffer of g, grown to at least `doubles`.
double* spart_reserve(bltc_targets g, int64_t doubles);
// The order of an evaluation launch's batches: by decreasing modelled work
// (see deal_batches in api_eval.cpp), dealt to the 8 XCDs in turn.  One
// group per launch: its degree and its batches (host ids, or NULL for all
// g->nb); group i's order goes to g->d_xmap + off[i] and its XCD ranges (in
// waves) to g->d_xstart + 9 i.  Reads the list counts back (synchronises).
struct DealGroup {
  int degree;
  const int32_t* ids;   // host, or NULL: batches 0 .. n-1
  int64_t n;
  int slices = 1;       // slices per batch of the group's launch
};
struct Dealt {
  int64_t off;          // in g->d_xmap
  int32_t xmax;         // longest XCD range in waves
};
std::vector<Dealt> deal_batches(bltc_targets g, const bltc::ListSet& L, hipStream_t s,
                                const std::vector<DealGroup>& groups);
void evaluate_tree(bltc_tree t, bltc_targets g, int kernel, double eps, int degree,
                   double theta, const bltc_options& o, double* out, hipStream_t s);
// The checks shared by the entry points that evaluate a built tree: handles,
// kernel and parameters, output pointer, weights of `degree` present.
int check_tree_eval(bltc_tree t, int64_t m, int kernel, double eps, int degree, double theta,
                    const bltc_options& o, const double* out);

}  // namespace api
}  // namespace bltc

// Device buffers that the cluster-cluster path (on the target tree) and the
// judge's repair pass (on the targets) keep between calls, grown on demand,
// so a repeated call allocates nothing.
struct bltc_dual_cache {
  bltc::api::DevBuf<int32_t> gnode, gbptr, gpptr, gpids, gdptr, gdids, giota, bptr, pptr, pids,
      dptr, dids, xptr, xgi, xnode;
  // the grid and target passes' batch orders and XCD ranges (in waves), and
  // their host copies (sources of the uploads)
  bltc::api::DevBuf<int32_t> gbmap, gxstart, tbmap, txstart;
  std::vector<int32_t> h_gbmap, h_gxstart, h_tbmap, h_txstart;
  // the device traversal's counts, offsets, slots and flags
  bltc::api::DevBuf<int32_t> leaves, ncc, ncp, ccptr, cpptr, flag, slot, npc, npp, xcnt, ovf;
  bltc::api::DevBuf<unsigned long long> work;
  bltc::api::DevBuf<uint32_t> mask;
  bltc::api::DevBuf<double4> bgeo, gbgeo;
  bltc::api::DevBuf<double> tgrid, g, gpts;
};
struct bltc_split_cache {
  bltc::api::DevBuf<int4> sl;
  bltc::api::DevBuf<int32_t> sptr;
  bltc::api::DevBuf<double> part;
};
