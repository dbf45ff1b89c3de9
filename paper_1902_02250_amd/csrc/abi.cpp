// The C ABI of include/bltc.h: argument checks, handle management, host
// tree building and the sequencing of the device kernels on the caller's
// stream.  No exception crosses the boundary.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <utility>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "bltc.h"
#include "internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError {
  int code;
  std::string msg;
};

// Throws inside the library only; every entry point catches.
void hipchk(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? BLTC_ENOMEM : BLTC_EDEVICE;
  throw HipError{code, std::string(what) + ": " + hipGetErrorString(e)};
}

template <typename T>
T* dalloc(size_t count) {
  void* p = nullptr;
  hipchk(hipMalloc(&p, sizeof(T) * (count ? count : 1)), "hipMalloc");
  return static_cast<T*>(p);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
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

void sync(hipStream_t s) { hipchk(hipStreamSynchronize(s), "hipStreamSynchronize"); }

// Library-owned streams (default priority) for independent launches, per
// device, created on first use and kept for the life of the process.
constexpr int kSideStreams = 4;
std::mutex g_side_mu;
std::map<int, std::array<hipStream_t, kSideStreams>> g_side;

hipStream_t side_stream(int i) {
  int dev = 0;
  hipchk(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_side_mu);
  auto it = g_side.find(dev);
  if (it == g_side.end()) it = g_side.emplace(dev, std::array<hipStream_t, kSideStreams>{}).first;
  hipStream_t& st = it->second[i % kSideStreams];
  if (!st) hipchk(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
  return st;
}

// Events without timing, destroyed with the holder.
struct Events {
  std::vector<hipEvent_t> ev;
  hipEvent_t make() {
    hipEvent_t e;
    hipchk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    ev.push_back(e);
    return e;
  }
  ~Events() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// True if p points into device (or managed) memory that kernels may read.
bool device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

int odim_of(int kernel) { return kernel == BLTC_ROTLET || kernel == BLTC_FULL ? 6 : 3; }
int wdim_of(int kernel) { return kernel == BLTC_FULL ? 6 : 3; }

bool valid_kernel(int k) {
  return k == BLTC_STOKESLET || k == BLTC_ROTLET || k == BLTC_FULL || k == BLTC_POLY;
}

int check_points(const double* x, const double* y, const double* z,
                 int64_t n, const char* what) {
  if (n < 0 || n > 0x7fffffffLL)
    return fail(BLTC_EINVAL, std::string(what) + ": count out of range [0, 2^31)");
  if (n > 0 && (!x || !y || !z))
    return fail(BLTC_EINVAL, std::string(what) + ": NULL coordinate array");
  if (n > 0 && (!device_ptr(x) || !device_ptr(y) || !device_ptr(z)))
    return fail(BLTC_EINVAL, std::string(what) + ": coordinates must be device pointers");
  return BLTC_OK;
}

int check_options(const bltc_options* o, int kernel) {
  if (o->size != (int32_t)sizeof(bltc_options))
    return fail(BLTC_EINVAL, "bltc_options.size mismatch");
  if (o->precision < BLTC_FP64 || o->precision > BLTC_FP32_KAHAN)
    return fail(BLTC_EINVAL, "unknown precision");
  if (kernel == BLTC_POLY && o->precision != BLTC_FP64)
    return fail(BLTC_EINVAL, "the polynomial test kernel runs in FP64 only");
  if (o->batch_size < 1 || o->batch_size > 1024)
    return fail(BLTC_EINVAL, "batch_size must be in [1, 1024]");
  if (o->order_leaf < 1) return fail(BLTC_EINVAL, "order_leaf must be >= 1");
  if (o->group_max < 1) return fail(BLTC_EINVAL, "group_max must be >= 1");
  if (o->poly_p < 0 || o->poly_p > 64) return fail(BLTC_EINVAL, "poly_p must be in [0, 64]");
  if (o->deg_min < 0 || o->deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  return BLTC_OK;
}

int check_eval(int kernel, double eps, int degree, double theta) {
  if (!valid_kernel(kernel)) return fail(BLTC_EINVAL, "unknown kernel");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BLTC_EINVAL, "eps must be finite and >= 0");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  return BLTC_OK;
}

void kernel_scales(int kernel, double* su, double* sw) {
  const double c = 1.0 / (8.0 * 3.14159265358979323846);
  if (kernel == BLTC_STOKESLET || kernel == BLTC_FULL) { *su = c; *sw = c; }
  else if (kernel == BLTC_ROTLET) { *su = 0.5 * c; *sw = 0.25 * c; }
  else { *su = 1.0; *sw = 1.0; }
}

// ---- stage timing ------------------------------------------------------------
struct Profiler {
  bool on = false;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipchk(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
};
Profiler g_prof;

// Records events around one stage on stream s when profiling is on.
struct StageTimer {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(int st, hipStream_t str) : stage(st), s(str) {
    if (!g_prof.on) return;
    a = g_prof.get();
    hipchk(hipEventRecord(a, s), "hipEventRecord");
  }
  void stop() {
    if (!a) return;
    hipEvent_t b = g_prof.get();
    hipchk(hipEventRecord(b, s), "hipEventRecord");
    g_prof.marks.push_back({stage, a, b});
    a = nullptr;
  }
};

// ---- tree ---------------------------------------------------------------------
void destroy_degree(bltc_degree_data& d) {
  dfree(d.grid);
  dfree(d.fhat64);
  dfree(d.p2p64);
  dfree(d.p2p32);
}

void destroy_dual_cache(bltc_dual_cache* c);

void destroy_tree(bltc_tree t) {
  if (!t) return;
  for (auto& kv : t->deg) destroy_degree(kv.second);
  for (auto& kv : t->spare) destroy_degree(kv.second);
  for (auto& kv : t->derived) destroy_degree(kv.second);
  for (auto& kv : t->spare_derived) destroy_degree(kv.second);
  dfree(t->d_perm); dfree(t->d_y); dfree(t->d_box); dfree(t->d_geo);
  dfree(t->d_range); dfree(t->d_kids); dfree(t->d_skip); dfree(t->d_w64); dfree(t->d_w32);
  dfree(t->d_chunks); dfree(t->d_chunk_ptr); dfree(t->d_partial); dfree(t->d_parents);
  destroy_dual_cache(t->dual);
  delete t;
}

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

}  // namespace

// Device buffers that the cluster-cluster path (on the target tree) and the
// judge's repair pass (on the targets) keep between calls, grown on demand,
// so a repeated call allocates nothing.
struct bltc_dual_cache {
  DevBuf<int32_t> gnode, gbptr, gpptr, gpids, gdptr, gdids, giota, bptr, pptr, pids, dptr, dids,
      xptr, xgi, xnode;
  DevBuf<double4> bgeo, gbgeo;
  DevBuf<double> tgrid, g, gpts;
};
struct bltc_split_cache {
  DevBuf<int4> sl;
  DevBuf<int32_t> sptr;
  DevBuf<double> part;
};

namespace {

void destroy_dual_cache(bltc_dual_cache* c) { delete c; }

// The cluster tree built on the device, level by level (Section 6 rules, the
// same results as bltc::build_host_tree bit for bit).  The host keeps the
// node ranges and numbers the children breadth first from one histogram per
// chunk; boxes, centers and radii come back with it.  Returns the
// tree-ordered coordinates [3][n] and the permutation in device memory.
void build_device_tree(const double* x, const double* y, const double* z, int64_t n,
                       int64_t leaf_max, hipStream_t s, bltc::HostTree& t, double** coords,
                       int32_t** perm) {
  t = bltc::HostTree();
  t.n = n;
  DevBuf<double> ca, cb, cmm;
  DevBuf<int32_t> pa, pb, dcptr, dhist, dpos;
  DevBuf<int4> dchunks;
  DevBuf<int2> drange;
  DevBuf<bltc::TreeLevelNode> dnodes;
  ca.reserve(3 * n);
  pa.reserve(n);
  hipchk(bltc::launch_tree_init(x, y, z, n, ca.p, pa.p, s), "tree init");
  if (n > 0) {
    cb.reserve(3 * n);
    pb.reserve(n);
    auto add = [&](int32_t b, int32_t e, int32_t lev) {
      t.begin.push_back(b);
      t.end.push_back(e);
      t.level.push_back(lev);
      t.first.push_back(-1);
      t.count.push_back(0);
      if (lev > t.depth) t.depth = lev;
    };
    add(0, (int32_t)n, 0);
    std::vector<int4> chunks;
    std::vector<int32_t> cptr, hist, pos;
    std::vector<int2> range;
    std::vector<bltc::TreeLevelNode> nodes;
    size_t lev_begin = 0;
    while (lev_begin < t.begin.size()) {
      const size_t lev_end = t.begin.size();
      const int nl = (int)(lev_end - lev_begin);
      chunks.clear();
      cptr.resize(nl + 1);
      range.resize(nl);
      for (int k = 0; k < nl; ++k) {
        const size_t q = lev_begin + k;
        cptr[k] = (int32_t)chunks.size();
        range[k] = make_int2(t.begin[q], t.end[q]);
        for (int64_t b = t.begin[q]; b < t.end[q]; b += bltc::kTreeChunk)
          chunks.push_back(make_int4(k, (int)b, (int)std::min<int64_t>(t.end[q], b + bltc::kTreeChunk), 0));
      }
      cptr[nl] = (int32_t)chunks.size();
      const int64_t nch = (int64_t)chunks.size();
      dchunks.reserve(nch);
      dcptr.reserve(nl + 1);
      drange.reserve(nl);
      cmm.reserve(6 * nch);
      dnodes.reserve(nl);
      dhist.reserve(8 * nch);
      dpos.reserve(9 * nch);
      h2d(dchunks.p, chunks.data(), nch, s);
      h2d(dcptr.p, cptr.data(), nl + 1, s);
      h2d(drange.p, range.data(), nl, s);
      hipchk(bltc::launch_tree_level(dchunks.p, nch, dcptr.p, drange.p, nl, ca.p, n, leaf_max,
                                     cmm.p, dnodes.p, dhist.p, s), "tree level");
      hist.resize(8 * nch);
      nodes.resize(nl);
      d2h(hist.data(), dhist.p, 8 * nch, s);
      d2h(nodes.data(), dnodes.p, nl, s);
      sync(s);
      // split decisions, child offsets and per-chunk positions (stable)
      pos.assign(9 * nch, 0);
      bool any = false;
      std::vector<std::array<int32_t, 8>> off(nl), tot(nl);
      std::vector<char> split(nl, 0);
      for (int k = 0; k < nl; ++k) {
        const size_t q = lev_begin + k;
        const bltc::TreeLevelNode& o = nodes[k];   // box, center, radius, split axes
        for (int a = 0; a < 3; ++a) t.box.push_back(o.lo[a]);
        for (int a = 0; a < 3; ++a) t.box.push_back(o.hi[a]);
        for (int a = 0; a < 3; ++a) t.ctr.push_back(o.ctr[a]);
        t.rad.push_back(o.rad);
        tot[k].fill(0);
        for (int c = cptr[k]; c < cptr[k + 1]; ++c)
          for (int k8 = 0; k8 < 8; ++k8) tot[k][k8] += hist[8 * c + k8];
        int used = 0;
        for (int k8 = 0; k8 < 8; ++k8) used += tot[k][k8] != 0;
        split[k] = o.mask != 0 && used >= 2;
        if (!split[k]) {
          for (int c = cptr[k]; c < cptr[k + 1]; ++c) pos[9 * c] = chunks[c].y;
          continue;
        }
        any = true;
        int32_t acc = t.begin[q];
        for (int k8 = 0; k8 < 8; ++k8) {
          off[k][k8] = acc;
          acc += tot[k][k8];
        }
        for (int k8 = 0; k8 < 8; ++k8) {
          int32_t p = off[k][k8];
          for (int c = cptr[k]; c < cptr[k + 1]; ++c) {
            pos[9 * c + k8] = p;
            p += hist[8 * c + k8];
          }
        }
        for (int c = cptr[k]; c < cptr[k + 1]; ++c) pos[9 * c + 8] = 1;
      }
      if (any) {
        h2d(dpos.p, pos.data(), 9 * nch, s);
        hipchk(bltc::launch_tree_scatter(dchunks.p, nch, dpos.p, n, dnodes.p, ca.p, pa.p, cb.p,
                                         pb.p, s), "tree scatter");
      }
      for (int k = 0; k < nl; ++k) {
        if (!split[k]) continue;
        const size_t q = lev_begin + k;
        t.first[q] = (int32_t)t.begin.size();
        int nch8 = 0;
        for (int k8 = 0; k8 < 8; ++k8) {
          if (!tot[k][k8]) continue;
          add(off[k][k8], off[k][k8] + tot[k][k8], t.level[q] + 1);
          ++nch8;
        }
        t.count[q] = nch8;
      }
      lev_begin = lev_end;
    }
    t.perm.resize(n);
    d2h(t.perm.data(), pa.p, n, s);
    sync(s);
  }
  *coords = ca.release();
  *perm = pa.release();
}

void build_tree(const double* x, const double* y, const double* z, int64_t n,
                int64_t leaf_max, hipStream_t s, bltc_tree t) {
  build_device_tree(x, y, z, n, leaf_max, s, t->host, &t->d_y, &t->d_perm);
  const bltc::HostTree& H = t->host;
  const int64_t nn = H.nnodes();
  std::vector<double4> geo(nn);
  std::vector<int2> range(nn), kids(nn);
  for (int64_t q = 0; q < nn; ++q) {
    geo[q] = make_double4(H.ctr[3 * q], H.ctr[3 * q + 1], H.ctr[3 * q + 2], H.rad[q]);
    range[q] = make_int2(H.begin[q], H.end[q]);
    kids[q] = make_int2(H.first[q], H.count[q]);
  }
  // depth-first successor past each subtree: the next sibling, else the
  // parent's successor (nodes are numbered breadth first, parents first)
  std::vector<int32_t> skip(nn, -1);
  for (int64_t q = 0; q < nn; ++q)
    for (int32_t k = 0; k < H.count[q]; ++k)
      skip[H.first[q] + k] = k + 1 < H.count[q] ? H.first[q] + k + 1 : skip[q];
  // upward-pass chunks: consecutive pieces of each leaf's particle range
  std::vector<int4> chunks;
  std::vector<int32_t> cptr(nn + 1);
  for (int64_t q = 0; q < nn; ++q) {
    cptr[q] = (int32_t)chunks.size();
    if (H.count[q] > 0) continue;
    for (int32_t b = H.begin[q]; b < H.end[q]; b += bltc::kUpwardChunk)
      chunks.push_back(make_int4((int)q, b, std::min(H.end[q], b + bltc::kUpwardChunk), 0));
  }
  cptr[nn] = (int32_t)chunks.size();
  t->nchunks = (int64_t)chunks.size();
  // parents by level, deepest first: their children are done before them
  int32_t maxlev = 0;
  for (int64_t q = 0; q < nn; ++q) maxlev = std::max(maxlev, H.level[q]);
  std::vector<int32_t> parents;
  t->parent_levels.clear();
  for (int32_t l = maxlev; l >= 0; --l) {
    const int64_t off = (int64_t)parents.size();
    for (int64_t q = 0; q < nn; ++q)
      if (H.level[q] == l && H.count[q] > 0) parents.push_back((int32_t)q);
    if ((int64_t)parents.size() > off) t->parent_levels.push_back({off, (int64_t)parents.size() - off});
  }

  t->d_box = dalloc<double>(6 * nn);
  t->d_geo = dalloc<double4>(nn);
  t->d_range = dalloc<int2>(nn);
  t->d_kids = dalloc<int2>(nn);
  t->d_skip = dalloc<int32_t>(nn);
  t->d_chunks = dalloc<int4>(chunks.size());
  t->d_chunk_ptr = dalloc<int32_t>(nn + 1);
  if (!parents.empty()) t->d_parents = dalloc<int32_t>(parents.size());
  h2d(t->d_box, H.box.data(), 6 * nn, s);
  h2d(t->d_geo, geo.data(), nn, s);
  h2d(t->d_range, range.data(), nn, s);
  h2d(t->d_kids, kids.data(), nn, s);
  h2d(t->d_skip, skip.data(), nn, s);
  h2d(t->d_chunks, chunks.data(), chunks.size(), s);
  h2d(t->d_chunk_ptr, cptr.data(), nn + 1, s);
  if (!parents.empty()) h2d(t->d_parents, parents.data(), parents.size(), s);
  sync(s);   // the host staging vectors go out of scope
}

// Grid and modified weights of one degree from the stored tree-ordered
// weights, cached per degree until the weights change: the leaves from
// their particles, then the parents level by level from their children.
void ensure_degree(bltc_tree t, int degree, hipStream_t s) {
  if (t->deg.count(degree)) return;
  const int64_t nn = t->host.nnodes();
  const int n1 = degree + 1;
  const int64_t nk = (int64_t)n1 * n1 * n1;
  bltc_degree_data d;
  try {
    const int wd = t->wdim;
    const auto sp = t->spare.find(degree);
    if (sp != t->spare.end()) {   // buffers of a stale table of this degree
      d = sp->second;
      t->spare.erase(sp);
    } else {
      d.grid = dalloc<double>(nn * 3 * n1);
      d.fhat64 = dalloc<double>(nn * wd * nk);
      d.p2p64 = dalloc<double>(nn * wd * nk);
      d.p2p32 = dalloc<float>(nn * wd * nk);
    }
    double tk[bltc::kMaxDegree + 1];
    bltc::cheb_points(degree, tk);
    StageTimer prep(BLTC_STAGE_PREP, s);
    hipchk(bltc::launch_grids(t->d_box, nn, degree, tk, d.grid, s), "grids");
    prep.stop();
    const size_t want = (size_t)t->nchunks * wd * nk;
    if (want > t->partial_cap) {
      dfree(t->d_partial);
      t->d_partial = dalloc<double>(want);
      t->partial_cap = want;
    }
    StageTimer up(BLTC_STAGE_UPWARD, s);
    hipchk(bltc::launch_upward(t->d_y, t->d_w64, t->n, wd, t->d_chunks,
                               t->nchunks, d.grid, degree, t->d_partial, s),
           "upward");
    hipchk(bltc::launch_upward_reduce(t->d_chunk_ptr, nn, t->d_partial, degree, wd,
                                      d.fhat64, d.p2p64, d.p2p32, s),
           "upward reduce");
    for (const auto& lv : t->parent_levels)
      hipchk(bltc::launch_m2m(t->d_parents + lv.first, lv.second, t->d_kids, degree, wd, d.grid,
                              d.fhat64, d.p2p64, d.p2p32, s),
             "upward transfer");
    up.stop();
  } catch (...) {
    destroy_degree(d);
    throw;
  }
  t->deg[degree] = d;
}

// L^d_k(t^n_m) on the reference Chebyshev nodes, in barycentric form with
// the exact-hit rule of Algorithm 1.
void restrict_matrix(int d, int n, double* R) {
  double td[bltc::kMaxDegree + 1], tn[bltc::kMaxDegree + 1];
  bltc::cheb_points(d, td);
  bltc::cheb_points(n, tn);
  for (int m = 0; m <= n; ++m) {
    double L[bltc::kMaxDegree + 1], sum = 0.0;
    int flag = -1;
    for (int k = 0; k <= d; ++k) {
      const double wk = (k == 0 || k == d) ? ((k & 1) ? -0.5 : 0.5) : ((k & 1) ? -1.0 : 1.0);
      const double diff = tn[m] - td[k];
      if (std::fabs(diff) <= DBL_MIN) {
        flag = k;
        L[k] = 0.0;
      } else {
        L[k] = wk / diff;
        sum += L[k];
      }
    }
    for (int k = 0; k <= d; ++k)
      R[k * (n + 1) + m] = flag >= 0 ? (k == flag ? 1.0 : 0.0) : L[k] / sum;
  }
}

// Weights of degree d < n derived from those of degree n (which must
// exist), cached under (d, n) until the weights change.  Lower degrees of
// the separation rule take these, so a batch's result depends only on its
// own top degree n, whichever other degrees a call uses.
const bltc_degree_data& ensure_derived(bltc_tree t, int d, int n, hipStream_t s) {
  if (d == n) return t->deg.at(n);
  const auto key = std::make_pair(d, n);
  auto it = t->derived.find(key);
  if (it != t->derived.end()) return it->second;
  const bltc_degree_data& src = t->deg.at(n);
  const int64_t nn = t->host.nnodes();
  const int d1 = d + 1;
  const int64_t nk = (int64_t)d1 * d1 * d1;
  bltc_degree_data e;
  try {
    const int wd = t->wdim;
    const auto sp = t->spare_derived.find(key);
    if (sp != t->spare_derived.end()) {
      e = sp->second;
      t->spare_derived.erase(sp);
    } else {
      e.grid = dalloc<double>(nn * 3 * d1);
      e.fhat64 = dalloc<double>(nn * wd * nk);
      e.p2p64 = dalloc<double>(nn * wd * nk);
      e.p2p32 = dalloc<float>(nn * wd * nk);
    }
    double tk[bltc::kMaxDegree + 1];
    bltc::cheb_points(d, tk);
    StageTimer up(BLTC_STAGE_UPWARD, s);
    hipchk(bltc::launch_grids(t->d_box, nn, d, tk, e.grid, s), "grids");
    bltc::RestrictArgs ra;
    ra.d1 = d1;
    ra.n1 = n + 1;
    restrict_matrix(d, n, ra.R);
    hipchk(bltc::launch_restrict(ra, nn, wd, src.fhat64, e.fhat64, e.p2p64, e.p2p32, s),
           "restrict");
    up.stop();
  } catch (...) {
    destroy_degree(e);
    throw;
  }
  return t->derived[key] = e;
}

void set_weights(bltc_tree t, const double* w, int wdim, hipStream_t s) {
  // the cached tables go stale; their buffers are kept for the next tables
  // of the same degree and width (no free or allocation per call)
  for (auto& kv : t->deg) {
    auto it = t->spare.find(kv.first);
    if (it != t->spare.end()) destroy_degree(it->second);
    t->spare[kv.first] = kv.second;
  }
  t->deg.clear();
  for (auto& kv : t->derived) {
    auto it = t->spare_derived.find(kv.first);
    if (it != t->spare_derived.end()) destroy_degree(it->second);
    t->spare_derived[kv.first] = kv.second;
  }
  t->derived.clear();
  t->has_w = false;
  if (t->wdim != wdim) {
    for (auto& kv : t->spare) destroy_degree(kv.second);
    t->spare.clear();
    for (auto& kv : t->spare_derived) destroy_degree(kv.second);
    t->spare_derived.clear();
  }
  if (t->d_w64 && t->wdim != wdim) {
    dfree(t->d_w64);
    dfree(t->d_w32);
    t->d_w64 = nullptr;
    t->d_w32 = nullptr;
  }
  t->wdim = wdim;
  if (!t->d_w64) {
    t->d_w64 = dalloc<double>(wdim * t->n);
    t->d_w32 = dalloc<float>(wdim * t->n);
  }
  StageTimer prep(BLTC_STAGE_PREP, s);
  hipchk(bltc::launch_gather_weights(w, t->d_perm, t->n, wdim, t->d_w64, t->d_w32, s),
         "gather weights");
  prep.stop();
  t->has_w = true;
}

// ---- targets -----------------------------------------------------------------
void destroy_targets(bltc_targets g) {
  if (!g) return;
  dfree(g->d_tperm); dfree(g->d_x); dfree(g->d_bptr); dfree(g->d_bgeo);
  dfree(g->d_flags);
  for (auto& L : g->ls) {
    dfree(L.cnt); dfree(L.ptr); dfree(L.pids); dfree(L.dids);
  }
  dfree(g->d_feat); dfree(g->d_Y); dfree(g->d_pc); dfree(g->d_sc);
  dfree(g->d_choice); dfree(g->d_bmap); dfree(g->d_theta_b); dfree(g->d_spos);
  dfree(g->d_sbatch); dfree(g->d_gflag); dfree(g->d_ufb);
  dfree(g->d_wt); dfree(g->d_usq); dfree(g->d_contrib); dfree(g->d_part); dfree(g->d_sums); dfree(g->d_lam);
  dfree(g->d_cost); dfree(g->d_e2); dfree(g->d_candT); dfree(g->d_candn);
  delete g->split;
  dfree(g->d_dmask);
  delete g;
}

void build_targets(const double* x, const double* y, const double* z,
                   int64_t m, int32_t bs, int32_t leaf, int64_t gmax,
                   hipStream_t s, bltc_targets g) {
  // the order tree on the device; groups and batch bounds on the host;
  // batch geometry on the device
  bltc::HostTree order;
  build_device_tree(x, y, z, m, leaf, s, order, &g->d_x, &g->d_tperm);
  bltc::HostBatches& B = g->host;
  B = bltc::HostBatches();
  B.perm.swap(order.perm);
  std::vector<int32_t> bend;
  bltc::batch_bounds(order, bs, gmax, B.bptr, bend);
  g->m = m;
  g->nb = (int64_t)B.bptr.size() - 1;
  g->batch_size = bs;
  g->order_leaf = leaf;
  g->group_max = gmax;
  const int64_t nb = g->nb;
  g->d_bptr = dalloc<int32_t>(nb + 1);
  g->d_bgeo = dalloc<double4>(nb);
  for (auto& L : g->ls) {
    L.cnt = dalloc<int32_t>(3 * nb);
    L.ptr = dalloc<int32_t>(2 * (nb + 1));
  }
  g->d_flags = dalloc<int32_t>(4);
  g->d_dmask = dalloc<uint32_t>(bltc::kMaxDegree + 1);
  h2d(g->d_bptr, B.bptr.data(), nb + 1, s);
  {
    int32_t* d_bend = dalloc<int32_t>(nb);
    try {
      h2d(d_bend, bend.data(), nb, s);
      hipchk(bltc::launch_batch_geo(g->d_x, m, g->d_bptr, d_bend, nb, g->d_bgeo, s),
             "batch geometry");
      B.geo.resize(4 * nb);
      d2h(reinterpret_cast<double4*>(B.geo.data()), g->d_bgeo, nb, s);
      sync(s);
    } catch (...) {
      dfree(d_bend);
      throw;
    }
    dfree(d_bend);
  }
  const int32_t zero[4] = {0, 0, 0, 0};
  h2d(g->d_flags, zero, 4, s);
  sync(s);
}

// Separation-rule thresholds for evaluation degree n and MAC theta: for d in
// [deg_min, n), T[d] = (2k / (1 + k^2))^2 with k = kappa(theta)^((n+1)/(d+1)),
// kappa(r) = r / (1 + sqrt(1 - r^2)); a cluster at ratio rho takes the first
// d with rho^2 <= T[d].  deg_min outside [1, n) turns the rule off.
bltc::Rule make_rule(double theta, int degree, int deg_min) {
  bltc::Rule r;
  if (deg_min < 1 || deg_min >= degree) return r;
  r.deg_min = deg_min;
  r.degree = degree;
  const double kt = theta / (1.0 + std::sqrt(1.0 - theta * theta));
  for (int d = deg_min; d < degree; ++d) {
    const double k = std::pow(kt, (double)(degree + 1) / (double)(d + 1));
    const double rho = (2.0 * k) / (1.0 + k * k);
    r.T[d] = rho * rho;
  }
  return r;
}

bltc::ListArgs list_args(bltc_tree t, bltc_targets g, double theta,
                         const double* theta_b, bltc::ListSet& L) {
  const int64_t nb = g->nb;
  bltc::ListArgs a;
  a.bgeo = g->d_bgeo;
  a.nb = nb;
  a.nodes.geo = t->d_geo;
  a.nodes.range = t->d_range;
  a.nodes.kids = t->d_kids;
  a.nodes.skip = t->d_skip;
  a.nodes.nn = t->host.nnodes();
  a.theta = theta;
  a.theta_b = theta_b;
  a.pcnt = L.cnt;
  a.dcnt = L.cnt + nb;
  a.scnt = L.cnt + 2 * nb;
  a.pptr = L.ptr;
  a.dptr = L.ptr + nb + 1;
  a.pids = nullptr;
  a.dids = nullptr;
  a.err = g->d_flags;
  return a;
}

// Device interaction lists of every batch (MAC theta, or theta_b[b] when
// theta_b is given) into L; returns the list sizes.
void build_lists(bltc_tree t, bltc_targets g, double theta, const double* theta_b,
                 bltc::ListSet& L, hipStream_t s, int64_t* np, int64_t* nd,
                 const bltc::Rule* rule = nullptr, const bltc::ListArgs* per_batch = nullptr) {
  const int64_t nb = g->nb;
  bltc::ListArgs a = list_args(t, g, theta, theta_b, L);
  const bool on = (rule && rule->deg_min > 0) || (per_batch && per_batch->rule_deg_min > 0);
  if (on && t->host.nnodes() > bltc::kIdMask)
    throw HipError{BLTC_EINVAL, "the separation rule supports at most 2^27 - 1 clusters"};
  if (rule) a.rule = *rule;
  if (per_batch) {
    a.choice = per_batch->choice;
    a.cand_T = per_batch->cand_T;
    a.cand_deg = per_batch->cand_deg;
    a.rule_deg_min = per_batch->rule_deg_min;
  }
  StageTimer lt(BLTC_STAGE_LISTS, s);
  hipchk(bltc::launch_lists(a, false, s), "list count");
  hipchk(bltc::launch_exclusive_scan(a.pcnt, nb, L.ptr, g->d_flags + 1, s), "scan");
  hipchk(bltc::launch_exclusive_scan(a.dcnt, nb, L.ptr + nb + 1, g->d_flags + 2, s), "scan");
  int32_t tot[2], flags[4];
  d2h(&tot[0], L.ptr + nb, 1, s);
  d2h(&tot[1], L.ptr + 2 * nb + 1, 1, s);
  d2h(flags, g->d_flags, 4, s);
  sync(s);
  if (flags[0] || flags[1] || flags[2])
    throw HipError{BLTC_EDEVICE, "interaction lists overflowed"};
  if (tot[0] > L.pcap) {
    dfree(L.pids);
    L.pids = dalloc<int32_t>(tot[0]);
    L.pcap = tot[0];
  }
  if (tot[1] > L.dcap) {
    dfree(L.dids);
    L.dids = dalloc<int32_t>(tot[1]);
    L.dcap = tot[1];
  }
  a.pids = L.pids;
  a.dids = L.dids;
  hipchk(bltc::launch_lists(a, true, s), "list fill");
  lt.stop();
  *np = tot[0];
  *nd = tot[1];
}

// The separation rule's lower degrees that each evaluation group uses, derived
// from the group's top degree: groups (top degree, batches bsel[0..count)),
// bsel NULL for all batches.
void derive_used_degrees(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int rule_min,
                         const std::vector<std::pair<int, std::pair<const int32_t*, int64_t>>>& grp,
                         hipStream_t s) {
  if (rule_min <= 0 || grp.empty()) return;
  for (size_t i = 0; i < grp.size(); ++i)
    hipchk(bltc::launch_degree_mask(grp[i].second.first, grp[i].second.second, L.ptr, L.pids,
                                    g->d_dmask + i, s),
           "degree mask");
  std::vector<uint32_t> mask(grp.size());
  d2h(mask.data(), g->d_dmask, grp.size(), s);
  sync(s);
  for (size_t i = 0; i < grp.size(); ++i)
    for (int dd = rule_min; dd < grp[i].first; ++dd)
      if (mask[i] >> dd & 1u) ensure_derived(t, dd, grp[i].first, s);
}

// The particle-cluster evaluation of the batches in bmap (all if NULL) with
// lists L and the modified weights of `degree`.
void run_p2p(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int kernel,
             double eps, int degree, const bltc_options& o, const int32_t* bmap,
             int64_t nmap, double* out, hipStream_t s, const int4* split = nullptr,
             int64_t nsplit = 0, double* partial = nullptr) {
  const bltc_degree_data& d = t->deg.at(degree);
  bltc::P2PArgs a;
  a.split = split;
  a.nsplit = nsplit;
  a.partial = partial;
  a.bmap = bmap;
  a.nmap = nmap;
  a.tx = g->d_x;
  a.m = g->m;
  a.tperm = g->d_tperm;
  a.bptr = g->d_bptr;
  a.bgeo = g->d_bgeo;
  a.nb = g->nb;
  a.wpb = (g->batch_size + bltc::kWave - 1) / bltc::kWave;
  a.pptr = L.ptr;
  a.pids = L.pids;
  a.dptr = L.ptr + g->nb + 1;
  a.dids = L.dids;
  a.range = t->d_range;
  a.grid = d.grid;
  a.fhat = o.precision == BLTC_FP64 ? (const void*)d.p2p64 : (const void*)d.p2p32;
  if (o.deg_min >= 1 && o.deg_min < degree) {
    for (int dd = o.deg_min; dd <= degree; ++dd) {   // lower degrees derived from the top
      const bltc_degree_data* e = &d;
      if (dd < degree) {
        const auto it = t->derived.find({dd, degree});
        if (it == t->derived.end()) continue;   // a degree no list entry carries
        e = &it->second;
      }
      a.grid_d[dd] = e->grid;
      a.fhat_d[dd] = o.precision == BLTC_FP64 ? (const void*)e->p2p64 : (const void*)e->p2p32;
    }
  }
  a.ys = t->d_y;
  a.w64 = t->d_w64;
  a.w32 = t->d_w32;
  a.n = t->n;
  a.eps = eps;
  a.poly_p = o.poly_p;
  a.poly_c = o.poly_c;
  kernel_scales(kernel, &a.scale_u, &a.scale_w);
  a.out = out;
  StageTimer ev(BLTC_STAGE_EVAL, s);
  hipchk(bltc::launch_p2p(kernel, o.precision, degree, a, s), "p2p");
  ev.stop();
}

void evaluate_tree(bltc_tree t, bltc_targets g, int kernel, double eps,
                   int degree, double theta, const bltc_options& o,
                   double* out, hipStream_t s) {
  if (g->m == 0) return;
  ensure_degree(t, degree, s);
  int64_t np = 0, nd = 0;
  const bltc::Rule rule = make_rule(theta, degree, o.deg_min);
  build_lists(t, g, theta, nullptr, g->ls[0], s, &np, &nd, &rule);
  derive_used_degrees(t, g, g->ls[0], rule.deg_min, {{degree, {nullptr, g->nb}}}, s);
  run_p2p(t, g, g->ls[0], kernel, eps, degree, o, nullptr, 0, out, s);
}

// ---- learned (n, theta) per batch -------------------------------------------
void compute_features(bltc_tree t, bltc_targets g, int kernel, double eps,
                      double theta_ref, const float* mean, const float* stdv,
                      float* feat, hipStream_t s) {
  bltc::FeatArgs a;
  a.bgeo = g->d_bgeo;
  a.bptr = g->d_bptr;
  a.nb = g->nb;
  a.nodes.geo = t->d_geo;
  a.nodes.range = t->d_range;
  a.nodes.kids = t->d_kids;
  a.nodes.skip = t->d_skip;
  a.nodes.nn = t->host.nnodes();
  a.box = t->d_box;
  a.theta_ref = theta_ref;
  a.eps = eps;
  a.kernel = kernel;
  a.n_src = t->n;
  a.mean = mean;
  a.stdv = stdv;
  a.feat = feat;
  hipchk(bltc::launch_features(a, s), "features");
}

// Per-batch proxy-cluster and near-source counts of the walk at theta.
void batch_counts(bltc_tree t, bltc_targets g, double theta, int32_t* pc,
                  int32_t* sc, hipStream_t s) {
  bltc::ListSet& L = g->ls[1];
  bltc::ListArgs a = list_args(t, g, theta, nullptr, L);
  a.pcnt = pc;
  a.scnt = sc;
  hipchk(bltc::launch_lists(a, false, s), "list count");
}

constexpr int kLamGrid = 64;   // multipliers per allocation pass

// Modelled wave cost of every batch under each of the k candidates
// (cand_n[j], cand_theta[j]) into cost[j][nb] (device), with the separation
// rule when deg_min >= 1: one walk per distinct theta.
void candidate_costs(bltc_tree t, bltc_targets g, int k, const int32_t* cand_n,
                     const double* cand_theta, int deg_min, const bltc::Costs& w,
                     float* cost, hipStream_t s) {
  // the rule's thresholds of every candidate, [k][kMaxDegree + 1], on the device
  if (!g->d_candT) {
    g->d_candT = dalloc<double>((size_t)bltc::kMlpMaxOut * (bltc::kMaxDegree + 1));
    g->d_candn = dalloc<int32_t>(bltc::kMlpMaxOut);
  }
  std::vector<double> T((size_t)k * (bltc::kMaxDegree + 1));
  for (int j = 0; j < k; ++j) {
    const bltc::Rule r = make_rule(cand_theta[j], cand_n[j], deg_min);
    for (int d = 0; d <= bltc::kMaxDegree; ++d) T[(size_t)j * (bltc::kMaxDegree + 1) + d] = r.T[d];
  }
  h2d(g->d_candT, T.data(), T.size(), s);
  h2d(g->d_candn, cand_n, k, s);
  // candidates grouped by theta (at most kMaxPerTheta per group), up to
  // kMaxThetaGroups groups per launch
  std::vector<bltc::CostGroup> groups;
  std::vector<bool> done(k, false);
  for (int j0 = 0; j0 < k; ++j0) {
    if (done[j0]) continue;
    bltc::CostGroup gr;
    std::memset(&gr, 0, sizeof gr);
    gr.theta = cand_theta[j0];
    for (int j = j0; j < k && gr.nc < bltc::kMaxPerTheta; ++j) {
      if (done[j] || cand_theta[j] != cand_theta[j0]) continue;
      done[j] = true;
      gr.deg[gr.nc] = cand_n[j];
      gr.row[gr.nc] = j;
      ++gr.nc;
    }
    groups.push_back(gr);
  }
  for (size_t g0 = 0; g0 < groups.size(); g0 += bltc::kMaxThetaGroups) {
    bltc::CostArgs a;
    std::memset(&a, 0, sizeof a);
    a.bgeo = g->d_bgeo;
    a.nb = g->nb;
    a.nodes.geo = t->d_geo;
    a.nodes.range = t->d_range;
    a.nodes.kids = t->d_kids;
  a.nodes.skip = t->d_skip;
    a.nodes.nn = t->host.nnodes();
    a.ngroups = (int32_t)std::min<size_t>(bltc::kMaxThetaGroups, groups.size() - g0);
    for (int i = 0; i < a.ngroups; ++i) a.grp[i] = groups[g0 + i];
    a.deg_min = deg_min;
    a.T = g->d_candT;
    a.w = w;
    a.cost = cost;
    a.err = g->d_flags;
    hipchk(bltc::launch_cand_costs(a, s), "candidate costs");
  }
}

void ensure_selection_scratch(bltc_targets g, int64_t k, int64_t nth) {
  const int64_t nb = g->nb;
  if (!g->d_feat) {
    g->d_feat = dalloc<float>(nb * bltc::kMlpIn);
    g->d_choice = dalloc<int32_t>(nb);
    g->d_bmap = dalloc<int32_t>(nb);
    g->d_theta_b = dalloc<double>(nb);
    g->d_gflag = dalloc<int32_t>(nb);
    g->d_ufb = dalloc<double>(6 * nb);
    g->d_wt = dalloc<double>(nb);
    g->d_contrib = dalloc<double>(nb);
    g->d_part = dalloc<double>(bltc::alloc_blocks(nb) * kLamGrid * 2);
    g->d_sums = dalloc<double>(2 * std::max(kLamGrid, bltc::kMlpMaxOut));
    g->d_lam = dalloc<double>(kLamGrid);
    // one judge sample per kJudgeStride batches, at a hashed position inside
    // the first batch of its group
    const int64_t ns = (nb + bltc::kJudgeStride - 1) / bltc::kJudgeStride;
    g->nsamp = (int32_t)ns;
    g->d_usq = dalloc<double>(ns);
    std::vector<int32_t> sp(ns), sb(ns);
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t b = i * bltc::kJudgeStride;
      const int32_t b0 = g->host.bptr[b], cnt = g->host.bptr[b + 1] - b0;
      const uint32_t h = (uint32_t)(b * 2654435761ull >> 7);
      sp[i] = b0 + (int32_t)(h % (uint32_t)cnt);
      sb[i] = (int32_t)b;
    }
    g->d_spos = dalloc<int32_t>(ns);
    g->d_sbatch = dalloc<int32_t>(ns);
    h2d(g->d_spos, sp.data(), ns, nullptr);
    h2d(g->d_sbatch, sb.data(), ns, nullptr);
    sync(nullptr);
  }
  if (nb * k > g->ycap) {
    dfree(g->d_Y);
    g->d_Y = dalloc<float>(nb * k);
    g->ycap = nb * k;
  }
  if (nb * k > g->costcap) {
    dfree(g->d_cost);
    dfree(g->d_e2);
    g->d_cost = dalloc<float>(nb * k);
    g->d_e2 = dalloc<double>(nb * k);
    g->costcap = nb * k;
  }
  if (!g->d_candT) {
    g->d_candT = dalloc<double>((size_t)bltc::kMlpMaxOut * (bltc::kMaxDegree + 1));
    g->d_candn = dalloc<int32_t>(bltc::kMlpMaxOut);
  }
  (void)nth;
}

// Judge sums (sum of cnt |u_fb|^2, sum of cnt |u - u_fb|^2) over the one
// sample per batch; `out` NULL gives the weights only.
void judge_sums(bltc_targets g, int kernel, const double* out, double sums[2],
                hipStream_t s) {
  hipchk(bltc::launch_judge(g->nsamp, bltc::kJudgeStride, g->nb, g->d_bptr, g->d_spos,
                            g->d_tperm, out, g->m, odim_of(kernel), g->d_ufb, g->d_usq,
                            g->d_contrib, g->d_part, g->d_sums, s),
         "judge");
  d2h(sums, g->d_sums, 2, s);
  sync(s);
}

// Evaluation with (n, theta) chosen per batch (see bltc_evaluate_adaptive).
// ---- cluster-cluster variant -------------------------------------------------
// Dual traversal of the target tree T and the source tree S (the target
// variable is interpolated too, Section 9).  For a pair (A, C):
//   MAC (R2 > 0 and (r_A + r_C)^2 <= theta^2 R2): CC if both hold more than
//   P = (n+1)^3 particles, PC if only C does, CP if only A does, else PP;
//   no MAC and both leaves: PP; otherwise refine A if C is a leaf or
//   (A is not a leaf and r_A >= r_C), else refine C.
struct DualPlan {
  std::vector<std::vector<int32_t>> cc, cp, pc, pp;   // source nodes, by target node
  int64_t cnt[5] = {0, 0, 0, 0, 0};                    // CC, PC, CP, PP evaluations, downward terms
};

void dual_traverse(const bltc::HostTree& T, const bltc::HostTree& S, int n1, double theta,
                   const bltc::Rule& rule, DualPlan& D) {
  const int64_t ntn = T.nnodes();
  D.cc.assign(ntn, {});
  D.cp.assign(ntn, {});
  D.pc.assign(ntn, {});
  D.pp.assign(ntn, {});
  if (T.n == 0 || S.n == 0) return;
  const int64_t P = (int64_t)n1 * n1 * n1;
  std::vector<std::pair<int32_t, int32_t>> st{{0, 0}};
  while (!st.empty()) {
    const int32_t A = st.back().first, C = st.back().second;
    st.pop_back();
    const int64_t na = T.end[A] - T.begin[A], nc = S.end[C] - S.begin[C];
    const double dx = T.ctr[3 * A] - S.ctr[3 * C];
    const double dy = T.ctr[3 * A + 1] - S.ctr[3 * C + 1];
    const double dz = T.ctr[3 * A + 2] - S.ctr[3 * C + 2];
    const double R2 = dx * dx + dy * dy + dz * dz;
    const double rr = T.rad[A] + S.rad[C];
    const bool mac = R2 > 0.0 && rr * rr <= (theta * theta) * R2;
    const bool leafA = T.count[A] == 0, leafC = S.count[C] == 0;
    // the source side's degree under the separation rule (n - 1 when off):
    // the entry carries it above kDegShift
    int d = n1 - 1;
    if (mac && rule.deg_min > 0) {
      const double qq = (rr * rr) / R2;
      d = rule.deg_min;
      while (d < rule.degree && !(qq <= rule.T[d])) ++d;
    }
    const int64_t Pd = (int64_t)(d + 1) * (d + 1) * (d + 1);
    const int32_t e = rule.deg_min > 0 ? (C | (d << bltc::kDegShift)) : C;
    if (mac && na > P && nc > P) {
      D.cc[A].push_back(e);
      D.cnt[0] += P * Pd;
    } else if (mac && nc > P) {
      D.pc[A].push_back(e);
      D.cnt[1] += na * Pd;
    } else if (mac && na > P) {
      D.cp[A].push_back(C);
      D.cnt[2] += P * nc;
    } else if (mac || (leafA && leafC)) {
      D.pp[A].push_back(C);
      D.cnt[3] += na * nc;
    } else if (leafC || (!leafA && T.rad[A] >= S.rad[C])) {
      for (int32_t k = T.count[A] - 1; k >= 0; --k) st.push_back({T.first[A] + k, C});
    } else {
      for (int32_t k = S.count[C] - 1; k >= 0; --k) st.push_back({A, S.first[C] + k});
    }
  }
}

void evaluate_dual(bltc_tree src, bltc_tree tgt, int kernel, double eps, int degree,
                   double theta, const bltc_options& o, double* out, int64_t* counts,
                   hipStream_t s) {
  const bltc::HostTree& T = tgt->host;
  const bltc::HostTree& S = src->host;
  const int64_t m = tgt->n, ntn = T.nnodes();
  if (m == 0) return;
  ensure_degree(src, degree, s);
  const bltc_degree_data& d = src->deg.at(degree);
  const int n1 = degree + 1;
  const int64_t P = (int64_t)n1 * n1 * n1;
  const int odim = odim_of(kernel);

  StageTimer lt(BLTC_STAGE_LISTS, s);
  DualPlan D;
  const bltc::Rule rule = make_rule(theta, degree, o.deg_min);
  if (rule.deg_min > 0 && S.nnodes() > bltc::kIdMask)
    throw HipError{BLTC_EINVAL, "too many source clusters for the separation rule's encoding"};
  dual_traverse(T, S, n1, theta, rule, D);
  // grid slots: target clusters with CC or CP work
  // (their grid points are evaluated as targets, one batch per cluster run
  // by several waves: CC clusters on the proxy list, CP clusters on the
  // direct list)
  std::vector<int32_t> slot(ntn, -1), gnode;
  std::vector<int32_t> gbptr, gpptr{0}, gpids, gdptr{0}, gdids;
  std::vector<double4> gbgeo;
  for (int64_t A = 0; A < ntn; ++A) {
    if (D.cc[A].empty() && D.cp[A].empty()) continue;
    const int32_t gi = (int32_t)gnode.size();
    slot[A] = gi;
    gnode.push_back((int32_t)A);
    gbptr.push_back((int32_t)(gi * P));
    gbgeo.push_back(make_double4(T.ctr[3 * A], T.ctr[3 * A + 1], T.ctr[3 * A + 2], T.rad[A]));
    gpids.insert(gpids.end(), D.cc[A].begin(), D.cc[A].end());
    gpptr.push_back((int32_t)gpids.size());
    gdids.insert(gdids.end(), D.cp[A].begin(), D.cp[A].end());
    gdptr.push_back((int32_t)gdids.size());
    D.cnt[4] += (int64_t)(T.end[A] - T.begin[A]) * P;
  }
  const int64_t ng = (int64_t)gnode.size(), M = ng * P, gnb = (int64_t)gbgeo.size();
  if (M > (int64_t)INT32_MAX || gpids.size() > (size_t)INT32_MAX)
    throw HipError{BLTC_EINVAL, "cluster-cluster grid pass exceeds 2^31 entries"};
  gbptr.push_back((int32_t)M);
  std::vector<int32_t> giota(M);
  std::iota(giota.begin(), giota.end(), 0);
  // one batch per target leaf (run by several waves of 64 targets), leaves
  // in position order; it takes the PC and PP entries and the grid slots of
  // the leaf and all its ancestors
  std::vector<int32_t> parent(ntn, -1), leaves;
  for (int64_t q = 0; q < ntn; ++q) {
    for (int32_t k = 0; k < T.count[q]; ++k) parent[T.first[q] + k] = (int32_t)q;
    if (T.count[q] == 0) leaves.push_back((int32_t)q);
  }
  std::sort(leaves.begin(), leaves.end(),
            [&](int32_t a, int32_t b) { return T.begin[a] < T.begin[b]; });
  std::vector<int32_t> bptr, pptr{0}, pids, dptr{0}, dids, xptr{0}, xgi, xnode, path;
  std::vector<double4> bgeo;
  std::vector<int32_t> lpc, lpp, lgi, lnode;
  int64_t lmax = 1;
  for (int32_t L : leaves) {
    path.clear();
    for (int32_t q = L; q >= 0; q = parent[q]) path.push_back(q);
    std::reverse(path.begin(), path.end());
    lpc.clear();
    lpp.clear();
    lgi.clear();
    lnode.clear();
    for (int32_t q : path) {
      lpc.insert(lpc.end(), D.pc[q].begin(), D.pc[q].end());
      lpp.insert(lpp.end(), D.pp[q].begin(), D.pp[q].end());
      if (slot[q] >= 0) {
        lgi.push_back(slot[q]);
        lnode.push_back(q);
      }
    }
    bptr.push_back(T.begin[L]);
    bgeo.push_back(make_double4(T.ctr[3 * L], T.ctr[3 * L + 1], T.ctr[3 * L + 2], T.rad[L]));
    pids.insert(pids.end(), lpc.begin(), lpc.end());
    pptr.push_back((int32_t)pids.size());
    dids.insert(dids.end(), lpp.begin(), lpp.end());
    dptr.push_back((int32_t)dids.size());
    xgi.insert(xgi.end(), lgi.begin(), lgi.end());
    xnode.insert(xnode.end(), lnode.begin(), lnode.end());
    xptr.push_back((int32_t)xgi.size());
    lmax = std::max<int64_t>(lmax, T.end[L] - T.begin[L]);
  }
  const int64_t nb = (int64_t)bgeo.size();
  const int wpb_t = (int)((lmax + bltc::kWave - 1) / bltc::kWave);
  const int wpb_g = (int)((P + bltc::kWave - 1) / bltc::kWave);
  bptr.push_back((int32_t)m);
  if (pids.size() > (size_t)INT32_MAX || dids.size() > (size_t)INT32_MAX)
    throw HipError{BLTC_EINVAL, "cluster-cluster lists exceed 2^31 entries"};

  if (!tgt->dual) tgt->dual = new bltc_dual_cache;
  bltc_dual_cache& C = *tgt->dual;
  DevBuf<int32_t>&d_gnode = C.gnode, &d_gbptr = C.gbptr, &d_gpptr = C.gpptr, &d_gpids = C.gpids,
      &d_gdptr = C.gdptr, &d_gdids = C.gdids, &d_giota = C.giota, &d_bptr = C.bptr,
      &d_pptr = C.pptr, &d_pids = C.pids, &d_dptr = C.dptr, &d_dids = C.dids, &d_xptr = C.xptr,
      &d_xgi = C.xgi, &d_xnode = C.xnode;
  DevBuf<double4>&d_bgeo = C.bgeo, &d_gbgeo = C.gbgeo;
  DevBuf<double>&d_tgrid = C.tgrid, &d_g = C.g, &d_gpts = C.gpts;
  auto up = [&](auto& buf, const auto& v) {
    buf.reserve(v.size());
    h2d(buf.p, v.data(), v.size(), s);
  };
  up(d_gnode, gnode);
  up(d_gbptr, gbptr);
  up(d_gpptr, gpptr);
  up(d_gpids, gpids);
  up(d_gdptr, gdptr);
  up(d_gdids, gdids);
  up(d_gbgeo, gbgeo);
  up(d_giota, giota);
  up(d_bptr, bptr);
  up(d_pptr, pptr);
  up(d_pids, pids);
  up(d_dptr, dptr);
  up(d_dids, dids);
  up(d_xptr, xptr);
  up(d_xgi, xgi);
  up(d_xnode, xnode);
  up(d_bgeo, bgeo);
  d_tgrid.reserve(ntn * 3 * n1);
  d_g.reserve(odim * M);
  d_gpts.reserve(3 * M);
  double tk[bltc::kMaxDegree + 1];
  bltc::cheb_points(degree, tk);
  hipchk(bltc::launch_grids(tgt->d_box, ntn, degree, tk, d_tgrid.p, s), "target grids");
  hipchk(bltc::launch_dual_points(d_gnode.p, ng, n1, d_tgrid.p, d_gpts.p, s), "grid points");
  lt.stop();
  // the rule's lower degrees that the source side uses, derived from the top
  // degree's weights
  if (rule.deg_min > 0) {
    std::vector<bool> used(degree, false);
    for (int64_t A = 0; A < ntn; ++A)
      for (const auto* lst : {&D.cc[A], &D.pc[A]})
        for (int32_t e : *lst) {
          const int dd = e >> bltc::kDegShift;
          if (dd < degree) used[dd] = true;
        }
    for (int dd = rule.deg_min; dd < degree; ++dd)
      if (used[dd]) ensure_derived(src, dd, degree, s);
  }

  StageTimer ev(BLTC_STAGE_EVAL, s);
  // the particle-cluster kernel over a point set: batches bp/bg, proxy
  // lists pp/pi, direct lists dp/di, output dst [odim][mm] via tperm
  auto p2p = [&](const double* tx, int64_t mm, const int32_t* tperm, const int32_t* bp,
                 const double4* bg, int64_t nbb, int wpb, const int32_t* pp, const int32_t* pi,
                 const int32_t* dp, const int32_t* di, double* dst) {
    bltc::P2PArgs a;
    a.tx = tx;
    a.m = mm;
    a.tperm = tperm;
    a.bptr = bp;
    a.bgeo = bg;
    a.nb = nbb;
    a.wpb = wpb;
    a.pptr = pp;
    a.pids = pi;
    a.dptr = dp;
    a.dids = di;
    a.range = src->d_range;
    a.grid = d.grid;
    a.fhat = o.precision == BLTC_FP64 ? (const void*)d.p2p64 : (const void*)d.p2p32;
    if (rule.deg_min > 0) {
      for (int dd = rule.deg_min; dd <= degree; ++dd) {   // lower degrees derived from the top
        const bltc_degree_data* e = &d;
        if (dd < degree) {
          const auto it = src->derived.find({dd, degree});
          if (it == src->derived.end()) continue;   // a degree no list entry carries
          e = &it->second;
        }
        a.grid_d[dd] = e->grid;
        a.fhat_d[dd] = o.precision == BLTC_FP64 ? (const void*)e->p2p64 : (const void*)e->p2p32;
      }
    }
    a.ys = src->d_y;
    a.w64 = src->d_w64;
    a.w32 = src->d_w32;
    a.n = src->n;
    a.eps = eps;
    a.poly_p = o.poly_p;
    a.poly_c = o.poly_c;
    kernel_scales(kernel, &a.scale_u, &a.scale_w);
    a.out = dst;
    hipchk(bltc::launch_p2p(kernel, o.precision, degree, a, s), "p2p");
  };
  // grid potentials g_A at the target clusters' grid points (CC and CP)
  if (gnb > 0)
    p2p(d_gpts.p, M, d_giota.p, d_gbptr.p, d_gbgeo.p, gnb, wpb_g, d_gpptr.p, d_gpids.p,
        d_gdptr.p, d_gdids.p, d_g.p);
  // targets: PC and PP of their leaf and its ancestors
  p2p(tgt->d_y, m, tgt->d_perm, d_bptr.p, d_bgeo.p, nb, wpb_t, d_pptr.p, d_pids.p, d_dptr.p,
      d_dids.p, out);

  bltc::DualDownArgs da;
  da.bptr = d_bptr.p;
  da.nb = nb;
  da.wpb = wpb_t;
  da.tx = tgt->d_y;
  da.m = m;
  da.tperm = tgt->d_perm;
  da.dptr = d_xptr.p;
  da.dgi = d_xgi.p;
  da.dnode = d_xnode.p;
  da.tgrid = d_tgrid.p;
  da.g = d_g.p;
  da.gstride = M;
  da.out = out;
  if (ng > 0) hipchk(bltc::launch_dual_down(odim, n1, da, s), "dual down");
  ev.stop();
  if (counts) std::memcpy(counts, D.cnt, sizeof D.cnt);
  sync(s);   // the device lists go out of scope
}

void evaluate_adaptive(bltc_tree t, bltc_targets g, int kernel, double eps,
                       bltc_selector sel, double tol, int mode, int fb_degree, double fb_theta,
                       const bltc_options& o, double* out, int32_t* choice_out,
                       int64_t* stats, double* judge, hipStream_t s) {
  const int64_t nb = g->nb;
  int64_t st[4] = {nb, 0, 0, 0};
  double jd[2] = {0.0, 0.0};
  if (g->m == 0) {
    if (stats) std::memcpy(stats, st, sizeof st);
    if (judge) std::memcpy(judge, jd, sizeof jd);
    return;
  }
  const int k = sel->k;
  const int rule_min = sel->deg_min;
  const bltc::Costs costs{(float)sel->cost_far, (float)sel->cost_row, (float)sel->cost_clu,
                          (float)sel->cost_near};
  ensure_selection_scratch(g, k, 0);

  // 1. predicted log10 errors of every candidate, and their modelled costs
  compute_features(t, g, kernel, eps, sel->theta_ref, sel->d_mean, sel->d_std, g->d_feat, s);
  hipchk(bltc::launch_mlp_forward(sel->d_params, g->d_feat, nb, k, g->d_Y, nullptr, s),
         "mlp forward");
  candidate_costs(t, g, k, sel->cand_n.data(), sel->cand_theta.data(), rule_min, costs,
                  g->d_cost, s);
  hipchk(bltc::launch_pred_err2(g->d_Y, k, nb, g->d_e2, s), "predicted errors");

  // 2. the judge: the fallback treecode at one sample per batch
  ensure_degree(t, fb_degree, s);
  int64_t np = 0, nd = 0;
  build_lists(t, g, fb_theta, nullptr, g->ls[1], s, &np, &nd);
  const bltc_degree_data& fd = t->deg.at(fb_degree);
  bltc::GuardArgs ga;
  ga.spos = g->d_spos;
  ga.sbatch = g->d_sbatch;
  ga.ns = g->nsamp;
  ga.tx = g->d_x;
  ga.m = g->m;
  ga.pptr = g->ls[1].ptr;
  ga.pids = g->ls[1].pids;
  ga.dptr = g->ls[1].ptr + nb + 1;
  ga.dids = g->ls[1].dids;
  ga.range = t->d_range;
  ga.grid = fd.grid;
  ga.fh32 = fd.p2p32;
  ga.ys = t->d_y;
  ga.w32 = t->d_w32;
  ga.n = t->n;
  ga.eps = eps;
  kernel_scales(kernel, &ga.scale_u, &ga.scale_w);
  ga.ufb = g->d_ufb;
  hipchk(bltc::launch_guard(kernel, fb_degree, ga, s), "judge samples");
  double ws[2];
  judge_sums(g, kernel, nullptr, ws, s);
  hipchk(bltc::launch_batch_weights(nb, bltc::kJudgeStride, g->d_bptr, g->d_usq, g->d_wt, s),
         "batch weights");
  const double wsum = ws[0];

  if (mode == BLTC_SELECT_RUN) {
    // 3. one candidate for the whole run: the cheapest whose predicted global
    //    error sqrt(sum_b wn_b e_b^2) is within tau = tol 10^-margin_global
    const double tau = tol * std::pow(10.0, -sel->margin_global);
    const double inv_w = wsum > 0.0 ? 1.0 / (wsum * tau * tau) : 0.0;
    hipchk(bltc::launch_cand_totals(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w, g->d_sums, s),
           "candidate totals");
    std::vector<double> tot(2 * (size_t)k);
    d2h(tot.data(), g->d_sums, 2 * (size_t)k, s);
    sync(s);
    int best = -1, most = 0;
    for (int j = 0; j < k; ++j) {
      if (tot[2 * j + 1] < tot[2 * most + 1]) most = j;
      if (tot[2 * j + 1] <= 1.0 && (best < 0 || tot[2 * j] < tot[2 * best])) best = j;
    }
    hipchk(bltc::launch_fill_i32(g->d_choice, nb, best >= 0 ? best : most, s), "choice");
  } else {
  // 3. error budget: minimise the modelled cost subject to
  //    sum_b wn_b e_b^2 <= tau^2,  wn_b = w_b / sum w,  tau = tol 10^-margin,
  //    by the multiplier lam of cost + lam wn e^2 / tau^2 (two grid passes)
  const double tau = tol * std::pow(10.0, -sel->margin);
  const double inv_w = wsum > 0.0 ? 1.0 / (wsum * tau * tau) : 0.0;
  double lam_star = 0.0;
  if (inv_w > 0.0) {
    double lo = 0.0, hi = 24.0;   // log10 of the multiplier range
    lam_star = std::pow(10.0, hi);
    std::vector<double> lam(kLamGrid), sums(2 * kLamGrid);
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < kLamGrid; ++i)
        lam[i] = std::pow(10.0, lo + (hi - lo) * i / (kLamGrid - 1));
      h2d(g->d_lam, lam.data(), kLamGrid, s);
      hipchk(bltc::launch_alloc(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w,
                                g->d_lam, kLamGrid, g->d_part, g->d_sums, s),
             "allocation");
      d2h(sums.data(), g->d_sums, 2 * kLamGrid, s);
      sync(s);
      // err sums are in units of tau^2 (wn carries 1/tau^2)
      int first = -1;
      for (int i = 0; i < kLamGrid; ++i)
        if (sums[2 * i + 1] <= 1.0) {
          first = i;
          break;
        }
      if (first < 0) {         // not even the most accurate choices meet it
        lam_star = lam[kLamGrid - 1];
        break;
      }
      lam_star = lam[first];
      if (first == 0) break;   // the cheapest choices already meet it
      const double step = (hi - lo) / (kLamGrid - 1);
      hi = lo + step * first;
      lo = hi - step;
    }
  }
  hipchk(bltc::launch_choose(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w,
                             lam_star, g->d_choice, s),
         "choose");
  }
  std::vector<int32_t> choice(nb);
  d2h(choice.data(), g->d_choice, nb, s);
  sync(s);

  // 4. lists at each batch's theta; modified weights of every chosen degree
  //    for the clusters its batches use; evaluation grouped by degree
  std::vector<double> th(nb);
  std::map<int, std::vector<int32_t>> by_degree;
  for (int64_t b = 0; b < nb; ++b) {
    th[b] = sel->cand_theta[choice[b]];
    by_degree[sel->cand_n[choice[b]]].push_back((int32_t)b);
  }
  st[1] = (int64_t)by_degree.size();
  h2d(g->d_theta_b, th.data(), nb, s);
  {
    bltc::ListArgs extra;
    extra.choice = g->d_choice;
    extra.cand_T = g->d_candT;
    extra.cand_deg = g->d_candn;
    extra.rule_deg_min = rule_min;
    build_lists(t, g, 0.0, g->d_theta_b, g->ls[0], s, &np, &nd, nullptr, &extra);
  }
  std::vector<int32_t> order;
  std::vector<std::pair<int, std::pair<int64_t, int64_t>>> spans;
  for (auto& kv : by_degree) {
    spans.push_back({kv.first, {(int64_t)order.size(), (int64_t)kv.second.size()}});
    order.insert(order.end(), kv.second.begin(), kv.second.end());
  }
  h2d(g->d_bmap, order.data(), nb, s);
  // each group's top degree and, with the rule, the lower degrees derived
  // from it (a batch's result then depends on its own top degree only)
  std::vector<std::pair<int, std::pair<const int32_t*, int64_t>>> grp;
  for (auto& sp : spans) {
    ensure_degree(t, sp.first, s);
    grp.push_back({sp.first, {g->d_bmap + sp.second.first, sp.second.second}});
  }
  derive_used_degrees(t, g, g->ls[0], rule_min, grp, s);
  bltc_options og = o;
  og.deg_min = rule_min;
  // the degree groups write disjoint targets: with more than one, they run
  // concurrently on side streams, largest first
  Events evs;
  if (spans.size() == 1) {
    run_p2p(t, g, g->ls[0], kernel, eps, spans[0].first, og, g->d_bmap, nb, out, s);
  } else {
    std::sort(spans.begin(), spans.end(), [](const auto& a, const auto& b) {
      const double wa = (double)a.second.second * std::pow(a.first + 1.0, 3);
      const double wb = (double)b.second.second * std::pow(b.first + 1.0, 3);
      return wa > wb;
    });
    hipEvent_t ready = evs.make();
    hipchk(hipEventRecord(ready, s), "hipEventRecord");
    std::vector<hipEvent_t> done;
    for (size_t i = 0; i < spans.size(); ++i) {
      hipStream_t ss = side_stream((int)i);
      hipchk(hipStreamWaitEvent(ss, ready, 0), "hipStreamWaitEvent");
      run_p2p(t, g, g->ls[0], kernel, eps, spans[i].first, og,
              g->d_bmap + spans[i].second.first, spans[i].second.second, out, ss);
      if (i + kSideStreams >= spans.size()) {   // last launch on this side stream
        hipEvent_t e = evs.make();
        hipchk(hipEventRecord(e, ss), "hipEventRecord");
        done.push_back(e);
      }
    }
    for (hipEvent_t e : done) hipchk(hipStreamWaitEvent(s, e, 0), "hipStreamWaitEvent");
  }

  // 5. the judge's estimate of the global error; when it exceeds tol, the
  //    batches with the largest sampled errors are evaluated again with the
  //    fallback until the estimate is at most 0.8 tol (the sampled estimate
  //    reads up to about 15% low where the error sits in a few clustered
  //    batches)
  double js[2];
  judge_sums(g, kernel, out, js, s);
  jd[0] = jd[1] = wsum > 0.0 ? std::sqrt(js[1] / wsum) : 0.0;
  if (js[1] > tol * tol * wsum) {
    // the fewest samples, largest terms first, whose removal brings the
    // estimate to (0.8 tol)^2; their batches go to the fallback
    const int ns = g->nsamp;
    std::vector<double> c(ns);
    d2h(c.data(), g->d_contrib, ns, s);
    sync(s);
    std::vector<int32_t> ord(ns);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return c[a] > c[b]; });
    double rest = js[1];
    std::vector<int32_t> redo;
    for (int32_t i : ord) {
      if (rest <= 0.64 * tol * tol * wsum) break;
      rest -= c[i];
      for (int64_t b = (int64_t)i * bltc::kJudgeStride;
           b < std::min<int64_t>(nb, (int64_t)(i + 1) * bltc::kJudgeStride); ++b) {
        redo.push_back((int32_t)b);
        choice[b] = -2;
      }
    }
    std::sort(redo.begin(), redo.end());
    st[2] = (int64_t)redo.size();
    if (!redo.empty()) {
      h2d(g->d_bmap, redo.data(), redo.size(), s);
      if (g->batch_size <= bltc::kWave) {
        // few batches: each batch's proxy list is cut into slices that run
        // as separate waves (the direct list goes with the first slice);
        // the slices' FP64 sums are added in slice order
        std::vector<int32_t> lp(nb + 1);
        d2h(lp.data(), g->ls[1].ptr, nb + 1, s);
        sync(s);
        int64_t tot = 0;
        for (int32_t b : redo) tot += lp[b + 1] - lp[b];
        const int64_t len = std::max<int64_t>(16, (tot + 4095) / 4096);
        std::vector<int4> sl;
        std::vector<int32_t> sptr{0};
        for (int32_t b : redo) {
          const int32_t p0 = lp[b], p1 = lp[b + 1];
          if (p0 == p1) sl.push_back(make_int4(b, p0, p0, 1));
          for (int64_t q = p0; q < p1; q += len)
            sl.push_back(make_int4(b, (int)q, (int)std::min<int64_t>(p1, q + len), q == p0));
          sptr.push_back((int32_t)sl.size());
        }
        const int odim = odim_of(kernel);
        if (!g->split) g->split = new bltc_split_cache;
        DevBuf<int4>& d_sl = g->split->sl;
        DevBuf<int32_t>& d_sptr = g->split->sptr;
        DevBuf<double>& d_part = g->split->part;
        d_sl.reserve(sl.size());
        d_sptr.reserve(sptr.size());
        d_part.reserve(sl.size() * odim * bltc::kWave);
        h2d(d_sl.p, sl.data(), sl.size(), s);
        h2d(d_sptr.p, sptr.data(), sptr.size(), s);
        run_p2p(t, g, g->ls[1], kernel, eps, fb_degree, o, g->d_bmap, (int64_t)redo.size(),
                out, s, d_sl.p, (int64_t)sl.size(), d_part.p);
        double su, sw;
        kernel_scales(kernel, &su, &sw);
        hipchk(bltc::launch_split_reduce(d_sptr.p, g->d_bmap, (int64_t)redo.size(), g->d_bptr,
                                         g->d_tperm, d_part.p, odim, su, sw, g->m, out, s),
               "split reduce");
        judge_sums(g, kernel, out, js, s);
      } else {
        run_p2p(t, g, g->ls[1], kernel, eps, fb_degree, o, g->d_bmap, (int64_t)redo.size(),
                out, s);
        judge_sums(g, kernel, out, js, s);
      }
      jd[1] = std::sqrt(js[1] / wsum);
    }
  }
  sync(s);
  if (choice_out) std::memcpy(choice_out, choice.data(), sizeof(int32_t) * nb);
  if (stats) std::memcpy(stats, st, sizeof st);
  if (judge) std::memcpy(judge, jd, sizeof jd);
}

// Selector model file (little endian):
//   char magic[8] "BLTCSEL1"; int32 version (4); int32 n_in (12);
//   int32 n_hidden (64); int32 k; int32 deg_min (separation rule, 0 = off);
//   int32 cand_n[k]; double cand_theta[k];
//   double theta_ref, cost_far, cost_row, cost_cluster, cost_near, margin,
//   margin_global;
//   float mean[12], stdv[12]; float params[bltc_mlp_params(k)];
//   uint64 FNV-1a hash of all preceding bytes.
uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

int load_selector(const char* path, bltc_selector sel) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(BLTC_EMODEL, std::string("cannot open selector model ") + path);
  std::vector<unsigned char> buf;
  unsigned char tmp[4096];
  size_t r;
  while ((r = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
  std::fclose(f);
  size_t off = 0;
  auto take = [&](void* dst, size_t n) {
    if (off + n > buf.size()) return false;
    std::memcpy(dst, buf.data() + off, n);
    off += n;
    return true;
  };
  char magic[8];
  int32_t hdr[5];
  if (!take(magic, 8) || std::memcmp(magic, "BLTCSEL1", 8) != 0 || !take(hdr, sizeof hdr))
    return fail(BLTC_EMODEL, "selector model: bad magic or header");
  if (hdr[4] < 0 || hdr[4] > bltc::kMaxDegree)
    return fail(BLTC_EMODEL, "selector model: deg_min out of range");
  if (hdr[0] != 4 || hdr[1] != bltc::kMlpIn || hdr[2] != bltc::kMlpHidden || hdr[3] < 1 ||
      hdr[3] > bltc::kMlpMaxOut)
    return fail(BLTC_EMODEL, "selector model: unsupported version or dimensions");
  const int32_t k = hdr[3];
  sel->k = k;
  sel->deg_min = hdr[4];
  sel->cand_n.resize(k);
  sel->cand_theta.resize(k);
  double tail[7];
  sel->mean.resize(bltc::kMlpIn);
  sel->stdv.resize(bltc::kMlpIn);
  sel->params.resize(bltc::mlp_params(k));
  if (!take(sel->cand_n.data(), 4 * (size_t)k) || !take(sel->cand_theta.data(), 8 * (size_t)k) ||
      !take(tail, sizeof tail) || !take(sel->mean.data(), 4 * bltc::kMlpIn) ||
      !take(sel->stdv.data(), 4 * bltc::kMlpIn) ||
      !take(sel->params.data(), 4 * sel->params.size()))
    return fail(BLTC_EMODEL, "selector model: truncated");
  const uint64_t want = fnv1a(buf.data(), off);
  uint64_t got = 0;
  if (!take(&got, 8) || got != want || off != buf.size())
    return fail(BLTC_EMODEL, "selector model: checksum mismatch or trailing bytes");
  sel->theta_ref = tail[0];
  sel->cost_far = tail[1];
  sel->cost_row = tail[2];
  sel->cost_clu = tail[3];
  sel->cost_near = tail[4];
  sel->margin = tail[5];
  sel->margin_global = tail[6];
  for (int i = 1; i < 5; ++i)
    if (!(tail[i] >= 0.0 && tail[i] < 1e6))
      return fail(BLTC_EMODEL, "selector model: cost weight out of range");
  if (!(tail[5] > -6.0 && tail[5] < 6.0) || !(tail[6] > -6.0 && tail[6] < 6.0))
    return fail(BLTC_EMODEL, "selector model: margin out of range");
  for (int j = 0; j < k; ++j)
    if (sel->cand_n[j] < 1 || sel->cand_n[j] > bltc::kMaxDegree ||
        !(sel->cand_theta[j] >= 0.0 && sel->cand_theta[j] <= 1.0))
      return fail(BLTC_EMODEL, "selector model: candidate out of range");
  for (int i = 0; i < bltc::kMlpIn; ++i)
    if (!(sel->stdv[i] > 0.f)) return fail(BLTC_EMODEL, "selector model: non-positive std");
  return BLTC_OK;
}

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

}  // namespace

// ============================================================================
extern "C" {

void bltc_options_default(bltc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->size = (int32_t)sizeof(bltc_options);
  o->precision = BLTC_FP64;
  o->batch_size = 64;
  o->order_leaf = 32;
  o->group_max = 512;
  o->poly_p = 2;
  o->poly_c = 1.0;
}

const char* bltc_last_error(void) { return g_err.c_str(); }

const char* bltc_version(void) { return "bltc 0.1 gfx950"; }

int bltc_build_tree(const double* x, const double* y, const double* z,
                    int64_t n, int64_t leaf_max, void* stream, bltc_tree* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (int rc = check_points(x, y, z, n, "sources")) return rc;
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  return guarded([&] {
    bltc_tree t = new bltc_tree_s;
    t->n = n;
    t->leaf_max = leaf_max;
    try {
      build_tree(x, y, z, n, leaf_max, (hipStream_t)stream, t);
    } catch (...) {
      destroy_tree(t);
      throw;
    }
    *out = t;
    return (int)BLTC_OK;
  });
}

int bltc_tree_destroy(bltc_tree t) {
  destroy_tree(t);
  return BLTC_OK;
}

int bltc_tree_info(bltc_tree t, int64_t* n_nodes, int32_t* depth) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  if (n_nodes) *n_nodes = t->host.nnodes();
  if (depth) *depth = t->host.depth;
  return BLTC_OK;
}

int bltc_tree_export(bltc_tree t, int64_t* perm, double* box, double* center,
                     double* radius, int32_t* child_first, int32_t* child_count,
                     int64_t* pbegin, int64_t* pend, int32_t* level) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  const bltc::HostTree& H = t->host;
  const int64_t nn = H.nnodes();
  for (int64_t i = 0; perm && i < t->n; ++i) perm[i] = H.perm[i];
  for (int64_t q = 0; q < nn; ++q) {
    if (box) for (int k = 0; k < 6; ++k) box[6 * q + k] = H.box[6 * q + k];
    if (center) for (int k = 0; k < 3; ++k) center[3 * q + k] = H.ctr[3 * q + k];
    if (radius) radius[q] = H.rad[q];
    if (child_first) child_first[q] = H.first[q];
    if (child_count) child_count[q] = H.count[q];
    if (pbegin) pbegin[q] = H.begin[q];
    if (pend) pend[q] = H.end[q];
    if (level) level[q] = H.level[q];
  }
  return BLTC_OK;
}

int bltc_compute_modified_weights(bltc_tree t, const double* w, int32_t wdim,
                                  int32_t degree, void* stream) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  if (wdim != 3 && wdim != 6) return fail(BLTC_EINVAL, "wdim must be 3 or 6");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (t->n > 0 && !device_ptr(w))
    return fail(BLTC_EINVAL, "weights must be a device pointer");
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    set_weights(t, w, wdim, s);
    ensure_degree(t, degree, s);
    return (int)BLTC_OK;
  });
}

int bltc_modified_weights_export(bltc_tree t, int32_t degree, double* fhat,
                                 double* grid) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  auto it = t->deg.find(degree);
  if (it == t->deg.end())
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return guarded([&] {
    const int64_t nn = t->host.nnodes();
    const int n1 = degree + 1;
    hipchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (fhat)
      hipchk(hipMemcpy(fhat, it->second.fhat64,
                       sizeof(double) * nn * t->wdim * n1 * n1 * n1,
                       hipMemcpyDeviceToHost), "hipMemcpy");
    if (grid)
      hipchk(hipMemcpy(grid, it->second.grid, sizeof(double) * nn * 3 * n1,
                       hipMemcpyDeviceToHost), "hipMemcpy");
    return (int)BLTC_OK;
  });
}

int bltc_build_targets(const double* x, const double* y, const double* z,
                       int64_t m, int32_t batch_size, int32_t order_leaf,
                       int64_t group_max, void* stream, bltc_targets* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (int rc = check_points(x, y, z, m, "targets")) return rc;
  if (batch_size < 1 || batch_size > 1024)
    return fail(BLTC_EINVAL, "batch_size must be in [1, 1024]");
  if (order_leaf < 1) return fail(BLTC_EINVAL, "order_leaf must be >= 1");
  if (group_max < 1) return fail(BLTC_EINVAL, "group_max must be >= 1");
  return guarded([&] {
    bltc_targets g = new bltc_targets_s;
    try {
      build_targets(x, y, z, m, batch_size, order_leaf, group_max, (hipStream_t)stream, g);
    } catch (...) {
      destroy_targets(g);
      throw;
    }
    *out = g;
    return (int)BLTC_OK;
  });
}

int bltc_targets_destroy(bltc_targets g) {
  destroy_targets(g);
  return BLTC_OK;
}

int bltc_targets_export(bltc_targets g, int64_t* nb, int64_t* tperm,
                        int64_t* bptr, double* bcenter, double* bradius) {
  if (!g) return fail(BLTC_EINVAL, "NULL targets");
  const bltc::HostBatches& B = g->host;
  if (nb) *nb = g->nb;
  for (int64_t i = 0; tperm && i < g->m; ++i) tperm[i] = B.perm[i];
  for (int64_t b = 0; b <= g->nb; ++b) {
    if (bptr) bptr[b] = B.bptr[b];
    if (b == g->nb) break;
    if (bcenter) for (int k = 0; k < 3; ++k) bcenter[3 * b + k] = B.geo[4 * b + k];
    if (bradius) bradius[b] = B.geo[4 * b + 3];
  }
  return BLTC_OK;
}

int bltc_host_tree(const double* hx, const double* hy, const double* hz,
                   int64_t n, int64_t leaf_max, int64_t* n_nodes,
                   int32_t* depth, int64_t* perm, double* box, double* center,
                   double* radius, int32_t* child_first, int32_t* child_count,
                   int64_t* pbegin, int64_t* pend, int32_t* level) {
  if (n < 0 || n > 0x7fffffffLL) return fail(BLTC_EINVAL, "count out of range [0, 2^31)");
  if (n > 0 && (!hx || !hy || !hz)) return fail(BLTC_EINVAL, "NULL coordinate array");
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  return guarded([&] {
    bltc_tree_s t;
    t.n = n;
    bltc::build_host_tree(hx, hy, hz, n, leaf_max, t.host);
    if (n_nodes) *n_nodes = t.host.nnodes();
    if (depth) *depth = t.host.depth;
    return bltc_tree_export(&t, perm, box, center, radius, child_first,
                            child_count, pbegin, pend, level);
  });
}

int bltc_host_batches(const double* hx, const double* hy, const double* hz,
                      int64_t m, int32_t batch_size, int32_t order_leaf,
                      int64_t group_max, int64_t* nb, int64_t* tperm,
                      int64_t* bptr, double* bcenter, double* bradius) {
  if (m < 0 || m > 0x7fffffffLL) return fail(BLTC_EINVAL, "count out of range [0, 2^31)");
  if (m > 0 && (!hx || !hy || !hz)) return fail(BLTC_EINVAL, "NULL coordinate array");
  if (batch_size < 1 || batch_size > 1024)
    return fail(BLTC_EINVAL, "batch_size must be in [1, 1024]");
  if (order_leaf < 1) return fail(BLTC_EINVAL, "order_leaf must be >= 1");
  if (group_max < 1) return fail(BLTC_EINVAL, "group_max must be >= 1");
  return guarded([&] {
    bltc_targets_s g;
    bltc::build_host_batches(hx, hy, hz, m, batch_size, order_leaf, group_max, g.host);
    g.m = m;
    g.nb = (int64_t)g.host.bptr.size() - 1;
    return bltc_targets_export(&g, nb, tperm, bptr, bcenter, bradius);
  });
}

int bltc_evaluate_tree(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt,
                       double* out, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (g->m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!t->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (t->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  if (!t->deg.count(degree))
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return guarded([&] {
    evaluate_tree(t, g, kernel, eps, degree, theta, o, out, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_evaluate_dual(bltc_tree src, bltc_tree tgt, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt, double* out,
                       int64_t* counts, void* stream) {
  if (counts) std::memset(counts, 0, 5 * sizeof(int64_t));
  if (!src || !tgt) return fail(BLTC_EINVAL, "NULL source or target tree");
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (tgt->n > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!src->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (src->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  if (!src->deg.count(degree))
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return guarded([&] {
    evaluate_dual(src, tgt, kernel, eps, degree, theta, o, out, counts, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_evaluate(const double* tx, const double* ty, const double* tz,
                  int64_t m, const double* sx, const double* sy,
                  const double* sz, int64_t n, const double* w, int32_t kernel,
                  double eps, int32_t degree, double theta, int64_t leaf_max,
                  const bltc_options* opt, double* out, void* stream) {
  if (int rc = check_points(tx, ty, tz, m, "targets")) return rc;
  if (int rc = check_points(sx, sy, sz, n, "sources")) return rc;
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (n > 0 && !device_ptr(w)) return fail(BLTC_EINVAL, "weights must be a device pointer");
  if (m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (m == 0) return BLTC_OK;   // nothing to write
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    bltc_tree t = new bltc_tree_s;
    bltc_targets g = nullptr;
    try {
      t->n = n;
      t->leaf_max = leaf_max;
      build_tree(sx, sy, sz, n, leaf_max, s, t);
      g = new bltc_targets_s;
      build_targets(tx, ty, tz, m, o.batch_size, o.order_leaf, o.group_max, s, g);
      set_weights(t, w, wdim_of(kernel), s);
      evaluate_tree(t, g, kernel, eps, degree, theta, o, out, s);
      sync(s);
    } catch (...) {
      destroy_targets(g);
      destroy_tree(t);
      throw;
    }
    destroy_targets(g);
    destroy_tree(t);
    return (int)BLTC_OK;
  });
}

int bltc_lists_export(bltc_tree t, bltc_targets g, double theta, int32_t degree,
                      int32_t deg_min, int64_t* nb, int64_t* n_prox, int64_t* n_dir,
                      int64_t* prox_ptr, int32_t* prox_ids, int32_t* prox_deg,
                      int64_t* dir_ptr, int32_t* dir_ids) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  return guarded([&] {
    int64_t np = 0, nd = 0;
    const bltc::Rule rule = make_rule(theta, degree, deg_min);
    if (g->nb > 0) build_lists(t, g, theta, nullptr, g->ls[0], nullptr, &np, &nd, &rule);
    if (nb) *nb = g->nb;
    if (n_prox) *n_prox = np;
    if (n_dir) *n_dir = nd;
    if (g->nb == 0) {
      if (prox_ptr) prox_ptr[0] = 0;
      if (dir_ptr) dir_ptr[0] = 0;
      return (int)BLTC_OK;
    }
    std::vector<int32_t> pp(g->nb + 1), dp(g->nb + 1), pe(np);
    const bltc::ListSet& L = g->ls[0];
    d2h(pp.data(), L.ptr, g->nb + 1, nullptr);
    d2h(dp.data(), L.ptr + g->nb + 1, g->nb + 1, nullptr);
    d2h(pe.data(), L.pids, np, nullptr);
    if (dir_ids) d2h(dir_ids, L.dids, nd, nullptr);
    sync(nullptr);
    for (int64_t i = 0; i < np; ++i) {
      if (prox_ids) prox_ids[i] = pe[i] & bltc::kIdMask;
      if (prox_deg) {
        const int dd = pe[i] >> bltc::kDegShift;
        prox_deg[i] = dd ? dd : degree;
      }
    }
    for (int64_t b = 0; b <= g->nb; ++b) {
      if (prox_ptr) prox_ptr[b] = pp[b];
      if (dir_ptr) dir_ptr[b] = dp[b];
    }
    return (int)BLTC_OK;
  });
}

int bltc_counts(bltc_tree t, bltc_targets g, int32_t degree, double theta, int32_t deg_min,
                int64_t* n_proxy_evals, int64_t* n_direct_evals) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  return guarded([&] {
    int64_t np = 0, nd = 0;
    const bltc::Rule rule = make_rule(theta, degree, deg_min);
    if (g->nb > 0) build_lists(t, g, theta, nullptr, g->ls[0], nullptr, &np, &nd, &rule);
    std::vector<int32_t> pp(g->nb + 1), dp(g->nb + 1), pi(np), di(nd);
    if (g->nb > 0) {
      const bltc::ListSet& L = g->ls[0];
      d2h(pp.data(), L.ptr, g->nb + 1, nullptr);
      d2h(dp.data(), L.ptr + g->nb + 1, g->nb + 1, nullptr);
      d2h(pi.data(), L.pids, np, nullptr);
      d2h(di.data(), L.dids, nd, nullptr);
      sync(nullptr);
    }
    int64_t cp = 0, cd = 0;
    const bltc::HostTree& H = t->host;
    for (int64_t b = 0; b < g->nb; ++b) {
      const int64_t cnt = g->host.bptr[b + 1] - g->host.bptr[b];
      int64_t prox = 0;
      for (int32_t k = pp[b]; k < pp[b + 1]; ++k) {
        const int dd = pi[k] >> bltc::kDegShift;
        const int64_t n1 = (dd ? dd : degree) + 1;
        prox += n1 * n1 * n1;
      }
      cp += cnt * prox;
      int64_t leaf = 0;
      for (int32_t k = dp[b]; k < dp[b + 1]; ++k) leaf += H.end[di[k]] - H.begin[di[k]];
      cd += cnt * leaf;
    }
    if (n_proxy_evals) *n_proxy_evals = cp;
    if (n_direct_evals) *n_direct_evals = cd;
    return (int)BLTC_OK;
  });
}

int bltc_direct(const double* tx, const double* ty, const double* tz,
                int64_t m, const int64_t* idx, int64_t k, const double* sx,
                const double* sy, const double* sz, int64_t n, const double* w,
                int32_t kernel, double eps, const bltc_options* opt,
                double* out, void* stream) {
  if (int rc = check_points(tx, ty, tz, m, "targets")) return rc;
  if (k < 0 || k > 0x7fffffffLL) return fail(BLTC_EINVAL, "k out of range [0, 2^31)");
  if (!idx && k > m) return fail(BLTC_EINVAL, "k exceeds the number of targets");
  if (int rc = check_points(sx, sy, sz, n, "sources")) return rc;
  if (!valid_kernel(kernel)) return fail(BLTC_EINVAL, "unknown kernel");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BLTC_EINVAL, "eps must be finite and >= 0");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (o.precision != BLTC_FP64 && o.precision != BLTC_FP32_FP64ACC)
    return fail(BLTC_EINVAL, "direct sum precision must be FP64 or FP32_FP64ACC");
  if (idx && !device_ptr(idx)) return fail(BLTC_EINVAL, "idx must be a device pointer");
  if (n > 0 && !device_ptr(w)) return fail(BLTC_EINVAL, "weights must be a device pointer");
  if (k > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  return guarded([&] {
    if (idx && k > 0) {   // every index must address a target
      std::vector<int64_t> h(k);
      d2h(h.data(), idx, k, (hipStream_t)stream);
      sync((hipStream_t)stream);
      for (int64_t v : h)
        if (v < 0 || v >= m) throw HipError{BLTC_EINVAL, "idx entry outside [0, m)"};
    }
    double su, sw;
    kernel_scales(kernel, &su, &sw);
    hipchk(bltc::launch_direct(kernel, o.precision, tx, ty, tz, idx, k, sx, sy,
                               sz, n, w, eps, o.poly_p, o.poly_c, su, sw, out,
                               (hipStream_t)stream),
           "direct");
    return (int)BLTC_OK;
  });
}

int bltc_selector_load(const char* path, bltc_selector* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (!path) return fail(BLTC_EINVAL, "NULL path");
  bltc_selector sel = new bltc_selector_s;
  if (int rc = load_selector(path, sel)) {
    delete sel;
    return rc;
  }
  int rc = guarded([&] {
    sel->d_params = dalloc<float>(sel->params.size());
    sel->d_mean = dalloc<float>(bltc::kMlpIn);
    sel->d_std = dalloc<float>(bltc::kMlpIn);
    h2d(sel->d_params, sel->params.data(), sel->params.size(), nullptr);
    h2d(sel->d_mean, sel->mean.data(), bltc::kMlpIn, nullptr);
    h2d(sel->d_std, sel->stdv.data(), bltc::kMlpIn, nullptr);
    sync(nullptr);
    return (int)BLTC_OK;
  });
  if (rc) {
    dfree(sel->d_params); dfree(sel->d_mean); dfree(sel->d_std);
    delete sel;
    return rc;
  }
  *out = sel;
  return BLTC_OK;
}

int bltc_selector_destroy(bltc_selector sel) {
  if (!sel) return BLTC_OK;
  dfree(sel->d_params); dfree(sel->d_mean); dfree(sel->d_std);
  delete sel;
  return BLTC_OK;
}

int bltc_selector_info(bltc_selector sel, int32_t* k, int32_t* cand_n,
                       double* cand_theta) {
  if (!sel) return fail(BLTC_EINVAL, "NULL selector");
  if (k) *k = sel->k;
  for (int j = 0; j < sel->k; ++j) {
    if (cand_n) cand_n[j] = sel->cand_n[j];
    if (cand_theta) cand_theta[j] = sel->cand_theta[j];
  }
  return BLTC_OK;
}

int bltc_batch_features(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                        double theta_ref, float* feat, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (kernel != BLTC_STOKESLET && kernel != BLTC_ROTLET)
    return fail(BLTC_EINVAL, "features are defined for the Stokeslet and rotlet kernels");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BLTC_EINVAL, "eps must be finite and >= 0");
  if (!(theta_ref > 0.0 && theta_ref <= 1.0)) return fail(BLTC_EINVAL, "theta_ref must be in (0, 1]");
  if (g->nb > 0 && !device_ptr(feat)) return fail(BLTC_EINVAL, "feat must be a device pointer");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    compute_features(t, g, kernel, eps, theta_ref, nullptr, nullptr, feat, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_batch_costs(bltc_tree t, bltc_targets g, int32_t k, const int32_t* cand_n,
                     const double* cand_theta, int32_t deg_min, const float* weights,
                     float* cost, void* stream) {
  if (!t || !g || !cand_n || !cand_theta || !weights)
    return fail(BLTC_EINVAL, "NULL tree, targets, candidates or weights");
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  for (int j = 0; j < k; ++j)
    if (cand_n[j] < 1 || cand_n[j] > bltc::kMaxDegree ||
        !(cand_theta[j] >= 0.0 && cand_theta[j] <= 1.0))
      return fail(BLTC_EINVAL, "candidate out of range");
  for (int i = 0; i < 4; ++i)
    if (!(weights[i] >= 0.f)) return fail(BLTC_EINVAL, "cost weights must be >= 0");
  if (g->nb > 0 && !device_ptr(cost)) return fail(BLTC_EINVAL, "cost must be a device pointer");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    const bltc::Costs w{weights[0], weights[1], weights[2], weights[3]};
    candidate_costs(t, g, k, cand_n, cand_theta, deg_min, w, cost, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_batch_counts(bltc_tree t, bltc_targets g, double theta, int32_t* n_proxy,
                      int32_t* n_near, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (g->nb > 0 && (!device_ptr(n_proxy) || !device_ptr(n_near)))
    return fail(BLTC_EINVAL, "n_proxy and n_near must be device pointers");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    batch_counts(t, g, theta, n_proxy, n_near, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_evaluate_adaptive(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                           bltc_selector sel, double tol, int32_t mode, int32_t fb_degree,
                           double fb_theta, const bltc_options* opt, double* out,
                           int32_t* choice, int64_t* stats, double* judge, void* stream) {
  if (!t || !g || !sel) return fail(BLTC_EINVAL, "NULL tree, targets or selector");
  if (kernel != BLTC_STOKESLET && kernel != BLTC_ROTLET)
    return fail(BLTC_EINVAL, "the selector serves the Stokeslet and rotlet kernels");
  if (int rc = check_eval(kernel, eps, fb_degree, fb_theta)) return rc;
  if (!(tol > 0.0 && tol < 1.0)) return fail(BLTC_EINVAL, "tol must be in (0, 1)");
  if (mode != BLTC_SELECT_BATCH && mode != BLTC_SELECT_RUN)
    return fail(BLTC_EINVAL, "mode must be BLTC_SELECT_BATCH or BLTC_SELECT_RUN");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  o.deg_min = 0;   // the candidates take the model's rule, the fallback none
  if (int rc = check_options(&o, kernel)) return rc;
  if (g->m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!t->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (t->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  return guarded([&] {
    evaluate_adaptive(t, g, kernel, eps, sel, tol, mode, fb_degree, fb_theta, o, out, choice,
                      stats, judge, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_mlp_params(int32_t k, int64_t* n_params) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (!n_params) return fail(BLTC_EINVAL, "NULL output");
  *n_params = bltc::mlp_params(k);
  return BLTC_OK;
}

int bltc_mlp_work_size(int64_t rows, int32_t k, int64_t* n_floats) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0 || !n_floats) return fail(BLTC_EINVAL, "bad rows or NULL output");
  *n_floats = std::max<int64_t>(bltc::mlp_work_floats(rows, k), (rows * k + 255) / 256 + 1);
  return BLTC_OK;
}

int bltc_mlp_forward(const float* params, const float* X, int64_t rows,
                     int32_t k, float* Y, float* cache, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (rows == 0) return BLTC_OK;
  if (!device_ptr(params) || !device_ptr(X) || !device_ptr(Y) || (cache && !device_ptr(cache)))
    return fail(BLTC_EINVAL, "params, X, Y and cache must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_forward(params, X, rows, k, Y, cache, (hipStream_t)stream),
           "mlp forward");
    return (int)BLTC_OK;
  });
}

int bltc_mlp_loss(const float* Y, const float* T, int64_t rows, int32_t k,
                  float* dY, float* loss, float* work, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (rows == 0) return BLTC_OK;
  if (!device_ptr(Y) || !device_ptr(T) || !device_ptr(dY) || !device_ptr(loss) || !device_ptr(work))
    return fail(BLTC_EINVAL, "Y, T, dY, loss and work must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_loss(Y, T, rows * k, dY, loss, work, (hipStream_t)stream),
           "mlp loss");
    return (int)BLTC_OK;
  });
}

int bltc_mlp_backward(const float* params, const float* X, const float* cache,
                      const float* dY, int64_t rows, int32_t k, float* grad,
                      float* work, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (!device_ptr(params) || !device_ptr(grad) || !device_ptr(work) ||
      (rows > 0 && (!device_ptr(X) || !device_ptr(cache) || !device_ptr(dY))))
    return fail(BLTC_EINVAL, "params, X, cache, dY, grad and work must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_backward(params, X, cache, dY, rows, k, grad, work,
                                     (hipStream_t)stream),
           "mlp backward");
    return (int)BLTC_OK;
  });
}

int bltc_adam_step(float* params, float* m, float* v, const float* grad,
                   int64_t n, float lr, float beta1, float beta2, float eps,
                   int64_t step, void* stream) {
  if (n < 0 || step < 1) return fail(BLTC_EINVAL, "n must be >= 0 and step >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return fail(BLTC_EINVAL, "beta1 and beta2 must be in [0, 1)");
  if (n == 0) return BLTC_OK;
  if (!device_ptr(params) || !device_ptr(m) || !device_ptr(v) || !device_ptr(grad))
    return fail(BLTC_EINVAL, "params, m, v and grad must be device pointers");
  return guarded([&] {
    const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
    hipchk(bltc::launch_adam(params, m, v, grad, n, lr, beta1, beta2, eps, (float)bc1,
                             (float)bc2, (hipStream_t)stream),
           "adam");
    return (int)BLTC_OK;
  });
}

int bltc_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  return BLTC_OK;
}

int bltc_profile_read(double* ms, int64_t* launches, int32_t reset) {
  return guarded([&] {
    double acc[BLTC_NSTAGES] = {0, 0, 0, 0};
    int64_t cnt[BLTC_NSTAGES] = {0, 0, 0, 0};
    for (const auto& mk : g_prof.marks) {
      hipchk(hipEventSynchronize(mk.b), "hipEventSynchronize");
      float t = 0.f;
      hipchk(hipEventElapsedTime(&t, mk.a, mk.b), "hipEventElapsedTime");
      acc[mk.stage] += t;
      cnt[mk.stage] += 1;
    }
    for (int k = 0; k < BLTC_NSTAGES; ++k) {
      if (ms) ms[k] = acc[k];
      if (launches) launches[k] = cnt[k];
    }
    if (reset) {
      for (const auto& mk : g_prof.marks) {
        g_prof.pool.push_back(mk.a);
        g_prof.pool.push_back(mk.b);
      }
      g_prof.marks.clear();
    }
    return (int)BLTC_OK;
  });
}

}  // extern "C"
