// Host-side internals shared by the units of the C ABI, and the ABI's
// process-wide calls: options, errors, version, stage timing.
#include "host.h"

#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

namespace bltc {
namespace api {

namespace {
thread_local std::string g_err;

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

std::mutex g_side_mu;
std::map<int, std::array<hipStream_t, kSideStreams>> g_side;
}  // namespace

int g_fail_alloc_after = 0;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void hipchk(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? BLTC_ENOMEM : BLTC_EDEVICE;
  throw HipError{code, std::string(what) + ": " + hipGetErrorString(e)};
}

void* dalloc_bytes(size_t bytes) {
  if (g_fail_alloc_after > 0 && --g_fail_alloc_after == 0)
    throw HipError{BLTC_ENOMEM, "hipMalloc: out of memory (injected by the test hook)"};
  void* p = nullptr;
  hipchk(hipMalloc(&p, bytes), "hipMalloc");
  return p;
}

void sync(hipStream_t s) { hipchk(hipStreamSynchronize(s), "hipStreamSynchronize"); }

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

hipEvent_t Events::make() {
  hipEvent_t e;
  hipchk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  ev.push_back(e);
  return e;
}

Events::~Events() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

bool device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

bool valid_kernel(int k) {
  return k == BLTC_STOKESLET || k == BLTC_ROTLET || k == BLTC_FULL || k == BLTC_POLY;
}

int check_points(const double* x, const double* y, const double* z, int64_t n,
                 const char* what) {
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
  if (o->order_leaf < 0) return fail(BLTC_EINVAL, "order_leaf must be >= 0 (0: balanced k-d batches)");
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

StageTimer::StageTimer(int st, hipStream_t str) : stage(st), s(str) {
  if (!g_prof.on) return;
  a = g_prof.get();
  hipchk(hipEventRecord(a, s), "hipEventRecord");
}

void StageTimer::stop() {
  if (!a) return;
  hipEvent_t b = g_prof.get();
  hipchk(hipEventRecord(b, s), "hipEventRecord");
  g_prof.marks.push_back({stage, a, b});
  a = nullptr;
}

}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

void bltc_options_default(bltc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->size = (int32_t)sizeof(bltc_options);
  o->precision = BLTC_FP64;
  o->batch_size = 64;
  o->order_leaf = 0;   // balanced k-d batches
  o->group_max = 512;
  o->poly_p = 2;
  o->poly_c = 1.0;
}

const char* bltc_last_error(void) { return bltc::api::g_err.c_str(); }

const char* bltc_version(void) { return "bltc 0.2 gfx950"; }

int bltc_test_fail_alloc(int32_t after) {
  if (after < 0) return fail(BLTC_EINVAL, "after must be >= 0");
  g_fail_alloc_after = after;
  return BLTC_OK;
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
