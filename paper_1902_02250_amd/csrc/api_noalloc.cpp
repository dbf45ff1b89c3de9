// Allocation-free evaluation of a built tree: bltc_evaluate_tree with its
// interaction lists, walk flags and degree mask in a fixed device array of
// this file instead of buffers grown in the targets handle, for callers that
// cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "host.h"

namespace bltc {
namespace api {
namespace {

// The fixed scratch: every device the library runs on holds its own copy
// for the life of the process.  Host code never uses the array's name as an
// address; it takes the device address from hipGetSymbolAddress, per device.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, unsigned char*> g_scratch;   // device -> the array's device address

// The current device's scratch address, looked up once per device.
unsigned char* scratch_ptr() {
  int dev = 0;
  hipchk(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) return it->second;
  void* p = nullptr;
  hipchk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
  if (!p) throw HipError{BLTC_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch"};
  g_scratch[dev] = static_cast<unsigned char*>(p);
  return static_cast<unsigned char*>(p);
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

void evaluate_tree_noalloc(bltc_tree t, bltc_targets g, int kernel, double eps, int degree,
                           double theta, const bltc_options& o, double* out, hipStream_t s) {
  const int64_t nb = g->nb;
  // the slices of a fixed evaluation (small launches), with their partial sums
  const int wpb = (g->batch_size + kWave - 1) / kWave;
  const int nsl = slices_for(nb, wpb, odim_of(kernel));
  const size_t spart_bytes = nsl > 1 ? (size_t)slices_bytes(nb, wpb, odim_of(kernel), nsl) : 0;
  // scratch layout: flags [4] | degree mask [kMaxDegree + 1] | counts [3][nb]
  // | pointers [2][nb + 1] | slice sums | proxy list, then leaf list
  const size_t o_mask = up256(4 * sizeof(int32_t));
  const size_t o_cnt = o_mask + up256((kMaxDegree + 1) * sizeof(uint32_t));
  const size_t o_ptr = o_cnt + up256(3 * (size_t)nb * sizeof(int32_t));
  const size_t o_spart = o_ptr + up256(2 * ((size_t)nb + 1) * sizeof(int32_t));
  const size_t o_ids = o_spart + up256(spart_bytes);
  if (o_ids >= kScratchBytes)
    throw HipError{BLTC_EINVAL, std::to_string(nb) + " batches need " + std::to_string(o_ids) +
                                    " bytes of scratch before any list entry; the fixed "
                                    "scratch holds " + std::to_string(kScratchBytes)};
  unsigned char* base = scratch_ptr();
  ListSet L;
  L.fixed = true;
  L.flags = reinterpret_cast<int32_t*>(base);
  uint32_t* mask = reinterpret_cast<uint32_t*>(base + o_mask);
  L.cnt = reinterpret_cast<int32_t*>(base + o_cnt);
  L.ptr = reinterpret_cast<int32_t*>(base + o_ptr);
  L.pids = reinterpret_cast<int32_t*>(base + o_ids);
  L.pcap = (int64_t)((kScratchBytes - o_ids) / sizeof(int32_t));
  // the previous call's flags stay in the array: clear them (a fill kernel,
  // which stream capture records as a kernel node)
  hipchk(launch_fill_i32(L.flags, 4, 0, s), "clear flags");
  int64_t np = 0, nd = 0;
  const Rule rule = make_rule(theta, degree, o.deg_min);
  build_lists(t, g, theta, nullptr, L, s, &np, &nd, &rule);
  if (rule.deg_min > 0) {
    // every lower degree the lists carry must have been derived already
    hipchk(launch_degree_mask(nullptr, nb, L.ptr, L.pids, mask, s), "degree mask");
    uint32_t used = 0;
    d2h(&used, mask, 1, s);
    sync(s);
    for (int dd = rule.deg_min; dd < degree; ++dd)
      if ((used >> dd & 1u) && !t->derived.count({dd, degree}))
        throw HipError{BLTC_ESTATE,
                       "the separation rule needs the degree-" + std::to_string(dd) +
                           " weights derived from degree " + std::to_string(degree) +
                           "; a call of bltc_evaluate_tree with the same options derives them"};
  }
  run_p2p(t, g, L, kernel, eps, degree, o, nullptr, 0, out, s, nullptr, 0, nullptr, nullptr, 0,
          nsl, nsl > 1 ? reinterpret_cast<double*>(base + o_spart) : nullptr);
}

}  // namespace
}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

int bltc_evaluate_tree_noalloc(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                               int32_t degree, double theta, const bltc_options* opt,
                               double* out, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_tree_eval(t, g->m, kernel, eps, degree, theta, o, out)) return rc;
  if (g->m == 0) return BLTC_OK;
  return guarded([&] {
    evaluate_tree_noalloc(t, g, kernel, eps, degree, theta, o, out, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_noalloc_scratch_bytes(int64_t* bytes) {
  if (!bytes) return fail(BLTC_EINVAL, "NULL output");
  *bytes = (int64_t)kScratchBytes;
  return BLTC_OK;
}

}  // extern "C"
