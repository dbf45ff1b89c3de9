// Interaction lists of the batch walk (Algorithm 2 shared by the targets of
// a batch).  One 64-lane wave walks the tree for one batch, the lanes
// splitting the work over the tree's cut (walk.h), depth first, children in
// their stored order:
//   MAC holds          -> the cluster goes on the proxy list,
//   else leaf          -> the cluster goes on the direct list,
//   else               -> visit the children.
// The MAC r/R <= theta (eq. MAC) is tested for the whole batch as
//   R2 > 0  and  (r_B + r_C)^2 <= (theta theta) R2,
// R2 = dx dx + dy dy + dz dz from the batch center to the cluster center,
// in FP64 without fused multiply-adds, so the integer lists are
// reproducible bit for bit.  The count pass sizes the lists; the fill pass
// counts each lane's share again, takes the lanes' offsets from a prefix sum
// across the wave and writes the lists in walk order.  Under the separation
// rule the fill pass also stores each accepted cluster's degree: the
// smallest d in [deg_min, degree) with rr^2 / R2 <= T[d], else degree (one
// division and comparisons, reproducible bit for bit).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "walk.h"

namespace bltc {

namespace {

constexpr int kListWaves = 4;   // batches (waves) per work group

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Exclusive prefix sum over the wave's lanes.
__device__ __forceinline__ int32_t wave_exclusive(int32_t v, int lane) {
  int32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  return inc - v;
}

template <bool FILL>
__global__ __launch_bounds__(64 * kListWaves) void k_lists(ListArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * kListWaves + (threadIdx.x >> 6);
  if (b >= a.nb) return;
  const double4 g = a.bgeo[b];
  const double th = a.theta_b ? a.theta_b[b] : a.theta;
  // under the separation rule every entry carries its degree
  bool enc = a.rule.deg_min > 0;
  int rmin = a.rule.deg_min, rdeg = a.rule.degree;
  const double* rT = a.rule.T;
  if (a.choice && a.rule_deg_min > 0) {
    const int j = a.choice[b];
    enc = true;
    rmin = a.rule_deg_min;
    rdeg = a.cand_deg[j];
    rT = a.cand_T + (int64_t)j * (kMaxDegree + 1);
  }
  const double th2 = th * th;
  int32_t np = 0, nd = 0;
  int64_t ns = 0;   // near-field sources
  cut_walk(a.nodes, g, th2, lane, [&](int32_t, double, double) { ++np; },
           [&](int32_t q) {
             ++nd;
             const int2 rg = a.nodes.range[q];
             ns += rg.y - rg.x;
           });
  if (!FILL) {
    const int64_t tp = wave_sum(np), td = wave_sum(nd), tn = wave_sum(ns);
    if (lane == 0) {
      a.pcnt[b] = (int32_t)tp;
      a.dcnt[b] = (int32_t)td;
      if (a.scnt) a.scnt[b] = (int32_t)(tn < 0x7fffffff ? tn : 0x7fffffff);
    }
    return;
  }
  int32_t* pout = a.pids + a.pptr[b] + wave_exclusive(np, lane);
  int32_t* dout = a.dids + a.dptr[b] + wave_exclusive(nd, lane);
  cut_walk(a.nodes, g, th2, lane,
           [&](int32_t q, double R2, double rr) {
             int32_t e = q;
             if (enc) {
               const double qq = (rr * rr) / R2;
               int d = rmin < rdeg ? rmin : rdeg;
               while (d < rdeg && !(qq <= rT[d])) ++d;
               e |= d << kDegShift;
             }
             *pout++ = e;
           },
           [&](int32_t q) { *dout++ = q; });
}

}  // namespace

hipError_t launch_lists(const ListArgs& a, bool fill, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  const unsigned nblk = (unsigned)((a.nb + kListWaves - 1) / kListWaves);
  if (fill)
    hipLaunchKernelGGL(k_lists<true>, dim3(nblk), dim3(64 * kListWaves), 0, s, a);
  else
    hipLaunchKernelGGL(k_lists<false>, dim3(nblk), dim3(64 * kListWaves), 0, s, a);
  return hipGetLastError();
}

}  // namespace bltc
