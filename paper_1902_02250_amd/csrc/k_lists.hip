// Interaction lists of the batch walk (Algorithm 2 shared by the targets of
// a batch).  One thread walks the tree for one batch depth first, children
// in their stored order, following each node's first child or, past its
// subtree, its depth-first successor (no stack):
//   MAC holds          -> the cluster goes on the proxy list,
//   else leaf          -> the cluster goes on the direct list,
//   else               -> visit the children.
// The MAC r/R <= theta (eq. MAC) is tested for the whole batch as
//   R2 > 0  and  (r_B + r_C)^2 <= (theta theta) R2,
// R2 = dx dx + dy dy + dz dz from the batch center to the cluster center,
// in FP64 without fused multiply-adds (this file is built with
// -ffp-contract=off), so the integer lists are reproducible bit for bit.
// The count pass sizes the lists; the fill pass writes them.  Under the
// separation rule the fill pass also stores each accepted cluster's degree:
// the smallest d in [deg_min, degree) with rr^2 / R2 <= T[d], else degree
// (one division and comparisons, reproducible bit for bit).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

template <bool FILL>
__global__ __launch_bounds__(128) void k_lists(ListArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
  int32_t* pout = nullptr;
  int32_t* dout = nullptr;
  if (FILL) {
    pout = a.pids + a.pptr[b];
    dout = a.dids + a.dptr[b];
  }
  int32_t q = a.nodes.nn > 0 ? 0 : -1;
  while (q >= 0) {
    const double4 c = a.nodes.geo[q];
    const double dx = g.x - c.x;
    const double dy = g.y - c.y;
    const double dz = g.z - c.z;
    const double R2 = dx * dx + dy * dy + dz * dz;
    const double rr = g.w + c.w;
    if (R2 > 0.0 && rr * rr <= th2 * R2) {
      if (FILL) {
        int32_t e = q;
        if (enc) {
          const double qq = (rr * rr) / R2;
          int d = rmin < rdeg ? rmin : rdeg;
          while (d < rdeg && !(qq <= rT[d])) ++d;
          e |= d << kDegShift;
        }
        pout[np] = e;
      }
      ++np;
      q = a.nodes.skip[q];
      continue;
    }
    const int2 kd = a.nodes.kids[q];
    if (kd.y == 0) {
      if (FILL) dout[nd] = q;
      ++nd;
      const int2 rg = a.nodes.range[q];
      ns += rg.y - rg.x;
      q = a.nodes.skip[q];
      continue;
    }
    q = kd.x;
  }
  if (!FILL) {
    a.pcnt[b] = np;
    a.dcnt[b] = nd;
    if (a.scnt) a.scnt[b] = (int32_t)(ns < 0x7fffffff ? ns : 0x7fffffff);
  }
}

}  // namespace

hipError_t launch_lists(const ListArgs& a, bool fill, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  const unsigned nblk = (unsigned)((a.nb + 127) / 128);
  if (fill)
    hipLaunchKernelGGL(k_lists<true>, dim3(nblk), dim3(128), 0, s, a);
  else
    hipLaunchKernelGGL(k_lists<false>, dim3(nblk), dim3(128), 0, s, a);
  return hipGetLastError();
}

}  // namespace bltc
