// Per-batch (n, theta) selection on the device: batch features, the
// cheapest candidate whose predicted error meets the tolerance, and the
// guard's comparison against the fallback.
#include <hip/hip_runtime.h>

#include "bltc.h"
#include "internal.h"

namespace bltc {

namespace {

// Features of batch b, from its geometry and one walk at theta_ref:
//  0 log2 targets             1 log10 r_B / R0         2 log10 eps / R0
//  3 log10 eps / r_B          4 log10(1 + proxy clusters)
//  5 log10(1 + near sources)  6 log10(1 + near leaves)
//  7 mean log10 r_C / R0 over accepted clusters
//  8 mean (r_B + r_C) / (theta_ref R) over accepted clusters
//  9 log10 near-field density relative to the mean density
// 10 kernel (0 Stokeslet, 1 rotlet)  11 log10 n
// R0 is the root radius; lengths below 1e-12 R0 are floored.
__global__ __launch_bounds__(128) void k_features(FeatArgs a) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.nb) return;
  const double4 g = a.bgeo[b];
  const double4 root = a.nodes.geo[0];
  const double R0 = root.w > 0.0 ? root.w : 1.0;
  const double tiny = 1e-12 * R0;
  const double th2 = a.theta_ref * a.theta_ref;
  int32_t stack[kStackMax];
  int sp = 0;
  double P = 0, L = 0, D = 0, slr = 0, stight = 0, vol = 0;
  if (a.nodes.nn > 0) stack[sp++] = 0;
  while (sp > 0) {
    const int32_t q = stack[--sp];
    const double4 c = a.nodes.geo[q];
    const double dx = g.x - c.x, dy = g.y - c.y, dz = g.z - c.z;
    const double R2 = dx * dx + dy * dy + dz * dz;
    const double rr = g.w + c.w;
    if (R2 > 0.0 && rr * rr <= th2 * R2) {
      P += 1;
      slr += log10((c.w + tiny) / R0);
      stight += rr / (a.theta_ref * sqrt(R2));
      continue;
    }
    const int2 kd = a.nodes.kids[q];
    if (kd.y == 0) {
      const int2 rg = a.nodes.range[q];
      L += 1;
      D += rg.y - rg.x;
      const double* bx = a.box + 6 * (int64_t)q;
      vol += (bx[3] - bx[0] + tiny) * (bx[4] - bx[1] + tiny) * (bx[5] - bx[2] + tiny);
      continue;
    }
    if (sp + kd.y > kStackMax) break;
    for (int k = kd.y - 1; k >= 0; --k) stack[sp++] = kd.x + k;
  }
  const double* rb = a.box;
  const double vroot = (rb[3] - rb[0] + tiny) * (rb[4] - rb[1] + tiny) * (rb[5] - rb[2] + tiny);
  const double mean_density = (double)(a.n_src > 0 ? a.n_src : 1) / vroot;
  const double cnt = (double)(a.bptr[b + 1] - a.bptr[b]);
  float f[kMlpIn];
  f[0] = (float)log2(cnt > 1 ? cnt : 1.0);
  f[1] = (float)log10((g.w + tiny) / R0);
  f[2] = (float)log10((a.eps + tiny) / R0);
  f[3] = (float)log10((a.eps + tiny) / (g.w + tiny));
  f[4] = (float)log10(1.0 + P);
  f[5] = (float)log10(1.0 + D);
  f[6] = (float)log10(1.0 + L);
  f[7] = P > 0 ? (float)(slr / P) : 0.f;
  f[8] = P > 0 ? (float)(stight / P) : 0.f;
  f[9] = (float)log10(((D + 1.0) / (vol + tiny * tiny * tiny)) / mean_density);
  f[10] = a.kernel == BLTC_ROTLET ? 1.f : 0.f;
  f[11] = (float)log10((double)(a.n_src > 0 ? a.n_src : 1));
  for (int i = 0; i < kMlpIn; ++i) {
    float v = f[i];
    if (a.mean) v = (v - a.mean[i]) / a.stdv[i];
    a.feat[b * kMlpIn + i] = v;
  }
}

// choice[b] = the candidate of least modelled cost whose predicted log10
// error plus margin is at most logtol, or -1 if none qualifies.  Modelled
// cost = targets x (proxy clusters x (n+1)^3 x cfar + near sources x cnear).
__global__ void k_select(const float* __restrict__ Y, int k, int64_t nb,
                         const int32_t* __restrict__ bptr,
                         const int32_t* __restrict__ pcnt,
                         const int32_t* __restrict__ scnt, Candidates c,
                         float logtol, float margin, float cfar, float cnear,
                         int32_t* __restrict__ choice) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double cnt = (double)(bptr[b + 1] - bptr[b]);
  int best = -1;
  double bestcost = 0.0;
  for (int j = 0; j < k; ++j) {
    if (!(Y[b * k + j] + margin <= logtol)) continue;
    const int ti = c.t[j];
    const double n1 = (double)(c.n[j] + 1);
    const double cost = cnt * ((double)pcnt[(int64_t)ti * nb + b] * n1 * n1 * n1 * cfar +
                               (double)scnt[(int64_t)ti * nb + b] * cnear);
    if (best < 0 || cost < bestcost) {
      best = j;
      bestcost = cost;
    }
  }
  choice[b] = best;
}

// flag[batch] = 1 when the learned result at a sampled target differs from
// the fallback result by more than tol relative (in the L2 norm over the
// components).
__global__ void k_guard_check(int ns, const int32_t* __restrict__ spos,
                              const int32_t* __restrict__ sbatch,
                              const int32_t* __restrict__ tperm,
                              const double* __restrict__ out, int64_t m, int od,
                              const double* __restrict__ ufb, double tol,
                              int32_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t o = tperm[spos[i]];
  double num = 0.0, den = 0.0;
  for (int c = 0; c < od; ++c) {
    const double r = ufb[(int64_t)i * od + c];
    const double d = out[c * m + o] - r;
    num += d * d;
    den += r * r;
  }
  if (num > tol * tol * den) atomicOr(&flag[sbatch[i]], 1);
}

}  // namespace

hipError_t launch_features(const FeatArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((a.nb + 127) / 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_select(const float* Y, int k, int64_t nb, const int32_t* bptr,
                         const int32_t* pcnt, const int32_t* scnt,
                         const Candidates& c, float logtol, float margin,
                         float cfar, float cnear, int32_t* choice, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_select, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, Y, k,
                     nb, bptr, pcnt, scnt, c, logtol, margin, cfar, cnear, choice);
  return hipGetLastError();
}

hipError_t launch_guard_check(int ns, const int32_t* spos, const int32_t* sbatch,
                              const int32_t* tperm, const double* out, int64_t m,
                              int od, const double* ufb, double tol,
                              int32_t* flag, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  hipLaunchKernelGGL(k_guard_check, dim3((ns + 255) / 256), dim3(256), 0, s, ns, spos,
                     sbatch, tperm, out, m, od, ufb, tol, flag);
  return hipGetLastError();
}

}  // namespace bltc
