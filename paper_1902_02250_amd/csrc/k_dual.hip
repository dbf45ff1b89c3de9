// Cluster-cluster variant of the treecode (the interpolation in the target
// variable that Section 9 names as the next step): the two kernels the
// particle-cluster path does not have.
//
//   k_dual_points: the Chebyshev grid points t_m of the target clusters that
//     receive CC or CP work, written as a point set [3][ng (n+1)^3].  The
//     particle-cluster kernel then evaluates these points against the CC
//     clusters' proxies (its far field) and the CP clusters' particles (its
//     near field), which gives the grid potentials
//       g_A[m] = sum_{C in CC(A)} sum_k K(t_m, s_k) fhat_C,k
//              + sum_{C in CP(A)} sum_{y in C} K(t_m, y) f_y
//     with the same tensor-product marginal sums as for targets.
//   k_dual_down: every target adds sum_m L_m(x) g_A[m] for the clusters A on
//     its list, with the tensor-product Lagrange basis on A's grid in the
//     barycentric form and the exact-hit rule of Algorithm 1 (FP64).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "bltc.h"
#include "internal.h"

namespace bltc {

namespace {

__global__ void k_dual_points(const int32_t* __restrict__ gnode, int64_t ng, int n1,
                              const double* __restrict__ tgrid, double* __restrict__ pts) {
  const int64_t P = (int64_t)n1 * n1 * n1, M = ng * P;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int64_t gi = i / P;
  const int m = (int)(i % P);
  const double* __restrict__ g = tgrid + (int64_t)gnode[gi] * 3 * n1;
  pts[i] = g[m / (n1 * n1)];
  pts[M + i] = g[n1 + (m / n1) % n1];
  pts[2 * M + i] = g[2 * n1 + m % n1];
}

// L_k(v), k < N1, on the nodes s (barycentric form, exact-hit rule).
template <int N1>
__device__ __forceinline__ void lagrange(const double* __restrict__ s, double v, double* L) {
  int flag = -1;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const double wk = (k == 0 || k == N1 - 1) ? ((k & 1) ? -0.5 : 0.5) : ((k & 1) ? -1.0 : 1.0);
    const double diff = v - s[k];
    if (fabs(diff) <= DBL_MIN) {
      flag = k;
      L[k] = 0.0;
    } else {
      L[k] = wk / diff;
      sum += L[k];
    }
  }
  if (flag >= 0) {
#pragma unroll
    for (int k = 0; k < N1; ++k) L[k] = k == flag ? 1.0 : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) L[k] = L[k] / sum;
  }
}

// One lane per target of a batch (wave wv of batch b serves its targets
// 64 wv ..): out += sum over the batch's down list.
template <int N1, int OD>
__global__ __launch_bounds__(64) void k_dual_down(DualDownArgs a) {
  constexpr int P = N1 * N1 * N1;
  const int b = blockIdx.x / a.wpb, wv = blockIdx.x % a.wpb;
  const int t0 = a.bptr[b], t1 = a.bptr[b + 1];
  const int ti = t0 + wv * 64 + (int)threadIdx.x;
  if (ti >= t1) return;
  const double x = a.tx[ti], y = a.tx[a.m + ti], z = a.tx[2 * a.m + ti];
  double u[OD];
#pragma unroll
  for (int c = 0; c < OD; ++c) u[c] = 0.0;
  for (int e = a.dptr[b]; e < a.dptr[b + 1]; ++e) {
    const int gi = a.dgi[e], A = a.dnode[e];
    const double* __restrict__ tg = a.tgrid + (int64_t)A * 3 * N1;
    double Lx[N1], Ly[N1], Lz[N1];
    lagrange<N1>(tg, x, Lx);
    lagrange<N1>(tg + N1, y, Ly);
    lagrange<N1>(tg + 2 * N1, z, Lz);
    const double* __restrict__ g = a.g + (int64_t)gi * P;   // row c at c * a.gstride
    for (int k1 = 0; k1 < N1; ++k1)
      for (int k2 = 0; k2 < N1; ++k2) {
        const double l12 = Lx[k1] * Ly[k2];
        const int r = (k1 * N1 + k2) * N1;
#pragma unroll
        for (int k3 = 0; k3 < N1; ++k3) {
          const double l = l12 * Lz[k3];
#pragma unroll
          for (int c = 0; c < OD; ++c) u[c] = fma(l, g[c * a.gstride + r + k3], u[c]);
        }
      }
  }
  const int64_t o = a.tperm[ti];
#pragma unroll
  for (int c = 0; c < OD; ++c) a.out[c * a.m + o] += u[c];
}

template <int OD>
hipError_t down_kern(const DualDownArgs& a, int n1, hipStream_t s) {
  switch (n1) {
#define BLTC_DN(N)                                                                        \
  case N:                                                                                 \
    hipLaunchKernelGGL((k_dual_down<N, OD>), dim3((unsigned)(a.nb * a.wpb)), dim3(64), 0, s, a); \
    break;
    BLTC_DN(2) BLTC_DN(3) BLTC_DN(4) BLTC_DN(5) BLTC_DN(6) BLTC_DN(7)
    BLTC_DN(8) BLTC_DN(9) BLTC_DN(10) BLTC_DN(11) BLTC_DN(12) BLTC_DN(13)
#undef BLTC_DN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dual_points(const int32_t* gnode, int64_t ng, int n1, const double* tgrid,
                              double* pts, hipStream_t s) {
  const int64_t M = ng * n1 * n1 * n1;
  if (M == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dual_points, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, gnode, ng,
                     n1, tgrid, pts);
  return hipGetLastError();
}

hipError_t launch_dual_down(int odim, int n1, const DualDownArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  return odim == 6 ? down_kern<6>(a, n1, s) : down_kern<3>(a, n1, s);
}

}  // namespace bltc
