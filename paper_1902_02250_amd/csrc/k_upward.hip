// Upward pass: modified weights of every cluster (eq. modified_weights),
//   fhat[c][k1][k2][k3] = sum_{j in C} L_k1(y_j1) L_k2(y_j2) L_k3(y_j3) f_j[c],
// with L_k in the 2nd barycentric form (eq. Barycentric-1D) on the cluster's
// mapped Chebyshev points and the simple weights (eq. barycentric_weights),
// and the exact-hit rule of Algorithm 1: a coordinate within DBL_MIN of a
// grid point (in practice equal to it) gets L = Kronecker delta, taking the
// last such point as Algorithm 1's loop does.
//
// Only the leaves are summed over their particles.  A parent's weights come
// from its children's: each L_k of the parent grid is a polynomial of degree
// n in each variable, which interpolation on a child's degree-n grid
// reproduces exactly, so
//   fhat_P[k] = sum_children sum_m L^P_k1(s_m1) L^P_k2(s_m2) L^P_k3(s_m3) fhat_child[m]
// over the child's grid points s_m, equal to the sum over the parent's
// particles up to rounding.  Each particle is then read once instead of once
// per tree level.
//
// Leaf work decomposition: the particles of every leaf are cut into chunks
// of at most kUpwardChunk; one work group owns one chunk.  Per sub-block of
// 64 particles, 3 x 64 threads first compute the 1D values L_k for one
// (particle, axis) each into LDS; then every thread accumulates the n1
// values k3 of its (k1, k2, c) items, a tensor-product contraction of
// (n1^2 x WD) by n1 over the chunk's particles (WD = 3 weight components, or
// 6 for force and torque).  Chunk partial sums land in a scratch array and a
// second kernel adds them per cluster in chunk order.  The child-to-parent
// step (k_m2m) runs one tree level at a time, deepest first, one work group
// per (parent, weight component), as three separable contractions per child
// through LDS, the children in order.  Every sum has a fixed order, so the
// result is deterministic.  FP64 throughout.
#include <float.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

constexpr int kSub = 64;        // particles per sub-block
constexpr int kThreads = 256;

// L_k(v), k < N1, on the nodes s (barycentric form, exact-hit rule).
template <int N1>
__device__ __forceinline__ void bary_row(const double* s, double v, double* L) {
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

template <int N1, int WD>
__global__ __launch_bounds__(kThreads) void k_upward(
    const double* __restrict__ ys, const double* __restrict__ w64, int64_t n,
    const int4* __restrict__ chunks, const double* __restrict__ grid,
    double* __restrict__ partial) {
  constexpr int NK = N1 * N1 * N1;
  constexpr int NITEM = N1 * N1 * WD;                      // (k1, k2, c)
  constexpr int IPT = (NITEM + kThreads - 1) / kThreads;   // items per thread
  __shared__ double sL[3][N1][kSub];
  __shared__ double sF[WD][kSub];
  __shared__ double sS[3][N1];

  const int4 ch = chunks[blockIdx.x];
  const int q = ch.x, b = ch.y, e = ch.z;
  const int t = threadIdx.x;
  if (t < 3 * N1) sS[t / N1][t % N1] = grid[(int64_t)q * 3 * N1 + t];

  double acc[IPT][N1];
#pragma unroll
  for (int i = 0; i < IPT; ++i)
#pragma unroll
    for (int k = 0; k < N1; ++k) acc[i][k] = 0.0;
  __syncthreads();

  for (int s0 = b; s0 < e; s0 += kSub) {
    if (t < 3 * kSub) {
      const int p = t % kSub, ax = t / kSub;
      const int j = s0 + p;
      double L[N1];
      if (j < e) {
        bary_row<N1>(sS[ax], ys[(int64_t)ax * n + j], L);
        if (ax == 0)
          for (int c = 0; c < WD; ++c) sF[c][p] = w64[(int64_t)c * n + j];
      } else {
#pragma unroll
        for (int k = 0; k < N1; ++k) L[k] = 0.0;
        if (ax == 0)
          for (int c = 0; c < WD; ++c) sF[c][p] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < N1; ++k) sL[ax][k][p] = L[k];
    }
    __syncthreads();
    const int cnt = min(kSub, e - s0);
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int it = t + i * kThreads;
      if (it < NITEM) {
        const int c = it % WD;
        const int k2 = (it / WD) % N1;
        const int k1 = it / (WD * N1);
        for (int p = 0; p < cnt; ++p) {
          const double a = sL[0][k1][p] * sL[1][k2][p] * sF[c][p];
#pragma unroll
          for (int k3 = 0; k3 < N1; ++k3) acc[i][k3] = fma(a, sL[2][k3][p], acc[i][k3]);
        }
      }
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.x * WD * NK;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int it = t + i * kThreads;
    if (it < NITEM) {
      const int c = it % WD;
      const int k2 = (it / WD) % N1;
      const int k1 = it / (WD * N1);
#pragma unroll
      for (int k3 = 0; k3 < N1; ++k3)
        out[(int64_t)c * NK + (k1 * N1 + k2) * N1 + k3] = acc[i][k3];
    }
  }
}

// fhat64[q][c][k1][k2][k3] = sum of the chunk partials of cluster q, and the
// evaluation layout p2p[q][k1][k2][c][k3] in FP64 and FP32 (c < wd).  A
// cluster without chunks (a parent) gets zeros here and its sums from k_m2m.
__global__ void k_upward_reduce(const int32_t* __restrict__ chunk_ptr,
                                int64_t nn, const double* __restrict__ partial,
                                int n1, int wd, double* __restrict__ fhat64,
                                double* __restrict__ p2p64,
                                float* __restrict__ p2p32) {
  const int nk = n1 * n1 * n1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * wd * nk) return;
  const int64_t q = i / (wd * nk);
  const int r = (int)(i % (wd * nk));
  double s = 0.0;
  for (int32_t c = chunk_ptr[q]; c < chunk_ptr[q + 1]; ++c)
    s += partial[(int64_t)c * wd * nk + r];
  fhat64[i] = s;
  const int comp = r / nk, kk = r % nk;
  const int k3 = kk % n1, k12 = kk / n1;
  const int64_t o = q * wd * nk + ((int64_t)k12 * wd + comp) * n1 + k3;
  p2p64[o] = s;
  p2p32[o] = (float)s;
}

// One work group per parent q = nodes[blockIdx.x], whose children all have
// their weights, and weight component c = blockIdx.y: per child,
// T_ax[k][m] = L^P_k(s_m) on each axis, then
//   A[k1][m2][m3] = sum_m1 T_0[k1][m1] F[m1][m2][m3]
//   B[k1][k2][m3] = sum_m2 T_1[k2][m2] A[k1][m2][m3]
//   fhat_P[k1][k2][k3] += sum_m3 T_2[k3][m3] B[k1][k2][m3]
// with F the child's weights of component c.
template <int N1, int WD>
__global__ __launch_bounds__(kThreads) void k_m2m(const int32_t* __restrict__ nodes,
                                                  const int2* __restrict__ kids,
                                                  const double* __restrict__ grid,
                                                  double* __restrict__ fhat64,
                                                  double* __restrict__ p2p64,
                                                  float* __restrict__ p2p32) {
  constexpr int NK = N1 * N1 * N1;
  constexpr int N2 = N1 * N1;
  constexpr int IPT = (NK + kThreads - 1) / kThreads;
  __shared__ double sP[3][N1];
  __shared__ double sT[3][N1][N1];
  __shared__ double sF[NK];
  __shared__ double sA[NK];

  const int q = nodes[blockIdx.x];
  const int2 kd = kids[q];
  const int t = threadIdx.x;
  if (t < 3 * N1) sP[t / N1][t % N1] = grid[(int64_t)q * 3 * N1 + t];

  const int c = blockIdx.y;   // weight component
  double acc[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) acc[i] = 0.0;
  for (int ch = kd.x; ch < kd.x + kd.y; ++ch) {
    __syncthreads();   // sP written; the previous child's sT and sF read
    if (t < 3 * N1) {
      const int ax = t / N1, m = t % N1;
      double L[N1];
      bary_row<N1>(sP[ax], grid[((int64_t)ch * 3 + ax) * N1 + m], L);
#pragma unroll
      for (int k = 0; k < N1; ++k) sT[ax][k][m] = L[k];
    }
    const double* __restrict__ F = fhat64 + ((int64_t)ch * WD + c) * NK;
    for (int i = t; i < NK; i += kThreads) sF[i] = F[i];
    __syncthreads();
    for (int i = t; i < NK; i += kThreads) {
      const int k1 = i / N2, r = i % N2;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < N1; ++m) s = fma(sT[0][k1][m], sF[m * N2 + r], s);
      sA[i] = s;
    }
    __syncthreads();
    for (int i = t; i < NK; i += kThreads) {
      const int k1 = i / N2, k2 = (i / N1) % N1, m3 = i % N1;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < N1; ++m) s = fma(sT[1][k2][m], sA[(k1 * N1 + m) * N1 + m3], s);
      sF[i] = s;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      const int i = t + it * kThreads;
      if (i < NK) {
        const int k12 = i / N1, k3 = i % N1;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) s = fma(sT[2][k3][m], sF[k12 * N1 + m], s);
        acc[it] += s;
      }
    }
  }
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int i = t + it * kThreads;
    if (i < NK) {
      const int k12 = i / N1, k3 = i % N1;
      fhat64[((int64_t)q * WD + c) * NK + i] = acc[it];
      const int64_t o = (int64_t)q * WD * NK + ((int64_t)k12 * WD + c) * N1 + k3;
      p2p64[o] = acc[it];
      p2p32[o] = (float)acc[it];
    }
  }
}

// Weights of a lower degree d from those of degree n of the same cluster
// (separation rule): every L^d_k is a polynomial of degree d <= n, which
// degree-n interpolation reproduces, so
//   fhat^d[k] = sum_m R[k1][m1] R[k2][m2] R[k3][m3] fhat^n[m],  R[k][m] = L^d_k(t^n_m)
// on the reference nodes (the same for every cluster and axis).  One work
// group per (cluster, weight row c = blockIdx.y); three separable
// contractions through LDS in a fixed order.
__global__ __launch_bounds__(kThreads) void k_restrict(RestrictArgs a, int wd,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ fhat64,
                                                       double* __restrict__ p2p64,
                                                       float* __restrict__ p2p32) {
  constexpr int M = kMaxDegree + 1;
  __shared__ double sR[M * M];
  __shared__ double sF[M * M * M];
  __shared__ double sA[M * M * M];
  const int64_t q = blockIdx.x;
  const int c = blockIdx.y, t = threadIdx.x;
  const int d1 = a.d1, n1 = a.n1;
  const int ns = n1 * n1 * n1, nd = d1 * d1 * d1;
  for (int i = t; i < d1 * n1; i += kThreads) sR[i] = a.R[i];
  const double* __restrict__ F = src + (q * wd + c) * ns;
  for (int i = t; i < ns; i += kThreads) sF[i] = F[i];
  __syncthreads();
  for (int i = t; i < d1 * n1 * n1; i += kThreads) {   // A[k1][m2][m3]
    const int k1 = i / (n1 * n1), r = i % (n1 * n1);
    double s = 0.0;
    for (int m = 0; m < n1; ++m) s = fma(sR[k1 * n1 + m], sF[m * n1 * n1 + r], s);
    sA[i] = s;
  }
  __syncthreads();
  for (int i = t; i < d1 * d1 * n1; i += kThreads) {   // B[k1][k2][m3], into sF
    const int k1 = i / (d1 * n1), k2 = (i / n1) % d1, m3 = i % n1;
    double s = 0.0;
    for (int m = 0; m < n1; ++m) s = fma(sR[k2 * n1 + m], sA[(k1 * n1 + m) * n1 + m3], s);
    sF[i] = s;
  }
  __syncthreads();
  for (int i = t; i < nd; i += kThreads) {             // fhat^d[k1][k2][k3]
    const int k12 = i / d1, k3 = i % d1;
    double s = 0.0;
    for (int m = 0; m < n1; ++m) s = fma(sR[k3 * n1 + m], sF[k12 * n1 + m], s);
    fhat64[(q * wd + c) * nd + i] = s;
    const int64_t o = q * wd * nd + ((int64_t)k12 * wd + c) * d1 + k3;
    p2p64[o] = s;
    p2p32[o] = (float)s;
  }
}

template <int N1>
hipError_t run_upward(const double* ys, const double* w64, int64_t n, int wd,
                      const int4* chunks, int64_t nchunks, const double* grid,
                      double* partial, hipStream_t s) {
  if (wd == 6)
    hipLaunchKernelGGL((k_upward<N1, 6>), dim3((unsigned)nchunks), dim3(kThreads), 0,
                       s, ys, w64, n, chunks, grid, partial);
  else
    hipLaunchKernelGGL((k_upward<N1, 3>), dim3((unsigned)nchunks), dim3(kThreads), 0,
                       s, ys, w64, n, chunks, grid, partial);
  return hipGetLastError();
}

template <int N1>
hipError_t run_m2m(const int32_t* nodes, int64_t count, const int2* kids, int wd,
                   const double* grid, double* fhat64, double* p2p64, float* p2p32,
                   hipStream_t s) {
  if (wd == 6)
    hipLaunchKernelGGL((k_m2m<N1, 6>), dim3((unsigned)count, 6), dim3(kThreads), 0, s, nodes,
                       kids, grid, fhat64, p2p64, p2p32);
  else
    hipLaunchKernelGGL((k_m2m<N1, 3>), dim3((unsigned)count, 3), dim3(kThreads), 0, s, nodes,
                       kids, grid, fhat64, p2p64, p2p32);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_upward(const double* ys, const double* w64, int64_t n, int wd,
                         const int4* chunks, int64_t nchunks,
                         const double* grid, int degree, double* partial, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  switch (degree + 1) {
#define BLTC_UP(N) \
  case N:          \
    return run_upward<N>(ys, w64, n, wd, chunks, nchunks, grid, partial, s);
    BLTC_UP(2) BLTC_UP(3) BLTC_UP(4) BLTC_UP(5) BLTC_UP(6) BLTC_UP(7)
    BLTC_UP(8) BLTC_UP(9) BLTC_UP(10) BLTC_UP(11) BLTC_UP(12) BLTC_UP(13)
#undef BLTC_UP
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_upward_reduce(const int32_t* chunk_ptr, int64_t nn,
                                const double* partial, int degree, int wd,
                                double* fhat64, double* p2p64, float* p2p32, hipStream_t s) {
  if (nn == 0) return hipSuccess;
  const int n1 = degree + 1;
  const int64_t tot = nn * wd * n1 * n1 * n1;
  hipLaunchKernelGGL(k_upward_reduce, dim3((unsigned)((tot + 255) / 256)),
                     dim3(256), 0, s, chunk_ptr, nn, partial, n1, wd, fhat64,
                     p2p64, p2p32);
  return hipGetLastError();
}

hipError_t launch_m2m(const int32_t* nodes, int64_t count, const int2* kids, int degree, int wd,
                      const double* grid, double* fhat64, double* p2p64, float* p2p32,
                      hipStream_t s) {
  if (count == 0) return hipSuccess;
  switch (degree + 1) {
#define BLTC_M2M(N) \
  case N:           \
    return run_m2m<N>(nodes, count, kids, wd, grid, fhat64, p2p64, p2p32, s);
    BLTC_M2M(2) BLTC_M2M(3) BLTC_M2M(4) BLTC_M2M(5) BLTC_M2M(6) BLTC_M2M(7)
    BLTC_M2M(8) BLTC_M2M(9) BLTC_M2M(10) BLTC_M2M(11) BLTC_M2M(12) BLTC_M2M(13)
#undef BLTC_M2M
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_restrict(const RestrictArgs& a, int64_t nn, int wd, const double* src,
                           double* fhat64, double* p2p64, float* p2p32, hipStream_t s) {
  if (nn == 0) return hipSuccess;
  if (a.d1 < 1 || a.n1 < a.d1 || a.n1 > kMaxDegree + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)nn, (unsigned)wd), dim3(kThreads), 0, s, a, wd,
                     src, fhat64, p2p64, p2p32);
  return hipGetLastError();
}

}  // namespace bltc
