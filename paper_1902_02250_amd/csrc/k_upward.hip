// Upward pass: modified weights of every cluster (eq. modified_weights),
//   fhat[c][k1][k2][k3] = sum_{j in C} L_k1(y_j1) L_k2(y_j2) L_k3(y_j3) f_j[c],
// with L_k in the 2nd barycentric form (eq. Barycentric-1D) on the cluster's
// mapped Chebyshev points and the simple weights (eq. barycentric_weights),
// and the exact-hit rule of Algorithm 1: a coordinate within DBL_MIN of a
// grid point (in practice equal to it) gets L = Kronecker delta, taking the
// last such point as Algorithm 1's loop does.
//
// Work decomposition: the particles of every cluster are cut into chunks of
// at most kUpwardChunk; one work group owns one chunk.  Per sub-block of 64
// particles, 3 x 64 threads first compute the 1D values L_k for one
// (particle, axis) each into LDS; then every thread accumulates the n1
// values k3 of its (k1, k2, c) items, a tensor-product contraction of
// (n1^2 x WD) by n1 over the chunk's particles (WD = 3 weight components, or
// 6 for force and torque).  Chunk partial sums land in
// a scratch array and a second kernel adds them per cluster in chunk order,
// so the result is deterministic.  FP64 throughout.  An optional need mask
// (one byte per cluster) restricts both kernels to the flagged clusters.
#include <float.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

constexpr int kSub = 64;        // particles per sub-block
constexpr int kThreads = 256;

template <int N1, int WD>
__global__ __launch_bounds__(kThreads) void k_upward(
    const double* __restrict__ ys, const double* __restrict__ w64, int64_t n,
    const int4* __restrict__ chunks, const double* __restrict__ grid,
    const uint8_t* __restrict__ need, double* __restrict__ partial) {
  constexpr int NK = N1 * N1 * N1;
  constexpr int NITEM = N1 * N1 * WD;                      // (k1, k2, c)
  constexpr int IPT = (NITEM + kThreads - 1) / kThreads;   // items per thread
  __shared__ double sL[3][N1][kSub];
  __shared__ double sF[WD][kSub];
  __shared__ double sS[3][N1];

  const int4 ch = chunks[blockIdx.x];
  const int q = ch.x, b = ch.y, e = ch.z;
  if (need && !need[q]) return;   // uniform over the work group
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
        const double y = ys[(int64_t)ax * n + j];
        int flag = -1;
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          const double wk = (k == 0 || k == N1 - 1) ? ((k & 1) ? -0.5 : 0.5)
                                                     : ((k & 1) ? -1.0 : 1.0);
          const double diff = y - sS[ax][k];
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
// evaluation layout p2p[q][k1][k2][c][k3] in FP64 and FP32 (c < wd).
__global__ void k_upward_reduce(const int32_t* __restrict__ chunk_ptr,
                                int64_t nn, const double* __restrict__ partial,
                                int n1, int wd, const uint8_t* __restrict__ need,
                                double* __restrict__ fhat64,
                                double* __restrict__ p2p64,
                                float* __restrict__ p2p32) {
  const int nk = n1 * n1 * n1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * wd * nk) return;
  const int64_t q = i / (wd * nk);
  if (need && !need[q]) return;
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

template <int N1>
hipError_t run_upward(const double* ys, const double* w64, int64_t n, int wd,
                      const int4* chunks, int64_t nchunks, const double* grid,
                      const uint8_t* need, double* partial, hipStream_t s) {
  if (wd == 6)
    hipLaunchKernelGGL((k_upward<N1, 6>), dim3((unsigned)nchunks), dim3(kThreads), 0,
                       s, ys, w64, n, chunks, grid, need, partial);
  else
    hipLaunchKernelGGL((k_upward<N1, 3>), dim3((unsigned)nchunks), dim3(kThreads), 0,
                       s, ys, w64, n, chunks, grid, need, partial);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_upward(const double* ys, const double* w64, int64_t n, int wd,
                         const int4* chunks, int64_t nchunks,
                         const double* grid, int degree, const uint8_t* need,
                         double* partial, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  switch (degree + 1) {
#define BLTC_UP(N) \
  case N:          \
    return run_upward<N>(ys, w64, n, wd, chunks, nchunks, grid, need, partial, s);
    BLTC_UP(2) BLTC_UP(3) BLTC_UP(4) BLTC_UP(5) BLTC_UP(6) BLTC_UP(7)
    BLTC_UP(8) BLTC_UP(9) BLTC_UP(10) BLTC_UP(11) BLTC_UP(12) BLTC_UP(13)
#undef BLTC_UP
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_upward_reduce(const int32_t* chunk_ptr, int64_t nn,
                                const double* partial, int degree, int wd,
                                const uint8_t* need, double* fhat64, double* p2p64,
                                float* p2p32, hipStream_t s) {
  if (nn == 0) return hipSuccess;
  const int n1 = degree + 1;
  const int64_t tot = nn * wd * n1 * n1 * n1;
  hipLaunchKernelGGL(k_upward_reduce, dim3((unsigned)((tot + 255) / 256)),
                     dim3(256), 0, s, chunk_ptr, nn, partial, n1, wd, need, fhat64,
                     p2p64, p2p32);
  return hipGetLastError();
}

}  // namespace bltc
