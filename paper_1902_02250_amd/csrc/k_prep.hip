// Data preparation kernels: gathers into tree order, cluster grids and the
// exclusive scan of the interaction-list sizes.  Built with
// -ffp-contract=off: the grid points c + h t_k must round exactly as written
// (Section 3, the linear map of [-1, 1] onto [a, b]).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

__global__ void k_gather_points(const double* __restrict__ x,
                                const double* __restrict__ y,
                                const double* __restrict__ z,
                                const int32_t* __restrict__ perm, int64_t n,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t j = perm[i];
  out[i] = x[j];
  out[n + i] = y[j];
  out[2 * n + i] = z[j];
}

__global__ void k_gather_weights(const double* __restrict__ w,
                                 const int32_t* __restrict__ perm, int64_t n, int wd,
                                 double* __restrict__ w64,
                                 float* __restrict__ w32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t j = perm[i];
  for (int c = 0; c < wd; ++c) {
    const double v = w[c * n + j];
    w64[c * n + i] = v;
    w32[c * n + i] = (float)v;
  }
}

struct UnitNodes {
  double t[kMaxDegree + 1];
};

// grid[q][a][k] = c_a + h_a t_k with c = 0.5 (lo + hi), h = 0.5 (hi - lo).
__global__ void k_grids(const double* __restrict__ box, int64_t nn, int n1,
                        UnitNodes u, double* __restrict__ grid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * 3 * n1) return;
  const int k = (int)(i % n1);
  const int64_t qa = i / n1;
  const int a = (int)(qa % 3);
  const int64_t q = qa / 3;
  const double lo = box[6 * q + a], hi = box[6 * q + 3 + a];
  const double c = 0.5 * (lo + hi);
  const double h = 0.5 * (hi - lo);
  const double ht = h * u.t[k];
  grid[i] = c + ht;
}

// Single-work-group exclusive scan: out[0..n] with out[n] = total.  Sums are
// kept in 64 bits; a total above INT32_MAX sets *overflow.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ in,
                                               int64_t n,
                                               int32_t* __restrict__ out,
                                               int32_t* __restrict__ overflow) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = t * per;
  const int64_t e = b + per < n ? b + per : n;
  long long s = 0;
  for (int64_t i = b; i < e; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    long long v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  long long run = part[t] - s;   // exclusive prefix of this segment
  for (int64_t i = b; i < e; ++i) {
    out[i] = (int32_t)run;
    run += in[i];
  }
  if (t == 1023) {
    out[n] = (int32_t)part[1023];
    *overflow = part[1023] > 2147483647LL ? 1 : 0;
  }
}

inline unsigned blocks(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}
}  // namespace

hipError_t launch_gather_points(const double* x, const double* y,
                                const double* z, const int32_t* perm,
                                int64_t n, double* out3, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_points, dim3(blocks(n, 256)), dim3(256), 0, s,
                     x, y, z, perm, n, out3);
  return hipGetLastError();
}

hipError_t launch_gather_weights(const double* w, const int32_t* perm,
                                 int64_t n, int wd, double* w64, float* w32,
                                 hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_weights, dim3(blocks(n, 256)), dim3(256), 0, s,
                     w, perm, n, wd, w64, w32);
  return hipGetLastError();
}

hipError_t launch_grids(const double* box, int64_t nn, int degree,
                        const double* unit_nodes, double* grid, hipStream_t s) {
  if (nn == 0) return hipSuccess;
  UnitNodes u;
  for (int k = 0; k <= kMaxDegree; ++k) u.t[k] = k <= degree ? unit_nodes[k] : 0.0;
  const int n1 = degree + 1;
  hipLaunchKernelGGL(k_grids, dim3(blocks(nn * 3 * n1, 256)), dim3(256), 0, s,
                     box, nn, n1, u, grid);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* out,
                                 int32_t* overflow, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, in, n, out, overflow);
  return hipGetLastError();
}

}  // namespace bltc
