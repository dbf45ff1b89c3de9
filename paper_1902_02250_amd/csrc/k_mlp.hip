// The per-batch (n, theta) selector network on the device: forward pass,
// loss gradient, backward pass and Adam, in FP32.
//
//   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3
// with 12 inputs, two hidden layers of 64 and K outputs (K <= kMlpMaxOut).
// Flat parameters: W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [K][64],
// b3 [K].  A work group takes kRows rows; the backward pass writes one
// partial gradient per work group and a second kernel adds the partials in
// work-group order, so gradients are deterministic.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

constexpr int NIN = kMlpIn, NH = kMlpHidden, KMAX = kMlpMaxOut;
constexpr int kRows = 32;
constexpr int kThreads = 256;

struct Offsets {
  int w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Offsets offsets(int k) {
  Offsets o;
  o.w1 = 0;
  o.b1 = o.w1 + NH * NIN;
  o.w2 = o.b1 + NH;
  o.b2 = o.w2 + NH * NH;
  o.w3 = o.b2 + NH;
  o.b3 = o.w3 + k * NH;
  o.total = o.b3 + k;
  return o;
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(
    const float* __restrict__ p, const float* __restrict__ X, int64_t rows,
    int k, float* __restrict__ Y, float* __restrict__ cache) {
  __shared__ float sx[kRows][NIN];
  __shared__ float s1[kRows][NH];
  __shared__ float s2[kRows][NH];
  const Offsets o = offsets(k);
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int t = threadIdx.x;
  for (int i = t; i < kRows * NIN; i += kThreads) {
    const int r = i / NIN, c = i % NIN;
    sx[r][c] = r0 + r < rows ? X[(r0 + r) * NIN + c] : 0.f;
  }
  __syncthreads();
  for (int i = t; i < kRows * NH; i += kThreads) {
    const int r = i / NH, j = i % NH;
    float z = p[o.b1 + j];
    for (int c = 0; c < NIN; ++c) z += p[o.w1 + j * NIN + c] * sx[r][c];
    s1[r][j] = tanhf(z);
  }
  __syncthreads();
  for (int i = t; i < kRows * NH; i += kThreads) {
    const int r = i / NH, j = i % NH;
    float z = p[o.b2 + j];
    for (int c = 0; c < NH; ++c) z += p[o.w2 + j * NH + c] * s1[r][c];
    s2[r][j] = tanhf(z);
  }
  __syncthreads();
  for (int i = t; i < kRows * k; i += kThreads) {
    const int r = i / k, j = i % k;
    if (r0 + r >= rows) continue;
    float z = p[o.b3 + j];
    for (int c = 0; c < NH; ++c) z += p[o.w3 + j * NH + c] * s2[r][c];
    Y[(r0 + r) * k + j] = z;
  }
  if (cache) {
    for (int i = t; i < kRows * NH; i += kThreads) {
      const int r = i / NH, j = i % NH;
      if (r0 + r >= rows) continue;
      cache[(r0 + r) * 2 * NH + j] = s1[r][j];
      cache[(r0 + r) * 2 * NH + NH + j] = s2[r][j];
    }
  }
}

// dY = 2 (Y - T) / (rows k); partial[b] = sum of (Y - T)^2 over the block.
__global__ __launch_bounds__(kThreads) void k_mlp_loss(
    const float* __restrict__ Y, const float* __restrict__ T, int64_t total,
    float* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[kThreads];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  float sq = 0.f;
  if (i < total) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d / (float)total;
    sq = d * d;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_mlp_loss_final(const float* __restrict__ partial, int nblk,
                                 int64_t total, float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[b];
  *loss = (float)(s / (double)total);
}

__global__ __launch_bounds__(kThreads) void k_mlp_backward(
    const float* __restrict__ p, const float* __restrict__ X,
    const float* __restrict__ cache, const float* __restrict__ dY,
    int64_t rows, int k, float* __restrict__ partial) {
  __shared__ float sx[kRows][NIN];
  __shared__ float s1[kRows][NH];
  __shared__ float s2[kRows][NH];
  __shared__ float sd[kRows][KMAX];
  __shared__ float z2[kRows][NH];
  __shared__ float z1[kRows][NH];
  const Offsets o = offsets(k);
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int t = threadIdx.x;
  for (int i = t; i < kRows * NIN; i += kThreads) {
    const int r = i / NIN, c = i % NIN;
    sx[r][c] = r0 + r < rows ? X[(r0 + r) * NIN + c] : 0.f;
  }
  for (int i = t; i < kRows * NH; i += kThreads) {
    const int r = i / NH, j = i % NH;
    const bool ok = r0 + r < rows;
    s1[r][j] = ok ? cache[(r0 + r) * 2 * NH + j] : 0.f;
    s2[r][j] = ok ? cache[(r0 + r) * 2 * NH + NH + j] : 0.f;
  }
  for (int i = t; i < kRows * k; i += kThreads) {
    const int r = i / k, j = i % k;
    sd[r][j] = r0 + r < rows ? dY[(r0 + r) * k + j] : 0.f;
  }
  __syncthreads();
  for (int i = t; i < kRows * NH; i += kThreads) {   // dz2 = (dY W3) (1 - h2^2)
    const int r = i / NH, j = i % NH;
    float a = 0.f;
    for (int c = 0; c < k; ++c) a += sd[r][c] * p[o.w3 + c * NH + j];
    z2[r][j] = a * (1.f - s2[r][j] * s2[r][j]);
  }
  __syncthreads();
  for (int i = t; i < kRows * NH; i += kThreads) {   // dz1 = (dz2 W2) (1 - h1^2)
    const int r = i / NH, j = i % NH;
    float a = 0.f;
    for (int c = 0; c < NH; ++c) a += z2[r][c] * p[o.w2 + c * NH + j];
    z1[r][j] = a * (1.f - s1[r][j] * s1[r][j]);
  }
  __syncthreads();
  float* g = partial + (int64_t)blockIdx.x * o.total;
  for (int i = t; i < o.total; i += kThreads) {
    float a = 0.f;
    if (i < o.b1) {                       // W1[j][c] += dz1[r][j] x[r][c]
      const int j = i / NIN, c = i % NIN;
      for (int r = 0; r < kRows; ++r) a += z1[r][j] * sx[r][c];
    } else if (i < o.w2) {
      const int j = i - o.b1;
      for (int r = 0; r < kRows; ++r) a += z1[r][j];
    } else if (i < o.b2) {
      const int j = (i - o.w2) / NH, c = (i - o.w2) % NH;
      for (int r = 0; r < kRows; ++r) a += z2[r][j] * s1[r][c];
    } else if (i < o.w3) {
      const int j = i - o.b2;
      for (int r = 0; r < kRows; ++r) a += z2[r][j];
    } else if (i < o.b3) {
      const int j = (i - o.w3) / NH, c = (i - o.w3) % NH;
      for (int r = 0; r < kRows; ++r) a += sd[r][j] * s2[r][c];
    } else {
      const int j = i - o.b3;
      for (int r = 0; r < kRows; ++r) a += sd[r][j];
    }
    g[i] = a;
  }
}

__global__ void k_mlp_reduce(const float* __restrict__ partial, int nblk, int np,
                             float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * np + i];
  grad[i] = s;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g,
                       int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

}  // namespace

int64_t mlp_params(int k) { return offsets(k).total; }

int64_t mlp_work_floats(int64_t rows, int k) {
  return ((rows + kRows - 1) / kRows) * (int64_t)offsets(k).total;
}

hipError_t launch_mlp_forward(const float* p, const float* X, int64_t rows,
                              int k, float* Y, float* cache, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + kRows - 1) / kRows)),
                     dim3(kThreads), 0, s, p, X, rows, k, Y, cache);
  return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* Y, const float* T, int64_t total,
                           float* dY, float* loss, float* work, hipStream_t s) {
  if (total == 0) return hipSuccess;
  const int nblk = (int)((total + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_mlp_loss, dim3(nblk), dim3(kThreads), 0, s, Y, T, total, dY, work);
  hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, s, work, nblk, total, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* p, const float* X,
                               const float* cache, const float* dY,
                               int64_t rows, int k, float* grad, float* work,
                               hipStream_t s) {
  const int np = offsets(k).total;
  const int nblk = (int)((rows + kRows - 1) / kRows);
  if (nblk > 0)
    hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(kThreads), 0, s, p, X,
                       cache, dY, rows, k, work);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((np + 255) / 256), dim3(256), 0, s, work,
                     nblk, np, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n,
                       float lr, float b1, float b2, float eps, float bc1,
                       float bc2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     p, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace bltc
