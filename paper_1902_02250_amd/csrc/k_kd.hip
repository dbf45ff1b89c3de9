// Balanced k-d target batches on the device.
//
// The rule (the same as the host builder's and the oracle's): a part of c
// targets with c > bs is cut along the longest side of its bounding box
// (the first axis among equals); the first part takes the bs floor(nb/2)
// smallest targets by (coordinate, index), nb = ceil(c / bs), the second the
// rest; a part of at most bs targets is a batch, its targets in index order.
// The sizes of all parts follow from c and bs alone, so the host lays out
// every level's parts; the device decides which targets go where.
//
// Large parts (above kKdLocal targets), one level at a time over all of
// them: bounding boxes from segment-aligned chunks (no atomics), the axis,
// then one sort of all positions by the key (part, coordinate, index) packed
// in 128 bits; afterwards every part's first bs floor(nb/2) positions hold
// its first child.  The sort is a bitonic network whose passes with a
// stride below kBitonicLocal run inside a work group in LDS.
// Small parts: one work group each finishes the recursion in LDS, sorting
// each sub-part by rank (every element counts the elements below it).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

constexpr int kBitonicLocal = 2048;    // elements per work group in the local passes
constexpr uint64_t kIdxMask = (1ull << 44) - 1;

// A double as an unsigned key with the same order (-0 taken as +0).
__device__ __forceinline__ uint64_t sortable(double v) {
  uint64_t b = __double_as_longlong(v);
  if (b == 0x8000000000000000ull) b = 0;
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ bool greater(uint64_t ah, uint64_t al, uint64_t bh, uint64_t bl) {
  return ah > bh || (ah == bh && al > bl);
}

__global__ void k_kd_init(uint64_t* __restrict__ hi, uint64_t* __restrict__ lo, int64_t m,
                          int64_t n2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n2) return;
  hi[p] = p < m ? 0ull : ~0ull;
  lo[p] = p < m ? (uint64_t)p : ~0ull;
}

// Per chunk (part, begin, end) of a part that is cut: min and max of x, y, z.
__global__ __launch_bounds__(256) void k_kd_bbox(const int4* __restrict__ chunks,
                                                 const int32_t* __restrict__ cut,
                                                 const uint64_t* __restrict__ lo,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 double* __restrict__ part) {
  __shared__ double red[6][256];
  const int4 ch = chunks[blockIdx.x];
  if (!cut[ch.x]) return;   // uniform over the block
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int p = ch.y + threadIdx.x; p < ch.z; p += blockDim.x) {
    const int64_t id = (int64_t)(lo[p] & kIdxMask);
    const double c[3] = {x[id], y[id], z[id]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a] = fmin(v[a], c[a]);
      v[3 + a] = fmax(v[3 + a], c[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + h]);
        red[3 + a][threadIdx.x] = fmax(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + h]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[(int64_t)blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Per part that is cut: its box from its chunks' and the cut axis.
__global__ void k_kd_axis(const int32_t* __restrict__ cut, const int32_t* __restrict__ cfirst,
                          int32_t nseg, const double* __restrict__ part,
                          int32_t* __restrict__ axis) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg || !cut[s]) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int c = cfirst[s]; c < cfirst[s + 1]; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], part[(int64_t)c * 6 + a]);
      hi[a] = fmax(hi[a], part[(int64_t)c * 6 + 3 + a]);
    }
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
  axis[s] = ax;
}

// Sort keys (part, coordinate on the part's axis, index); parts that are not
// cut take coordinate 0, which orders them by index.
__global__ __launch_bounds__(256) void k_kd_keys(const int4* __restrict__ chunks,
                                                 const int32_t* __restrict__ cut,
                                                 const int32_t* __restrict__ axis,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ z,
                                                 uint64_t* __restrict__ hi,
                                                 uint64_t* __restrict__ lo) {
  const int4 ch = chunks[blockIdx.x];
  const bool c = cut[ch.x] != 0;
  const int ax = c ? axis[ch.x] : 0;
  const double* __restrict__ coord = ax == 0 ? x : (ax == 1 ? y : z);
  for (int p = ch.y + threadIdx.x; p < ch.z; p += blockDim.x) {
    const uint64_t id = lo[p] & kIdxMask;
    const uint64_t ck = c ? sortable(coord[id]) : 0ull;
    hi[p] = ((uint64_t)ch.x << 44) | (ck >> 20);
    lo[p] = (ck << 44) | id;
  }
}

// One global pass of the bitonic network: stage k, stride j >= kBitonicLocal.
__global__ void k_bitonic_global(uint64_t* __restrict__ hi, uint64_t* __restrict__ lo,
                                 int64_t n2, int64_t k, int64_t j) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n2 / 2) return;
  const int64_t i = (t / j) * 2 * j + (t % j);
  const int64_t q = i + j;
  const bool asc = (i & k) == 0;
  const uint64_t ah = hi[i], al = lo[i], bh = hi[q], bl = lo[q];
  if (greater(ah, al, bh, bl) == asc) {
    hi[i] = bh;
    lo[i] = bl;
    hi[q] = ah;
    lo[q] = al;
  }
}

// The passes with strides below kBitonicLocal inside one work group: all
// stages up to kBitonicLocal (k0 = 0), or the tail of stage k0.
__global__ __launch_bounds__(kBitonicLocal / 2) void k_bitonic_local(uint64_t* __restrict__ hi,
                                                                     uint64_t* __restrict__ lo,
                                                                     int64_t k0) {
  __shared__ uint64_t sh[kBitonicLocal], sl[kBitonicLocal];
  const int64_t base = (int64_t)blockIdx.x * kBitonicLocal;
  const int t = threadIdx.x;
  sh[t] = hi[base + t];
  sl[t] = lo[base + t];
  sh[t + kBitonicLocal / 2] = hi[base + t + kBitonicLocal / 2];
  sl[t + kBitonicLocal / 2] = lo[base + t + kBitonicLocal / 2];
  __syncthreads();
  auto pass = [&](int64_t k, int j) {
    const int i = (t / j) * 2 * j + (t % j);
    const int q = i + j;
    const bool asc = ((base + i) & k) == 0;
    const uint64_t ah = sh[i], al = sl[i], bh = sh[q], bl = sl[q];
    if (greater(ah, al, bh, bl) == asc) {
      sh[i] = bh;
      sl[i] = bl;
      sh[q] = ah;
      sl[q] = al;
    }
    __syncthreads();
  };
  if (k0 == 0) {
    for (int64_t k = 2; k <= kBitonicLocal; k <<= 1)
      for (int j = (int)(k >> 1); j > 0; j >>= 1) pass(k, j);
  } else {
    for (int j = kBitonicLocal / 2; j > 0; j >>= 1) pass(k0, j);
  }
  hi[base + t] = sh[t];
  lo[base + t] = sl[t];
  hi[base + t + kBitonicLocal / 2] = sh[t + kBitonicLocal / 2];
  lo[base + t + kBitonicLocal / 2] = sl[t + kBitonicLocal / 2];
}

// One small part (start, count <= kKdLocal) per work group: the rest of the
// recursion in LDS; writes the batches' targets, in index order, to perm.
__global__ __launch_bounds__(512) void k_kd_local(const int2* __restrict__ parts,
                                                  const uint64_t* __restrict__ lo,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ z, int32_t bs,
                                                  int32_t* __restrict__ perm) {
  __shared__ double sc[3][kKdLocal];
  __shared__ int32_t sid[kKdLocal];
  __shared__ uint16_t ord[kKdLocal], tmp[kKdLocal];
  __shared__ int32_t stk[2][32];
  __shared__ int32_t top, cur_s, cur_c, cur_ax;
  __shared__ double red[6][512 / 64];
  const int2 pt = parts[blockIdx.x];
  const int c0 = pt.y;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int u = t; u < c0; u += nt) {
    const int64_t id = (int64_t)(lo[pt.x + u] & kIdxMask);
    sid[u] = (int32_t)id;
    sc[0][u] = x[id];
    sc[1][u] = y[id];
    sc[2][u] = z[id];
    ord[u] = (uint16_t)u;
  }
  if (t == 0) {
    stk[0][0] = 0;
    stk[1][0] = c0;
    top = 1;
  }
  __syncthreads();
  while (true) {
    if (t == 0) {
      --top;
      cur_s = stk[0][top];
      cur_c = stk[1][top];
    }
    __syncthreads();
    const int ss = cur_s, cc = cur_c;
    int ax = -1;   // -1: order by index (a batch)
    if (cc > bs) {
      // the sub-part's box and its longest side
      double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
      for (int u = t; u < cc; u += nt) {
        const int e = ord[ss + u];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          v[a] = fmin(v[a], sc[a][e]);
          v[3 + a] = fmax(v[3 + a], sc[a][e]);
        }
      }
      for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          v[a] = fmin(v[a], __shfl_xor(v[a], off));
          v[3 + a] = fmax(v[3 + a], __shfl_xor(v[3 + a], off));
        }
      if ((t & 63) == 0)
#pragma unroll
        for (int a = 0; a < 6; ++a) red[a][t >> 6] = v[a];
      __syncthreads();
      if (t == 0) {
        double lo3[3], hi3[3];
        for (int a = 0; a < 3; ++a) {
          lo3[a] = red[a][0];
          hi3[a] = red[3 + a][0];
          for (int w = 1; w < nt / 64; ++w) {
            lo3[a] = fmin(lo3[a], red[a][w]);
            hi3[a] = fmax(hi3[a], red[3 + a][w]);
          }
        }
        int a0 = 0;
        for (int a = 1; a < 3; ++a)
          if (hi3[a] - lo3[a] > hi3[a0] - lo3[a0]) a0 = a;
        cur_ax = a0;
      }
      __syncthreads();
      ax = cur_ax;
    }
    // rank sort of ord[ss, ss + cc) by (coordinate on ax, index), or by index
    for (int u = t; u < cc; u += nt) {
      const int e = ord[ss + u];
      const double ke = ax >= 0 ? sc[ax][e] : 0.0;
      const int32_t ie = sid[e];
      int r = 0;
      for (int v2 = 0; v2 < cc; ++v2) {
        const int f = ord[ss + v2];
        const double kf = ax >= 0 ? sc[ax][f] : 0.0;
        r += (kf < ke || (kf == ke && sid[f] < ie)) ? 1 : 0;
      }
      tmp[ss + r] = (uint16_t)e;
    }
    __syncthreads();
    for (int u = t; u < cc; u += nt) ord[ss + u] = tmp[ss + u];
    __syncthreads();
    if (t == 0 && cc > bs) {
      const int nb = (cc + bs - 1) / bs;
      const int left = bs * (nb / 2);
      stk[0][top] = ss + left;
      stk[1][top] = cc - left;
      stk[0][top + 1] = ss;
      stk[1][top + 1] = left;
      top += 2;
    }
    __syncthreads();
    const int remaining = top;   // read by every thread before thread 0 pops again
    __syncthreads();
    if (remaining == 0) break;
  }
  for (int u = t; u < c0; u += nt) perm[pt.x + u] = sid[ord[u]];
}

}  // namespace

hipError_t launch_kd_init(uint64_t* hi, uint64_t* lo, int64_t m, int64_t n2, hipStream_t s) {
  hipLaunchKernelGGL(k_kd_init, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, hi, lo, m,
                     n2);
  return hipGetLastError();
}

hipError_t launch_kd_level(const int4* chunks, int32_t nchunks, const int32_t* cut,
                           const int32_t* cfirst, int32_t nseg, const double* x,
                           const double* y, const double* z, double* part, int32_t* axis,
                           uint64_t* hi, uint64_t* lo, int64_t n2, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kd_bbox, dim3(nchunks), dim3(256), 0, s, chunks, cut, lo, x, y, z, part);
  hipLaunchKernelGGL(k_kd_axis, dim3((nseg + 255) / 256), dim3(256), 0, s, cut, cfirst, nseg,
                     part, axis);
  hipLaunchKernelGGL(k_kd_keys, dim3(nchunks), dim3(256), 0, s, chunks, cut, axis, x, y, z, hi,
                     lo);
  // the bitonic network over n2 (a power of two >= kBitonicLocal) keys
  hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(n2 / kBitonicLocal)),
                     dim3(kBitonicLocal / 2), 0, s, hi, lo, (int64_t)0);
  for (int64_t k = 2 * kBitonicLocal; k <= n2; k <<= 1) {
    for (int64_t j = k / 2; j >= kBitonicLocal; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((n2 / 2 + 255) / 256)), dim3(256), 0,
                         s, hi, lo, n2, k, j);
    hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(n2 / kBitonicLocal)),
                       dim3(kBitonicLocal / 2), 0, s, hi, lo, k);
  }
  return hipGetLastError();
}

hipError_t launch_kd_local(const int2* parts, int32_t nparts, const uint64_t* lo,
                           const double* x, const double* y, const double* z, int32_t bs,
                           int32_t* perm, hipStream_t s) {
  if (nparts == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kd_local, dim3(nparts), dim3(512), 0, s, parts, lo, x, y, z, bs, perm);
  return hipGetLastError();
}

}  // namespace bltc
