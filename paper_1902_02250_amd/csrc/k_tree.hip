// Device construction of the cluster tree (Section 6), level by level, with
// the same rules and the same FP64 expressions as the host builder, so the
// two trees are identical bit for bit:
//   * a cluster's box is the tight box of its particles (min and max are
//     exact in any order);
//   * a cluster holding more than leaf_max particles with l_max > 0 bisects
//     every side longer than l_max / sqrt(2) at 0.5 (lo + hi); a coordinate
//     below the midpoint goes low;
//   * its particles are partitioned stably by the code bx + 2 by + 4 bz, and
//     the split is kept only if two or more codes occur.
// A level's clusters are cut into chunks of at most kTreeChunk consecutive
// particles; each kernel below runs one work group per chunk.  The host
// reads back one histogram per chunk to number the children breadth first;
// the scatter kernel writes the splitting clusters' partitioned order into a
// second buffer, and their ranges are copied back.  Compiled with
// -ffp-contract=off.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

namespace {

constexpr int kTreeThreads = 256;
constexpr int kTreeWaves = kTreeThreads / 64;

__global__ void k_tree_init(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, int64_t n, double* __restrict__ c,
                            int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  c[i] = x[i];
  c[n + i] = y[i];
  c[2 * n + i] = z[i];
  perm[i] = (int32_t)i;
}

// Min and max of each axis over one chunk: cmm[chunk] = lo xyz, hi xyz.
__global__ __launch_bounds__(kTreeThreads) void k_tree_minmax(
    const int4* __restrict__ chunks, const double* __restrict__ c, int64_t n,
    double* __restrict__ cmm) {
  const int4 ck = chunks[blockIdx.x];   // (level node, begin, end, -)
  const int t = threadIdx.x;
  double mn[3], mx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) mn[a] = mx[a] = c[a * n + ck.y];
  for (int i = ck.y + t; i < ck.z; i += kTreeThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double v = c[a * n + i];
      mn[a] = v < mn[a] ? v : mn[a];
      mx[a] = v > mx[a] ? v : mx[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    for (int off = 32; off > 0; off >>= 1) {
      const double u = __shfl_xor(mn[a], off), w = __shfl_xor(mx[a], off);
      mn[a] = u < mn[a] ? u : mn[a];
      mx[a] = w > mx[a] ? w : mx[a];
    }
  __shared__ double sm[kTreeWaves][6];
  if ((t & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      sm[t >> 6][a] = mn[a];
      sm[t >> 6][3 + a] = mx[a];
    }
  __syncthreads();
  if (t < 6) {
    double v = sm[0][t];
    for (int w = 1; w < kTreeWaves; ++w) {
      const double u = sm[w][t];
      if (t < 3) v = u < v ? u : v;
      else v = u > v ? u : v;
    }
    cmm[(int64_t)blockIdx.x * 6 + t] = v;
  }
}

// One thread per cluster of the level: its box from its chunks, center,
// radius, and the split test.
__global__ void k_tree_nodes(const int32_t* __restrict__ cptr, const int2* __restrict__ range,
                             int nl, const double* __restrict__ cmm, int64_t leaf_max,
                             TreeLevelNode* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nl) return;
  TreeLevelNode o;
  const int c0 = cptr[k], c1 = cptr[k + 1];
  for (int a = 0; a < 3; ++a) {
    double lo = cmm[(int64_t)c0 * 6 + a], hi = cmm[(int64_t)c0 * 6 + 3 + a];
    for (int c = c0 + 1; c < c1; ++c) {
      const double u = cmm[(int64_t)c * 6 + a], w = cmm[(int64_t)c * 6 + 3 + a];
      lo = u < lo ? u : lo;
      hi = w > hi ? w : hi;
    }
    o.lo[a] = lo;
    o.hi[a] = hi;
  }
  double side[3], hsq[3];
  for (int a = 0; a < 3; ++a) {
    side[a] = o.hi[a] - o.lo[a];
    o.ctr[a] = 0.5 * (o.lo[a] + o.hi[a]);
    const double half = 0.5 * (o.hi[a] - o.lo[a]);
    hsq[a] = half * half;
  }
  o.rad = sqrt((hsq[0] + hsq[1]) + hsq[2]);
  const double m12 = side[1] < side[2] ? side[2] : side[1];
  const double lmax = side[0] < m12 ? m12 : side[0];
  const int64_t cnt = (int64_t)range[k].y - range[k].x;
  o.mask = 0;
  if (cnt > leaf_max && lmax > 0.0) {
    const double cut = lmax * 0.70710678118654752440;   // l_max / sqrt(2)
    for (int a = 0; a < 3; ++a)
      if (side[a] > cut) o.mask |= 1 << a;
  }
  out[k] = o;
}

__device__ __forceinline__ int tree_code(const double* __restrict__ c, int64_t n, int i,
                                         int mask, const double* ctr) {
  int cd = 0;
  if ((mask & 1) && !(c[i] < ctr[0])) cd |= 1;
  if ((mask & 2) && !(c[n + i] < ctr[1])) cd |= 2;
  if ((mask & 4) && !(c[2 * n + i] < ctr[2])) cd |= 4;
  return cd;
}

// Per-chunk histogram of the child codes (all in code 0 for clusters that do
// not try to split).
__global__ __launch_bounds__(kTreeThreads) void k_tree_codes(
    const int4* __restrict__ chunks, const double* __restrict__ c, int64_t n,
    const TreeLevelNode* __restrict__ nodes, int32_t* __restrict__ hist) {
  const int4 ck = chunks[blockIdx.x];
  const TreeLevelNode nd = nodes[ck.x];
  __shared__ int h[8];
  const int t = threadIdx.x;
  if (t < 8) h[t] = 0;
  __syncthreads();
  if (nd.mask == 0) {
    if (t == 0) h[0] = ck.z - ck.y;
  } else {
    for (int i = ck.y + t; i < ck.z; i += kTreeThreads)
      atomicAdd(&h[tree_code(c, n, i, nd.mask, nd.ctr)], 1);
  }
  __syncthreads();
  if (t < 8) hist[(int64_t)blockIdx.x * 8 + t] = h[t];
}

// Stable scatter of one chunk of a splitting cluster into the second
// buffer: a particle of code k goes to pos[k] plus the number of earlier
// particles of the chunk with code k.  Chunks of clusters that do not split
// (split flag 0) are left alone.
__global__ __launch_bounds__(kTreeThreads) void k_tree_scatter(
    const int4* __restrict__ chunks, const int32_t* __restrict__ pos, int64_t n,
    const TreeLevelNode* __restrict__ nodes, const double* __restrict__ cin,
    const int32_t* __restrict__ pin, double* __restrict__ cout, int32_t* __restrict__ pout) {
  const int4 ck = chunks[blockIdx.x];
  const int32_t* __restrict__ P = pos + (int64_t)blockIdx.x * 9;
  if (P[8] == 0) return;   // uniform over the work group
  const TreeLevelNode nd = nodes[ck.x];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  __shared__ int base[8];
  __shared__ int wtot[kTreeWaves][8];
  if (t < 8) base[t] = P[t];
  __syncthreads();
  for (int r0 = ck.y; r0 < ck.z; r0 += kTreeThreads) {
    const int i = r0 + t;
    const bool valid = i < ck.z;
    const int cd = valid ? tree_code(cin, n, i, nd.mask, nd.ctr) : 8;
    int rank = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t m = __ballot(cd == k);
      if (cd == k) rank = __popcll(m & lt);
      if (lane == 0) wtot[wid][k] = __popcll(m);
    }
    __syncthreads();
    if (valid) {
      int d = base[cd] + rank;
      for (int w = 0; w < wid; ++w) d += wtot[w][cd];
      if ((uint32_t)d < (uint32_t)n) {   // positions come from the host's plan
        pout[d] = pin[i];
        cout[d] = cin[i];
        cout[n + d] = cin[n + i];
        cout[2 * n + d] = cin[2 * n + i];
      }
    }
    __syncthreads();
    if (t < 8) {
      int s = 0;
      for (int w = 0; w < kTreeWaves; ++w) s += wtot[w][t];
      base[t] += s;
    }
    __syncthreads();
  }
}

// Copies the scattered chunks of splitting clusters back into the first
// buffer, which thus always holds every particle in the current tree order.
__global__ __launch_bounds__(kTreeThreads) void k_tree_copyback(
    const int4* __restrict__ chunks, const int32_t* __restrict__ pos, int64_t n,
    const double* __restrict__ cin, const int32_t* __restrict__ pin, double* __restrict__ cout,
    int32_t* __restrict__ pout) {
  const int4 ck = chunks[blockIdx.x];
  if (pos[(int64_t)blockIdx.x * 9 + 8] == 0) return;
  for (int i = ck.y + threadIdx.x; i < ck.z; i += kTreeThreads) {
    pout[i] = pin[i];
    cout[i] = cin[i];
    cout[n + i] = cin[n + i];
    cout[2 * n + i] = cin[2 * n + i];
  }
}

// Batch geometry: tight box of [bptr[b], bend[b]) in tree order; center and
// radius as for a cluster.
__global__ void k_batch_geo(const double* __restrict__ c, int64_t m,
                            const int32_t* __restrict__ bptr, const int32_t* __restrict__ bend,
                            int64_t nb, double4* __restrict__ geo) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int s = bptr[b], e = bend[b];
  double r[3], sq[3];
  for (int a = 0; a < 3; ++a) {
    double lo = c[a * m + s], hi = lo;
    for (int i = s + 1; i < e; ++i) {
      const double v = c[a * m + i];
      if (v < lo) lo = v;
      if (v > hi) hi = v;
    }
    r[a] = 0.5 * (lo + hi);
    const double h = 0.5 * (hi - lo);
    sq[a] = h * h;
  }
  geo[b] = make_double4(r[0], r[1], r[2], sqrt((sq[0] + sq[1]) + sq[2]));
}

}  // namespace

hipError_t launch_tree_init(const double* x, const double* y, const double* z, int64_t n,
                            double* c, int32_t* perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tree_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, z,
                     n, c, perm);
  return hipGetLastError();
}

hipError_t launch_tree_level(const int4* chunks, int64_t nch, const int32_t* cptr,
                             const int2* range, int nl, const double* c, int64_t n,
                             int64_t leaf_max, double* cmm, TreeLevelNode* nodes,
                             int32_t* hist, hipStream_t s) {
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tree_minmax, dim3((unsigned)nch), dim3(kTreeThreads), 0, s, chunks, c,
                     n, cmm);
  hipLaunchKernelGGL(k_tree_nodes, dim3((unsigned)((nl + 127) / 128)), dim3(128), 0, s, cptr,
                     range, nl, cmm, leaf_max, nodes);
  hipLaunchKernelGGL(k_tree_codes, dim3((unsigned)nch), dim3(kTreeThreads), 0, s, chunks, c, n,
                     nodes, hist);
  return hipGetLastError();
}

hipError_t launch_tree_scatter(const int4* chunks, int64_t nch, const int32_t* pos, int64_t n,
                               const TreeLevelNode* nodes, double* c, int32_t* perm,
                               double* tc, int32_t* tperm, hipStream_t s) {
  if (nch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tree_scatter, dim3((unsigned)nch), dim3(kTreeThreads), 0, s, chunks, pos,
                     n, nodes, c, perm, tc, tperm);
  hipLaunchKernelGGL(k_tree_copyback, dim3((unsigned)nch), dim3(kTreeThreads), 0, s, chunks, pos,
                     n, tc, tperm, c, perm);
  return hipGetLastError();
}

hipError_t launch_batch_geo(const double* c, int64_t m, const int32_t* bptr, const int32_t* bend,
                            int64_t nb, double4* geo, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_geo, dim3((unsigned)((nb + 127) / 128)), dim3(128), 0, s, c, m,
                     bptr, bend, nb, geo);
  return hipGetLastError();
}

}  // namespace bltc
