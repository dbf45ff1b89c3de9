// Particle-cluster evaluation over the batch interaction lists: the hot path.
//
// One 64-lane wave evaluates up to 64 targets of one batch (the targets are
// in tree order, so a batch is a compact group) against the batch's shared
// lists:
//   proxy list:  u += sum_k K(x, s_k) fhat_k      (eq. pc_approximation_3D)
//   direct list: u += sum_{y_j in L} K(x, y_j) f_j (eq. pc_interaction_3D)
// Every lane handles one target; all lanes walk the same list, so cluster
// data and sources are wave-uniform: grids and modified weights are read
// through scalar loads, leaf sources are staged through LDS and read by
// broadcast.  Consecutive leaves whose particle ranges touch are merged into
// one run.
//
// Far field: the grid is a tensor product, so the per-axis differences
// x - s_k1, y - s_k2, z - s_k3 are formed once per (target, cluster) in FP64
// and rounded to FP32; r^2 of a proxy then costs one add.
// Near field, FP32 modes: the target and the staged sources are rounded to
// FP32 relative to the batch center (the differences are formed in FP64), so
// the FP32 difference x - y carries an absolute error of order 1e-7 times
// the batch size instead of the domain size.
//
// Kernel algebra (eq. MRS_kernels with rho^2 = r^2 + eps^2, inv = 1/rho):
//   8 pi H1 = inv + eps^2 inv^3,          8 pi H2 = inv^3,
//   8 pi Q  = 2 inv^3 + 3 eps^2 inv^5,
//   8 pi D1 = 15 eps^4 inv^7 - 3 eps^2 inv^5 - 2 inv^3,
//   8 pi D2 = 6 inv^5 + 15 eps^2 inv^7,
// obtained by substituting r^2 = rho^2 - eps^2 in the printed forms; the
// 1/(8 pi), 1/2 and 1/4 factors are applied once per target at the end.
//
// Accumulation: FP64 mode sums in FP64; FP32 modes sum each tile (one
// cluster's proxies, or up to 64 staged sources) in FP32 and fold the tile
// into an FP64 accumulator (BLTC_FP32_FP64ACC) or an FP32 compensated pair
// (BLTC_FP32_KAHAN, Neumaier/Kahan TwoSum).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bltc.h"
#include "internal.h"
#include "kmath.h"

namespace bltc {

namespace {

// ---- far field ---------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// Sums K(x, s_k) fhat_k over one cluster's (n+1)^3 proxies into p.  The grid
// is a tensor product: a row (k1, k2) shares dx and dy, and a k3 column
// shares dz.  A term c_k d_k (c a scalar per proxy) is therefore summed as
//   dx * (row sum of c),  dy * (row sum of c),  sum_k3 dz_k3 * (column sum of c),
// so the d-weighted parts of the kernels cost one multiply-add per proxy and
// marginal instead of a product and a multiply-add per component.  Every
// sum runs over a grid row first (n+1 terms) and then over the rows, which
// keeps the FP32 rounding of a cluster's sum near that of n+1 + (n+1)^2
// additions instead of (n+1)^3.  The per-axis differences are
// formed once per (target, cluster): dz and dz^2 in registers (the k3 loop
// is unrolled), dy and (FP32) dy^2 in this lane's entries of an LDS table
// (sd[k2 * SdStride<T>]) because the k2 loop is not, so a grid row costs
// one LDS read instead of an FP64 difference, a conversion and a square.
// In FP64 the table holds dy alone and a row forms dy^2 + (dx^2 + eps^2)
// with one fused multiply-add, the same instruction count as the add it
// replaces: half the LDS per wave, which is what limits FP64 occupancy.
// LDS stride (elements) between grid rows of a lane's dy table: (dy, dy^2)
// pairs in FP32, dy alone in FP64, 64 lanes per row.
template <typename T>
constexpr int SdStride = sizeof(T) == 8 ? 64 : 128;

// dy^2 + (dx^2 + eps^2) of grid row k2
template <typename T>
__device__ __forceinline__ T row_r2(const T* __restrict__ sd, int k2, T dy, T dx2e) {
  if constexpr (sizeof(T) == 8) return fmat(dy, dy, dx2e);
  else return sd[k2 * SdStride<T> + 1] + dx2e;
}

template <int KERN, int N1, bool ZEPS, typename T, typename F>
__device__ __forceinline__ void proxies(double x, double y, double z,
                                        const double* __restrict__ g,
                                        const F* __restrict__ fh, T e2,
                                        T* __restrict__ sd, T* p) {
  T dz[N1], dz2[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    dz[k] = (T)(z - g[2 * N1 + k]);
    dz2[k] = dz[k] * dz[k];
    const T d = (T)(y - g[N1 + k]);
    sd[k * SdStride<T>] = d;
    if constexpr (sizeof(T) == 4) sd[k * SdStride<T> + 1] = d * d;
  }
  if constexpr (KERN == KSTOKES) {
    // u = sum f H1 + sum (f.d) H2 d,  H2 = inv^3
    T cz[N1];   // column sums of (f.d) inv^3
#pragma unroll
    for (int k = 0; k < N1; ++k) cz[k] = 0;
    for (int k1 = 0; k1 < N1; ++k1) {
      const T dx = (T)(x - g[k1]);
      const T dx2e = dx * dx + e2;
      for (int k2 = 0; k2 < N1; ++k2) {
        const T dy = sd[k2 * SdStride<T>];
        const T dxy2 = row_r2(sd, k2, dy, dx2e);
        const F* __restrict__ R = fh + (k1 * N1 + k2) * 3 * N1;   // [c][k3], c < 3
        T S = 0, ax = 0, ay = 0, az = 0;
#pragma unroll
        for (int k3 = 0; k3 < N1; ++k3) {
          const T fx = (T)R[k3], fy = (T)R[N1 + k3], fz = (T)R[2 * N1 + k3];
          const T inv = inv_rho<ZEPS>(dxy2 + dz2[k3]);
          const T inv3 = (inv * inv) * inv;
          const T fd = fz * dz[k3] + (fy * dy + fx * dx);
          const T h1 = e2 * inv3 + inv;
          ax = fmat(fx, h1, ax);
          ay = fmat(fy, h1, ay);
          az = fmat(fz, h1, az);
          S = fmat(fd, inv3, S);
          cz[k3] = fmat(fd, inv3, cz[k3]);
        }
        // row sums first: FP32 partials of (n+1) terms, then (n+1)^2 rows
        p[0] += fmat(dx, S, ax);
        p[1] += fmat(dy, S, ay);
        p[2] += az;
      }
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) p[2] = dz[k] * cz[k] + p[2];
  } else if constexpr (KERN == KFULL) {
    // u = sum f H1 + (f.d) H2 d + Q/2 (n x d),
    // w = sum Q/2 (f x d) + D1/4 n + D2/4 (n.d) d
    T cz[N1], cqx[N1], cqy[N1], cfx[N1], cfy[N1], cg[N1];   // column sums
#pragma unroll
    for (int k = 0; k < N1; ++k) cz[k] = cqx[k] = cqy[k] = cfx[k] = cfy[k] = cg[k] = 0;
    const T qa = T(1.5) * e2, d2a = T(3.75) * e2, d1a = T(3.75) * e2 * e2, d1b = T(-0.75) * e2;
    for (int k1 = 0; k1 < N1; ++k1) {
      const T dx = (T)(x - g[k1]);
      const T dx2e = dx * dx + e2;
      for (int k2 = 0; k2 < N1; ++k2) {
        const T dy = sd[k2 * SdStride<T>];
        const T dxy2 = row_r2(sd, k2, dy, dx2e);
        const F* __restrict__ R = fh + (k1 * N1 + k2) * 6 * N1;   // [c][k3], c < 6
        T ax = 0, ay = 0, az = 0, S = 0, Qx = 0, Qy = 0, Qz = 0;
        T Fx = 0, Fy = 0, Fz = 0, Wx = 0, Wy = 0, Wz = 0, G = 0;
#pragma unroll
        for (int k3 = 0; k3 < N1; ++k3) {
          const T fx = (T)R[k3], fy = (T)R[N1 + k3], fz = (T)R[2 * N1 + k3];
          const T nx = (T)R[3 * N1 + k3], ny = (T)R[4 * N1 + k3], nz = (T)R[5 * N1 + k3];
          const T inv = inv_rho<ZEPS>(dxy2 + dz2[k3]);
          const T inv2 = inv * inv;
          const T inv3 = inv2 * inv;
          const T inv5 = inv3 * inv2;
          const T h1 = e2 * inv3 + inv;                                 // H1
          const T qh = (qa * inv2 + T(1)) * inv3;                       // Q/2
          const T d1q = (inv2 * (d1a * inv2 + d1b) + T(-0.5)) * inv3;   // D1/4
          const T d2q = (d2a * inv2 + T(1.5)) * inv5;                   // D2/4
          const T fd = fz * dz[k3] + (fy * dy + fx * dx);
          const T nd = nz * dz[k3] + (ny * dy + nx * dx);
          ax = fmat(fx, h1, ax);
          ay = fmat(fy, h1, ay);
          az = fmat(fz, h1, az);
          S = fmat(fd, inv3, S);
          cz[k3] = fmat(fd, inv3, cz[k3]);
          Qx = fmat(qh, nx, Qx);
          Qy = fmat(qh, ny, Qy);
          Qz = fmat(qh, nz, Qz);
          cqx[k3] = fmat(qh, nx, cqx[k3]);
          cqy[k3] = fmat(qh, ny, cqy[k3]);
          Fx = fmat(qh, fx, Fx);
          Fy = fmat(qh, fy, Fy);
          Fz = fmat(qh, fz, Fz);
          cfx[k3] = fmat(qh, fx, cfx[k3]);
          cfy[k3] = fmat(qh, fy, cfy[k3]);
          Wx = fmat(d1q, nx, Wx);
          Wy = fmat(d1q, ny, Wy);
          Wz = fmat(d1q, nz, Wz);
          G = fmat(d2q, nd, G);
          cg[k3] = fmat(d2q, nd, cg[k3]);
        }
        // f x d and n x d split into the row's dx, dy and the column's dz
        p[0] += fmat(dx, S, ax) - dy * Qz;
        p[1] += fmat(dy, S, ay) + dx * Qz;
        p[2] += fmat(dy, Qx, az) - dx * Qy;
        p[3] += fmat(dx, G, Wx) - dy * Fz;
        p[4] += fmat(dy, G, Wy) + dx * Fz;
        p[5] += fmat(dy, Fx, Wz) - dx * Fy;
      }
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      p[0] = dz[k] * cqy[k] + p[0];
      p[1] = -dz[k] * cqx[k] + p[1];
      p[2] = dz[k] * cz[k] + p[2];
      p[3] = dz[k] * cfy[k] + p[3];
      p[4] = -dz[k] * cfx[k] + p[4];
      p[5] = dz[k] * cg[k] + p[5];
    }
  } else {
    // u = sum Q (n x d),  w = sum D1 n + sum D2 (n.d) d
    T cqx[N1], cqy[N1], cg[N1];   // column sums of Q nx, Q ny, D2 (n.d)
#pragma unroll
    for (int k = 0; k < N1; ++k) cqx[k] = cqy[k] = cg[k] = 0;
    const T q2 = T(3) * e2, d2c = T(15) * e2, d1a = T(15) * e2 * e2, d1b = T(-3) * e2;
    for (int k1 = 0; k1 < N1; ++k1) {
      const T dx = (T)(x - g[k1]);
      const T dx2e = dx * dx + e2;
      for (int k2 = 0; k2 < N1; ++k2) {
        const T dy = sd[k2 * SdStride<T>];
        const T dxy2 = row_r2(sd, k2, dy, dx2e);
        const F* __restrict__ R = fh + (k1 * N1 + k2) * 3 * N1;
        T qx = 0, qy = 0, qz = 0, G = 0, wx = 0, wy = 0, wz = 0;
#pragma unroll
        for (int k3 = 0; k3 < N1; ++k3) {
          const T nx = (T)R[k3], ny = (T)R[N1 + k3], nz = (T)R[2 * N1 + k3];
          const T inv = inv_rho<ZEPS>(dxy2 + dz2[k3]);
          const T inv2 = inv * inv;
          const T inv3 = inv2 * inv;
          const T inv5 = inv3 * inv2;
          const T q = (q2 * inv2 + T(2)) * inv3;                      // Q
          const T d1 = (inv2 * (d1a * inv2 + d1b) + T(-2)) * inv3;    // D1
          const T d2 = (d2c * inv2 + T(6)) * inv5;                    // D2
          const T nd = nz * dz[k3] + (ny * dy + nx * dx);
          qx = fmat(q, nx, qx);
          qy = fmat(q, ny, qy);
          qz = fmat(q, nz, qz);
          cqx[k3] = fmat(q, nx, cqx[k3]);
          cqy[k3] = fmat(q, ny, cqy[k3]);
          wx = fmat(d1, nx, wx);
          wy = fmat(d1, ny, wy);
          wz = fmat(d1, nz, wz);
          G = fmat(d2, nd, G);
          cg[k3] = fmat(d2, nd, cg[k3]);
        }
        // n x d = (ny dz - nz dy, nz dx - nx dz, nx dy - ny dx)
        p[0] = -dy * qz + p[0];
        p[1] = dx * qz + p[1];
        p[2] += dy * qx - dx * qy;
        p[3] += fmat(dx, G, wx);
        p[4] += fmat(dy, G, wy);
        p[5] += wz;
      }
    }
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      p[0] = dz[k] * cqy[k] + p[0];
      p[1] = -dz[k] * cqx[k] + p[1];
      p[5] = dz[k] * cg[k] + p[5];
    }
  }
}

// Polynomial test kernel (FP64): (c + x.s)^p with s the grid point.
template <int N1>
__device__ __forceinline__ void proxies_poly(double x, double y, double z,
                                             const double* __restrict__ g,
                                             const double* __restrict__ fh,
                                             int pp, double pc, double* p) {
  for (int k1 = 0; k1 < N1; ++k1)
    for (int k2 = 0; k2 < N1; ++k2) {
      const double* __restrict__ R = fh + (k1 * N1 + k2) * 3 * N1;
#pragma unroll
      for (int k3 = 0; k3 < N1; ++k3) {
        double dot = x * g[k1];
        dot = dot + y * g[N1 + k2];
        dot = dot + z * g[2 * N1 + k3];
        const double base = pc + dot;
        double v = 1.0;
        for (int e = 0; e < pp; ++e) v *= base;
        p[0] += v * R[k3];
        p[1] += v * R[N1 + k3];
        p[2] += v * R[2 * N1 + k3];
      }
    }
}

// The far field of a cluster whose degree (separation rule) is n1 - 1 for
// some n1 in [2, M]: one unrolled instance per degree, chosen by the
// wave-uniform n1.
template <int KERN, int M, bool ZEPS, typename T, typename F>
__device__ __forceinline__ void proxies_low(int n1, double x, double y, double z,
                                            const double* __restrict__ g,
                                            const F* __restrict__ fh, T e2,
                                            T* __restrict__ sd, T* p) {
  if constexpr (M >= 2) {
    if (n1 == M) {
      proxies<KERN, M, ZEPS, T, F>(x, y, z, g, fh, e2, sd, p);
      return;
    }
    proxies_low<KERN, M - 1, ZEPS, T, F>(n1, x, y, z, g, fh, e2, sd, p);
  }
}

template <int M>
__device__ __forceinline__ void proxies_poly_low(int n1, double x, double y, double z,
                                                 const double* __restrict__ g,
                                                 const double* __restrict__ fh, int pp,
                                                 double pc, double* p) {
  if constexpr (M >= 2) {
    if (n1 == M) {
      proxies_poly<M>(x, y, z, g, fh, pp, pc, p);
      return;
    }
    proxies_poly_low<M - 1>(n1, x, y, z, g, fh, pp, pc, p);
  }
}

// ---- accumulators --------------------------------------------------------------
template <int PREC, int OD>
struct Acc {
  double s[OD];
  float hi[OD], lo[OD];
  __device__ void init() {
#pragma unroll
    for (int c = 0; c < OD; ++c) { s[c] = 0.0; hi[c] = 0.f; lo[c] = 0.f; }
  }
  template <typename T>
  __device__ void fold(const T* p) {
#pragma unroll
    for (int c = 0; c < OD; ++c) {
      if (PREC == BLTC_FP32_KAHAN) {
        const float v = (float)p[c];
        const float t = hi[c] + v;
        const float bp = t - hi[c];
        lo[c] += (hi[c] - (t - bp)) + (v - bp);
        hi[c] = t;
      } else {
        s[c] += (double)p[c];
      }
    }
  }
  __device__ double get(int c) const {
    return PREC == BLTC_FP32_KAHAN ? (double)hi[c] + (double)lo[c] : s[c];
  }
};

// Blocks are dispatched round robin over the 8 XCDs; without a launch order
// each XCD takes a contiguous range of batches, so neighbouring batches,
// which share most of their lists, share an L2.  The evaluations pass their
// own order instead (bmap, by decreasing modelled work, dealt to the XCDs)
// with each XCD's range of it (xstart).
__device__ __forceinline__ int xcd_block(int blk, int nblk) {
  const int per = nblk / 8, rem = nblk % 8;
  const int xcd = blk % 8, idx = blk / 8;
  return xcd * per + min(xcd, rem) + idx;
}

// Orders this wave's LDS accesses: a wave's LDS instructions execute in
// program order, so only the compiler must be kept from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walks the direct list as maximal runs of contiguous particles.
struct Runs {
  const int32_t* __restrict__ ids;
  const int2* __restrict__ range;
  int li, le, rb, re;
  __device__ bool next() {
    if (li >= le) return false;
    const int2 r0 = range[ids[li]];
    rb = r0.x;
    re = r0.y;
    ++li;
    while (li < le) {
      const int2 r1 = range[ids[li]];
      if (r1.x != re) break;
      re = r1.y;
      ++li;
    }
    return true;
  }
};

// One wave per work group: a group's slot is held until its slowest wave
// ends, and batches differ widely in work, so waves are scheduled singly.
constexpr int kWavesPerBlock = 1;

// Wave gw serves targets
// [bptr[b] + 64 wv, ...) of batch b = gw / wpb, wv = gw % wpb.
// Per-degree grids and modified weights for entries that carry their own
// degree (separation rule).
struct DegTables {
  const double* grid[kMaxDegree + 1];
  const void* fh[kMaxDegree + 1];
};

template <int KERN, int PREC, int N1, bool ZEPS, bool RULE>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_p2p(
    const double* __restrict__ tx, int64_t m, const int32_t* __restrict__ tperm,
    const int32_t* __restrict__ bptr, const double4* __restrict__ bgeo,
    int nblk, int nwaves, int wpb, const int32_t* __restrict__ bmap,
    const int32_t* __restrict__ pptr,
    const int32_t* __restrict__ pids, const int32_t* __restrict__ dptr,
    const int32_t* __restrict__ dids, const int2* __restrict__ range,
    const double* __restrict__ grid, const float* __restrict__ fh32,
    const double* __restrict__ fh64, const double* __restrict__ ys,
    const float* __restrict__ w32, const double* __restrict__ w64, int64_t n,
    double eps, int poly_p, double poly_c, double su, double sw,
    double* __restrict__ out, DegTables dt, const int4* __restrict__ split,
    double* __restrict__ partial, const int32_t* __restrict__ xstart, int nslice,
    double* __restrict__ spart) {
  constexpr int OD = Dims<KERN>::OD;
  constexpr int WD = Dims<KERN>::WD;
  constexpr int NK = N1 * N1 * N1;
  constexpr bool F64 = PREC == BLTC_FP64;
  using T = typename std::conditional<F64, double, float>::type;
  __shared__ T sA[kWavesPerBlock][4][64];        // source x, y, z, weight 0
  __shared__ T sB[kWavesPerBlock][WD - 1][64];   // weights 1 .. WD-1
  // far field: each lane's dy (and, in FP32, dy^2) per grid row
  __shared__ T sY[kWavesPerBlock][N1][SdStride<T>];

  // the wave index is uniform across the wave; readfirstlane tells the
  // compiler so, which keeps everything derived from it in scalar registers
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int gw;
  if (xstart) {   // XCD x serves the waves [xstart[x], xstart[x + 1])
    const int xcd = blockIdx.x % 8;
    gw = xstart[xcd] + (int)(blockIdx.x / 8) * kWavesPerBlock + wid;
    if (gw >= xstart[xcd + 1]) return;
  } else {
    gw = xcd_block(blockIdx.x, nblk) * kWavesPerBlock + wid;
  }
  if (gw >= nwaves) return;
  int b, bi = 0, wv, sl = 0, pbeg, pend, dbeg, dend;
  if (split) {   // a slice of a batch's proxy list or of its direct list
    const int4 sp = split[gw];
    b = sp.x;
    wv = 0;
    const bool far = sp.w == 0;
    pbeg = far ? sp.y : 0;
    pend = far ? sp.z : 0;
    dbeg = far ? 0 : sp.y;
    dend = far ? 0 : sp.z;
  } else {   // slice sl of nslice equal parts of both lists (all of them at 1)
    const int per = wpb * nslice;
    bi = gw / per;
    const int rem = gw % per;
    b = bmap ? bmap[bi] : bi;
    wv = rem / nslice;
    sl = rem % nslice;
    const int p0 = pptr[b], p1 = pptr[b + 1], d0 = dptr[b], d1 = dptr[b + 1];
    pbeg = p0 + (int)((int64_t)(p1 - p0) * sl / nslice);
    pend = p0 + (int)((int64_t)(p1 - p0) * (sl + 1) / nslice);
    // the direct list is sliced by tiles in the near-field loop
    dbeg = d0;
    dend = d1;
  }
  const int t0 = bptr[b] + wv * 64, t1 = bptr[b + 1];
  if (t0 >= t1) return;
  const int ti = t0 + lane;
  const bool active = ti < t1;
  const int tc = active ? ti : t0;
  const double x = tx[tc], y = tx[m + tc], z = tx[2 * m + tc];
  const double4 cb = bgeo[b];
  const T e2 = (T)(eps * eps);
  T (*A)[64] = sA[wid];
  T (*B)[64] = sB[wid];
  T* sd = &sY[wid][0][lane * (SdStride<T> / 64)];

  Acc<PREC, OD> acc;
  acc.init();

  // far field
  for (int li = pbeg; li < pend; ++li) {
    const int e = pids[li];
    const int q = e & kIdMask;
    const int dd = e >> kDegShift;
    const int n1 = (RULE && dd) ? dd + 1 : N1;
    T p[OD];
#pragma unroll
    for (int c = 0; c < OD; ++c) p[c] = 0;
    if (n1 == N1) {
      const double* __restrict__ g = grid + (int64_t)q * 3 * N1;
      if constexpr (KERN == KPOLY)
        proxies_poly<N1>(x, y, z, g, fh64 + (int64_t)q * 3 * NK, poly_p, poly_c, p);
      else if constexpr (F64)
        proxies<KERN, N1, ZEPS, T, double>(x, y, z, g, fh64 + (int64_t)q * WD * NK, e2, sd, p);
      else
        proxies<KERN, N1, ZEPS, T, float>(x, y, z, g, fh32 + (int64_t)q * WD * NK, e2, sd, p);
    } else if (RULE && n1 >= 2 && n1 < N1) {
      const double* __restrict__ g = dt.grid[n1 - 1] + (int64_t)q * 3 * n1;
      const int64_t o = (int64_t)q * WD * n1 * n1 * n1;
      if constexpr (KERN == KPOLY)
        proxies_poly_low<N1 - 1>(n1, x, y, z, g, (const double*)dt.fh[n1 - 1] + o, poly_p,
                                 poly_c, p);
      else if constexpr (F64)
        proxies_low<KERN, N1 - 1, ZEPS, T, double>(n1, x, y, z, g,
                                                   (const double*)dt.fh[n1 - 1] + o, e2, sd, p);
      else
        proxies_low<KERN, N1 - 1, ZEPS, T, float>(n1, x, y, z, g,
                                                  (const float*)dt.fh[n1 - 1] + o, e2, sd, p);
    }
    acc.fold(p);
  }

  // near field: runs of contiguous leaf particles in chunks of 64; the next
  // chunk's sources are loaded into registers while the current one is
  // evaluated from LDS
  const T xr = F64 ? (T)x : (T)(x - cb.x);
  const T yr = F64 ? (T)y : (T)(y - cb.y);
  const T zr = F64 ? (T)z : (T)(z - cb.z);
  Runs it{dids, range, dbeg, dend, 0, 0};
  bool have = it.next();
  int s0 = it.rb, re = it.re;
  // slice sl of nslice: the tiles [tl, th) of the batch's tiles (each run of
  // contiguous leaves cut into tiles of 64 sources from its start), so every
  // tile is the unsliced one and slices change only the order of the FP64
  // sums
  int tiles_left = 0x7fffffff;
  if (nslice > 1 && !split) {
    int nt = 0;
    for (Runs c{dids, range, dbeg, dend, 0, 0}; c.next();) nt += (c.re - c.rb + 63) >> 6;
    const int tl = (int)((int64_t)nt * sl / nslice);
    tiles_left = (int)((int64_t)nt * (sl + 1) / nslice) - tl;
    if (tiles_left == 0) {
      have = false;
    } else {
      int t = 0;   // tiles before the current run
      while (have && t + ((it.re - it.rb + 63) >> 6) <= tl) {
        t += (it.re - it.rb + 63) >> 6;
        have = it.next();
      }
      s0 = it.rb + 64 * (tl - t);
      re = it.re;
    }
  }
  double py0 = 0, py1 = 0, py2 = 0;   // prefetched source (FP64 position)
  T pf[WD];                           // and weights
#pragma unroll
  for (int c = 0; c < WD; ++c) pf[c] = 0;
  auto fetch = [&](int start, int end) {
    const int j = start + lane;
    if (j < end) {
      py0 = ys[j];
      py1 = ys[n + j];
      py2 = ys[2 * n + j];
#pragma unroll
      for (int c = 0; c < WD; ++c) {
        if constexpr (F64) pf[c] = w64[c * n + j];
        else pf[c] = w32[c * n + j];
      }
    }
  };
  if (have) fetch(s0, re);
  while (have) {
    const int cnt = min(64, re - s0);
    if (lane < cnt) {
      if constexpr (F64) {
        A[0][lane] = py0;
        A[1][lane] = py1;
        A[2][lane] = py2;
      } else {
        A[0][lane] = (T)(py0 - cb.x);
        A[1][lane] = (T)(py1 - cb.y);
        A[2][lane] = (T)(py2 - cb.z);
      }
      A[3][lane] = pf[0];
#pragma unroll
      for (int c = 1; c < WD; ++c) B[c - 1][lane] = pf[c];
    }
    wave_lds_sync();
    int ns0 = s0 + 64, nre = re;
    bool nhave = --tiles_left > 0;
    if (nhave && ns0 >= re) {
      nhave = it.next();
      ns0 = it.rb;
      nre = it.re;
    }
    if (nhave) fetch(ns0, nre);
    T p[OD];
#pragma unroll
    for (int c = 0; c < OD; ++c) p[c] = 0;
    if constexpr (KERN == KPOLY) {
      for (int jj = 0; jj < cnt; ++jj) {
        double dot = x * (double)A[0][jj];
        dot = dot + y * (double)A[1][jj];
        dot = dot + z * (double)A[2][jj];
        const double base = poly_c + dot;
        double v = 1.0;
        for (int e = 0; e < poly_p; ++e) v *= base;
        p[0] += (T)(v * (double)A[3][jj]);
        p[1] += (T)(v * (double)B[0][jj]);
        p[2] += (T)(v * (double)B[1][jj]);
      }
    } else {
#pragma unroll 8
      for (int jj = 0; jj < cnt; ++jj) {
        const T dx = xr - A[0][jj];
        const T dy = yr - A[1][jj];
        const T dz = zr - A[2][jj];
        const T r2 = dz * dz + (dy * dy + (dx * dx + e2));
        if constexpr (KERN == KFULL)
          pair_full<ZEPS, T>(dx, dy, dz, r2, e2, A[3][jj], B[0][jj], B[1][jj], B[2][jj],
                             B[3][jj], B[4][jj], p);
        else
          pair<KERN, ZEPS, T>(dx, dy, dz, r2, e2, A[3][jj], B[0][jj], B[1][jj], p);
      }
    }
    acc.fold(p);
    wave_lds_sync();
    s0 = ns0;
    re = nre;
    have = nhave;
  }

  if (active) {
    if (split) {
#pragma unroll
      for (int c = 0; c < OD; ++c) partial[((int64_t)gw * OD + c) * 64 + lane] = acc.get(c);
    } else if (nslice > 1) {
      const int64_t u = ((int64_t)bi * wpb + wv) * nslice + sl;   // by launch position
#pragma unroll
      for (int c = 0; c < OD; ++c) spart[(u * OD + c) * 64 + lane] = acc.get(c);
    } else {
      const int64_t o = tperm[ti];
#pragma unroll
      for (int c = 0; c < OD; ++c) out[c * m + o] = acc.get(c) * (c < 3 ? su : sw);
    }
  }
}

// Sums the slices of each split batch in slice order and scatters.
__global__ void k_split_reduce(const int32_t* __restrict__ sptr, const int32_t* __restrict__ bmap,
                               int64_t nr, const int32_t* __restrict__ bptr,
                               const int32_t* __restrict__ tperm, const double* __restrict__ partial,
                               int od, double su, double sw, int64_t m, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr * 64) return;
  const int64_t r = i / 64;
  const int lane = (int)(i % 64);
  const int b = bmap[r];
  const int t = bptr[b] + lane;
  if (t >= bptr[b + 1]) return;
  const int64_t o = tperm[t];
  for (int c = 0; c < od; ++c) {
    double v = 0.0;
    for (int sl = sptr[r]; sl < sptr[r + 1]; ++sl) v += partial[((int64_t)sl * od + c) * 64 + lane];
    out[c * m + o] = v * (c < 3 ? su : sw);
  }
}

// Sums the slices of each (launch position, wave) in slice order and
// scatters to the targets of the batch at that position.
__global__ void k_slice_reduce(const int32_t* __restrict__ bmap, int64_t n,
                               const int32_t* __restrict__ bptr, int wpb, int nslice,
                               const int32_t* __restrict__ tperm,
                               const double* __restrict__ spart, int od, double su, double sw,
                               int64_t m, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * wpb * 64) return;
  const int64_t r = i / (64 * wpb);
  const int wv = (int)(i / 64 % wpb);
  const int lane = (int)(i % 64);
  const int b = bmap ? bmap[r] : (int)r;
  const int t = bptr[b] + wv * 64 + lane;
  if (t >= bptr[b + 1]) return;
  const int64_t o = tperm[t];
  const int64_t u0 = (r * wpb + wv) * nslice;
  for (int c = 0; c < od; ++c) {
    double v = 0.0;
    for (int j = 0; j < nslice; ++j) v += spart[((u0 + j) * od + c) * 64 + lane];
    out[c * m + o] = v * (c < 3 ? su : sw);
  }
}

template <int KERN, int PREC, int N1>
hipError_t run_p2p(const P2PArgs& a, hipStream_t s) {
  const int nslice = a.split ? 1 : a.slices;
  if (nslice < 1 || (nslice > 1 && !a.spart)) return hipErrorInvalidValue;
  const int64_t nw64 =
      a.split ? a.nsplit : (a.bmap ? a.nmap : a.nb) * (int64_t)a.wpb * nslice;
  if (nw64 == 0) return hipSuccess;
  if (nw64 > 0x7fffffff - kWavesPerBlock) return hipErrorInvalidValue;
  const int nwaves = (int)nw64;
  // with work-balanced XCD ranges: 8 x the longest range's blocks
  const int nblk = a.xstart ? 8 * ((a.xmax + kWavesPerBlock - 1) / kWavesPerBlock)
                            : (nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (nblk == 0) return hipSuccess;
  const bool zeps = a.eps == 0.0;
  DegTables dt;
  bool rule = false;
  for (int d = 0; d <= kMaxDegree; ++d) {
    dt.grid[d] = a.grid_d[d];
    dt.fh[d] = a.fhat_d[d];
    if (d < N1 - 1 && a.grid_d[d]) rule = true;
  }
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(64 * kWavesPerBlock), 0, s, a.tx, a.m,
                       a.tperm, a.bptr, a.bgeo, nblk, nwaves, a.wpb, a.bmap, a.pptr, a.pids,
                       a.dptr, a.dids, a.range, a.grid, (const float*)a.fhat,
                       (const double*)a.fhat, a.ys, a.w32, a.w64, a.n, a.eps,
                       a.poly_p, a.poly_c, a.scale_u, a.scale_w, a.out, dt, a.split, a.partial,
                       a.xstart, nslice, a.spart);
  };
  if (rule) {
    if (zeps)
      go(k_p2p<KERN, PREC, N1, true, true>);
    else
      go(k_p2p<KERN, PREC, N1, false, true>);
  } else {
    if (zeps)
      go(k_p2p<KERN, PREC, N1, true, false>);
    else
      go(k_p2p<KERN, PREC, N1, false, false>);
  }
  return hipGetLastError();
}

template <int KERN, int PREC>
hipError_t dispatch_degree(int degree, const P2PArgs& a, hipStream_t s) {
  switch (degree + 1) {
#define BLTC_P2P(N) \
  case N:           \
    return run_p2p<KERN, PREC, N>(a, s);
    BLTC_P2P(2) BLTC_P2P(3) BLTC_P2P(4) BLTC_P2P(5) BLTC_P2P(6) BLTC_P2P(7)
    BLTC_P2P(8) BLTC_P2P(9) BLTC_P2P(10) BLTC_P2P(11) BLTC_P2P(12) BLTC_P2P(13)
#undef BLTC_P2P
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

#if defined(BLTC_P2P_KERN) && defined(BLTC_P2P_PREC)
// This object holds the kernels of one (kernel, precision) pair: the source
// is compiled once per pair (with -DBLTC_P2P_KERN and -DBLTC_P2P_PREC) so the
// template matrix builds in parallel, and once without them for the
// dispatcher below.
#define BLTC_P2P_NAME2(k, p) p2p_k##k##_p##p
#define BLTC_P2P_NAME(k, p) BLTC_P2P_NAME2(k, p)
hipError_t BLTC_P2P_NAME(BLTC_P2P_KERN, BLTC_P2P_PREC)(int degree, const P2PArgs& a,
                                                      hipStream_t s) {
  return dispatch_degree<BLTC_P2P_KERN, BLTC_P2P_PREC>(degree, a, s);
}
#else
// one entry per (kernel, precision) pair, each in its own object
hipError_t p2p_k0_p0(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k0_p1(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k0_p2(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k1_p0(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k1_p1(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k1_p2(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k2_p0(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k2_p1(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k2_p2(int degree, const P2PArgs& a, hipStream_t s);
hipError_t p2p_k100_p0(int degree, const P2PArgs& a, hipStream_t s);
static_assert(KSTOKES == 0 && KROT == 1 && KFULL == 2 && KPOLY == 100 && BLTC_FP64 == 0 &&
                  BLTC_FP32_FP64ACC == 1 && BLTC_FP32_KAHAN == 2,
              "the entry names follow the kernel and precision codes");

hipError_t launch_split_reduce(const int32_t* sptr, const int32_t* bmap, int64_t nr,
                               const int32_t* bptr, const int32_t* tperm, const double* partial,
                               int odim, double su, double sw, int64_t m, double* out,
                               hipStream_t s) {
  if (nr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((nr * 64 + 255) / 256)), dim3(256), 0, s,
                     sptr, bmap, nr, bptr, tperm, partial, odim, su, sw, m, out);
  return hipGetLastError();
}

hipError_t launch_slice_reduce(const int32_t* bmap, int64_t n, const int32_t* bptr, int wpb,
                               int slices, const int32_t* tperm, const double* spart, int odim,
                               double su, double sw, int64_t m, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t th = n * wpb * 64;
  hipLaunchKernelGGL(k_slice_reduce, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, s, bmap,
                     n, bptr, wpb, slices, tperm, spart, odim, su, sw, m, out);
  return hipGetLastError();
}

hipError_t launch_p2p(int kernel, int precision, int degree, const P2PArgs& a,
                      hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  if (kernel == KPOLY) {
    if (precision != BLTC_FP64) return hipErrorInvalidValue;
    return p2p_k100_p0(degree, a, s);
  }
  if (kernel == KSTOKES) {
    if (precision == BLTC_FP64) return p2p_k0_p0(degree, a, s);
    if (precision == BLTC_FP32_FP64ACC) return p2p_k0_p1(degree, a, s);
    return p2p_k0_p2(degree, a, s);
  }
  if (kernel == KFULL) {
    if (precision == BLTC_FP64) return p2p_k2_p0(degree, a, s);
    if (precision == BLTC_FP32_FP64ACC) return p2p_k2_p1(degree, a, s);
    return p2p_k2_p2(degree, a, s);
  }
  if (precision == BLTC_FP64) return p2p_k1_p0(degree, a, s);
  if (precision == BLTC_FP32_FP64ACC) return p2p_k1_p1(degree, a, s);
  return p2p_k1_p2(degree, a, s);
}
#endif

}  // namespace bltc
