// Cluster-cluster variant of the treecode (the interpolation in the target
// variable that Section 9 names as the next step): kernels for the two parts
// that the particle-cluster path does not have.
//
//   k_dual_grid: potentials at a target cluster's Chebyshev grid points,
//       g_A[m] = sum_{C in CC(A)} sum_k K(t_m, s_k) fhat_C,k
//              + sum_{C in CP(A)} sum_{y in C} K(t_m, y) f_y,
//     one thread per grid point, 256 grid points per work group; the
//     proxies (or sources) of each C are staged through LDS 256 at a time
//     and read by broadcast.  FP32 evaluation with the coordinates taken
//     relative to A's center and each tile folded into FP64, or FP64.
//   k_dual_down: every target adds sum_m L_m(x) g_A[m] for the clusters A on
//     its list, with the tensor-product Lagrange basis on A's grid in the
//     barycentric form and the exact-hit rule of Algorithm 1 (FP64).
// The accepted particle-cluster and direct pairs of the dual traversal run
// through the particle-cluster evaluation kernel first; k_dual_down adds to
// its output.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <type_traits>

#include "bltc.h"
#include "internal.h"
#include "kmath.h"

namespace bltc {

namespace {

constexpr int kDualThreads = 256;

template <typename T>
__device__ __forceinline__ T poly_value(T dot, int pp, double pc) {
  const double base = pc + (double)dot;
  double v = 1.0;
  for (int e = 0; e < pp; ++e) v *= base;
  return (T)v;
}

// One pair for any kernel; f holds WD weights.
template <int KERN, bool ZEPS, typename T>
__device__ __forceinline__ void any_pair(T dx, T dy, T dz, T e2, const T* f, T* p,
                                         double tx, double ty, double tz, double sx, double sy,
                                         double sz, int pp, double pc) {
  if constexpr (KERN == KPOLY) {
    const double v = poly_value<double>(tx * sx + ty * sy + tz * sz, pp, pc);
    p[0] += (T)(v * (double)f[0]);
    p[1] += (T)(v * (double)f[1]);
    p[2] += (T)(v * (double)f[2]);
  } else {
    const T r2 = dz * dz + (dy * dy + (dx * dx + e2));
    if constexpr (KERN == KFULL)
      pair_full<ZEPS, T>(dx, dy, dz, r2, e2, f[0], f[1], f[2], f[3], f[4], f[5], p);
    else
      pair<KERN, ZEPS, T>(dx, dy, dz, r2, e2, f[0], f[1], f[2], p);
  }
}

template <int KERN, bool F64, bool ZEPS>
__global__ __launch_bounds__(kDualThreads) void k_dual_grid(DualGridArgs a) {
  constexpr int OD = Dims<KERN>::OD;
  constexpr int WD = Dims<KERN>::WD;
  using T = typename std::conditional<F64, double, float>::type;
  __shared__ T sP[3 + WD][kDualThreads];   // staged proxies or sources (relative to A)
  __shared__ double sPd[3][kDualThreads];  // FP64 positions for the polynomial kernel

  const int4 it = a.items[blockIdx.x];     // (grid slot gi, target node A, first point, -)
  const int gi = it.x, A = it.y;
  const int n1 = a.n1, P = n1 * n1 * n1;
  const int t = threadIdx.x;
  const int mm = it.z + t;
  const bool active = mm < P;
  const int m = active ? mm : 0;
  const double* __restrict__ tg = a.tgrid + (int64_t)A * 3 * n1;
  const double gx = tg[m / (n1 * n1)], gy = tg[n1 + (m / n1) % n1], gz = tg[2 * n1 + m % n1];
  const double4 cA = a.tgeo[A];
  const T xr = F64 ? (T)gx : (T)(gx - cA.x);
  const T yr = F64 ? (T)gy : (T)(gy - cA.y);
  const T zr = F64 ? (T)gz : (T)(gz - cA.z);
  const T e2 = (T)(a.eps * a.eps);
  double acc[OD];
#pragma unroll
  for (int c = 0; c < OD; ++c) acc[c] = 0.0;

  // tile loop shared by both lists: entries [0, ncc) are CC, the rest CP
  const int c0 = a.ccptr[gi], c1 = a.ccptr[gi + 1];
  const int p0 = a.cpptr[gi], p1 = a.cpptr[gi + 1];
  const int nent = (c1 - c0) + (p1 - p0);
  for (int e = 0; e < nent; ++e) {
    const bool cc = e < c1 - c0;
    const int C = cc ? a.ccids[c0 + e] : a.cpids[p0 + e - (c1 - c0)];
    const int cnt = cc ? P : a.srange[C].y - a.srange[C].x;
    const int j0 = cc ? 0 : a.srange[C].x;
    const double* __restrict__ sg = a.sgrid + (int64_t)C * 3 * n1;
    const double* __restrict__ fh = a.fhat + (int64_t)C * WD * P;
    for (int s0 = 0; s0 < cnt; s0 += kDualThreads) {
      const int tc = min(kDualThreads, cnt - s0);
      __syncthreads();   // the previous tile is consumed
      if (t < tc) {
        const int k = s0 + t;
        double px, py, pz;
        if (cc) {
          px = sg[k / (n1 * n1)];
          py = sg[n1 + (k / n1) % n1];
          pz = sg[2 * n1 + k % n1];
#pragma unroll
          for (int w = 0; w < WD; ++w) sP[3 + w][t] = (T)fh[(int64_t)w * P + k];
        } else {
          const int64_t j = j0 + k;
          px = a.ys[j];
          py = a.ys[a.n + j];
          pz = a.ys[2 * a.n + j];
#pragma unroll
          for (int w = 0; w < WD; ++w) sP[3 + w][t] = (T)a.w64[(int64_t)w * a.n + j];
        }
        if constexpr (KERN == KPOLY) {
          sPd[0][t] = px;
          sPd[1][t] = py;
          sPd[2][t] = pz;
        }
        sP[0][t] = F64 ? (T)px : (T)(px - cA.x);
        sP[1][t] = F64 ? (T)py : (T)(py - cA.y);
        sP[2][t] = F64 ? (T)pz : (T)(pz - cA.z);
      }
      __syncthreads();
      T p[OD];
#pragma unroll
      for (int c = 0; c < OD; ++c) p[c] = 0;
      for (int jj = 0; jj < tc; ++jj) {
        T f[WD];
#pragma unroll
        for (int w = 0; w < WD; ++w) f[w] = sP[3 + w][jj];
        if constexpr (KERN == KPOLY)
          any_pair<KERN, ZEPS, T>(0, 0, 0, e2, f, p, gx, gy, gz, sPd[0][jj], sPd[1][jj],
                                  sPd[2][jj], a.poly_p, a.poly_c);
        else
          any_pair<KERN, ZEPS, T>(xr - sP[0][jj], yr - sP[1][jj], zr - sP[2][jj], e2, f, p, 0,
                                  0, 0, 0, 0, 0, 0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < OD; ++c) acc[c] += (double)p[c];
    }
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < OD; ++c)
      a.g[((int64_t)gi * OD + c) * P + m] = acc[c] * (c < 3 ? a.scale_u : a.scale_w);
  }
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

// One lane per target of a batch: out += sum over the batch's down list.
template <int N1, int OD>
__global__ __launch_bounds__(64) void k_dual_down(DualDownArgs a) {
  constexpr int P = N1 * N1 * N1;
  const int b = blockIdx.x;
  const int t0 = a.bptr[b], t1 = a.bptr[b + 1];
  const int ti = t0 + (int)threadIdx.x;
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
    const double* __restrict__ g = a.g + (int64_t)gi * OD * P;
    for (int k1 = 0; k1 < N1; ++k1)
      for (int k2 = 0; k2 < N1; ++k2) {
        const double l12 = Lx[k1] * Ly[k2];
        const int r = (k1 * N1 + k2) * N1;
#pragma unroll
        for (int k3 = 0; k3 < N1; ++k3) {
          const double l = l12 * Lz[k3];
#pragma unroll
          for (int c = 0; c < OD; ++c) u[c] = fma(l, g[c * P + r + k3], u[c]);
        }
      }
  }
  const int64_t o = a.tperm[ti];
#pragma unroll
  for (int c = 0; c < OD; ++c) a.out[c * a.m + o] += u[c];
}

template <int KERN>
hipError_t grid_kern(const DualGridArgs& a, bool f64, hipStream_t s) {
  const bool z = a.eps == 0.0;
  auto go = [&](auto k) {
    hipLaunchKernelGGL(k, dim3((unsigned)a.nitems), dim3(kDualThreads), 0, s, a);
  };
  if (f64) {
    if (z) go(k_dual_grid<KERN, true, true>);
    else go(k_dual_grid<KERN, true, false>);
  } else {
    if (z) go(k_dual_grid<KERN, false, true>);
    else go(k_dual_grid<KERN, false, false>);
  }
  return hipGetLastError();
}

template <int OD>
hipError_t down_kern(const DualDownArgs& a, int n1, hipStream_t s) {
  switch (n1) {
#define BLTC_DN(N)                                                                        \
  case N:                                                                                 \
    hipLaunchKernelGGL((k_dual_down<N, OD>), dim3((unsigned)a.nb), dim3(64), 0, s, a);   \
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

hipError_t launch_dual_grid(int kernel, int precision, const DualGridArgs& a, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  const bool f64 = precision == BLTC_FP64;
  if (kernel == KSTOKES) return grid_kern<KSTOKES>(a, f64, s);
  if (kernel == KROT) return grid_kern<KROT>(a, f64, s);
  if (kernel == KFULL) return grid_kern<KFULL>(a, f64, s);
  if (kernel == KPOLY) return f64 ? grid_kern<KPOLY>(a, true, s) : hipErrorInvalidValue;
  return hipErrorInvalidValue;
}

hipError_t launch_dual_down(int odim, int n1, const DualDownArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  return odim == 6 ? down_kern<6>(a, n1, s) : down_kern<3>(a, n1, s);
}

}  // namespace bltc
