// Direct sum on the device (eq. N-body): u(x_i) = sum_j K(x_i, y_j) f_j for a
// list of target indices against every source, sources in caller order.
// One thread per target; sources are staged 256 at a time through LDS and
// read by broadcast.  FP64, or FP32 evaluation (differences formed in FP64)
// with each 256-source tile folded into an FP64 accumulator.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bltc.h"
#include "internal.h"
#include "kmath.h"

namespace bltc {

namespace {

constexpr int kTile = 256;

template <int KERN, int PREC, bool ZEPS>
__global__ __launch_bounds__(kTile) void k_direct(
    const double* __restrict__ tx, const double* __restrict__ ty,
    const double* __restrict__ tz, const int64_t* __restrict__ idx, int64_t k,
    const double* __restrict__ sx, const double* __restrict__ sy,
    const double* __restrict__ sz, int64_t n, const double* __restrict__ w,
    double eps, int poly_p, double poly_c, double su, double sw,
    double* __restrict__ out) {
  constexpr int OD = Dims<KERN>::OD;
  constexpr int WD = Dims<KERN>::WD;
  constexpr bool F64 = PREC == BLTC_FP64;
  using T = typename std::conditional<F64, double, float>::type;
  __shared__ double sh[3 + WD][kTile];
  const int64_t i = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const bool active = i < k;
  const int64_t ti = active ? (idx ? idx[i] : i) : 0;
  const double x = tx[ti], y = ty[ti], z = tz[ti];
  const T e2 = (T)(eps * eps);
  double acc[OD];
#pragma unroll
  for (int c = 0; c < OD; ++c) acc[c] = 0.0;

  for (int64_t s0 = 0; s0 < n; s0 += kTile) {
    const int64_t j = s0 + threadIdx.x;
    if (j < n) {
      sh[0][threadIdx.x] = sx[j];
      sh[1][threadIdx.x] = sy[j];
      sh[2][threadIdx.x] = sz[j];
#pragma unroll
      for (int c = 0; c < WD; ++c) sh[3 + c][threadIdx.x] = w[c * n + j];
    }
    __syncthreads();
    const int cnt = (int)(n - s0 < kTile ? n - s0 : kTile);
    T p[OD];
#pragma unroll
    for (int c = 0; c < OD; ++c) p[c] = 0;
    for (int jj = 0; jj < cnt; ++jj) {
      if constexpr (KERN == KPOLY) {
        double dot = x * sh[0][jj];
        dot = dot + y * sh[1][jj];
        dot = dot + z * sh[2][jj];
        const double base = poly_c + dot;
        double v = 1.0;
        for (int e = 0; e < poly_p; ++e) v *= base;
        p[0] += (T)(v * sh[3][jj]);
        p[1] += (T)(v * sh[4][jj]);
        p[2] += (T)(v * sh[5][jj]);
      } else {
        const T dx = (T)(x - sh[0][jj]);
        const T dy = (T)(y - sh[1][jj]);
        const T dz = (T)(z - sh[2][jj]);
        const T r2 = dz * dz + (dy * dy + (dx * dx + e2));
        if constexpr (KERN == KFULL)
          pair_full<ZEPS, T>(dx, dy, dz, r2, e2, (T)sh[3][jj], (T)sh[4][jj], (T)sh[5][jj],
                             (T)sh[6][jj], (T)sh[7][jj], (T)sh[8][jj], p);
        else
          pair<KERN, ZEPS, T>(dx, dy, dz, r2, e2, (T)sh[3][jj], (T)sh[4][jj],
                              (T)sh[5][jj], p);
      }
    }
#pragma unroll
    for (int c = 0; c < OD; ++c) acc[c] += (double)p[c];
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < OD; ++c) out[c * k + i] = acc[c] * (c < 3 ? su : sw);
  }
}

template <int KERN, int PREC>
hipError_t run(const double* tx, const double* ty, const double* tz,
               const int64_t* idx, int64_t k, const double* sx,
               const double* sy, const double* sz, int64_t n, const double* w,
               double eps, int32_t pp, double pc, double su, double sw,
               double* out, hipStream_t s) {
  const unsigned nblk = (unsigned)((k + kTile - 1) / kTile);
  if (eps == 0.0)
    hipLaunchKernelGGL((k_direct<KERN, PREC, true>), dim3(nblk), dim3(kTile),
                       0, s, tx, ty, tz, idx, k, sx, sy, sz, n, w, eps, pp, pc,
                       su, sw, out);
  else
    hipLaunchKernelGGL((k_direct<KERN, PREC, false>), dim3(nblk), dim3(kTile),
                       0, s, tx, ty, tz, idx, k, sx, sy, sz, n, w, eps, pp, pc,
                       su, sw, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_direct(int kernel, int precision, const double* tx,
                         const double* ty, const double* tz,
                         const int64_t* idx, int64_t k, const double* sx,
                         const double* sy, const double* sz, int64_t n,
                         const double* w, double eps, int32_t poly_p,
                         double poly_c, double su, double sw, double* out,
                         hipStream_t s) {
  if (k == 0) return hipSuccess;
  const bool f64 = precision == BLTC_FP64;
  if (kernel == KPOLY)
    return run<KPOLY, BLTC_FP64>(tx, ty, tz, idx, k, sx, sy, sz, n, w, eps,
                                 poly_p, poly_c, su, sw, out, s);
  if (kernel == KSTOKES)
    return f64 ? run<KSTOKES, BLTC_FP64>(tx, ty, tz, idx, k, sx, sy, sz, n, w,
                                          eps, poly_p, poly_c, su, sw, out, s)
               : run<KSTOKES, BLTC_FP32_FP64ACC>(tx, ty, tz, idx, k, sx, sy,
                                                 sz, n, w, eps, poly_p, poly_c,
                                                 su, sw, out, s);
  if (kernel == KFULL)
    return f64 ? run<KFULL, BLTC_FP64>(tx, ty, tz, idx, k, sx, sy, sz, n, w,
                                        eps, poly_p, poly_c, su, sw, out, s)
               : run<KFULL, BLTC_FP32_FP64ACC>(tx, ty, tz, idx, k, sx, sy,
                                               sz, n, w, eps, poly_p, poly_c,
                                               su, sw, out, s);
  return f64 ? run<KROT, BLTC_FP64>(tx, ty, tz, idx, k, sx, sy, sz, n, w, eps,
                                     poly_p, poly_c, su, sw, out, s)
             : run<KROT, BLTC_FP32_FP64ACC>(tx, ty, tz, idx, k, sx, sy, sz, n,
                                            w, eps, poly_p, poly_c, su, sw,
                                            out, s);
}

}  // namespace bltc
