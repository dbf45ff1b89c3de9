// Device-side kernel algebra shared by the evaluation kernels.
//
// With rho^2 = r^2 + eps^2 and inv = 1/rho, the MRS functions of
// eq. MRS_kernels become (substituting r^2 = rho^2 - eps^2 in the printed
// numerators; every function here omits the common 1/(8 pi)):
//   H1 = inv + eps^2 inv^3,   H2 = inv^3,   Q = 2 inv^3 + 3 eps^2 inv^5,
//   D1 = 15 eps^4 inv^7 - 3 eps^2 inv^5 - 2 inv^3,
//   D2 = 6 inv^5 + 15 eps^2 inv^7.
// pair() adds one interaction K(x, y) f to u for the difference d = x - y:
//   Stokeslet: u += f H1 + (f.d) d H2                       (eq. Velocity_1)
//   rotlet:    u += Q (n x d),  w += D1 n + D2 (n.d) d      (eq. MRS_2)
// (the 1/2 and 1/4 of the rotlet are applied with the 1/(8 pi) at the end).
// pair_full() adds both parts of eq. MRS_2 for a force f and a torque n:
//   u += f H1 + (f.d) d H2 + Q/2 (n x d)
//   w += Q/2 (f x d) + D1/4 n + D2/4 (n.d) d
// with the 1/2 and 1/4 folded into the coefficients.
#pragma once
#include <hip/hip_runtime.h>

namespace bltc {

enum { KSTOKES = 0, KROT = 1, KFULL = 2, KPOLY = 100 };

template <int KERN>
struct Dims {
  static constexpr int OD = (KERN == KROT || KERN == KFULL) ? 6 : 3;   // outputs
  static constexpr int WD = KERN == KFULL ? 6 : 3;                     // weights
};

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }
// FP64: the hardware estimate y (about 23 correct bits) and one second-order
// Newton step for 1/sqrt(v): with e = 1 - v y^2, 1/sqrt(v) = y (1 - e)^(-1/2)
// = y (1 + e/2 + 3e^2/8 + O(e^3)), and e^3 is below an FP64 ulp.  The
// argument is rho^2 >= eps^2 > 0, or r^2 > 0 when eps = 0 (inv_rho tests
// it), always positive and finite, so no special values are handled.
__device__ __forceinline__ double rsq(double v) {
  const double y = __builtin_amdgcn_rsq(v);
  const double e = __builtin_fma(-v * y, y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

template <bool ZEPS, typename T>
__device__ __forceinline__ T inv_rho(T r2) {
  if (ZEPS) return r2 > T(0) ? rsq(r2) : T(0);   // eps = 0: drop r = 0
  return rsq(r2);
}

// One interaction with difference d, rho^2 = r2, weights f; u += K f.
template <int KERN, bool ZEPS, typename T>
__device__ __forceinline__ void pair(T dx, T dy, T dz, T r2, T e2, T fx, T fy,
                                     T fz, T* u) {
  const T inv = inv_rho<ZEPS>(r2);
  const T inv2 = inv * inv;
  const T inv3 = inv2 * inv;
  if constexpr (KERN == KSTOKES) {
    const T fd = fz * dz + (fy * dy + fx * dx);
    const T h1 = e2 * inv3 + inv;
    const T s = fd * inv3;
    u[0] = fx * h1 + u[0];
    u[0] = dx * s + u[0];
    u[1] = fy * h1 + u[1];
    u[1] = dy * s + u[1];
    u[2] = fz * h1 + u[2];
    u[2] = dz * s + u[2];
  } else {  // rotlet: f holds the torque n
    const T inv5 = inv3 * inv2;
    const T inv7 = inv5 * inv2;
    const T q = T(3) * e2 * inv5 + (inv3 + inv3);
    const T d1 = T(15) * e2 * e2 * inv7 + (T(-3) * e2 * inv5 + T(-2) * inv3);
    const T d2 = T(15) * e2 * inv7 + T(6) * inv5;
    const T cx = fy * dz - fz * dy;
    const T cy = fz * dx - fx * dz;
    const T cz = fx * dy - fy * dx;
    const T nd = fz * dz + (fy * dy + fx * dx);
    const T g = d2 * nd;
    u[0] = q * cx + u[0];
    u[1] = q * cy + u[1];
    u[2] = q * cz + u[2];
    u[3] = d1 * fx + u[3];
    u[3] = g * dx + u[3];
    u[4] = d1 * fy + u[4];
    u[4] = g * dy + u[4];
    u[5] = d1 * fz + u[5];
    u[5] = g * dz + u[5];
  }
}

// Both parts of eq. MRS_2 for one pair: force (fx, fy, fz), torque
// (nx, ny, nz); u[0..2] velocity, u[3..5] angular velocity.
template <bool ZEPS, typename T>
__device__ __forceinline__ void pair_full(T dx, T dy, T dz, T r2, T e2, T fx, T fy,
                                          T fz, T nx, T ny, T nz, T* u) {
  const T inv = inv_rho<ZEPS>(r2);
  const T inv2 = inv * inv;
  const T inv3 = inv2 * inv;
  const T inv5 = inv3 * inv2;
  const T h1 = e2 * inv3 + inv;
  const T qh = (T(1.5) * e2 * inv2 + T(1)) * inv3;                              // Q/2
  const T d1q = (inv2 * (T(3.75) * e2 * e2 * inv2 + T(-0.75) * e2) + T(-0.5)) * inv3;  // D1/4
  const T d2q = (T(3.75) * e2 * inv2 + T(1.5)) * inv5;                          // D2/4
  const T s = (fz * dz + (fy * dy + fx * dx)) * inv3;
  const T g = (nz * dz + (ny * dy + nx * dx)) * d2q;
  u[0] = fx * h1 + u[0];
  u[0] = dx * s + u[0];
  u[0] = qh * (ny * dz - nz * dy) + u[0];
  u[1] = fy * h1 + u[1];
  u[1] = dy * s + u[1];
  u[1] = qh * (nz * dx - nx * dz) + u[1];
  u[2] = fz * h1 + u[2];
  u[2] = dz * s + u[2];
  u[2] = qh * (nx * dy - ny * dx) + u[2];
  u[3] = qh * (fy * dz - fz * dy) + u[3];
  u[3] = d1q * nx + u[3];
  u[3] = g * dx + u[3];
  u[4] = qh * (fz * dx - fx * dz) + u[4];
  u[4] = d1q * ny + u[4];
  u[4] = g * dy + u[4];
  u[5] = qh * (fx * dy - fy * dx) + u[5];
  u[5] = d1q * nz + u[5];
  u[5] = g * dz + u[5];
}

}  // namespace bltc
