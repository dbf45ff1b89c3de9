// Per-batch (n, theta) selection on the device: batch features, the
// allocation of an error budget over the batches, the judge's sums against
// the fallback, and the clusters a degree needs.
#include <hip/hip_runtime.h>

#include "bltc.h"
#include "internal.h"
#include "walk.h"

namespace bltc {

namespace {

constexpr int kSelWaves = 4;   // batches (waves) per work group of the walk kernels

__device__ __forceinline__ double wave_sumd(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Features of batch b, from its geometry and one walk at theta_ref (one
// wave-shared walk, walk.h; the lanes' sums are added across the wave):
//  0 log2 targets             1 log10 r_B / R0         2 log10 eps / R0
//  3 log10 eps / r_B          4 log10(1 + proxy clusters)
//  5 log10(1 + near sources)  6 log10(1 + near leaves)
//  7 mean log10 r_C / R0 over accepted clusters
//  8 mean (r_B + r_C) / (theta_ref R) over accepted clusters
//  9 log10 near-field density relative to the mean density
// 10 kernel (0 Stokeslet, 1 rotlet)  11 log10 n
// R0 is the root radius; lengths below 1e-12 R0 are floored.
__global__ __launch_bounds__(64 * kSelWaves) void k_features(FeatArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * kSelWaves + (threadIdx.x >> 6);
  if (b >= a.nb) return;
  const double4 g = a.bgeo[b];
  const double4 root = a.nodes.geo[0];
  const double R0 = root.w > 0.0 ? root.w : 1.0;
  const double tiny = 1e-12 * R0;
  const double th2 = a.theta_ref * a.theta_ref;
  double P = 0, L = 0, D = 0, slr = 0, stight = 0, vol = 0;
  cut_walk(a.nodes, g, th2, lane,
           [&](int32_t q, double R2, double rr) {
             P += 1;
             slr += log10((a.nodes.geo[q].w + tiny) / R0);
             stight += rr / (a.theta_ref * sqrt(R2));
           },
           [&](int32_t q) {
             const int2 rg = a.nodes.range[q];
             L += 1;
             D += rg.y - rg.x;
             const double* bx = a.box + 6 * (int64_t)q;
             vol += (bx[3] - bx[0] + tiny) * (bx[4] - bx[1] + tiny) * (bx[5] - bx[2] + tiny);
           });
  P = wave_sumd(P);
  L = wave_sumd(L);
  D = wave_sumd(D);
  slr = wave_sumd(slr);
  stight = wave_sumd(stight);
  vol = wave_sumd(vol);
  if (lane != 0) return;
  const double* rb = a.box;
  const double vroot = (rb[3] - rb[0] + tiny) * (rb[4] - rb[1] + tiny) * (rb[5] - rb[2] + tiny);
  const double mean_density = (double)(a.n_src > 0 ? a.n_src : 1) / vroot;
  const double cnt = (double)(a.bptr[b + 1] - a.bptr[b]);
  float f[kMlpIn];
  f[0] = (float)log2(cnt > 1 ? cnt : 1.0);
  f[1] = (float)log10((g.w + tiny) / R0);
  f[2] = (float)log10((a.eps + tiny) / R0);
  f[3] = (float)log10((a.eps + tiny) / (g.w + tiny));
  f[4] = (float)log10(1.0 + P);
  f[5] = (float)log10(1.0 + D);
  f[6] = (float)log10(1.0 + L);
  f[7] = P > 0 ? (float)(slr / P) : 0.f;
  f[8] = P > 0 ? (float)(stight / P) : 0.f;
  f[9] = (float)log10(((D + 1.0) / (vol + tiny * tiny * tiny)) / mean_density);
  f[10] = a.kernel == BLTC_ROTLET ? 1.f : 0.f;
  f[11] = (float)log10((double)(a.n_src > 0 ? a.n_src : 1));
  for (int i = 0; i < kMlpIn; ++i) {
    float v = f[i];
    if (a.mean) v = (v - a.mean[i]) / a.stdv[i];
    a.feat[b * kMlpIn + i] = v;
  }
}

// Modelled wave costs of the candidates (CostArgs): one wave-shared walk
// (walk.h) per batch and theta group (grid y).  An accepted cluster at
// ratio^2 qq = (rr/R)^2 costs (far n1 + row) n1^2 + clu with n1 - 1 the
// candidate's degree, or under the separation rule the first d >= deg_min
// with qq <= T[d].  Which degree every candidate of the group takes depends
// on qq only through its bucket among the group's distinct thresholds, so a
// cluster costs one binary search over them (staged in LDS) and one table
// row read per candidate; the host fills the table.  The candidate loop is
// unrolled to kMaxPerTheta so the sums stay in registers; the theta groups
// run in one launch so their walks overlap.
__global__ __launch_bounds__(64 * kSelWaves) void k_cand_costs(CostArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * kSelWaves + (threadIdx.x >> 6);
  const CostGroup& gr = a.grp[blockIdx.y];
  __shared__ double sU[kMaxBuckets];
  __shared__ float sC[kMaxPerTheta][kMaxBuckets + 1];
  const int nu = gr.nu;
  for (int i = threadIdx.x; i < nu; i += blockDim.x) sU[i] = a.U[gr.u_off + i];
  for (int i = threadIdx.x; i < gr.nc * (nu + 1); i += blockDim.x)
    sC[i / (nu + 1)][i % (nu + 1)] = a.C[gr.c_off + i];
  __syncthreads();
  if (b >= a.nb) return;
  const double4 g = a.bgeo[b];
  const double th2 = gr.theta * gr.theta;
  float far[kMaxPerTheta];
#pragma unroll
  for (int i = 0; i < kMaxPerTheta; ++i) far[i] = 0.f;
  double S = 0.0;
  cut_walk(a.nodes, g, th2, lane,
           [&](int32_t, double R2, double rr) {
             int k = 0;
             if (nu > 0) {
               // the number of thresholds below qq
               const double qq = (rr * rr) / R2;
               int hi = nu;
               while (k < hi) {
                 const int mid = (k + hi) >> 1;
                 if (sU[mid] < qq) k = mid + 1;
                 else hi = mid;
               }
             }
#pragma unroll
             for (int i = 0; i < kMaxPerTheta; ++i)
               if (i < gr.nc) far[i] += sC[i][k];
           },
           [&](int32_t q) {
             const int2 rg = a.nodes.range[q];
             S += rg.y - rg.x;
           });
  S = wave_sumd(S);
#pragma unroll
  for (int i = 0; i < kMaxPerTheta; ++i)
    for (int off = 32; off > 0; off >>= 1) far[i] += __shfl_xor(far[i], off);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < kMaxPerTheta; ++i)
      if (i < gr.nc) a.cost[(int64_t)gr.row[i] * a.nb + b] = far[i] + (float)S * a.nearf;
  }
}

// e2[j][b] = 10^(2 Y[b][j]): the predicted squared relative errors.
__global__ void k_pred_err2(const float* __restrict__ Y, int k, int64_t nb,
                            double* __restrict__ e2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * k) return;
  const int64_t b = i % nb, j = i / nb;
  e2[i] = exp10(2.0 * (double)Y[b * k + j]);
}

// The candidate minimising cost + lam wn e^2 with e = 10^Y the predicted
// relative error; ties go to the lower index.
__device__ __forceinline__ int best_candidate(const double* __restrict__ e2_jb, int k,
                                             int64_t nb, int64_t b,
                                             const float* __restrict__ cost_jb,
                                             double lw, double* cost, double* err2) {
  int best = 0;
  double bv = 0.0, bc = 0.0, be = 0.0;
  for (int j = 0; j < k; ++j) {
    const double e2 = e2_jb[(int64_t)j * nb + b];
    const double cj = (double)cost_jb[(int64_t)j * nb + b];
    const double v = cj + lw * e2;
    if (j == 0 || v < bv) {
      best = j;
      bv = v;
      bc = cj;
      be = e2;
    }
  }
  *cost = bc;
  *err2 = be;
  return best;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums (a, b) over the work group's threads in a fixed order.
template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double* out2) {
  __shared__ double red[2][NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < NT / 64; ++i) {
      sa += red[0][i];
      sb += red[1][i];
    }
    out2[0] = sa;
    out2[1] = sb;
  }
  __syncthreads();
}

constexpr int kSelThreads = 256;

// For every multiplier lam[g], g < G: each batch takes its best candidate
// for lam[g] wn_b (wn_b = wt[b] / sum wt); partial[blk][g] = (sum of cost,
// sum of wn e^2) over the work group's batches.
__global__ __launch_bounds__(kSelThreads) void k_alloc(
    const double* __restrict__ E2, int k, int64_t nb, const float* __restrict__ costs,
    const double* __restrict__ wt, double inv_wsum, const double* __restrict__ lam,
    int G, double* __restrict__ partial) {
  const int64_t b = (int64_t)blockIdx.x * kSelThreads + threadIdx.x;
  const bool act = b < nb;
  const double wn = act ? wt[b] * inv_wsum : 0.0;
  for (int g = 0; g < G; ++g) {
    double cost = 0.0, e2 = 0.0;
    if (act) best_candidate(E2, k, nb, b, costs, lam[g] * wn, &cost, &e2);
    block_sum2<kSelThreads>(cost, wn * e2, partial + ((int64_t)blockIdx.x * G + g) * 2);
  }
}

// Whole-run totals of every candidate j (one work group each): out[j] =
// (sum over batches of cost[j][b], sum of wn_b e2[j][b]), wn_b = wt[b] inv_wsum.
__global__ __launch_bounds__(kSelThreads) void k_cand_totals(
    const double* __restrict__ E2, int64_t nb, const float* __restrict__ costs,
    const double* __restrict__ wt, double inv_wsum, double* __restrict__ out) {
  const int j = blockIdx.x;
  double c = 0.0, e = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kSelThreads) {
    c += (double)costs[(int64_t)j * nb + b];
    e += wt[b] * inv_wsum * E2[(int64_t)j * nb + b];
  }
  block_sum2<kSelThreads>(c, e, out + 2 * j);
}

__global__ void k_choose(const double* __restrict__ E2, int k, int64_t nb,
                         const float* __restrict__ costs, const double* __restrict__ wt,
                         double inv_wsum, double lam, int32_t* __restrict__ choice) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double cost, e2;
  choice[b] = best_candidate(E2, k, nb, b, costs, lam * wt[b] * inv_wsum, &cost, &e2);
}

// Judge sums over the sampled targets: sample i lies in batch i * stride and
// stands for the group of batches [i * stride, (i + 1) * stride), which
// holds G_i targets:
//   usq[i]     = |u_fb|^2
//   contrib[i] = G_i |u - u_fb|^2   (when out is given, else 0)
// with u_fb the fallback treecode at the sample; partial[blk] = the work
// group's sums of (G_i |u_fb|^2, contrib).
__global__ __launch_bounds__(kSelThreads) void k_judge(
    int ns, int stride, int64_t nb, const int32_t* __restrict__ bptr,
    const int32_t* __restrict__ spos, const int32_t* __restrict__ tperm,
    const double* __restrict__ out, int64_t m, int od, const double* __restrict__ ufb,
    double* __restrict__ usq, double* __restrict__ contrib, double* __restrict__ partial) {
  const int i = blockIdx.x * kSelThreads + threadIdx.x;
  double wv = 0.0, cv = 0.0;
  if (i < ns) {
    const int64_t g0 = (int64_t)i * stride, g1 = g0 + stride < nb ? g0 + stride : nb;
    const double cnt = (double)(bptr[g1] - bptr[g0]);
    const int64_t o = out ? tperm[spos[i]] : 0;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < od; ++c) {
      const double r = ufb[(int64_t)i * od + c];
      den += r * r;
      if (out) {
        const double d = out[c * m + o] - r;
        num += d * d;
      }
    }
    wv = cnt * den;
    cv = cnt * num;
    usq[i] = den;
    contrib[i] = cv;
  }
  block_sum2<kSelThreads>(wv, cv, partial + (int64_t)blockIdx.x * 2);
}

// wt[b] = targets_b |u_fb|^2 of the sample standing for batch b.
__global__ void k_batch_weights(int64_t nb, int stride, const int32_t* __restrict__ bptr,
                                const double* __restrict__ usq, double* __restrict__ wt) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  wt[b] = (double)(bptr[b + 1] - bptr[b]) * usq[b / stride];
}

// out[c] = sum over blk of partial[blk][c], in work-group order.
__global__ void k_sum_columns(const double* __restrict__ partial, int nblk, int ncol,
                              double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * ncol + c];
  out[c] = s;
}

__global__ void k_flag(int ns, const double* __restrict__ contrib, double thr,
                       int32_t* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) flag[i] = contrib[i] > thr ? 1 : 0;
}

// mask[0] |= 1 << d for every degree d that the proxy lists of the batches
// bsel[0..nsel) carry (all batches when bsel is NULL); mask[0] starts at 0.
__global__ void k_degree_mask(const int32_t* __restrict__ bsel, int64_t nsel,
                              const int32_t* __restrict__ pptr,
                              const int32_t* __restrict__ pids, uint32_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsel) return;
  const int64_t b = bsel ? bsel[i] : i;
  uint32_t m = 0;
  for (int l = pptr[b]; l < pptr[b + 1]; ++l) m |= 1u << (pids[l] >> kDegShift);
  if (m) atomicOr(mask, m);
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_features(const FeatArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((a.nb + kSelWaves - 1) / kSelWaves)),
                     dim3(64 * kSelWaves), 0, s, a);
  return hipGetLastError();
}

int64_t alloc_blocks(int64_t nb) { return (nb + kSelThreads - 1) / kSelThreads; }

hipError_t launch_pred_err2(const float* Y, int k, int64_t nb, double* e2, hipStream_t s) {
  const int64_t tot = nb * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pred_err2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y, k,
                     nb, e2);
  return hipGetLastError();
}

hipError_t launch_alloc(const double* e2, int k, int64_t nb, const float* cost,
                        const double* wt, double inv_wsum, const double* lam, int G,
                        double* partial, double* sums, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  const int nblk = (int)alloc_blocks(nb);
  hipLaunchKernelGGL(k_alloc, dim3(nblk), dim3(kSelThreads), 0, s, e2, k, nb, cost, wt,
                     inv_wsum, lam, G, partial);
  hipLaunchKernelGGL(k_sum_columns, dim3((2 * G + 63) / 64), dim3(64), 0, s, partial, nblk,
                     2 * G, sums);
  return hipGetLastError();
}

hipError_t launch_cand_totals(const double* e2, int k, int64_t nb, const float* cost,
                              const double* wt, double inv_wsum, double* out, hipStream_t s) {
  if (nb == 0 || k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cand_totals, dim3(k), dim3(kSelThreads), 0, s, e2, nb, cost, wt,
                     inv_wsum, out);
  return hipGetLastError();
}

hipError_t launch_choose(const double* e2, int k, int64_t nb, const float* cost,
                         const double* wt, double inv_wsum, double lam, int32_t* choice,
                         hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_choose, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, e2, k, nb,
                     cost, wt, inv_wsum, lam, choice);
  return hipGetLastError();
}

hipError_t launch_judge(int ns, int stride, int64_t nb, const int32_t* bptr,
                        const int32_t* spos, const int32_t* tperm, const double* out,
                        int64_t m, int od, const double* ufb, double* usq, double* contrib,
                        double* partial, double* sums, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  const int nblk = (int)alloc_blocks(ns);
  hipLaunchKernelGGL(k_judge, dim3(nblk), dim3(kSelThreads), 0, s, ns, stride, nb, bptr, spos,
                     tperm, out, m, od, ufb, usq, contrib, partial);
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(64), 0, s, partial, nblk, 2, sums);
  return hipGetLastError();
}

hipError_t launch_batch_weights(int64_t nb, int stride, const int32_t* bptr,
                                const double* usq, double* wt, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_weights, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, nb,
                     stride, bptr, usq, wt);
  return hipGetLastError();
}

hipError_t launch_flag(int ns, const double* contrib, double thr, int32_t* flag,
                       hipStream_t s) {
  if (ns == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flag, dim3((ns + 255) / 256), dim3(256), 0, s, ns, contrib, thr, flag);
  return hipGetLastError();
}

hipError_t launch_cand_costs(const CostArgs& a, hipStream_t s) {
  if (a.nb == 0) return hipSuccess;
  if (a.ngroups < 1 || a.ngroups > kMaxThetaGroups) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cand_costs,
                     dim3((unsigned)((a.nb + kSelWaves - 1) / kSelWaves), (unsigned)a.ngroups),
                     dim3(64 * kSelWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_degree_mask(const int32_t* bsel, int64_t nsel, const int32_t* pptr,
                              const int32_t* pids, uint32_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t*)mask, (int64_t)1, 0);
  if (nsel > 0)
    hipLaunchKernelGGL(k_degree_mask, dim3((unsigned)((nsel + 127) / 128)), dim3(128), 0, s,
                       bsel, nsel, pptr, pids, mask);
  return hipGetLastError();
}

}  // namespace bltc
