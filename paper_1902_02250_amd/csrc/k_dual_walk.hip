// The dual traversal of the cluster-cluster variant (the interpolation in
// the target variable that Section 9 names as the next step), on the device.
//
// The traversal visits pairs (A, C) of a target and a source cluster from
// (root, root).  For a pair:
//   MAC (R2 > 0 and (r_A + r_C)^2 <= theta^2 R2): CC if both hold more than
//   P = (n+1)^3 particles, PC if only C does, CP if only A does, else PP;
//   no MAC and both leaves: PP; otherwise refine A (its children with C) if
//   C is a leaf or (A is not a leaf and r_A >= r_C), else refine C.
// Seen from one target node A with root path A_0 .. A_k = A, the pairs that
// involve the path form a walk over the source tree whose state is the level
// i of the path: refining A moves to (A_{i+1}, C) with the same C, refining
// C visits (A_i, C') for its children C'.  So every target node (or leaf)
// can walk the source tree on its own, depth first, and meets its pairs in
// the order of the serial traversal.  The 64 lanes of the wave share the
// walk over the source tree's cut as the batch walk does (walk.h): a lane
// replays the chain of its cut node's ancestors from the root pair (the
// level advances on the way exactly as in the serial walk), reports a
// terminal pair above the cut once, from the first cut node under it, and
// otherwise walks the cut node's subtree, keeping for every source depth the
// level at which that depth's nodes are entered.
//
// Per-node mode: the pairs at the node's own level: its CC and CP lists (in
// traversal order) and the evaluation counts.  Per-leaf mode: the PC and PP
// pairs at every level of the leaf's path, which are the leaf's far and near
// lists.  All decisions are FP64 comparisons rounded as written (no
// contraction), those of the traversal the oracle runs.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "walk.h"

namespace bltc {

namespace {

enum { kCC = 0, kPC = 1, kCP = 2, kPP = 3, kRefineA = 4, kRefineC = 5 };

struct Tgt {          // one level of the target path
  double4 g;
  int64_t n;
  int32_t leaf;
};

// The traversal's decision for the pair (target level t, source node C);
// *deg is the source side's degree (the rule's, else n), *nc C's count.
__device__ __forceinline__ int decide(const DualArgs& a, const Tgt& t, int32_t C, int* deg,
                                      int64_t* nc) {
#pragma clang fp contract(off)
  const double4 gc = a.src.geo[C];
  const int2 rc = a.src.range[C];
  *nc = rc.y - rc.x;
  const double dx = t.g.x - gc.x;
  const double dy = t.g.y - gc.y;
  const double dz = t.g.z - gc.z;
  const double R2 = dx * dx + dy * dy + dz * dz;
  const double rr = t.g.w + gc.w;
  const bool mac = R2 > 0.0 && rr * rr <= a.th2 * R2;
  const bool leafC = a.src.kids[C].y == 0;
  int d = a.n1 - 1;
  if (mac && a.rule.deg_min > 0) {
    const double qq = (rr * rr) / R2;
    d = a.rule.deg_min;
    while (d < a.rule.degree && !(qq <= a.rule.T[d])) ++d;
  }
  *deg = d;
  if (mac && t.n > a.P && *nc > a.P) return kCC;
  if (mac && *nc > a.P) return kPC;
  if (mac && t.n > a.P) return kCP;
  if (mac || (t.leaf && leafC)) return kPP;
  if (leafC || (!t.leaf && t.g.w >= gc.w)) return kRefineA;
  return kRefineC;
}

// Levels at which the nodes of each source depth are entered, 8 bits each.
struct LevelStack {
  uint64_t w[kDualMaxDepth / 8] = {0, 0, 0, 0};
  __device__ __forceinline__ void set(int d, int v) {
    const int k = d >> 3, sh = (d & 7) * 8;
#pragma unroll
    for (int j = 0; j < kDualMaxDepth / 8; ++j)
      if (j == k) w[j] = (w[j] & ~(0xffull << sh)) | ((uint64_t)v << sh);
  }
  __device__ __forceinline__ int get(int d) const {
    const int k = d >> 3, sh = (d & 7) * 8;
    uint64_t x = 0;
#pragma unroll
    for (int j = 0; j < kDualMaxDepth / 8; ++j)
      if (j == k) x = w[j];
    return (int)((x >> sh) & 0xff);
  }
};

__device__ __forceinline__ int32_t wave_excl(int32_t v, int lane) {
  int32_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  return inc - v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <bool LEAF, bool FILL>
__global__ __launch_bounds__(64) void k_dual_walk(DualArgs a) {
  __shared__ Tgt sT[kDualMaxDepth];
  __shared__ int32_t sK;
  const int64_t it = blockIdx.x;
  if (it >= a.nitems) return;
  const int lane = threadIdx.x;
  const int32_t A = LEAF ? a.items[it] : (int32_t)it;
  if (lane == 0) {   // the target's root path, root first
    int k = 0;
    for (int32_t q = A; q >= 0; q = a.tparent[q]) ++k;
    int j = k - 1;
    for (int32_t q = A; q >= 0; q = a.tparent[q], --j) {
      const int2 r = a.trange[q];
      sT[j].g = a.tgeo[q];
      sT[j].n = r.y - r.x;
      sT[j].leaf = a.tkids[q].y == 0;
    }
    sK = k - 1;
  }
  __syncthreads();
  const int kk = sK;
  const bool rule = a.rule.deg_min > 0;
  int32_t n0 = 0, n1 = 0;
  int64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  int32_t* out0 = nullptr;
  int32_t* out1 = nullptr;
  bool wr = false;   // second walk of the fill pass: write
  // a terminal pair (level i, source node C)
  auto emit = [&](int dec, int i, int32_t C, int deg, int64_t nc) {
    if (LEAF) {
      if (dec == kPC) {
        if (wr) *out0++ = rule ? (C | (deg << kDegShift)) : C;
        else ++n0;
      } else if (dec == kPP) {
        if (wr) *out1++ = C;
        else ++n1;
      }
      return;
    }
    if (i != kk) return;   // an ancestor's pair
    const int64_t Pd = (int64_t)(deg + 1) * (deg + 1) * (deg + 1);
    if (dec == kCC) {
      if (wr) *out0++ = rule ? (C | (deg << kDegShift)) : C;
      else { ++n0; w0 += a.P * Pd; }
    } else if (dec == kCP) {
      if (wr) *out1++ = C;
      else { ++n1; w2 += a.P * nc; }
    } else if (dec == kPC) {
      w1 += sT[kk].n * Pd;
    } else {
      w3 += sT[kk].n * nc;
    }
  };
  // decide at (level i, C), refining the target while the traversal does;
  // kRefineA comes back when the pair passes below the walk's own node
  auto step = [&](int* i, int32_t C, int* deg, int64_t* nc) {
    int dec;
    while (true) {
      dec = decide(a, sT[*i], C, deg, nc);
      if (dec != kRefineA || *i == kk) break;
      ++*i;
    }
    return dec;
  };
  auto walk = [&]() {
    int c0, c1;
    cut_chunk(a.src, lane, &c0, &c1);
    LevelStack lv;
    for (int c = c0; c < c1; ++c) {
      const int32_t root = a.src.cut[c];
      const uint32_t first = a.src.cut_first[c];
      const int32_t* anc = a.src.cut_anc + (int64_t)c * kCutMaxDepth;
      int i = 0;
      bool subtree = false;
      for (int j = 0; j <= kCutMaxDepth; ++j) {
        const bool at_cut = j == kCutMaxDepth || anc[j] < 0;
        const int32_t s = at_cut ? root : anc[j];
        int deg;
        int64_t nc;
        const int dec = step(&i, s, &deg, &nc);
        if (dec == kRefineA) break;   // below the walk's own node: nothing here
        if (dec != kRefineC) {
          if (at_cut || (first >> j & 1u)) emit(dec, i, s, deg, nc);
          break;
        }
        if (at_cut) {
          subtree = true;
          break;
        }
      }
      if (!subtree) continue;
      // the cut node is refined at level i: walk its subtree
      lv.set(a.slevel[root] + 1, i);
      int32_t q = a.src.kids[root].x;
      const int32_t end = a.src.skip[root];
      while (q != end) {
        int iq = lv.get(a.slevel[q]);
        int deg;
        int64_t nc;
        const int dec = step(&iq, q, &deg, &nc);
        if (dec == kRefineA) {
          q = a.src.skip[q];
          continue;
        }
        if (dec != kRefineC) {
          emit(dec, iq, q, deg, nc);
          q = a.src.skip[q];
          continue;
        }
        lv.set(a.slevel[q] + 1, iq);
        q = a.src.kids[q].x;
      }
    }
  };
  walk();
  if (!FILL) {
    const int64_t t0 = wave_sum64(n0), t1 = wave_sum64(n1);
    if (!LEAF) {
      w0 = wave_sum64(w0);
      w1 = wave_sum64(w1);
      w2 = wave_sum64(w2);
      w3 = wave_sum64(w3);
    }
    if (lane == 0) {
      a.cnt0[it] = (int32_t)t0;
      a.cnt1[it] = (int32_t)t1;
      if (!LEAF) {
        atomicAdd(a.work + 0, (unsigned long long)w0);
        atomicAdd(a.work + 1, (unsigned long long)w1);
        atomicAdd(a.work + 2, (unsigned long long)w2);
        atomicAdd(a.work + 3, (unsigned long long)w3);
      }
    }
    return;
  }
  // fill: this lane's entries go after those of the lanes before it
  out0 = a.ids0 + a.ptr0[it] + wave_excl(n0, lane);
  out1 = a.ids1 + a.ptr1[it] + wave_excl(n1, lane);
  wr = true;
  walk();
}

__global__ void k_dual_flags(const int32_t* __restrict__ ncc, const int32_t* __restrict__ ncp,
                             int64_t nn, int32_t* __restrict__ flag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nn) flag[q] = (ncc[q] + ncp[q]) > 0 ? 1 : 0;
}

__global__ void k_dual_slots(const int32_t* __restrict__ flag, const int32_t* __restrict__ slot,
                             int64_t nn, int64_t ng, int64_t P,
                             const double4* __restrict__ tgeo, const int2* __restrict__ trange,
                             const int32_t* __restrict__ ccptr, const int32_t* __restrict__ cpptr,
                             int32_t* __restrict__ gnode, double4* __restrict__ gbgeo,
                             int32_t* __restrict__ gbptr, int32_t* __restrict__ gpptr,
                             int32_t* __restrict__ gdptr, unsigned long long* __restrict__ work) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) {
    gbptr[ng] = (int32_t)(ng * P);
    gpptr[ng] = ccptr[nn];
    gdptr[ng] = cpptr[nn];
  }
  if (q >= nn || !flag[q]) return;
  const int32_t gi = slot[q];
  gnode[gi] = (int32_t)q;
  gbgeo[gi] = tgeo[q];
  gbptr[gi] = (int32_t)(gi * P);
  gpptr[gi] = ccptr[q];
  gdptr[gi] = cpptr[q];
  const int2 r = trange[q];
  atomicAdd(work + 4, (unsigned long long)((int64_t)(r.y - r.x) * P));
}

template <bool FILL>
__global__ void k_dual_xlists(const int32_t* __restrict__ leaves, int64_t nl,
                              const int32_t* __restrict__ tparent,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ slot,
                              int32_t* __restrict__ xcnt, const int32_t* __restrict__ xptr,
                              int32_t* __restrict__ xgi, int32_t* __restrict__ xnode) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  int32_t cnt = 0;
  for (int32_t q = leaves[l]; q >= 0; q = tparent[q]) cnt += flag[q];
  if (!FILL) {
    xcnt[l] = cnt;
    return;
  }
  int32_t o = xptr[l] + cnt;   // root first: written from the leaf backwards
  for (int32_t q = leaves[l]; q >= 0; q = tparent[q])
    if (flag[q]) {
      --o;
      xgi[o] = slot[q];
      xnode[o] = q;
    }
}

__global__ void k_iota(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

}  // namespace

hipError_t launch_dual_walk(const DualArgs& a, bool per_leaf, bool fill, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  if (a.nitems > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.nitems), block(64);
  if (per_leaf) {
    if (fill) hipLaunchKernelGGL((k_dual_walk<true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_dual_walk<true, false>), grid, block, 0, s, a);
  } else {
    if (fill) hipLaunchKernelGGL((k_dual_walk<false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_dual_walk<false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_dual_flags(const int32_t* ncc, const int32_t* ncp, int64_t nn, int32_t* flag,
                             hipStream_t s) {
  if (nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dual_flags, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, ncc, ncp,
                     nn, flag);
  return hipGetLastError();
}

hipError_t launch_dual_slots(const int32_t* flag, const int32_t* slot, int64_t nn, int64_t ng,
                             int64_t P, const double4* tgeo, const int2* trange,
                             const int32_t* ccptr, const int32_t* cpptr, int32_t* gnode,
                             double4* gbgeo, int32_t* gbptr, int32_t* gpptr, int32_t* gdptr,
                             unsigned long long* work, hipStream_t s) {
  const int64_t nt = nn > 0 ? nn : 1;
  hipLaunchKernelGGL(k_dual_slots, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, flag,
                     slot, nn, ng, P, tgeo, trange, ccptr, cpptr, gnode, gbgeo, gbptr, gpptr,
                     gdptr, work);
  return hipGetLastError();
}

hipError_t launch_dual_xlists(const int32_t* leaves, int64_t nl, const int32_t* tparent,
                              const int32_t* flag, const int32_t* slot, int32_t* xcnt,
                              const int32_t* xptr, int32_t* xgi, int32_t* xnode, bool fill,
                              hipStream_t s) {
  if (nl == 0) return hipSuccess;
  const dim3 grid((unsigned)((nl + 255) / 256)), block(256);
  if (fill)
    hipLaunchKernelGGL(k_dual_xlists<true>, grid, block, 0, s, leaves, nl, tparent, flag, slot,
                       xcnt, xptr, xgi, xnode);
  else
    hipLaunchKernelGGL(k_dual_xlists<false>, grid, block, 0, s, leaves, nl, tparent, flag, slot,
                       xcnt, xptr, xgi, xnode);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace bltc
