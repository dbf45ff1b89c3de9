// The batch walk of Algorithm 2 shared by a wave's 64 lanes.
//
// A walk from the root visits the tree depth first: an accepted cluster
// (the batch MAC) ends the descent into it, a leaf that fails the MAC goes
// on the direct list, any other cluster is refined.  One thread walking a
// whole tree is a chain of dependent loads; here the tree is cut into
// subtrees whose roots (the cut: the clusters at the cut depth plus the
// shallower leaves, in depth-first order) are split into 64 contiguous
// chunks, one per lane.  For a cut node the lane first tests its ancestors
// from the root down: the shallowest accepted ancestor replaces the whole
// subtree and is reported once, by the first cut node under it (the
// walk's own order: an ancestor comes before its descendants).  Otherwise
// the lane walks the cut node's subtree, first child or depth-first
// successor, until the successor of the subtree.  Concatenated in lane
// order, the lanes' reports are exactly the serial walk's, in its order.
//
// The MAC is R2 > 0 and (r_B + r_C)^2 <= (theta theta) R2 with
// R2 = dx dx + dy dy + dz dz, rounded exactly as written (no contraction),
// the oracle's test bit for bit.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bltc {

// MAC of batch g against cluster c; R2 and rr for the caller.
__device__ __forceinline__ bool batch_mac(const double4& g, const double4& c, double th2,
                                          double* R2o, double* rro) {
#pragma clang fp contract(off)
  const double dx = g.x - c.x;
  const double dy = g.y - c.y;
  const double dz = g.z - c.z;
  const double R2 = dx * dx + dy * dy + dz * dz;
  const double rr = g.w + c.w;
  *R2o = R2;
  *rro = rr;
  return R2 > 0.0 && rr * rr <= th2 * R2;
}

// The cut nodes lane `lane` of 64 handles: [*c0, *c1).
__device__ __forceinline__ void cut_chunk(const Nodes& nd, int lane, int* c0, int* c1) {
  const int per = (nd.ncut + 63) / 64;
  *c0 = min(nd.ncut, lane * per);
  *c1 = min(nd.ncut, *c0 + per);
}

// Runs this lane's part of the walk of batch g under MAC th2:
// accept(q, R2, rr) for every accepted cluster, leaf(q) for every leaf on
// the direct list, in walk order.
template <typename Accept, typename Leaf>
__device__ __forceinline__ void cut_walk(const Nodes& nd, const double4& g, double th2, int lane,
                                         Accept&& accept, Leaf&& leaf) {
  int c0, c1;
  cut_chunk(nd, lane, &c0, &c1);
  for (int c = c0; c < c1; ++c) {
    const int32_t root = nd.cut[c];
    const uint32_t first = nd.cut_first[c];
    const int32_t* anc = nd.cut_anc + (int64_t)c * kCutMaxDepth;
    bool covered = false;
    for (int j = 0; j < kCutMaxDepth; ++j) {
      const int32_t a = anc[j];
      if (a < 0) break;
      double R2, rr;
      if (batch_mac(g, nd.geo[a], th2, &R2, &rr)) {
        if (first >> j & 1u) accept(a, R2, rr);
        covered = true;
        break;
      }
    }
    if (covered) continue;
    const int32_t end = nd.skip[root];
    int32_t q = root;
    while (q != end) {
      double R2, rr;
      if (batch_mac(g, nd.geo[q], th2, &R2, &rr)) {
        accept(q, R2, rr);
        q = nd.skip[q];
        continue;
      }
      const int2 kd = nd.kids[q];
      if (kd.y == 0) {
        leaf(q);
        q = nd.skip[q];
        continue;
      }
      q = kd.x;
    }
  }
}

}  // namespace bltc
