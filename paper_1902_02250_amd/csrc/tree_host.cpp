// Host construction of the source cluster tree and of the target batches.
//
// Tree rules (Section 6 of the paper, with the readings the library uses):
//   * a cluster's box is the tight box of its own particles;
//   * a cluster is split when it holds more than leaf_max particles, its
//     longest side l_max is positive and the bisection separates something;
//   * each side longer than l_max / sqrt(2) is bisected at the box midpoint
//     0.5 (lo + hi); a coordinate below the midpoint goes low, others high;
//   * children are ordered by the code bx + 2 by + 4 bz over the bisected
//     axes, empty ones are dropped, and the partition is stable;
//   * center = 0.5 (lo + hi), radius = sqrt(hx^2 + hy^2 + hz^2) with
//     h = 0.5 (hi - lo); nodes are numbered breadth first.
// Built with -ffp-contract=off so the FP64 expressions round exactly as
// written.  The coordinates travel with the permutation, so each box is a
// scan over contiguous memory.
#include <cmath>
#include <cstring>
#include <numeric>
#include <utility>

#include "internal.h"

namespace bltc {

namespace {

struct Builder {
  std::vector<double> c[3];       // coordinates in current tree order
  std::vector<int32_t> perm;
  std::vector<double> tc[3];      // scratch for the partition
  std::vector<int32_t> tperm;
  std::vector<uint8_t> code;
};

void node_geometry(const Builder& B, int32_t b, int32_t e, double lo[3],
                   double hi[3]) {
  for (int a = 0; a < 3; ++a) {
    const double* v = B.c[a].data();
    double mn = v[b], mx = v[b];
    for (int32_t i = b + 1; i < e; ++i) {
      if (v[i] < mn) mn = v[i];
      if (v[i] > mx) mx = v[i];
    }
    lo[a] = mn;
    hi[a] = mx;
  }
}

}  // namespace

void cheb_points(int degree, double* t) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k <= degree; ++k)
    t[k] = std::sin(pi * (double)(degree - 2 * k) / (2.0 * degree));
}

void build_host_tree(const double* x, const double* y, const double* z,
                     int64_t n, int64_t leaf_max, HostTree& t) {
  t = HostTree();
  t.n = n;
  if (n == 0) return;
  Builder B;
  const double* src[3] = {x, y, z};
  for (int a = 0; a < 3; ++a) {
    B.c[a].assign(src[a], src[a] + n);
    B.tc[a].resize(n);
  }
  B.perm.resize(n);
  std::iota(B.perm.begin(), B.perm.end(), 0);
  B.tperm.resize(n);
  B.code.resize(n);

  auto add = [&](int32_t b, int32_t e, int32_t lev) {
    t.begin.push_back(b);
    t.end.push_back(e);
    t.level.push_back(lev);
    t.first.push_back(-1);
    t.count.push_back(0);
    if (lev > t.depth) t.depth = lev;
  };
  add(0, (int32_t)n, 0);
  for (size_t q = 0; q < t.begin.size(); ++q) {
    const int32_t b = t.begin[q], e = t.end[q];
    double lo[3], hi[3], side[3], hsq[3];
    node_geometry(B, b, e, lo, hi);
    for (int a = 0; a < 3; ++a) t.box.push_back(lo[a]);
    for (int a = 0; a < 3; ++a) t.box.push_back(hi[a]);
    for (int a = 0; a < 3; ++a) {
      side[a] = hi[a] - lo[a];
      t.ctr.push_back(0.5 * (lo[a] + hi[a]));
      const double half = 0.5 * (hi[a] - lo[a]);
      hsq[a] = half * half;
    }
    t.rad.push_back(std::sqrt((hsq[0] + hsq[1]) + hsq[2]));
    double lmax = std::max(side[0], std::max(side[1], side[2]));
    if ((int64_t)(e - b) <= leaf_max || !(lmax > 0.0)) continue;

    const double cut = lmax * 0.70710678118654752440;   // l_max / sqrt(2)
    bool split[3];
    double mid[3];
    for (int a = 0; a < 3; ++a) {
      split[a] = side[a] > cut;
      mid[a] = t.ctr[3 * q + a];
    }
    int32_t hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t i = b; i < e; ++i) {
      uint8_t cd = 0;
      if (split[0] && !(B.c[0][i] < mid[0])) cd |= 1;
      if (split[1] && !(B.c[1][i] < mid[1])) cd |= 2;
      if (split[2] && !(B.c[2][i] < mid[2])) cd |= 4;
      B.code[i] = cd;
      ++hist[cd];
    }
    int used = 0;
    for (int k = 0; k < 8; ++k) used += hist[k] != 0;
    if (used < 2) continue;

    int32_t off[8];
    int32_t acc = b;
    for (int k = 0; k < 8; ++k) {
      off[k] = acc;
      acc += hist[k];
    }
    int32_t pos[8];
    std::memcpy(pos, off, sizeof pos);
    for (int32_t i = b; i < e; ++i) {
      const int32_t d = pos[B.code[i]]++;
      B.tperm[d] = B.perm[i];
      for (int a = 0; a < 3; ++a) B.tc[a][d] = B.c[a][i];
    }
    std::memcpy(B.perm.data() + b, B.tperm.data() + b, sizeof(int32_t) * (e - b));
    for (int a = 0; a < 3; ++a)
      std::memcpy(B.c[a].data() + b, B.tc[a].data() + b, sizeof(double) * (e - b));

    const int32_t child0 = (int32_t)t.begin.size();
    int32_t nch = 0;
    for (int k = 0; k < 8; ++k) {
      if (!hist[k]) continue;
      add(off[k], off[k] + hist[k], t.level[q] + 1);
      ++nch;
    }
    t.first[q] = child0;
    t.count[q] = nch;
  }
  t.perm.swap(B.perm);
}

namespace {

// Group nodes: the maximal nodes holding at most group_max targets, plus
// oversized (degenerate) leaves, in tree order.
void groups_of(const HostTree& t, int32_t q, int64_t group_max,
               std::vector<std::pair<int32_t, int32_t>>& out) {
  const int64_t cnt = t.end[q] - t.begin[q];
  if (cnt <= group_max || t.count[q] == 0) {
    out.emplace_back(t.begin[q], t.end[q]);
    return;
  }
  for (int32_t c = 0; c < t.count[q]; ++c) groups_of(t, t.first[q] + c, group_max, out);
}

}  // namespace

void build_host_batches(const double* x, const double* y, const double* z,
                        int64_t m, int32_t batch_size, int32_t order_leaf,
                        int64_t group_max, HostBatches& out) {
  out = HostBatches();
  out.bptr.push_back(0);
  if (m == 0) return;
  HostTree order;
  build_host_tree(x, y, z, m, order_leaf, order);
  out.perm.swap(order.perm);
  std::vector<std::pair<int32_t, int32_t>> groups;
  groups_of(order, 0, group_max, groups);
  out.bptr.clear();
  const double* src[3] = {x, y, z};
  for (const auto& g : groups) {
    for (int64_t s = g.first; s < g.second; s += batch_size) {
      const int64_t e = std::min<int64_t>(g.second, s + batch_size);
      out.bptr.push_back((int32_t)s);
      double sq[3];
      for (int a = 0; a < 3; ++a) {
        double lo = src[a][out.perm[s]], hi = lo;
        for (int64_t i = s + 1; i < e; ++i) {
          const double v = src[a][out.perm[i]];
          if (v < lo) lo = v;
          if (v > hi) hi = v;
        }
        out.geo.push_back(0.5 * (lo + hi));
        const double h = 0.5 * (hi - lo);
        sq[a] = h * h;
      }
      out.geo.push_back(std::sqrt((sq[0] + sq[1]) + sq[2]));
    }
  }
  out.bptr.push_back((int32_t)m);
}

}  // namespace bltc
