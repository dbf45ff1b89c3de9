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
// scan over contiguous memory.  The nodes of one level own disjoint particle
// ranges, so a level is processed by several host threads and its children
// are numbered afterwards in node order: the result does not depend on the
// thread count.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
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

// Runs fn(i) for i in [0, n) on up to hardware_concurrency threads (at most
// 16), handing out indices in order.
template <typename F>
void parallel_for(int64_t n, F&& fn) {
  const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(16, std::thread::hardware_concurrency()));
  const int64_t nt = std::min<int64_t>(hw, n);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next(0);
  auto work = [&] {
    for (int64_t i = next++; i < n; i = next++) fn(i);
  };
  std::vector<std::thread> th;
  for (int64_t k = 1; k < nt; ++k) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
}

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
  // what the processing of one node leaves for the numbering pass
  struct NodeOut {
    double lo[3], hi[3], ctr[3], rad;
    int32_t off[8], cnt[8];
    int nch;
  };
  add(0, (int32_t)n, 0);
  size_t lev_begin = 0;
  while (lev_begin < t.begin.size()) {
    const size_t lev_end = t.begin.size();
    std::vector<NodeOut> res(lev_end - lev_begin);
    auto process = [&](int64_t k, bool intra) {
      const size_t q = lev_begin + (size_t)k;
      NodeOut& o = res[k];
      o.nch = 0;
      const int32_t b = t.begin[q], e = t.end[q];
      // chunks of the node's range for the intra-node parallel passes
      const int64_t nck = intra ? std::min<int64_t>(64, std::max<int64_t>(1, (e - b) >> 15)) : 1;
      auto cb = [&](int64_t c) { return (int32_t)(b + ((int64_t)(e - b) * c) / nck); };
      double side[3], hsq[3];
      if (nck == 1) {
        node_geometry(B, b, e, o.lo, o.hi);
      } else {   // min and max are exact in any order
        std::vector<double> clo(3 * nck), chi(3 * nck);
        parallel_for(nck, [&](int64_t c) {
          node_geometry(B, cb(c), cb(c + 1), &clo[3 * c], &chi[3 * c]);
        });
        for (int a = 0; a < 3; ++a) {
          o.lo[a] = clo[a];
          o.hi[a] = chi[a];
          for (int64_t c = 1; c < nck; ++c) {
            if (clo[3 * c + a] < o.lo[a]) o.lo[a] = clo[3 * c + a];
            if (chi[3 * c + a] > o.hi[a]) o.hi[a] = chi[3 * c + a];
          }
        }
      }
      for (int a = 0; a < 3; ++a) {
        side[a] = o.hi[a] - o.lo[a];
        o.ctr[a] = 0.5 * (o.lo[a] + o.hi[a]);
        const double half = 0.5 * (o.hi[a] - o.lo[a]);
        hsq[a] = half * half;
      }
      o.rad = std::sqrt((hsq[0] + hsq[1]) + hsq[2]);
      const double lmax = std::max(side[0], std::max(side[1], side[2]));
      if ((int64_t)(e - b) <= leaf_max || !(lmax > 0.0)) return;

      const double cut = lmax * 0.70710678118654752440;   // l_max / sqrt(2)
      bool split[3];
      for (int a = 0; a < 3; ++a) split[a] = side[a] > cut;
      // codes and per-chunk histograms; the stable partition places chunk c's
      // particles of code k after those of the chunks before it
      std::vector<int32_t> hist(8 * nck, 0);
      auto codes = [&](int64_t c) {
        int32_t* h = &hist[8 * c];
        for (int32_t i = cb(c); i < cb(c + 1); ++i) {
          uint8_t cd = 0;
          if (split[0] && !(B.c[0][i] < o.ctr[0])) cd |= 1;
          if (split[1] && !(B.c[1][i] < o.ctr[1])) cd |= 2;
          if (split[2] && !(B.c[2][i] < o.ctr[2])) cd |= 4;
          B.code[i] = cd;
          ++h[cd];
        }
      };
      if (nck == 1) codes(0); else parallel_for(nck, codes);
      int32_t tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int64_t c = 0; c < nck; ++c)
        for (int k8 = 0; k8 < 8; ++k8) tot[k8] += hist[8 * c + k8];
      int used = 0;
      for (int k8 = 0; k8 < 8; ++k8) used += tot[k8] != 0;
      if (used < 2) return;

      int32_t off[8];
      int32_t acc = b;
      for (int k8 = 0; k8 < 8; ++k8) {
        off[k8] = acc;
        acc += tot[k8];
      }
      std::vector<int32_t> pos(8 * nck);
      for (int k8 = 0; k8 < 8; ++k8) {
        int32_t p = off[k8];
        for (int64_t c = 0; c < nck; ++c) {
          pos[8 * c + k8] = p;
          p += hist[8 * c + k8];
        }
      }
      auto scatter = [&](int64_t c) {
        int32_t* ps = &pos[8 * c];
        for (int32_t i = cb(c); i < cb(c + 1); ++i) {
          const int32_t d = ps[B.code[i]]++;
          B.tperm[d] = B.perm[i];
          for (int a = 0; a < 3; ++a) B.tc[a][d] = B.c[a][i];
        }
      };
      auto copyback = [&](int64_t c) {
        const int32_t lo = cb(c), hi = cb(c + 1);
        std::memcpy(B.perm.data() + lo, B.tperm.data() + lo, sizeof(int32_t) * (hi - lo));
        for (int a = 0; a < 3; ++a)
          std::memcpy(B.c[a].data() + lo, B.tc[a].data() + lo, sizeof(double) * (hi - lo));
      };
      if (nck == 1) {
        scatter(0);
        copyback(0);
      } else {
        parallel_for(nck, scatter);
        parallel_for(nck, copyback);
      }
      for (int k8 = 0; k8 < 8; ++k8) {
        if (!tot[k8]) continue;
        o.off[o.nch] = off[k8];
        o.cnt[o.nch] = tot[k8];
        ++o.nch;
      }
    };
    const int64_t nlev = (int64_t)(lev_end - lev_begin);
    if (nlev < 8) {
      for (int64_t k = 0; k < nlev; ++k) process(k, true);
    } else {
      parallel_for(nlev, [&](int64_t k) { process(k, false); });
    }
    // geometry and children of the level, in node order (breadth first)
    for (size_t q = lev_begin; q < lev_end; ++q) {
      const NodeOut& o = res[q - lev_begin];
      for (int a = 0; a < 3; ++a) t.box.push_back(o.lo[a]);
      for (int a = 0; a < 3; ++a) t.box.push_back(o.hi[a]);
      for (int a = 0; a < 3; ++a) t.ctr.push_back(o.ctr[a]);
      t.rad.push_back(o.rad);
      if (o.nch == 0) continue;
      t.first[q] = (int32_t)t.begin.size();
      t.count[q] = o.nch;
      for (int c = 0; c < o.nch; ++c) add(o.off[c], o.off[c] + o.cnt[c], t.level[q] + 1);
    }
    lev_begin = lev_end;
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

void batch_bounds(const HostTree& order, int32_t batch_size, int64_t group_max,
                  std::vector<int32_t>& bptr, std::vector<int32_t>& bend) {
  bptr.clear();
  bend.clear();
  if (order.n == 0) {
    bptr.push_back(0);
    return;
  }
  std::vector<std::pair<int32_t, int32_t>> groups;
  groups_of(order, 0, group_max, groups);
  // every batch ends at the next batch's start or at its group's end
  for (const auto& g : groups)
    for (int64_t s = g.first; s < g.second; s += batch_size) {
      bptr.push_back((int32_t)s);
      bend.push_back((int32_t)std::min<int64_t>(g.second, s + batch_size));
    }
  bptr.push_back((int32_t)order.n);
}

namespace {

// One part of the balanced k-d cut: idx[0, c) holds the part's targets and
// `base` its first position in the final order.
void kd_part(int32_t* idx, int64_t c, int32_t bs, const double* const xyz[3], int64_t base,
             int depth, std::vector<int64_t>& starts) {
  if (c <= bs) {
    std::sort(idx, idx + c);
    starts.push_back(base);
    return;
  }
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = hi[a] = xyz[a][idx[0]];
    for (int64_t i = 1; i < c; ++i) {
      const double v = xyz[a][idx[i]];
      if (v < lo[a]) lo[a] = v;
      if (v > hi[a]) hi[a] = v;
    }
  }
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
  const double* key = xyz[ax];
  const int64_t nb = (c + bs - 1) / bs;
  const int64_t left = (int64_t)bs * (nb / 2);
  // the `left` smallest by (coordinate, index): a strict total order, so
  // the set is unique whatever the selection algorithm
  std::nth_element(idx, idx + left, idx + c, [key](int32_t i, int32_t j) {
    return key[i] < key[j] || (key[i] == key[j] && i < j);
  });
  if (depth < 4 && c > (1 << 17)) {   // large parts: the two halves in parallel
    std::vector<int64_t> other;
    std::thread th([&] { kd_part(idx, left, bs, xyz, base, depth + 1, other); });
    kd_part(idx + left, c - left, bs, xyz, base + left, depth + 1, starts);
    th.join();
    starts.insert(starts.end(), other.begin(), other.end());
  } else {
    kd_part(idx, left, bs, xyz, base, depth + 1, starts);
    kd_part(idx + left, c - left, bs, xyz, base + left, depth + 1, starts);
  }
}

}  // namespace

void kd_batches(const double* x, const double* y, const double* z, int64_t m, int32_t bs,
                std::vector<int32_t>& perm, std::vector<int32_t>& bptr) {
  perm.resize(m);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<int64_t> starts;
  const double* const xyz[3] = {x, y, z};
  if (m > 0) kd_part(perm.data(), m, bs, xyz, 0, 0, starts);
  std::sort(starts.begin(), starts.end());   // parts in cut order, first part first
  bptr.assign(starts.begin(), starts.end());
  bptr.push_back((int32_t)m);
}

void build_host_batches(const double* x, const double* y, const double* z,
                        int64_t m, int32_t batch_size, int32_t order_leaf,
                        int64_t group_max, HostBatches& out) {
  out = HostBatches();
  out.bptr.push_back(0);
  if (m == 0) return;
  std::vector<int32_t> bend;
  if (order_leaf == 0) {
    kd_batches(x, y, z, m, batch_size, out.perm, out.bptr);
    bend.assign(out.bptr.begin() + 1, out.bptr.end());
  } else {
    HostTree order;
    build_host_tree(x, y, z, m, order_leaf, order);
    out.perm.swap(order.perm);
    batch_bounds(order, batch_size, group_max, out.bptr, bend);
  }
  const int64_t nb = (int64_t)bend.size();
  const double* src[3] = {x, y, z};
  out.geo.resize(4 * nb);
  parallel_for(nb, [&](int64_t b) {
    const int64_t s = out.bptr[b], e = bend[b];
    double sq[3];
    for (int a = 0; a < 3; ++a) {
      double lo = src[a][out.perm[s]], hi = lo;
      for (int64_t i = s + 1; i < e; ++i) {
        const double v = src[a][out.perm[i]];
        if (v < lo) lo = v;
        if (v > hi) hi = v;
      }
      out.geo[4 * b + a] = 0.5 * (lo + hi);
      const double h = 0.5 * (hi - lo);
      sq[a] = h * h;
    }
    out.geo[4 * b + 3] = std::sqrt((sq[0] + sq[1]) + sq[2]);
  });
}

}  // namespace bltc
