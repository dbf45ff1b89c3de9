// Test driver built with AddressSanitizer and UndefinedBehaviorSanitizer:
// runs the oracle (the C sources under oracle/) and the library's host
// builders (tree_host.cpp) on small synthetic sets, including degenerate
// ones, and checks that the two builders agree.  Any sanitizer report or
// mismatch ends the process with a non-zero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "internal.h"
extern "C" {
#include "oracle.h"
}

static int fails = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++fails;                                                       \
    }                                                                \
  } while (0)

static void points(int kind, int64_t n, uint64_t seed, std::vector<double>& p) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  p.resize(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double v = u(g);
      if (kind == 1) v = std::round(v * 2.0);          // lattice with repeats
      if (kind == 2) v = 0.25;                          // all points equal
      if (kind == 3 && a == 2) v = 0.0;                 // a flat set
      p[a * n + i] = v;
    }
}

static void compare_tree(const std::vector<double>& p, int64_t n, int64_t leaf) {
  bltc::HostTree H;
  bltc::build_host_tree(p.data(), p.data() + n, p.data() + 2 * n, n, leaf, H);
  orc_tree* t = orc_tree_new(p.data(), p.data() + n, p.data() + 2 * n, n, leaf);
  const int64_t nn = orc_tree_nnodes(t);
  CHECK(nn == H.nnodes());
  std::vector<int64_t> perm(n > 0 ? n : 1), pb(nn > 0 ? nn : 1), pe(nn > 0 ? nn : 1);
  std::vector<double> ctr(3 * (nn > 0 ? nn : 1)), rad(nn > 0 ? nn : 1);
  orc_tree_export(t, perm.data(), nullptr, ctr.data(), rad.data(), nullptr, nullptr,
                  pb.data(), pe.data(), nullptr, nullptr);
  if (nn == H.nnodes()) {
    for (int64_t i = 0; i < n; ++i) CHECK(perm[i] == H.perm[i]);
    for (int64_t q = 0; q < nn; ++q) {
      CHECK(pb[q] == H.begin[q] && pe[q] == H.end[q] && rad[q] == H.rad[q]);
      for (int a = 0; a < 3; ++a) CHECK(ctr[3 * q + a] == H.ctr[3 * q + a]);
    }
  }
  orc_tree_free(t);
}

static void compare_batches(const std::vector<double>& p, int64_t m, int bs, int leaf,
                            int64_t gmax) {
  bltc::HostBatches B;
  bltc::build_host_batches(p.data(), p.data() + m, p.data() + 2 * m, m, bs, leaf, gmax, B);
  const int64_t nb = orc_batches(p.data(), p.data() + m, p.data() + 2 * m, m, bs, leaf, gmax,
                                 nullptr, nullptr, nullptr, nullptr);
  CHECK(nb == (int64_t)B.bptr.size() - 1);
  std::vector<int64_t> tperm(m > 0 ? m : 1), bptr(nb + 1);
  std::vector<double> bc(3 * (nb > 0 ? nb : 1)), br(nb > 0 ? nb : 1);
  orc_batches(p.data(), p.data() + m, p.data() + 2 * m, m, bs, leaf, gmax, tperm.data(),
              bptr.data(), bc.data(), br.data());
  if (nb == (int64_t)B.bptr.size() - 1) {
    for (int64_t i = 0; i < m; ++i) CHECK(tperm[i] == B.perm[i]);
    for (int64_t b = 0; b <= nb; ++b) CHECK(bptr[b] == B.bptr[b]);
    for (int64_t b = 0; b < nb; ++b) {
      CHECK(br[b] == B.geo[4 * b + 3]);
      for (int a = 0; a < 3; ++a) CHECK(bc[3 * b + a] == B.geo[4 * b + a]);
    }
  }
}

int main() {
  for (int kind = 0; kind < 4; ++kind)
    for (int64_t n : {0L, 1L, 7L, 300L, 2501L}) {
      std::vector<double> p;
      points(kind, n, 11 + kind, p);
      for (int64_t leaf : {1L, 5L, 64L}) compare_tree(p, n, leaf);
      compare_batches(p, n, 64, 0, 512);
      compare_batches(p, n, 7, 0, 512);
      compare_batches(p, n, 16, 8, 40);
      compare_batches(p, n, 1, 4, 1);
    }
  // the oracle's arithmetic on a small set: every kernel, both MAC modes,
  // the separation rule, the cluster-cluster variant and the direct sum
  const int64_t n = 900;
  std::vector<double> p, w(6 * n);
  points(0, n, 5, p);
  std::mt19937_64 g(6);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  for (double& v : w) v = u(g);
  const double* x = p.data();
  const double* y = p.data() + n;
  const double* z = p.data() + 2 * n;
  for (int kernel : {ORC_STOKESLET, ORC_ROTLET, ORC_FULL}) {
    const int od = kernel == ORC_STOKESLET ? 3 : 6;
    std::vector<double> ref(od * n), out(od * n);
    CHECK(orc_direct(kernel, 0.01, 0, 0.0, x, y, z, n, x, y, z, n, w.data(), 0, ref.data()) == 0);
    for (int mode : {0, 1})
      for (int dm : {0, 2}) {
        orc_params prm{kernel, 0.01, 0, 0.0, 6, 0.7, 60, mode, 64, 0, 512, dm};
        int64_t np = 0, nd = 0;
        CHECK(orc_treecode(&prm, x, y, z, n, x, y, z, n, w.data(), nullptr, 0, out.data(),
                           &np, &nd) == 0);
        double num = 0, den = 0;
        for (int64_t i = 0; i < od * n; ++i) {
          num += (out[i] - ref[i]) * (out[i] - ref[i]);
          den += ref[i] * ref[i];
        }
        CHECK(std::sqrt(num / den) < 1e-3);
      }
    orc_params prm{kernel, 0.01, 0, 0.0, 5, 0.7, 60, 0, 1, 1, 1, 0};
    std::vector<int64_t> cnt(5);
    CHECK(orc_dual_treecode(&prm, 40, x, y, z, n, x, y, z, n, w.data(), out.data(),
                            cnt.data()) == 0);
  }
  std::printf("sanitized driver: %d failed checks\n", fails);
  return fails ? 1 : 0;
}
