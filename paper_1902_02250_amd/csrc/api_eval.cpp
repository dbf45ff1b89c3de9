// The C ABI's fixed-(n, theta) evaluation: device interaction lists under
// the batch MAC (eq. MAC, Algorithm 2), the separation rule's degrees, the
// particle-cluster kernel, and the direct sum and work counts.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace bltc {
namespace api {

// Separation-rule thresholds for evaluation degree n and MAC theta: for d in
// [deg_min, n), T[d] = (2k / (1 + k^2))^2 with k = kappa(theta)^((n+1)/(d+1)),
// kappa(r) = r / (1 + sqrt(1 - r^2)); a cluster at ratio rho takes the first
// d with rho^2 <= T[d].  deg_min outside [1, n) turns the rule off.
bltc::Rule make_rule(double theta, int degree, int deg_min) {
  bltc::Rule r;
  if (deg_min < 1 || deg_min >= degree) return r;
  r.deg_min = deg_min;
  r.degree = degree;
  const double kt = theta / (1.0 + std::sqrt(1.0 - theta * theta));
  for (int d = deg_min; d < degree; ++d) {
    const double k = std::pow(kt, (double)(degree + 1) / (double)(d + 1));
    const double rho = (2.0 * k) / (1.0 + k * k);
    r.T[d] = rho * rho;
  }
  return r;
}

bltc::ListArgs list_args(bltc_tree t, bltc_targets g, double theta,
                         const double* theta_b, bltc::ListSet& L) {
  const int64_t nb = g->nb;
  bltc::ListArgs a;
  a.bgeo = g->d_bgeo;
  a.nb = nb;
  a.nodes = tree_nodes(t);
  a.theta = theta;
  a.theta_b = theta_b;
  a.pcnt = L.cnt;
  a.dcnt = L.cnt + nb;
  a.scnt = L.cnt + 2 * nb;
  a.pptr = L.ptr;
  a.dptr = L.ptr + nb + 1;
  a.pids = nullptr;
  a.dids = nullptr;
  a.err = g->d_flags;
  return a;
}

// Device interaction lists of every batch (MAC theta, or theta_b[b] when
// theta_b is given) into L; returns the list sizes.
void build_lists(bltc_tree t, bltc_targets g, double theta, const double* theta_b,
                 bltc::ListSet& L, hipStream_t s, int64_t* np, int64_t* nd,
                 const bltc::Rule* rule, const bltc::ListArgs* per_batch) {
  const int64_t nb = g->nb;
  bltc::ListArgs a = list_args(t, g, theta, theta_b, L);
  const bool on = (rule && rule->deg_min > 0) || (per_batch && per_batch->rule_deg_min > 0);
  if (on && t->host.nnodes() > bltc::kIdMask)
    throw HipError{BLTC_EINVAL, "the separation rule supports at most 2^27 - 1 clusters"};
  if (rule) a.rule = *rule;
  if (per_batch) {
    a.choice = per_batch->choice;
    a.cand_T = per_batch->cand_T;
    a.cand_deg = per_batch->cand_deg;
    a.rule_deg_min = per_batch->rule_deg_min;
  }
  StageTimer lt(BLTC_STAGE_LISTS, s);
  int32_t* fl = L.flags ? L.flags : g->d_flags;
  if (L.flags) a.err = L.flags;
  hipchk(bltc::launch_lists(a, false, s), "list count");
  hipchk(bltc::launch_exclusive_scan(a.pcnt, nb, L.ptr, fl + 1, s), "scan");
  hipchk(bltc::launch_exclusive_scan(a.dcnt, nb, L.ptr + nb + 1, fl + 2, s), "scan");
  int32_t tot[2], flags[4];
  d2h(&tot[0], L.ptr + nb, 1, s);
  d2h(&tot[1], L.ptr + 2 * nb + 1, 1, s);
  d2h(flags, fl, 4, s);
  sync(s);
  if (flags[0] || flags[1] || flags[2])
    throw HipError{BLTC_EDEVICE, "interaction lists overflowed"};
  if (L.fixed) {
    const int64_t off = ((int64_t)tot[0] + 63) / 64 * 64;
    if (off + tot[1] > L.pcap)
      throw HipError{BLTC_EINVAL,
                     "the interaction lists need " + std::to_string(4 * (off + tot[1])) +
                         " bytes, more than the " + std::to_string(4 * L.pcap) +
                         " bytes of fixed scratch left for them"};
    L.dids = L.pids + off;
  } else if (tot[0] > L.pcap) {
    dfree(L.pids);
    L.pcap = 0;
    L.pids = dalloc<int32_t>(tot[0]);
    L.pcap = tot[0];
  }
  if (!L.fixed && tot[1] > L.dcap) {
    dfree(L.dids);
    L.dcap = 0;
    L.dids = dalloc<int32_t>(tot[1]);
    L.dcap = tot[1];
  }
  a.pids = L.pids;
  a.dids = L.dids;
  hipchk(bltc::launch_lists(a, true, s), "list fill");
  lt.stop();
  *np = tot[0];
  *nd = tot[1];
}

// The separation rule's lower degrees that each evaluation group uses, derived
// from the group's top degree: groups (top degree, batches bsel[0..count)),
// bsel NULL for all batches.
void derive_used_degrees(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int rule_min,
                         const DegreeGroups& grp, hipStream_t s) {
  if (rule_min <= 0 || grp.empty()) return;
  for (size_t i = 0; i < grp.size(); ++i)
    hipchk(bltc::launch_degree_mask(grp[i].second.first, grp[i].second.second, L.ptr, L.pids,
                                    g->d_dmask + i, s),
           "degree mask");
  std::vector<uint32_t> mask(grp.size());
  d2h(mask.data(), g->d_dmask, grp.size(), s);
  sync(s);
  for (size_t i = 0; i < grp.size(); ++i)
    for (int dd = rule_min; dd < grp[i].first; ++dd)
      if (mask[i] >> dd & 1u) ensure_derived(t, dd, grp[i].first, s);
}

// The particle-cluster evaluation of the batches in bmap (all if NULL) with
// lists L and the modified weights of `degree`.
bltc::P2PArgs p2p_args(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int kernel,
                       double eps, int degree, const bltc_options& o, const int32_t* bmap,
                       int64_t nmap, double* out) {
  const bltc_degree_data& d = t->deg.at(degree);
  bltc::P2PArgs a;
  a.bmap = bmap;
  a.nmap = nmap;
  a.tx = g->d_x;
  a.m = g->m;
  a.tperm = g->d_tperm;
  a.bptr = g->d_bptr;
  a.bgeo = g->d_bgeo;
  a.nb = g->nb;
  a.wpb = (g->batch_size + bltc::kWave - 1) / bltc::kWave;
  a.pptr = L.ptr;
  a.pids = L.pids;
  a.dptr = L.ptr + g->nb + 1;
  a.dids = L.dids;
  a.range = t->d_range;
  a.grid = d.grid;
  a.fhat = o.precision == BLTC_FP64 ? (const void*)d.p2p64 : (const void*)d.p2p32;
  if (o.deg_min >= 1 && o.deg_min < degree) {
    for (int dd = o.deg_min; dd <= degree; ++dd) {   // lower degrees derived from the top
      const bltc_degree_data* e = &d;
      if (dd < degree) {
        const auto it = t->derived.find({dd, degree});
        if (it == t->derived.end()) continue;   // a degree no list entry carries
        e = &it->second;
      }
      a.grid_d[dd] = e->grid;
      a.fhat_d[dd] = o.precision == BLTC_FP64 ? (const void*)e->p2p64 : (const void*)e->p2p32;
    }
  }
  a.ys = t->d_y;
  a.w64 = t->d_w64;
  a.w32 = t->d_w32;
  a.n = t->n;
  a.eps = eps;
  a.poly_p = o.poly_p;
  a.poly_c = o.poly_c;
  kernel_scales(kernel, &a.scale_u, &a.scale_w);
  a.out = out;
  return a;
}

void run_p2p(bltc_tree t, bltc_targets g, const bltc::ListSet& L, int kernel, double eps,
             int degree, const bltc_options& o, const int32_t* bmap, int64_t nmap,
             double* out, hipStream_t s, const int4* split, int64_t nsplit, double* partial,
             const int32_t* xstart, int32_t xmax, int slices, double* spart) {
  bltc::P2PArgs a = p2p_args(t, g, L, kernel, eps, degree, o, bmap, nmap, out);
  a.split = split;
  a.nsplit = nsplit;
  a.partial = partial;
  if (xstart && xmax > 0 && !split) {
    a.xstart = xstart;
    a.xmax = xmax;
  }
  const bool sliced = !split && slices > 1;
  if (sliced) {
    a.slices = slices;
    a.spart = spart;
  }
  StageTimer ev(BLTC_STAGE_EVAL, s);
  hipchk(bltc::launch_p2p(kernel, o.precision, degree, a, s), "p2p");
  if (sliced)
    hipchk(bltc::launch_slice_reduce(bmap, bmap ? nmap : g->nb, g->d_bptr, a.wpb, slices,
                                     g->d_tperm, spart, odim_of(kernel), a.scale_u, a.scale_w,
                                     g->m, out, s),
           "slice reduce");
  ev.stop();
}

double* spart_reserve(bltc_targets g, int64_t doubles) {
  if (doubles > g->spart_cap) {
    dfree(g->d_spart);
    g->spart_cap = 0;
    g->d_spart = dalloc<double>((size_t)doubles);
    g->spart_cap = doubles;
  }
  return g->d_spart;
}

void evaluate_tree(bltc_tree t, bltc_targets g, int kernel, double eps,
                   int degree, double theta, const bltc_options& o,
                   double* out, hipStream_t s) {
  if (g->m == 0) return;
  ensure_degree(t, degree, s);
  int64_t np = 0, nd = 0;
  const bltc::Rule rule = make_rule(theta, degree, o.deg_min);
  build_lists(t, g, theta, nullptr, g->ls[0], s, &np, &nd, &rule);
  derive_used_degrees(t, g, g->ls[0], rule.deg_min, {{degree, {nullptr, g->nb}}}, s);
  const int wpb = (g->batch_size + bltc::kWave - 1) / bltc::kWave;
  const int k = slices_for(g->nb, wpb, odim_of(kernel));
  double* spart =
      k > 1 ? spart_reserve(g, slices_bytes(g->nb, wpb, odim_of(kernel), k) / 8) : nullptr;
  const std::vector<Dealt> d = deal_batches(g, g->ls[0], s, {{degree, nullptr, g->nb, k}});
  run_p2p(t, g, g->ls[0], kernel, eps, degree, o, g->d_xmap + d[0].off, g->nb, out, s, nullptr,
          0, nullptr, g->d_xstart, d[0].xmax, k, spart);
}

// The launch order of the evaluation's batches.  A wave's time is modelled
// from its lists: an accepted cluster costs (0.69 n1 + 0.5) n1^2 + 2.5
// near-field pair-equivalents (n1 = n + 1: the grid's proxies at the far
// field's per-proxy cost, plus its per-row and per-cluster set-up), a near
// source one.  The batches go by decreasing modelled time (ties in batch
// order), dealt to XCDs 0, 1, .., 7, 0, 1, ..: each XCD gets an eighth of
// the work and runs its share longest first, so the batches that start last
// are the shortest.  In tree order the long batches of a dense region sit
// together and could start last, each then holding its SIMD to the end of
// the launch.  The order changes no result (every wave's sums are its own).
// The sort is a stable counting sort over 4096 levels of the group's largest
// modelled time (batches within 1/4096 of it count as equal), linear in the
// batches, since the device waits for it.
std::vector<Dealt> deal_batches(bltc_targets g, const bltc::ListSet& L, hipStream_t s,
                                const std::vector<DealGroup>& groups) {
  constexpr int kLevels = 4096;
  const int64_t nb = g->nb;
  std::vector<Dealt> res(groups.size(), Dealt{0, 0});
  int64_t total = 0;
  for (const DealGroup& gr : groups) total += gr.n;
  if (total == 0) return res;
  // proxy, leaf and near-source counts of every batch ([3][nb]), one copy
  g->h_cnt.resize(3 * nb);
  d2h(g->h_cnt.data(), L.cnt, 3 * nb, s);
  sync(s);
  ensure_alloc(g->d_xmap, nb);
  ensure_alloc(g->d_xstart, 9 * (bltc::kMaxDegree + 1));
  g->h_xmap.resize(total);
  g->h_xstart.assign(9 * groups.size(), 0);
  const int wpb0 = (g->batch_size + bltc::kWave - 1) / bltc::kWave;
  std::vector<double> w;
  std::vector<int32_t> ord, lev, first(kLevels + 1);
  int64_t off = 0;
  for (size_t i = 0; i < groups.size(); ++i) {
    const DealGroup& gr = groups[i];
    const int wpb = wpb0 * gr.slices;   // waves per batch: of 64 targets, times slices
    const double n1 = gr.degree + 1;
    const double per_cluster = (0.69 * n1 + 0.5) * n1 * n1 + 2.5;
    w.resize(gr.n);
    ord.resize(gr.n);
    lev.resize(gr.n);
    double wmax = 0.0;
    for (int64_t k = 0; k < gr.n; ++k) {
      const int32_t b = gr.ids ? gr.ids[k] : (int32_t)k;
      w[k] = (double)g->h_cnt[b] * per_cluster + (double)g->h_cnt[2 * nb + b];
      wmax = std::max(wmax, w[k]);
    }
    // level 0 holds the longest batches; stable within a level
    const double scale = wmax > 0.0 ? (kLevels - 1) / wmax : 0.0;
    std::fill(first.begin(), first.end(), 0);
    for (int64_t k = 0; k < gr.n; ++k) {
      lev[k] = kLevels - 1 - std::min(kLevels - 1, (int)(w[k] * scale));
      ++first[lev[k] + 1];
    }
    for (int l = 0; l < kLevels; ++l) first[l + 1] += first[l];
    for (int64_t k = 0; k < gr.n; ++k) ord[first[lev[k]]++] = (int32_t)k;
    int32_t* xm = g->h_xmap.data() + off;
    int32_t* xs = g->h_xstart.data() + 9 * i;
    int64_t pos = 0;
    for (int x = 0; x < 8; ++x) {
      xs[x] = (int32_t)(pos * wpb);
      for (int64_t r = x; r < gr.n; r += 8) xm[pos++] = gr.ids ? gr.ids[ord[r]] : ord[r];
    }
    xs[8] = (int32_t)(pos * wpb);
    for (int x = 0; x < 8; ++x) res[i].xmax = std::max(res[i].xmax, xs[x + 1] - xs[x]);
    res[i].off = off;
    off += gr.n;
  }
  h2d(g->d_xmap, g->h_xmap.data(), total, s);
  h2d(g->d_xstart, g->h_xstart.data(), 9 * groups.size(), s);
  return res;
}

int check_tree_eval(bltc_tree t, int64_t m, int kernel, double eps, int degree, double theta,
                    const bltc_options& o, const double* out) {
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  if (int rc = check_options(&o, kernel)) return rc;
  if (m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!t->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (t->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  if (!t->deg.count(degree))
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return BLTC_OK;
}

}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

int bltc_evaluate_tree(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt,
                       double* out, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_tree_eval(t, g->m, kernel, eps, degree, theta, o, out)) return rc;
  return guarded([&] {
    evaluate_tree(t, g, kernel, eps, degree, theta, o, out, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_evaluate(const double* tx, const double* ty, const double* tz,
                  int64_t m, const double* sx, const double* sy,
                  const double* sz, int64_t n, const double* w, int32_t kernel,
                  double eps, int32_t degree, double theta, int64_t leaf_max,
                  const bltc_options* opt, double* out, void* stream) {
  if (int rc = check_points(tx, ty, tz, m, "targets")) return rc;
  if (int rc = check_points(sx, sy, sz, n, "sources")) return rc;
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (n > 0 && !device_ptr(w)) return fail(BLTC_EINVAL, "weights must be a device pointer");
  if (m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (m == 0) return BLTC_OK;   // nothing to write
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    bltc_tree t = new bltc_tree_s;
    bltc_targets g = nullptr;
    try {
      t->n = n;
      t->leaf_max = leaf_max;
      build_tree(sx, sy, sz, n, leaf_max, s, t);
      g = new bltc_targets_s;
      build_targets(tx, ty, tz, m, o.batch_size, o.order_leaf, o.group_max, s, g);
      set_weights(t, w, wdim_of(kernel), s);
      evaluate_tree(t, g, kernel, eps, degree, theta, o, out, s);
      sync(s);
    } catch (...) {
      destroy_targets(g);
      destroy_tree(t);
      throw;
    }
    destroy_targets(g);
    destroy_tree(t);
    return (int)BLTC_OK;
  });
}

int bltc_lists_export(bltc_tree t, bltc_targets g, double theta, int32_t degree,
                      int32_t deg_min, int64_t* nb, int64_t* n_prox, int64_t* n_dir,
                      int64_t* prox_ptr, int32_t* prox_ids, int32_t* prox_deg,
                      int64_t* dir_ptr, int32_t* dir_ids) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  return guarded([&] {
    int64_t np = 0, nd = 0;
    const bltc::Rule rule = make_rule(theta, degree, deg_min);
    if (g->nb > 0) build_lists(t, g, theta, nullptr, g->ls[0], nullptr, &np, &nd, &rule);
    if (nb) *nb = g->nb;
    if (n_prox) *n_prox = np;
    if (n_dir) *n_dir = nd;
    if (g->nb == 0) {
      if (prox_ptr) prox_ptr[0] = 0;
      if (dir_ptr) dir_ptr[0] = 0;
      return (int)BLTC_OK;
    }
    std::vector<int32_t> pp(g->nb + 1), dp(g->nb + 1), pe(np);
    const bltc::ListSet& L = g->ls[0];
    d2h(pp.data(), L.ptr, g->nb + 1, nullptr);
    d2h(dp.data(), L.ptr + g->nb + 1, g->nb + 1, nullptr);
    d2h(pe.data(), L.pids, np, nullptr);
    if (dir_ids) d2h(dir_ids, L.dids, nd, nullptr);
    sync(nullptr);
    for (int64_t i = 0; i < np; ++i) {
      if (prox_ids) prox_ids[i] = pe[i] & bltc::kIdMask;
      if (prox_deg) {
        const int dd = pe[i] >> bltc::kDegShift;
        prox_deg[i] = dd ? dd : degree;
      }
    }
    for (int64_t b = 0; b <= g->nb; ++b) {
      if (prox_ptr) prox_ptr[b] = pp[b];
      if (dir_ptr) dir_ptr[b] = dp[b];
    }
    return (int)BLTC_OK;
  });
}

int bltc_counts(bltc_tree t, bltc_targets g, int32_t degree, double theta, int32_t deg_min,
                int64_t* n_proxy_evals, int64_t* n_direct_evals) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  return guarded([&] {
    int64_t np = 0, nd = 0;
    const bltc::Rule rule = make_rule(theta, degree, deg_min);
    if (g->nb > 0) build_lists(t, g, theta, nullptr, g->ls[0], nullptr, &np, &nd, &rule);
    std::vector<int32_t> pp(g->nb + 1), dp(g->nb + 1), pi(np), di(nd);
    if (g->nb > 0) {
      const bltc::ListSet& L = g->ls[0];
      d2h(pp.data(), L.ptr, g->nb + 1, nullptr);
      d2h(dp.data(), L.ptr + g->nb + 1, g->nb + 1, nullptr);
      d2h(pi.data(), L.pids, np, nullptr);
      d2h(di.data(), L.dids, nd, nullptr);
      sync(nullptr);
    }
    int64_t cp = 0, cd = 0;
    const bltc::HostTree& H = t->host;
    for (int64_t b = 0; b < g->nb; ++b) {
      const int64_t cnt = g->host.bptr[b + 1] - g->host.bptr[b];
      int64_t prox = 0;
      for (int32_t k = pp[b]; k < pp[b + 1]; ++k) {
        const int dd = pi[k] >> bltc::kDegShift;
        const int64_t n1 = (dd ? dd : degree) + 1;
        prox += n1 * n1 * n1;
      }
      cp += cnt * prox;
      int64_t leaf = 0;
      for (int32_t k = dp[b]; k < dp[b + 1]; ++k) leaf += H.end[di[k]] - H.begin[di[k]];
      cd += cnt * leaf;
    }
    if (n_proxy_evals) *n_proxy_evals = cp;
    if (n_direct_evals) *n_direct_evals = cd;
    return (int)BLTC_OK;
  });
}

int bltc_direct(const double* tx, const double* ty, const double* tz,
                int64_t m, const int64_t* idx, int64_t k, const double* sx,
                const double* sy, const double* sz, int64_t n, const double* w,
                int32_t kernel, double eps, const bltc_options* opt,
                double* out, void* stream) {
  if (int rc = check_points(tx, ty, tz, m, "targets")) return rc;
  if (k < 0 || k > 0x7fffffffLL) return fail(BLTC_EINVAL, "k out of range [0, 2^31)");
  if (!idx && k > m) return fail(BLTC_EINVAL, "k exceeds the number of targets");
  if (int rc = check_points(sx, sy, sz, n, "sources")) return rc;
  if (!valid_kernel(kernel)) return fail(BLTC_EINVAL, "unknown kernel");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BLTC_EINVAL, "eps must be finite and >= 0");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (o.precision != BLTC_FP64 && o.precision != BLTC_FP32_FP64ACC)
    return fail(BLTC_EINVAL, "direct sum precision must be FP64 or FP32_FP64ACC");
  if (idx && !device_ptr(idx)) return fail(BLTC_EINVAL, "idx must be a device pointer");
  if (n > 0 && !device_ptr(w)) return fail(BLTC_EINVAL, "weights must be a device pointer");
  if (k > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  return guarded([&] {
    if (idx && k > 0) {   // every index must address a target
      std::vector<int64_t> h(k);
      d2h(h.data(), idx, k, (hipStream_t)stream);
      sync((hipStream_t)stream);
      for (int64_t v : h)
        if (v < 0 || v >= m) throw HipError{BLTC_EINVAL, "idx entry outside [0, m)"};
    }
    double su, sw;
    kernel_scales(kernel, &su, &sw);
    hipchk(bltc::launch_direct(kernel, o.precision, tx, ty, tz, idx, k, sx, sy,
                               sz, n, w, eps, o.poly_p, o.poly_c, su, sw, out,
                               (hipStream_t)stream),
           "direct");
    return (int)BLTC_OK;
  });
}

}  // extern "C"
