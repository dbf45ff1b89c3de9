// The C ABI's cluster-cluster variant: interpolation in the target
// variable too (the next step Section 9 names), through a dual traversal of
// the target and source trees.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.h"

namespace bltc {
namespace api {

namespace {

// ---- cluster-cluster variant -------------------------------------------------
// The dual traversal of the target tree T and the source tree S (the target
// variable is interpolated too, Section 9) runs on the device
// (k_dual_walk.hip): per target node its CC and CP lists and the evaluation
// counts, per target leaf the PC and PP entries of the leaf and its
// ancestors.  Each target cluster with CC or CP work gets a grid slot: its
// grid points are evaluated as targets (one batch per cluster run by several
// waves: CC clusters on the proxy list, CP clusters on the direct list), and
// every target adds the interpolated grid potentials of the slots on its
// root path.

void evaluate_dual(bltc_tree src, bltc_tree tgt, int kernel, double eps, int degree,
                   double theta, const bltc_options& o, double* out, int64_t* counts,
                   hipStream_t s) {
  const bltc::HostTree& T = tgt->host;
  const bltc::HostTree& S = src->host;
  const int64_t m = tgt->n, ntn = T.nnodes();
  if (m == 0) return;
  if (T.depth + 1 > bltc::kDualMaxDepth || S.depth + 2 > bltc::kDualMaxDepth)
    throw HipError{BLTC_EINVAL, "the cluster-cluster traversal supports trees of at most " +
                                    std::to_string(bltc::kDualMaxDepth - 2) + " levels"};
  ensure_degree(src, degree, s);
  const bltc_degree_data& d = src->deg.at(degree);
  const int n1 = degree + 1;
  const int64_t P = (int64_t)n1 * n1 * n1;
  const int odim = odim_of(kernel);
  const bltc::Rule rule = make_rule(theta, degree, o.deg_min);
  if (rule.deg_min > 0 && S.nnodes() > bltc::kIdMask)
    throw HipError{BLTC_EINVAL, "too many source clusters for the separation rule's encoding"};

  if (!tgt->dual) tgt->dual = new bltc_dual_cache;
  bltc_dual_cache& C = *tgt->dual;
  StageTimer lt(BLTC_STAGE_LISTS, s);
  // the target leaves in position order: one batch each
  std::vector<int32_t> leaves, bptr;
  std::vector<double4> bgeo;
  int64_t lmax = 1;
  for (int64_t q = 0; q < ntn; ++q)
    if (T.count[q] == 0) leaves.push_back((int32_t)q);
  std::sort(leaves.begin(), leaves.end(),
            [&](int32_t a, int32_t b) { return T.begin[a] < T.begin[b]; });
  for (int32_t L : leaves) {
    bptr.push_back(T.begin[L]);
    bgeo.push_back(make_double4(T.ctr[3 * L], T.ctr[3 * L + 1], T.ctr[3 * L + 2], T.rad[L]));
    lmax = std::max<int64_t>(lmax, T.end[L] - T.begin[L]);
  }
  bptr.push_back((int32_t)m);
  const int64_t nl = (int64_t)leaves.size(), nb = nl;
  auto up = [&](auto& buf, const auto& v) {
    buf.reserve(v.size());
    h2d(buf.p, v.data(), v.size(), s);
  };
  up(C.leaves, leaves);
  up(C.bptr, bptr);
  up(C.bgeo, bgeo);
  C.ncc.reserve(ntn);
  C.ncp.reserve(ntn);
  C.ccptr.reserve(ntn + 1);
  C.cpptr.reserve(ntn + 1);
  C.flag.reserve(ntn);
  C.slot.reserve(ntn + 1);
  C.npc.reserve(nl);
  C.npp.reserve(nl);
  C.xcnt.reserve(nl);
  C.pptr.reserve(nl + 1);
  C.dptr.reserve(nl + 1);
  C.xptr.reserve(nl + 1);
  C.work.reserve(5);
  C.ovf.reserve(8);
  hipchk(bltc::launch_fill_i32(reinterpret_cast<int32_t*>(C.work.p), 10, 0, s), "clear");
  hipchk(bltc::launch_fill_i32(C.ovf.p, 8, 0, s), "clear");

  bltc::DualArgs a;
  a.src = tree_nodes(src);
  a.slevel = src->d_level;
  a.tgeo = tgt->d_geo;
  a.trange = tgt->d_range;
  a.tkids = tgt->d_kids;
  a.tparent = tgt->d_parent;
  a.th2 = theta * theta;
  a.P = P;
  a.n1 = n1;
  a.rule = rule;
  a.work = C.work.p;
  // per target node: CC and CP lists, counts, grid slots
  a.items = nullptr;
  a.nitems = ntn;
  a.cnt0 = C.ncc.p;
  a.cnt1 = C.ncp.p;
  hipchk(bltc::launch_dual_walk(a, false, false, s), "dual walk (nodes)");
  hipchk(bltc::launch_exclusive_scan(C.ncc.p, ntn, C.ccptr.p, C.ovf.p, s), "scan");
  hipchk(bltc::launch_exclusive_scan(C.ncp.p, ntn, C.cpptr.p, C.ovf.p + 1, s), "scan");
  hipchk(bltc::launch_dual_flags(C.ncc.p, C.ncp.p, ntn, C.flag.p, s), "grid slots");
  hipchk(bltc::launch_exclusive_scan(C.flag.p, ntn, C.slot.p, C.ovf.p + 2, s), "scan");
  // per target leaf: PC and PP entries of its path, and its path's slots
  a.items = C.leaves.p;
  a.nitems = nl;
  a.cnt0 = C.npc.p;
  a.cnt1 = C.npp.p;
  hipchk(bltc::launch_dual_walk(a, true, false, s), "dual walk (leaves)");
  hipchk(bltc::launch_exclusive_scan(C.npc.p, nl, C.pptr.p, C.ovf.p + 3, s), "scan");
  hipchk(bltc::launch_exclusive_scan(C.npp.p, nl, C.dptr.p, C.ovf.p + 4, s), "scan");
  hipchk(bltc::launch_dual_xlists(C.leaves.p, nl, tgt->d_parent, C.flag.p, C.slot.p, C.xcnt.p,
                                  nullptr, nullptr, nullptr, false, s),
         "slot lists");
  hipchk(bltc::launch_exclusive_scan(C.xcnt.p, nl, C.xptr.p, C.ovf.p + 5, s), "scan");
  int32_t tot[6], ovf[8];
  d2h(&tot[0], C.ccptr.p + ntn, 1, s);
  d2h(&tot[1], C.cpptr.p + ntn, 1, s);
  d2h(&tot[2], C.slot.p + ntn, 1, s);
  d2h(&tot[3], C.pptr.p + nl, 1, s);
  d2h(&tot[4], C.dptr.p + nl, 1, s);
  d2h(&tot[5], C.xptr.p + nl, 1, s);
  d2h(ovf, C.ovf.p, 8, s);
  sync(s);
  for (int q = 0; q < 6; ++q)
    if (ovf[q]) throw HipError{BLTC_EINVAL, "cluster-cluster lists exceed 2^31 entries"};
  const int64_t ng = tot[2], M = ng * P, gnb = ng;
  if (M > (int64_t)INT32_MAX)
    throw HipError{BLTC_EINVAL, "cluster-cluster grid pass exceeds 2^31 entries"};
  DevBuf<int32_t>&d_gnode = C.gnode, &d_gbptr = C.gbptr, &d_gpptr = C.gpptr, &d_gpids = C.gpids,
      &d_gdptr = C.gdptr, &d_gdids = C.gdids, &d_giota = C.giota, &d_bptr = C.bptr,
      &d_pptr = C.pptr, &d_pids = C.pids, &d_dptr = C.dptr, &d_dids = C.dids, &d_xptr = C.xptr,
      &d_xgi = C.xgi, &d_xnode = C.xnode;
  DevBuf<double4>&d_bgeo = C.bgeo, &d_gbgeo = C.gbgeo;
  DevBuf<double>&d_tgrid = C.tgrid, &d_g = C.g, &d_gpts = C.gpts;
  d_gpids.reserve(tot[0]);
  d_gdids.reserve(tot[1]);
  d_gnode.reserve(ng);
  d_gbgeo.reserve(ng);
  d_gbptr.reserve(ng + 1);
  d_gpptr.reserve(ng + 1);
  d_gdptr.reserve(ng + 1);
  d_pids.reserve(tot[3]);
  d_dids.reserve(tot[4]);
  d_xgi.reserve(tot[5]);
  d_xnode.reserve(tot[5]);
  d_giota.reserve(M);
  a.items = nullptr;
  a.nitems = ntn;
  a.ptr0 = C.ccptr.p;
  a.ptr1 = C.cpptr.p;
  a.ids0 = d_gpids.p;
  a.ids1 = d_gdids.p;
  hipchk(bltc::launch_dual_walk(a, false, true, s), "dual walk (nodes)");
  hipchk(bltc::launch_dual_slots(C.flag.p, C.slot.p, ntn, ng, P, tgt->d_geo, tgt->d_range,
                                 C.ccptr.p, C.cpptr.p, d_gnode.p, d_gbgeo.p, d_gbptr.p,
                                 d_gpptr.p, d_gdptr.p, C.work.p, s),
         "grid slots");
  a.items = C.leaves.p;
  a.nitems = nl;
  a.ptr0 = d_pptr.p;
  a.ptr1 = d_dptr.p;
  a.ids0 = d_pids.p;
  a.ids1 = d_dids.p;
  hipchk(bltc::launch_dual_walk(a, true, true, s), "dual walk (leaves)");
  hipchk(bltc::launch_dual_xlists(C.leaves.p, nl, tgt->d_parent, C.flag.p, C.slot.p, C.xcnt.p,
                                  d_xptr.p, d_xgi.p, d_xnode.p, true, s),
         "slot lists");
  hipchk(bltc::launch_iota(d_giota.p, M, s), "grid point order");
  const int wpb_t = (int)((lmax + bltc::kWave - 1) / bltc::kWave);
  const int wpb_g = (int)((P + bltc::kWave - 1) / bltc::kWave);
  d_tgrid.reserve(ntn * 3 * n1);
  d_g.reserve(odim * M);
  d_gpts.reserve(3 * M);
  double tk[bltc::kMaxDegree + 1];
  bltc::cheb_points(degree, tk);
  hipchk(bltc::launch_grids(tgt->d_box, ntn, degree, tk, d_tgrid.p, s), "target grids");
  hipchk(bltc::launch_dual_points(d_gnode.p, ng, n1, d_tgrid.p, d_gpts.p, s), "grid points");
  lt.stop();
  // the rule's lower degrees that the source side uses, derived from the top
  // degree's weights
  if (rule.deg_min > 0) {
    uint32_t mk[2] = {0, 0};
    C.mask.reserve(2);
    hipchk(bltc::launch_degree_mask(nullptr, ng, d_gpptr.p, d_gpids.p, C.mask.p, s), "degrees");
    hipchk(bltc::launch_degree_mask(nullptr, nl, d_pptr.p, d_pids.p, C.mask.p + 1, s),
           "degrees");
    d2h(mk, C.mask.p, 2, s);
    sync(s);
    for (int dd = rule.deg_min; dd < degree; ++dd)
      if ((mk[0] | mk[1]) >> dd & 1u) ensure_derived(src, dd, degree, s);
  }

  // Schedules of the two passes: batches by decreasing modelled work, dealt
  // to the 8 XCDs in turn, each XCD running its share longest first.  List
  // lengths vary with a cluster's level and place, and in tree order the
  // longest batches could start last and hold a launch open; every wave's
  // sums are independent, so the order does not change any result.  A proxy
  // entry costs its cluster's grid size, a direct entry about half a full
  // source leaf.
  const double leaf_half = 0.5 * (double)src->leaf_max;
  auto schedule = [&](const int32_t* d_pp, const int32_t* d_dp, int64_t nbb, int wpb,
                      DevBuf<int32_t>& d_map, DevBuf<int32_t>& d_xs, std::vector<int32_t>& bm,
                      std::vector<int32_t>& xs) -> int32_t {
    if (nbb == 0) return 0;
    std::vector<int32_t> pp(nbb + 1), dp(nbb + 1);
    d2h(pp.data(), d_pp, nbb + 1, s);
    d2h(dp.data(), d_dp, nbb + 1, s);
    sync(s);
    std::vector<double> w(nbb);
    for (int64_t i = 0; i < nbb; ++i)
      w[i] = (double)(pp[i + 1] - pp[i]) * (double)P + (double)(dp[i + 1] - dp[i]) * leaf_half;
    std::vector<int32_t> ord(nbb);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t i, int32_t j) { return w[i] > w[j]; });
    bm.resize(nbb);
    xs.assign(9, 0);
    int64_t pos = 0;
    for (int x = 0; x < 8; ++x) {
      xs[x] = (int32_t)(pos * wpb);
      for (int64_t r = x; r < nbb; r += 8) bm[pos++] = ord[r];
    }
    xs[8] = (int32_t)(pos * wpb);
    int32_t xmax = 0;
    for (int x = 0; x < 8; ++x) xmax = std::max(xmax, xs[x + 1] - xs[x]);
    d_map.reserve(nbb);
    d_xs.reserve(9);
    h2d(d_map.p, bm.data(), nbb, s);
    h2d(d_xs.p, xs.data(), 9, s);
    return xmax;
  };
  const int32_t gxmax =
      schedule(d_gpptr.p, d_gdptr.p, gnb, wpb_g, C.gbmap, C.gxstart, C.h_gbmap, C.h_gxstart);
  const int32_t txmax =
      schedule(d_pptr.p, d_dptr.p, nb, wpb_t, C.tbmap, C.txstart, C.h_tbmap, C.h_txstart);

  StageTimer ev(BLTC_STAGE_EVAL, s);
  // the particle-cluster kernel over a point set: batches bp/bg, proxy
  // lists pp/pi, direct lists dp/di, output dst [odim][mm] via tperm;
  // optionally batches in the order bmap with XCD ranges xstart
  auto p2p = [&](const double* tx, int64_t mm, const int32_t* tperm, const int32_t* bp,
                 const double4* bg, int64_t nbb, int wpb, const int32_t* pp, const int32_t* pi,
                 const int32_t* dp, const int32_t* di, double* dst, const int32_t* bmap,
                 const int32_t* xstart, int32_t xmax) {
    bltc::P2PArgs a;
    if (bmap) {
      a.bmap = bmap;
      a.nmap = nbb;
      a.xstart = xstart;
      a.xmax = xmax;
    }
    a.tx = tx;
    a.m = mm;
    a.tperm = tperm;
    a.bptr = bp;
    a.bgeo = bg;
    a.nb = nbb;
    a.wpb = wpb;
    a.pptr = pp;
    a.pids = pi;
    a.dptr = dp;
    a.dids = di;
    a.range = src->d_range;
    a.grid = d.grid;
    a.fhat = o.precision == BLTC_FP64 ? (const void*)d.p2p64 : (const void*)d.p2p32;
    if (rule.deg_min > 0) {
      for (int dd = rule.deg_min; dd <= degree; ++dd) {   // lower degrees derived from the top
        const bltc_degree_data* e = &d;
        if (dd < degree) {
          const auto it = src->derived.find({dd, degree});
          if (it == src->derived.end()) continue;   // a degree no list entry carries
          e = &it->second;
        }
        a.grid_d[dd] = e->grid;
        a.fhat_d[dd] = o.precision == BLTC_FP64 ? (const void*)e->p2p64 : (const void*)e->p2p32;
      }
    }
    a.ys = src->d_y;
    a.w64 = src->d_w64;
    a.w32 = src->d_w32;
    a.n = src->n;
    a.eps = eps;
    a.poly_p = o.poly_p;
    a.poly_c = o.poly_c;
    kernel_scales(kernel, &a.scale_u, &a.scale_w);
    a.out = dst;
    hipchk(bltc::launch_p2p(kernel, o.precision, degree, a, s), "p2p");
  };
  // grid potentials g_A at the target clusters' grid points (CC and CP)
  if (gnb > 0)
    p2p(d_gpts.p, M, d_giota.p, d_gbptr.p, d_gbgeo.p, gnb, wpb_g, d_gpptr.p, d_gpids.p,
        d_gdptr.p, d_gdids.p, d_g.p, C.gbmap.p, C.gxstart.p, gxmax);
  // targets: PC and PP of their leaf and its ancestors
  p2p(tgt->d_y, m, tgt->d_perm, d_bptr.p, d_bgeo.p, nb, wpb_t, d_pptr.p, d_pids.p, d_dptr.p,
      d_dids.p, out, C.tbmap.p, C.txstart.p, txmax);

  bltc::DualDownArgs da;
  da.bptr = d_bptr.p;
  da.nb = nb;
  da.wpb = wpb_t;
  da.tx = tgt->d_y;
  da.m = m;
  da.tperm = tgt->d_perm;
  da.dptr = d_xptr.p;
  da.dgi = d_xgi.p;
  da.dnode = d_xnode.p;
  da.tgrid = d_tgrid.p;
  da.g = d_g.p;
  da.gstride = M;
  da.out = out;
  if (ng > 0) hipchk(bltc::launch_dual_down(odim, n1, da, s), "dual down");
  ev.stop();
  if (counts) {
    unsigned long long w[5];
    d2h(w, C.work.p, 5, s);
    sync(s);
    for (int q = 0; q < 5; ++q) counts[q] = (int64_t)w[q];
  }
  sync(s);
}

}  // namespace

}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

int bltc_evaluate_dual(bltc_tree src, bltc_tree tgt, int32_t kernel, double eps,
                       int32_t degree, double theta, const bltc_options* opt, double* out,
                       int64_t* counts, void* stream) {
  if (counts) std::memset(counts, 0, 5 * sizeof(int64_t));
  if (!src || !tgt) return fail(BLTC_EINVAL, "NULL source or target tree");
  if (int rc = check_eval(kernel, eps, degree, theta)) return rc;
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o, kernel)) return rc;
  if (tgt->n > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!src->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (src->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  if (!src->deg.count(degree))
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return guarded([&] {
    evaluate_dual(src, tgt, kernel, eps, degree, theta, o, out, counts, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

}  // extern "C"
