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

// Evaluation with (n, theta) chosen per batch (see bltc_evaluate_adaptive).
// ---- cluster-cluster variant -------------------------------------------------
// Dual traversal of the target tree T and the source tree S (the target
// variable is interpolated too, Section 9).  For a pair (A, C):
//   MAC (R2 > 0 and (r_A + r_C)^2 <= theta^2 R2): CC if both hold more than
//   P = (n+1)^3 particles, PC if only C does, CP if only A does, else PP;
//   no MAC and both leaves: PP; otherwise refine A if C is a leaf or
//   (A is not a leaf and r_A >= r_C), else refine C.
struct DualPlan {
  std::vector<std::vector<int32_t>> cc, cp, pc, pp;   // source nodes, by target node
  int64_t cnt[5] = {0, 0, 0, 0, 0};                    // CC, PC, CP, PP evaluations, downward terms
};

void dual_traverse(const bltc::HostTree& T, const bltc::HostTree& S, int n1, double theta,
                   const bltc::Rule& rule, DualPlan& D) {
  const int64_t ntn = T.nnodes();
  D.cc.assign(ntn, {});
  D.cp.assign(ntn, {});
  D.pc.assign(ntn, {});
  D.pp.assign(ntn, {});
  if (T.n == 0 || S.n == 0) return;
  const int64_t P = (int64_t)n1 * n1 * n1;
  std::vector<std::pair<int32_t, int32_t>> st{{0, 0}};
  while (!st.empty()) {
    const int32_t A = st.back().first, C = st.back().second;
    st.pop_back();
    const int64_t na = T.end[A] - T.begin[A], nc = S.end[C] - S.begin[C];
    const double dx = T.ctr[3 * A] - S.ctr[3 * C];
    const double dy = T.ctr[3 * A + 1] - S.ctr[3 * C + 1];
    const double dz = T.ctr[3 * A + 2] - S.ctr[3 * C + 2];
    const double R2 = dx * dx + dy * dy + dz * dz;
    const double rr = T.rad[A] + S.rad[C];
    const bool mac = R2 > 0.0 && rr * rr <= (theta * theta) * R2;
    const bool leafA = T.count[A] == 0, leafC = S.count[C] == 0;
    // the source side's degree under the separation rule (n - 1 when off):
    // the entry carries it above kDegShift
    int d = n1 - 1;
    if (mac && rule.deg_min > 0) {
      const double qq = (rr * rr) / R2;
      d = rule.deg_min;
      while (d < rule.degree && !(qq <= rule.T[d])) ++d;
    }
    const int64_t Pd = (int64_t)(d + 1) * (d + 1) * (d + 1);
    const int32_t e = rule.deg_min > 0 ? (C | (d << bltc::kDegShift)) : C;
    if (mac && na > P && nc > P) {
      D.cc[A].push_back(e);
      D.cnt[0] += P * Pd;
    } else if (mac && nc > P) {
      D.pc[A].push_back(e);
      D.cnt[1] += na * Pd;
    } else if (mac && na > P) {
      D.cp[A].push_back(C);
      D.cnt[2] += P * nc;
    } else if (mac || (leafA && leafC)) {
      D.pp[A].push_back(C);
      D.cnt[3] += na * nc;
    } else if (leafC || (!leafA && T.rad[A] >= S.rad[C])) {
      for (int32_t k = T.count[A] - 1; k >= 0; --k) st.push_back({T.first[A] + k, C});
    } else {
      for (int32_t k = S.count[C] - 1; k >= 0; --k) st.push_back({A, S.first[C] + k});
    }
  }
}

void evaluate_dual(bltc_tree src, bltc_tree tgt, int kernel, double eps, int degree,
                   double theta, const bltc_options& o, double* out, int64_t* counts,
                   hipStream_t s) {
  const bltc::HostTree& T = tgt->host;
  const bltc::HostTree& S = src->host;
  const int64_t m = tgt->n, ntn = T.nnodes();
  if (m == 0) return;
  ensure_degree(src, degree, s);
  const bltc_degree_data& d = src->deg.at(degree);
  const int n1 = degree + 1;
  const int64_t P = (int64_t)n1 * n1 * n1;
  const int odim = odim_of(kernel);

  StageTimer lt(BLTC_STAGE_LISTS, s);
  DualPlan D;
  const bltc::Rule rule = make_rule(theta, degree, o.deg_min);
  if (rule.deg_min > 0 && S.nnodes() > bltc::kIdMask)
    throw HipError{BLTC_EINVAL, "too many source clusters for the separation rule's encoding"};
  dual_traverse(T, S, n1, theta, rule, D);
  // grid slots: target clusters with CC or CP work
  // (their grid points are evaluated as targets, one batch per cluster run
  // by several waves: CC clusters on the proxy list, CP clusters on the
  // direct list)
  std::vector<int32_t> slot(ntn, -1), gnode;
  std::vector<int32_t> gbptr, gpptr{0}, gpids, gdptr{0}, gdids;
  std::vector<double4> gbgeo;
  for (int64_t A = 0; A < ntn; ++A) {
    if (D.cc[A].empty() && D.cp[A].empty()) continue;
    const int32_t gi = (int32_t)gnode.size();
    slot[A] = gi;
    gnode.push_back((int32_t)A);
    gbptr.push_back((int32_t)(gi * P));
    gbgeo.push_back(make_double4(T.ctr[3 * A], T.ctr[3 * A + 1], T.ctr[3 * A + 2], T.rad[A]));
    gpids.insert(gpids.end(), D.cc[A].begin(), D.cc[A].end());
    gpptr.push_back((int32_t)gpids.size());
    gdids.insert(gdids.end(), D.cp[A].begin(), D.cp[A].end());
    gdptr.push_back((int32_t)gdids.size());
    D.cnt[4] += (int64_t)(T.end[A] - T.begin[A]) * P;
  }
  const int64_t ng = (int64_t)gnode.size(), M = ng * P, gnb = (int64_t)gbgeo.size();
  if (M > (int64_t)INT32_MAX || gpids.size() > (size_t)INT32_MAX)
    throw HipError{BLTC_EINVAL, "cluster-cluster grid pass exceeds 2^31 entries"};
  gbptr.push_back((int32_t)M);
  std::vector<int32_t> giota(M);
  std::iota(giota.begin(), giota.end(), 0);
  // one batch per target leaf (run by several waves of 64 targets), leaves
  // in position order; it takes the PC and PP entries and the grid slots of
  // the leaf and all its ancestors
  std::vector<int32_t> parent(ntn, -1), leaves;
  for (int64_t q = 0; q < ntn; ++q) {
    for (int32_t k = 0; k < T.count[q]; ++k) parent[T.first[q] + k] = (int32_t)q;
    if (T.count[q] == 0) leaves.push_back((int32_t)q);
  }
  std::sort(leaves.begin(), leaves.end(),
            [&](int32_t a, int32_t b) { return T.begin[a] < T.begin[b]; });
  std::vector<int32_t> bptr, pptr{0}, pids, dptr{0}, dids, xptr{0}, xgi, xnode, path;
  std::vector<double4> bgeo;
  std::vector<int32_t> lpc, lpp, lgi, lnode;
  int64_t lmax = 1;
  for (int32_t L : leaves) {
    path.clear();
    for (int32_t q = L; q >= 0; q = parent[q]) path.push_back(q);
    std::reverse(path.begin(), path.end());
    lpc.clear();
    lpp.clear();
    lgi.clear();
    lnode.clear();
    for (int32_t q : path) {
      lpc.insert(lpc.end(), D.pc[q].begin(), D.pc[q].end());
      lpp.insert(lpp.end(), D.pp[q].begin(), D.pp[q].end());
      if (slot[q] >= 0) {
        lgi.push_back(slot[q]);
        lnode.push_back(q);
      }
    }
    bptr.push_back(T.begin[L]);
    bgeo.push_back(make_double4(T.ctr[3 * L], T.ctr[3 * L + 1], T.ctr[3 * L + 2], T.rad[L]));
    pids.insert(pids.end(), lpc.begin(), lpc.end());
    pptr.push_back((int32_t)pids.size());
    dids.insert(dids.end(), lpp.begin(), lpp.end());
    dptr.push_back((int32_t)dids.size());
    xgi.insert(xgi.end(), lgi.begin(), lgi.end());
    xnode.insert(xnode.end(), lnode.begin(), lnode.end());
    xptr.push_back((int32_t)xgi.size());
    lmax = std::max<int64_t>(lmax, T.end[L] - T.begin[L]);
  }
  const int64_t nb = (int64_t)bgeo.size();
  const int wpb_t = (int)((lmax + bltc::kWave - 1) / bltc::kWave);
  const int wpb_g = (int)((P + bltc::kWave - 1) / bltc::kWave);
  bptr.push_back((int32_t)m);
  if (pids.size() > (size_t)INT32_MAX || dids.size() > (size_t)INT32_MAX)
    throw HipError{BLTC_EINVAL, "cluster-cluster lists exceed 2^31 entries"};

  if (!tgt->dual) tgt->dual = new bltc_dual_cache;
  bltc_dual_cache& C = *tgt->dual;
  DevBuf<int32_t>&d_gnode = C.gnode, &d_gbptr = C.gbptr, &d_gpptr = C.gpptr, &d_gpids = C.gpids,
      &d_gdptr = C.gdptr, &d_gdids = C.gdids, &d_giota = C.giota, &d_bptr = C.bptr,
      &d_pptr = C.pptr, &d_pids = C.pids, &d_dptr = C.dptr, &d_dids = C.dids, &d_xptr = C.xptr,
      &d_xgi = C.xgi, &d_xnode = C.xnode;
  DevBuf<double4>&d_bgeo = C.bgeo, &d_gbgeo = C.gbgeo;
  DevBuf<double>&d_tgrid = C.tgrid, &d_g = C.g, &d_gpts = C.gpts;
  auto up = [&](auto& buf, const auto& v) {
    buf.reserve(v.size());
    h2d(buf.p, v.data(), v.size(), s);
  };
  up(d_gnode, gnode);
  up(d_gbptr, gbptr);
  up(d_gpptr, gpptr);
  up(d_gpids, gpids);
  up(d_gdptr, gdptr);
  up(d_gdids, gdids);
  up(d_gbgeo, gbgeo);
  up(d_giota, giota);
  up(d_bptr, bptr);
  up(d_pptr, pptr);
  up(d_pids, pids);
  up(d_dptr, dptr);
  up(d_dids, dids);
  up(d_xptr, xptr);
  up(d_xgi, xgi);
  up(d_xnode, xnode);
  up(d_bgeo, bgeo);
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
    std::vector<bool> used(degree, false);
    for (int64_t A = 0; A < ntn; ++A)
      for (const auto* lst : {&D.cc[A], &D.pc[A]})
        for (int32_t e : *lst) {
          const int dd = e >> bltc::kDegShift;
          if (dd < degree) used[dd] = true;
        }
    for (int dd = rule.deg_min; dd < degree; ++dd)
      if (used[dd]) ensure_derived(src, dd, degree, s);
  }

  StageTimer ev(BLTC_STAGE_EVAL, s);
  // the particle-cluster kernel over a point set: batches bp/bg, proxy
  // lists pp/pi, direct lists dp/di, output dst [odim][mm] via tperm
  auto p2p = [&](const double* tx, int64_t mm, const int32_t* tperm, const int32_t* bp,
                 const double4* bg, int64_t nbb, int wpb, const int32_t* pp, const int32_t* pi,
                 const int32_t* dp, const int32_t* di, double* dst) {
    bltc::P2PArgs a;
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
        d_gdptr.p, d_gdids.p, d_g.p);
  // targets: PC and PP of their leaf and its ancestors
  p2p(tgt->d_y, m, tgt->d_perm, d_bptr.p, d_bgeo.p, nb, wpb_t, d_pptr.p, d_pids.p, d_dptr.p,
      d_dids.p, out);

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
  if (counts) std::memcpy(counts, D.cnt, sizeof D.cnt);
  sync(s);   // the device lists go out of scope
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
