// The C ABI's source and target handles: the cluster tree of Section 6
// built on the device, the weights in tree order, the modified weights of
// eq. modified_weights (Algorithm 1) per degree, and the target batches.
#include <algorithm>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "host.h"

namespace bltc {
namespace api {

// ---- tree ---------------------------------------------------------------------
void destroy_degree(bltc_degree_data& d) {
  dfree(d.grid);
  dfree(d.fhat64);
  dfree(d.p2p64);
  dfree(d.p2p32);
}

void destroy_tree(bltc_tree t) {
  if (!t) return;
  for (auto& kv : t->deg) destroy_degree(kv.second);
  for (auto& kv : t->spare) destroy_degree(kv.second);
  for (auto& kv : t->derived) destroy_degree(kv.second);
  for (auto& kv : t->spare_derived) destroy_degree(kv.second);
  dfree(t->d_perm); dfree(t->d_y); dfree(t->d_box); dfree(t->d_geo);
  dfree(t->d_range); dfree(t->d_kids); dfree(t->d_skip); dfree(t->d_w64); dfree(t->d_w32);
  dfree(t->d_level); dfree(t->d_parent);
  dfree(t->d_cut); dfree(t->d_cut_anc); dfree(t->d_cut_first);
  dfree(t->d_chunks); dfree(t->d_chunk_ptr); dfree(t->d_partial); dfree(t->d_parents);
  delete t->dual;
  delete t;
}

// The cluster tree built on the device, level by level (Section 6 rules, the
// same results as bltc::build_host_tree bit for bit).  The host keeps the
// node ranges and numbers the children breadth first from one histogram per
// chunk; boxes, centers and radii come back with it.  Returns the
// tree-ordered coordinates [3][n] and the permutation in device memory.
void build_device_tree(const double* x, const double* y, const double* z, int64_t n,
                       int64_t leaf_max, hipStream_t s, bltc::HostTree& t, double** coords,
                       int32_t** perm) {
  t = bltc::HostTree();
  t.n = n;
  DevBuf<double> ca, cb, cmm;
  DevBuf<int32_t> pa, pb, dcptr, dhist, dpos;
  DevBuf<int4> dchunks;
  DevBuf<int2> drange;
  DevBuf<bltc::TreeLevelNode> dnodes;
  ca.reserve(3 * n);
  pa.reserve(n);
  hipchk(bltc::launch_tree_init(x, y, z, n, ca.p, pa.p, s), "tree init");
  if (n > 0) {
    cb.reserve(3 * n);
    pb.reserve(n);
    auto add = [&](int32_t b, int32_t e, int32_t lev) {
      t.begin.push_back(b);
      t.end.push_back(e);
      t.level.push_back(lev);
      t.first.push_back(-1);
      t.count.push_back(0);
      if (lev > t.depth) t.depth = lev;
    };
    add(0, (int32_t)n, 0);
    std::vector<int4> chunks;
    std::vector<int32_t> cptr, hist, pos;
    std::vector<int2> range;
    std::vector<bltc::TreeLevelNode> nodes;
    size_t lev_begin = 0;
    while (lev_begin < t.begin.size()) {
      const size_t lev_end = t.begin.size();
      const int nl = (int)(lev_end - lev_begin);
      chunks.clear();
      cptr.resize(nl + 1);
      range.resize(nl);
      for (int k = 0; k < nl; ++k) {
        const size_t q = lev_begin + k;
        cptr[k] = (int32_t)chunks.size();
        range[k] = make_int2(t.begin[q], t.end[q]);
        for (int64_t b = t.begin[q]; b < t.end[q]; b += bltc::kTreeChunk)
          chunks.push_back(make_int4(k, (int)b, (int)std::min<int64_t>(t.end[q], b + bltc::kTreeChunk), 0));
      }
      cptr[nl] = (int32_t)chunks.size();
      const int64_t nch = (int64_t)chunks.size();
      dchunks.reserve(nch);
      dcptr.reserve(nl + 1);
      drange.reserve(nl);
      cmm.reserve(6 * nch);
      dnodes.reserve(nl);
      dhist.reserve(8 * nch);
      dpos.reserve(9 * nch);
      h2d(dchunks.p, chunks.data(), nch, s);
      h2d(dcptr.p, cptr.data(), nl + 1, s);
      h2d(drange.p, range.data(), nl, s);
      hipchk(bltc::launch_tree_level(dchunks.p, nch, dcptr.p, drange.p, nl, ca.p, n, leaf_max,
                                     cmm.p, dnodes.p, dhist.p, s), "tree level");
      hist.resize(8 * nch);
      nodes.resize(nl);
      d2h(hist.data(), dhist.p, 8 * nch, s);
      d2h(nodes.data(), dnodes.p, nl, s);
      sync(s);
      // split decisions, child offsets and per-chunk positions (stable)
      pos.assign(9 * nch, 0);
      bool any = false;
      std::vector<std::array<int32_t, 8>> off(nl), tot(nl);
      std::vector<char> split(nl, 0);
      for (int k = 0; k < nl; ++k) {
        const size_t q = lev_begin + k;
        const bltc::TreeLevelNode& o = nodes[k];   // box, center, radius, split axes
        for (int a = 0; a < 3; ++a) t.box.push_back(o.lo[a]);
        for (int a = 0; a < 3; ++a) t.box.push_back(o.hi[a]);
        for (int a = 0; a < 3; ++a) t.ctr.push_back(o.ctr[a]);
        t.rad.push_back(o.rad);
        tot[k].fill(0);
        for (int c = cptr[k]; c < cptr[k + 1]; ++c)
          for (int k8 = 0; k8 < 8; ++k8) tot[k][k8] += hist[8 * c + k8];
        int used = 0;
        for (int k8 = 0; k8 < 8; ++k8) used += tot[k][k8] != 0;
        split[k] = o.mask != 0 && used >= 2;
        if (!split[k]) {
          for (int c = cptr[k]; c < cptr[k + 1]; ++c) pos[9 * c] = chunks[c].y;
          continue;
        }
        any = true;
        int32_t acc = t.begin[q];
        for (int k8 = 0; k8 < 8; ++k8) {
          off[k][k8] = acc;
          acc += tot[k][k8];
        }
        for (int k8 = 0; k8 < 8; ++k8) {
          int32_t p = off[k][k8];
          for (int c = cptr[k]; c < cptr[k + 1]; ++c) {
            pos[9 * c + k8] = p;
            p += hist[8 * c + k8];
          }
        }
        for (int c = cptr[k]; c < cptr[k + 1]; ++c) pos[9 * c + 8] = 1;
      }
      if (any) {
        h2d(dpos.p, pos.data(), 9 * nch, s);
        hipchk(bltc::launch_tree_scatter(dchunks.p, nch, dpos.p, n, dnodes.p, ca.p, pa.p, cb.p,
                                         pb.p, s), "tree scatter");
      }
      for (int k = 0; k < nl; ++k) {
        if (!split[k]) continue;
        const size_t q = lev_begin + k;
        t.first[q] = (int32_t)t.begin.size();
        int nch8 = 0;
        for (int k8 = 0; k8 < 8; ++k8) {
          if (!tot[k][k8]) continue;
          add(off[k][k8], off[k][k8] + tot[k][k8], t.level[q] + 1);
          ++nch8;
        }
        t.count[q] = nch8;
      }
      lev_begin = lev_end;
    }
    t.perm.resize(n);
    d2h(t.perm.data(), pa.p, n, s);
    sync(s);
  }
  *coords = ca.release();
  *perm = pa.release();
}

void build_tree(const double* x, const double* y, const double* z, int64_t n,
                int64_t leaf_max, hipStream_t s, bltc_tree t) {
  build_device_tree(x, y, z, n, leaf_max, s, t->host, &t->d_y, &t->d_perm);
  const bltc::HostTree& H = t->host;
  const int64_t nn = H.nnodes();
  std::vector<double4> geo(nn);
  std::vector<int2> range(nn), kids(nn);
  for (int64_t q = 0; q < nn; ++q) {
    geo[q] = make_double4(H.ctr[3 * q], H.ctr[3 * q + 1], H.ctr[3 * q + 2], H.rad[q]);
    range[q] = make_int2(H.begin[q], H.end[q]);
    kids[q] = make_int2(H.first[q], H.count[q]);
  }
  // depth-first successor past each subtree: the next sibling, else the
  // parent's successor (nodes are numbered breadth first, parents first)
  std::vector<int32_t> skip(nn, -1);
  for (int64_t q = 0; q < nn; ++q)
    for (int32_t k = 0; k < H.count[q]; ++k)
      skip[H.first[q] + k] = k + 1 < H.count[q] ? H.first[q] + k + 1 : skip[q];
  // upward-pass chunks: consecutive pieces of each leaf's particle range
  std::vector<int4> chunks;
  std::vector<int32_t> cptr(nn + 1);
  for (int64_t q = 0; q < nn; ++q) {
    cptr[q] = (int32_t)chunks.size();
    if (H.count[q] > 0) continue;
    for (int32_t b = H.begin[q]; b < H.end[q]; b += bltc::kUpwardChunk)
      chunks.push_back(make_int4((int)q, b, std::min(H.end[q], b + bltc::kUpwardChunk), 0));
  }
  cptr[nn] = (int32_t)chunks.size();
  t->nchunks = (int64_t)chunks.size();
  // parents by level, deepest first: their children are done before them
  int32_t maxlev = 0;
  for (int64_t q = 0; q < nn; ++q) maxlev = std::max(maxlev, H.level[q]);
  std::vector<int32_t> parents;
  t->parent_levels.clear();
  for (int32_t l = maxlev; l >= 0; --l) {
    const int64_t off = (int64_t)parents.size();
    for (int64_t q = 0; q < nn; ++q)
      if (H.level[q] == l && H.count[q] > 0) parents.push_back((int32_t)q);
    if ((int64_t)parents.size() > off) t->parent_levels.push_back({off, (int64_t)parents.size() - off});
  }

  // the cut for lane-shared walks: the shallowest depth (up to
  // kCutMaxDepth) with at least 64 cut nodes, cut nodes in depth-first order
  int32_t cut_depth = 0;
  std::vector<int32_t> cut;
  {
    std::vector<int32_t> parent(nn, -1);
    for (int64_t q = 0; q < nn; ++q)
      for (int32_t k = 0; k < H.count[q]; ++k) parent[H.first[q] + k] = (int32_t)q;
    auto collect = [&](int32_t L, std::vector<int32_t>& out) {
      out.clear();
      if (nn == 0) return;
      std::vector<int32_t> st{0};
      while (!st.empty()) {
        const int32_t q = st.back();
        st.pop_back();
        if (H.level[q] == L || H.count[q] == 0) {
          out.push_back(q);
          continue;
        }
        for (int32_t k = H.count[q] - 1; k >= 0; --k) st.push_back(H.first[q] + k);
      }
    };
    for (cut_depth = 0; cut_depth <= bltc::kCutMaxDepth; ++cut_depth) {
      collect(cut_depth, cut);
      if ((int64_t)cut.size() >= 64 || cut_depth >= H.depth || cut_depth == bltc::kCutMaxDepth)
        break;
    }
    const int64_t nc = (int64_t)cut.size();
    std::vector<int32_t> anc(nc * bltc::kCutMaxDepth, -1);
    std::vector<uint32_t> first(nc, 0);
    for (int64_t c = 0; c < nc; ++c) {
      std::vector<int32_t> chain;
      for (int32_t a = parent[cut[c]]; a >= 0; a = parent[a]) chain.push_back(a);
      std::reverse(chain.begin(), chain.end());   // root first; depth = index
      for (size_t j = 0; j < chain.size(); ++j) anc[c * bltc::kCutMaxDepth + j] = chain[j];
      for (size_t j = 0; j < chain.size(); ++j) {
        const bool prev_under = c > 0 && anc[(c - 1) * bltc::kCutMaxDepth + j] == chain[j];
        if (!prev_under) first[c] |= 1u << j;
      }
    }
    t->ncut = (int32_t)nc;
    t->d_cut = dalloc<int32_t>(nc);
    t->d_cut_anc = dalloc<int32_t>(nc * bltc::kCutMaxDepth);
    t->d_cut_first = dalloc<uint32_t>(nc);
    h2d(t->d_cut, cut.data(), nc, s);
    h2d(t->d_cut_anc, anc.data(), anc.size(), s);
    h2d(t->d_cut_first, first.data(), nc, s);
  }

  t->d_box = dalloc<double>(6 * nn);
  t->d_geo = dalloc<double4>(nn);
  t->d_range = dalloc<int2>(nn);
  t->d_kids = dalloc<int2>(nn);
  t->d_skip = dalloc<int32_t>(nn);
  t->d_level = dalloc<int32_t>(nn);
  t->d_parent = dalloc<int32_t>(nn);
  t->d_chunks = dalloc<int4>(chunks.size());
  t->d_chunk_ptr = dalloc<int32_t>(nn + 1);
  if (!parents.empty()) t->d_parents = dalloc<int32_t>(parents.size());
  h2d(t->d_box, H.box.data(), 6 * nn, s);
  h2d(t->d_geo, geo.data(), nn, s);
  h2d(t->d_range, range.data(), nn, s);
  h2d(t->d_kids, kids.data(), nn, s);
  h2d(t->d_skip, skip.data(), nn, s);
  h2d(t->d_level, H.level.data(), nn, s);
  {
    std::vector<int32_t> par(nn, -1);
    for (int64_t q = 0; q < nn; ++q)
      for (int32_t k = 0; k < H.count[q]; ++k) par[H.first[q] + k] = (int32_t)q;
    h2d(t->d_parent, par.data(), nn, s);
    sync(s);   // par goes out of scope
  }
  h2d(t->d_chunks, chunks.data(), chunks.size(), s);
  h2d(t->d_chunk_ptr, cptr.data(), nn + 1, s);
  if (!parents.empty()) h2d(t->d_parents, parents.data(), parents.size(), s);
  sync(s);   // the host staging vectors go out of scope
}

// Grid and modified weights of one degree from the stored tree-ordered
// weights, cached per degree until the weights change: the leaves from
// their particles, then the parents level by level from their children.
void ensure_degree(bltc_tree t, int degree, hipStream_t s) {
  if (t->deg.count(degree)) return;
  const int64_t nn = t->host.nnodes();
  const int n1 = degree + 1;
  const int64_t nk = (int64_t)n1 * n1 * n1;
  bltc_degree_data d;
  try {
    const int wd = t->wdim;
    const auto sp = t->spare.find(degree);
    if (sp != t->spare.end()) {   // buffers of a stale table of this degree
      d = sp->second;
      t->spare.erase(sp);
    } else {
      d.grid = dalloc<double>(nn * 3 * n1);
      d.fhat64 = dalloc<double>(nn * wd * nk);
      d.p2p64 = dalloc<double>(nn * wd * nk);
      d.p2p32 = dalloc<float>(nn * wd * nk);
    }
    double tk[bltc::kMaxDegree + 1];
    bltc::cheb_points(degree, tk);
    StageTimer prep(BLTC_STAGE_PREP, s);
    hipchk(bltc::launch_grids(t->d_box, nn, degree, tk, d.grid, s), "grids");
    prep.stop();
    const size_t want = (size_t)t->nchunks * wd * nk;
    if (want > t->partial_cap) {
      dfree(t->d_partial);
      t->partial_cap = 0;
      t->d_partial = dalloc<double>(want);
      t->partial_cap = want;
    }
    StageTimer up(BLTC_STAGE_UPWARD, s);
    hipchk(bltc::launch_upward(t->d_y, t->d_w64, t->n, wd, t->d_chunks,
                               t->nchunks, d.grid, degree, t->d_partial, s),
           "upward");
    hipchk(bltc::launch_upward_reduce(t->d_chunk_ptr, nn, t->d_partial, degree, wd,
                                      d.fhat64, d.p2p64, d.p2p32, s),
           "upward reduce");
    for (const auto& lv : t->parent_levels)
      hipchk(bltc::launch_m2m(t->d_parents + lv.first, lv.second, t->d_kids, degree, wd, d.grid,
                              d.fhat64, d.p2p64, d.p2p32, s),
             "upward transfer");
    up.stop();
  } catch (...) {
    destroy_degree(d);
    throw;
  }
  t->deg[degree] = d;
}

namespace {

// L^d_k(t^n_m) on the reference Chebyshev nodes, in barycentric form with
// the exact-hit rule of Algorithm 1.
void restrict_matrix(int d, int n, double* R) {
  double td[bltc::kMaxDegree + 1], tn[bltc::kMaxDegree + 1];
  bltc::cheb_points(d, td);
  bltc::cheb_points(n, tn);
  for (int m = 0; m <= n; ++m) {
    double L[bltc::kMaxDegree + 1], sum = 0.0;
    int flag = -1;
    for (int k = 0; k <= d; ++k) {
      const double wk = (k == 0 || k == d) ? ((k & 1) ? -0.5 : 0.5) : ((k & 1) ? -1.0 : 1.0);
      const double diff = tn[m] - td[k];
      if (std::fabs(diff) <= DBL_MIN) {
        flag = k;
        L[k] = 0.0;
      } else {
        L[k] = wk / diff;
        sum += L[k];
      }
    }
    for (int k = 0; k <= d; ++k)
      R[k * (n + 1) + m] = flag >= 0 ? (k == flag ? 1.0 : 0.0) : L[k] / sum;
  }
}

}  // namespace

// Weights of degree d < n derived from those of degree n (which must
// exist), cached under (d, n) until the weights change.  Lower degrees of
// the separation rule take these, so a batch's result depends only on its
// own top degree n, whichever other degrees a call uses.
const bltc_degree_data& ensure_derived(bltc_tree t, int d, int n, hipStream_t s) {
  if (d == n) return t->deg.at(n);
  const auto key = std::make_pair(d, n);
  auto it = t->derived.find(key);
  if (it != t->derived.end()) return it->second;
  const bltc_degree_data& src = t->deg.at(n);
  const int64_t nn = t->host.nnodes();
  const int d1 = d + 1;
  const int64_t nk = (int64_t)d1 * d1 * d1;
  bltc_degree_data e;
  try {
    const int wd = t->wdim;
    const auto sp = t->spare_derived.find(key);
    if (sp != t->spare_derived.end()) {
      e = sp->second;
      t->spare_derived.erase(sp);
    } else {
      e.grid = dalloc<double>(nn * 3 * d1);
      e.fhat64 = dalloc<double>(nn * wd * nk);
      e.p2p64 = dalloc<double>(nn * wd * nk);
      e.p2p32 = dalloc<float>(nn * wd * nk);
    }
    double tk[bltc::kMaxDegree + 1];
    bltc::cheb_points(d, tk);
    StageTimer up(BLTC_STAGE_UPWARD, s);
    hipchk(bltc::launch_grids(t->d_box, nn, d, tk, e.grid, s), "grids");
    bltc::RestrictArgs ra;
    ra.d1 = d1;
    ra.n1 = n + 1;
    restrict_matrix(d, n, ra.R);
    hipchk(bltc::launch_restrict(ra, nn, wd, src.fhat64, e.fhat64, e.p2p64, e.p2p32, s),
           "restrict");
    up.stop();
  } catch (...) {
    destroy_degree(e);
    throw;
  }
  return t->derived[key] = e;
}

bltc::Nodes tree_nodes(bltc_tree t) {
  bltc::Nodes n;
  n.geo = t->d_geo;
  n.range = t->d_range;
  n.kids = t->d_kids;
  n.skip = t->d_skip;
  n.nn = t->host.nnodes();
  n.cut = t->d_cut;
  n.cut_anc = t->d_cut_anc;
  n.cut_first = t->d_cut_first;
  n.ncut = t->ncut;
  return n;
}

void set_weights(bltc_tree t, const double* w, int wdim, hipStream_t s) {
  // the cached tables go stale; their buffers are kept for the next tables
  // of the same degree and width (no free or allocation per call)
  for (auto& kv : t->deg) {
    auto it = t->spare.find(kv.first);
    if (it != t->spare.end()) destroy_degree(it->second);
    t->spare[kv.first] = kv.second;
  }
  t->deg.clear();
  for (auto& kv : t->derived) {
    auto it = t->spare_derived.find(kv.first);
    if (it != t->spare_derived.end()) destroy_degree(it->second);
    t->spare_derived[kv.first] = kv.second;
  }
  t->derived.clear();
  t->has_w = false;
  if (t->wdim != wdim) {
    for (auto& kv : t->spare) destroy_degree(kv.second);
    t->spare.clear();
    for (auto& kv : t->spare_derived) destroy_degree(kv.second);
    t->spare_derived.clear();
  }
  if (t->d_w64 && t->wdim != wdim) {
    dfree(t->d_w64);
    dfree(t->d_w32);
    t->d_w64 = nullptr;
    t->d_w32 = nullptr;
  }
  t->wdim = wdim;
  if (!t->d_w64 || !t->d_w32) {   // both or neither (a failed call may leave one)
    dfree(t->d_w64);
    dfree(t->d_w32);
    t->d_w64 = dalloc<double>(wdim * t->n);
    t->d_w32 = dalloc<float>(wdim * t->n);
  }
  StageTimer prep(BLTC_STAGE_PREP, s);
  hipchk(bltc::launch_gather_weights(w, t->d_perm, t->n, wdim, t->d_w64, t->d_w32, s),
         "gather weights");
  prep.stop();
  t->has_w = true;
}

// ---- targets -----------------------------------------------------------------
void destroy_targets(bltc_targets g) {
  if (!g) return;
  dfree(g->d_tperm); dfree(g->d_x); dfree(g->d_bptr); dfree(g->d_bgeo);
  dfree(g->d_flags);
  for (auto& L : g->ls) {
    dfree(L.cnt); dfree(L.ptr); dfree(L.pids); dfree(L.dids);
  }
  dfree(g->d_feat); dfree(g->d_Y); dfree(g->d_pc); dfree(g->d_sc);
  dfree(g->d_choice); dfree(g->d_bmap); dfree(g->d_theta_b); dfree(g->d_spos);
  dfree(g->d_xmap); dfree(g->d_xstart); dfree(g->d_spart);
  dfree(g->d_ufb); dfree(g->d_sgeo); dfree(g->d_sflags);
  dfree(g->ls_samp.cnt); dfree(g->ls_samp.ptr); dfree(g->ls_samp.pids); dfree(g->ls_samp.dids);
  dfree(g->d_wt); dfree(g->d_usq); dfree(g->d_contrib); dfree(g->d_part); dfree(g->d_sums); dfree(g->d_lam);
  dfree(g->d_cost); dfree(g->d_e2); dfree(g->d_candT); dfree(g->d_candn);
  dfree(g->d_costtab);
  delete g->split;
  dfree(g->d_dmask);
  delete g;
}

namespace {

// The starts of the balanced k-d batches of m targets in position order: a
// part of c > bs targets has a first part of bs floor(nb/2), nb = ceil(c/bs).
void kd_batch_starts(int64_t m, int32_t bs, std::vector<int32_t>& bptr) {
  bptr.clear();
  std::vector<std::pair<int64_t, int64_t>> st;
  if (m > 0) st.push_back({0, m});
  while (!st.empty()) {
    const auto [b, c] = st.back();
    st.pop_back();
    if (c <= bs) {
      bptr.push_back((int32_t)b);
      continue;
    }
    const int64_t nb = (c + bs - 1) / bs, left = (int64_t)bs * (nb / 2);
    st.push_back({b + left, c - left});
    st.push_back({b, left});
  }
  bptr.push_back((int32_t)m);
}

// perm (device, m): the balanced k-d order (k_kd.hip).
void kd_batches_device(const double* x, const double* y, const double* z, int64_t m,
                       int32_t bs, int32_t* perm, hipStream_t s) {
  if (m == 0) return;
  std::vector<std::pair<int64_t, int64_t>> segs{{0, m}};
  int64_t n2 = 2048;
  while (n2 < m) n2 <<= 1;
  DevBuf<uint64_t> hi, lo;
  hi.reserve(n2);
  lo.reserve(n2);
  hipchk(bltc::launch_kd_init(hi.p, lo.p, m, n2, s), "k-d keys");
  DevBuf<int4> d_chunks;
  DevBuf<int32_t> d_cut, d_cfirst, d_axis;
  DevBuf<double> d_part;
  auto large = [&] {
    for (const auto& sg : segs)
      if (sg.second > bltc::kKdLocal) return true;
    return false;
  };
  while (large()) {
    if (segs.size() >= (size_t)(1 << 20))
      throw HipError{BLTC_EINVAL, "too many targets for the k-d batches"};
    std::vector<int4> chunks;
    std::vector<int32_t> cut(segs.size()), cfirst(segs.size() + 1);
    for (size_t q = 0; q < segs.size(); ++q) {
      const int64_t b = segs[q].first, c = segs[q].second;
      cut[q] = c > bltc::kKdLocal ? 1 : 0;
      cfirst[q] = (int32_t)chunks.size();
      for (int64_t p = b; p < b + c; p += bltc::kKdChunk)
        chunks.push_back(make_int4((int)q, (int)p, (int)std::min(b + c, p + bltc::kKdChunk), 0));
    }
    cfirst[segs.size()] = (int32_t)chunks.size();
    d_chunks.reserve(chunks.size());
    d_cut.reserve(cut.size());
    d_cfirst.reserve(cfirst.size());
    d_axis.reserve(segs.size());
    d_part.reserve(6 * chunks.size());
    h2d(d_chunks.p, chunks.data(), chunks.size(), s);
    h2d(d_cut.p, cut.data(), cut.size(), s);
    h2d(d_cfirst.p, cfirst.data(), cfirst.size(), s);
    hipchk(bltc::launch_kd_level(d_chunks.p, (int32_t)chunks.size(), d_cut.p, d_cfirst.p,
                                 (int32_t)segs.size(), x, y, z, d_part.p, d_axis.p, hi.p, lo.p,
                                 n2, s),
           "k-d level");
    sync(s);   // the staged layout goes out of scope
    std::vector<std::pair<int64_t, int64_t>> next;
    for (const auto& sg : segs) {
      const int64_t b = sg.first, c = sg.second;
      if (c <= bltc::kKdLocal) {
        next.push_back(sg);
        continue;
      }
      const int64_t nb = (c + bs - 1) / bs, left = (int64_t)bs * (nb / 2);
      next.push_back({b, left});
      next.push_back({b + left, c - left});
    }
    segs.swap(next);
  }
  std::vector<int2> parts(segs.size());
  for (size_t q = 0; q < segs.size(); ++q)
    parts[q] = make_int2((int)segs[q].first, (int)segs[q].second);
  DevBuf<int2> d_parts;
  d_parts.reserve(parts.size());
  h2d(d_parts.p, parts.data(), parts.size(), s);
  hipchk(bltc::launch_kd_local(d_parts.p, (int32_t)parts.size(), lo.p, x, y, z, bs, perm, s),
         "k-d parts");
  sync(s);
}

}  // namespace

void build_targets(const double* x, const double* y, const double* z,
                   int64_t m, int32_t bs, int32_t leaf, int64_t gmax,
                   hipStream_t s, bltc_targets g) {
  bltc::HostBatches& B = g->host;
  B = bltc::HostBatches();
  std::vector<int32_t> bend;
  if (leaf == 0) {
    // balanced k-d batches, cut on the device; the part sizes follow from m
    // and bs alone, so the layout of every level comes from the host
    g->d_tperm = dalloc<int32_t>(m);
    g->d_x = dalloc<double>(3 * m);
    kd_batches_device(x, y, z, m, bs, g->d_tperm, s);
    B.perm.resize(m);
    d2h(B.perm.data(), g->d_tperm, m, s);
    kd_batch_starts(m, bs, B.bptr);
    bend.assign(B.bptr.begin() + 1, B.bptr.end());
    hipchk(bltc::launch_gather_points(x, y, z, g->d_tperm, m, g->d_x, s), "gather targets");
    sync(s);
  } else {
    // the order tree on the device; groups and batch bounds on the host;
    // batch geometry on the device
    bltc::HostTree order;
    build_device_tree(x, y, z, m, leaf, s, order, &g->d_x, &g->d_tperm);
    B.perm.swap(order.perm);
    bltc::batch_bounds(order, bs, gmax, B.bptr, bend);
  }
  g->m = m;
  g->nb = (int64_t)B.bptr.size() - 1;
  g->batch_size = bs;
  g->order_leaf = leaf;
  g->group_max = gmax;
  const int64_t nb = g->nb;
  g->d_bptr = dalloc<int32_t>(nb + 1);
  g->d_bgeo = dalloc<double4>(nb);
  for (auto& L : g->ls) {
    L.cnt = dalloc<int32_t>(3 * nb);
    L.ptr = dalloc<int32_t>(2 * (nb + 1));
  }
  g->d_flags = dalloc<int32_t>(4);
  g->d_dmask = dalloc<uint32_t>(bltc::kMaxDegree + 1);
  h2d(g->d_bptr, B.bptr.data(), nb + 1, s);
  {
    int32_t* d_bend = dalloc<int32_t>(nb);
    try {
      h2d(d_bend, bend.data(), nb, s);
      hipchk(bltc::launch_batch_geo(g->d_x, m, g->d_bptr, d_bend, nb, g->d_bgeo, s),
             "batch geometry");
      B.geo.resize(4 * nb);
      d2h(reinterpret_cast<double4*>(B.geo.data()), g->d_bgeo, nb, s);
      sync(s);
    } catch (...) {
      dfree(d_bend);
      throw;
    }
    dfree(d_bend);
  }
  const int32_t zero[4] = {0, 0, 0, 0};
  h2d(g->d_flags, zero, 4, s);
  sync(s);
}

}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

int bltc_build_tree(const double* x, const double* y, const double* z,
                    int64_t n, int64_t leaf_max, void* stream, bltc_tree* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (int rc = check_points(x, y, z, n, "sources")) return rc;
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  return guarded([&] {
    bltc_tree t = new bltc_tree_s;
    t->n = n;
    t->leaf_max = leaf_max;
    try {
      build_tree(x, y, z, n, leaf_max, (hipStream_t)stream, t);
    } catch (...) {
      destroy_tree(t);
      throw;
    }
    *out = t;
    return (int)BLTC_OK;
  });
}

int bltc_tree_destroy(bltc_tree t) {
  destroy_tree(t);
  return BLTC_OK;
}

int bltc_tree_info(bltc_tree t, int64_t* n_nodes, int32_t* depth) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  if (n_nodes) *n_nodes = t->host.nnodes();
  if (depth) *depth = t->host.depth;
  return BLTC_OK;
}

int bltc_tree_export(bltc_tree t, int64_t* perm, double* box, double* center,
                     double* radius, int32_t* child_first, int32_t* child_count,
                     int64_t* pbegin, int64_t* pend, int32_t* level) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  const bltc::HostTree& H = t->host;
  const int64_t nn = H.nnodes();
  for (int64_t i = 0; perm && i < t->n; ++i) perm[i] = H.perm[i];
  for (int64_t q = 0; q < nn; ++q) {
    if (box) for (int k = 0; k < 6; ++k) box[6 * q + k] = H.box[6 * q + k];
    if (center) for (int k = 0; k < 3; ++k) center[3 * q + k] = H.ctr[3 * q + k];
    if (radius) radius[q] = H.rad[q];
    if (child_first) child_first[q] = H.first[q];
    if (child_count) child_count[q] = H.count[q];
    if (pbegin) pbegin[q] = H.begin[q];
    if (pend) pend[q] = H.end[q];
    if (level) level[q] = H.level[q];
  }
  return BLTC_OK;
}

int bltc_compute_modified_weights(bltc_tree t, const double* w, int32_t wdim,
                                  int32_t degree, void* stream) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  if (wdim != 3 && wdim != 6) return fail(BLTC_EINVAL, "wdim must be 3 or 6");
  if (degree < 1 || degree > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "degree must be in [1, 12]");
  if (t->n > 0 && !device_ptr(w))
    return fail(BLTC_EINVAL, "weights must be a device pointer");
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    set_weights(t, w, wdim, s);
    ensure_degree(t, degree, s);
    return (int)BLTC_OK;
  });
}

int bltc_modified_weights_export(bltc_tree t, int32_t degree, double* fhat,
                                 double* grid) {
  if (!t) return fail(BLTC_EINVAL, "NULL tree");
  auto it = t->deg.find(degree);
  if (it == t->deg.end())
    return fail(BLTC_ESTATE, "modified weights of this degree are not computed");
  return guarded([&] {
    const int64_t nn = t->host.nnodes();
    const int n1 = degree + 1;
    hipchk(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (fhat)
      hipchk(hipMemcpy(fhat, it->second.fhat64,
                       sizeof(double) * nn * t->wdim * n1 * n1 * n1,
                       hipMemcpyDeviceToHost), "hipMemcpy");
    if (grid)
      hipchk(hipMemcpy(grid, it->second.grid, sizeof(double) * nn * 3 * n1,
                       hipMemcpyDeviceToHost), "hipMemcpy");
    return (int)BLTC_OK;
  });
}

int bltc_build_targets(const double* x, const double* y, const double* z,
                       int64_t m, int32_t batch_size, int32_t order_leaf,
                       int64_t group_max, void* stream, bltc_targets* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (int rc = check_points(x, y, z, m, "targets")) return rc;
  if (batch_size < 1 || batch_size > 1024)
    return fail(BLTC_EINVAL, "batch_size must be in [1, 1024]");
  if (order_leaf < 0) return fail(BLTC_EINVAL, "order_leaf must be >= 0 (0: balanced k-d batches)");
  if (group_max < 1) return fail(BLTC_EINVAL, "group_max must be >= 1");
  return guarded([&] {
    bltc_targets g = new bltc_targets_s;
    try {
      build_targets(x, y, z, m, batch_size, order_leaf, group_max, (hipStream_t)stream, g);
    } catch (...) {
      destroy_targets(g);
      throw;
    }
    *out = g;
    return (int)BLTC_OK;
  });
}

int bltc_targets_destroy(bltc_targets g) {
  destroy_targets(g);
  return BLTC_OK;
}

int bltc_targets_export(bltc_targets g, int64_t* nb, int64_t* tperm,
                        int64_t* bptr, double* bcenter, double* bradius) {
  if (!g) return fail(BLTC_EINVAL, "NULL targets");
  const bltc::HostBatches& B = g->host;
  if (nb) *nb = g->nb;
  for (int64_t i = 0; tperm && i < g->m; ++i) tperm[i] = B.perm[i];
  for (int64_t b = 0; b <= g->nb; ++b) {
    if (bptr) bptr[b] = B.bptr[b];
    if (b == g->nb) break;
    if (bcenter) for (int k = 0; k < 3; ++k) bcenter[3 * b + k] = B.geo[4 * b + k];
    if (bradius) bradius[b] = B.geo[4 * b + 3];
  }
  return BLTC_OK;
}

int bltc_host_tree(const double* hx, const double* hy, const double* hz,
                   int64_t n, int64_t leaf_max, int64_t* n_nodes,
                   int32_t* depth, int64_t* perm, double* box, double* center,
                   double* radius, int32_t* child_first, int32_t* child_count,
                   int64_t* pbegin, int64_t* pend, int32_t* level) {
  if (n < 0 || n > 0x7fffffffLL) return fail(BLTC_EINVAL, "count out of range [0, 2^31)");
  if (n > 0 && (!hx || !hy || !hz)) return fail(BLTC_EINVAL, "NULL coordinate array");
  if (leaf_max < 1) return fail(BLTC_EINVAL, "leaf_max must be >= 1");
  return guarded([&] {
    bltc_tree_s t;
    t.n = n;
    bltc::build_host_tree(hx, hy, hz, n, leaf_max, t.host);
    if (n_nodes) *n_nodes = t.host.nnodes();
    if (depth) *depth = t.host.depth;
    return bltc_tree_export(&t, perm, box, center, radius, child_first,
                            child_count, pbegin, pend, level);
  });
}

int bltc_host_batches(const double* hx, const double* hy, const double* hz,
                      int64_t m, int32_t batch_size, int32_t order_leaf,
                      int64_t group_max, int64_t* nb, int64_t* tperm,
                      int64_t* bptr, double* bcenter, double* bradius) {
  if (m < 0 || m > 0x7fffffffLL) return fail(BLTC_EINVAL, "count out of range [0, 2^31)");
  if (m > 0 && (!hx || !hy || !hz)) return fail(BLTC_EINVAL, "NULL coordinate array");
  if (batch_size < 1 || batch_size > 1024)
    return fail(BLTC_EINVAL, "batch_size must be in [1, 1024]");
  if (order_leaf < 0) return fail(BLTC_EINVAL, "order_leaf must be >= 0 (0: balanced k-d batches)");
  if (group_max < 1) return fail(BLTC_EINVAL, "group_max must be >= 1");
  return guarded([&] {
    bltc_targets_s g;
    bltc::build_host_batches(hx, hy, hz, m, batch_size, order_leaf, group_max, g.host);
    g.m = m;
    g.nb = (int64_t)g.host.bptr.size() - 1;
    return bltc_targets_export(&g, nb, tperm, bptr, bcenter, bradius);
  });
}

}  // extern "C"
