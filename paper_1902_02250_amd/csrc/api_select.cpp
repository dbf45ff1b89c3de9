// The C ABI's learned (n, theta) per batch: batch features, candidate
// costs, the selector network's kernels and model file, the judge (the
// fixed treecode of Algorithm 2 at sampled targets) and the adaptive
// evaluation.  Not part of the paper's method.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>

#include "host.h"

namespace bltc {
namespace api {

namespace {

// ---- learned (n, theta) per batch -------------------------------------------
void compute_features(bltc_tree t, bltc_targets g, int kernel, double eps,
                      double theta_ref, const float* mean, const float* stdv,
                      float* feat, hipStream_t s) {
  bltc::FeatArgs a;
  a.bgeo = g->d_bgeo;
  a.bptr = g->d_bptr;
  a.nb = g->nb;
  a.nodes = tree_nodes(t);
  a.box = t->d_box;
  a.theta_ref = theta_ref;
  a.eps = eps;
  a.kernel = kernel;
  a.n_src = t->n;
  a.mean = mean;
  a.stdv = stdv;
  a.feat = feat;
  hipchk(bltc::launch_features(a, s), "features");
}

// Per-batch proxy-cluster and near-source counts of the walk at theta.
void batch_counts(bltc_tree t, bltc_targets g, double theta, int32_t* pc,
                  int32_t* sc, hipStream_t s) {
  bltc::ListSet& L = g->ls[1];
  bltc::ListArgs a = list_args(t, g, theta, nullptr, L);
  a.pcnt = pc;
  a.scnt = sc;
  hipchk(bltc::launch_lists(a, false, s), "list count");
}

constexpr int kLamGrid = 64;   // multipliers per allocation pass

// The judge re-evaluates batches when its estimate exceeds kJudgeTrigger tol,
// down to kJudgeTarget tol; the choices aim below the trigger.
constexpr double kJudgeTrigger = 0.8, kJudgeTarget = 0.6;

// Modelled wave cost of every batch under each of the k candidates
// (cand_n[j], cand_theta[j]) into cost[j][nb] (device), with the separation
// rule when deg_min >= 1: one walk per distinct theta.
void candidate_costs(bltc_tree t, bltc_targets g, int k, const int32_t* cand_n,
                     const double* cand_theta, int deg_min, const bltc::Costs& w,
                     float* cost, hipStream_t s) {
  // the rule's thresholds of every candidate, [k][kMaxDegree + 1], on the device
  ensure_alloc(g->d_candT, (size_t)bltc::kMlpMaxOut * (bltc::kMaxDegree + 1));
  ensure_alloc(g->d_candn, bltc::kMlpMaxOut);
  std::vector<double> T((size_t)k * (bltc::kMaxDegree + 1));
  for (int j = 0; j < k; ++j) {
    const bltc::Rule r = make_rule(cand_theta[j], cand_n[j], deg_min);
    for (int d = 0; d <= bltc::kMaxDegree; ++d) T[(size_t)j * (bltc::kMaxDegree + 1) + d] = r.T[d];
  }
  h2d(g->d_candT, T.data(), T.size(), s);
  h2d(g->d_candn, cand_n, k, s);
  // candidates grouped by theta (at most kMaxPerTheta per group), up to
  // kMaxThetaGroups groups per launch
  std::vector<bltc::CostGroup> groups;
  std::vector<bool> done(k, false);
  for (int j0 = 0; j0 < k; ++j0) {
    if (done[j0]) continue;
    bltc::CostGroup gr;
    std::memset(&gr, 0, sizeof gr);
    gr.theta = cand_theta[j0];
    for (int j = j0; j < k && gr.nc < bltc::kMaxPerTheta; ++j) {
      if (done[j] || cand_theta[j] != cand_theta[j0]) continue;
      done[j] = true;
      gr.deg[gr.nc] = cand_n[j];
      gr.row[gr.nc] = j;
      ++gr.nc;
    }
    groups.push_back(gr);
  }
  // each group's distinct thresholds U (sorted) and bucket costs C[i][k]:
  // candidate i's degree for qq in bucket k (U[k-1] < qq <= U[k]) is the
  // first d in [deg_min, n_i) with T_i[d] >= U[k] (qq <= T_i[d] exactly
  // then), else n_i; bucket nu (qq above every threshold) takes n_i
  std::vector<double> U;
  std::vector<float> C;
  for (bltc::CostGroup& gr : groups) {
    std::vector<bltc::Rule> rules(gr.nc);
    std::vector<double> u;
    for (int i = 0; i < gr.nc; ++i) {
      rules[i] = make_rule(gr.theta, gr.deg[i], deg_min);
      for (int d = rules[i].deg_min; d < rules[i].degree; ++d) u.push_back(rules[i].T[d]);
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    gr.nu = (int32_t)u.size();
    gr.u_off = (int32_t)U.size();
    gr.c_off = (int32_t)C.size();
    U.insert(U.end(), u.begin(), u.end());
    for (int i = 0; i < gr.nc; ++i) {
      for (int kb = 0; kb <= gr.nu; ++kb) {
        int d = gr.deg[i];
        if (kb < gr.nu) {
          for (int dd = rules[i].deg_min; dd < rules[i].degree; ++dd)
            if (rules[i].T[dd] >= u[kb]) {
              d = dd;
              break;
            }
        }
        const float n1 = (float)(d + 1);
        C.push_back((w.far * n1 + w.row) * n1 * n1 + w.clu);
      }
    }
  }
  const size_t ub = (U.size() * sizeof(double) + 255) / 256 * 256;
  const size_t need = ub + C.size() * sizeof(float);
  if ((int64_t)need > g->costtab_cap) {
    dfree(g->d_costtab);
    g->costtab_cap = 0;
    g->d_costtab = dalloc_bytes(need);
    g->costtab_cap = (int64_t)need;
  }
  double* dU = static_cast<double*>(g->d_costtab);
  float* dC = reinterpret_cast<float*>(static_cast<char*>(g->d_costtab) + ub);
  h2d(dU, U.data(), U.size(), s);
  h2d(dC, C.data(), C.size(), s);
  for (size_t g0 = 0; g0 < groups.size(); g0 += bltc::kMaxThetaGroups) {
    bltc::CostArgs a;
    std::memset(&a, 0, sizeof a);
    a.bgeo = g->d_bgeo;
    a.nb = g->nb;
    a.nodes = tree_nodes(t);
    a.ngroups = (int32_t)std::min<size_t>(bltc::kMaxThetaGroups, groups.size() - g0);
    for (int i = 0; i < a.ngroups; ++i) a.grp[i] = groups[g0 + i];
    a.U = dU;
    a.C = dC;
    a.nearf = w.nearf;
    a.cost = cost;
    a.err = g->d_flags;
    hipchk(bltc::launch_cand_costs(a, s), "candidate costs");
  }
}

// The judge's sample targets: one per judge_stride(nb) batches, at a hashed
// position inside the first batch of its group, and their geometry as
// batches of one target; their fallback values go to g->d_ufb.
void ensure_judge_samples(bltc_targets g) {
  if (g->nsamp > 0) return;
  const int64_t nb = g->nb;
  const int st = bltc::judge_stride(nb);
  const int64_t ns = (nb + st - 1) / st;
  ensure_alloc(g->d_ufb, 6 * ns);
  ensure_alloc(g->d_spos, ns);
  ensure_alloc(g->d_sgeo, ns);
  ensure_alloc(g->d_sflags, 4);
  bltc::ListSet& L = g->ls_samp;
  ensure_alloc(L.cnt, 3 * ns);
  ensure_alloc(L.ptr, 2 * (ns + 1));
  std::vector<int32_t> sp(ns);
  for (int64_t i = 0; i < ns; ++i) {
    const int64_t b = i * st;
    const int32_t b0 = g->host.bptr[b], cnt = g->host.bptr[b + 1] - b0;
    const uint32_t h = (uint32_t)(b * 2654435761ull >> 7);
    sp[i] = b0 + (int32_t)(h % (uint32_t)cnt);
  }
  h2d(g->d_spos, sp.data(), ns, nullptr);
  hipchk(bltc::launch_sample_geo(g->d_spos, (int)ns, g->d_x, g->m, g->d_sgeo, nullptr),
         "sample geometry");
  hipchk(bltc::launch_fill_i32(g->d_sflags, 4, 0, nullptr), "clear flags");
  sync(nullptr);
  g->sstride = st;
  g->nsamp = (int32_t)ns;   // last: a failed allocation leaves it 0
}

// The samples' lists: the batch walk of every sample (a batch of one target
// at radius 0, so the batch MAC is the per-target MAC) at fb_theta.
void sample_lists(bltc_tree t, bltc_targets g, double fb_theta, hipStream_t s) {
  const int64_t ns = g->nsamp;
  bltc::ListSet& L = g->ls_samp;
  bltc::ListArgs a;
  a.bgeo = g->d_sgeo;
  a.nb = ns;
  a.nodes = tree_nodes(t);
  a.theta = fb_theta;
  a.pcnt = L.cnt;
  a.dcnt = L.cnt + ns;
  a.scnt = L.cnt + 2 * ns;
  a.pptr = L.ptr;
  a.dptr = L.ptr + ns + 1;
  a.pids = nullptr;
  a.dids = nullptr;
  a.err = g->d_sflags;
  hipchk(bltc::launch_lists(a, false, s), "sample list count");
  hipchk(bltc::launch_exclusive_scan(a.pcnt, ns, L.ptr, g->d_sflags + 1, s), "scan");
  hipchk(bltc::launch_exclusive_scan(a.dcnt, ns, L.ptr + ns + 1, g->d_sflags + 2, s), "scan");
  int32_t tot[2], flags[4];
  d2h(&tot[0], L.ptr + ns, 1, s);
  d2h(&tot[1], L.ptr + 2 * ns + 1, 1, s);
  d2h(flags, g->d_sflags, 4, s);
  sync(s);
  if (flags[0] || flags[1] || flags[2])
    throw HipError{BLTC_EDEVICE, "the judge samples' lists overflowed"};
  if (tot[0] > L.pcap) {
    dfree(L.pids);
    L.pcap = 0;
    L.pids = dalloc<int32_t>(tot[0]);
    L.pcap = tot[0];
  }
  if (tot[1] > L.dcap) {
    dfree(L.dids);
    L.dcap = 0;
    L.dids = dalloc<int32_t>(tot[1]);
    L.dcap = tot[1];
  }
  a.pids = L.pids;
  a.dids = L.dids;
  hipchk(bltc::launch_lists(a, true, s), "sample list fill");
}

// The fallback treecode (fb_degree, fb_theta) at the judge's samples, into
// g->d_ufb [nsamp][odim].
void fallback_samples(bltc_tree t, bltc_targets g, int kernel, double eps, int fb_degree,
                      double fb_theta, hipStream_t s) {
  ensure_judge_samples(g);
  ensure_degree(t, fb_degree, s);
  sample_lists(t, g, fb_theta, s);
  const bltc_degree_data& fd = t->deg.at(fb_degree);
  const int64_t ns = g->nsamp;
  bltc::SampleArgs a;
  a.spos = g->d_spos;
  a.ns = g->nsamp;
  a.tx = g->d_x;
  a.m = g->m;
  a.range = tree_nodes(t).range;
  a.pptr = g->ls_samp.ptr;
  a.pids = g->ls_samp.pids;
  a.dptr = g->ls_samp.ptr + ns + 1;
  a.dids = g->ls_samp.dids;
  a.grid = fd.grid;
  a.fh32 = fd.p2p32;
  a.ys = t->d_y;
  a.w32 = t->d_w32;
  a.n = t->n;
  a.eps = eps;
  kernel_scales(kernel, &a.scale_u, &a.scale_w);
  a.ufb = g->d_ufb;
  hipchk(bltc::launch_fallback_samples(kernel, fb_degree, a, s), "judge samples");
}

void ensure_selection_scratch(bltc_targets g, int64_t k) {
  const int64_t nb = g->nb;
  if (!g->d_lam) {   // allocated last: a failed call leaves it NULL
    ensure_alloc(g->d_feat, nb * bltc::kMlpIn);
    ensure_alloc(g->d_choice, nb);
    ensure_alloc(g->d_bmap, nb);
    ensure_alloc(g->d_theta_b, nb);
    ensure_alloc(g->d_wt, nb);
    ensure_alloc(g->d_contrib, nb);
    ensure_alloc(g->d_usq, nb);
    ensure_alloc(g->d_part, bltc::alloc_blocks(nb) * kLamGrid * 2);
    ensure_alloc(g->d_sums, 2 * std::max(kLamGrid, bltc::kMlpMaxOut));
    ensure_alloc(g->d_lam, kLamGrid);
  }
  ensure_judge_samples(g);
  if (nb * k > g->ycap) {
    dfree(g->d_Y);
    g->ycap = 0;
    g->d_Y = dalloc<float>(nb * k);
    g->ycap = nb * k;
  }
  if (nb * k > g->costcap) {
    dfree(g->d_cost);
    dfree(g->d_e2);
    g->costcap = 0;
    g->d_cost = dalloc<float>(nb * k);
    g->d_e2 = dalloc<double>(nb * k);
    g->costcap = nb * k;
  }
  ensure_alloc(g->d_candT, (size_t)bltc::kMlpMaxOut * (bltc::kMaxDegree + 1));
  ensure_alloc(g->d_candn, bltc::kMlpMaxOut);
}

// Judge sums (sum of cnt |u_fb|^2, sum of cnt |u - u_fb|^2) over the one
// sample per batch; `out` NULL gives the weights only.
void judge_sums(bltc_targets g, int kernel, const double* out, double sums[2],
                hipStream_t s) {
  hipchk(bltc::launch_judge(g->nsamp, g->sstride, g->nb, g->d_bptr, g->d_spos,
                            g->d_tperm, out, g->m, odim_of(kernel), g->d_ufb, g->d_usq,
                            g->d_contrib, g->d_part, g->d_sums, s),
         "judge");
  d2h(sums, g->d_sums, 2, s);
  sync(s);
}

void evaluate_adaptive(bltc_tree t, bltc_targets g, int kernel, double eps,
                       bltc_selector sel, double tol, int mode, int fb_degree, double fb_theta,
                       const bltc_options& o, double* out, int32_t* choice_out,
                       int64_t* stats, double* judge, hipStream_t s) {
  const int64_t nb = g->nb;
  int64_t st[4] = {nb, 0, 0, 0};
  double jd[2] = {0.0, 0.0};
  if (g->m == 0) {
    if (stats) std::memcpy(stats, st, sizeof st);
    if (judge) std::memcpy(judge, jd, sizeof jd);
    return;
  }
  const int k = sel->k;
  const int rule_min = sel->deg_min;
  const bltc::Costs costs{(float)sel->cost_far, (float)sel->cost_row, (float)sel->cost_clu,
                          (float)sel->cost_near};
  ensure_selection_scratch(g, k);

  Events evs;
  hipEvent_t start = evs.make();
  hipchk(hipEventRecord(start, s), "hipEventRecord");

  // 1. predicted log10 errors of every candidate, and their modelled costs
  compute_features(t, g, kernel, eps, sel->theta_ref, sel->d_mean, sel->d_std, g->d_feat, s);
  hipchk(bltc::launch_mlp_forward(sel->d_params, g->d_feat, nb, k, g->d_Y, nullptr, s),
         "mlp forward");
  candidate_costs(t, g, k, sel->cand_n.data(), sel->cand_theta.data(), rule_min, costs,
                  g->d_cost, s);
  hipchk(bltc::launch_pred_err2(g->d_Y, k, nb, g->d_e2, s), "predicted errors");

  // 2. on a library stream, concurrent with step 1 (the two are independent;
  //    enqueued second because sizing the samples' lists waits on the host),
  //    the judge: the fallback treecode (Algorithm 2 with the per-target MAC)
  //    at one sample per judge_stride(nb) batches
  hipStream_t jstream = side_stream(0);
  hipchk(hipStreamWaitEvent(jstream, start, 0), "hipStreamWaitEvent");
  fallback_samples(t, g, kernel, eps, fb_degree, fb_theta, jstream);
  hipEvent_t judged = evs.make();
  hipchk(hipEventRecord(judged, jstream), "hipEventRecord");
  hipchk(hipStreamWaitEvent(s, judged, 0), "hipStreamWaitEvent");

  double ws[2];
  judge_sums(g, kernel, nullptr, ws, s);
  hipchk(bltc::launch_batch_weights(nb, g->sstride, g->d_bptr, g->d_usq, g->d_wt, s),
         "batch weights");
  const double wsum = ws[0];

  if (mode == BLTC_SELECT_RUN) {
    // 3. one candidate for the whole run: the cheapest whose predicted global
    //    error sqrt(sum_b wn_b e_b^2) is within tau = kJudgeTrigger tol
    //    10^-margin_global (the judge's trigger, so a choice as predicted is
    //    not re-evaluated)
    const double tau = kJudgeTrigger * tol * std::pow(10.0, -sel->margin_global);
    const double inv_w = wsum > 0.0 ? 1.0 / (wsum * tau * tau) : 0.0;
    hipchk(bltc::launch_cand_totals(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w, g->d_sums, s),
           "candidate totals");
    std::vector<double> tot(2 * (size_t)k);
    d2h(tot.data(), g->d_sums, 2 * (size_t)k, s);
    sync(s);
    int best = -1, most = 0;
    for (int j = 0; j < k; ++j) {
      if (tot[2 * j + 1] < tot[2 * most + 1]) most = j;
      if (tot[2 * j + 1] <= 1.0 && (best < 0 || tot[2 * j] < tot[2 * best])) best = j;
    }
    hipchk(bltc::launch_fill_i32(g->d_choice, nb, best >= 0 ? best : most, s), "choice");
  } else {
  // 3. error budget: minimise the modelled cost subject to
  //    sum_b wn_b e_b^2 <= tau^2,  wn_b = w_b / sum w,
  //    tau = kJudgeTrigger tol 10^-margin,
  //    by the multiplier lam of cost + lam wn e^2 / tau^2 (two grid passes)
  const double tau = kJudgeTrigger * tol * std::pow(10.0, -sel->margin);
  const double inv_w = wsum > 0.0 ? 1.0 / (wsum * tau * tau) : 0.0;
  double lam_star = 0.0;
  if (inv_w > 0.0) {
    double lo = 0.0, hi = 24.0;   // log10 of the multiplier range
    lam_star = std::pow(10.0, hi);
    std::vector<double> lam(kLamGrid), sums(2 * kLamGrid);
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < kLamGrid; ++i)
        lam[i] = std::pow(10.0, lo + (hi - lo) * i / (kLamGrid - 1));
      h2d(g->d_lam, lam.data(), kLamGrid, s);
      hipchk(bltc::launch_alloc(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w,
                                g->d_lam, kLamGrid, g->d_part, g->d_sums, s),
             "allocation");
      d2h(sums.data(), g->d_sums, 2 * kLamGrid, s);
      sync(s);
      // err sums are in units of tau^2 (wn carries 1/tau^2)
      int first = -1;
      for (int i = 0; i < kLamGrid; ++i)
        if (sums[2 * i + 1] <= 1.0) {
          first = i;
          break;
        }
      if (first < 0) {         // not even the most accurate choices meet it
        lam_star = lam[kLamGrid - 1];
        break;
      }
      lam_star = lam[first];
      if (first == 0) break;   // the cheapest choices already meet it
      const double step = (hi - lo) / (kLamGrid - 1);
      hi = lo + step * first;
      lo = hi - step;
    }
  }
  hipchk(bltc::launch_choose(g->d_e2, k, nb, g->d_cost, g->d_wt, inv_w,
                             lam_star, g->d_choice, s),
         "choose");
  }
  std::vector<int32_t> choice(nb);
  d2h(choice.data(), g->d_choice, nb, s);
  sync(s);

  // 4. lists at each batch's theta; modified weights of every chosen degree
  //    for the clusters its batches use; evaluation grouped by degree
  std::vector<double> th(nb);
  std::map<int, std::vector<int32_t>> by_degree;
  for (int64_t b = 0; b < nb; ++b) {
    th[b] = sel->cand_theta[choice[b]];
    by_degree[sel->cand_n[choice[b]]].push_back((int32_t)b);
  }
  st[1] = (int64_t)by_degree.size();
  h2d(g->d_theta_b, th.data(), nb, s);
  {
    bltc::ListArgs extra;
    extra.choice = g->d_choice;
    extra.cand_T = g->d_candT;
    extra.cand_deg = g->d_candn;
    extra.rule_deg_min = rule_min;
    int64_t np = 0, nd = 0;
    build_lists(t, g, 0.0, g->d_theta_b, g->ls[0], s, &np, &nd, nullptr, &extra);
  }
  std::vector<int32_t> order;
  std::vector<std::pair<int, std::pair<int64_t, int64_t>>> spans;
  for (auto& kv : by_degree) {
    spans.push_back({kv.first, {(int64_t)order.size(), (int64_t)kv.second.size()}});
    order.insert(order.end(), kv.second.begin(), kv.second.end());
  }
  h2d(g->d_bmap, order.data(), nb, s);
  // each group's top degree and, with the rule, the lower degrees derived
  // from it (a batch's result then depends on its own top degree only)
  std::vector<std::pair<int, std::pair<const int32_t*, int64_t>>> grp;
  for (auto& sp : spans) {
    ensure_degree(t, sp.first, s);
    grp.push_back({sp.first, {g->d_bmap + sp.second.first, sp.second.second}});
  }
  derive_used_degrees(t, g, g->ls[0], rule_min, grp, s);
  bltc_options og = o;
  og.deg_min = rule_min;
  // the degree groups write disjoint targets: with more than one, they run
  // concurrently on side streams, largest first; each group's batches in the
  // launch order of a fixed evaluation (by decreasing modelled work, dealt
  // to the XCDs)
  // (a launch under 8 waves per SIMD slices its batches' lists: a lone group
  // as a fixed evaluation, bit for bit; a small degree group more finely)
  const int wpb = (g->batch_size + bltc::kWave - 1) / bltc::kWave;
  const int od = odim_of(kernel);
  if (spans.size() == 1) {
    const int nsl = slices_for(nb, wpb, od);
    double* spart = nsl > 1 ? spart_reserve(g, slices_bytes(nb, wpb, od, nsl) / 8) : nullptr;
    const std::vector<Dealt> d =
        deal_batches(g, g->ls[0], s, {{spans[0].first, order.data(), nb, nsl}});
    run_p2p(t, g, g->ls[0], kernel, eps, spans[0].first, og, g->d_xmap + d[0].off, nb, out, s,
            nullptr, 0, nullptr, g->d_xstart, d[0].xmax, nsl, spart);
  } else {
    std::sort(spans.begin(), spans.end(), [](const auto& a, const auto& b) {
      const double wa = (double)a.second.second * std::pow(a.first + 1.0, 3);
      const double wb = (double)b.second.second * std::pow(b.first + 1.0, 3);
      return wa > wb;
    });
    std::vector<DealGroup> dg;
    std::vector<int64_t> soff;   // each group's slice sums in the shared buffer
    int64_t stot = 0;
    for (auto& sp : spans) {
      const int k = slices_for(sp.second.second, wpb, od);
      dg.push_back({sp.first, order.data() + sp.second.first, sp.second.second, k});
      soff.push_back(stot);
      if (k > 1) stot += slices_bytes(sp.second.second, wpb, od, k) / 8;
    }
    double* spart = stot > 0 ? spart_reserve(g, stot) : nullptr;
    const std::vector<Dealt> d = deal_batches(g, g->ls[0], s, dg);
    hipEvent_t ready = evs.make();
    hipchk(hipEventRecord(ready, s), "hipEventRecord");
    std::vector<hipEvent_t> done;
    for (size_t i = 0; i < spans.size(); ++i) {
      hipStream_t ss = side_stream((int)i);
      hipchk(hipStreamWaitEvent(ss, ready, 0), "hipStreamWaitEvent");
      run_p2p(t, g, g->ls[0], kernel, eps, spans[i].first, og, g->d_xmap + d[i].off,
              spans[i].second.second, out, ss, nullptr, 0, nullptr, g->d_xstart + 9 * i,
              d[i].xmax, dg[i].slices, dg[i].slices > 1 ? spart + soff[i] : nullptr);
      if (i + kSideStreams >= spans.size()) {   // last launch on this side stream
        hipEvent_t e = evs.make();
        hipchk(hipEventRecord(e, ss), "hipEventRecord");
        done.push_back(e);
      }
    }
    for (hipEvent_t e : done) hipchk(hipStreamWaitEvent(s, e, 0), "hipStreamWaitEvent");
  }

  // 5. the judge's estimate of the global error; when it exceeds
  //    kJudgeTrigger tol, the batches with the largest sampled errors are
  //    evaluated again with the fallback until the estimate is at most
  //    kJudgeTarget tol.  The margins
  //    cover the sampled estimate's spread: the per-target errors are heavy
  //    tailed (a few targets next to accepted clusters of a dense region
  //    carry much of the sum), so one sample per batch reads low more often
  //    than high, and the samples with the largest terms overstate their
  //    batches' errors, so their removal lowers the estimate by more than
  //    it lowers the error.
  double js[2];
  judge_sums(g, kernel, out, js, s);
  jd[0] = jd[1] = wsum > 0.0 ? std::sqrt(js[1] / wsum) : 0.0;
  if (js[1] > kJudgeTrigger * kJudgeTrigger * tol * tol * wsum) {
    // the fewest samples, largest terms first, whose removal brings the
    // estimate to (kJudgeTarget tol)^2; their batches go to the fallback
    const int ns = g->nsamp;
    std::vector<double> c(ns);
    d2h(c.data(), g->d_contrib, ns, s);
    sync(s);
    std::vector<int32_t> ord(ns);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return c[a] > c[b]; });
    double rest = js[1];
    std::vector<int32_t> redo;
    for (int32_t i : ord) {
      if (rest <= kJudgeTarget * kJudgeTarget * tol * tol * wsum) break;
      rest -= c[i];
      for (int64_t b = (int64_t)i * g->sstride;
           b < std::min<int64_t>(nb, (int64_t)(i + 1) * g->sstride); ++b) {
        redo.push_back((int32_t)b);
        choice[b] = -2;
      }
    }
    std::sort(redo.begin(), redo.end());
    st[2] = (int64_t)redo.size();
    if (!redo.empty()) {
      int64_t np = 0, nd = 0;   // the fallback's batch lists
      build_lists(t, g, fb_theta, nullptr, g->ls[1], s, &np, &nd);
      h2d(g->d_bmap, redo.data(), redo.size(), s);
      if (g->batch_size <= bltc::kWave) {
        // few batches: each batch's proxy list and its direct list are cut
        // into slices that run as separate waves (about 4096 of each over
        // all batches); the slices' FP64 sums are added in slice order.  A
        // direct slice starts only where a new run of contiguous leaf
        // particles starts, so the near field's 64-source chunks, and their
        // FP32 sums, are those of the uncut list.
        std::vector<int32_t> lp(2 * (nb + 1));
        std::vector<int32_t> dl(nd);
        d2h(lp.data(), g->ls[1].ptr, 2 * (nb + 1), s);
        d2h(dl.data(), g->ls[1].dids, nd, s);
        sync(s);
        const int32_t* ld = lp.data() + nb + 1;
        const std::vector<int32_t>& lb = t->host.begin;
        const std::vector<int32_t>& le = t->host.end;
        int64_t tot = 0, tsrc = 0;
        for (int32_t b : redo) {
          tot += lp[b + 1] - lp[b];
          for (int32_t e = ld[b]; e < ld[b + 1]; ++e) tsrc += le[dl[e]] - lb[dl[e]];
        }
        const int64_t len = std::max<int64_t>(16, (tot + 4095) / 4096);
        const int64_t srcs = std::max<int64_t>(1024, (tsrc + 4095) / 4096);
        std::vector<int4> sl;   // (batch, begin, end, 0: proxy entries / 1: direct entries)
        std::vector<int32_t> sptr{0};
        for (int32_t b : redo) {
          const int32_t p0 = lp[b], p1 = lp[b + 1], d0 = ld[b], d1 = ld[b + 1];
          for (int64_t q = p0; q < p1; q += len)
            sl.push_back(make_int4(b, (int)q, (int)std::min<int64_t>(p1, q + len), 0));
          int32_t q = d0;
          int64_t acc = 0;
          for (int32_t e = d0; e < d1; ++e) {
            if (e > q && acc >= srcs && lb[dl[e]] != le[dl[e - 1]]) {
              sl.push_back(make_int4(b, q, e, 1));
              q = e;
              acc = 0;
            }
            acc += le[dl[e]] - lb[dl[e]];
          }
          if (q < d1) sl.push_back(make_int4(b, q, d1, 1));
          if (p0 == p1 && d0 == d1) sl.push_back(make_int4(b, p0, p0, 0));
          sptr.push_back((int32_t)sl.size());
        }
        const int odim = odim_of(kernel);
        if (!g->split) g->split = new bltc_split_cache;
        DevBuf<int4>& d_sl = g->split->sl;
        DevBuf<int32_t>& d_sptr = g->split->sptr;
        DevBuf<double>& d_part = g->split->part;
        d_sl.reserve(sl.size());
        d_sptr.reserve(sptr.size());
        d_part.reserve(sl.size() * odim * bltc::kWave);
        h2d(d_sl.p, sl.data(), sl.size(), s);
        h2d(d_sptr.p, sptr.data(), sptr.size(), s);
        run_p2p(t, g, g->ls[1], kernel, eps, fb_degree, o, g->d_bmap, (int64_t)redo.size(),
                out, s, d_sl.p, (int64_t)sl.size(), d_part.p);
        double su, sw;
        kernel_scales(kernel, &su, &sw);
        hipchk(bltc::launch_split_reduce(d_sptr.p, g->d_bmap, (int64_t)redo.size(), g->d_bptr,
                                         g->d_tperm, d_part.p, odim, su, sw, g->m, out, s),
               "split reduce");
        judge_sums(g, kernel, out, js, s);
      } else {
        run_p2p(t, g, g->ls[1], kernel, eps, fb_degree, o, g->d_bmap, (int64_t)redo.size(),
                out, s);
        judge_sums(g, kernel, out, js, s);
      }
      jd[1] = std::sqrt(js[1] / wsum);
    }
  }
  sync(s);
  if (choice_out) std::memcpy(choice_out, choice.data(), sizeof(int32_t) * nb);
  if (stats) std::memcpy(stats, st, sizeof st);
  if (judge) std::memcpy(judge, jd, sizeof jd);
}

// Selector model file (little endian):
//   char magic[8] "BLTCSEL1"; int32 version (4); int32 n_in (12);
//   int32 n_hidden (64); int32 k; int32 deg_min (separation rule, 0 = off);
//   int32 cand_n[k]; double cand_theta[k];
//   double theta_ref, cost_far, cost_row, cost_cluster, cost_near, margin,
//   margin_global;
//   float mean[12], stdv[12]; float params[bltc_mlp_params(k)];
//   uint64 FNV-1a hash of all preceding bytes.
uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

int load_selector(const char* path, bltc_selector sel) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(BLTC_EMODEL, std::string("cannot open selector model ") + path);
  std::vector<unsigned char> buf;
  unsigned char tmp[4096];
  size_t r;
  while ((r = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
  std::fclose(f);
  size_t off = 0;
  auto take = [&](void* dst, size_t n) {
    if (off + n > buf.size()) return false;
    std::memcpy(dst, buf.data() + off, n);
    off += n;
    return true;
  };
  char magic[8];
  int32_t hdr[5];
  if (!take(magic, 8) || std::memcmp(magic, "BLTCSEL1", 8) != 0 || !take(hdr, sizeof hdr))
    return fail(BLTC_EMODEL, "selector model: bad magic or header");
  if (hdr[4] < 0 || hdr[4] > bltc::kMaxDegree)
    return fail(BLTC_EMODEL, "selector model: deg_min out of range");
  if (hdr[0] != 4 || hdr[1] != bltc::kMlpIn || hdr[2] != bltc::kMlpHidden || hdr[3] < 1 ||
      hdr[3] > bltc::kMlpMaxOut)
    return fail(BLTC_EMODEL, "selector model: unsupported version or dimensions");
  const int32_t k = hdr[3];
  sel->k = k;
  sel->deg_min = hdr[4];
  sel->cand_n.resize(k);
  sel->cand_theta.resize(k);
  double tail[7];
  sel->mean.resize(bltc::kMlpIn);
  sel->stdv.resize(bltc::kMlpIn);
  sel->params.resize(bltc::mlp_params(k));
  if (!take(sel->cand_n.data(), 4 * (size_t)k) || !take(sel->cand_theta.data(), 8 * (size_t)k) ||
      !take(tail, sizeof tail) || !take(sel->mean.data(), 4 * bltc::kMlpIn) ||
      !take(sel->stdv.data(), 4 * bltc::kMlpIn) ||
      !take(sel->params.data(), 4 * sel->params.size()))
    return fail(BLTC_EMODEL, "selector model: truncated");
  const uint64_t want = fnv1a(buf.data(), off);
  uint64_t got = 0;
  if (!take(&got, 8) || got != want || off != buf.size())
    return fail(BLTC_EMODEL, "selector model: checksum mismatch or trailing bytes");
  sel->theta_ref = tail[0];
  sel->cost_far = tail[1];
  sel->cost_row = tail[2];
  sel->cost_clu = tail[3];
  sel->cost_near = tail[4];
  sel->margin = tail[5];
  sel->margin_global = tail[6];
  for (int i = 1; i < 5; ++i)
    if (!(tail[i] >= 0.0 && tail[i] < 1e6))
      return fail(BLTC_EMODEL, "selector model: cost weight out of range");
  if (!(tail[5] > -6.0 && tail[5] < 6.0) || !(tail[6] > -6.0 && tail[6] < 6.0))
    return fail(BLTC_EMODEL, "selector model: margin out of range");
  for (int j = 0; j < k; ++j)
    if (sel->cand_n[j] < 1 || sel->cand_n[j] > bltc::kMaxDegree ||
        !(sel->cand_theta[j] >= 0.0 && sel->cand_theta[j] <= 1.0))
      return fail(BLTC_EMODEL, "selector model: candidate out of range");
  for (int i = 0; i < bltc::kMlpIn; ++i)
    if (!(sel->stdv[i] > 0.f)) return fail(BLTC_EMODEL, "selector model: non-positive std");
  return BLTC_OK;
}

}  // namespace

}  // namespace api
}  // namespace bltc

using namespace bltc::api;

extern "C" {

int bltc_selector_load(const char* path, bltc_selector* out) {
  if (!out) return fail(BLTC_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  if (!path) return fail(BLTC_EINVAL, "NULL path");
  bltc_selector sel = new bltc_selector_s;
  if (int rc = load_selector(path, sel)) {
    delete sel;
    return rc;
  }
  int rc = guarded([&] {
    sel->d_params = dalloc<float>(sel->params.size());
    sel->d_mean = dalloc<float>(bltc::kMlpIn);
    sel->d_std = dalloc<float>(bltc::kMlpIn);
    h2d(sel->d_params, sel->params.data(), sel->params.size(), nullptr);
    h2d(sel->d_mean, sel->mean.data(), bltc::kMlpIn, nullptr);
    h2d(sel->d_std, sel->stdv.data(), bltc::kMlpIn, nullptr);
    sync(nullptr);
    return (int)BLTC_OK;
  });
  if (rc) {
    dfree(sel->d_params); dfree(sel->d_mean); dfree(sel->d_std);
    delete sel;
    return rc;
  }
  *out = sel;
  return BLTC_OK;
}

int bltc_selector_destroy(bltc_selector sel) {
  if (!sel) return BLTC_OK;
  dfree(sel->d_params); dfree(sel->d_mean); dfree(sel->d_std);
  delete sel;
  return BLTC_OK;
}

int bltc_selector_info(bltc_selector sel, int32_t* k, int32_t* cand_n,
                       double* cand_theta) {
  if (!sel) return fail(BLTC_EINVAL, "NULL selector");
  if (k) *k = sel->k;
  for (int j = 0; j < sel->k; ++j) {
    if (cand_n) cand_n[j] = sel->cand_n[j];
    if (cand_theta) cand_theta[j] = sel->cand_theta[j];
  }
  return BLTC_OK;
}

int bltc_batch_features(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                        double theta_ref, float* feat, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (kernel != BLTC_STOKESLET && kernel != BLTC_ROTLET)
    return fail(BLTC_EINVAL, "features are defined for the Stokeslet and rotlet kernels");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BLTC_EINVAL, "eps must be finite and >= 0");
  if (!(theta_ref > 0.0 && theta_ref <= 1.0)) return fail(BLTC_EINVAL, "theta_ref must be in (0, 1]");
  if (g->nb > 0 && !device_ptr(feat)) return fail(BLTC_EINVAL, "feat must be a device pointer");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    compute_features(t, g, kernel, eps, theta_ref, nullptr, nullptr, feat, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_batch_costs(bltc_tree t, bltc_targets g, int32_t k, const int32_t* cand_n,
                     const double* cand_theta, int32_t deg_min, const float* weights,
                     float* cost, void* stream) {
  if (!t || !g || !cand_n || !cand_theta || !weights)
    return fail(BLTC_EINVAL, "NULL tree, targets, candidates or weights");
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (deg_min < 0 || deg_min > bltc::kMaxDegree)
    return fail(BLTC_EINVAL, "deg_min must be in [0, 12]");
  for (int j = 0; j < k; ++j)
    if (cand_n[j] < 1 || cand_n[j] > bltc::kMaxDegree ||
        !(cand_theta[j] >= 0.0 && cand_theta[j] <= 1.0))
      return fail(BLTC_EINVAL, "candidate out of range");
  for (int i = 0; i < 4; ++i)
    if (!(weights[i] >= 0.f)) return fail(BLTC_EINVAL, "cost weights must be >= 0");
  if (g->nb > 0 && !device_ptr(cost)) return fail(BLTC_EINVAL, "cost must be a device pointer");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    const bltc::Costs w{weights[0], weights[1], weights[2], weights[3]};
    candidate_costs(t, g, k, cand_n, cand_theta, deg_min, w, cost, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_batch_counts(bltc_tree t, bltc_targets g, double theta, int32_t* n_proxy,
                      int32_t* n_near, void* stream) {
  if (!t || !g) return fail(BLTC_EINVAL, "NULL tree or targets");
  if (!(theta >= 0.0 && theta <= 1.0)) return fail(BLTC_EINVAL, "theta must be in [0, 1]");
  if (g->nb > 0 && (!device_ptr(n_proxy) || !device_ptr(n_near)))
    return fail(BLTC_EINVAL, "n_proxy and n_near must be device pointers");
  if (g->nb == 0) return BLTC_OK;
  return guarded([&] {
    batch_counts(t, g, theta, n_proxy, n_near, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_evaluate_adaptive(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                           bltc_selector sel, double tol, int32_t mode, int32_t fb_degree,
                           double fb_theta, const bltc_options* opt, double* out,
                           int32_t* choice, int64_t* stats, double* judge, void* stream) {
  if (!t || !g || !sel) return fail(BLTC_EINVAL, "NULL tree, targets or selector");
  if (kernel != BLTC_STOKESLET && kernel != BLTC_ROTLET)
    return fail(BLTC_EINVAL, "the selector serves the Stokeslet and rotlet kernels");
  if (int rc = check_eval(kernel, eps, fb_degree, fb_theta)) return rc;
  if (!(tol > 0.0 && tol < 1.0)) return fail(BLTC_EINVAL, "tol must be in (0, 1)");
  if (mode != BLTC_SELECT_BATCH && mode != BLTC_SELECT_RUN)
    return fail(BLTC_EINVAL, "mode must be BLTC_SELECT_BATCH or BLTC_SELECT_RUN");
  bltc_options o;
  bltc_options_default(&o);
  if (opt) o = *opt;
  o.deg_min = 0;   // the candidates take the model's rule, the fallback none
  if (int rc = check_options(&o, kernel)) return rc;
  if (g->m > 0 && !device_ptr(out)) return fail(BLTC_EINVAL, "out must be a device pointer");
  if (!t->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (t->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  return guarded([&] {
    evaluate_adaptive(t, g, kernel, eps, sel, tol, mode, fb_degree, fb_theta, o, out, choice,
                      stats, judge, (hipStream_t)stream);
    return (int)BLTC_OK;
  });
}

int bltc_judge_samples(bltc_tree t, bltc_targets g, int32_t kernel, double eps,
                       int32_t fb_degree, double fb_theta, int64_t* n_samples,
                       int64_t* target_idx, double* ufb, void* stream) {
  if (!t || !g || !n_samples) return fail(BLTC_EINVAL, "NULL tree, targets or n_samples");
  if (kernel != BLTC_STOKESLET && kernel != BLTC_ROTLET)
    return fail(BLTC_EINVAL, "the judge serves the Stokeslet and rotlet kernels");
  if (int rc = check_eval(kernel, eps, fb_degree, fb_theta)) return rc;
  if (!t->has_w) return fail(BLTC_ESTATE, "no weights: call bltc_compute_modified_weights first");
  if (t->wdim != wdim_of(kernel))
    return fail(BLTC_ESTATE, "the tree's weights have the wrong number of components for this kernel");
  const int st = bltc::judge_stride(g->nb);
  *n_samples = g->m > 0 ? (g->nb + st - 1) / st : 0;
  if (!target_idx && !ufb) return BLTC_OK;
  if (g->m == 0) return BLTC_OK;
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    fallback_samples(t, g, kernel, eps, fb_degree, fb_theta, s);
    const int64_t ns = g->nsamp;
    std::vector<int32_t> sp(ns);
    std::vector<double> u((size_t)ns * odim_of(kernel));
    d2h(sp.data(), g->d_spos, ns, s);
    d2h(u.data(), g->d_ufb, u.size(), s);
    sync(s);
    for (int64_t i = 0; i < ns; ++i)
      if (target_idx) target_idx[i] = g->host.perm[sp[i]];
    if (ufb) std::memcpy(ufb, u.data(), sizeof(double) * u.size());
    return (int)BLTC_OK;
  });
}

int bltc_mlp_params(int32_t k, int64_t* n_params) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (!n_params) return fail(BLTC_EINVAL, "NULL output");
  *n_params = bltc::mlp_params(k);
  return BLTC_OK;
}

int bltc_mlp_work_size(int64_t rows, int32_t k, int64_t* n_floats) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0 || !n_floats) return fail(BLTC_EINVAL, "bad rows or NULL output");
  *n_floats = std::max<int64_t>(bltc::mlp_work_floats(rows, k), (rows * k + 255) / 256 + 1);
  return BLTC_OK;
}

int bltc_mlp_forward(const float* params, const float* X, int64_t rows,
                     int32_t k, float* Y, float* cache, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (rows == 0) return BLTC_OK;
  if (!device_ptr(params) || !device_ptr(X) || !device_ptr(Y) || (cache && !device_ptr(cache)))
    return fail(BLTC_EINVAL, "params, X, Y and cache must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_forward(params, X, rows, k, Y, cache, (hipStream_t)stream),
           "mlp forward");
    return (int)BLTC_OK;
  });
}

int bltc_mlp_loss(const float* Y, const float* T, int64_t rows, int32_t k,
                  float* dY, float* loss, float* work, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (rows == 0) return BLTC_OK;
  if (!device_ptr(Y) || !device_ptr(T) || !device_ptr(dY) || !device_ptr(loss) || !device_ptr(work))
    return fail(BLTC_EINVAL, "Y, T, dY, loss and work must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_loss(Y, T, rows * k, dY, loss, work, (hipStream_t)stream),
           "mlp loss");
    return (int)BLTC_OK;
  });
}

int bltc_mlp_backward(const float* params, const float* X, const float* cache,
                      const float* dY, int64_t rows, int32_t k, float* grad,
                      float* work, void* stream) {
  if (k < 1 || k > bltc::kMlpMaxOut) return fail(BLTC_EINVAL, "k must be in [1, 128]");
  if (rows < 0) return fail(BLTC_EINVAL, "rows must be >= 0");
  if (!device_ptr(params) || !device_ptr(grad) || !device_ptr(work) ||
      (rows > 0 && (!device_ptr(X) || !device_ptr(cache) || !device_ptr(dY))))
    return fail(BLTC_EINVAL, "params, X, cache, dY, grad and work must be device pointers");
  return guarded([&] {
    hipchk(bltc::launch_mlp_backward(params, X, cache, dY, rows, k, grad, work,
                                     (hipStream_t)stream),
           "mlp backward");
    return (int)BLTC_OK;
  });
}

int bltc_adam_step(float* params, float* m, float* v, const float* grad,
                   int64_t n, float lr, float beta1, float beta2, float eps,
                   int64_t step, void* stream) {
  if (n < 0 || step < 1) return fail(BLTC_EINVAL, "n must be >= 0 and step >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return fail(BLTC_EINVAL, "beta1 and beta2 must be in [0, 1)");
  if (n == 0) return BLTC_OK;
  if (!device_ptr(params) || !device_ptr(m) || !device_ptr(v) || !device_ptr(grad))
    return fail(BLTC_EINVAL, "params, m, v and grad must be device pointers");
  return guarded([&] {
    const double bc1 = 1.0 - std::pow((double)beta1, (double)step);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)step);
    hipchk(bltc::launch_adam(params, m, v, grad, n, lr, beta1, beta2, eps, (float)bc1,
                             (float)bc2, (hipStream_t)stream),
           "adam");
    return (int)BLTC_OK;
  });
}

}  // extern "C"
