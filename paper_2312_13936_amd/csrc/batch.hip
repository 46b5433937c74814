// Fused batch driver: many graphs as one disjoint union, one launch sequence.
//
// The graphs of a batch are laid side by side in one union CSR; every pass
// of Alg. 1 runs on the union, so each kernel launch works on all graphs
// that are still running, and a thousand small graphs cost about as many
// launches as one.  Each graph keeps its own state where Alg. 1 and Alg. 2
// are per graph: its total weight W and resolution (the gains of Eq. 2),
// the sum of its move gains and its own stop of local-moving (Alg. 2), its
// refinement moves, community count and zero-degree vertices (the stop tests
// of Alg. 1), the pass at which it ends, and its own vertex ids for the
// sub-sweep groups.  Labels of a graph are its solo labels shifted by a
// per-graph constant, so every comparison (lowest id on ties, the min-label
// rule) falls the same way: a graph's result is the one gvl_leiden returns
// for it alone (bit-identical in deterministic mode).
//
// Per pass, with A the graphs still running:
//   bins / hub plan / K' of the union; W and the gains' constants per graph
//   local-moving: per iteration read back each graph's gain sum; a graph
//     whose sum is <= tau stops (its flags are cleared)
//   refinement: sweeps until no vertex of the union moves (a graph with no
//     move in a sweep has none in any later sweep: nothing it reads changed)
//   per graph: communities, zero-degree vertices, refinement moves -> stop
//     (converged, low shrink, last pass) or continue
//   graphs that stop write their refined labels into the dendrogram, moved
//   into their own id range; the others are renumbered, looked up and
//   aggregated into the next union
// then the canonical relabelling per graph, the results written to each
// graph's output, and Eq. 1 per graph.
#include "host.hpp"

namespace gvl {
namespace {

// union graphs stay below 2^31 arcs (int32 offsets)
constexpr int64_t kFusedMaxArcs = 1500000000;
constexpr int64_t kFusedMaxVerts = 1500000000;

// Per-graph device arrays of one fused run, carved after the union
// workspace.
struct BatchArea {
  const int32_t** off;
  const int32_t** idx;
  const float** w;
  int32_t** out;
  int64_t *n, *m, *vb, *ub, *uab;
  int32_t *src, *flags, *vcur, *pos, *gath, *goff0, *nz, *cb, *gsh;
  double *W, *dqg, *s1g, *s2d;
  unsigned long long *dqg128, *mvg, *s2u;
  GraphParam* gp;
  uint8_t *active, *keep, *state;
  // union
  int32_t *uoff, *uidx, *gid0, *gidA, *gidB, *top;
  float* uw;
  size_t bytes;
};

BatchArea carve_batch(int64_t G, int64_t N, int64_t M, char* base) {
  BatchArea b;
  memset(&b, 0, sizeof(b));
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + o : nullptr;
    o += align_up(bytes);
    return p;
  };
  const size_t g = (size_t)std::max<int64_t>(G, 1), n = (size_t)std::max<int64_t>(N, 1),
               m = (size_t)std::max<int64_t>(M, 1);
  b.off = (const int32_t**)take(sizeof(void*) * g);
  b.idx = (const int32_t**)take(sizeof(void*) * g);
  b.w = (const float**)take(sizeof(void*) * g);
  b.out = (int32_t**)take(sizeof(void*) * g);
  b.n = (int64_t*)take(8 * g);
  b.m = (int64_t*)take(8 * g);
  b.vb = (int64_t*)take(8 * (g + 1));
  b.ub = (int64_t*)take(8 * (g + 1));
  b.uab = (int64_t*)take(8 * (g + 1));
  b.src = (int32_t*)take(4 * g);
  b.flags = (int32_t*)take(4 * g);
  b.vcur = (int32_t*)take(4 * g);
  b.gsh = (int32_t*)take(4 * g);
  b.pos = (int32_t*)take(4 * (g + 1));
  b.gath = (int32_t*)take(4 * (g + 1));
  b.goff0 = (int32_t*)take(4 * (g + 1));
  b.nz = (int32_t*)take(4 * g);
  b.cb = (int32_t*)take(4 * (g + 1));
  b.W = (double*)take(8 * g);
  b.dqg = (double*)take(8 * g);
  b.s1g = (double*)take(8 * g);
  b.s2d = (double*)take(8 * g);
  b.dqg128 = (unsigned long long*)take(16 * g);
  b.mvg = (unsigned long long*)take(8 * g);
  b.s2u = (unsigned long long*)take(16 * g);
  b.gp = (GraphParam*)take(sizeof(GraphParam) * g);
  b.active = (uint8_t*)take(g);
  b.keep = (uint8_t*)take(g);
  b.state = (uint8_t*)take(g);
  b.uoff = (int32_t*)take(4 * (n + 1));
  b.uidx = (int32_t*)take(4 * m);
  b.uw = (float*)take(4 * m);
  b.gid0 = (int32_t*)take(4 * n);
  b.gidA = (int32_t*)take(4 * n);
  b.gidB = (int32_t*)take(4 * n);
  b.top = (int32_t*)take(4 * n);
  b.bytes = o;
  return b;
}

// Graphs [g0, g1) of the batch form one fused run.
struct Chunk {
  int32_t g0, g1;
  int64_t n, m, nmax;  // vertices, arcs, largest graph
};

std::vector<Chunk> plan_chunks(int32_t num, const gvl_graph_desc* gs) {
  std::vector<Chunk> out;
  Chunk c{0, 0, 0, 0, 0};
  for (int32_t g = 0; g < num; ++g) {
    const int64_t n = std::max<int64_t>(gs[g].n, 0), m = std::max<int64_t>(gs[g].m, 0);
    if (c.g1 > c.g0 && (c.n + n > kFusedMaxVerts || c.m + m > kFusedMaxArcs)) {
      out.push_back(c);
      c = Chunk{g, g, 0, 0, 0};
    }
    c.g1 = g + 1;
    c.n += n;
    c.m += m;
    c.nmax = std::max(c.nmax, n);
  }
  if (c.g1 > c.g0) out.push_back(c);
  return out;
}

size_t chunk_bytes(const Chunk& c, bool det) {
  return align_up(carve(c.n, c.m, det, nullptr, c.nmax).bytes) + carve_batch(c.g1 - c.g0, c.n, c.m, nullptr).bytes;
}

// Host-to-device copy of a small host array; waits, so the host array may
// change right after.
template <class T>
gvl_status upload(hipStream_t st, T* dst, const std::vector<T>& src) {
  if (src.empty()) return GVL_OK;
  HIP_TRY(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return GVL_OK;
}
template <class T>
gvl_status download(hipStream_t st, std::vector<T>& dst, const T* src, size_t count) {
  dst.resize(count);
  if (count == 0) return GVL_OK;
  HIP_TRY(hipMemcpyAsync(dst.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return GVL_OK;
}

gvl_status fused_chunk(gvl_ctx* ctx, int32_t G, const gvl_graph_desc* gs, const gvl_options* opt, char* wsbase,
                       const Chunk& ch, double* qs, gvl_status* sts) {
  hipStream_t st = ctx->stream;
  const bool det = opt->mode == GVL_MODE_DET;
  Workspace ws = carve(ch.n, ch.m, det, wsbase, ch.nmax);
  BatchArea B = carve_batch(G, ch.n, ch.m, wsbase + align_up(ws.bytes));
  gvl_status s = GVL_OK;

  // ---- per-graph argument checks (host), then validation of the CSRs
  std::vector<int32_t> ok(G, 0);
  std::vector<int64_t> hn(G, 0), hm(G, 0), hvb(G + 1, 0);
  std::vector<const int32_t*> hoff(G, nullptr), hidx(G, nullptr);
  std::vector<const float*> hw(G, nullptr);
  for (int32_t g = 0; g < G; ++g) {
    const gvl_graph_desc& d = gs[g];
    qs[g] = 0.0;
    gvl_status e = GVL_OK;
    if (d.n < 0 || d.m < 0 || (d.n > 0 && (!d.d_offsets || !d.d_membership)) || (d.m > 0 && !d.d_indices) ||
        (d.n == 0 && d.m > 0))
      e = GVL_E_INVALID_ARG;
    else if (!(d.resolution >= 0.0) || !std::isfinite(d.resolution))
      e = GVL_E_RESOLUTION;
    else if (det) {
      const double pd = d.resolution * 65536.0;
      if (pd != std::floor(pd) || pd > 16777216.0) e = GVL_E_RESOLUTION;
    }
    sts[g] = e;
    if (e == GVL_OK && d.n > 0) {
      ok[g] = 1;
      hn[g] = d.n;
      hm[g] = d.m;
      hoff[g] = d.d_offsets;
      hidx[g] = d.d_indices;
      hw[g] = d.d_weights;
    }
    hvb[g + 1] = hvb[g] + hn[g];
  }
  HIP_TRY(hipMemcpyAsync(B.off, hoff.data(), sizeof(void*) * G, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.idx, hidx.data(), sizeof(void*) * G, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(B.w, hw.data(), sizeof(void*) * G, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  if ((s = upload(st, B.n, hn)) != GVL_OK) return s;
  if ((s = upload(st, B.m, hm)) != GVL_OK) return s;
  if ((s = upload(st, B.vb, hvb)) != GVL_OK) return s;
  fill_i32(st, B.flags, 0, G);
  fill_f64(st, B.W, 0.0, G);
  BatchDesc bd{B.off, B.idx, B.w, B.n, B.m, B.vb, B.ub, B.uab};
  batch_validate(st, bd, G, hvb[G], B.flags, B.W);
  std::vector<int32_t> hflags;
  std::vector<double> hW;
  if ((s = download(st, hflags, B.flags, G)) != GVL_OK) return s;
  if ((s = download(st, hW, B.W, G)) != GVL_OK) return s;
  std::vector<unsigned long long> hsym;
  if (opt->validate >= 2) {  // symmetry of every graph whose CSR is in range (B.s2u as scratch)
    fill_u64(st, B.s2u, 0ull, 2 * (int64_t)G);
    for (int32_t g = 0; g < G; ++g)
      if (ok[g] && !(hflags[g] & 1))
        symmetry_check(st, gs[g].d_offsets, gs[g].d_indices, gs[g].d_weights, gs[g].n, B.s2u + 2 * g);
    if ((s = download(st, hsym, B.s2u, 2 * (size_t)G)) != GVL_OK) return s;
  }

  // ---- kept graphs: valid, with arcs; edgeless graphs are singletons
  std::vector<int32_t> src;
  std::vector<int64_t> hub(1, 0), huab(1, 0);
  std::vector<int32_t*> hout;
  for (int32_t g = 0; g < G; ++g) {
    if (!ok[g]) continue;
    const int f = hflags[g];
    if (f & 1) { sts[g] = GVL_E_BAD_CSR; continue; }
    if (f & 2) { sts[g] = GVL_E_NONINTEGER_WEIGHT; continue; }
    if (!hsym.empty() && (hsym[2 * g] != 0 || hsym[2 * g + 1] != 0)) { sts[g] = GVL_E_NOT_SYMMETRIC; continue; }
    if (det && ((f & 4) || hW[g] > 1099511627776.0)) { sts[g] = GVL_E_NONINTEGER_WEIGHT; continue; }
    if (hW[g] == 0.0) {
      iota_i32(st, gs[g].d_membership, gs[g].n);
      continue;
    }
    src.push_back(g);
    hub.push_back(hub.back() + gs[g].n);
    huab.push_back(huab.back() + gs[g].m);
    hout.push_back(gs[g].d_membership);
  }
  const int32_t K = (int32_t)src.size();
  if (K == 0) {
    HIP_TRY(hipStreamSynchronize(st));
    return GVL_OK;
  }
  const int64_t N0 = hub[K], M0 = huab[K];
  if ((s = upload(st, B.src, src)) != GVL_OK) return s;
  if ((s = upload(st, B.ub, hub)) != GVL_OK) return s;
  if ((s = upload(st, B.uab, huab)) != GVL_OK) return s;
  HIP_TRY(hipMemcpyAsync(B.out, hout.data(), sizeof(void*) * K, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  batch_build(st, bd, B.src, K, N0, B.uoff, B.uidx, B.uw, B.gidA);
  fill_i32(st, B.uoff + N0, (int32_t)M0, 1);
  copy_i32(st, B.gid0, B.gidA, N0);

  // per-graph constants of Eq. 2
  std::vector<GraphParam> hgp(K);
  std::vector<double> Wk(K), gam(K);
  std::vector<int32_t> goff0(K + 1);
  std::vector<uint8_t> integral(K);
  for (int32_t k = 0; k < K; ++k) {
    const gvl_graph_desc& d = gs[src[k]];
    Wk[k] = hW[src[k]];
    gam[k] = d.resolution;
    integral[k] = (hflags[src[k]] & 4) == 0;
    hgp[k].inv_m = 2.0 / Wk[k];
    hgp[k].gk_scale = 2.0 * d.resolution / (Wk[k] * Wk[k]);
    hgp[k].W = det ? (long long)Wk[k] : 0;
    hgp[k].p = det ? (long long)(d.resolution * 65536.0) : 0;
    goff0[k] = (int32_t)hub[k];
  }
  goff0[K] = (int32_t)N0;
  if ((s = upload(st, B.gp, hgp)) != GVL_OK) return s;
  if ((s = upload(st, B.goff0, goff0)) != GVL_OK) return s;
  // sub-sweep groups: the option, or per graph by its longest row; a graph
  // with fewer groups than the union puts its group k into union group
  // k << gsh (its groups run in the same order as alone)
  int S_union = opt->subsweeps;
  std::vector<int32_t> gsh(K, 0);
  if (opt->subsweeps == 0) {
    S_union = kAutoFewGroups;
    for (int32_t k = 0; k < K; ++k)
      if (hflags[src[k]] & 8) S_union = kAutoGroups;
    for (int32_t k = 0; k < K; ++k) {
      const int Sg = (hflags[src[k]] & 8) ? kAutoGroups : kAutoFewGroups;
      while ((Sg << gsh[k]) < S_union) ++gsh[k];
    }
  }
  if ((s = upload(st, B.gsh, gsh)) != GVL_OK) return s;

  // ---- state of the pass loop
  fill_u64(st, (unsigned long long*)ws.sc, 0ull, sizeof(Scalars) / 8);
  fill_i32(st, ws.hp_done, 0, ch.n);
  fill_i32(st, ws.hp_lcnt, 0, ch.n);
  fill_i32(st, ws.wd_done, 0, ws.max_wide);
  fill_i32(st, ws.wd_ctr, 0, 2);
  ScanArgs a;
  memset(&a, 0, sizeof(a));
  a.C = ws.C; a.CB = ws.CB; a.Sig = ws.Sig; a.size = ws.size; a.K = ws.K; a.flag = ws.flag;
  a.CP = ws.CP;
  a.mark_after = INT32_MAX;
  a.ident_after = -1;
  a.target = ws.target; a.targeted = ws.targeted;
  a.dq = ws.sc->dq; a.dq128 = &ws.sc->dq128[0][0]; a.cnt = &ws.sc->cnt[0][0];
  a.ovf = &ws.sc->ovf;
  a.gainf = ws.gainf; a.gaink = ws.gaink; a.last = ws.last; a.mv = ws.mv; a.it_dev = &ws.sc->iter;
  if (!scan_state_ready(a, det)) return GVL_E_INVALID_ARG;
  a.gsh = B.gsh;
  a.wd_g = ws.wd_g; a.wd_k = ws.wd_k; a.wd_c = ws.wd_c; a.wd_ok = ws.wd_ok; a.wd_done = ws.wd_done;
  a.wd_next = ws.wd_ctr; a.wd_exit = ws.wd_ctr + 1;
  a.gp = B.gp; a.dqg = B.dqg; a.dqg128 = B.dqg128; a.mvg = B.mvg;
  const bool sync_mv = det || opt->sync_moves != 0;
  a.sync_moves = det ? 3 : (opt->sync_moves & 3);
  // launch shapes of the batch class (tuning.hip)
  const gvl_tuning tune = gvl_tuning_of(GVL_CLASS_BATCH);
  ctx->lim = bin_limits(tune);
  const int grid_cap = tune.decide_grid, agg_grid_cap = tune.agg_grid;
  a.commit_grid = tune.commit_grid;
  int64_t dummy_launches = 0;
  TableState tstate;

  GraphDesc cur{N0, B.uoff, nullptr, B.uidx, B.uw, false};
  int32_t* gid = B.gidA;
  int32_t* gidn = B.gidB;
  int buf = 0;
  double tau = opt->tolerance;
  unsigned long long moves_before = 0;
  // per kept graph: running, its vertices in the current union, base
  std::vector<uint8_t> run(K, 1);
  std::vector<int64_t> ncur(K);
  std::vector<int32_t> vcur(K);
  for (int32_t k = 0; k < K; ++k) { ncur[k] = gs[src[k]].n; vcur[k] = goff0[k]; }
  if ((s = upload(st, B.vcur, vcur)) != GVL_OK) return s;
  int32_t alive = K;

  a.seed = opt->seed;
  a.vbase = B.vcur;
  for (int32_t pass = 0; pass < opt->max_passes && alive > 0; ++pass) {
    const int64_t nn = cur.n;
    a.gid = gid;
    a.pass = pass;
    a.rnd = 0;
    // ---- bins, hub plan, K', initial labels
    BinInfo bins;
    s = make_bins(ctx, ws, cur.off, cur.deg, nn, S_union, true, bins, gid, B.vcur, B.gsh);
    if (s != GVL_OK) return s;
    HubPlan plan;
    s = build_hub_plan(ctx, ws, bins, false, cur, nullptr, 0, plan);
    if (s != GVL_OK) return s;
    // K' of the inputs here; of a super-vertex graph, written by the
    // aggregation that built it (its community totals)
    if (pass == 0) graph_weights(ctx, ws, cur, M0, bins, plan, 0);
    fill_i32(st, B.nz, 0, K);
    graph_nonzero(st, cur, gid, B.nz);
    if (pass > 0) {
      copy_i32(st, ws.C, ws.start, nn);
      fill_f64(st, ws.Sig, 0.0, nn);
      fill_i32(st, ws.size, 0, nn);
      community_totals(st, ws.C, ws.K, ws.Sig, ws.size, nn);
    } else {
      iota_i32(st, ws.C, nn);
      copy_f64(st, ws.Sig, ws.K, nn);
      set_size_one(st, ws.size, nn);
    }
    HubArgs hargs = hub_args(ws, bins);
    fill_u8(st, ws.flag, 1, nn);
    fill_i32(st, ws.target, -1, nn);
    fill_i32(st, (int32_t*)ws.last, kNoLastMove, 2 * nn);  // no vertex has moved in this pass
    fill_i32(st, (int32_t*)ws.mv, 0, 4 * nn);     // no move recorded (stamps start at 1)
    fill_i32(st, &ws.sc->iter, 0, 1);

    // (bx, lx: the short-row bins and their list, thinned during refinement;
    // the hubs always come from bins and ws.list)
    auto decide_group = [&](hipStream_t q, int grp, int phase, const BinInfo& bx, const int32_t* lx) {
      // (thinned refinement: no lone hub left in the group)
      const bool hubs = bx.count[grp][kHubBin] > 0 && !plan.groups[grp].empty();
      const int32_t h0 = hubs ? plan.groups[grp].front().h0 : 0, h1 = hubs ? plan.groups[grp].back().h1 : 0;
      if (phase == kMove)
        launch_decide_move(q, cur, a, lx, bx.count[grp], bx.start[grp], det, grid_cap, hargs, h0, h1, &dummy_launches);
      else
        launch_decide_refine(q, cur, a, lx, bx.count[grp], bx.start[grp], det, grid_cap, hargs, h0, h1, &dummy_launches);
      if (hubs)
        for (const HubBatch& hb : plan.groups[grp]) {
          tstate.ensure(q, ws, hb.tend - hb.tbase);
          hargs.tbase = hb.tbase;
          hub_decide(q, cur, a, hargs, hb.h0, hb.h1, hb.c0, hb.c1, hb.s0, hb.s1, hb.tend > hb.tbase, phase, det,
                     &dummy_launches);
        }
    };
    auto commit_group = [&](hipStream_t q, int grp, int phase, const BinInfo& bx, const int32_t* lx) {
      CommitLaunch cl;
      memset(&cl, 0, sizeof(cl));
      const int32_t n0 = bx.gend[grp] - bx.gstart[grp];  // bins 0 .. kHubBin-1 of the group
      const int32_t n0s = bx.start[grp][5] - bx.gstart[grp];  // rows of at most kBinMax[4] arcs
      cl.l0 = lx + bx.gstart[grp];
      cl.l2 = ws.list + bins.start[grp][kHubBin];
      cl.n2 = bx.count[grp][kHubBin] > 0 ? bins.count[grp][kHubBin] : 0;
      if (phase == kMove) {
        cl.n0 = n0s;
        cl.l1 = cl.l0 + n0s;
        cl.n1 = n0 - n0s;
        if (!plan.groups[grp].empty()) {
          cl.c0 = plan.groups[grp].front().c0;
          cl.c1 = plan.groups[grp].back().c1;
        }
      } else {
        cl.n0 = n0;
      }
      launch_commit(q, cur, a, hargs, cl, phase);
    };

    // every local-moving iteration, and every refinement sweep after the
    // first, repeats one launch sequence with the same arguments: replayed as
    // one HIP graph
    const bool replay = !opt->no_graph_replay;

    // ---- local-moving (Alg. 2), each graph stopping on its own gain sum
    std::vector<uint8_t> iter(run), first_conv(K, 0);
    a.groups = bins.S;
    Replay move_graph;
    for (int32_t it = 0; it < opt->max_iterations; ++it) {
      const int64_t clean = tstate.clean;
      s = move_graph.run(ctx, replay, &dummy_launches, [&](hipStream_t q) {
        if (det) fill_u64(q, B.dqg128, 0ull, 2 * (int64_t)K);
        else fill_f64(q, B.dqg, 0.0, K);
        for (int32_t grp = 0; grp < bins.S; ++grp) {
          a.grp = grp;
          decide_group(q, grp, kMove, bins, ws.list);
          if (sync_mv) {
            commit_group(q, grp, kMove, bins, ws.list);
          }
        }
        add_one_i32(q, &ws.sc->iter);
      }, [&] { tstate.clean = clean; });
      if (s != GVL_OK) return s;
      bool any = false, stopped = false;
      if (det) {
        std::vector<unsigned long long> h;
        if ((s = download(st, h, B.dqg128, 2 * (size_t)K)) != GVL_OK) return s;
        for (int32_t k = 0; k < K; ++k) {
          if (!iter[k]) continue;
          const double W = Wk[k];
          const double dq = i128_to_double(h[2 * k], h[2 * k + 1]) * 2.0 / (65536.0 * W * W);
          if (dq <= tau) { iter[k] = 0; stopped = true; if (it == 0) first_conv[k] = 1; }
          else any = true;
        }
      } else {
        std::vector<double> h;
        if ((s = download(st, h, B.dqg, K)) != GVL_OK) return s;
        for (int32_t k = 0; k < K; ++k) {
          if (!iter[k]) continue;
          if (h[k] <= tau) { iter[k] = 0; stopped = true; if (it == 0) first_conv[k] = 1; }
          else any = true;
        }
      }
      if (!any) break;
      if (stopped && it + 1 < opt->max_iterations) {
        if ((s = upload(st, B.active, iter)) != GVL_OK) return s;
        mask_flags(st, ws.flag, gid, B.active, nn);
      }
    }

    // ---- refinement (Alg. 3); the Louvain method keeps the local-moving
    // communities as they are (C' = C'_B)
    copy_i32(st, ws.CB, ws.C, nn);
    if (!opt->louvain) {
      iota_i32(st, ws.C, nn);
      copy_f64(st, ws.Sig, ws.K, nn);
      set_size_one(st, ws.size, nn);
      fill_i32(st, ws.targeted, 0, nn);
      pack_labels(st, ws.C, ws.CB, ws.CP, nn);
      fill_i32(st, &ws.sc->sweep, 0, 1);
    }
    fill_u64(st, B.mvg, 0ull, K);
    s = readback(ctx, ws.sc);
    if (s != GVL_OK) return s;
    if (det && ctx->host->ovf) return GVL_E_TABLE_OVERFLOW;
    moves_before = counter(ctx->host, 3);
    BinInfo rbins;  // after the first sweep: the short-row bins thinned to lone vertices
    const BinInfo* rb = &bins;
    const int32_t* rl = ws.list;
    // one sweep: group stamps grp + 1 + sweep * S (unique within the pass),
    // the sweep number read from the device and advanced by the sweep itself
    a.rnd = opt->refine_random;
    a.sweep_dev = &ws.sc->sweep;
    auto refine_sweep = [&](hipStream_t q) {
      for (int32_t grp = 0; grp < bins.S; ++grp) {
        a.stamp = grp + 1;
        decide_group(q, grp, kRefine, *rb, rl);
        commit_group(q, grp, kRefine, *rb, rl);
      }
      add_one_i32(q, &ws.sc->sweep);
    };
    Replay refine_graph;  // sweeps from the second on (the thinned bins stay fixed)
    for (int32_t sw = 0; sw < (opt->louvain ? 0 : opt->refine_sweeps); ++sw) {
      if (sw == 0) {
        refine_sweep(st);
      } else {
        const int64_t clean = tstate.clean;
        s = refine_graph.run(ctx, replay, &dummy_launches, refine_sweep, [&] { tstate.clean = clean; });
        if (s != GVL_OK) return s;
      }
      s = readback(ctx, ws.sc);
      if (s != GVL_OK) return s;
      if (det && ctx->host->ovf) return GVL_E_TABLE_OVERFLOW;
      const unsigned long long mv = counter(ctx->host, 3) - moves_before;
      moves_before = counter(ctx->host, 3);
      if (mv == 0) break;
      if (sw == 0 && sw + 1 < opt->refine_sweeps) {
        s = thin_refine_bins(ctx, ws, bins, rbins);
        if (s != GVL_OK) return s;
        rb = &rbins;
        rl = ws.list2;
      }
    }
    a.rnd = 0;
    a.sweep_dev = nullptr;
    std::vector<unsigned long long> hmv;
    if ((s = download(st, hmv, B.mvg, K)) != GVL_OK) return s;
    std::vector<int32_t> hnz;
    if ((s = download(st, hnz, B.nz, K)) != GVL_OK) return s;

    // ---- communities per graph; who stops
    fill_i32(st, ws.newid, 0, nn + 1);
    mark_used(st, ws.C, nn, ws.newid);
    exclusive_scan(st, ws.newid, nn, ws.scan_tmp);
    std::vector<int32_t> alive_k, hpos;
    for (int32_t k = 0; k < K; ++k)
      if (run[k]) { alive_k.push_back(k); hpos.push_back(vcur[k]); }
    hpos.push_back((int32_t)nn);
    const int32_t A = (int32_t)alive_k.size();
    if ((s = upload(st, B.pos, hpos)) != GVL_OK) return s;
    gather_at(st, ws.newid, B.pos, A + 1, B.gath);
    std::vector<int32_t> hg;
    if ((s = download(st, hg, B.gath, A + 1)) != GVL_OK) return s;
    std::vector<uint8_t> state(K, kBatchDone), keep(K, 0);
    int32_t cont = 0;
    for (int32_t j = 0; j < A; ++j) {
      const int32_t k = alive_k[j];
      const int64_t n_k = ncur[k];
      const int64_t ncom = hg[j + 1] - hg[j];
      const int64_t z = opt->shrink_excludes_isolated ? n_k - hnz[k] : 0;
      bool stop = false;
      if (first_conv[k] && hmv[k] == 0) stop = true;
      else if (n_k == z || (double)(ncom - z) / (double)(n_k - z) > opt->aggregation_tolerance) stop = true;
      if (!stop && pass + 1 >= opt->max_passes) stop = true;
      if (stop) {
        state[k] = kBatchEnd;
      } else {
        state[k] = kBatchCont;
        keep[k] = 1;
        ++cont;
      }
    }
    // renumbering over the continuing graphs only
    if (cont < A) {
      if ((s = upload(st, B.keep, keep)) != GVL_OK) return s;
      fill_i32(st, ws.newid, 0, nn + 1);
      mark_used(st, ws.C, nn, ws.newid, gid, B.keep);
      exclusive_scan(st, ws.newid, nn, ws.scan_tmp);
    }
    if ((s = upload(st, B.state, state)) != GVL_OK) return s;
    lookup_batch(st, B.top, N0, ws.C, ws.newid, B.gid0, B.state, B.vcur, B.goff0, pass == 0);
    for (int32_t j = 0; j < A; ++j) {
      const int32_t k = alive_k[j];
      if (state[k] == kBatchEnd) { run[k] = 0; --alive; }
    }
    if (cont == 0) break;

    // ---- aggregation (Alg. 4) of the continuing graphs
    if ((s = upload(st, B.keep, keep)) != GVL_OK) return s;
    std::vector<int32_t> hnc;
    if ((s = download(st, hnc, ws.newid + nn, 1)) != GVL_OK) return s;
    const int64_t ncom_all = hnc[0];
    const int nb = buf;
    buf ^= 1;
    int32_t* yoff = ws.off[nb];
    int32_t* ydeg = ws.deg[nb];
    fill_i32(st, ws.cnt, 0, ncom_all + 1);
    fill_i32(st, yoff, 0, ncom_all + 1);
    agg_count(st, cur, ws.C, ws.newid, ws.lab, ws.rank, ws.cnt, yoff, gid, B.keep);
    // K' of the next pass: each super-vertex row sums its members' rows
    next_weights(st, ws.Sig, ws.newid, nn, ws.K);
    exclusive_scan(st, ws.cnt, ncom_all, ws.scan_tmp);
    exclusive_scan(st, yoff, ncom_all, ws.scan_tmp);
    agg_fill(st, ws.lab, ws.rank, ws.cnt, nn, ws.cv);
    fill_i32(st, ydeg, 0, ncom_all);
    BinInfo cb;
    s = make_bins(ctx, ws, yoff, nullptr, ncom_all, 1, false, cb);
    if (s != GVL_OK) return s;
    HubPlan gp;
    s = build_hub_plan(ctx, ws, cb, true, cur, yoff, ncom_all, gp);
    if (s != GVL_OK) return s;
    AggArgs g;
    memset(&g, 0, sizeof(g));
    g.lab = ws.lab; g.coff = ws.cnt; g.cv = ws.cv; g.yoff = yoff; g.ydeg = ydeg;
    g.yidx = ws.idx[nb]; g.yw = ws.w[nb]; g.yw_double = det; g.cnt = &ws.sc->cnt[0][0];
    g.ncom = ncom_all;
    launch_agg_rows(st, cur, g, ws.list, cb.count[0], cb.start[0], agg_grid_cap, 0, &dummy_launches);
    if (gp.H > 0) {
      // members: the vertices of the continuing graphs
      int64_t nkept = 0;
      for (int32_t k = 0; k < K; ++k)
        if (keep[k]) nkept += ncur[k];
      member_degrees(st, cur, ws.cv, nkept, ws.apre);
      exclusive_scan(st, ws.apre, nkept, ws.scan_tmp);
      HubArgs gh = hub_args(ws, cb);
      for (const HubBatch& hb : gp.groups[0]) {
        tstate.ensure(st, ws, hb.tend - hb.tbase);
        gh.tbase = hb.tbase;
        gagg_rows(st, cur, g, gh, hb.c0, hb.c1, hb.s0, hb.s1, &dummy_launches);
      }
    }
    // labels of the super-vertices (move-based, Alg. 1; or refine-based,
    // Sec. 4.1: every super-vertex alone, its union id being its solo id
    // shifted by its graph's base), their graphs and bases
    if (opt->refine_based) {
      iota_i32(st, ws.start, ncom_all);
    } else {
      fill_i32(st, ws.brank, 0, nn + 1);
      mark_used(st, ws.CB, nn, ws.brank, gid, B.keep);
      exclusive_scan(st, ws.brank, nn, ws.scan_tmp);
      next_labels(st, ws.lab, ws.CB, ws.brank, nn, ws.start);
    }
    gid_next(st, ws.C, ws.newid, gid, B.keep, nn, gidn);
    std::vector<int32_t> cont_k, cpos;
    for (int32_t k = 0; k < K; ++k)
      if (keep[k]) { cont_k.push_back(k); cpos.push_back(vcur[k]); }
    if ((s = upload(st, B.pos, cpos)) != GVL_OK) return s;
    gather_at(st, ws.newid, B.pos, (int32_t)cont_k.size(), B.gath);
    std::vector<int32_t> hv;
    if ((s = download(st, hv, B.gath, cont_k.size())) != GVL_OK) return s;
    for (size_t j = 0; j < cont_k.size(); ++j) {
      const int32_t k = cont_k[j];
      const int64_t nxt = (j + 1 < cont_k.size()) ? hv[j + 1] : ncom_all;
      ncur[k] = nxt - hv[j];
      vcur[k] = hv[j];
    }
    if ((s = upload(st, B.vcur, vcur)) != GVL_OK) return s;
    cur = GraphDesc{ncom_all, yoff, ydeg, ws.idx[nb], ws.w[nb], det};
    std::swap(gid, gidn);
    tau = tau / opt->tolerance_drop;
  }

  // ---- canonical labels per graph, outputs, Eq. 1 per graph
  const int64_t N = N0;
  fill_i32(st, ws.rank, std::numeric_limits<int32_t>::max(), N);
  first_occurrence(st, B.top, N, ws.rank);
  first_flags(st, B.top, ws.rank, N, ws.newid);
  exclusive_scan(st, ws.newid, N, ws.scan_tmp);
  apply_canonical(st, B.top, ws.rank, ws.newid, N);
  batch_outputs(st, B.top, N, B.gid0, B.goff0, B.out);
  gather_at(st, B.top, B.goff0, K, B.cb);
  copy_i32(st, B.cb + K, ws.newid + N, 1);
  std::vector<int32_t> htot;
  if ((s = download(st, htot, ws.newid + N, 1)) != GVL_OK) return s;
  const GraphDesc input{N0, B.uoff, nullptr, B.uidx, B.uw, false};
  BinInfo mb;
  s = make_bins(ctx, ws, input.off, input.deg, N0, 1, true, mb);
  if (s != GVL_OK) return s;
  HubPlan mp;
  s = build_hub_plan(ctx, ws, mb, false, input, nullptr, 0, mp);
  if (s != GVL_OK) return s;
  fill_f64(st, ws.Sig, 0.0, N0);
  fill_f64(st, B.s1g, 0.0, K);
  fill_f64(st, B.s2d, 0.0, K);
  fill_u64(st, B.s2u, 0ull, 2 * (int64_t)K);
  modularity_partial(st, input, B.top, ws.Sig, ws.sc->acc_d, B.gid0, B.s1g);
  if (mp.H > 0) hub_modularity(st, input, hub_args(ws, mb), 0, mp.T, B.top, ws.Sig, ws.sc->acc_d, B.gid0, B.s1g);
  mod_squares_batch(st, ws.Sig, htot[0], B.cb, K, B.s2d, B.s2u);
  std::vector<double> hs1, hs2;
  std::vector<unsigned long long> hs2u;
  if ((s = download(st, hs1, B.s1g, K)) != GVL_OK) return s;
  if ((s = download(st, hs2, B.s2d, K)) != GVL_OK) return s;
  if ((s = download(st, hs2u, B.s2u, 2 * (size_t)K)) != GVL_OK) return s;
  for (int32_t k = 0; k < K; ++k) {
    const double W = Wk[k];
    const double S2 = integral[k] ? i128_to_double(hs2u[2 * k], hs2u[2 * k + 1]) : hs2[k];
    qs[src[k]] = hs1[k] / W - gam[k] * (S2 / (W * W));
  }
  return GVL_OK;
}

}  // namespace
}  // namespace gvl

using namespace gvl;

extern "C" {

gvl_status gvl_fused_workspace_bytes(int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                                     size_t* bytes) {
  if (!bytes || !opt || num_graphs < 0 || (num_graphs > 0 && !graphs)) return GVL_E_INVALID_ARG;
  size_t mx = 256;
  for (const Chunk& c : plan_chunks(num_graphs, graphs)) mx = std::max(mx, chunk_bytes(c, opt->mode == GVL_MODE_DET));
  *bytes = mx;
  return GVL_OK;
}

gvl_status gvl_leiden_fused(gvl_ctx_t ctx, int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                            void* d_workspace, size_t workspace_bytes, double* modularities, gvl_status* statuses) {
  if (!ctx || !opt || num_graphs < 0 || (num_graphs > 0 && (!graphs || !modularities || !statuses)))
    return GVL_E_INVALID_ARG;
  if (opt->mode != GVL_MODE_FAST && opt->mode != GVL_MODE_DET) return GVL_E_INVALID_ARG;
  if (opt->max_iterations < 1 || opt->max_iterations > kMaxIterationsSync || opt->max_passes < 1 ||
      opt->refine_sweeps < 1 || opt->subsweeps < 0 ||
      (opt->subsweeps == 0 && opt->mode == GVL_MODE_DET) || opt->subsweeps > kMaxGroups ||
      !(opt->tolerance_drop > 0.0))
    return GVL_E_INVALID_ARG;
  size_t need = 0;
  gvl_status s = gvl_fused_workspace_bytes(num_graphs, graphs, opt, &need);
  if (s != GVL_OK) return s;
  if (num_graphs == 0) return GVL_OK;
  if (!d_workspace || workspace_bytes < need) return GVL_E_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GVL_E_HIP;
  bool failed = false;
  for (const Chunk& c : plan_chunks(num_graphs, graphs)) {
    s = fused_chunk(ctx, c.g1 - c.g0, graphs + c.g0, opt, (char*)d_workspace, c, modularities + c.g0,
                    statuses + c.g0);
    if (s != GVL_OK) return s;
    for (int32_t g = c.g0; g < c.g1; ++g) failed |= statuses[g] != GVL_OK;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return GVL_E_HIP;
  return failed ? GVL_E_BATCH : GVL_OK;
}

}  // extern "C"
