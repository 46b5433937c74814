// Host driver of the Leiden pass loop (Alg. 1) and the C ABI of libgvl.so.
//
// Per pass on the current graph G' (the input at pass 0, then a holey
// super-vertex graph):
//   1. vertex weights K', initial labels C' and community totals Sigma'
//   2. degree binning of the vertices
//   3. local-moving iterations (Alg. 2) until the summed gain <= tau
//   4. refinement sweeps inside the local-moving bounds (Alg. 3)
//   5. |Gamma| = distinct refined labels; stop on convergence / low shrink
//   6. renumbering, dendrogram lookup, aggregation (Alg. 4) into the other
//      graph buffer, move-based labels of the super-vertices, tau /= drop
// then the canonical relabelling of the result and Eq. 1.
#include "host.hpp"


extern "C" {

const char* gvl_status_string(gvl_status s) {
  switch (s) {
    case GVL_E_BUSY: return "request busy";
    case GVL_E_BATCH: return "some graphs of the batch failed";
    case GVL_E_TABLE_OVERFLOW: return "a key partition of a wide row or hub overflowed its table";
    case GVL_OK: return "ok";
    case GVL_E_INVALID_ARG: return "invalid argument";
    case GVL_E_BAD_CSR: return "malformed CSR input";
    case GVL_E_NOT_SYMMETRIC: return "graph not symmetric (an arc has no reverse arc of the same weight)";
    case GVL_E_NONINTEGER_WEIGHT: return "weights not valid for this mode";
    case GVL_E_RESOLUTION: return "invalid resolution";
    case GVL_E_WORKSPACE: return "workspace missing or too small";
    case GVL_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

gvl_status gvl_default_options(gvl_options* o, int32_t mode) {
  if (!o || (mode != GVL_MODE_FAST && mode != GVL_MODE_DET)) return GVL_E_INVALID_ARG;
  memset(o, 0, sizeof(*o));
  o->mode = mode;
  o->tolerance = 0.01;
  o->tolerance_drop = 10.0;
  o->aggregation_tolerance = 0.8;
  o->max_iterations = 20;
  o->max_passes = 20;
  o->refine_sweeps = 20;
  // deterministic mode: 32 groups, as the oracle's default; fast mode: 8 or
  // 32 by the longest row of the input (kAutoShortRow)
  o->subsweeps = mode == GVL_MODE_DET ? kAutoGroups : 0;
  o->validate = 1;
  // group-synchronous local-moving (faster and higher modularity than
  // committing every move at once on the R-MAT benchmark graph)
  o->sync_moves = 3;
  return GVL_OK;
}

gvl_status gvl_workspace_bytes(int64_t n, int64_t m, const gvl_options* opt, size_t* bytes) {
  if (!bytes || n < 0 || m < 0) return GVL_E_INVALID_ARG;
  const bool det = opt && opt->mode == GVL_MODE_DET;
  *bytes = carve(n, m, det, nullptr).bytes;
  return GVL_OK;
}

gvl_status gvl_create(gvl_ctx_t* out, int device, void* hip_stream) {
  if (!out) return GVL_E_INVALID_ARG;
  *out = nullptr;
  gvl_ctx* c = new gvl_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&c->host, sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->hbins, sizeof(BinBuf), hipHostMallocDefault) != hipSuccess) {
    if (c->host) (void)hipHostFree(c->host);
    delete c;
    return GVL_E_HIP;
  }
  memset(c->host, 0, sizeof(Scalars));
  memset(c->hbins, 0, sizeof(BinBuf));
  // device address of gvl_leiden_static's array on this device (once per device)
  const gvl_status s = gvl_static_scratch_setup(device);
  if (s != GVL_OK) {
    (void)hipHostFree(c->host);
    (void)hipHostFree(c->hbins);
    delete c;
    return s;
  }
  gvl_tuning_load_once();  // launch shapes per class of graph, from the tune file if there is one
  // private stream for recording launch sequences into graphs (default
  // priority; nothing runs on it); without it every launch goes eagerly
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->cap = nullptr;
    (void)hipGetLastError();
  }
  *out = c;
  return GVL_OK;
}

gvl_status gvl_destroy(gvl_ctx_t c) {
  if (!c) return GVL_E_INVALID_ARG;
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->host) (void)hipHostFree(c->host);
  if (c->hbins) (void)hipHostFree(c->hbins);
  delete c;
  return GVL_OK;
}

gvl_status gvl_modularity(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_off, const int32_t* d_idx,
                          const float* d_w, const int32_t* d_membership, double resolution, void* d_ws,
                          size_t ws_bytes, double* modularity) {
  gvl_options opt;
  gvl_default_options(&opt, GVL_MODE_FAST);
  gvl_status s = check_args(ctx, n, m, d_off, d_idx, resolution, &opt, d_ws, ws_bytes);
  if (s != GVL_OK) return s;
  if (!modularity || (n > 0 && !d_membership)) return GVL_E_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GVL_E_HIP;
  Workspace ws = carve(n, m, false, (char*)d_ws);
  hipStream_t st = ctx->stream;
  *modularity = 0.0;
  if (n == 0) return GVL_OK;
  GraphDesc in{n, d_off, nullptr, d_idx, d_w, false};
  fill_u64(st, (unsigned long long*)ws.sc, 0ull, sizeof(Scalars) / 8);
  check_offsets(st, d_off, n, m, ws.sc->flags);
  s = readback(ctx, ws.sc);
  if (s != GVL_OK) return s;
  if (ctx->host->flags[0]) return GVL_E_BAD_CSR;
  BinInfo bins;
  s = make_bins(ctx, ws, d_off, nullptr, n, 1, true, bins);
  if (s != GVL_OK) return s;
  HubPlan plan;
  s = build_hub_plan(ctx, ws, bins, false, in, nullptr, 0, plan);
  if (s != GVL_OK) return s;
  graph_weights(ctx, ws, in, m, bins, plan, 1);
  s = readback(ctx, ws.sc);
  if (s != GVL_OK) return s;
  if (ctx->host->flags[0]) return GVL_E_BAD_CSR;
  if (ctx->host->flags[2]) return GVL_E_NONINTEGER_WEIGHT;
  const double W = ctx->host->accW;
  const bool integral = ctx->host->flags[1] == 0;
  return modularity_device(ctx, ws, in, d_membership, W, integral, resolution, modularity);
}

gvl_status gvl_disconnected_communities(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_off,
                                        const int32_t* d_idx, const int32_t* d_membership, void* d_ws,
                                        size_t ws_bytes, int32_t* d_flags, int64_t* count) {
  gvl_options opt;
  gvl_default_options(&opt, GVL_MODE_FAST);
  gvl_status s = check_args(ctx, n, m, d_off, d_idx, 1.0, &opt, d_ws, ws_bytes);
  if (s != GVL_OK) return s;
  if (!count || (n > 0 && !d_membership)) return GVL_E_INVALID_ARG;
  *count = 0;
  if (n == 0) return GVL_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return GVL_E_HIP;
  Workspace ws = carve(n, m, false, (char*)d_ws);
  hipStream_t st = ctx->stream;
  fill_u64(st, (unsigned long long*)ws.sc, 0ull, sizeof(Scalars) / 8);
  check_offsets(st, d_off, n, m, ws.sc->flags);
  s = readback(ctx, ws.sc);
  if (s != GVL_OK) return s;
  if (ctx->host->flags[0]) return GVL_E_BAD_CSR;
  disconnected_communities(st, d_off, d_idx, d_membership, n, ws.C, ws.start, ws.CB,
                           d_flags ? d_flags : ws.target, &ws.sc->acc_u[0]);
  s = readback(ctx, ws.sc);
  if (s != GVL_OK) return s;
  *count = (int64_t)ctx->host->acc_u[0];
  return GVL_OK;
}

gvl_status gvl_leiden(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_off, const int32_t* d_idx,
                      const float* d_w, double resolution, const gvl_options* opt, void* d_ws,
                      size_t ws_bytes, int32_t* d_membership, double* modularity, gvl_stats* stats) {
  gvl_status s = check_args(ctx, n, m, d_off, d_idx, resolution, opt, d_ws, ws_bytes);
  if (s != GVL_OK) return s;
  if (!modularity || (n > 0 && !d_membership)) return GVL_E_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GVL_E_HIP;
  const bool det = opt->mode == GVL_MODE_DET;
  gvl_stats st_local;
  gvl_stats* S = stats ? stats : &st_local;
  memset(S, 0, sizeof(*S));
  ctx->trace.clear();
  ctx->ev_used = 0;
  *modularity = 0.0;
  if (n == 0) { S->termination = 3; return GVL_OK; }

  hipStream_t st = ctx->stream;
  Workspace ws = carve(n, m, det, (char*)d_ws);
  Timer tm{ctx, opt->profile != 0, {}};
  const GraphDesc input{n, d_off, nullptr, d_idx, d_w, false};
  int32_t* top = d_membership;
  TableState tstate;

  // ---- input checks
  int h = tm.begin(kEvOther);
  fill_u64(st, (unsigned long long*)ws.sc, 0ull, sizeof(Scalars) / 8);
  fill_i32(st, ws.hp_done, 0, n);
  fill_i32(st, ws.hp_lcnt, 0, n);
  fill_i32(st, ws.wd_done, 0, ws.max_wide);
  fill_i32(st, ws.wd_ctr, 0, 2);
  if (opt->validate) {
    check_offsets(st, d_off, n, m, ws.sc->flags);
    s = readback(ctx, ws.sc);
    if (s != GVL_OK) return s;
    if (ctx->host->flags[0]) return GVL_E_BAD_CSR;
  }

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
  a.wd_g = ws.wd_g; a.wd_k = ws.wd_k; a.wd_c = ws.wd_c; a.wd_ok = ws.wd_ok; a.wd_done = ws.wd_done;
  a.wd_next = ws.wd_ctr; a.wd_exit = ws.wd_ctr + 1;
  const bool sync_mv = det || opt->sync_moves != 0;
  a.sync_moves = det ? 3 : (opt->sync_moves & 3);

  // launch shapes of the graph's class (tuning.hip): bin limits, workgroups
  // per decision, commit and aggregation launch
  const gvl_tuning tune = gvl_tuning_of(gvl_class_of(n, m, false));
  ctx->lim = bin_limits(tune);
  const int grid_cap = tune.decide_grid, agg_grid_cap = tune.agg_grid;
  a.commit_grid = tune.commit_grid;
  GraphDesc cur = input;
  int buf = 0;
  double tau = opt->tolerance;
  bool ended = false;
  int32_t pass = 0;
  S->termination = 2;
  int64_t ncom = n;
  unsigned long long moves_before = 0, out_before = 0;
  double Wd = 0.0;
  bool integral = true;
  long long Wi = 0, p = 0;
  tm.end(h);

  a.seed = opt->seed;
  int S_run = opt->subsweeps > 0 ? opt->subsweeps : kAutoGroups;  // sub-sweep groups of every pass
  for (pass = 0; pass < opt->max_passes; ++pass) {
    a.pass = pass;
    a.rnd = 0;
    const int64_t nn = cur.n;
    PassDebug pd;
    pd.n = nn;
    // ---- 1. degree bins, hub plan, vertex weights K', initial labels
    h = tm.begin(kEvOther);
    BinInfo bins;
    s = make_bins(ctx, ws, cur.off, cur.deg, nn, S_run, true, bins);
    if (s != GVL_OK) return s;
    if (pass == 0 && opt->subsweeps == 0) {  // automatic S: by the longest row of the input
      int32_t longest = 0;
      for (int b = 0; b < kNumBins; ++b) longest = std::max(longest, bins.maxsize[b]);
      if (longest <= kAutoShortRow) {
        S_run = kAutoFewGroups;
        s = make_bins(ctx, ws, cur.off, cur.deg, nn, S_run, true, bins);
        if (s != GVL_OK) return s;
      }
    }
    HubPlan plan;
    s = build_hub_plan(ctx, ws, bins, false, cur, nullptr, 0, plan);
    if (s != GVL_OK) return s;
    // K' of the input here; of a super-vertex graph, written by the
    // aggregation that built it (its community totals)
    fill_f64(st, &ws.sc->accW, 0.0, 1);
    if (pass == 0) graph_weights(ctx, ws, cur, m, bins, plan, opt->validate);
    s = readback(ctx, ws.sc);
    if (s != GVL_OK) return s;
    if (pass == 0) {
      if (ctx->host->flags[0]) return GVL_E_BAD_CSR;
      if (ctx->host->flags[2]) return GVL_E_NONINTEGER_WEIGHT;
      if (opt->validate >= 2) {  // offsets and neighbour ids are known to be in range here
        fill_u64(st, ws.sc->acc_u, 0ull, 2);
        symmetry_check(st, d_off, d_idx, d_w, n, ws.sc->acc_u);
        s = readback(ctx, ws.sc);
        if (s != GVL_OK) return s;
        if (ctx->host->acc_u[0] != 0 || ctx->host->acc_u[1] != 0) return GVL_E_NOT_SYMMETRIC;
      }
      Wd = ctx->host->accW;
      integral = ctx->host->flags[1] == 0;
      if (det) {
        if (!integral || Wd > 1099511627776.0) return GVL_E_NONINTEGER_WEIGHT;
        const double pd_ = resolution * 65536.0;
        if (pd_ != std::floor(pd_) || pd_ > 16777216.0) return GVL_E_RESOLUTION;
        Wi = (long long)Wd;
        p = (long long)pd_;
      }
      if (Wd == 0.0) {
        iota_i32(st, d_membership, n);
        HIP_TRY(hipStreamSynchronize(st));
        S->termination = 3;
        S->num_communities = n;
        return GVL_OK;
      }
      a.inv_m = 2.0 / Wd;
      a.gk_scale = 2.0 * resolution / (Wd * Wd);
      a.W = Wi;
      a.p = p;
    }
    if (pass < GVL_MAX_PASS_STATS) {
      S->nv[pass] = nn;
      S->ne[pass] = (pass == 0) ? m : (int64_t)(counter(ctx->host, 6) - out_before);
    }
    out_before = counter(ctx->host, 6);
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
    tm.end(h);

    // Decisions of one group: short rows by the binned kernels, hubs by the
    // chunked path (batch by batch through the table region).
    // (bx, lx: the short-row bins and their list, thinned during refinement;
    // the hubs always come from bins and ws.list)
    auto decide_group = [&](hipStream_t q, int grp, int phase, const BinInfo& bx, const int32_t* lx) {
      // (thinned refinement: no lone hub left in the group)
      const bool hubs = bx.count[grp][kHubBin] > 0 && !plan.groups[grp].empty();
      const int32_t h0 = hubs ? plan.groups[grp].front().h0 : 0, h1 = hubs ? plan.groups[grp].back().h1 : 0;
      if (phase == kMove)
        launch_decide_move(q, cur, a, lx, bx.count[grp], bx.start[grp], det, grid_cap, hargs, h0, h1, &S->scan_launches);
      else
        launch_decide_refine(q, cur, a, lx, bx.count[grp], bx.start[grp], det, grid_cap, hargs, h0, h1, &S->scan_launches);
      if (hubs)
        for (const HubBatch& hb : plan.groups[grp]) {
          tstate.ensure(q, ws, hb.tend - hb.tbase);
          hargs.tbase = hb.tbase;
          hub_decide(q, cur, a, hargs, hb.h0, hb.h1, hb.c0, hb.c1, hb.s0, hb.s1, hb.tend > hb.tbase, phase, det,
                     &S->scan_launches);
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
    // Iterations and sweeps after the first of a phase repeat one launch
    // sequence with the same arguments: they are replayed as one HIP graph
    // (not while kernel classes are timed: see Replay).
    const bool replay = !tm.on && !opt->no_graph_replay;

    // ---- 2. local-moving (Alg. 2)
    h = tm.begin(kEvMove);
    int32_t iters = 0;
    bool first_conv = false;
    a.groups = bins.S;
    // one iteration: every group decides on the state its predecessors left
    // (and commits, synchronous schedules); the first iteration of a pass
    // knows which vertices are still unmarked or (pass 0) unmoved
    auto move_iteration = [&](hipStream_t q, int32_t it) {
      fill_u64(q, (unsigned long long*)ws.sc->dq, 0ull, 3 * kCntSlots);
      int hk = sync_mv ? -1 : tm.begin(kEvScanMoveK);
      for (int32_t grp = 0; grp < bins.S; ++grp) {
        if (sync_mv) hk = tm.begin(kEvScanMoveK);
        a.ident_after = (pass == 0 && it == 0) ? grp : -1;
        a.grp = grp;
        decide_group(q, grp, kMove, bins, ws.list);
        a.ident_after = -1;
        if (sync_mv) {
          tm.end(hk);
          a.mark_after = (it == 0) ? grp : INT32_MAX;
          commit_group(q, grp, kMove, bins, ws.list);
          a.mark_after = INT32_MAX;
        }
      }
      if (!sync_mv) tm.end(hk);
      add_one_i32(q, &ws.sc->iter);
    };
    Replay move_graph;
    for (int32_t it = 0; it < opt->max_iterations; ++it) {
      if (it == 0) {
        move_iteration(st, 0);
      } else {
        const int64_t clean = tstate.clean;
        s = move_graph.run(ctx, replay, &S->scan_launches, [&](hipStream_t q) { move_iteration(q, it); },
                           [&] { tstate.clean = clean; });
        if (s != GVL_OK) return s;
      }
      s = readback(ctx, ws.sc);
      if (s != GVL_OK) return s;
      if (det && ctx->host->ovf) return GVL_E_TABLE_OVERFLOW;
      if (move_graph.launched) ++S->graph_launches;
      ++iters;
      const unsigned long long mv = counter(ctx->host, 3) - moves_before;
      moves_before = counter(ctx->host, 3);
      pd.movers.push_back((int64_t)mv);
      double dq;
      if (det) {
        unsigned __int128 sum = 0;
        for (int k = 0; k < kCntSlots; ++k)
          sum += ((unsigned __int128)ctx->host->dq128[k][1] << 64) | ctx->host->dq128[k][0];
        dq = i128_to_double((unsigned long long)sum, (unsigned long long)(sum >> 64)) * 2.0 /
             (65536.0 * (double)Wi * (double)Wi);
      } else {
        dq = 0.0;
        for (int k = 0; k < kCntSlots; ++k) dq += ctx->host->dq[k];
      }
      if (dq <= tau) {
        if (it == 0) first_conv = true;
        break;
      }
    }
    tm.end(h);
    // ---- 3. refinement (Alg. 3); the Louvain method keeps the local-moving
    // communities as they are (C' = C'_B)
    h = tm.begin(kEvRefine);
    copy_i32(st, ws.CB, ws.C, nn);
    int32_t sweeps = 0;
    int64_t refine_moved = 0;
    if (!opt->louvain) {
      iota_i32(st, ws.C, nn);
      copy_f64(st, ws.Sig, ws.K, nn);
      set_size_one(st, ws.size, nn);
      fill_i32(st, ws.targeted, 0, nn);
      pack_labels(st, ws.C, ws.CB, ws.CP, nn);
      fill_i32(st, &ws.sc->sweep, 0, 1);
    }
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
        const int hk = tm.begin(kEvScanRefineK);
        decide_group(q, grp, kRefine, *rb, rl);
        tm.end(hk);
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
        s = refine_graph.run(ctx, replay, &S->scan_launches, refine_sweep, [&] { tstate.clean = clean; });
        if (s != GVL_OK) return s;
      }
      s = readback(ctx, ws.sc);
      if (s != GVL_OK) return s;
      if (det && ctx->host->ovf) return GVL_E_TABLE_OVERFLOW;
      if (refine_graph.launched) ++S->graph_launches;
      ++sweeps;
      const unsigned long long mv = counter(ctx->host, 3) - moves_before;
      moves_before = counter(ctx->host, 3);
      pd.refine_movers.push_back((int64_t)mv);
      refine_moved += (int64_t)mv;
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
    tm.end(h);
    // ---- 4. count communities; stop on convergence or low shrink
    h = tm.begin(kEvOther);
    fill_i32(st, ws.newid, 0, nn + 1);
    mark_used(st, ws.C, nn, ws.newid);
    exclusive_scan(st, ws.newid, nn, ws.scan_tmp);
    HIP_TRY(hipMemcpyAsync(&ctx->host->total, ws.newid + nn, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ncom = ctx->host->total;
    if (pass < GVL_MAX_PASS_STATS) {
      S->iterations[pass] = iters;
      S->refine_sweeps[pass] = sweeps;
      S->ncom[pass] = ncom;
    }
    pd.ncom = ncom;
    if (opt->debug_trace) {
      pd.bound = to_host(ctx, ws.CB, nn);
      pd.refined = to_host(ctx, ws.C, nn);
    }
    // Alg. 1 low shrink, |Gamma| / |V'|; the variant leaves the vertices
    // without arcs (singletons for ever) out of both counts
    const int64_t z = opt->shrink_excludes_isolated ? nn - bins.binned : 0;
    bool stop = false;
    if (first_conv && refine_moved == 0) { S->termination = 0; stop = true; }
    else if (nn == z || (double)(ncom - z) / (double)(nn - z) > opt->aggregation_tolerance) {
      S->termination = 1;
      stop = true;
    }
    if (stop) {
      if (opt->debug_trace) ctx->trace.push_back(std::move(pd));
      ended = true;
      tm.end(h);
      break;
    }
    // ---- 5. renumber + dendrogram lookup
    lookup_top(st, top, n, ws.C, ws.newid, pass == 0);
    tm.end(h);
    if (pass + 1 < opt->max_passes) {
      // ---- 6. aggregation (Alg. 4)
      h = tm.begin(kEvAgg);
      const int nb = buf;
      buf ^= 1;
      int32_t* yoff = ws.off[nb];
      int32_t* ydeg = ws.deg[nb];
      fill_i32(st, ws.cnt, 0, ncom + 1);
      fill_i32(st, yoff, 0, ncom + 1);
      agg_count(st, cur, ws.C, ws.newid, ws.lab, ws.rank, ws.cnt, yoff);
      // K' of the next pass: each super-vertex row sums its members' rows
      // (no later step of this pass reads K')
      next_weights(st, ws.Sig, ws.newid, nn, ws.K);
      exclusive_scan(st, ws.cnt, ncom, ws.scan_tmp);
      exclusive_scan(st, yoff, ncom, ws.scan_tmp);
      agg_fill(st, ws.lab, ws.rank, ws.cnt, nn, ws.cv);
      fill_i32(st, ydeg, 0, ncom);
      BinInfo cb;
      s = make_bins(ctx, ws, yoff, nullptr, ncom, 1, false, cb);
      if (s != GVL_OK) return s;
      HubPlan gp;
      s = build_hub_plan(ctx, ws, cb, true, cur, yoff, ncom, gp);
      if (s != GVL_OK) return s;
      AggArgs g;
      memset(&g, 0, sizeof(g));
      g.lab = ws.lab; g.coff = ws.cnt; g.cv = ws.cv; g.yoff = yoff; g.ydeg = ydeg;
      g.yidx = ws.idx[nb]; g.yw = ws.w[nb]; g.yw_double = det; g.cnt = &ws.sc->cnt[0][0];
      g.ncom = ncom;
      const int hk = tm.begin(kEvAggK);
      launch_agg_rows(st, cur, g, ws.list, cb.count[0], cb.start[0], agg_grid_cap, 0, &S->agg_launches);
      if (gp.H > 0) {
        member_degrees(st, cur, ws.cv, nn, ws.apre);
        exclusive_scan(st, ws.apre, nn, ws.scan_tmp);
        HubArgs gh = hub_args(ws, cb);
        for (const HubBatch& hb : gp.groups[0]) {
          tstate.ensure(st, ws, hb.tend - hb.tbase);
          gh.tbase = hb.tbase;
          gagg_rows(st, cur, g, gh, hb.c0, hb.c1, hb.s0, hb.s1, &S->agg_launches);
        }
      }
      tm.end(hk);
      if (opt->refine_based) {
        // refine-based labels (Sec. 4.1): every super-vertex starts alone
        iota_i32(st, ws.start, ncom);
      } else {
        // move-based labels of the super-vertices (Alg. 1)
        fill_i32(st, ws.brank, 0, nn + 1);
        mark_used(st, ws.CB, nn, ws.brank);
        exclusive_scan(st, ws.brank, nn, ws.scan_tmp);
        next_labels(st, ws.lab, ws.CB, ws.brank, nn, ws.start);
      }
      GraphDesc nxt{ncom, yoff, ydeg, ws.idx[nb], ws.w[nb], det};
      if (opt->debug_trace) export_graph(ctx, nxt, ncom, pd);
      cur = nxt;
      tm.end(h);
    }
    if (opt->debug_trace) ctx->trace.push_back(std::move(pd));
    tau = tau / opt->tolerance_drop;
  }
  // ---- result: flatten the last refinement, canonical labels, Eq. 1
  h = tm.begin(kEvOther);
  if (ended) lookup_raw(st, top, n, ws.C, pass == 0);
  S->passes = ended ? pass + 1 : pass;
  fill_i32(st, ws.rank, std::numeric_limits<int32_t>::max(), n);
  first_occurrence(st, top, n, ws.rank);
  first_flags(st, top, ws.rank, n, ws.newid);
  exclusive_scan(st, ws.newid, n, ws.scan_tmp);
  apply_canonical(st, top, ws.rank, ws.newid, n);
  HIP_TRY(hipMemcpyAsync(&ctx->host->total, ws.newid + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  S->num_communities = ctx->host->total;
  s = modularity_device(ctx, ws, input, top, Wd, integral, resolution, modularity);
  if (s != GVL_OK) return s;
  tm.end(h);
  HIP_TRY(hipStreamSynchronize(st));
  S->scan_vertices = (int64_t)counter(ctx->host, 0);
  S->scan_arcs = (int64_t)counter(ctx->host, 1);
  S->scan_candidates = (int64_t)counter(ctx->host, 2);
  S->scan_moves = (int64_t)counter(ctx->host, 3);
  S->agg_vertices = (int64_t)counter(ctx->host, 4);
  S->agg_arcs = (int64_t)counter(ctx->host, 5);
  S->agg_out_arcs = (int64_t)counter(ctx->host, 6);
  S->scan_refine_arcs = (int64_t)counter(ctx->host, 7);
  S->table_overflows = (int64_t)ctx->host->ovf;
  if (tm.on) {
    double ms[kEvClasses];
    tm.totals(ms);
    S->ms_move = ms[kEvMove];
    S->ms_refine = ms[kEvRefine];
    S->ms_aggregate = ms[kEvAgg];
    S->ms_other = ms[kEvOther];
    S->ms_total = ms[kEvMove] + ms[kEvRefine] + ms[kEvAgg] + ms[kEvOther];
    S->ms_scan_kernels = ms[kEvScanMoveK] + ms[kEvScanRefineK];
    S->ms_scan_move_kernels = ms[kEvScanMoveK];
    S->ms_agg_kernels = ms[kEvAggK];
  }
  return GVL_OK;
}

gvl_status gvl_debug_pass_info(gvl_ctx_t ctx, int32_t pass, int64_t* n_out, int64_t* ncom_out, int64_t* m_out) {
  if (!ctx || pass < 0 || pass >= (int32_t)ctx->trace.size()) return GVL_E_INVALID_ARG;
  const PassDebug& p = ctx->trace[pass];
  if (n_out) *n_out = p.n;
  if (ncom_out) *ncom_out = p.ncom;
  if (m_out) *m_out = p.m;
  return GVL_OK;
}

gvl_status gvl_debug_export_pass(gvl_ctx_t ctx, int32_t pass, int32_t* bound, int32_t* refined, int32_t* y_off,
                                 int32_t* y_idx, double* y_w) {
  if (!ctx || pass < 0 || pass >= (int32_t)ctx->trace.size()) return GVL_E_INVALID_ARG;
  const PassDebug& p = ctx->trace[pass];
  if (bound && !p.bound.empty()) memcpy(bound, p.bound.data(), sizeof(int32_t) * p.bound.size());
  if (refined && !p.refined.empty()) memcpy(refined, p.refined.data(), sizeof(int32_t) * p.refined.size());
  if (p.m >= 0) {
    if (y_off) memcpy(y_off, p.y_off.data(), sizeof(int32_t) * p.y_off.size());
    if (y_idx && p.m > 0) memcpy(y_idx, p.y_idx.data(), sizeof(int32_t) * p.y_idx.size());
    if (y_w && p.m > 0) memcpy(y_w, p.y_w.data(), sizeof(double) * p.y_w.size());
  }
  return GVL_OK;
}

gvl_status gvl_debug_pass_movers(gvl_ctx_t ctx, int32_t pass, int64_t* movers, int32_t max_it,
                                 int64_t* refine_movers, int32_t max_sw) {
  if (!ctx || pass < 0 || pass >= (int32_t)ctx->trace.size()) return GVL_E_INVALID_ARG;
  const PassDebug& p = ctx->trace[pass];
  for (int32_t k = 0; movers && k < max_it && k < (int32_t)p.movers.size(); ++k) movers[k] = p.movers[k];
  for (int32_t k = 0; refine_movers && k < max_sw && k < (int32_t)p.refine_movers.size(); ++k)
    refine_movers[k] = p.refine_movers[k];
  return GVL_OK;
}

}  // extern "C"

// Stream of a context (used by the batch runner, same library).
hipStream_t gvl_context_stream(gvl_ctx_t ctx) { return ctx ? ctx->stream : nullptr; }
