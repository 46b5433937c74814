// Host-side internals shared by the single-graph driver and the fused batch
// driver: the workspace layout, the context, binning, hub plans and the
// device read-backs.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "gvl.h"
#include "kernels.hpp"

namespace gvl {

// Scalars shared between the device and one pinned host mirror.
struct Scalars {
  double dq[kCntSlots];                        // fast: summed move gains of an iteration
  unsigned long long dq128[kCntSlots][2];      // det: exact summed move keys (lo, hi)
  unsigned long long cnt[kCntSlots][8];        // kernel work counters (cumulative)
  int32_t flags[4];                 // input checks
  double accW;                      // total weight
  double acc_d[2];                  // modularity: S1, S2 (floating)
  unsigned long long acc_u[2];      // modularity: S2 exact (lo, hi)
  int32_t total;                    // scan totals read back
  int32_t sweep;                    // refinement sweep number, read by replayed sweeps (ScanArgs::sweep_dev)
  unsigned long long ovf;           // decisions cancelled by a partition table overflow (cumulative)
  int32_t iter;                     // local-moving iteration of the pass, read by the kernels (ScanArgs::it_dev)
};

static inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static inline int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Device workspace, carved out of the caller's buffer.
struct Workspace {
  double *K, *Sig;
  int32_t *size, *C, *CB, *start, *target, *newid, *brank, *lab, *rank, *cnt, *cv, *list, *scan_tmp;
  uint8_t* flag;
  int32_t* targeted;
  int2* CP;
  int32_t* list2;  // refinement: the thinned short-row bins
  // synchronous local-moving: decided gains (FP64, or exact keys in
  // deterministic mode), last move of each vertex, move records (ScanArgs)
  double* gainf;
  i128_t* gaink;
  int2* last;
  int4* mv;
  int32_t *off[2], *deg[2], *idx[2];
  void* w[2];
  TblSlot* tbl;
  int32_t* lbuf;  // partitioned hubs: sorted candidates, their weights, chunk offsets
  double* wbuf;
  uint16_t* poff;
  int64_t tbl_entries;
  // hub path
  int32_t *hp_chunk, *hp_tbl, *hp_slice, *hp_active, *hp_done, *hp_lcnt, *apre, *tbl_list;
  double* hp_kid;
  int2 *chunk_tasks, *slice_tasks;
  double* pb_g;
  i128_t* pb_k;
  int32_t* pb_c;
  int64_t max_tasks;
  // wide rows
  double* wd_g;
  i128_t* wd_k;
  int32_t *wd_c, *wd_ok, *wd_done, *wd_ctr;
  int64_t max_wide;

  Scalars* sc;
  BinBuf* bb;
  size_t bytes;
};

static int64_t table_entries(int64_t n) { return std::max<int64_t>(4 * next_pow2(2 * std::max<int64_t>(n, 1)), 1 << 16); }

// tbl_n: the largest vertex count of one graph (hub tables never span two
// graphs of a fused batch); < 0 means n.
static Workspace carve(int64_t n, int64_t m, bool det, char* base, int64_t tbl_n = -1) {
  Workspace w;
  memset(&w, 0, sizeof(w));
  size_t o = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + o : nullptr;
    o += align_up(bytes);
    return p;
  };
  const size_t N = (size_t)std::max<int64_t>(n, 1), M = (size_t)std::max<int64_t>(m, 1);
  const size_t ws = det ? sizeof(double) : sizeof(float);
  w.sc = (Scalars*)take(sizeof(Scalars));
  w.bb = (BinBuf*)take(sizeof(BinBuf));
  w.K = (double*)take(8 * N);
  w.Sig = (double*)take(8 * N);
  w.size = (int32_t*)take(4 * N);
  w.C = (int32_t*)take(4 * N);
  w.CB = (int32_t*)take(4 * N);
  w.start = (int32_t*)take(4 * N);
  w.target = (int32_t*)take(4 * N);
  w.newid = (int32_t*)take(4 * (N + 1));
  w.brank = (int32_t*)take(4 * (N + 1));
  w.lab = (int32_t*)take(4 * N);
  w.rank = (int32_t*)take(4 * (N + 1));
  w.cnt = (int32_t*)take(4 * (N + 1));
  w.cv = (int32_t*)take(4 * N);
  w.list = (int32_t*)take(4 * N);
  w.scan_tmp = (int32_t*)take(4 * ((size_t)scan_tiles((int64_t)N + 1) + 2));
  w.flag = (uint8_t*)take(N);
  w.targeted = (int32_t*)take(4 * N);
  w.CP = (int2*)take(8 * N);
  w.list2 = (int32_t*)take(4 * N);
  if (det) w.gaink = (i128_t*)take(16 * N); else w.gainf = (double*)take(8 * N);
  w.last = (int2*)take(8 * N);
  w.mv = (int4*)take(16 * N);
  for (int b = 0; b < 2; ++b) {
    w.off[b] = (int32_t*)take(4 * (N + 1));
    w.deg[b] = (int32_t*)take(4 * N);
    w.idx[b] = (int32_t*)take(4 * M);
    w.w[b] = (void*)take(ws * M);
  }
  w.tbl_entries = table_entries(tbl_n < 0 ? n : std::min(tbl_n, n));
  w.tbl = (TblSlot*)take(sizeof(TblSlot) * (size_t)w.tbl_entries);
  w.lbuf = (int32_t*)take(4 * M);
  w.wbuf = (double*)take(8 * M);
  // chunk tasks of one plan: sum of ceil(arcs / kHubChunk) over items of
  // more than kBinMax[kAggLastBin] arcs (aggregation; vertex hubs are longer)
  w.poff = (uint16_t*)take(2 * (kPartMaxP + 1) *
                           ((size_t)M / kHubChunk + (size_t)M / ((size_t)kBinMax[kAggLastBin] + 1) + 2));
  w.hp_chunk = (int32_t*)take(4 * (N + 1));
  w.hp_tbl = (int32_t*)take(4 * (N + 1));
  w.hp_slice = (int32_t*)take(4 * (N + 1));
  w.hp_active = (int32_t*)take(4 * N);
  w.hp_done = (int32_t*)take(4 * N);
  w.hp_lcnt = (int32_t*)take(4 * N);
  w.tbl_list = (int32_t*)take(4 * (size_t)w.tbl_entries);
  w.apre = (int32_t*)take(4 * (N + 1));
  w.hp_kid = (double*)take(8 * N);
  // chunk tasks <= H + M / kHubChunk; slice tasks <= H + M / (kHubSlice / 4)
  w.max_tasks = (int64_t)N + (int64_t)M / 1024 + 2;
  w.chunk_tasks = (int2*)take(sizeof(int2) * (size_t)w.max_tasks);
  w.slice_tasks = (int2*)take(sizeof(int2) * (size_t)w.max_tasks);
  w.pb_g = (double*)take(8 * (size_t)w.max_tasks);
  w.pb_k = (i128_t*)take(16 * (size_t)w.max_tasks);
  w.pb_c = (int32_t*)take(4 * (size_t)w.max_tasks);
  // vertices of the wide bins: degree above the bin-5 limit, at least kMinBin5
  w.max_wide = std::min<int64_t>((int64_t)N, (int64_t)M / (kMinBin5 + 1) + 1);
  const size_t wq = (size_t)w.max_wide * kWideMaxParts;
  w.wd_g = (double*)take(8 * wq);
  w.wd_k = (i128_t*)take(16 * wq);
  w.wd_c = (int32_t*)take(4 * wq);
  w.wd_ok = (int32_t*)take(4 * wq);
  w.wd_done = (int32_t*)take(4 * (size_t)w.max_wide);
  w.wd_ctr = (int32_t*)take(4 * 2);
  w.bytes = o;
  return w;
}

static unsigned long long counter(const Scalars* h, int k) {
  unsigned long long s = 0;
  for (int j = 0; j < kCntSlots; ++j) s += h->cnt[j][k];
  return s;
}

// Deterministic int128 -> double: hi * 2^64 + lo (one rounding in the add).
static double i128_to_double(unsigned long long lo, unsigned long long hi) {
  return (double)(long long)hi * 18446744073709551616.0 + (double)lo;
}

struct PassDebug {
  int64_t n = 0, ncom = 0, m = -1;
  std::vector<int32_t> bound, refined, y_off, y_idx;
  std::vector<double> y_w;
  std::vector<int64_t> movers, refine_movers;
};

}  // namespace gvl

using namespace gvl;

struct gvl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream on which launch sequences are recorded into HIP graphs
  BinLimits lim = {{4, 8, 16, 32, 128, 1024, 4096, 8192, 16384, 0x7fffffff}};  // bin limits of the call
  Scalars* host = nullptr;  // pinned
  BinBuf* hbins = nullptr;  // pinned
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  std::vector<PassDebug> trace;
};

// gvl_leiden_static's device array: resolves its address on `device` (the
// current device) once per device; called by gvl_create (static_ws.hip).
gvl_status gvl_static_scratch_setup(int device);

// Launch-shape tuning (tuning.hip): the table is loaded from the tune file
// once per process; class of a graph; the values of a class; bin limits.
void gvl_tuning_load_once();
int32_t gvl_class_of(int64_t n, int64_t m, bool fused);
gvl_tuning gvl_tuning_of(int32_t cls);
BinLimits bin_limits(const gvl_tuning& t);

namespace {

#define HIP_TRY(x)                                   \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) {                          \
      fprintf(stderr, "gvl: %s failed: %s\n", #x, hipGetErrorString(e_)); \
      return GVL_E_HIP;                              \
    }                                                \
  } while (0)

// Event pairs for per-phase timing (profile = 1).  Phase spans include the
// host read-backs between launches; kernel spans bracket only the launches
// of one kernel class.
enum { kEvMove = 0, kEvRefine = 1, kEvAgg = 2, kEvOther = 3, kEvScanMoveK = 4, kEvScanRefineK = 5,
       kEvAggK = 6, kEvClasses = 7 };

// Checks a HIP call whose failure the caller handles itself: reports it on
// stderr (the first 32 in a process) and clears the thread's last-error
// state so that it does not surface in the caller's later HIP calls.
inline bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  static int reported = 0;
  if (reported < 32) {
    ++reported;
    fprintf(stderr, "gvl: %s failed: %s\n", what, hipGetErrorString(e));
  }
  (void)hipGetLastError();
  return false;
}

struct Timer {
  gvl_ctx* ctx;
  bool on;
  struct Span { int cls; hipEvent_t a, b; };
  std::vector<Span> spans;
  hipEvent_t get() {
    if (ctx->ev_used == ctx->events.size()) {
      hipEvent_t e;
      if (!hip_ok(hipEventCreate(&e), "hipEventCreate")) return nullptr;
      ctx->events.push_back(e);
    }
    return ctx->events[ctx->ev_used++];
  }
  int begin(int cls) {
    if (!on) return -1;
    hipEvent_t e = get();
    if (!e || !hip_ok(hipEventRecord(e, ctx->stream), "hipEventRecord")) return -1;
    spans.push_back({cls, e, nullptr});
    return (int)spans.size() - 1;
  }
  void end(int h) {
    if (h < 0) return;
    hipEvent_t e = get();
    if (!e || !hip_ok(hipEventRecord(e, ctx->stream), "hipEventRecord")) return;
    spans[h].b = e;
  }
  void totals(double* ms) {
    for (int k = 0; k < kEvClasses; ++k) ms[k] = 0.0;
    for (auto& sp : spans) {
      float t = 0.f;
      if (sp.b && hip_ok(hipEventElapsedTime(&t, sp.a, sp.b), "hipEventElapsedTime")) ms[sp.cls] += t;
    }
  }
};

// A launch sequence (one local-moving iteration, one refinement sweep)
// recorded once into a HIP graph on the context's private stream, then
// launched as one graph on the context's stream, so its kernels run back to
// back instead of each waiting for the host to issue it.  body(stream) must
// enqueue only kernel launches whose arguments stay valid for every launch
// of the graph.  If recording fails the sequence runs eagerly from then on.
// *launches counts the kernels of every launch.  Not used while kernel
// classes are timed: HIP reports no elapsed time between events recorded by
// graph nodes, so timed runs launch every kernel from the host.
struct Replay {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool broken = false;
  bool launched = false;
  int64_t per_launch = 0;
  Replay() = default;
  Replay(const Replay&) = delete;
  Replay& operator=(const Replay&) = delete;
  ~Replay() { reset(); }
  void reset() {
    if (exec) hip_ok(hipGraphExecDestroy(exec), "hipGraphExecDestroy");
    if (graph) hip_ok(hipGraphDestroy(graph), "hipGraphDestroy");
    exec = nullptr;
    graph = nullptr;
    broken = false;
    per_launch = 0;
  }
  // undo(): restores host-side state the body changed while it was only
  // being recorded (called before the eager fallback of a failed recording)
  template <class F, class U>
  gvl_status run(gvl_ctx* ctx, bool use, int64_t* launches, F&& body, U&& undo) {
    launched = false;
    if (use && !broken && !exec && ctx->cap) {
      const int64_t before = *launches;
      if (hip_ok(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")) {
        body(ctx->cap);
        hipGraph_t g = nullptr;
        const bool ended = hip_ok(hipStreamEndCapture(ctx->cap, &g), "hipStreamEndCapture");
        if (ended && g && hip_ok(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "hipGraphInstantiate")) {
          graph = g;
          per_launch = *launches - before;
          *launches = before;
        } else {
          if (g) hip_ok(hipGraphDestroy(g), "hipGraphDestroy");
          exec = nullptr;
          broken = true;
          *launches = before;
          undo();
          (void)hipGetLastError();
        }
      } else {
        broken = true;
        (void)hipGetLastError();
      }
    }
    if (use && exec) {
      HIP_TRY(hipGraphLaunch(exec, ctx->stream));
      *launches += per_launch;
      launched = true;
      return GVL_OK;
    }
    body(ctx->stream);
    return GVL_OK;
  }
};

gvl_status readback(gvl_ctx* ctx, Scalars* dev) {
  HIP_TRY(hipMemcpyAsync(ctx->host, dev, sizeof(Scalars), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return GVL_OK;
}

// Bin the items of a graph (or of a capacity array) into S groups and fill
// `list`: bins 0..kHubBin-1 of every group (group-major), then the hub bin
// of every group in group order.
gvl_status make_bins(gvl_ctx* ctx, Workspace& ws, const int32_t* off, const int32_t* deg, int64_t n, int S,
                     bool wide, BinInfo& bins, const int32_t* gid = nullptr, const int32_t* vbase = nullptr,
                     const int32_t* gsh = nullptr) {
  hipStream_t st = ctx->stream;
  fill_i32(st, (int32_t*)ws.bb, 0, (int64_t)(sizeof(BinBuf) / sizeof(int32_t)));
  bin_count(st, off, deg, n, S, wide, gid, vbase, gsh, ctx->lim, ws.bb);
  HIP_TRY(hipMemcpyAsync(ctx->hbins, ws.bb, sizeof(BinBuf), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  bins.S = S;
  int32_t acc = 0;
  for (int g = 0; g < S; ++g) {
    bins.gstart[g] = acc;
    for (int b = 0; b < kHubBin; ++b) {
      bins.count[g][b] = ctx->hbins->counts[g * kNumBins + b];
      bins.start[g][b] = acc;
      ctx->hbins->cursors[g * kNumBins + b] = acc;
      acc += bins.count[g][b];
    }
    bins.gend[g] = acc;
  }
  bins.gstart[S] = acc;
  bins.H0 = acc;
  for (int g = 0; g < S; ++g) {
    bins.count[g][kHubBin] = ctx->hbins->counts[g * kNumBins + kHubBin];
    bins.start[g][kHubBin] = acc;
    ctx->hbins->cursors[g * kNumBins + kHubBin] = acc;
    acc += bins.count[g][kHubBin];
  }
  bins.H = acc - bins.H0;
  bins.binned = acc;
  for (int b = 0; b < kNumBins; ++b) bins.maxsize[b] = ctx->hbins->maxsize[b];
  HIP_TRY(hipMemcpyAsync(ws.bb->cursors, ctx->hbins->cursors, sizeof(int32_t) * S * kNumBins,
                         hipMemcpyHostToDevice, st));
  bin_scatter(st, off, deg, n, S, wide, gid, vbase, gsh, ctx->lim, ws.bb, ws.list);
  return GVL_OK;
}

// Every per-vertex array the synchronous local-moving kernels write or read
// (gains, last moves, move records, iteration counter) is set.
static inline bool scan_state_ready(const ScanArgs& a, bool det) {
  return a.last && a.mv && a.it_dev && (det ? a.gaink != nullptr : a.gainf != nullptr);
}

// Refinement (Alg. 3) after a sweep: the short-row bins of `bins` (in
// ws.list) reduced to their vertices still alone in their refined community,
// in ws.list2 with the same group-major layout; `rb` describes them (its hub
// counts are the lone hubs, which stay where `bins` has them, in ws.list).
gvl_status thin_refine_bins(gvl_ctx* ctx, Workspace& ws, const BinInfo& bins, BinInfo& rb) {
  hipStream_t st = ctx->stream;
  BinBuf* hb = ctx->hbins;
  memset(hb, 0, sizeof(BinBuf));
  for (int g = 0; g < bins.S; ++g)
    for (int b = 0; b < kNumBins; ++b) {
      hb->cursors[g * kNumBins + b] = bins.start[g][b];
      hb->counts[g * kNumBins + b] = bins.count[g][b];
    }
  HIP_TRY(hipMemcpyAsync(ws.bb, hb, sizeof(BinBuf), hipMemcpyHostToDevice, st));
  thin_count(st, ws.list, ws.bb, bins.S, ws.C, ws.size, ws.K);
  HIP_TRY(hipMemcpyAsync(hb->kept, ws.bb->kept, sizeof(hb->kept), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  rb = bins;
  int32_t acc = 0;
  for (int g = 0; g < bins.S; ++g) {
    rb.gstart[g] = acc;
    for (int b = 0; b < kHubBin; ++b) {
      const int s = g * kNumBins + b;
      rb.count[g][b] = hb->kept[s];
      rb.start[g][b] = acc;
      hb->nstart[s] = acc;
      acc += hb->kept[s];
    }
    rb.gend[g] = acc;
    rb.count[g][kHubBin] = hb->kept[g * kNumBins + kHubBin];  // lone hubs (they stay in ws.list)
  }
  rb.gstart[bins.S] = acc;
  HIP_TRY(hipMemcpyAsync(ws.bb->nstart, hb->nstart, sizeof(hb->nstart), hipMemcpyHostToDevice, st));
  thin_scatter(st, ws.list, ws.bb, bins.S, ws.C, ws.size, ws.K, ws.list2);
  return GVL_OK;
}

// Hub plan of one graph (or of the giant communities of an aggregation):
// chunk / table / slice offsets on the device, task lists, and batches of
// consecutive hubs of one group whose tables fit the table region together.
struct HubBatch {
  int32_t h0, h1, c0, c1, s0, s1;
  int64_t tbase, tend;
};
struct HubPlan {
  int32_t H = 0;
  int32_t T = 0;
  std::vector<std::vector<HubBatch>> groups;  // per group
};

gvl_status build_hub_plan(gvl_ctx* ctx, Workspace& ws, const BinInfo& bins, bool agg, const GraphDesc& g,
                          const int32_t* yoff, int64_t ncom, HubPlan& plan) {
  hipStream_t st = ctx->stream;
  plan = HubPlan();
  plan.H = bins.H;
  plan.groups.assign(bins.S, {});
  if (bins.H == 0) return GVL_OK;
  const int32_t* items = ws.list + bins.H0;
  const int32_t H = bins.H;
  // Distinct keys of one table are at most the items with arcs (bins.binned):
  // communities / vertices without arcs are never anyone's neighbour.
  if (agg) gagg_setup(st, yoff, items, H, ws.hp_chunk, ws.hp_tbl, ws.hp_slice);
  else hub_setup(st, g.off, g.deg, items, H, bins.binned, ws.hp_chunk, ws.hp_tbl, ws.hp_slice);
  exclusive_scan(st, ws.hp_chunk, H, ws.scan_tmp);
  exclusive_scan(st, ws.hp_tbl, H, ws.scan_tmp);
  exclusive_scan(st, ws.hp_slice, H, ws.scan_tmp);
  std::vector<int32_t> hc(H + 1), ht(H + 1), hs(H + 1);
  HIP_TRY(hipMemcpyAsync(hc.data(), ws.hp_chunk, sizeof(int32_t) * (H + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(ht.data(), ws.hp_tbl, sizeof(int32_t) * (H + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(hs.data(), ws.hp_slice, sizeof(int32_t) * (H + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hc[H] > ws.max_tasks || hs[H] > ws.max_tasks) return GVL_E_WORKSPACE;
  plan.T = hc[H];
  hub_tasks(st, H, ws.hp_chunk, ws.hp_slice, ws.chunk_tasks, ws.slice_tasks);
  const int64_t region = ws.tbl_entries;
  for (int grp = 0; grp < bins.S; ++grp) {
    int32_t a = bins.start[grp][kHubBin] - bins.H0;
    const int32_t e = a + bins.count[grp][kHubBin];
    while (a < e) {
      int32_t b = a + 1;
      while (b < e && (int64_t)(ht[b + 1] - ht[a]) * kTblUnit <= region) ++b;
      HubBatch hb;
      hb.h0 = a; hb.h1 = b;
      hb.c0 = hc[a]; hb.c1 = hc[b];
      hb.s0 = hs[a]; hb.s1 = hs[b];
      hb.tbase = (int64_t)ht[a] * kTblUnit;
      hb.tend = (int64_t)ht[b] * kTblUnit;
      plan.groups[grp].push_back(hb);
      a = b;
    }
  }
  return GVL_OK;
}

HubArgs hub_args(Workspace& ws, const BinInfo& bins) {
  HubArgs h;
  memset(&h, 0, sizeof(h));
  h.items = ws.list + bins.H0;
  h.chunk_off = ws.hp_chunk; h.tbl_off = ws.hp_tbl; h.slice_off = ws.hp_slice;
  h.chunk_tasks = ws.chunk_tasks; h.slice_tasks = ws.slice_tasks;
  h.active = ws.hp_active; h.kid = ws.hp_kid; h.done = ws.hp_done;
  h.pb_g = ws.pb_g; h.pb_k = ws.pb_k; h.pb_c = ws.pb_c;
  h.tbl = ws.tbl;
  h.lbuf = ws.lbuf;
  h.wbuf = ws.wbuf;
  h.poff = ws.poff;
  h.tbl_list = ws.tbl_list; h.lcnt = ws.hp_lcnt;
  h.apre = ws.apre;
  return h;
}

// Table slots below `clean` are known to be empty: every use leaves its
// slots empty, so only the first use of a slot in a call needs clearing.
struct TableState {
  int64_t clean = 0;
  void ensure(hipStream_t st, Workspace& ws, int64_t extent) {
    if (extent <= clean) return;
    fill_slots(st, ws.tbl + clean, extent - clean);
    clean = extent;
  }
};

// K' (row sums) of a graph: short rows by kernel, hub rows by chunks.
void graph_weights(gvl_ctx* ctx, Workspace& ws, const GraphDesc& g, int64_t m, const BinInfo& bins,
                   const HubPlan& plan, int validate) {
  hipStream_t st = ctx->stream;
  vertex_weights(st, g, m, ws.K, &ws.sc->accW, ws.sc->flags, validate);
  if (plan.H > 0) {
    HubArgs h = hub_args(ws, bins);
    hub_weights(st, g, h, 0, plan.T, ws.K, &ws.sc->accW, ws.sc->flags, validate);
  }
}

void export_graph(gvl_ctx* ctx, const GraphDesc& g, int64_t ncom, PassDebug& pd) {
  std::vector<int32_t> off(ncom + 1), deg(ncom);
  (void)hipMemcpyAsync(off.data(), g.off, sizeof(int32_t) * (ncom + 1), hipMemcpyDeviceToHost, ctx->stream);
  (void)hipMemcpyAsync(deg.data(), g.deg, sizeof(int32_t) * ncom, hipMemcpyDeviceToHost, ctx->stream);
  (void)hipStreamSynchronize(ctx->stream);
  const int64_t cap = off[ncom];
  std::vector<int32_t> idx(std::max<int64_t>(cap, 1));
  std::vector<double> wd(std::max<int64_t>(cap, 1));
  std::vector<float> wf;
  (void)hipMemcpyAsync(idx.data(), g.idx, sizeof(int32_t) * cap, hipMemcpyDeviceToHost, ctx->stream);
  if (g.w_double) {
    (void)hipMemcpyAsync(wd.data(), g.w, sizeof(double) * cap, hipMemcpyDeviceToHost, ctx->stream);
  } else {
    wf.resize(std::max<int64_t>(cap, 1));
    (void)hipMemcpyAsync(wf.data(), g.w, sizeof(float) * cap, hipMemcpyDeviceToHost, ctx->stream);
  }
  (void)hipStreamSynchronize(ctx->stream);
  pd.y_off.assign(ncom + 1, 0);
  pd.y_idx.clear();
  pd.y_w.clear();
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t r = 0; r < ncom; ++r) {
    row.clear();
    for (int32_t k = 0; k < deg[r]; ++k) {
      const int64_t e = (int64_t)off[r] + k;
      row.push_back({idx[e], g.w_double ? wd[e] : (double)wf[e]});
    }
    std::sort(row.begin(), row.end());
    for (auto& x : row) { pd.y_idx.push_back(x.first); pd.y_w.push_back(x.second); }
    pd.y_off[r + 1] = (int32_t)pd.y_idx.size();
  }
  pd.m = (int64_t)pd.y_idx.size();
}

template <class T>
std::vector<T> to_host(gvl_ctx* ctx, const T* d, int64_t n) {
  std::vector<T> h(std::max<int64_t>(n, 1));
  (void)hipMemcpyAsync(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, ctx->stream);
  (void)hipStreamSynchronize(ctx->stream);
  h.resize(n);
  return h;
}

// Eq. 1 of `membership` on the input graph, computed on the device.
gvl_status modularity_device(gvl_ctx* ctx, Workspace& ws, const GraphDesc& in, const int32_t* membership,
                             double W, bool integral, double gamma, double* q) {
  hipStream_t st = ctx->stream;
  BinInfo bins;
  gvl_status s = make_bins(ctx, ws, in.off, in.deg, in.n, 1, true, bins);
  if (s != GVL_OK) return s;
  HubPlan plan;
  s = build_hub_plan(ctx, ws, bins, false, in, nullptr, 0, plan);
  if (s != GVL_OK) return s;
  fill_f64(st, ws.Sig, 0.0, in.n);
  fill_f64(st, ws.sc->acc_d, 0.0, 2);
  fill_u64(st, ws.sc->acc_u, 0ull, 2);
  modularity_partial(st, in, membership, ws.Sig, ws.sc->acc_d);
  if (plan.H > 0) hub_modularity(st, in, hub_args(ws, bins), 0, plan.T, membership, ws.Sig, ws.sc->acc_d);
  modularity_squares(st, ws.Sig, in.n, integral, ws.sc->acc_d, ws.sc->acc_u);
  s = readback(ctx, ws.sc);
  if (s != GVL_OK) return s;
  const double S1 = ctx->host->acc_d[0];
  const double S2 = integral ? i128_to_double(ctx->host->acc_u[0], ctx->host->acc_u[1]) : ctx->host->acc_d[1];
  *q = (W == 0.0) ? 0.0 : S1 / W - gamma * (S2 / (W * W));
  return GVL_OK;
}

gvl_status check_args(gvl_ctx* ctx, int64_t n, int64_t m, const int32_t* off, const int32_t* idx,
                      double resolution, const gvl_options* opt, void* wsp, size_t wsb) {
  if (!ctx || !opt || n < 0 || m < 0 || m > 2147483647LL || n > 2147483646LL) return GVL_E_INVALID_ARG;
  if (n > 0 && !off) return GVL_E_INVALID_ARG;
  if (m > 0 && !idx) return GVL_E_INVALID_ARG;
  if (!(resolution >= 0.0) || !std::isfinite(resolution)) return GVL_E_RESOLUTION;
  if (opt->mode != GVL_MODE_FAST && opt->mode != GVL_MODE_DET) return GVL_E_INVALID_ARG;
  if ((opt->louvain != 0 && opt->louvain != 1) || (opt->refine_random != 0 && opt->refine_random != 1) ||
      (opt->shrink_excludes_isolated != 0 && opt->shrink_excludes_isolated != 1) ||
      (opt->refine_based != 0 && opt->refine_based != 1) || opt->validate < 0 ||
      opt->validate > 2)
    return GVL_E_INVALID_ARG;
  if (opt->max_iterations < 1 || opt->max_iterations > kMaxIterationsSync || opt->max_passes < 1 ||
      opt->refine_sweeps < 1 || opt->subsweeps < 0 ||
      (opt->subsweeps == 0 && opt->mode == GVL_MODE_DET) || opt->subsweeps > kMaxGroups ||
      !(opt->tolerance_drop > 0.0) || !(opt->aggregation_tolerance >= 0.0))
    return GVL_E_INVALID_ARG;
  size_t need = 0;
  gvl_workspace_bytes(n, m, opt, &need);
  if (!wsp || wsb < need) return GVL_E_WORKSPACE;
  return GVL_OK;
}

}  // namespace
