// Neighbour-community scan: the decision kernels shared by local-moving
// (Alg. 2, scanCommunities) and refinement (Alg. 3, scanBounded), and the
// commit kernel of the synchronous variants.
//
// For a vertex i the scan accumulates H[C[j]] += w_ij over the arcs of i
// (j != i; refinement also requires CB[j] == CB[i]), evaluates the
// delta-modularity of Eq. 2 for every community in H other than d = C[i],
// and picks the best one (largest gain, lowest id on ties).
//   fast mode:  gain = (K_ic - K_id) / m - gamma K_i (K_i + Sigma_c - Sigma_d) / (2 m^2)  (FP64)
//   det mode:   key  = 2^16 W (K_ic - K_id) - p K_i (K_i + Sigma_c - Sigma_d)             (int128)
//               with gamma = p / 2^16, so that gain = 2 key / (2^16 W^2) exactly.
// Local-moving in fast mode commits a move at once (asynchronous updates,
// Sec. 4.1): Sigma and sizes by atomics, C[i] by a plain store, neighbours
// marked unprocessed.  Deterministic local-moving, fast local-moving with
// sync_moves, and refinement record the choice in target[] and a separate
// commit kernel applies it.
//
// Singleton-to-singleton moves go only towards the lower community id
// (min-label rule), which stops pairs of singletons from swapping.
#pragma once

#include "device.hpp"
#include "kernels.hpp"

namespace gvl {

// Refinement stamp of the current group and the current sweep number (see
// ScanArgs::sweep_dev).
__device__ __forceinline__ int32_t cur_stamp(const ScanArgs& a) {
  return a.sweep_dev ? a.stamp + *a.sweep_dev * a.groups : a.stamp;
}
__device__ __forceinline__ int32_t cur_sweep(const ScanArgs& a) { return a.sweep_dev ? *a.sweep_dev : a.sweep; }

template <int PH, bool DET>
struct Decide {
  // Returns true if vertex i is to be scanned in this launch.
  __device__ static __forceinline__ bool eligible(const ScanArgs& a, int32_t i) {
    if (PH == kMove) return a.flag[i] != 0;
    return a.size[a.C[i]] == 1 && a.K[i] > 0.0;
  }
};

// Accumulators of one thread, reduced once per workgroup at kernel end.
struct Acc {
  double dq = 0.0;
  i128 dqk = 0;
  unsigned long long nv = 0, na = 0, nc = 0, nm = 0;
};

template <int PH, bool DET>
__device__ __forceinline__ void flush_acc(const ScanArgs& a, Acc& acc) {
  __shared__ double red_d[16];
  __shared__ unsigned long long red_u[16];
  __shared__ i128 red_k[16];
  unsigned long long nv = block_sum<unsigned long long>(acc.nv, red_u);
  unsigned long long na = block_sum<unsigned long long>(acc.na, red_u);
  unsigned long long nc = block_sum<unsigned long long>(acc.nc, red_u);
  unsigned long long nm = block_sum<unsigned long long>(acc.nm, red_u);
  if (DET) {
    i128 k = block_sum_i128(acc.dqk, red_k);
    if (threadIdx.x == 0 && k != 0) atomic_add_i128(a.dq128 + 2 * cslot(), k);
  } else {
    double d = block_sum<double>(acc.dq, red_d);
    if (threadIdx.x == 0 && d != 0.0) atomicAdd(a.dq + cslot(), d);
  }
  if (threadIdx.x == 0) {
    if (nv) atomicAdd(&cnt_of(a.cnt)[0], nv);
    if (na) atomicAdd(&cnt_of(a.cnt)[1], na);
    if (PH == kRefine && na) atomicAdd(&cnt_of(a.cnt)[7], na);
    if (nc) atomicAdd(&cnt_of(a.cnt)[2], nc);
    if (nm) atomicAdd(&cnt_of(a.cnt)[3], nm);
  }
}

// Gain of one candidate; updates the running best.  With the randomized
// refinement (a.rnd) only positive gains compete, each by the score
// gain / (-ln u) of its own draw (the largest wins: c is chosen with
// probability proportional to its gain); in deterministic mode the score of
// the exact key is carried in the key slot as its IEEE bit pattern, which
// orders positive doubles like their values.
template <bool DET>
struct Eval {
  double kid, ki, sd, gk, inv_m;
  long long kidi, kii, sdi;
  i128 A, B;
  int32_t rnd, il, base;
  // i: the vertex (its graph's constants in a fused batch)
  __device__ __forceinline__ Eval(const ScanArgs& a, int32_t i, double kid_, double ki_, double sd_) {
    double im = a.inv_m, gks = a.gk_scale;
    long long W = a.W, p = a.p;
    base = 0;
    if (a.gid) {
      const GraphParam q = a.gp[a.gid[i]];
      im = q.inv_m; gks = q.gk_scale; W = q.W; p = q.p;
      if (a.rnd) base = a.vbase[a.gid[i]];
    }
    rnd = a.rnd;
    il = i - base;
    kid = kid_; ki = ki_; sd = sd_;
    inv_m = im;
    gk = gks * ki_;
    kidi = (long long)kid_; kii = (long long)ki_; sdi = (long long)sd_;
    A = (i128)65536 * (i128)W;
    B = (i128)p * (i128)kii;
  }
  // Every arc from i into a candidate community c also counts in the weight
  // of its member, so Sigma_c >= K_{i->c}; Eq. 2 with Sigma_c = K_{i->c}
  // then bounds the gain from above (the gain falls as Sigma_c grows).  A
  // candidate whose bound is not positive is never chosen (a move needs a
  // positive gain, also in randomized refinement), so its total is not read.
  __device__ __forceinline__ bool may_gain(double kic) const {
    if (DET) {
      const long long k = (long long)kic;
      return A * (i128)(k - kidi) - B * (i128)(kii + k - sdi) > 0;
    }
    return (kic - kid) * inv_m - gk * (ki + kic - sd) > 0.0;
  }
  __device__ __forceinline__ double score(const ScanArgs& a, double gain, int32_t c) const {
    return gain / neg_ln_unit(draw32(a.seed, a.pass, cur_sweep(a), il, c - base));
  }
  __device__ __forceinline__ void operator()(const ScanArgs& a, int32_t c, double kic, double sc,
                                             double& bg, i128& bk, int32_t& bc) const {
    if (DET) {
      i128 k = A * (i128)((long long)kic - kidi) - B * (i128)(kii + (long long)sc - sdi);
      if (rnd) {
        if (!(k > 0)) return;
        k = (i128)__double_as_longlong(score(a, key_to_double(k), c));
      }
      if (better_k(k, c, bk, bc)) { bk = k; bc = c; }
    } else {
      double x = (kic - kid) * inv_m - gk * (ki + sc - sd);
      if (rnd) {
        if (!(x > 0.0)) return;
        x = score(a, x, c);
      }
      if (better_f(x, c, bg, bc)) { bg = x; bc = c; }
    }
  }
};

// Adds the gain of a move of vertex i to the iteration's sum: the
// workgroup's accumulator for a single graph, the graph's own sum in a
// fused batch.
template <bool DET>
__device__ __forceinline__ void add_gain(const ScanArgs& a, Acc& acc, int32_t i, double bg, i128 bk) {
  if (a.gid) {
    const int32_t g = a.gid[i];
    if (DET) atomic_add_i128(a.dqg128 + 2 * g, bk);
    else atomicAdd(a.dqg + g, bg);
  } else {
    if (DET) acc.dqk += bk; else acc.dq += bg;
  }
}

// Records the gain of a synchronous local-moving decision of a row of at
// most kSwapRowMax arcs; the commit adds it if the move is applied.
template <bool DET>
__device__ __forceinline__ void store_gain(const ScanArgs& a, int32_t i, double bg, i128 bk) {
  if (DET) a.gaink[i] = bk; else a.gainf[i] = bg;
}

// Sub-sweep group of neighbour j of a vertex whose graph starts at vbase
// (group shift sh in a fused batch).
__device__ __forceinline__ int group_in_pass(const ScanArgs& a, int32_t j, int32_t vbase, int sh) {
  return group_of(j - vbase, a.groups >> sh) << sh;
}

// Stamp of the current (iteration, group) of the synchronous local-moving,
// unique within a pass and > 0; and the move record of a decision: partner
// = the one neighbour of the group in the target (a row of at most
// kSwapRowMax arcs), -2 for several (the commit reads the row), -1 for a
// row that never yields.
__device__ __forceinline__ int32_t move_stamp(const ScanArgs& a) { return *a.it_dev * a.groups + a.grp + 1; }
__device__ __forceinline__ void record_move(const ScanArgs& a, int32_t i, int32_t d, int32_t t, int32_t partner) {
  a.mv[i] = make_int4(d, t, move_stamp(a), partner);
}

template <int G>
__device__ __forceinline__ int sum_lanes(int f) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) f += __shfl_xor(f, o, G);
  return f;
}
template <int G>
__device__ __forceinline__ int max_lanes(int f) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) f = max(f, __shfl_xor(f, o, G));
  return f;
}

// Workgroup argmax of (gain or key, id) over NW wavefronts; the result is
// valid in every thread.
template <bool DET, int NW = kBlock / kWave>
__device__ __forceinline__ void block_argmax(double& bg, i128& bk, int32_t& bc, double* s_g, i128* s_k,
                                             int32_t* s_c) {
  if (DET) argmax_k<kWave>(bk, bc); else argmax_f<kWave>(bg, bc);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) { s_g[w] = bg; s_k[w] = bk; s_c[w] = bc; }
  __syncthreads();
  bc = s_c[0]; bg = s_g[0]; bk = s_k[0];
  for (int k = 1; k < NW; ++k) {
    if (DET) { if (better_k(s_k[k], s_c[k], bk, bc)) { bk = s_k[k]; bc = s_c[k]; } }
    else { if (better_f(s_g[k], s_c[k], bg, bc)) { bg = s_g[k]; bc = s_c[k]; } }
  }
}

// Whether a synchronous commit must mark neighbour j (see mark_after).
__device__ __forceinline__ bool mark_needed(const ScanArgs& a, int32_t j) {
  return a.mark_after == INT32_MAX || group_of(j, a.groups) <= a.mark_after;
}

// Marks the neighbours j != i of a moved vertex i as unprocessed (Alg. 2):
// the arcs e0, e0 + nt, ... < deg of its row, kMarkUnroll per thread per
// step with their index loads issued together (the marks do not depend on
// each other).  check (synchronous commits): only where mark_needed, and a
// flag is read before it is written: a vertex with many moving neighbours
// is marked by each of them, and the read of a set flag stays in the cache
// where each store would travel to memory.  (No flag is cleared while a
// commit runs, so a skipped store is never needed; the asynchronous
// schedule clears flags concurrently and always stores.)  The flag reads
// are branch-guarded and so issued one at a time; reading every lane's
// flag through a valid index instead measured no faster.
constexpr int kMarkUnroll = 8;
template <class WT>
__device__ __forceinline__ void mark_row(const GraphView<WT>& g, const ScanArgs& a, int32_t i, int32_t beg,
                                         int32_t deg, int32_t e0, int32_t nt, bool check) {
  for (int32_t base = e0; base < deg; base += kMarkUnroll * nt) {
    int32_t j[kMarkUnroll];
    uint8_t f[kMarkUnroll];
#pragma unroll
    for (int u = 0; u < kMarkUnroll; ++u) {
      const int32_t e = base + u * nt;
      j[u] = (e < deg) ? g.idx[beg + e] : i;
    }
#pragma unroll
    for (int u = 0; u < kMarkUnroll; ++u) {
      const bool want = j[u] != i && (!check || mark_needed(a, j[u]));
      f[u] = !want ? 1 : (check ? a.flag[j[u]] : 0);
    }
#pragma unroll
    for (int u = 0; u < kMarkUnroll; ++u)
      if (f[u] == 0) a.flag[j[u]] = 1;
  }
}

// Bounce rule of the synchronous local-moving: a vertex that moved in each
// of the two previous iterations does not go straight back to the community
// it left in the last one (it is cycling with a neighbour of its group).
// (l: the vertex's last-move entry, it: the current iteration)
__device__ __forceinline__ bool bounced(int2 l, int32_t bc, int32_t it) {
  return l.x == bc && (int16_t)(l.y & 0xFFFF) == it - 1 && (int16_t)((uint32_t)l.y >> 16) == it - 2;
}
__device__ __forceinline__ bool bounces(const ScanArgs& a, int32_t i, int32_t bc) {
  return bounced(a.last[i], bc, *a.it_dev);
}

// After the argmax: apply the min-label rule, the sign test and, for a
// synchronous local-moving decision (sync), the bounce rule.
template <int PH, bool DET>
__device__ __forceinline__ bool accept(const ScanArgs& a, int32_t i, int32_t d, int32_t bc, double bg, i128 bk,
                                       bool sync) {
  if (bc < 0) return false;
  if (DET ? !(bk > 0) : !(bg > 0.0)) return false;
  if (PH == kMove) {
    if (a.size[d] == 1 && a.size[bc] == 1 && bc > d) return false;
    if (sync && bounces(a, i, bc)) return false;
  } else {
    if (a.size[bc] == 1 && bc > d) return false;
  }
  return true;
}

// A row's own state, loaded ahead of its scan: row bounds, bound label
// (refinement), label, K', and the pruning flag (local-moving).  Only the
// loads go out here; nothing waits for them.
struct RowState {
  int32_t beg = 0, deg = 0, bi = 0, d = 0;
  double ki = 0.0;
  uint8_t flag = 0;
};
template <int PH, class WT>
__device__ __forceinline__ RowState load_row_state(const GraphView<WT>& g, const ScanArgs& a, int32_t i) {
  RowState r;
  r.beg = g.begin(i);
  r.deg = g.degree(i);
  if (PH == kRefine) r.bi = a.CB[i];
  r.d = a.C[i];
  r.ki = a.K[i];
  if (PH == kMove) r.flag = a.flag[i];
  return r;
}
// Decide::eligible on a loaded state (refinement reads the size of the own
// community here: the row's label is already loaded).  sync: the loaded
// pruning flag is current (no decision of a synchronous schedule sets a
// flag); the asynchronous schedule marks neighbours while others decide,
// so there the flag of vertex i is read again now.
template <int PH>
__device__ __forceinline__ bool row_eligible(const ScanArgs& a, const RowState& r, int32_t i, bool sync) {
  if (PH == kMove) return (sync ? r.flag : a.flag[i]) != 0;
  return a.size[r.d] == 1 && r.ki > 0.0;
}

// The state of vertex i (own community d) that the tests after the argmax
// read, loaded before the scan so that the only load left between the
// argmax and the decision is size[c*] for a singleton (see accept_pre).
// sync: synchronous local-moving (the bounce rule applies); it: the
// iteration (read once per launch).
struct Pre {
  int32_t size_d = 0;
  int2 last = make_int2(kEmpty, 0);
  int32_t it = 0;
};
template <int PH>
__device__ __forceinline__ Pre prefetch_state(const ScanArgs& a, int32_t i, int32_t d, bool sync, int32_t it) {
  Pre p;
  if (PH == kMove) {
    p.size_d = a.size[d];
    if (sync) p.last = a.last[i];
    p.it = it;
  }
  return p;
}
// accept() on prefetched state: the same tests in an order that reads
// size[bc] only where it decides.
template <int PH, bool DET>
__device__ __forceinline__ bool accept_pre(const ScanArgs& a, const Pre& p, int32_t d, int32_t bc, double bg,
                                           i128 bk, bool sync) {
  if (bc < 0) return false;
  if (DET ? !(bk > 0) : !(bg > 0.0)) return false;
  if (PH == kMove) {
    if (p.size_d == 1 && bc > d && a.size[bc] == 1) return false;
    if (sync && bounced(p.last, bc, p.it)) return false;
  } else {
    if (bc > d && a.size[bc] == 1) return false;
  }
  return true;
}
// The iteration number for the bounce rule, once per launch (sync only).
template <int PH>
__device__ __forceinline__ int32_t launch_iteration(const ScanArgs& a, bool sync) {
  return (PH == kMove && sync) ? *a.it_dev : 0;
}

// Accumulates the arcs e0, e0 + NT, ... of row i: arcs to the vertex's own
// community d are summed into the returned K_{i->d} (kept out of the table,
// whose slot would otherwise take an atomic per intra-community arc), every
// other neighbour community goes to ins(c, w).  U arcs per round, with their
// index, weight, label (and bound) loads issued together.
// note(u, j, c) sees arc u of the lane's round (j: neighbour, c: its label,
// kEmpty past the row or outside the bound).
template <int U, int NT, int PH, class WT, class Ins, class Note>
__device__ __forceinline__ double scan_row(const GraphView<WT>& g, const ScanArgs& a, int32_t i, int32_t beg,
                                           int32_t deg, int32_t e0, int32_t d, int32_t bi, Ins ins, Note note) {
  double kid = 0.0;
  for (int32_t base = e0; base < deg; base += U * NT) {
    int32_t j[U];
    WT wr[U];  // raw weights: converted where used, so the round's loads are all in flight first
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = base + u * NT;
      j[u] = i;
      wr[u] = WT(1);
      if (e < deg) {
        j[u] = g.idx[beg + e];
        wr[u] = g.weight(beg + e);
      }
    }
    // The label loads of the round go out first and land in registers
    // nothing else writes (a value merged into a load's register from
    // another branch would make the compiler wait for that load there).
    int2 cb[U];  // (label, bound label) of each neighbour
    bool own[U];  // label known without a load (its id)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = j[u] != i;
      own[u] = PH == kMove && a.ident_after >= 0 && ok && group_of(j[u], a.groups) > a.ident_after;
      cb[u] = make_int2(kEmpty, bi);
      if (PH == kRefine && a.CP) {
        if (ok) cb[u] = a.CP[j[u]];
      } else if (ok && !own[u]) {
        cb[u].x = a.C[j[u]];
        if (PH == kRefine) cb[u].y = a.CB[j[u]];
      }
    }
    int32_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = own[u] ? j[u] : cb[u].x;
      if (PH == kRefine && cb[u].y != bi) c[u] = kEmpty;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      note(u, j[u], c[u]);
      if (c[u] == kEmpty) continue;
      const double w = (double)wr[u];
      if (c[u] == d) kid += w;
      else ins(c[u], w);
    }
  }
  return kid;
}
template <int U, int NT, int PH, class WT, class Ins>
__device__ __forceinline__ double scan_row(const GraphView<WT>& g, const ScanArgs& a, int32_t i, int32_t beg,
                                           int32_t deg, int32_t e0, int32_t d, int32_t bi, Ins ins) {
  return scan_row<U, NT, PH>(g, a, i, beg, deg, e0, d, bi, ins, [](int, int32_t, int32_t) {});
}

// Evaluates the table slots s0, s0 + NT, ... < ts (no slot holds d) and
// clears them; U slots per round with their Sigma loads issued together.
template <int U, int NT, bool DET>
__device__ __forceinline__ void eval_table(int32_t* keys, double* vals, int ts, int s0, const ScanArgs& a,
                                           const Eval<DET>& ev, Acc& acc, double& bg, i128& bk, int32_t& bc) {
  for (int base = s0; base < ts; base += U * NT) {
    int32_t c[U];
    double v[U], sg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = base + u * NT;
      c[u] = (s < ts) ? keys[s] : kEmpty;
      v[u] = (c[u] != kEmpty) ? vals[s] : 0.0;
    }
    bool e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) e[u] = c[u] != kEmpty && ev.may_gain(v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) sg[u] = e[u] ? a.Sig[c[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = base + u * NT;
      if (e[u]) {
        ++acc.nc;
        ev(a, c[u], v[u], sg[u], bg, bk, bc);
      }
      if (c[u] != kEmpty) {
        keys[s] = kEmpty;
        vals[s] = 0.0;
      }
    }
  }
}

// ------------------------------------------------ group of G lanes per vertex ---
// Bins 0-5 in one launch (k_decide_groups): blocks [blk[b], blk[b+1]) serve
// bin b, bins 0-4 with groups of G lanes per vertex (the bin's rows have at
// most BMAX arcs), bin 5 with one workgroup per vertex.
struct GroupLaunch {
  int32_t count[6];
  int32_t start[6];
  // the group's hub snapshot, served by blocks [blk[6], blk[7]): hubs
  // [h0, h1) of HubArgs::items, with its active and kid arrays
  const int32_t* h_items;
  int32_t* h_active;
  double* h_kid;
  int32_t h0, h1;
  int32_t blk[8];
};
constexpr int kGroupSlots = 2048;  // LDS slots of one workgroup: the largest GPB * 2^LG of bins 0-4, bin 5's table
static_assert(kBinLanes[5] == kBlock, "bin 5: one workgroup per vertex");

// Body of one workgroup of bin (G, LG): workgroup `bid` of `nb` strides over
// the bin's vertices; skeys / svals: the workgroup's kGroupSlots LDS slots.
template <int G, int LG, int BMAX, class WT, int PH, bool DET>
__device__ __forceinline__ void decide_group_body(const GraphView<WT>& g, const ScanArgs& a,
                                                  const int32_t* __restrict__ list, int32_t count, int32_t bid,
                                                  int32_t nb, int32_t* skeys, double* svals) {
  constexpr int TS = 1 << LG;
  constexpr int GPB = kBlock / G;
  static_assert(GPB * TS <= kGroupSlots, "group tables fit the workgroup's LDS");
  const int gl = threadIdx.x % G;
  const int gb = threadIdx.x / G;
  int32_t* keys = skeys + gb * TS;
  double* vals = svals + gb * TS;
  for (int s = gl; s < TS; s += G) { keys[s] = kEmpty; vals[s] = 0.0; }
  wave_sync();
  Acc acc;
  const bool sync = DET || (a.sync_moves & 1);
  const int32_t it = launch_iteration<PH>(a, sync);
  // rows software pipelined as in decide_block_body: a row's state is loaded
  // while the row before it is scanned, its list entry one row earlier
  const int64_t step = (int64_t)nb * GPB;
  const int64_t v0 = (int64_t)bid * GPB + gb;
  int32_t i_next = 0, i_after = 0;
  RowState nx;
  if (v0 < count) {
    i_next = list[v0];
    if (v0 + step < count) i_after = list[v0 + step];
    nx = load_row_state<PH>(g, a, i_next);
  }
  for (int64_t v = v0; v < count; v += step) {
    const int32_t i = i_next;
    const RowState cur = nx;
    if (v + step < count) nx = load_row_state<PH>(g, a, i_after);
    i_next = i_after;
    if (v + 2 * step < count) i_after = list[v + 2 * step];
    const int32_t beg = cur.beg, deg = cur.deg, bi = cur.bi, d = cur.d;
    const double ki = cur.ki;
    // One lane decides on the (possibly concurrently updated) eligibility state.
    int ok = (gl == 0) ? (int)row_eligible<PH>(a, cur, i, sync) : 0;
    ok = __shfl(ok, 0, G);
    if (!ok) continue;
    if (PH == kMove && gl == 0) a.flag[i] = 0;  // processed (Alg. 2 prune)
    // and those that need d, before the scan's
    const double sd = a.Sig[d];
    const Pre pre = prefetch_state<PH>(a, i, d, sync, it);
    // table of next_pow2(2 deg) <= TS slots: at most deg distinct keys
    const int lg = min(LG, ceil_log2(2 * (int64_t)deg));
    const int ts = 1 << lg;
    constexpr int UA = (BMAX + G - 1) / G;  // (one round: the row's arcs gl, gl + G, ... stay in registers)
    // labels of the lane's arcs gl + u G (kEmpty past the row: a lane whose
    // first arc lies past it sees none), kept for the swap-rule candidate test
    int32_t rc[UA], rj[UA];  // (rj: the neighbour ids, set wherever rc is)
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      rc[u] = kEmpty;
      rj[u] = i;
    }
    double kid = scan_row<UA, G, PH>(
        g, a, i, beg, deg, gl, d, bi, [&](int32_t c, double w) { lds_insert(keys, vals, lg, c, w); },
        [&](int u, int32_t j, int32_t c) {
          rc[u] = c;
          rj[u] = j;
        });
    kid = sum_xor<G>(kid);
    wave_sync();
    const Eval<DET> ev(a, i, kid, ki, sd);
    int32_t bc = -1;
    double bg = 0.0;
    i128 bk = 0;
    eval_table<(TS / G > 2 ? 2 : TS / G), G, DET>(keys, vals, ts, gl, a, ev, acc, bg, bk, bc);
    if (DET) argmax_k<G>(bk, bc); else argmax_f<G>(bg, bc);
    wave_sync();
    if (gl == 0) { ++acc.nv; acc.na += (unsigned long long)deg; }
    int take = (gl == 0) ? (int)accept_pre<PH, DET>(a, pre, d, bc, bg, bk, sync) : 0;
    take = __shfl(take, 0, G);
    if (!take) continue;
    if (PH == kMove && !DET && !(a.sync_moves & 1)) {
      if (gl == 0) {
        atomicAdd(&a.Sig[d], -ki);
        atomicAdd(&a.Sig[bc], ki);
        atomicSub(&a.size[d], 1);
        atomicAdd(&a.size[bc], 1);
        a.C[i] = bc;
        add_gain<DET>(a, acc, i, bg, bk);
        ++acc.nm;
      }
      mark_row(g, a, i, beg, deg, gl, G, false);
    } else if (PH == kMove) {
      // swap-rule candidate if the target holds a neighbour of the group:
      // its move record names that neighbour (-2: several)
      const int32_t vb = a.gid ? a.vbase[a.gid[i]] : 0;
      const int sh = (a.gid && a.gsh) ? a.gsh[a.gid[i]] : 0;
      int np = 0, pj = -1;
#pragma unroll
      for (int u = 0; u < UA; ++u)
        if (rc[u] == bc) {  // (bc is not the own community, so the arc is not a self-loop)
          const int32_t j = rj[u];
          if (group_in_pass(a, j, vb, sh) == a.grp) {
            ++np;
            pj = j;
          }
        }
      np = sum_lanes<G>(np);
      pj = max_lanes<G>(pj);
      if (gl == 0) {
        add_gain<DET>(a, acc, i, bg, bk);
        if (np > 0) {
          a.target[i] = -2 - bc;
          store_gain<DET>(a, i, bg, bk);
          record_move(a, i, d, bc, np == 1 ? pj : -2);
        } else {
          a.target[i] = bc;
        }
      }
    } else {
      if (gl == 0) { a.target[i] = bc; a.targeted[bc] = cur_stamp(a); }
    }
  }
  flush_acc<PH, DET>(a, acc);
}

// ------------------------------------------------ one workgroup per vertex ---
// Body of one workgroup of bin 5: workgroup `bid` of `nb` strides over the
// bin's vertices with an LDS table of 2^LG slots (keys, vals).
template <int LG, class WT, int PH, bool DET>
__device__ __forceinline__ void decide_block_body(const GraphView<WT>& g, const ScanArgs& a,
                                                  const int32_t* __restrict__ list, int32_t count, int32_t bid,
                                                  int32_t nb, int32_t* keys, double* vals) {
  constexpr int TS = 1 << LG;
  __shared__ double s_g[kBlock / kWave];
  __shared__ i128 s_k[kBlock / kWave];
  __shared__ int32_t s_c[kBlock / kWave];
  __shared__ int s_flag, s_take;
  for (int s = threadIdx.x; s < TS; s += kBlock) { keys[s] = kEmpty; vals[s] = 0.0; }
  __syncthreads();
  Acc acc;
  const bool sync = DET || (a.sync_moves & 2);
  const int32_t it = launch_iteration<PH>(a, sync);
  // stable: while this launch runs, nothing else writes a row's flag, the
  // community sizes or the last-move entries (refinement and synchronous
  // local-moving only record targets), so every thread reaches the
  // eligibility and acceptance decisions from its own loads and no thread
  // has to publish them.  The row's own flag is cleared once every
  // wavefront has read it.
  const bool stable = PH == kRefine || sync;
  // The workgroup's rows v = bid + r nb are software
  // pipelined: a row's own state is loaded while the row before it is
  // scanned, and its list entry one row earlier still, so that neither
  // sits on the path from one row's scan to the next.
  const int64_t step = nb;
  int32_t i_next = 0, i_after = 0;
  RowState nx;
  if ((int64_t)bid < count) {
    i_next = list[bid];
    if ((int64_t)bid + step < count) i_after = list[bid + step];
    nx = load_row_state<PH>(g, a, i_next);
  }
  for (int64_t v = bid; v < count; v += step) {
    const int32_t i = i_next;
    const RowState cur = nx;
    if (v + step < count) nx = load_row_state<PH>(g, a, i_after);
    i_next = i_after;
    if (v + 2 * step < count) i_after = list[v + 2 * step];
    const int32_t beg = cur.beg, deg = cur.deg, bi = cur.bi, d = cur.d;
    const double ki = cur.ki;
    int ok;
    if (stable) {
      ok = (int)row_eligible<PH>(a, cur, i, sync);
    } else {
      if (threadIdx.x == 0) s_flag = (int)row_eligible<PH>(a, cur, i, sync);
      __syncthreads();
      ok = s_flag;
      __syncthreads();
    }
    if (!ok) continue;  // uniform over the workgroup
    if (PH == kMove && !stable && threadIdx.x == 0) a.flag[i] = 0;  // processed (Alg. 2 prune)
    const int lg = min(LG, ceil_log2(2 * (int64_t)deg));
    const int ts = 1 << lg;
    // and those that need d, before the scan's
    const double sd = a.Sig[d];
    Pre pre;
    if (stable || threadIdx.x == 0) pre = prefetch_state<PH>(a, i, d, sync, it);
    double kid = scan_row<4, kBlock, PH>(g, a, i, beg, deg, threadIdx.x, d, bi, [&](int32_t c, double w) {
      lds_insert(keys, vals, lg, c, w);
    });
    kid = block_allsum<double>(kid, s_g);
    // Every wavefront has read this row's flag by now (it decided on it).
    if (PH == kMove && stable && threadIdx.x == 0) a.flag[i] = 0;
    const Eval<DET> ev(a, i, kid, ki, sd);
    int32_t bc = -1;
    double bg = 0.0;
    i128 bk = 0;
    eval_table<(TS / kBlock > 4 ? 4 : TS / kBlock), kBlock, DET>(keys, vals, ts, threadIdx.x, a, ev, acc, bg, bk,
                                                                 bc);
    block_argmax<DET>(bg, bk, bc, s_g, s_k, s_c);
    if (threadIdx.x == 0) {
      ++acc.nv;
      acc.na += (unsigned long long)deg;
    }
    int take;
    if (stable) {
      take = (int)accept_pre<PH, DET>(a, pre, d, bc, bg, bk, sync);
    } else {
      if (threadIdx.x == 0) s_take = (int)accept_pre<PH, DET>(a, pre, d, bc, bg, bk, sync);
      __syncthreads();  // s_take published
      take = s_take;
    }
    if (!take) continue;
    if (PH == kMove && !DET && !(a.sync_moves & 2)) {
      if (threadIdx.x == 0) {
        atomicAdd(&a.Sig[d], -ki);
        atomicAdd(&a.Sig[bc], ki);
        atomicSub(&a.size[d], 1);
        atomicAdd(&a.size[bc], 1);
        a.C[i] = bc;
        add_gain<DET>(a, acc, i, bg, bk);
        ++acc.nm;
      }
      mark_row(g, a, i, beg, deg, threadIdx.x, kBlock, false);
    } else if (PH == kMove) {
      if (threadIdx.x == 0) {
        add_gain<DET>(a, acc, i, bg, bk);
        if (deg <= kSwapRowMax) {  // (only with a tuned lane-group limit below kSwapRowMax) a candidate
          a.target[i] = -2 - bc;
          store_gain<DET>(a, i, bg, bk);
          record_move(a, i, d, bc, -2);
        } else {  // a possible partner
          a.target[i] = bc;
          record_move(a, i, d, bc, -1);
        }
      }
    } else {
      if (threadIdx.x == 0) { a.target[i] = bc; a.targeted[bc] = cur_stamp(a); }
    }
  }
  flush_acc<PH, DET>(a, acc);
}

// Eligibility snapshot of hubs p = t0, t0 + stride, ... < h1 of a group,
// taken before any of their chunks is gathered: active[p], K_{i->d} and the
// target reset (a synchronous local-moving commit applies a hub's target
// without forgetting it), the pruning flag cleared (Alg. 2).
template <int PH, bool DET>
__device__ __forceinline__ void hub_prep_body(const ScanArgs& a, const GroupLaunch& gl, int64_t t0, int64_t stride) {
  for (int64_t p = t0; p < gl.h1; p += stride) {
    const int32_t i = gl.h_items[p];
    const bool act = Decide<PH, DET>::eligible(a, i);
    gl.h_active[p] = act ? 1 : 0;
    gl.h_kid[p] = 0.0;
    a.target[i] = -1;
    if (PH == kMove && act) a.flag[i] = 0;  // processed (Alg. 2 prune)
  }
}

// The short-row decisions of a group: bins 0-5 in one launch, so the rows of
// bin 5 fill the CUs that the lane-group bins leave as they finish; the
// last blocks take the group's hub snapshot (the hub kernels follow on the
// same stream).
template <class WT, int PH, bool DET>
__global__ __launch_bounds__(kBlock) void k_decide_groups(GraphView<WT> g, ScanArgs a,
                                                          const int32_t* __restrict__ list, GroupLaunch gl) {
  __shared__ int32_t skeys[kGroupSlots];
  __shared__ double svals[kGroupSlots];
  int b = 0;
  while (b < 6 && (int32_t)blockIdx.x >= gl.blk[b + 1]) ++b;  // uniform over the workgroup
  const int32_t bid = (int32_t)blockIdx.x - gl.blk[b], nb = gl.blk[b + 1] - gl.blk[b];
  const int32_t* l = list + (b < 6 ? gl.start[b] : 0);
  switch (b) {
    case 0: decide_group_body<kBinLanes[0], 3, kBinMax[0], WT, PH, DET>(g, a, l, gl.count[0], bid, nb, skeys, svals); break;
    case 1: decide_group_body<kBinLanes[1], 4, kBinMax[1], WT, PH, DET>(g, a, l, gl.count[1], bid, nb, skeys, svals); break;
    case 2: decide_group_body<kBinLanes[2], 5, kBinMax[2], WT, PH, DET>(g, a, l, gl.count[2], bid, nb, skeys, svals); break;
    case 3: decide_group_body<kBinLanes[3], 6, kBinMax[3], WT, PH, DET>(g, a, l, gl.count[3], bid, nb, skeys, svals); break;
    case 4: decide_group_body<kBinLanes[4], 8, kBinMax[4], WT, PH, DET>(g, a, l, gl.count[4], bid, nb, skeys, svals); break;
    case 5: decide_block_body<11, WT, PH, DET>(g, a, l, gl.count[5], bid, nb, skeys, svals); break;
    default:
      hub_prep_body<PH, DET>(a, gl, (int64_t)gl.h0 + (int64_t)bid * kBlock + threadIdx.x, (int64_t)nb * kBlock);
      break;
  }
}

// ------------------------------------ wide rows: P workgroups per vertex ---
// Vertices of the wide bins (kBinMax[5] < deg <= kBinMax[kHubBin - 1]).  The
// P = 2^kWideShift[k] workgroups of a vertex of wide class k each stream the
// whole row, but accumulate only the neighbour communities c with
// wide_part(c) mod P equal to their partition, in an LDS table of up to
// kWideSlots slots, so no global table or global atomics are needed.  Rows
// of up to 8192 arcs fit one table (P = 1, load factor <= 2/3) and are read
// once.  K_{i->d} is a plain sum over the row.  Every partition evaluates
// its own candidates; the last one to finish reduces the partial bests and
// applies the decision.  Only partition 0 tests (and, for local-moving,
// clears) the pruning flag: the others scan regardless, and the decision
// follows partition 0.  A partition whose keys overflow the table (more than
// kWideSlots distinct; statistically out of reach for rows of at most 8192 P
// arcs, but ids can be chosen to put every neighbour into one partition)
// cancels the move of its vertex and is counted in *a.ovf.
constexpr int kWideThreads = 1024;
constexpr int64_t kWideGrid = 256;  // persistent workgroups: one per CU (the LDS table fits once)
static_assert(kWideSlots % kWideThreads == 0, "wide table: whole slots per thread");

struct WideLaunch {
  int32_t count[kWideClasses];  // vertices of class k in this launch
  int32_t start[kWideClasses];  // their offset in the list
  int32_t tasks;                // sum of count[k] << k
};

template <class WT, int PH, bool DET>
__global__ __launch_bounds__(kWideThreads) void k_decide_wide(GraphView<WT> g, ScanArgs a,
                                                              const int32_t* __restrict__ list, WideLaunch wl) {
  constexpr int TS = kWideSlots;
  constexpr int NW = kWideThreads / kWave;
  __shared__ int32_t keys[TS];
  __shared__ double vals[TS];
  __shared__ double s_g[NW];
  __shared__ i128 s_k[NW];
  __shared__ int32_t s_c[NW];
  __shared__ double s_d[NW];
  __shared__ int s_ok, s_ovf, s_last, s_take, s_task;
  // the table starts empty; every task leaves it empty (eval_table clears
  // what it reads, and nothing is inserted for a skipped vertex)
  for (int s = threadIdx.x; s < TS; s += kWideThreads) { keys[s] = kEmpty; vals[s] = 0.0; }
  Acc acc;
  const bool sync = DET || (a.sync_moves & 2);
  const int32_t it = launch_iteration<PH>(a, sync);
  // persistent workgroups take tasks from a counter, so a vertex that is
  // skipped (not flagged, not isolated) costs a few loads, not a dispatch
  // stable: as in decide_block_body (every thread decides eligibility
  // itself; the flag is cleared once every wavefront has read it).
  const bool stable = PH == kRefine || sync;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      s_task = atomicAdd(a.wd_next, 1);
      s_ovf = 0;
    }
    __syncthreads();
    int32_t b = s_task;
    if (b >= wl.tasks) break;  // uniform
    // task -> (class k, vertex r of the launch, partition)
    int32_t r = 0;
    int k = 0;
    for (; k < kWideClasses - 1; ++k) {
      const int32_t tk = wl.count[k] << kWideShift[k];
      if (b < tk) break;
      b -= tk;
      r += wl.count[k];
    }
    const int sh = kWideShift[k];
    const int P = 1 << sh;
    const int32_t vloc = b >> sh;
    const int part = b & (P - 1);
    r += vloc;
    const int32_t i = list[wl.start[k] + vloc];
    // the loads that need only i go out together with the eligibility test
    const int32_t beg = g.begin(i), deg = g.degree(i);
    const int32_t d = a.C[i];
    const double ki = a.K[i];
    // P == 1: 2 deg slots (whole multiples of the workgroup), at most TS
    int ts = TS;
    if (P == 1) {
      const int64_t want = ((2 * (int64_t)deg + kWideThreads - 1) / kWideThreads) * kWideThreads;
      if (want < ts) ts = (int)want;
    }
    int ok;
    if (stable) {
      ok = (part == 0 || PH == kRefine) ? (int)Decide<PH, DET>::eligible(a, i) : 1;
    } else {
      if (threadIdx.x == 0) {
        int o = 1;
        if (part == 0 || PH == kRefine) o = (int)Decide<PH, DET>::eligible(a, i);
        if (PH == kMove && part == 0 && o) a.flag[i] = 0;  // processed (Alg. 2 prune)
        s_ok = o;
      }
      __syncthreads();
      ok = s_ok;
    }
    if (!ok && P == 1) continue;  // uniform: nothing to decide, nothing to combine
    int32_t bc = -1;
    double bg = 0.0;
    i128 bk = 0;
    Pre pre;
    if (ok) {  // uniform
      // the loads that need d, before the scan's
      const double sd = a.Sig[d];
      if (threadIdx.x == 0) pre = prefetch_state<PH>(a, i, d, sync, it);
      const int32_t bi = (PH == kRefine) ? a.CB[i] : 0;
      double kid = scan_row<4, kWideThreads, PH>(g, a, i, beg, deg, threadIdx.x, d, bi, [&](int32_t c, double w) {
        if ((int)(wide_part(c) & (uint32_t)(P - 1)) != part) return;
        if (!lds_insert_sized(keys, vals, (uint32_t)ts, c, w)) s_ovf = 1;
      });
      kid = block_allsum<double>(kid, s_d);
      if (PH == kMove && stable && part == 0 && threadIdx.x == 0) a.flag[i] = 0;  // processed (Alg. 2 prune)
      const Eval<DET> ev(a, i, kid, ki, sd);
      eval_table<TS / kWideThreads / 2, kWideThreads, DET>(keys, vals, ts, threadIdx.x, a, ev, acc, bg, bk, bc);
      block_argmax<DET, NW>(bg, bk, bc, s_g, s_k, s_c);
    }
    const int ovf = s_ovf;
    int last = 1;
    if (P > 1) {
      if (threadIdx.x == 0) {
        const int64_t q = (int64_t)r * kWideMaxParts + part;
        a.wd_g[q] = bg;
        a.wd_k[q] = bk;
        a.wd_c[q] = bc;
        a.wd_ok[q] = ok | (ovf << 1);
        __threadfence();
        const int prev = atomicAdd(&a.wd_done[r], 1);
        s_last = (prev == P - 1) ? 1 : 0;
      }
      __syncthreads();
      last = s_last;
    }
    if (!last) continue;  // uniform
    int ok0 = ok, ovf_any = ovf;
    if (P > 1) {
      __threadfence();
      if (threadIdx.x == 0) {
        bc = -1; bg = 0.0; bk = 0;
        for (int q2 = 0; q2 < P; ++q2) {
          const int64_t q = (int64_t)r * kWideMaxParts + q2;
          const int f = __hip_atomic_load(a.wd_ok + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (q2 == 0) ok0 = f & 1;
          ovf_any |= (f >> 1) & 1;
          const int32_t c2 = __hip_atomic_load(a.wd_c + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (DET) {
            const unsigned long long* kw = (const unsigned long long*)(a.wd_k + q);
            const unsigned long long lo = __hip_atomic_load(kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long hi = __hip_atomic_load(kw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const i128 k2 = make_i128((long long)hi, lo);
            if (better_k(k2, c2, bk, bc)) { bk = k2; bc = c2; }
          } else {
            const double g2 = __hip_atomic_load(a.wd_g + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (better_f(g2, c2, bg, bc)) { bg = g2; bc = c2; }
          }
        }
        a.wd_done[r] = 0;
      }
    }
    if (threadIdx.x == 0) {
      int take = 0;
      if (ok0) {
        ++acc.nv;
        acc.na += (unsigned long long)deg;
        if (ovf_any) atomicAdd(a.ovf, 1ull);
        // (with ok0 set, the last partition scanned and loaded pre too)
        take = (!ovf_any && accept_pre<PH, DET>(a, pre, d, bc, bg, bk, sync)) ? 1 : 0;
      }
      if (take) {
        if (PH == kMove && !DET && !(a.sync_moves & 2)) {
          atomicAdd(&a.Sig[d], -ki);
          atomicAdd(&a.Sig[bc], ki);
          atomicSub(&a.size[d], 1);
          atomicAdd(&a.size[bc], 1);
          a.C[i] = bc;
          add_gain<DET>(a, acc, i, bg, bk);
          ++acc.nm;
        } else if (PH == kMove) {
          a.target[i] = bc;
          add_gain<DET>(a, acc, i, bg, bk);
          record_move(a, i, d, bc, -1);
        } else {
          a.target[i] = bc;
          a.targeted[bc] = cur_stamp(a);
        }
      }
      s_take = take;
    }
    if (!stable) {
      __syncthreads();
      if (PH == kMove && s_take) mark_row(g, a, i, beg, deg, threadIdx.x, kWideThreads, false);
    }
  }
  // the last workgroup out resets the task counter for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(a.wd_exit, 1) == (int)gridDim.x - 1) {
      *a.wd_next = 0;
      *a.wd_exit = 0;
    }
  }
  flush_acc<PH, DET>(a, acc);
}

// ------------------------------------------------------------- commit ---
// Applies the recorded synchronous decisions of the vertices list[0..count)
// (one group); the community totals go through the workgroup-combined
// table.  Refinement: vertex i moves only if its own community was not
// chosen as a target in this group.  Local-moving with MARK: every recorded
// move applies, the target is forgotten and the neighbours of movers are
// marked unprocessed; the workgroup lays its movers' rows end to end and
// every lane marks one arc per step.  Without MARK (long rows, hubs) the
// targets stay for the marking kernels.
// An applied local-moving move of vertex i out of community d: its record
// for the bounce rule.  A move that yields under the swap rule (rare) takes
// its gain back out of the iteration's sum with one atomic (per graph in a
// fused batch).
__device__ __forceinline__ void note_move(const ScanArgs& a, int32_t i, int32_t d) {
  const int2 l = a.last[i];
  a.last[i] = make_int2(d, (int32_t)(((uint32_t)l.y << 16) | ((uint32_t)*a.it_dev & 0xFFFFu)));
}
__device__ __forceinline__ void untake_gain(const ScanArgs& a, int32_t i) {
  if (a.gaink) {
    const i128 k = -a.gaink[i];
    atomic_add_i128(a.gid ? a.dqg128 + 2 * a.gid[i] : a.dq128 + 2 * cslot(), k);
  } else {
    const double x = -a.gainf[i];
    atomicAdd(a.gid ? a.dqg + a.gid[i] : a.dq + cslot(), x);
  }
}

// Swap rule of the synchronous local-moving, in the commit of a group: a
// recorded move of vertex i (community d, target t) of a row of at most
// kSwapRowMax arcs yields if an adjacent vertex j of the same group chose d
// while in t (its move record of this iteration and group), and j has the
// lower id or more than kSwapRowMax arcs (such rows never yield).  Two such
// vertices would trade places and trade back in the next iteration.  The
// records are written by the decisions only, so the answer does not depend
// on which moves of the group were applied before.  Only candidates (their
// target holds a neighbour of the group; target stored as -2 - t) can have
// such a partner.
template <class WT>
__device__ __forceinline__ bool swap_yields(const GraphView<WT>& g, const ScanArgs& a, int32_t i, int32_t d,
                                            int32_t t) {
  const int32_t stamp = move_stamp(a);
  const int4 own = a.mv[i];
  if (own.z != stamp || own.w == -1) return false;
  if (own.w >= 0) {  // the one neighbour of the group in the target
    const int32_t j = own.w;
    if ((int64_t)j >= g.n) return false;
    const int4 r = a.mv[j];
    return r.z == stamp && r.x == t && r.y == d && (j < i || g.degree(j) > kSwapRowMax);
  }
  const int32_t beg = g.begin(i), deg = g.degree(i);
  const int32_t vb = a.gid ? a.vbase[a.gid[i]] : 0;
  const int sh = (a.gid && a.gsh) ? a.gsh[a.gid[i]] : 0;
  // four arcs per step: their ids, then their records (a lane without a
  // same-group neighbour reads its own record), each batch in flight
  // together; a row walked one arc at a time (two dependent loads per arc)
  // could hold up a whole commit launch
  constexpr int U = 4;
  for (int32_t e0 = 0; e0 < deg; e0 += U) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = g.idx[beg + min(e0 + u, deg - 1)];
    bool same[U];
    int4 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      same[u] = e0 + u < deg && j[u] != i && group_in_pass(a, j[u], vb, sh) == a.grp;
      r[u] = a.mv[same[u] ? j[u] : i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (same[u] && r[u].z == stamp && r[u].x == t && r[u].y == d && (j[u] < i || g.degree(j[u]) > kSwapRowMax))
        return true;
  }
  return false;
}

// Shared memory of the commit roles.
struct CommitLds {
  KeyedLds<kBlock> kt;
  int32_t off[kBlock + 1], beg[kBlock], vi[kBlock];
  int32_t w[kBlock / kWave];
  int mv;
};

// Tiles of kBlock entries of list[0..count): workgroup `bid` of `nb`.
template <class WT, int PH, bool MARK>
__device__ __forceinline__ unsigned long long commit_tiles(const GraphView<WT>& g, const ScanArgs& a,
                                                           const int32_t* __restrict__ list, int32_t count,
                                                           int32_t bid, int32_t nb, CommitLds& L) {
  unsigned long long nm = 0;
  for (int64_t base = (int64_t)bid * kBlock; base < count; base += (int64_t)nb * kBlock) {
    const int64_t k = base + threadIdx.x;
    const int32_t i = (k < count) ? list[k] : 0;
    int32_t t = -1;
    if (k < count) t = a.target[i];
    const bool cand = PH == kMove && MARK && t <= -2;
    if (cand) t = -2 - t;
    bool mv = t >= 0;
    if (mv) {
      const int32_t d = a.C[i];
      if (PH == kMove && MARK) {
        a.target[i] = -1;
        if (cand && swap_yields(g, a, i, d, t)) {  // the neighbour takes this vertex's place
          mv = false;
          untake_gain(a, i);
        }
      }
      if (PH == kRefine) {
        a.target[i] = -1;
        if (a.targeted[d] == cur_stamp(a)) mv = false;  // own community chosen by this group
      }
      if (mv) {
        const double ki = a.K[i];
        keyed_put(L.kt, d, -ki, -1);
        keyed_put(L.kt, t, ki, 1);
        a.C[i] = t;
        if (PH == kRefine && a.CP) a.CP[i].x = t;
        if (PH == kMove) note_move(a, i, d);
        ++nm;
        if (PH == kRefine && a.gid) atomicAdd(&a.mvg[a.gid[i]], 1ull);
      }
    }
    keyed_flush(L.kt, a.Sig, a.size);
    if (PH == kMove && MARK) {  // uniform: the tile's movers' rows end to end
      const int32_t deg = mv ? g.degree(i) : 0;
      int incl = deg;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int x = __shfl_up(incl, o);
        if (lane_id() >= o) incl += x;
      }
      const int w = threadIdx.x / kWave;
      if (lane_id() == kWave - 1) L.w[w] = incl;
      __syncthreads();
      int before = 0, total = 0;
      for (int q = 0; q < kBlock / kWave; ++q) {
        if (q < w) before += L.w[q];
        total += L.w[q];
      }
      L.off[threadIdx.x] = before + incl - deg;
      if (threadIdx.x == 0) L.off[kBlock] = total;
      L.beg[threadIdx.x] = mv ? g.begin(i) : 0;
      L.vi[threadIdx.x] = i;
      __syncthreads();
      for (int32_t q0 = threadIdx.x; q0 < total; q0 += kMarkUnroll * kBlock) {  // (as mark_row)
        int32_t j[kMarkUnroll], v[kMarkUnroll];
#pragma unroll
        for (int u = 0; u < kMarkUnroll; ++u) {
          const int32_t q = q0 + u * kBlock;
          j[u] = 0;
          v[u] = 0;  // (j == v: no mark)
          if (q < total) {
            int lo = 0, hi = kBlock;  // off[lo] <= q < off[hi]
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (L.off[mid] <= q) lo = mid; else hi = mid;
            }
            j[u] = g.idx[(int64_t)L.beg[lo] + (q - L.off[lo])];
            v[u] = L.vi[lo];
          }
        }
        uint8_t f[kMarkUnroll];
#pragma unroll
        for (int u = 0; u < kMarkUnroll; ++u) f[u] = (j[u] != v[u] && mark_needed(a, j[u])) ? a.flag[j[u]] : 1;
#pragma unroll
        for (int u = 0; u < kMarkUnroll; ++u)
          if (f[u] == 0) a.flag[j[u]] = 1;
      }
      __syncthreads();  // L.* are rewritten by the next entries
    }
  }
  return nm;
}

// Long rows: one workgroup per entry applies the move, forgets the target
// and marks the mover's neighbours with all its threads.
template <class WT>
__device__ __forceinline__ unsigned long long commit_long(const GraphView<WT>& g, const ScanArgs& a,
                                                          const int32_t* __restrict__ list, int32_t count,
                                                          int32_t bid, int32_t nb, CommitLds& L) {
  unsigned long long nm = 0;
  for (int64_t k = bid; k < count; k += nb) {
    const int32_t i = list[k];
    if (threadIdx.x == 0) {
      int32_t t = a.target[i];
      const bool cand = t <= -2;  // (rows of bin 5 up to kSwapRowMax arcs, with a tuned lane-group limit)
      if (cand) t = -2 - t;
      L.mv = t >= 0;
      if (t >= 0) {
        a.target[i] = -1;
        const int32_t d = a.C[i];
        if (cand && swap_yields(g, a, i, d, t)) {
          L.mv = 0;
          untake_gain(a, i);
        } else {
          const double ki = a.K[i];
          atomicAdd(&a.Sig[d], -ki);
          atomicAdd(&a.Sig[t], ki);
          atomicSub(&a.size[d], 1);
          atomicAdd(&a.size[t], 1);
          a.C[i] = t;
          note_move(a, i, d);
          ++nm;
        }
      }
    }
    __syncthreads();
    if (L.mv) mark_row(g, a, i, g.begin(i), g.degree(i), threadIdx.x, kBlock, true);
    __syncthreads();
  }
  return nm;
}

// Applies the recorded synchronous decisions of one group (CommitLaunch).
template <class WT, int PH>
__global__ __launch_bounds__(kBlock) void k_commit(GraphView<WT> g, ScanArgs a, CommitLaunch cl) {
  __shared__ CommitLds L;
  __shared__ unsigned long long red_u[16];
  keyed_clear(L.kt);
  const int32_t x = (int32_t)blockIdx.x;
  int r = 0;
  while (r < 3 && x >= cl.b[r + 1]) ++r;  // uniform over the workgroup
  const int32_t bid = x - cl.b[r], nb = cl.b[r + 1] - cl.b[r];
  unsigned long long nm = 0;
  if (PH == kRefine) {
    if (r == 0) nm = commit_tiles<WT, kRefine, false>(g, a, cl.l0, cl.n0, bid, nb, L);
    else nm = commit_tiles<WT, kRefine, false>(g, a, cl.l2, cl.n2, bid, nb, L);
  } else if (r == 0) {
    nm = commit_tiles<WT, kMove, true>(g, a, cl.l0, cl.n0, bid, nb, L);
  } else if (r == 1) {
    nm = commit_long<WT>(g, a, cl.l1, cl.n1, bid, nb, L);
  } else if (r == 2) {
    nm = commit_tiles<WT, kMove, false>(g, a, cl.l2, cl.n2, bid, nb, L);
  } else {
    for (int64_t t = cl.c0 + (int64_t)bid; t < cl.c1; t += nb) {
      const int2 task = cl.chunk_tasks[t];
      const int32_t i = cl.hub_items[task.x];
      if (a.target[i] < 0) continue;  // uniform: no move
      const int32_t beg = g.begin(i), deg = g.degree(i);
      const int32_t e0 = task.y * kHubChunk;
      const int32_t e1 = (deg - e0 < kHubChunk) ? deg : e0 + kHubChunk;
      mark_row(g, a, i, beg + e0, e1 - e0, threadIdx.x, kBlock, true);
    }
  }
  nm = block_sum<unsigned long long>(nm, red_u);
  if (threadIdx.x == 0 && nm) atomicAdd(&cnt_of(a.cnt)[3], nm);
}

// ------------------------------------------------------------- launchers ---
template <class WT>
inline GraphView<WT> view(const GraphDesc& g) {
  GraphView<WT> v;
  v.n = g.n; v.off = g.off; v.deg = g.deg; v.idx = g.idx; v.w = (const WT*)g.w;
  return v;
}

inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

template <class WT, int PH, bool DET>
void decide_bins(hipStream_t st, const GraphDesc& gd, const ScanArgs& a, const int32_t* list,
                 const int32_t* count, const int32_t* start, int grid_cap, const HubArgs& h, int32_t h0, int32_t h1,
                 int64_t* launches) {
  const GraphView<WT> g = view<WT>(gd);
  {  // bins 0-5 and the hub snapshot: one launch
    GroupLaunch gl;
    gl.blk[0] = 0;
    for (int b = 0; b < 6; ++b) {
      gl.count[b] = count[b];
      gl.start[b] = start[b];
      gl.blk[b + 1] = gl.blk[b] + (count[b] > 0 ? grid_for(count[b], kBlock / kBinLanes[b], grid_cap) : 0);
    }
    gl.h_items = h.items;
    gl.h_active = h.active;
    gl.h_kid = h.kid;
    gl.h0 = h0;
    gl.h1 = h1;
    gl.blk[7] = gl.blk[6] + (h1 > h0 ? grid_for(h1 - h0, kBlock, 1024) : 0);
    if (gl.blk[7] > 0) {
      hipLaunchKernelGGL((k_decide_groups<WT, PH, DET>), dim3(gl.blk[7]), dim3(kBlock), 0, st, g, a, list, gl);
      ++*launches;
    }
  }
  WideLaunch wl;
  int64_t tasks = 0;
  for (int k = 0; k < kWideClasses; ++k) {
    wl.count[k] = count[kWideBin0 + k];
    wl.start[k] = start[kWideBin0 + k];
    tasks += (int64_t)wl.count[k] << kWideShift[k];
  }
  if (tasks > 0) {
    wl.tasks = (int32_t)tasks;
    const unsigned grid = (unsigned)(tasks < kWideGrid ? tasks : kWideGrid);
    hipLaunchKernelGGL((k_decide_wide<WT, PH, DET>), dim3(grid), dim3(kWideThreads), 0, st, g, a, list, wl);
    ++*launches;
  }
}

// One launch for the commits of a group (see k_commit).
template <class WT, int PH>
void commit_group_launch(hipStream_t st, const GraphDesc& gd, const ScanArgs& a, const HubArgs& h,
                         CommitLaunch cl) {
  const GraphView<WT> g = view<WT>(gd);
  int32_t nblk[4];
  const int cap = a.commit_grid > 0 ? a.commit_grid : 2048;
  if (PH == kRefine) {
    nblk[0] = cl.n0 > 0 ? grid_for(cl.n0, kBlock, cap) : 0;
    nblk[1] = cl.n2 > 0 ? grid_for(cl.n2, kBlock, cap) : 0;
    nblk[2] = nblk[3] = 0;
  } else {
    nblk[0] = cl.n0 > 0 ? grid_for(cl.n0, kBlock, cap) : 0;
    nblk[1] = cl.n1 > 0 ? grid_for(cl.n1, 1, 4 * cap) : 0;
    nblk[2] = cl.n2 > 0 ? grid_for(cl.n2, kBlock, 64) : 0;
    nblk[3] = cl.c1 > cl.c0 ? grid_for(cl.c1 - cl.c0, 1, 4096) : 0;
  }
  cl.chunk_tasks = h.chunk_tasks;
  cl.hub_items = h.items;
  cl.b[0] = 0;
  for (int r = 0; r < 4; ++r) cl.b[r + 1] = cl.b[r] + nblk[r];
  if (cl.b[4] > 0)
    hipLaunchKernelGGL((k_commit<WT, PH>), dim3(cl.b[4]), dim3(kBlock), 0, st, g, a, cl);
}

}  // namespace gvl
