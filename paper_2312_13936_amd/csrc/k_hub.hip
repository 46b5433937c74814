// Hub path of the neighbour-community scan (Alg. 2 / Alg. 3) and of the
// aggregation rows (Alg. 4) for items with very long rows: R-MAT hubs reach
// hundreds of thousands of arcs, and a single workgroup per hub would leave
// the GPU idle behind them.
//
// Every item's arcs are cut into chunks of kHubChunk, and one workgroup per
// chunk pre-aggregates the chunk in an LDS table.  Vertex hubs of up to
// kPartMaxDeg arcs and every giant community are split by key partitions:
// the chunk's distinct (community, weight) pairs are sorted by partition and
// staged at the chunk's arc positions, and one workgroup per partition sums
// its runs in LDS, then (scan) computes its best candidate (Eq. 2), the last
// partition to finish reducing the partial bests and applying the decision,
// or (aggregation) appends its entries to the super-vertex row.  Longer
// vertex hubs merge the chunks into a global table read back in slices.
#include "scan_kernels.hpp"

namespace gvl {

static inline int grid_items(int64_t n, int per, int cap) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

__device__ __forceinline__ int64_t table_slots(int64_t arcs, int64_t n) {
  int64_t x = arcs < n ? arcs : n;
  int64_t t = kTblUnit;
  while (t < 2 * x) t <<= 1;
  return t;
}

__device__ __forceinline__ TblSlot* tbl_of(const HubArgs& h, int32_t p) {
  return h.tbl + ((int64_t)h.tbl_off[p] * kTblUnit - h.tbase);
}
__device__ __forceinline__ int32_t* tbl_list_of(const HubArgs& h, int32_t p) {
  return h.tbl_list + ((int64_t)h.tbl_off[p] * kTblUnit - h.tbase);
}
__device__ __forceinline__ int tbl_lg(const HubArgs& h, int32_t p) {
  return ceil_log2((int64_t)(h.tbl_off[p + 1] - h.tbl_off[p]) * kTblUnit);
}

// ------------------------------------------------------------------ plan ---
__global__ void k_hub_setup(const int32_t* off, const int32_t* deg, const int32_t* items, int32_t H, int64_t n,
                            int32_t* chunk_off, int32_t* tbl_off, int32_t* slice_off) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < H; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = items[p];
    const int64_t d = deg ? deg[i] : off[i + 1] - off[i];
    chunk_off[p] = (int32_t)((d + kHubChunk - 1) / kHubChunk);
    if (hub_partitioned(d)) {  // no table; one task per key partition
      tbl_off[p] = 0;
      slice_off[p] = hub_parts(d);
    } else {
      const int64_t ts = table_slots(d, n);
      tbl_off[p] = (int32_t)(ts / kTblUnit);
      slice_off[p] = (int32_t)((ts + kHubSlice - 1) / kHubSlice);
    }
  }
}
void hub_setup(hipStream_t st, const int32_t* off, const int32_t* deg, const int32_t* items, int32_t H, int64_t n,
               int32_t* chunk_off, int32_t* tbl_off, int32_t* slice_off) {
  if (H > 0)
    hipLaunchKernelGGL(k_hub_setup, dim3(grid_items(H, kBlock, 4096)), dim3(kBlock), 0, st, off, deg, items, H, n,
                       chunk_off, tbl_off, slice_off);
}

__global__ void k_gagg_setup(const int32_t* yoff, const int32_t* items, int32_t H, int32_t* chunk_off,
                             int32_t* tbl_off, int32_t* slice_off) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < H; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = items[p];
    const int64_t cap = (int64_t)yoff[c + 1] - yoff[c];
    chunk_off[p] = (int32_t)((cap + kHubChunk - 1) / kHubChunk);
    tbl_off[p] = 0;  // no table; one task per key partition
    slice_off[p] = agg_parts(cap);
  }
}
void gagg_setup(hipStream_t st, const int32_t* yoff, const int32_t* items, int32_t H, int32_t* chunk_off,
                int32_t* tbl_off, int32_t* slice_off) {
  if (H > 0)
    hipLaunchKernelGGL(k_gagg_setup, dim3(grid_items(H, kBlock, 4096)), dim3(kBlock), 0, st, yoff, items, H,
                       chunk_off, tbl_off, slice_off);
}

// One workgroup per item writes its (item, chunk) and (item, slice) tasks.
__global__ void k_hub_tasks(int32_t H, const int32_t* chunk_off, const int32_t* slice_off, int2* chunk_tasks,
                            int2* slice_tasks) {
  for (int64_t p = blockIdx.x; p < H; p += gridDim.x) {
    const int32_t c0 = chunk_off[p], nc = chunk_off[p + 1] - c0;
    const int32_t s0 = slice_off[p], ns = slice_off[p + 1] - s0;
    for (int32_t c = threadIdx.x; c < nc; c += blockDim.x) chunk_tasks[c0 + c] = make_int2((int)p, c);
    for (int32_t c = threadIdx.x; c < ns; c += blockDim.x) slice_tasks[s0 + c] = make_int2((int)p, c);
  }
}
void hub_tasks(hipStream_t st, int32_t H, const int32_t* chunk_off, const int32_t* slice_off, int2* chunk_tasks,
               int2* slice_tasks) {
  if (H > 0)
    hipLaunchKernelGGL(k_hub_tasks, dim3(grid_items(H, 1, 4096)), dim3(kBlock), 0, st, H, chunk_off, slice_off,
                       chunk_tasks, slice_tasks);
}

// ------------------------------------------------------------------ scan ---
// Merge the LDS pre-aggregation table of one chunk into item p's global
// table; the slots of keys new to the global table are appended to p's
// occupied-slot list (one reservation per workgroup).  Leaves the LDS table
// empty.
__device__ __forceinline__ void flush_chunk(const HubArgs& h, int32_t p, int32_t* skeys, double* svals,
                                            int32_t* snew, int* s_nnew, int* s_base) {
  constexpr int TS = 1 << kHubGatherLg;
  TblSlot* gt = tbl_of(h, p);
  const int lg = tbl_lg(h, p);
  if (threadIdx.x == 0) *s_nnew = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < TS; s += kBlock) {
    const int32_t c = skeys[s];
    if (c != kEmpty) {
      const int64_t slot = slot_insert_new(gt, lg, c, svals[s]);
      if (slot >= 0) snew[atomicAdd(s_nnew, 1)] = (int32_t)slot;
      skeys[s] = kEmpty;
      svals[s] = 0.0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *s_base = *s_nnew ? atomicAdd(&h.lcnt[p], *s_nnew) : 0;
  __syncthreads();
  int32_t* lst = tbl_list_of(h, p);
  for (int k = threadIdx.x; k < *s_nnew; k += kBlock) lst[*s_base + k] = snew[k];
  __syncthreads();
}

// The distinct entries of a chunk's LDS table (2^kHubGatherLg slots), sorted
// by key partition (wide_part mod P), are written to lb / wb[0..n) with the
// partition offsets to po[0..P]; the table is left empty.  s_cnt: P + 1
// ints of LDS, zeroed by the caller before the table was filled and made
// visible by a barrier since; s_wsum: kBlock / kWave ints of LDS.
__device__ __forceinline__ void stage_chunk_partitions(int32_t* skeys, double* svals, int32_t* s_cnt, int* s_wsum,
                                                       int P, int32_t* lb, double* wb, uint16_t* po) {
  constexpr int TS = 1 << kHubGatherLg;
  // the table's entries into registers (the table is left empty), with
  // their rank inside their partition
  constexpr int R = TS / kBlock;
  int32_t ck[R], rk[R];
  double cw[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int sl = r * kBlock + threadIdx.x;
    ck[r] = skeys[sl];
    cw[r] = svals[sl];
    rk[r] = 0;
    if (ck[r] != kEmpty) {
      skeys[sl] = kEmpty;
      svals[sl] = 0.0;
      rk[r] = atomicAdd(&s_cnt[wide_part(ck[r]) & (uint32_t)(P - 1)], 1);
    }
  }
  __syncthreads();
  {  // exclusive scan of the P <= kBlock counts; s_cnt[P] = total
    const int v = ((int)threadIdx.x < P) ? s_cnt[threadIdx.x] : 0;
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_up(incl, o);
      if (lane_id() >= o) incl += x;
    }
    const int wv = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) s_wsum[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < kBlock / kWave; ++k) {
      if (k < wv) before += s_wsum[k];
      total += s_wsum[k];
    }
    if ((int)threadIdx.x < P) s_cnt[threadIdx.x] = before + incl - v;
    if (threadIdx.x == 0) s_cnt[P] = total;
    __syncthreads();
  }
  // staged in partition order at the front of the (empty) table
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (ck[r] == kEmpty) continue;
    const int pos = s_cnt[wide_part(ck[r]) & (uint32_t)(P - 1)] + rk[r];
    skeys[pos] = ck[r];
    svals[pos] = cw[r];
  }
  __syncthreads();
  // out; the table is emptied again
  const int n = s_cnt[P];
  for (int k = threadIdx.x; k < n; k += kBlock) {
    lb[k] = skeys[k];
    wb[k] = svals[k];
    skeys[k] = kEmpty;
    svals[k] = 0.0;
  }
  for (int k = threadIdx.x; k <= P; k += kBlock) po[k] = (uint16_t)s_cnt[k];
  __syncthreads();  // s_cnt is read above before the caller reuses it
}

// Chunk gather: H_chunk[C[j]] += w over the chunk's arcs (j != i; in
// refinement only j inside i's bound), staged by key partition (PART: hubs
// of up to kPartMaxDeg arcs) or merged into the hub's global table (longer
// hubs).  Two instances, so the partitioned one keeps the LDS of the
// table's new-slot list free (three workgroups per CU instead of two).
template <class WT, int PH, bool PART>
__global__ __launch_bounds__(kBlock) void k_hub_gather(GraphView<WT> g, ScanArgs a, HubArgs h, int32_t t0,
                                                       int32_t t1) {
  constexpr int TS = 1 << kHubGatherLg;
  __shared__ int32_t skeys[TS];
  __shared__ double svals[TS];
  __shared__ int32_t snew[PART ? kPartMaxP + 1 : kHubChunk];
  __shared__ int s_nnew, s_base;
  __shared__ double s_red[kBlock / kWave];
  __shared__ int s_wsum[kBlock / kWave];
  static_assert(kPartMaxP <= kBlock && kPartMaxP < kHubChunk, "partition counts: one per thread");
  static_assert(kHubChunk % kBlock == 0 && kHubChunk <= (1 << kHubGatherLg), "chunk staging in the LDS table");
  for (int s = threadIdx.x; s < TS; s += kBlock) { skeys[s] = kEmpty; svals[s] = 0.0; }
  __syncthreads();
  unsigned long long na = 0;
  for (int64_t t = t0 + (int64_t)blockIdx.x; t < t1; t += gridDim.x) {
    const int2 task = h.chunk_tasks[t];
    const int32_t p = task.x;
    if (!h.active[p]) continue;  // uniform over the workgroup
    const int32_t i = h.items[p];
    const int32_t beg = g.begin(i), deg = g.degree(i);
    if (hub_partitioned(deg) != PART) continue;  // uniform: the other instance
    const int32_t e0 = task.y * kHubChunk;
    const int32_t e1 = (deg - e0 < kHubChunk) ? deg : e0 + kHubChunk;
    const int32_t bi = (PH == kRefine) ? a.CB[i] : 0;
    const int32_t d = a.C[i];
    if (PART) {  // sum the chunk's candidates, sort them by partition
      const int P = h.slice_off[p + 1] - h.slice_off[p];
      int32_t* s_cnt = snew;  // [P + 1] counts, then offsets
      for (int k = threadIdx.x; k <= P; k += kBlock) s_cnt[k] = 0;
      // 1. candidates into the LDS table (equal communities summed)
      double kid = scan_row<4, kBlock, PH>(g, a, i, beg, e1, e0 + threadIdx.x, d, bi, [&](int32_t c, double w) {
        lds_insert(skeys, svals, kHubGatherLg, c, w);
      });
      __syncthreads();
      stage_chunk_partitions(skeys, svals, s_cnt, s_wsum, P, h.lbuf + (int64_t)beg + e0, h.wbuf + (int64_t)beg + e0,
                             h.poff + t * (kPartMaxP + 1));
      kid = block_sum<double>(kid, s_red);  // (its barriers also end this chunk's LDS use)
      if (threadIdx.x == 0) {
        na += (unsigned long long)(e1 - e0);
        if (kid != 0.0) atomicAdd(&h.kid[p], kid);
      }
      continue;
    }
    // arcs to the hub's own community are summed apart into kid[p]
    double kid = scan_row<4, kBlock, PH>(g, a, i, beg, e1, e0 + threadIdx.x, d, bi, [&](int32_t c, double w) {
      lds_insert(skeys, svals, kHubGatherLg, c, w);
    });
    kid = block_sum<double>(kid, s_red);
    if (threadIdx.x == 0) {
      na += (unsigned long long)(e1 - e0);
      if (kid != 0.0) atomicAdd(&h.kid[p], kid);
    }
    __syncthreads();
    flush_chunk(h, p, skeys, svals, snew, &s_nnew, &s_base);
  }
  if (threadIdx.x == 0 && na) {
    atomicAdd(&cnt_of(a.cnt)[1], na);
    if (PH == kRefine) atomicAdd(&cnt_of(a.cnt)[7], na);
  }
}

// Slice evaluation: best candidate among the slice's entries of the hub's
// occupied-slot list (the slots are cleared for the next use); the last
// slice of a hub reduces the partial bests, applies the min-label rule and
// the sign test, and commits (fast local-moving) or records the decision.
template <class WT, int PH, bool DET>
__global__ __launch_bounds__(kBlock) void k_hub_eval(GraphView<WT> g, ScanArgs a, HubArgs h, int32_t s0,
                                                     int32_t s1) {
  __shared__ double s_g[kBlock / kWave];
  __shared__ i128 s_k[kBlock / kWave];
  __shared__ int32_t s_c[kBlock / kWave];
  __shared__ int s_last, s_take;
  unsigned long long nc = 0, nv = 0, nm = 0;
  double dq = 0.0;
  i128 dqk = 0;
  for (int64_t t = s0 + (int64_t)blockIdx.x; t < s1; t += gridDim.x) {
    const int2 task = h.slice_tasks[t];
    const int32_t p = task.x;
    if (!h.active[p]) continue;  // uniform
    const int32_t i = h.items[p];
    if (hub_partitioned(g.degree(i))) continue;  // uniform: k_hub_part_eval
    const int32_t d = a.C[i];
    const double ki = a.K[i];
    const Eval<DET> ev(a, i, h.kid[p], ki, a.Sig[d]);
    TblSlot* gt = tbl_of(h, p);
    const int32_t* lst = tbl_list_of(h, p);
    const int32_t len = h.lcnt[p];
    const int64_t ts = (int64_t)1 << tbl_lg(h, p);
    // dense tables are scanned slot by slot (coalesced), sparse ones through
    // their occupied-slot list; slice sl covers kHubSlice slots or entries
    const bool dense = (int64_t)len * 8 > ts;
    const int64_t lim = dense ? ts : len;
    const int64_t q0 = (int64_t)task.y * kHubSlice;
    const int64_t q1 = (lim - q0 < kHubSlice) ? lim : q0 + kHubSlice;
    int32_t bc = -1;
    double bg = 0.0;
    i128 bk = 0;
    // a slice past the end of a sparse table's list has nothing to read: it
    // only reports an empty partial result (no workgroup-wide reduction)
    const bool empty = q0 >= lim;
    if (!empty) {  // uniform
      // U positions per thread per step: all slot reads, then all Sigma
      // gathers, are in flight together
      constexpr int U = 8;
      for (int64_t qb = q0; qb < q1; qb += U * kBlock) {
        uint32_t sl[U];
        int32_t ck[U];
        double cw[U], sg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t q = qb + u * kBlock + threadIdx.x;
          sl[u] = 0;
          ck[u] = kEmpty;
          cw[u] = 0.0;
          if (q < q1) {
            sl[u] = dense ? (uint32_t)q : (uint32_t)lst[q];
            const TblSlot e = gt[sl[u]];
            ck[u] = e.key;
            cw[u] = e.val;
          }
        }
        bool e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = ck[u] != kEmpty && ck[u] != d && ev.may_gain(cw[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) sg[u] = e[u] ? a.Sig[ck[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (ck[u] == kEmpty) continue;
          gt[sl[u]] = TblSlot{kEmpty, 0, 0.0};
          if (!e[u]) continue;
          ++nc;
          ev(a, ck[u], cw[u], sg[u], bg, bk, bc);
        }
      }
      block_argmax<DET>(bg, bk, bc, s_g, s_k, s_c);
    }
    if (threadIdx.x == 0) {
      h.pb_g[t] = bg;
      h.pb_k[t] = bk;
      h.pb_c[t] = bc;
      __threadfence();
      const int nsl = h.slice_off[p + 1] - h.slice_off[p];
      const int prev = atomicAdd(&h.done[p], 1);
      s_last = (prev == nsl - 1) ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      const int32_t sb = h.slice_off[p], se = h.slice_off[p + 1];
      bc = -1; bg = 0.0; bk = 0;
      for (int32_t k = sb + (int32_t)threadIdx.x; k < se; k += kBlock) {
        const int32_t c2 = __hip_atomic_load(h.pb_c + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (DET) {
          const unsigned long long* kw = (const unsigned long long*)(h.pb_k + k);
          const unsigned long long lo = __hip_atomic_load(kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const unsigned long long hi = __hip_atomic_load(kw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const i128 k2 = make_i128((long long)hi, lo);
          if (better_k(k2, c2, bk, bc)) { bk = k2; bc = c2; }
        } else {
          const double g2 = __hip_atomic_load(h.pb_g + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (better_f(g2, c2, bg, bc)) { bg = g2; bc = c2; }
        }
      }
      block_argmax<DET>(bg, bk, bc, s_g, s_k, s_c);
      if (threadIdx.x == 0) {
        h.done[p] = 0;
        h.lcnt[p] = 0;
        ++nv;
        const bool take = accept<PH, DET>(a, i, d, bc, bg, bk, DET || (a.sync_moves & 2));
        s_take = take ? 1 : 0;
        if (take) {
          if (PH == kMove && !DET && !(a.sync_moves & 2)) {
            atomicAdd(&a.Sig[d], -ki);
            atomicAdd(&a.Sig[bc], ki);
            atomicSub(&a.size[d], 1);
            atomicAdd(&a.size[bc], 1);
            a.C[i] = bc;
            if (a.gid) atomicAdd(a.dqg + a.gid[i], bg); else dq += bg;
            ++nm;
          } else if (PH == kMove) {
            a.target[i] = bc;
            record_move(a, i, d, bc, -1);
            if (a.gid) {
              if (DET) atomic_add_i128(a.dqg128 + 2 * a.gid[i], bk); else atomicAdd(a.dqg + a.gid[i], bg);
            } else {
              if (DET) dqk += bk; else dq += bg;
            }
          } else {
            a.target[i] = bc;
            a.targeted[bc] = cur_stamp(a);
          }
        }
      }
      __syncthreads();
      if (PH == kMove && !DET && !(a.sync_moves & 2) && s_take)
        mark_row(g, a, i, g.begin(i), g.degree(i), threadIdx.x, kBlock, false);
    }
    __syncthreads();
  }
  // one thread per workgroup carries the counters
  if (threadIdx.x == 0) {
    if (nv) atomicAdd(&cnt_of(a.cnt)[0], nv);
    if (nm) atomicAdd(&cnt_of(a.cnt)[3], nm);
    if (DET) { if (dqk != 0) atomic_add_i128(a.dq128 + 2 * cslot(), dqk); }
    else { if (dq != 0.0) atomicAdd(a.dq + cslot(), dq); }
  }
  __shared__ unsigned long long red_u[16];
  nc = block_sum<unsigned long long>(nc, red_u);
  if (threadIdx.x == 0 && nc) atomicAdd(&cnt_of(a.cnt)[2], nc);
}

// Partition evaluation of the partitioned hubs: task (p, q) accumulates the
// candidates c of hub p with wide_part(c) mod P == q from lbuf into an LDS
// table, evaluates them (Eq. 2) and leaves its partial best at the task's
// index; the last partition of p to finish reduces them, applies the
// min-label rule and the sign test, and commits (fast local-moving) or
// records the decision.  A partition whose keys overflow the table
// (statistically out of reach: at most kPartKeys expected per kPartSlots
// slots) reports kOverflow, cancels the hub's move and counts it in *a.ovf.
constexpr int32_t kOverflow = -2;
template <class WT, int PH, bool DET>
__global__ __launch_bounds__(kPartThreads) void k_hub_part_eval(GraphView<WT> g, ScanArgs a, HubArgs h, int32_t s0,
                                                                int32_t s1) {
  constexpr int NT = kPartThreads;
  constexpr int NW = NT / kWave;
  constexpr int TS = kPartSlots;
  static_assert(TS % NT == 0, "whole slots per thread");
  __shared__ int32_t keys[TS];
  __shared__ double vals[TS];
  __shared__ double s_g[NW];
  __shared__ i128 s_k[NW];
  __shared__ int32_t s_c[NW];
  __shared__ int s_ovf, s_last, s_take;
  __shared__ int32_t s_pre[NT + 1];
  __shared__ int32_t s_r0[NT];
  __shared__ int32_t s_w[NW];
  static_assert(kPartMaxDeg / kHubChunk <= NT, "one chunk per thread");
  for (int s = threadIdx.x; s < TS; s += NT) { keys[s] = kEmpty; vals[s] = 0.0; }
  Acc acc;
  for (int64_t t = s0 + (int64_t)blockIdx.x; t < s1; t += gridDim.x) {
    const int2 task = h.slice_tasks[t];
    const int32_t p = task.x;
    if (!h.active[p]) continue;  // uniform
    const int32_t i = h.items[p];
    const int32_t beg = g.begin(i), deg = g.degree(i);
    if (!hub_partitioned(deg)) continue;  // uniform: k_hub_eval
    // the hub's own label, K', K_{i->d} and total go out before the table
    // is filled, not after it
    const int32_t d = a.C[i];
    const double ki = a.K[i], kid = h.kid[p];
    const double sd = a.Sig[d];
    const int32_t sb = h.slice_off[p], se = h.slice_off[p + 1];
    const uint32_t pm = (uint32_t)(se - sb) - 1u;  // P - 1
    const uint32_t q = (uint32_t)task.y;
    // this partition's run in every chunk of p: start inside the chunk and
    // prefix of the run lengths
    const int32_t nch = h.chunk_off[p + 1] - h.chunk_off[p];
    int32_t r0 = 0, len = 0;
    if ((int)threadIdx.x < nch) {
      const uint16_t* po = h.poff + ((int64_t)h.chunk_off[p] + threadIdx.x) * (kPartMaxP + 1);
      r0 = po[q];
      len = (int32_t)po[q + 1] - r0;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_up(incl, o);
      if (lane_id() >= o) incl += x;
    }
    __syncthreads();  // the previous task's reads of s_pre / s_r0 and of the table are done
    if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = incl;
    if (threadIdx.x == 0) s_ovf = 0;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NW; ++k) {
      if (k < (int)(threadIdx.x / kWave)) before += s_w[k];
      total += s_w[k];
    }
    s_pre[threadIdx.x] = before + incl - len;
    s_r0[threadIdx.x] = r0;
    if (threadIdx.x == 0) s_pre[NT] = total;
    __syncthreads();
    const double* wb = h.wbuf;
    constexpr int U = 4;  // entries per thread per step, their loads in flight together
    for (int32_t kb = threadIdx.x; kb < total; kb += U * NT) {
      int32_t ck[U];
      double cw[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t k = kb + u * NT;
        ck[u] = kEmpty;
        cw[u] = 0.0;
        if (k < total) {
          int lo = 0, hi = nch;  // s_pre[lo] <= k < s_pre[hi] (s_pre[nch] = total)
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pre[mid] <= k) lo = mid; else hi = mid;
          }
          const int64_t pos = (int64_t)beg + (int64_t)lo * kHubChunk + s_r0[lo] + (k - s_pre[lo]);
          ck[u] = h.lbuf[pos];
          cw[u] = wb[pos];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ck[u] != kEmpty && !lds_insert_sized(keys, vals, (uint32_t)TS, ck[u], cw[u])) s_ovf = 1;
    }
    __syncthreads();
    const Eval<DET> ev(a, i, kid, ki, sd);
    int32_t bc = -1;
    double bg = 0.0;
    i128 bk = 0;
    eval_table<4, NT, DET>(keys, vals, TS, threadIdx.x, a, ev, acc, bg, bk, bc);  // (fewer registers: two workgroups per CU)
    block_argmax<DET, NW>(bg, bk, bc, s_g, s_k, s_c);
    if (threadIdx.x == 0) {
      h.pb_g[t] = bg;
      h.pb_k[t] = bk;
      h.pb_c[t] = s_ovf ? kOverflow : bc;
      __threadfence();
      const int prev = atomicAdd(&h.done[p], 1);
      s_last = (prev == (int)pm) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) continue;  // uniform
    __threadfence();
    bc = -1; bg = 0.0; bk = 0;
    int ovf = 0;
    for (int32_t k = sb + (int32_t)threadIdx.x; k < se; k += NT) {
      const int32_t c2 = __hip_atomic_load(h.pb_c + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c2 == kOverflow) { ovf = 1; continue; }
      if (DET) {
        const unsigned long long* kw = (const unsigned long long*)(h.pb_k + k);
        const unsigned long long lo = __hip_atomic_load(kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long hi = __hip_atomic_load(kw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const i128 k2 = make_i128((long long)hi, lo);
        if (better_k(k2, c2, bk, bc)) { bk = k2; bc = c2; }
      } else {
        const double g2 = __hip_atomic_load(h.pb_g + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (better_f(g2, c2, bg, bc)) { bg = g2; bc = c2; }
      }
    }
    ovf = __syncthreads_or(ovf);
    block_argmax<DET, NW>(bg, bk, bc, s_g, s_k, s_c);
    if (threadIdx.x == 0) {
      h.done[p] = 0;
      ++acc.nv;
      if (ovf) atomicAdd(a.ovf, 1ull);
      const bool take = !ovf && accept<PH, DET>(a, i, d, bc, bg, bk, DET || (a.sync_moves & 2));
      s_take = take ? 1 : 0;
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
          record_move(a, i, d, bc, -1);
          add_gain<DET>(a, acc, i, bg, bk);
        } else {
          a.target[i] = bc;
          a.targeted[bc] = cur_stamp(a);
        }
      }
    }
    __syncthreads();
    if (PH == kMove && !DET && !(a.sync_moves & 2) && s_take) mark_row(g, a, i, beg, deg, threadIdx.x, NT, false);
  }
  flush_acc<PH, DET>(a, acc);  // (the arcs were counted by the chunk pass)
}

template <class WT, int PH, bool DET>
static void hub_decide_t(hipStream_t st, const GraphDesc& gd, const ScanArgs& a, const HubArgs& h, int32_t h0,
                         int32_t h1, int32_t c0, int32_t c1, int32_t s0, int32_t s1, bool tables, int64_t* launches) {
  const GraphView<WT> g = view<WT>(gd);
  if (c1 > c0) {
    hipLaunchKernelGGL((k_hub_gather<WT, PH, true>), dim3(grid_items(c1 - c0, 1, 2048)), dim3(kBlock), 0, st, g, a,
                       h, c0, c1);
    if (tables)
      hipLaunchKernelGGL((k_hub_gather<WT, PH, false>), dim3(grid_items(c1 - c0, 1, 2048)), dim3(kBlock), 0, st, g,
                         a, h, c0, c1);
  }
  if (s1 > s0) {
    if (tables)
      hipLaunchKernelGGL((k_hub_eval<WT, PH, DET>), dim3(grid_items(s1 - s0, 1, 2048)), dim3(kBlock), 0, st, g, a,
                         h, s0, s1);
    // two workgroups per CU (their LDS tables fill it) take the partitions in turn
    hipLaunchKernelGGL((k_hub_part_eval<WT, PH, DET>), dim3(grid_items(s1 - s0, 1, 512)), dim3(kPartThreads), 0,
                       st, g, a, h, s0, s1);
  }
  *launches += tables ? 4 : 2;
}

void hub_decide(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const HubArgs& h, int32_t h0, int32_t h1,
                int32_t c0, int32_t c1, int32_t s0, int32_t s1, bool tables, int phase, bool det, int64_t* launches) {
  if (h1 <= h0) return;
#define GVL_HUB(WT, PH, DET) hub_decide_t<WT, PH, DET>(st, g, a, h, h0, h1, c0, c1, s0, s1, tables, launches)
  if (g.w_double) {
    if (phase == kMove) { if (det) GVL_HUB(double, kMove, true); else GVL_HUB(double, kMove, false); }
    else { if (det) GVL_HUB(double, kRefine, true); else GVL_HUB(double, kRefine, false); }
  } else {
    if (phase == kMove) { if (det) GVL_HUB(float, kMove, true); else GVL_HUB(float, kMove, false); }
    else { if (det) GVL_HUB(float, kRefine, true); else GVL_HUB(float, kRefine, false); }
  }
#undef GVL_HUB
}

// ------------------------------------------------------ row sums of hubs ---
template <class WT>
__global__ __launch_bounds__(kBlock) void k_hub_weights(GraphView<WT> g, HubArgs h, int32_t t0, int32_t t1, double* K,
                                                        double* accW, int32_t* flags, int validate) {
  __shared__ double red[16];
  int bad_csr = 0, bad_w = 0, bad_sign = 0;
  for (int64_t t = t0 + (int64_t)blockIdx.x; t < t1; t += gridDim.x) {
    const int2 task = h.chunk_tasks[t];
    const int32_t i = h.items[task.x];
    const int32_t beg = g.begin(i), deg = g.degree(i);
    const int32_t e0 = task.y * kHubChunk;
    const int32_t e1 = (deg - e0 < kHubChunk) ? deg : e0 + kHubChunk;
    double s = 0.0;
    for (int32_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
      const double w = g.weight(beg + e);
      if (validate) {
        const int32_t j = g.idx[beg + e];
        if (j < 0 || j >= g.n) bad_csr = 1;
      }
      if (!(w >= 1.0 && w <= 16777216.0 && w == floor(w))) bad_w = 1;
      if (!(w > 0.0 && w < INFINITY)) bad_sign = 1;
      s += w;
    }
    s = block_sum<double>(s, red);
    if (threadIdx.x == 0) {
      atomicAdd(&K[i], s);
      atomicAdd(accW, s);
    }
  }
  if (bad_csr) atomicOr(&flags[0], 1);
  if (bad_w) atomicOr(&flags[1], 1);
  if (bad_sign) atomicOr(&flags[2], 1);
}

void hub_weights(hipStream_t st, const GraphDesc& gd, const HubArgs& h, int32_t c0, int32_t c1, double* K,
                 double* accW, int32_t* flags, int validate) {
  if (c1 <= c0) return;
  const int grid = grid_items(c1 - c0, 1, 2048);
  if (gd.w_double)
    hipLaunchKernelGGL(k_hub_weights<double>, dim3(grid), dim3(kBlock), 0, st, view<double>(gd), h, c0, c1, K, accW,
                       flags, validate);
  else
    hipLaunchKernelGGL(k_hub_weights<float>, dim3(grid), dim3(kBlock), 0, st, view<float>(gd), h, c0, c1, K, accW,
                       flags, validate);
}

// --------------------------------------------------- modularity of hub rows ---
template <class WT>
__global__ __launch_bounds__(kBlock) void k_hub_modularity(GraphView<WT> g, HubArgs h, int32_t t0, int32_t t1,
                                                           const int32_t* C, double* tot, double* acc_d,
                                                           const int32_t* gid, double* s1g) {
  __shared__ double red[16];
  double s1 = 0.0;
  for (int64_t t = t0 + (int64_t)blockIdx.x; t < t1; t += gridDim.x) {
    const int2 task = h.chunk_tasks[t];
    const int32_t i = h.items[task.x];
    const int32_t beg = g.begin(i), deg = g.degree(i), ci = C[i];
    const int32_t e0 = task.y * kHubChunk;
    const int32_t e1 = (deg - e0 < kHubChunk) ? deg : e0 + kHubChunk;
    double k = 0.0, sc = 0.0;
    constexpr int U = 8;  // arcs per thread per round, their loads issued together
    for (int32_t eb = e0 + threadIdx.x; eb < e1; eb += U * kBlock) {
      int32_t j[U];
      WT w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        j[u] = i;  // (past the chunk: an unused, valid label load)
        w[u] = WT(0);
        if (eb + u * kBlock < e1) {
          j[u] = g.idx[beg + eb + u * kBlock];
          w[u] = g.weight(beg + eb + u * kBlock);
        }
      }
      int32_t cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cj[u] = C[j[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        k += (double)w[u];
        if (eb + u * kBlock < e1 && cj[u] == ci) sc += (double)w[u];
      }
    }
    k = block_sum<double>(k, red);
    if (threadIdx.x == 0) atomicAdd(&tot[ci], k);
    if (gid) {
      sc = block_sum<double>(sc, red);
      if (threadIdx.x == 0 && sc != 0.0) atomicAdd(&s1g[gid[i]], sc);
    } else {
      s1 += sc;
    }
  }
  s1 = block_sum<double>(s1, red);
  if (threadIdx.x == 0 && s1 != 0.0) atomicAdd(&acc_d[0], s1);
}

void hub_modularity(hipStream_t st, const GraphDesc& gd, const HubArgs& h, int32_t c0, int32_t c1, const int32_t* C,
                    double* tot, double* acc_d, const int32_t* gid, double* s1g) {
  if (c1 <= c0) return;
  const int grid = grid_items(c1 - c0, 1, 2048);
  if (gd.w_double)
    hipLaunchKernelGGL(k_hub_modularity<double>, dim3(grid), dim3(kBlock), 0, st, view<double>(gd), h, c0, c1, C, tot,
                       acc_d, gid, s1g);
  else
    hipLaunchKernelGGL(k_hub_modularity<float>, dim3(grid), dim3(kBlock), 0, st, view<float>(gd), h, c0, c1, C, tot,
                       acc_d, gid, s1g);
}

// ------------------------------------------------ giant community rows ---
template <class WT>
__global__ void k_member_degrees(GraphView<WT> g, const int32_t* cv, int64_t n, int32_t* mdeg) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    mdeg[k] = g.degree(cv[k]);
}
void member_degrees(hipStream_t st, const GraphDesc& gd, const int32_t* cv, int64_t n, int32_t* mdeg) {
  if (n > 0) hipLaunchKernelGGL(k_member_degrees<float>, dim3(grid_items(n, kBlock, 16384)), dim3(kBlock), 0, st,
                                view<float>(gd), cv, n, mdeg);
}

// Chunk gather over the concatenated member rows of community c: arcs
// [apre[coff[c]] + chunk * kHubChunk, ...) of the community-vertex order.
// One wavefront finds the member holding the chunk's first arc (a 65-way
// search over the member offsets, one load per step), the workgroup copies
// the offsets and row starts of the chunk's members to LDS, and thread t
// takes the chunk's arcs t, t + kBlock, ... (coalesced), each finding its
// member by a binary search in LDS.
template <class WT>
__global__ __launch_bounds__(kBlock) void k_gagg_gather(GraphView<WT> g, AggArgs a, HubArgs h, int32_t t0,
                                                        int32_t t1) {
  constexpr int TS = 1 << kHubGatherLg;
  constexpr int PER = kHubChunk / kBlock;  // arcs per thread
  __shared__ int32_t skeys[TS];
  __shared__ double svals[TS];
  __shared__ int32_t s_cnt[kPartMaxP + 1];
  __shared__ double s_red[kBlock / kWave];
  __shared__ int s_wsum[kBlock / kWave];
  __shared__ int32_t s_mo[kHubChunk + 1];  // member offsets (apre) from the chunk's first member on
  __shared__ int32_t s_mb[kHubChunk];      // their row starts
  __shared__ int32_t s_k0;
  for (int s = threadIdx.x; s < TS; s += kBlock) { skeys[s] = kEmpty; svals[s] = 0.0; }
  __syncthreads();
  unsigned long long na = 0;
  for (int64_t t = t0 + (int64_t)blockIdx.x; t < t1; t += gridDim.x) {
    const int2 task = h.chunk_tasks[t];
    const int32_t p = task.x;
    const int32_t c = h.items[p];
    const int32_t mb = a.coff[c], me = a.coff[c + 1];
    const int P = h.slice_off[p + 1] - h.slice_off[p];
    for (int k = threadIdx.x; k <= P; k += kBlock) s_cnt[k] = 0;
    const int64_t cend = h.apre[me];
    const int64_t A0 = (int64_t)h.apre[mb] + (int64_t)task.y * kHubChunk;
    const int64_t A1 = (A0 + kHubChunk < cend) ? A0 + kHubChunk : cend;
    if (threadIdx.x < kWave) {  // member k0 of [mb, me) with apre[k0] <= A0 < apre[k0 + 1]
      int32_t lo = mb, hi = me;
      const int l = lane_id();
      while (hi - lo > 1) {  // uniform over the wavefront
        const int64_t span = hi - lo;
        int32_t x;
        bool ok;
        if (span <= kWave) {
          x = lo + 1 + l;
          ok = x < hi && h.apre[x] <= A0;
        } else {
          x = lo + (int32_t)((span * (l + 1)) / (kWave + 1));  // strictly increasing in (lo, hi)
          ok = h.apre[x] <= A0;
        }
        const int L = __popcll(__ballot(ok));  // the probes are ordered and apre is monotone
        const int32_t xlo = __shfl(x, L > 0 ? L - 1 : 0);
        const int32_t xhi = __shfl(x, L < kWave ? L : kWave - 1);
        if (span <= kWave) {
          lo = L > 0 ? xlo : lo;
          hi = lo + 1;
        } else {
          if (L > 0) lo = xlo;
          if (L < kWave) hi = xhi;
        }
      }
      if (l == 0) s_k0 = lo;
    }
    __syncthreads();
    const int32_t k0 = s_k0;
    // offsets and row starts of the members k0, k0 + 1, ... that start
    // before A1 (at most kHubChunk: each holds an arc of the chunk)
    int32_t nm = 0;
    for (int32_t r = 0; r < kHubChunk; r += kBlock) {  // uniform
      const int32_t k = k0 + r + (int32_t)threadIdx.x;
      int in = 0;
      if (k < me) {
        const int32_t o = h.apre[k];
        if (o < A1) {
          s_mo[r + threadIdx.x] = o;
          s_mb[r + threadIdx.x] = g.begin(a.cv[k]);
          in = 1;
        }
      }
      const int cnt = __syncthreads_count(in);  // members start in order, so these are a prefix
      nm += cnt;
      if (cnt < kBlock) break;
    }
    double self = 0.0;  // arcs inside c: the super-vertex's self-loop
    int32_t j[PER];
    WT w[PER];  // widened where used (see GraphView::weight)
    bool in[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      const int64_t q = A0 + (int64_t)x * kBlock + threadIdx.x;
      in[x] = q < A1;
      j[x] = 0;  // (past the chunk: an unused, valid label load)
      w[x] = WT(0);
      if (in[x]) {
        int lo = 0, hi = nm;  // s_mo[lo] <= q < s_mo[hi] (s_mo[nm] taken as A1)
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_mo[mid] <= q) lo = mid; else hi = mid;
        }
        const int64_t e = (int64_t)s_mb[lo] + (q - s_mo[lo]);
        j[x] = g.idx[e];
        w[x] = g.weight(e);
      }
    }
    int32_t dl[PER];
#pragma unroll
    for (int x = 0; x < PER; ++x) dl[x] = a.lab[j[x]];
#pragma unroll
    for (int x = 0; x < PER; ++x) {
      if (!in[x] || dl[x] == kEmpty) continue;
      if (dl[x] == c) self += (double)w[x];
      else lds_insert(skeys, svals, kHubGatherLg, dl[x], (double)w[x]);
    }
    na += (unsigned long long)((A1 - A0 + kBlock - 1 - threadIdx.x) / kBlock);
    self = block_sum<double>(self, s_red);
    if (threadIdx.x == 0 && self != 0.0) lds_insert(skeys, svals, kHubGatherLg, c, self);
    // the distinct entries, by partition, at the chunk's arc positions
    __syncthreads();
    stage_chunk_partitions(skeys, svals, s_cnt, s_wsum, P, h.lbuf + A0, h.wbuf + A0, h.poff + t * (kPartMaxP + 1));
  }
  __shared__ unsigned long long red_u[16];
  na = block_sum<unsigned long long>(na, red_u);
  if (threadIdx.x == 0 && na) atomicAdd(&cnt_of(a.cnt)[5], na);
}

// Partition emit of the giant communities: task (p, q) sums the entries of
// partition q of every chunk of community c = items[p] in an LDS table and
// appends its distinct (d, H[d]) to row c.  The chunks are taken kPartThreads
// at a time (their run offsets in LDS).  Entries are inserted kPartBatch at a
// time; a batch that could overfill the table first flushes it to the row
// (then a key can occur twice in the row, with partial sums, which every
// later step adds up).  Up to kPartMaxDeg member arcs this is statistically
// out of reach (the table holds 1.5 times the expected keys of a
// partition); beyond, it happens when a partition has more distinct keys
// than its table.
constexpr int kPartBatch = 1024;
__device__ __forceinline__ int lds_insert_new_sized(int32_t* keys, double* vals, uint32_t ts, int32_t c, double w) {
  uint32_t h = (uint32_t)(((u64)((uint32_t)c * 0x9E3779B1u) * (u64)ts) >> 32);
  for (uint32_t probe = 0; probe < ts; ++probe) {
    int32_t k = keys[h];
    if (k == c) { atomicAdd(&vals[h], w); return 0; }
    if (k == kEmpty) {
      const int32_t old = atomicCAS(&keys[h], kEmpty, c);
      if (old == kEmpty || old == c) { atomicAdd(&vals[h], w); return old == kEmpty ? 1 : 0; }
    }
    h = (h + 1u == ts) ? 0u : h + 1u;
  }
  return -1;
}

template <class WTout>
__global__ __launch_bounds__(kPartThreads) void k_gagg_part_emit(AggArgs a, HubArgs h, int32_t s0, int32_t s1) {
  constexpr int NT = kPartThreads;
  constexpr int NW = NT / kWave;
  constexpr int TS = kPartSlots;
  constexpr int R = TS / NT;
  static_assert(TS % NT == 0 && kPartBatch < TS, "table rounds, batch below the table size");
  __shared__ int32_t keys[TS];
  __shared__ double vals[TS];
  __shared__ int32_t s_pre[NT + 1];
  __shared__ int32_t s_r0[NT];
  __shared__ int32_t s_w[NW];
  __shared__ int s_occ, s_base;
  WTout* yw = (WTout*)a.yw;
  unsigned long long no = 0;
  for (int s = threadIdx.x; s < TS; s += NT) { keys[s] = kEmpty; vals[s] = 0.0; }
  // appends the table's entries to row c and empties the table (every
  // thread; starts and ends with a barrier)
  auto flush = [&](int32_t c) {
    __syncthreads();
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) cnt += (keys[r * NT + threadIdx.x] != kEmpty);
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_up(incl, o);
      if (lane_id() >= o) incl += x;
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < NW; ++k) {
      if (k < w) before += s_w[k];
      total += s_w[k];
    }
    if (threadIdx.x == 0) {
      s_base = total ? atomicAdd(&a.ydeg[c], total) : 0;
      s_occ = 0;
      no += (unsigned long long)total;
    }
    __syncthreads();
    int64_t pos = (int64_t)a.yoff[c] + s_base + before + (incl - cnt);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = r * NT + threadIdx.x;
      const int32_t k = keys[sl];
      if (k == kEmpty) continue;
      a.yidx[pos] = k;
      yw[pos] = (WTout)vals[sl];
      ++pos;
      keys[sl] = kEmpty;
      vals[sl] = 0.0;
    }
    __syncthreads();
  };
  for (int64_t t = s0 + (int64_t)blockIdx.x; t < s1; t += gridDim.x) {
    const int2 task = h.slice_tasks[t];
    const int32_t p = task.x;
    const int32_t c = h.items[p];
    const int32_t q = task.y;
    const int64_t A0 = h.apre[a.coff[c]];
    const int32_t nch = h.chunk_off[p + 1] - h.chunk_off[p];
    if (threadIdx.x == 0) s_occ = 0;
    for (int32_t cb = 0; cb < nch; cb += NT) {  // uniform
      // this partition's run in chunks cb .. cb + nb - 1 of c
      const int32_t nb = (nch - cb < NT) ? nch - cb : NT;
      int32_t r0 = 0, len = 0;
      if ((int)threadIdx.x < nb) {
        const uint16_t* po = h.poff + ((int64_t)h.chunk_off[p] + cb + threadIdx.x) * (kPartMaxP + 1);
        r0 = po[q];
        len = (int32_t)po[q + 1] - r0;
      }
      int incl = len;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int x = __shfl_up(incl, o);
        if (lane_id() >= o) incl += x;
      }
      __syncthreads();  // the previous block's reads of s_pre / s_r0 are done
      if (lane_id() == kWave - 1) s_w[threadIdx.x / kWave] = incl;
      __syncthreads();
      int before = 0, total = 0;
      for (int k = 0; k < NW; ++k) {
        if (k < (int)(threadIdx.x / kWave)) before += s_w[k];
        total += s_w[k];
      }
      s_pre[threadIdx.x] = before + incl - len;
      s_r0[threadIdx.x] = r0;
      if (threadIdx.x == 0) s_pre[NT] = total;
      __syncthreads();
      const int64_t base = A0 + (int64_t)cb * kHubChunk;
      for (int32_t kb = 0; kb < total; kb += kPartBatch) {  // uniform
        if (s_occ + kPartBatch > TS) flush(c);  // (s_occ is read after a barrier)
        const int32_t ke = (kb + kPartBatch < total) ? kb + kPartBatch : total;
        for (int32_t k = kb + threadIdx.x; k < ke; k += NT) {
          int lo = 0, hi = nb;  // s_pre[lo] <= k < s_pre[hi] (s_pre[nb] = total)
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pre[mid] <= k) lo = mid; else hi = mid;
          }
          const int64_t pos = base + (int64_t)lo * kHubChunk + s_r0[lo] + (k - s_pre[lo]);
          if (lds_insert_new_sized(keys, vals, (uint32_t)TS, h.lbuf[pos], h.wbuf[pos]) > 0) atomicAdd(&s_occ, 1);
        }
        __syncthreads();
      }
    }
    flush(c);
  }
  if (threadIdx.x == 0 && no) atomicAdd(&cnt_of(a.cnt)[6], no);
}

void gagg_rows(hipStream_t st, const GraphDesc& gd, const AggArgs& a, const HubArgs& h, int32_t c0, int32_t c1,
               int32_t s0, int32_t s1, int64_t* launches) {
  if (c1 > c0) {
    const int grid = grid_items(c1 - c0, 1, 2048);
    if (gd.w_double)
      hipLaunchKernelGGL(k_gagg_gather<double>, dim3(grid), dim3(kBlock), 0, st, view<double>(gd), a, h, c0, c1);
    else
      hipLaunchKernelGGL(k_gagg_gather<float>, dim3(grid), dim3(kBlock), 0, st, view<float>(gd), a, h, c0, c1);
    ++*launches;
  }
  if (s1 > s0) {
    const int grid = grid_items(s1 - s0, 1, 2048);
    if (a.yw_double)
      hipLaunchKernelGGL(k_gagg_part_emit<double>, dim3(grid), dim3(kPartThreads), 0, st, a, h, s0, s1);
    else
      hipLaunchKernelGGL(k_gagg_part_emit<float>, dim3(grid), dim3(kPartThreads), 0, st, a, h, s0, s1);
    ++*launches;
  }
}

}  // namespace gvl
