// Aggregation (Alg. 4): rows of the super-vertex graph G''.
//
// For each community c (a super-vertex), every arc (j, w) of every member i
// of c -- self-loops included -- adds w to H[lab[j]], where lab[j] is the
// renumbered community of j.  The distinct (d, H[d]) pairs are written into
// row c of the holey CSR, whose capacity yoff[c+1] - yoff[c] is the total
// degree of c's members (an over-estimate), and ydeg[c] receives the count.
//
// Communities are binned by that capacity; small ones map a group of G lanes
// with an LDS table, large ones a workgroup with an LDS table; giant ones are
// split by key partitions (k_hub.hip).  Members with fewer than G arcs are
// walked one per lane; larger members are walked by all lanes of the group
// so that their rows stream coalesced.
#include "device.hpp"
#include "kernels.hpp"

namespace gvl {

// Arcs per lane per round in the row loops: their index, weight and label
// loads are all in flight before the LDS inserts of the round.
constexpr int kAggUnroll = 4;

template <class WTin, class WTout, int G, int LG>
__global__ __launch_bounds__(kBlock) void k_agg_group(GraphView<WTin> g, AggArgs a,
                                                      const int32_t* __restrict__ list,
                                                      int32_t count) {
  constexpr int TS = 1 << LG;
  constexpr int GPB = kBlock / G;
  __shared__ int32_t skeys[GPB * TS];
  __shared__ double svals[GPB * TS];
  __shared__ unsigned long long red_u[16];
  const int gl = threadIdx.x % G;
  const int gb = threadIdx.x / G;
  const int gbase = (lane_id() / G) * G;  // first lane of this group in the wavefront
  const u64 gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  int32_t* keys = skeys + gb * TS;
  double* vals = svals + gb * TS;
  WTout* yw = (WTout*)a.yw;
  for (int s = gl; s < TS; s += G) { keys[s] = kEmpty; vals[s] = 0.0; }
  wave_sync();
  unsigned long long nv = 0, na = 0, no = 0;
  for (int64_t v = (int64_t)blockIdx.x * GPB + gb; v < count; v += (int64_t)gridDim.x * GPB) {
    const int32_t c = list[v];
    const int32_t mb = a.coff[c], me = a.coff[c + 1];
    double self = 0.0;  // arcs inside c: the super-vertex's self-loop
    // members with short rows: one lane each
    for (int32_t k = mb + gl; k < me; k += G) {
      const int32_t i = a.cv[k];
      const int32_t beg = g.begin(i), deg = g.degree(i);
      ++nv;
      if (deg >= G) continue;
      na += (unsigned long long)deg;
      for (int32_t e0 = 0; e0 < deg; e0 += kAggUnroll) {
        int32_t j[kAggUnroll];
        WTin wr[kAggUnroll];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) {
          j[u] = 0;  // (past the row: an unused, valid label load)
          wr[u] = WTin(0);
          if (e0 + u < deg) {
            j[u] = g.idx[beg + e0 + u];
            wr[u] = g.weight(beg + e0 + u);
          }
        }
        int32_t d[kAggUnroll];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) d[u] = a.lab[j[u]];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) {
          if (e0 + u >= deg) continue;
          if (d[u] == c) self += (double)wr[u];
          else lds_insert(keys, vals, LG, d[u], (double)wr[u]);
        }
      }
    }
    // members with long rows: the whole group
    for (int32_t kb = mb; kb < me; kb += G) {
      const int32_t k = kb + gl;
      const int32_t i = (k < me) ? a.cv[k] : 0;
      const bool big = (k < me) && g.degree(i) >= G;
      u64 mask = (__ballot(big) >> gbase) & gmask;
      while (mask) {
        const int q = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int32_t ii = __shfl(i, q, G);
        const int32_t beg = g.begin(ii), deg = g.degree(ii);
        if (gl == 0) na += (unsigned long long)deg;
        for (int32_t e0 = gl; e0 < deg; e0 += kAggUnroll * G) {
          int32_t j[kAggUnroll];
          WTin wr[kAggUnroll];
#pragma unroll
          for (int u = 0; u < kAggUnroll; ++u) {
            j[u] = 0;  // (past the row: an unused, valid label load)
            wr[u] = WTin(0);
            if (e0 + u * G < deg) {
              j[u] = g.idx[beg + e0 + u * G];
              wr[u] = g.weight(beg + e0 + u * G);
            }
          }
          int32_t d[kAggUnroll];
#pragma unroll
          for (int u = 0; u < kAggUnroll; ++u) d[u] = a.lab[j[u]];
#pragma unroll
          for (int u = 0; u < kAggUnroll; ++u) {
            if (e0 + u * G >= deg) continue;
            if (d[u] == c) self += (double)wr[u];
            else lds_insert(keys, vals, LG, d[u], (double)wr[u]);
          }
        }
      }
    }
    self = sum_xor<G>(self);
    wave_sync();
    if (gl == 0 && self != 0.0) lds_insert(keys, vals, LG, c, self);
    wave_sync();
    // emit the row: group exclusive scan of per-lane occupied counts
    int cnt = 0;
    for (int s = gl; s < TS; s += G) cnt += (keys[s] != kEmpty);
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int t = __shfl_up(incl, o, G);
      if (gl >= o) incl += t;
    }
    const int total = __shfl(incl, G - 1, G);
    int32_t pos = a.yoff[c] + (incl - cnt);
    for (int s = gl; s < TS; s += G) {
      const int32_t d = keys[s];
      if (d == kEmpty) continue;
      a.yidx[pos] = d;
      yw[pos] = (WTout)vals[s];
      ++pos;
    }
    if (gl == 0) { a.ydeg[c] = total; no += (unsigned long long)total; }
    wave_sync();
    for (int s = gl; s < TS; s += G) { keys[s] = kEmpty; vals[s] = 0.0; }
    wave_sync();
  }
  nv = block_sum<unsigned long long>(nv, red_u);
  na = block_sum<unsigned long long>(na, red_u);
  no = block_sum<unsigned long long>(no, red_u);
  if (threadIdx.x == 0) {
    if (nv) atomicAdd(&cnt_of(a.cnt)[4], nv);
    if (na) atomicAdd(&cnt_of(a.cnt)[5], na);
    if (no) atomicAdd(&cnt_of(a.cnt)[6], no);
  }
}

// One workgroup of NT threads per community, LDS table of up to TS slots
// (2 cap slots rounded up to whole multiples of NT, at most TS; the bins
// keep cap <= 2 TS / 3, so the load factor stays <= 2/3 and the table never
// fills: a row has at most cap distinct keys).  The members' rows are laid
// end to end, NT members at a time, and every lane takes one arc per step
// (row of an arc by binary search over the members' offsets in LDS), so
// short and long member rows alike stream coalesced.  Used for capacities
// kBinMax[4] < cap <= kBinMax[5] (NT = 256) and kBinMax[5] < cap <=
// kBinMax[kAggLastBin] (NT = 1024, kWideSlots slots).
constexpr int kAggWideThreads = 1024;
template <class WTin, class WTout, int NT, int TS>
__global__ __launch_bounds__(NT) void k_agg_rows(GraphView<WTin> g, AggArgs a, const int32_t* __restrict__ list,
                                                 int32_t count) {
  constexpr int NW = NT / kWave;
  constexpr int R = TS / NT;  // emit rounds
  static_assert(TS % NT == 0, "whole rounds");
  static_assert(R * NW <= 3 * kWave, "emit scan: at most three entries per lane");
  __shared__ int32_t keys[TS];
  __shared__ double vals[TS];
  __shared__ int32_t s_off[NT + 1];
  __shared__ int32_t s_beg[NT];
  __shared__ int32_t s_w[NW];
  __shared__ int32_t s_cnt[3 * kWave];
  __shared__ double s_red[NW];
  __shared__ unsigned long long red_u[16];
  WTout* yw = (WTout*)a.yw;
  const int t = threadIdx.x;
  const int w = t / kWave;
  for (int s = t; s < TS; s += NT) { keys[s] = kEmpty; vals[s] = 0.0; }
  unsigned long long nv = 0, na = 0, no = 0;
  for (int64_t v = blockIdx.x; v < count; v += gridDim.x) {
    const int32_t c = list[v];
    const int32_t mb = a.coff[c], me = a.coff[c + 1];
    const int64_t cap = (int64_t)a.yoff[c + 1] - a.yoff[c];
    int ts = TS;
    if (2 * cap < ts) ts = (int)(((2 * cap + NT - 1) / NT) * NT);
    double self = 0.0;  // arcs inside c: the super-vertex's self-loop
    for (int32_t kb = mb; kb < me; kb += NT) {  // uniform
      const int32_t k = kb + t;
      int32_t deg = 0, beg = 0;
      if (k < me) {
        const int32_t i = a.cv[k];
        beg = g.begin(i);
        deg = g.degree(i);
        ++nv;
      }
      int incl = deg;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int x = __shfl_up(incl, o);
        if (lane_id() >= o) incl += x;
      }
      __syncthreads();  // the previous members' s_off / s_beg are no longer read
      if (lane_id() == kWave - 1) s_w[w] = incl;
      __syncthreads();
      int before = 0, total = 0;
      for (int q = 0; q < NW; ++q) {
        if (q < w) before += s_w[q];
        total += s_w[q];
      }
      s_off[t] = before + incl - deg;
      if (t == 0) s_off[NT] = total;
      s_beg[t] = beg;
      __syncthreads();
      na += (unsigned long long)deg;
      for (int32_t q0 = t; q0 < total; q0 += kAggUnroll * NT) {  // uniform
        int32_t j[kAggUnroll];
        WTin wr[kAggUnroll];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) {
          const int32_t q = q0 + u * NT;
          j[u] = 0;  // (past the arcs: an unused, valid label load)
          wr[u] = WTin(0);
          if (q < total) {
            int lo = 0, hi = NT;  // s_off[lo] <= q < s_off[hi]
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (s_off[mid] <= q) lo = mid; else hi = mid;
            }
            const int64_t e = (int64_t)s_beg[lo] + (q - s_off[lo]);
            j[u] = g.idx[e];
            wr[u] = g.weight(e);
          }
        }
        int32_t d[kAggUnroll];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) d[u] = a.lab[j[u]];
#pragma unroll
        for (int u = 0; u < kAggUnroll; ++u) {
          if (q0 + u * NT >= total) continue;
          const double wt = (double)wr[u];
          if (d[u] == c) self += wt;
          else lds_insert_sized(keys, vals, (uint32_t)ts, d[u], wt);
        }
      }
    }
    self = block_sum<double>(self, s_red);
    if (t == 0 && self != 0.0) lds_insert_sized(keys, vals, (uint32_t)ts, c, self);
    __syncthreads();
    // emit: round r covers slots [r NT, (r + 1) NT); entries of (round,
    // wavefront) are written contiguously
    int32_t key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = r * NT + t;
      key[r] = (s < ts) ? keys[s] : kEmpty;
      const u64 b = __ballot(key[r] != kEmpty);
      if (lane_id() == 0) s_cnt[r * NW + w] = __popcll(b);
    }
    for (int q = R * NW + t; q < 3 * kWave; q += NT) s_cnt[q] = 0;
    __syncthreads();
    if (w == 0) {
      const int v0 = s_cnt[3 * lane_id()], v1 = s_cnt[3 * lane_id() + 1], v2 = s_cnt[3 * lane_id() + 2];
      int incl = v0 + v1 + v2;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int x = __shfl_up(incl, o);
        if (lane_id() >= o) incl += x;
      }
      const int excl = incl - v0 - v1 - v2;
      s_cnt[3 * lane_id()] = excl;
      s_cnt[3 * lane_id() + 1] = excl + v0;
      s_cnt[3 * lane_id() + 2] = excl + v0 + v1;
      if (lane_id() == kWave - 1) {
        a.ydeg[c] = incl;
        no += (unsigned long long)incl;
      }
    }
    __syncthreads();
    const int64_t base = a.yoff[c];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const u64 b = __ballot(key[r] != kEmpty);
      if (key[r] != kEmpty) {
        const int s = r * NT + t;
        const int64_t pos = base + s_cnt[r * NW + w] + __popcll(b & lanemask_lt());
        a.yidx[pos] = key[r];
        yw[pos] = (WTout)vals[s];
        keys[s] = kEmpty;
        vals[s] = 0.0;
      }
    }
    __syncthreads();  // table empty again; s_cnt reusable
  }
  nv = block_sum<unsigned long long>(nv, red_u);
  na = block_sum<unsigned long long>(na, red_u);
  if (t == 0) {
    if (nv) atomicAdd(&cnt_of(a.cnt)[4], nv);
    if (na) atomicAdd(&cnt_of(a.cnt)[5], na);
  }
  if (t == kWave - 1 && no) atomicAdd(&cnt_of(a.cnt)[6], no);
}

template <class WTin, class WTout>
static void agg_bins(hipStream_t st, const GraphDesc& gd, const AggArgs& a, const int32_t* list,
                     const int32_t* count, const int32_t* start, int grid_cap, int hub_grid, int64_t* launches) {
  GraphView<WTin> g;
  g.n = gd.n; g.off = gd.off; g.deg = gd.deg; g.idx = gd.idx; g.w = (const WTin*)gd.w;
  auto grid_for = [&](int64_t items, int per_block, int cap) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
  };
#define GVL_AGG_BIN(B, G, LG)                                                                   \
  if (count[B] > 0) {                                                                      \
    hipLaunchKernelGGL((k_agg_group<WTin, WTout, G, LG>),                                       \
                       dim3(grid_for(count[B], kBlock / (G), grid_cap)), dim3(kBlock), 0, st, \
                       g, a, list + start[B], count[B]);                              \
    ++*launches;                                                                                \
  }
  GVL_AGG_BIN(0, kBinLanes[0], 3)
  GVL_AGG_BIN(1, kBinLanes[1], 4)
  GVL_AGG_BIN(2, kBinLanes[2], 5)
  GVL_AGG_BIN(3, kBinLanes[3], 6)
  GVL_AGG_BIN(4, kBinLanes[4], 8)
#undef GVL_AGG_BIN
  if (count[5] > 0) {
    hipLaunchKernelGGL((k_agg_rows<WTin, WTout, kBlock, 2048>), dim3(grid_for(count[5], 1, grid_cap)),
                       dim3(kBlock), 0, st, g, a, list + start[5], count[5]);
    ++*launches;
  }
  // bins kWideBin0 .. kAggLastBin are contiguous in the list (one group)
  int32_t nwide = 0;
  for (int b = kWideBin0; b <= kAggLastBin; ++b) nwide += count[b];
  if (nwide > 0) {
    hipLaunchKernelGGL((k_agg_rows<WTin, WTout, kAggWideThreads, kWideSlots>), dim3(grid_for(nwide, 1, grid_cap)),
                       dim3(kAggWideThreads), 0, st, g, a, list + start[kWideBin0], nwide);
    ++*launches;
  }
  (void)hub_grid;  // giant communities go through the chunked hub path
}

void launch_agg_rows(hipStream_t st, const GraphDesc& g, const AggArgs& a, const int32_t* list,
                     const int32_t* count, const int32_t* start, int grid_cap, int hub_grid,
                     int64_t* launches) {
  if (g.w_double) {
    agg_bins<double, double>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
  } else if (a.yw_double) {
    agg_bins<float, double>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
  } else {
    agg_bins<float, float>(st, g, a, list, count, start, grid_cap, hub_grid, launches);
  }
}

}  // namespace gvl
