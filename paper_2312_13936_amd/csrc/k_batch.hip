// Kernels of the fused batch: many graphs run as one disjoint union.
//
// The union graph holds the graphs side by side (graph g's vertices are
// [vbase[g], vbase[g] + n_g) in every pass); gid[i] names the graph of
// vertex i.  Every kernel of the single-graph path runs on the union
// unchanged except where a graph's own constants enter (gains, the vertex
// groups, the stop tests), so each graph follows exactly the steps it
// follows alone.
#include "device.hpp"
#include "kernels.hpp"

namespace gvl {

static inline int grid_b(int64_t n, int per = kBlock, int cap = 16384) {
  int64_t b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

// Graph of global item v: the last g with base[g] <= v (base sorted, G + 1
// entries, base[G] = total).
__device__ __forceinline__ int32_t graph_of(const int64_t* base, int32_t G, int64_t v) {
  int32_t lo = 0, hi = G;  // base[lo] <= v < base[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (base[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------ validation ---
// Over the vertices of every graph (concatenated, vertex v of the batch in
// graph g = graph_of(vb, v)): offsets start at 0, never decrease and end at
// m_g; neighbours lie in [0, n_g); weights are positive and finite (flag
// bit 1 otherwise), integers in [1, 2^24] (bit 2 otherwise); W[g] += row
// sums.  flags bit 0: bad CSR; bit 3: a row of more than kAutoShortRow arcs
// (the automatic sub-sweep count).
__global__ __launch_bounds__(kBlock) void k_batch_validate(BatchDesc d, int32_t G, int64_t total, int32_t* flags,
                                                           double* W) {
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < total; base += (int64_t)gridDim.x * kBlock) {
    const int64_t v = base + threadIdx.x;
    const bool on = v < total;
    int32_t g = 0, beg = 0, deg = 0, f = 0;
    int64_t n = 0;
    if (on) {
      g = graph_of(d.vb, G, v);
      const int64_t k = v - d.vb[g];
      n = d.n[g];
      const int32_t* off = d.off[g];
      beg = off[k];
      const int32_t end = off[k + 1];
      // rows are read only inside [0, m): a bad offset is flagged, not followed
      if ((k == 0 && beg != 0) || beg < 0 || end < beg || (int64_t)end > d.m[g] ||
          (k == n - 1 && (int64_t)end != d.m[g]))
        f |= 1;
      deg = (f & 1) ? 0 : end - beg;
      if (deg > kAutoShortRow) f |= 8;
    }
    double s = 0.0;
    const float* w = on ? d.w[g] : nullptr;
    const int32_t* idx = on ? d.idx[g] : nullptr;
    if (deg < kWave) {
      for (int32_t e = 0; e < deg; ++e) {
        const int32_t j = idx[beg + e];
        if (j < 0 || (int64_t)j >= n) f |= 1;
        const double x = w ? (double)w[beg + e] : 1.0;
        if (!(x > 0.0 && x < INFINITY)) f |= 2;
        if (!(x >= 1.0 && x <= 16777216.0 && x == floor(x))) f |= 4;
        s += x;
      }
    }
    u64 mask = __ballot(on && deg >= kWave);
    while (mask) {
      const int q = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const int32_t gq = __shfl(g, q), bq = __shfl(beg, q), dq = __shfl(deg, q);
      const int64_t nq = (int64_t)__shfl((long long)n, q);
      const int32_t* iq = d.idx[gq];
      const float* wq = d.w[gq];
      double part = 0.0;
      int fq = 0;
      for (int32_t e = lane_id(); e < dq; e += kWave) {
        const int32_t j = iq[bq + e];
        if (j < 0 || (int64_t)j >= nq) fq |= 1;
        const double x = wq ? (double)wq[bq + e] : 1.0;
        if (!(x > 0.0 && x < INFINITY)) fq |= 2;
        if (!(x >= 1.0 && x <= 16777216.0 && x == floor(x))) fq |= 4;
        part += x;
      }
      part = sum_xor<kWave>(part);
      if (fq) atomicOr(&flags[gq], fq);
      if (lane_id() == q) s = part;
    }
    if (f) atomicOr(&flags[g], f);
    atomic_add_keyed<double>(W, g, s, on && s != 0.0);
  }
}
void batch_validate(hipStream_t st, const BatchDesc& d, int32_t G, int64_t total, int32_t* flags, double* W) {
  if (total > 0)
    hipLaunchKernelGGL(k_batch_validate, dim3(grid_b(total)), dim3(kBlock), 0, st, d, G, total, flags, W);
}

// ------------------------------------------------------------ union build ---
// Vertex v of the union belongs to kept graph g (vertex k = v - vb[g] of
// desc graph src[g]): uoff[v] = ab[g] + off[k], neighbours shifted by vb[g],
// weights copied (1 for unit-weight graphs), gid[v] = g.
__global__ __launch_bounds__(kBlock) void k_batch_build(BatchDesc d, const int32_t* src, int32_t G, int64_t total,
                                                        int32_t* uoff, int32_t* uidx, float* uw, int32_t* gid) {
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < total; base += (int64_t)gridDim.x * kBlock) {
    const int64_t v = base + threadIdx.x;
    const bool on = v < total;
    int32_t g = 0, s = 0, beg = 0, deg = 0, nb = 0;
    if (on) {
      g = graph_of(d.ub, G, v);
      s = src[g];
      const int64_t k = v - d.ub[g];
      const int32_t* off = d.off[s];
      beg = off[k];
      deg = off[k + 1] - beg;
      nb = (int32_t)(d.uab[g] + beg);
      uoff[v] = nb;
      gid[v] = g;
    }
    if (deg < kWave) {
      const int32_t shift = (int32_t)d.ub[g];
      for (int32_t e = 0; e < deg; ++e) {
        uidx[nb + e] = d.idx[s][beg + e] + shift;
        uw[nb + e] = d.w[s] ? d.w[s][beg + e] : 1.0f;
      }
    }
    u64 mask = __ballot(on && deg >= kWave);
    while (mask) {
      const int q = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const int32_t gq = __shfl(g, q), sq = __shfl(s, q), bq = __shfl(beg, q), dq = __shfl(deg, q),
                    nq = __shfl(nb, q);
      const int32_t shift = (int32_t)d.ub[gq];
      const int32_t* iq = d.idx[sq];
      const float* wq = d.w[sq];
      for (int32_t e = lane_id(); e < dq; e += kWave) {
        uidx[nq + e] = iq[bq + e] + shift;
        uw[nq + e] = wq ? wq[bq + e] : 1.0f;
      }
    }
  }
}
void batch_build(hipStream_t st, const BatchDesc& d, const int32_t* src, int32_t G, int64_t total, int32_t* uoff,
                 int32_t* uidx, float* uw, int32_t* gid) {
  if (total > 0)
    hipLaunchKernelGGL(k_batch_build, dim3(grid_b(total)), dim3(kBlock), 0, st, d, src, G, total, uoff, uidx, uw,
                       gid);
}

// --------------------------------------------------------- pass helpers ---
// flag[i] = 0 for vertices of graphs whose local-moving has stopped.
__global__ void k_mask_flags(uint8_t* flag, const int32_t* gid, const uint8_t* active, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!active[gid[i]]) flag[i] = 0;
}
void mask_flags(hipStream_t st, uint8_t* flag, const int32_t* gid, const uint8_t* active, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_mask_flags, dim3(grid_b(n)), dim3(kBlock), 0, st, flag, gid, active, n);
}

// nz[g] += 1 for every vertex of graph g with at least one arc.
template <class WT>
__global__ void k_graph_nonzero(GraphView<WT> g, const int32_t* gid, int32_t* nz) {
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < g.n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool on = i < g.n && g.degree(i) > 0;
    atomic_add_keyed<int32_t>(nz, on ? gid[i] : 0, 1, on);
  }
}
void graph_nonzero(hipStream_t st, const GraphDesc& gd, const int32_t* gid, int32_t* nz) {
  if (gd.n <= 0) return;
  GraphView<float> g{gd.n, gd.off, gd.deg, gd.idx, nullptr};
  hipLaunchKernelGGL(k_graph_nonzero<float>, dim3(grid_b(gd.n)), dim3(kBlock), 0, st, g, gid, nz);
}

// out[g] = data[pos[g]] for g < count.
__global__ void k_gather_at(const int32_t* data, const int32_t* pos, int32_t count, int32_t* out) {
  for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < count; g += gridDim.x * blockDim.x)
    out[g] = data[pos[g]];
}
void gather_at(hipStream_t st, const int32_t* data, const int32_t* pos, int32_t count, int32_t* out) {
  if (count > 0) hipLaunchKernelGGL(k_gather_at, dim3(grid_b(count)), dim3(kBlock), 0, st, data, pos, count, out);
}

// gid_next[newid[C[i]]] = gid[i] for vertices of continuing graphs.
__global__ void k_gid_next(const int32_t* C, const int32_t* newid, const int32_t* gid, const uint8_t* keep,
                           int64_t n, int32_t* gid_next) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = gid[i];
    if (keep[g]) gid_next[newid[C[i]]] = g;
  }
}
void gid_next(hipStream_t st, const int32_t* C, const int32_t* newid, const int32_t* gid, const uint8_t* keep,
              int64_t n, int32_t* out) {
  if (n > 0) hipLaunchKernelGGL(k_gid_next, dim3(grid_b(n)), dim3(kBlock), 0, st, C, newid, gid, keep, n, out);
}

// Dendrogram lookup of the batch (over the original union vertices v, graph
// gid0[v]): continuing graphs take the renumbered label, graphs that end
// this pass take their refined label moved into the graph's own range
// [goff0[g], goff0[g] + n_g) (label - vcur[g] + goff0[g]), finished graphs
// are left alone.  first: top[v] is v itself (pass 0).
__global__ void k_lookup_batch(int32_t* top, int64_t N, const int32_t* C, const int32_t* newid, const int32_t* gid0,
                               const uint8_t* state, const int32_t* vcur, const int32_t* goff0, int first) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = gid0[v];
    const uint8_t s = state[g];
    if (s == kBatchDone) continue;
    const int32_t t = first ? (int32_t)v : top[v];
    top[v] = (s == kBatchCont) ? newid[C[t]] : C[t] - vcur[g] + goff0[g];
  }
}
void lookup_batch(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, const int32_t* newid,
                  const int32_t* gid0, const uint8_t* state, const int32_t* vcur, const int32_t* goff0, bool first) {
  if (N > 0)
    hipLaunchKernelGGL(k_lookup_batch, dim3(grid_b(N)), dim3(kBlock), 0, st, top, N, C, newid, gid0, state, vcur,
                       goff0, (int)first);
}

// Results: out[g][v - goff0[g]] = canon[v] - canon[goff0[g]] (labels of each
// graph counted from 0 in first-occurrence order).
__global__ void k_batch_outputs(const int32_t* canon, int64_t N, const int32_t* gid0, const int32_t* goff0,
                                int32_t* const* out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = gid0[v];
    out[g][v - goff0[g]] = canon[v] - canon[goff0[g]];
  }
}
void batch_outputs(hipStream_t st, const int32_t* canon, int64_t N, const int32_t* gid0, const int32_t* goff0,
                   int32_t* const* out) {
  if (N > 0) hipLaunchKernelGGL(k_batch_outputs, dim3(grid_b(N)), dim3(kBlock), 0, st, canon, N, gid0, goff0, out);
}

// Eq. 1 per graph, second half: S2[g] = sum over the graph's communities c
// (canonical ids [cb[g], cb[g + 1])) of tot[c]^2, exact (int128) and FP64.
__global__ __launch_bounds__(kBlock) void k_mod_squares_batch(const double* tot, int64_t n, const int32_t* cb,
                                                              int32_t G, double* s2d, unsigned long long* s2u) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = G;  // cb[lo] <= c < cb[hi]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (cb[mid] <= c) lo = mid; else hi = mid;
    }
    const double t = tot[c];
    if (t == 0.0) continue;
    atomicAdd(&s2d[lo], t * t);
    const long long ti = (long long)t;
    atomic_add_i128(s2u + 2 * lo, (i128)ti * (i128)ti);
  }
}
void mod_squares_batch(hipStream_t st, const double* tot, int64_t n, const int32_t* cb, int32_t G, double* s2d,
                       unsigned long long* s2u) {
  if (n > 0)
    hipLaunchKernelGGL(k_mod_squares_batch, dim3(grid_b(n)), dim3(kBlock), 0, st, tot, n, cb, G, s2d, s2u);
}

}  // namespace gvl
