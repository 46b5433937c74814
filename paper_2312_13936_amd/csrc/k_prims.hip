// Primitives of the pass loop (Alg. 1): vertex weights, community totals,
// degree binning, device-wide exclusive scan, renumbering, dendrogram
// lookup, community-vertex CSR (Alg. 4, first half), move-based labels,
// canonical relabelling and the modularity of Eq. 1.
#include "device.hpp"
#include "kernels.hpp"

namespace gvl {

static inline int grid_n(int64_t n, int per_block = kBlock, int cap = 16384) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ fills ---
template <class T>
__global__ void k_fill(T* p, T v, int64_t n) { GRID_STRIDE(i, n) p[i] = v; }
__global__ void k_iota(int32_t* p, int64_t n) { GRID_STRIDE(i, n) p[i] = (int32_t)i; }
template <class T>
__global__ void k_copy(T* d, const T* s, int64_t n) { GRID_STRIDE(i, n) d[i] = s[i]; }

void fill_i32(hipStream_t st, int32_t* p, int32_t v, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_n(n)), dim3(kBlock), 0, st, p, v, n);
}
void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_n(n)), dim3(kBlock), 0, st, p, v, n);
}
void fill_f64(hipStream_t st, double* p, double v, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill<double>, dim3(grid_n(n)), dim3(kBlock), 0, st, p, v, n);
}
__global__ void k_fill_slots(TblSlot* p, int64_t n) {
  GRID_STRIDE(k, n) p[k] = TblSlot{kEmpty, 0, 0.0};
}
void fill_slots(hipStream_t st, TblSlot* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill_slots, dim3(grid_n(n)), dim3(kBlock), 0, st, p, n);
}
void fill_u64(hipStream_t st, unsigned long long* p, unsigned long long v, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid_n(n)), dim3(kBlock), 0, st, p, v, n);
}
void iota_i32(hipStream_t st, int32_t* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(grid_n(n)), dim3(kBlock), 0, st, p, n);
}
__global__ void k_add_one(int32_t* p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p += 1;
}
void add_one_i32(hipStream_t st, int32_t* p) { hipLaunchKernelGGL(k_add_one, dim3(1), dim3(64), 0, st, p); }
void copy_i32(hipStream_t st, int32_t* d, const int32_t* s, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_copy<int32_t>, dim3(grid_n(n)), dim3(kBlock), 0, st, d, s, n);
}
__global__ void k_pack_labels(const int32_t* C, const int32_t* CB, int2* CP, int64_t n) {
  GRID_STRIDE(i, n) CP[i] = make_int2(C[i], CB[i]);
}
void pack_labels(hipStream_t st, const int32_t* C, const int32_t* CB, int2* CP, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_pack_labels, dim3(grid_n(n)), dim3(kBlock), 0, st, C, CB, CP, n);
}
// ------------------------------------------------- refinement thinning ---
// Alg. 3 moves only vertices alone in their refined community, and a
// refined community never drops back to one member (only lone vertices
// leave theirs), so a vertex that has company stays out for the rest of the
// refinement.
__device__ __forceinline__ bool still_alone(const int32_t* C, const int32_t* size, const double* K, int32_t i) {
  return size[C[i]] == 1 && K[i] > 0.0;
}
constexpr int kThinTiles = 64;  // workgroups per segment
__global__ __launch_bounds__(kBlock) void k_thin_count(const int32_t* list, BinBuf* bb, const int32_t* C,
                                                       const int32_t* size, const double* K) {
  const int s = (int)blockIdx.y;  // every bin, hubs included (they are counted, not moved)
  const int32_t beg = bb->cursors[s], cnt = bb->counts[s];
  int32_t mine = 0;
  for (int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x); k < cnt; k += kThinTiles * kBlock)
    mine += still_alone(C, size, K, list[beg + k]) ? 1 : 0;
  __shared__ int32_t red[kBlock / kWave];
  const int32_t tot = block_sum<int32_t>(mine, red);
  if (threadIdx.x == 0 && tot) atomicAdd(&bb->kept[s], tot);
}
__global__ __launch_bounds__(kBlock) void k_thin_scatter(const int32_t* list, BinBuf* bb, const int32_t* C,
                                                         const int32_t* size, const double* K, int32_t* out) {
  const int s = (int)(blockIdx.y / kHubBin) * kNumBins + (int)(blockIdx.y % kHubBin);
  const int32_t beg = bb->cursors[s], cnt = bb->counts[s], dst = bb->nstart[s], lim = bb->kept[s];
  __shared__ int32_t s_w[kBlock / kWave];
  __shared__ int32_t s_base;
  for (int32_t k0 = (int32_t)(blockIdx.x * kBlock); k0 < cnt; k0 += kThinTiles * kBlock) {  // uniform
    const int32_t k = k0 + (int32_t)threadIdx.x;
    const int32_t i = (k < cnt) ? list[beg + k] : -1;
    const bool keep = i >= 0 && still_alone(C, size, K, i);
    const u64 bal = __ballot(keep);
    const int wv = threadIdx.x / kWave;
    const int lr = __popcll(bal & ((1ull << lane_id()) - 1ull));
    if (lane_id() == 0) s_w[wv] = __popcll(bal);
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < kBlock / kWave; ++q) {
      if (q < wv) before += s_w[q];
      total += s_w[q];
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(&bb->ncur[s], total) : 0;
    __syncthreads();
    const int32_t q = s_base + before + lr;
    if (keep && q < lim) out[dst + q] = i;  // (the count pass saw the same state: q < lim always)
    __syncthreads();  // s_w / s_base are rewritten by the next tile
  }
}
void thin_count(hipStream_t st, const int32_t* list, BinBuf* bb, int S, const int32_t* C, const int32_t* size,
                const double* K) {
  hipLaunchKernelGGL(k_thin_count, dim3(kThinTiles, S * kNumBins), dim3(kBlock), 0, st, list, bb, C, size, K);
}
void thin_scatter(hipStream_t st, const int32_t* list, BinBuf* bb, int S, const int32_t* C, const int32_t* size,
                  const double* K, int32_t* out) {
  hipLaunchKernelGGL(k_thin_scatter, dim3(kThinTiles, S * kHubBin), dim3(kBlock), 0, st, list, bb, C, size, K,
                     out);
}

void copy_f64(hipStream_t st, double* d, const double* s, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_copy<double>, dim3(grid_n(n)), dim3(kBlock), 0, st, d, s, n);
}
void set_size_one(hipStream_t st, int32_t* size, int64_t n) { fill_i32(st, size, 1, n); }

// ---------------------------------------------------------- vertex weights ---
// K[i] = sum of the weights of row i (a self-loop is stored, and counted,
// once).  Also reduces W = sum K and checks the input.
template <class WT>
__global__ __launch_bounds__(kBlock) void k_vertex_weights(GraphView<WT> g, int64_t m, double* K,
                                                           double* accW, int32_t* flags, int validate) {
  __shared__ double red[16];
  double wsum = 0.0;
  int bad_csr = 0, bad_w = 0, bad_sign = 0;
  // a wavefront walks 64 vertices: short rows one lane each, long rows together
  const int64_t n = g.n;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    int32_t beg = 0, deg = 0;
    if (i < n) {
      beg = g.begin(i);
      deg = g.degree(i);
      if (validate && (deg < 0 || beg < 0 || (int64_t)beg + deg > m)) { bad_csr = 1; deg = 0; }
      if (deg > kBinMax[kHubBin - 1]) deg = 0;  // hub rows: hub_weights
    }
    // four arcs per step, their loads issued before the first use
    constexpr int U = 4;
    auto step = [&](int32_t b0, int32_t e0, int32_t stride, int32_t end, double& acc) {
      WT wr[U];
      int32_t j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        wr[u] = WT(1);
        j[u] = 0;
        if (e0 + u * stride < end) {
          wr[u] = g.weight(b0 + e0 + u * stride);
          if (validate) j[u] = g.idx[b0 + e0 + u * stride];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u * stride >= end) continue;
        const double w = (double)wr[u];
        if (validate && (j[u] < 0 || j[u] >= n)) bad_csr = 1;
        if (!(w >= 1.0 && w <= 16777216.0 && w == floor(w))) bad_w = 1;
        if (!(w > 0.0 && w < INFINITY)) bad_sign = 1;
        acc += w;
      }
    };
    double s = 0.0;
    if (deg < kWave)
      for (int32_t e = 0; e < deg; e += U) step(beg, e, 1, deg, s);
    u64 mask = __ballot(i < n && deg >= kWave);
    while (mask) {
      const int q = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const int32_t bq = __shfl(beg, q), dq = __shfl(deg, q);
      double part = 0.0;
      for (int32_t e = lane_id(); e < dq; e += U * kWave) step(bq, e, kWave, dq, part);
      part = sum_xor<kWave>(part);
      if (lane_id() == q) s = part;
    }
    if (i < n) {
      K[i] = s;
      wsum += s;
    }
  }
  const double t = block_sum<double>(wsum, red);
  if (threadIdx.x == 0) atomicAdd(accW, t);
  if (bad_csr) atomicOr(&flags[0], 1);
  if (bad_w) atomicOr(&flags[1], 1);
  if (bad_sign) atomicOr(&flags[2], 1);
}

void vertex_weights(hipStream_t st, const GraphDesc& gd, int64_t m, double* K, double* accW,
                    int32_t* flags, int validate) {
  if (gd.n <= 0) return;
  if (gd.w_double) {
    GraphView<double> g{gd.n, gd.off, gd.deg, gd.idx, (const double*)gd.w};
    hipLaunchKernelGGL(k_vertex_weights<double>, dim3(grid_n(gd.n, kBlock, 2048)), dim3(kBlock), 0, st,
                       g, m, K, accW, flags, validate);
  } else {
    GraphView<float> g{gd.n, gd.off, gd.deg, gd.idx, (const float*)gd.w};
    hipLaunchKernelGGL(k_vertex_weights<float>, dim3(grid_n(gd.n, kBlock, 2048)), dim3(kBlock), 0, st,
                       g, m, K, accW, flags, validate);
  }
}

__global__ void k_check_offsets(const int32_t* off, int64_t n, int64_t m, int32_t* flags) {
  GRID_STRIDE(i, n) {
    if (off[i] > off[i + 1]) atomicOr(&flags[0], 1);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (off[0] != 0 || off[n] != m) atomicOr(&flags[0], 1);
  }
}

// Symmetry check (validate = 2): one wavefront per row, acc[0..1] += the
// row's multiset-hash differences (zero in total for a symmetric CSR).
// Offsets must have been checked (rows stay inside [0, m)); neighbour ids
// are hashed, never followed.
__global__ __launch_bounds__(kBlock) void k_symmetry(const int32_t* off, const int32_t* idx, const float* w, int64_t n,
                                                     unsigned long long* acc) {
  u64 d0 = 0, d1 = 0;
  const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < n; i += nw) {
    const int32_t beg = off[i], end = off[i + 1];
    for (int32_t e = beg + lane_id(); e < end; e += kWave)
      arc_sym((int32_t)i, idx[e], w ? __float_as_uint(w[e]) : 0x3f800000u, d0, d1);
  }
  d0 = sum_xor<kWave>(d0);
  d1 = sum_xor<kWave>(d1);
  if (lane_id() == 0) {
    if (d0) atomicAdd(&acc[0], (unsigned long long)d0);
    if (d1) atomicAdd(&acc[1], (unsigned long long)d1);
  }
}
void symmetry_check(hipStream_t st, const int32_t* off, const int32_t* idx, const float* w, int64_t n,
                    unsigned long long* acc) {
  if (n > 0) hipLaunchKernelGGL(k_symmetry, dim3(grid_n(n, kBlock / kWave)), dim3(kBlock), 0, st, off, idx, w, n, acc);
}

// ------------------------------------------------------- community totals ---
__global__ __launch_bounds__(kBlock) void k_community_totals(const int32_t* C, const double* K, double* Sig,
                                                             int32_t* size, int64_t n) {
  __shared__ KeyedLds<kBlock> kt;
  keyed_clear(kt);
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    if (i < n) keyed_put(kt, C[i], K[i], 1);
    keyed_flush(kt, Sig, size);
  }
}
void community_totals(hipStream_t st, const int32_t* C, const double* K, double* Sig, int32_t* size,
                      int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_community_totals, dim3(grid_n(n)), dim3(kBlock), 0, st, C, K, Sig, size, n);
}

// ---------------------------------------------------------------- binning ---
__device__ __forceinline__ int bin_of(int32_t d, bool wide, const BinLimits& lim) {
  if (d <= 0) return -1;
#pragma unroll
  for (int b = 0; b < kNumBins; ++b) {
    if (!wide && b > kAggLastBin) return kHubBin;
    if (d <= lim.v[b]) return b;
  }
  return kHubBin;
}

__device__ __forceinline__ int32_t size_of(const int32_t* off, const int32_t* deg, int64_t i) {
  return deg ? deg[i] : off[i + 1] - off[i];
}

// Binning key of item i: group_of(i, S) * kNumBins + bin(size).  Counts
// per key and the largest size per bin go to bb.
__device__ __forceinline__ int group_local(int64_t i, int S, const int32_t* gid, const int32_t* vbase,
                                           const int32_t* gsh) {
  if (!gid) return group_of(i, S);
  const int32_t g = gid[i];
  const int sh = gsh ? gsh[g] : 0;
  return group_of(i - vbase[g], S >> sh) << sh;
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const int32_t* off, const int32_t* deg, int64_t n, int S,
                                                      bool wide, const int32_t* gid, const int32_t* vbase,
                                                      const int32_t* gsh, BinLimits lim, BinBuf* bb) {
  __shared__ int32_t h[kMaxGroups * kNumBins], mx[kNumBins];
  const int nk = S * kNumBins;
  for (int k = threadIdx.x; k < nk; k += kBlock) h[k] = 0;
  if (threadIdx.x < kNumBins) mx[threadIdx.x] = 0;
  __syncthreads();
  GRID_STRIDE(i, n) {
    const int32_t d = size_of(off, deg, i);
    const int b = bin_of(d, wide, lim);
    if (b >= 0) {
      const int grp = (S > 1) ? group_local(i, S, gid, vbase, gsh) : 0;
      atomicAdd(&h[grp * kNumBins + b], 1);
      atomicMax(&mx[b], d);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nk; k += kBlock)
    if (h[k]) atomicAdd(&bb->counts[k], h[k]);
  if (threadIdx.x < kNumBins && mx[threadIdx.x]) atomicMax(&bb->maxsize[threadIdx.x], mx[threadIdx.x]);
}
void bin_count(hipStream_t st, const int32_t* off, const int32_t* deg, int64_t n, int S, bool wide,
               const int32_t* gid, const int32_t* vbase, const int32_t* gsh, const BinLimits& lim, BinBuf* bb) {
  if (n > 0)
    hipLaunchKernelGGL(k_bin_count, dim3(grid_n(n, kBlock, 2048)), dim3(kBlock), 0, st, off, deg, n, S, wide, gid,
                       vbase, gsh, lim, bb);
}

// Each workgroup takes a contiguous chunk of items, reserves room per key
// with one global atomic, then places its items (chunk locality is kept so
// that rows of consecutive list entries sit close together in memory).
constexpr int kBinChunk = 4096;
__global__ __launch_bounds__(kBlock) void k_bin_scatter(const int32_t* off, const int32_t* deg, int64_t n, int S,
                                                        bool wide, const int32_t* gid, const int32_t* vbase,
                                                        const int32_t* gsh, BinLimits lim, BinBuf* bb,
                                                        int32_t* list) {
  __shared__ int32_t h[kMaxGroups * kNumBins], base[kMaxGroups * kNumBins];
  const int nk = S * kNumBins;
  for (int64_t c0 = (int64_t)blockIdx.x * kBinChunk; c0 < n; c0 += (int64_t)gridDim.x * kBinChunk) {
    for (int k = threadIdx.x; k < nk; k += kBlock) h[k] = 0;
    __syncthreads();
    const int64_t c1 = (c0 + kBinChunk < n) ? c0 + kBinChunk : n;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kBlock) {
      const int b = bin_of(size_of(off, deg, i), wide, lim);
      if (b >= 0) atomicAdd(&h[((S > 1) ? group_local(i, S, gid, vbase, gsh) : 0) * kNumBins + b], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += kBlock) {
      base[k] = h[k] ? atomicAdd(&bb->cursors[k], h[k]) : 0;
      h[k] = 0;
    }
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kBlock) {
      const int b = bin_of(size_of(off, deg, i), wide, lim);
      if (b >= 0) {
        const int k = ((S > 1) ? group_local(i, S, gid, vbase, gsh) : 0) * kNumBins + b;
        list[base[k] + atomicAdd(&h[k], 1)] = (int32_t)i;
      }
    }
    __syncthreads();
  }
}
void bin_scatter(hipStream_t st, const int32_t* off, const int32_t* deg, int64_t n, int S, bool wide,
                 const int32_t* gid, const int32_t* vbase, const int32_t* gsh, const BinLimits& lim, BinBuf* bb,
                 int32_t* list) {
  if (n > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid_n(n, kBinChunk, 2048)), dim3(kBlock), 0, st, off, deg, n, S,
                       wide, gid, vbase, gsh, lim, bb, list);
}

// ---------------------------------------------------------- exclusive scan ---
// Three phases over tiles of kScanTile items: tile sums, scan of the tile
// sums by one workgroup, then each tile scans itself from its offset.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

int scan_tiles(int64_t n) { return (int)((n + kScanTile - 1) / kScanTile); }

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ int32_t block_exscan(int32_t v, int32_t* excl, int32_t* wsum) {
  int32_t incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(incl, o);
    if (lane_id() >= o) incl += t;
  }
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  if (threadIdx.x < kWave) {
    int32_t x = (threadIdx.x < nw) ? wsum[threadIdx.x] : 0;
    int32_t y = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t t = __shfl_up(y, o);
      if (lane_id() >= o) y += t;
    }
    if (threadIdx.x < nw) wsum[kWave + threadIdx.x] = y - x;
    if (threadIdx.x == kWave - 1) wsum[2 * kWave] = y;
  }
  __syncthreads();
  *excl = wsum[kWave + w] + incl - v;
  const int32_t total = wsum[2 * kWave];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* data, int64_t n, int32_t* tsum) {
  __shared__ int32_t wsum[2 * kWave + 1];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = t0 + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) s += data[i];
  }
  int32_t ex;
  const int32_t tot = block_exscan(s, &ex, wsum);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tilesums(int32_t* tsum, int32_t ntiles) {
  __shared__ int32_t wsum[2 * kWave + 1];
  int32_t carry = 0;
  for (int32_t b = 0; b < ntiles; b += kScanThreads) {
    const int32_t i = b + threadIdx.x;
    const int32_t v = (i < ntiles) ? tsum[i] : 0;
    int32_t ex;
    const int32_t tot = block_exscan(v, &ex, wsum);
    if (i < ntiles) tsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) tsum[ntiles] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(int32_t* data, int64_t n, const int32_t* tsum,
                                                            int32_t ntiles) {
  __shared__ int32_t wsum[2 * kWave + 1];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  int32_t v[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = t0 + (int64_t)threadIdx.x * kScanItems + k;
    v[k] = (i < n) ? data[i] : 0;
    s += v[k];
  }
  int32_t ex;
  block_exscan(s, &ex, wsum);
  int32_t run = tsum[blockIdx.x] + ex;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = t0 + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) data[i] = run;
    run += v[k];
  }
  if (blockIdx.x == ntiles - 1 && threadIdx.x == 0) data[n] = tsum[ntiles];
}

void exclusive_scan(hipStream_t st, int32_t* data, int64_t n, int32_t* tmp) {
  if (n <= 0) {
    fill_i32(st, data, 0, 1);
    return;
  }
  const int nt = scan_tiles(n);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(kScanThreads), 0, st, data, n, tmp);
  hipLaunchKernelGGL(k_scan_tilesums, dim3(1), dim3(kScanThreads), 0, st, tmp, nt);
  hipLaunchKernelGGL(k_scan_down, dim3(nt), dim3(kScanThreads), 0, st, data, n, tmp, nt);
}

// ------------------------------------------------------------ relabelling ---
__global__ void k_mark_used(const int32_t* C, int64_t n, int32_t* used, const int32_t* gid, const uint8_t* keep) {
  GRID_STRIDE(i, n) if (!gid || keep[gid[i]]) used[C[i]] = 1;
}
void mark_used(hipStream_t st, const int32_t* C, int64_t n, int32_t* used, const int32_t* gid,
               const uint8_t* keep) {
  if (n > 0) hipLaunchKernelGGL(k_mark_used, dim3(grid_n(n)), dim3(kBlock), 0, st, C, n, used, gid, keep);
}

__global__ void k_lookup_top(int32_t* top, int64_t N, const int32_t* C, const int32_t* newid, int first) {
  GRID_STRIDE(v, N) {
    const int32_t t = first ? (int32_t)v : top[v];
    top[v] = newid ? newid[C[t]] : C[t];
  }
}
void lookup_top(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, const int32_t* newid, bool first) {
  if (N > 0) hipLaunchKernelGGL(k_lookup_top, dim3(grid_n(N)), dim3(kBlock), 0, st, top, N, C, newid, (int)first);
}
void lookup_raw(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, bool first) {
  if (N > 0)
    hipLaunchKernelGGL(k_lookup_top, dim3(grid_n(N)), dim3(kBlock), 0, st, top, N, C, (const int32_t*)nullptr,
                       (int)first);
}

// ------------------------------------------------ community-vertex CSR ---
// countCommunityVertices and communityTotalDegree of Alg. 4 in one pass;
// each vertex also keeps its slot inside its community's member list.
template <class WT>
__global__ __launch_bounds__(kBlock) void k_agg_count(GraphView<WT> g, const int32_t* C, const int32_t* newid,
                                                      int32_t* lab, int32_t* rank, int32_t* cnt, int32_t* cap,
                                                      const int32_t* gid, const uint8_t* keep) {
  // The workgroup's vertices are first counted per community in LDS (local
  // rank, members, arcs), then each community present reserves its block of
  // member slots with one global atomic: a community of a million members
  // costs one atomic per workgroup, not one per member on one address.
  constexpr int TS = 2 * kBlock;
  constexpr uint32_t mask = TS - 1;
  __shared__ int32_t skey[TS];
  __shared__ int32_t scnt[TS];
  __shared__ int32_t scap[TS];
  for (int s = threadIdx.x; s < TS; s += kBlock) { skey[s] = kEmpty; scnt[s] = 0; scap[s] = 0; }
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < g.n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    int32_t c = -1, lr = 0;
    uint32_t h = 0;
    if (i < g.n) {
      if (gid && !keep[gid[i]]) {
        lab[i] = -1;
      } else {
        c = newid[C[i]];
        lab[i] = c;
        h = hslot(c, __builtin_ctz(TS));
        while (true) {
          const int32_t k = skey[h];
          if (k == c) break;
          if (k == kEmpty) {
            const int32_t old = atomicCAS(&skey[h], kEmpty, c);
            if (old == kEmpty || old == c) break;
          }
          h = (h + 1u) & mask;
        }
        lr = atomicAdd(&scnt[h], 1);
        const int32_t d = g.degree(i);
        if (d) atomicAdd(&scap[h], d);
      }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < TS; s += kBlock) {
      const int32_t k = skey[s];
      if (k != kEmpty) {
        const int32_t n = scnt[s];
        scnt[s] = atomicAdd(&cnt[k], n);  // the block's first slot
        if (scap[s]) atomicAdd(&cap[k], scap[s]);
      }
    }
    __syncthreads();
    if (c >= 0) rank[i] = scnt[h] + lr;
    __syncthreads();
    for (int s = threadIdx.x; s < TS; s += kBlock) { skey[s] = kEmpty; scnt[s] = 0; scap[s] = 0; }
    __syncthreads();
  }
}
void agg_count(hipStream_t st, const GraphDesc& gd, const int32_t* C, const int32_t* newid, int32_t* lab,
               int32_t* rank, int32_t* cnt, int32_t* cap, const int32_t* gid, const uint8_t* keep) {
  if (gd.n <= 0) return;
  GraphView<float> g{gd.n, gd.off, gd.deg, gd.idx, nullptr};
  hipLaunchKernelGGL(k_agg_count<float>, dim3(grid_n(gd.n, kBlock, 4096)), dim3(kBlock), 0, st, g, C, newid, lab,
                     rank, cnt, cap, gid, keep);
}

__global__ void k_agg_fill(const int32_t* lab, const int32_t* rank, const int32_t* coff, int64_t n,
                           int32_t* cv) {
  GRID_STRIDE(i, n) if (lab[i] >= 0) cv[coff[lab[i]] + rank[i]] = (int32_t)i;
}
void agg_fill(hipStream_t st, const int32_t* lab, const int32_t* rank, const int32_t* coff, int64_t n,
              int32_t* cv) {
  if (n > 0) hipLaunchKernelGGL(k_agg_fill, dim3(grid_n(n)), dim3(kBlock), 0, st, lab, rank, coff, n, cv);
}

// K' of the next pass: super-vertex newid[c] is community c, and its row
// (self-loop included) sums the rows of c's members, i.e. Sigma'_c.
__global__ void k_next_weights(const double* Sig, const int32_t* newid, int64_t n, double* K) {
  GRID_STRIDE(c, n) if (newid[c + 1] != newid[c]) K[newid[c]] = Sig[c];
}
void next_weights(hipStream_t st, const double* Sig, const int32_t* newid, int64_t n, double* K) {
  if (n > 0) hipLaunchKernelGGL(k_next_weights, dim3(grid_n(n)), dim3(kBlock), 0, st, Sig, newid, n, K);
}

__global__ void k_next_labels(const int32_t* lab, const int32_t* CB, const int32_t* brank, int64_t n,
                              int32_t* start) {
  GRID_STRIDE(i, n) if (lab[i] >= 0) start[lab[i]] = brank[CB[i]];
}
void next_labels(hipStream_t st, const int32_t* lab, const int32_t* CB, const int32_t* brank, int64_t n,
                 int32_t* start) {
  if (n > 0) hipLaunchKernelGGL(k_next_labels, dim3(grid_n(n)), dim3(kBlock), 0, st, lab, CB, brank, n, start);
}

// ------------------------------------------------- canonical relabelling ---
__global__ void k_first_occurrence(const int32_t* top, int64_t N, int32_t* first) {
  GRID_STRIDE(v, N) {
    const int32_t c = top[v];
    if (first[c] > (int32_t)v) atomicMin(&first[c], (int32_t)v);
  }
}
void first_occurrence(hipStream_t st, const int32_t* top, int64_t N, int32_t* first) {
  if (N > 0) hipLaunchKernelGGL(k_first_occurrence, dim3(grid_n(N)), dim3(kBlock), 0, st, top, N, first);
}
__global__ void k_first_flags(const int32_t* top, const int32_t* first, int64_t N, int32_t* flags) {
  GRID_STRIDE(v, N) flags[v] = (first[top[v]] == (int32_t)v) ? 1 : 0;
}
void first_flags(hipStream_t st, const int32_t* top, const int32_t* first, int64_t N, int32_t* flags) {
  if (N > 0) hipLaunchKernelGGL(k_first_flags, dim3(grid_n(N)), dim3(kBlock), 0, st, top, first, N, flags);
}
__global__ void k_apply_canonical(int32_t* top, const int32_t* first, const int32_t* scan, int64_t N) {
  GRID_STRIDE(v, N) top[v] = scan[first[top[v]]];
}
void apply_canonical(hipStream_t st, int32_t* top, const int32_t* first, const int32_t* scan, int64_t N) {
  if (N > 0) hipLaunchKernelGGL(k_apply_canonical, dim3(grid_n(N)), dim3(kBlock), 0, st, top, first, scan, N);
}

// ------------------------------------------------------------ modularity ---
// Per vertex i: sigma_i = sum of w_ij over arcs with C[j] == C[i] (into
// acc_d[0]) and tot[C[i]] += K_i with K_i the row sum.
template <class WT>
__global__ __launch_bounds__(kBlock) void k_mod_partial(GraphView<WT> g, const int32_t* C, double* tot,
                                                        double* acc_d, const int32_t* gid, double* s1g) {
  __shared__ double red[16];
  double s1 = 0.0;
  const int64_t n = g.n;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    int32_t beg = 0, deg = 0, ci = -1;
    if (i < n) { beg = g.begin(i); deg = g.degree(i); ci = C[i]; }
    if (deg > kBinMax[kHubBin - 1]) deg = 0;  // hub rows: hub_modularity
    // four arcs per step: index and weight loads, then the label loads, all
    // issued before the first use
    constexpr int U = 4;
    auto step = [&](int32_t b0, int32_t e0, int32_t stride, int32_t end, int32_t cc, double& kk, double& ss) {
      WT wr[U];
      int32_t j[U], cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        wr[u] = WT(0);
        j[u] = 0;  // (past the row: an unused, valid label load)
        if (e0 + u * stride < end) {
          wr[u] = g.weight(b0 + e0 + u * stride);
          j[u] = g.idx[b0 + e0 + u * stride];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) cj[u] = C[j[u]];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u * stride >= end) continue;
        kk += (double)wr[u];
        if (cj[u] == cc) ss += (double)wr[u];
      }
    };
    double k = 0.0, sg = 0.0;
    if (deg < kWave)
      for (int32_t e = 0; e < deg; e += U) step(beg, e, 1, deg, ci, k, sg);
    u64 mask = __ballot(i < n && deg >= kWave);
    while (mask) {
      const int q = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const int32_t bq = __shfl(beg, q), dq = __shfl(deg, q), cq = __shfl(ci, q);
      double pk = 0.0, ps = 0.0;
      for (int32_t e = lane_id(); e < dq; e += U * kWave) step(bq, e, kWave, dq, cq, pk, ps);
      pk = sum_xor<kWave>(pk);
      ps = sum_xor<kWave>(ps);
      if (lane_id() == q) { k = pk; sg = ps; }
    }
    atomic_add_keyed<double>(tot, ci, k, i < n && k != 0.0);
    if (gid) atomic_add_keyed<double>(s1g, i < n ? gid[i] : 0, sg, i < n && sg != 0.0);
    else if (i < n) s1 += sg;
  }
  const double t = block_sum<double>(s1, red);
  if (threadIdx.x == 0) atomicAdd(&acc_d[0], t);
}
// The same partials for one graph, arc-parallel: a workgroup takes kBlock
// consecutive rows (hub rows excluded), lays their arcs end to end, and
// every lane takes one arc per step, so the label gathers of short and long
// rows alike are issued by full wavefronts.  The row of an arc comes from a
// binary search over the workgroup's row offsets in LDS; the row sums K_i
// are reduced per row by a segmented wavefront scan (rows of consecutive
// arcs are non-decreasing across the lanes) and one LDS add per segment,
// and added to the community totals through the workgroup-combined table.
template <class WT>
__global__ __launch_bounds__(kBlock) void k_mod_rows(GraphView<WT> g, const int32_t* C, double* tot,
                                                     double* acc_d) {
  constexpr int U = 4;  // arcs per lane per step
  __shared__ int32_t s_off[kBlock + 1];
  __shared__ int32_t s_beg[kBlock];
  __shared__ int32_t s_c[kBlock];
  __shared__ double s_k[kBlock];
  __shared__ int32_t s_wsum[kBlock / kWave];
  __shared__ double red[16];
  __shared__ KeyedLds<kBlock> kt;
  keyed_clear(kt);
  double s1 = 0.0;
  const int64_t n = g.n;
  const int t = threadIdx.x;
  const int wv = t / kWave;
  for (int64_t r0 = (int64_t)blockIdx.x * kBlock; r0 < n; r0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = r0 + t;
    int32_t deg = 0, beg = 0, ci = -1;
    if (i < n) { beg = g.begin(i); deg = g.degree(i); ci = C[i]; }
    if (deg > kBinMax[kHubBin - 1]) deg = 0;  // hub rows: hub_modularity
    int incl = deg;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_up(incl, o);
      if (lane_id() >= o) incl += x;
    }
    if (lane_id() == kWave - 1) s_wsum[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int k = 0; k < kBlock / kWave; ++k) {
      if (k < wv) before += s_wsum[k];
      total += s_wsum[k];
    }
    s_off[t] = before + incl - deg;
    if (t == 0) s_off[kBlock] = total;
    s_beg[t] = beg;
    s_c[t] = ci;
    s_k[t] = 0.0;
    __syncthreads();
    for (int32_t qb = 0; qb < total; qb += U * kBlock) {  // uniform over the workgroup
      int32_t row[U], j[U];
      WT w[U];  // widened where used (see GraphView::weight)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t q = qb + u * kBlock + t;
        row[u] = -1;
        j[u] = 0;
        w[u] = WT(0);
        if (q < total) {
          int lo = 0, hi = kBlock;  // s_off[lo] <= q < s_off[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= q) lo = mid; else hi = mid;
          }
          const int64_t e = (int64_t)s_beg[lo] + (q - s_off[lo]);
          row[u] = lo;
          j[u] = g.idx[e];
          w[u] = g.weight(e);
        }
      }
      int32_t cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cj[u] = C[j[u]];  // (j = 0 past the rows: an unused, valid load)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double v = (double)w[u];  // (0 past the rows)
        if (row[u] >= 0 && cj[u] == s_c[row[u]]) s1 += v;
        const int32_t r = row[u];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const double v2 = __shfl_down(v, o);
          const int32_t r2 = __shfl_down(r, o);
          if (lane_id() + o < kWave && r2 == r) v += v2;
        }
        const int32_t rp = __shfl_up(r, 1);
        if (r >= 0 && (lane_id() == 0 || rp != r)) atomicAdd(&s_k[r], v);
      }
    }
    __syncthreads();
    const double k = s_k[t];
    if (i < n && k != 0.0) keyed_put(kt, ci, k, 0);
    keyed_flush(kt, tot, (int32_t*)nullptr);  // also: s_* are rewritten by the next rows
  }
  const double s = block_sum<double>(s1, red);
  if (threadIdx.x == 0) atomicAdd(&acc_d[0], s);
}

void modularity_partial(hipStream_t st, const GraphDesc& gd, const int32_t* C, double* tot, double* acc_d,
                        const int32_t* gid, double* s1g) {
  if (gd.n <= 0) return;
  if (!gid) {
    const int grid = grid_n(gd.n, kBlock, 8192);
    if (gd.w_double)
      hipLaunchKernelGGL(k_mod_rows<double>, dim3(grid), dim3(kBlock), 0, st,
                         GraphView<double>{gd.n, gd.off, gd.deg, gd.idx, (const double*)gd.w}, C, tot, acc_d);
    else
      hipLaunchKernelGGL(k_mod_rows<float>, dim3(grid), dim3(kBlock), 0, st,
                         GraphView<float>{gd.n, gd.off, gd.deg, gd.idx, (const float*)gd.w}, C, tot, acc_d);
    return;
  }
  if (gd.w_double) {
    GraphView<double> g{gd.n, gd.off, gd.deg, gd.idx, (const double*)gd.w};
    hipLaunchKernelGGL(k_mod_partial<double>, dim3(grid_n(gd.n, kBlock, 2048)), dim3(kBlock), 0, st, g, C,
                       tot, acc_d, gid, s1g);
  } else {
    GraphView<float> g{gd.n, gd.off, gd.deg, gd.idx, (const float*)gd.w};
    hipLaunchKernelGGL(k_mod_partial<float>, dim3(grid_n(gd.n, kBlock, 2048)), dim3(kBlock), 0, st, g, C,
                       tot, acc_d, gid, s1g);
  }
}

__global__ __launch_bounds__(kBlock) void k_mod_squares(const double* tot, int64_t n, int integral,
                                                        double* acc_d, unsigned long long* acc_u) {
  __shared__ double red[16];
  __shared__ i128 redk[16];
  double sd = 0.0;
  i128 sk = 0;
  GRID_STRIDE(c, n) {
    const double t = tot[c];
    if (integral) {
      const long long ti = (long long)t;
      sk += (i128)ti * (i128)ti;
    } else {
      sd += t * t;
    }
  }
  if (integral) {
    const i128 k = block_sum_i128(sk, redk);
    if (threadIdx.x == 0 && k != 0) atomic_add_i128(acc_u, k);
  } else {
    const double d = block_sum<double>(sd, red);
    if (threadIdx.x == 0) atomicAdd(&acc_d[1], d);
  }
}
void modularity_squares(hipStream_t st, const double* tot, int64_t n, bool integral, double* acc_d,
                        unsigned long long* acc_u) {
  if (n > 0)
    hipLaunchKernelGGL(k_mod_squares, dim3(grid_n(n, kBlock, 4096)), dim3(kBlock), 0, st, tot, n,
                       (int)integral, acc_d, acc_u);
}

void check_offsets(hipStream_t st, const int32_t* off, int64_t n, int64_t m, int32_t* flags) {
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_n(n)), dim3(kBlock), 0, st, off, n, m, flags);
}

}  // namespace gvl
