// Disconnected-community check (Alg. 5) on the device.
//
// A community is disconnected when its members are not all reachable from
// one another through arcs that stay inside the community.  The connected
// components of the subgraph of intra-community arcs are built by
// union-find with lock-free hooking: every intra-community edge {i, j}
// (taken once, from its i < j arc) joins the trees of i and j by a CAS that
// points the larger root at the smaller one; finds halve their paths.  A
// failed CAS means that another edge changed that root, so the edge
// retries from the new roots; the number of roots only falls, so every
// edge finishes.  Then each community keeps the root of one of its members
// (plain stores: any member's root will do) and a community is flagged when
// a member's root differs from it.  Reads and writes of the parent array
// during the union pass are device-scope atomics, so that workgroups on
// different XCDs see one another's links.
#include "device.hpp"
#include "kernels.hpp"

namespace gvl {

__device__ __forceinline__ int32_t cc_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cc_store(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x; every visited vertex is re-pointed to its grandparent (path
// halving: parents only ever move towards the root).
__device__ __forceinline__ int32_t cc_find(int32_t* comp, int32_t x) {
  int32_t p = cc_load(comp + x);
  while (p != x) {
    const int32_t gp = cc_load(comp + p);
    if (gp == p) return p;
    cc_store(comp + x, gp);
    x = gp;
    p = cc_load(comp + x);
  }
  return x;
}

__global__ void k_cc_init(int32_t* comp, int32_t* rep, int32_t* dis, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    comp[i] = (int32_t)i;
    rep[i] = -1;
    dis[i] = 0;
  }
}

// Union pass, arc-parallel: a workgroup takes kBlock consecutive rows and
// lays their arcs end to end (row of an arc by binary search in LDS).
__global__ __launch_bounds__(kBlock) void k_cc_union(const int32_t* off, const int32_t* idx, const int32_t* C,
                                                     int64_t n, int32_t* comp) {
  __shared__ int32_t s_off[kBlock + 1];
  __shared__ int32_t s_beg[kBlock];
  __shared__ int32_t s_c[kBlock];
  __shared__ int32_t s_w[kBlock / kWave];
  const int t = threadIdx.x;
  const int wv = t / kWave;
  for (int64_t r0 = (int64_t)blockIdx.x * kBlock; r0 < n; r0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = r0 + t;
    int32_t deg = 0, beg = 0, ci = -1;
    if (i < n) {
      beg = off[i];
      deg = off[i + 1] - beg;
      ci = C[i];
    }
    int incl = deg;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int x = __shfl_up(incl, o);
      if (lane_id() >= o) incl += x;
    }
    __syncthreads();  // the previous rows' s_* are no longer read
    if (lane_id() == kWave - 1) s_w[wv] = incl;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int k = 0; k < kBlock / kWave; ++k) {
      if (k < wv) before += s_w[k];
      total += s_w[k];
    }
    s_off[t] = (int32_t)(before + incl - deg);
    if (t == 0) s_off[kBlock] = (int32_t)total;
    s_beg[t] = beg;
    s_c[t] = ci;
    __syncthreads();
    for (int32_t q = t; q < (int32_t)total; q += kBlock) {
      int lo = 0, hi = kBlock;  // s_off[lo] <= q < s_off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= q) lo = mid; else hi = mid;
      }
      const int32_t a = (int32_t)(r0 + lo);
      const int32_t b = idx[(int64_t)s_beg[lo] + (q - s_off[lo])];
      if (b <= a || C[b] != s_c[lo]) continue;  // each edge once; intra-community only
      int32_t ra = cc_find(comp, a), rb = cc_find(comp, b);
      while (ra != rb) {
        if (ra > rb) { const int32_t x = ra; ra = rb; rb = x; }
        const int32_t old = atomicCAS(comp + rb, rb, ra);  // hook the larger root
        if (old == rb) break;
        rb = cc_find(comp, old);
        ra = cc_find(comp, ra);
      }
    }
  }
}

// root[i] = root of i; rep[C[i]] = the root of some member of C[i].  The
// roots go to their own array: finds of other threads keep halving paths in
// comp during this kernel and may store an intermediate ancestor over a
// root written there.
__global__ void k_cc_flatten(int32_t* comp, const int32_t* C, int64_t n, int32_t* root, int32_t* rep) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = cc_find(comp, (int32_t)i);
    root[i] = r;
    rep[C[i]] = r;
  }
}

// dis[c] = 1 for communities with a member outside rep[c]'s component;
// cnt[0] counts them.
__global__ void k_cc_mark(const int32_t* root, const int32_t* C, const int32_t* rep, int64_t n, int32_t* dis,
                          unsigned long long* cnt) {
  unsigned long long mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = C[i];
    if (root[i] == rep[c] || dis[c]) continue;  // (a stale 0 is settled by the exchange)
    if (atomicExch(&dis[c], 1) == 0) ++mine;
  }
  if (mine) atomicAdd(cnt, mine);
}

static inline int grid_of(int64_t n, int cap) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

void disconnected_communities(hipStream_t st, const int32_t* off, const int32_t* idx, const int32_t* C, int64_t n,
                              int32_t* comp, int32_t* root, int32_t* rep, int32_t* dis, unsigned long long* cnt) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cc_init, dim3(grid_of(n, 16384)), dim3(kBlock), 0, st, comp, rep, dis, n);
  hipLaunchKernelGGL(k_cc_union, dim3(grid_of(n, 8192)), dim3(kBlock), 0, st, off, idx, C, n, comp);
  hipLaunchKernelGGL(k_cc_flatten, dim3(grid_of(n, 16384)), dim3(kBlock), 0, st, comp, C, n, root, rep);
  hipLaunchKernelGGL(k_cc_mark, dim3(grid_of(n, 16384)), dim3(kBlock), 0, st, root, C, rep, n, dis, cnt);
}

}  // namespace gvl
