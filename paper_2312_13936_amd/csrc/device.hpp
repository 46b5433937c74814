// Device-side building blocks shared by the gvl kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace gvl {

constexpr int kWave = 64;
constexpr int kBlock = 256;

typedef __int128 i128;
typedef unsigned long long u64;

// ------------------------------------------------------------- graph view ---
// CSR row i occupies [off[i], off[i] + degree(i)).  Input graphs are plain
// CSR (deg == nullptr, degree = off[i+1] - off[i]); super-vertex graphs are
// "holey": rows are allocated with an over-estimated capacity and deg[] holds
// the filled length (Alg. 4).  w == nullptr means unit weights.
template <class WT>
struct GraphView {
  int64_t n;
  const int32_t* off;
  const int32_t* deg;
  const int32_t* idx;
  const WT* w;
  __device__ __forceinline__ int32_t begin(int64_t i) const { return off[i]; }
  __device__ __forceinline__ int32_t degree(int64_t i) const {
    return deg ? deg[i] : off[i + 1] - off[i];
  }
  // Weight of arc e (1 for an unweighted graph) in the graph's own type.
  // Loops that issue several loads keep it in that type and widen it to
  // FP64 where it is used: a conversion next to its load, inside the
  // branch on w, makes the compiler wait for that load before the next
  // load of the round goes out.
  __device__ __forceinline__ WT weight(int64_t e) const {
    WT x = WT(1);
    if (w) x = w[e];
    return x;
  }
};

// ------------------------------------------------------------ wave helpers ---
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// This workgroup's copy of the counters / sums (see kCntSlots).
__device__ __forceinline__ int cslot() { return (int)(blockIdx.x & (kCntSlots - 1)); }
__device__ __forceinline__ unsigned long long* cnt_of(unsigned long long* cnt) { return cnt + 8 * cslot(); }

// Orders the LDS traffic of one wavefront: every lane's earlier LDS
// operations complete before any lane's later ones.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ u64 lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <int W>
__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, W); }
template <int W>
__device__ __forceinline__ int shfl_xor_i(int v, int m) { return __shfl_xor(v, m, W); }
template <int W>
__device__ __forceinline__ long long shfl_xor_ll(long long v, int m) { return __shfl_xor(v, m, W); }

__device__ __forceinline__ i128 make_i128(long long hi, unsigned long long lo) {
  return (i128)(((unsigned __int128)(unsigned long long)hi << 64) | (unsigned __int128)lo);
}

template <int W>
__device__ __forceinline__ i128 shfl_xor_i128(i128 v, int m) {
  long long hi = (long long)(v >> 64);
  long long lo = (long long)(unsigned long long)v;
  hi = __shfl_xor(hi, m, W);
  lo = __shfl_xor(lo, m, W);
  return make_i128(hi, (unsigned long long)lo);
}

// (gain, id) ordering: larger gain wins, equal gains go to the lower id;
// id < 0 means "no candidate".
__device__ __forceinline__ bool better_f(double g2, int32_t c2, double g, int32_t c) {
  return c2 >= 0 && (c < 0 || g2 > g || (g2 == g && c2 < c));
}
__device__ __forceinline__ bool better_k(i128 k2, int32_t c2, i128 k, int32_t c) {
  return c2 >= 0 && (c < 0 || k2 > k || (k2 == k && c2 < c));
}

template <int W>
__device__ __forceinline__ void argmax_f(double& g, int32_t& c) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    double g2 = shfl_xor_d<W>(g, o);
    int32_t c2 = shfl_xor_i<W>(c, o);
    if (better_f(g2, c2, g, c)) { g = g2; c = c2; }
  }
}
template <int W>
__device__ __forceinline__ void argmax_k(i128& k, int32_t& c) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    i128 k2 = shfl_xor_i128<W>(k, o);
    int32_t c2 = shfl_xor_i<W>(c, o);
    if (better_k(k2, c2, k, c)) { k = k2; c = c2; }
  }
}

template <int W, class T>
__device__ __forceinline__ T sum_xor(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Exact 128-bit accumulation into two 64-bit words (lo, hi) with carry:
// correct modulo 2^128 for any order of concurrent callers.
__device__ __forceinline__ void atomic_add_i128(u64* lohi, i128 v) {
  const u64 lo = (u64)v;
  u64 hi = (u64)(v >> 64);
  const u64 old = atomicAdd(&lohi[0], lo);
  if (old + lo < old) hi += 1ull;
  atomicAdd(&lohi[1], hi);
}

// -------------------------------------------------------------- hashing ---
// Open addressing with linear probing, power-of-two capacity 2^lg.
// Multiplicative (Fibonacci) hashing of the community id.
__device__ __forceinline__ uint32_t hslot(int32_t c, int lg) {
  return ((uint32_t)c * 0x9E3779B1u) >> (32 - lg);
}

// LDS table insert: H[c] += w.
__device__ __forceinline__ void lds_insert(int32_t* keys, double* vals, int lg, int32_t c, double w) {
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t h = hslot(c, lg);
  while (true) {
    int32_t k = keys[h];
    if (k == c) { atomicAdd(&vals[h], w); return; }
    if (k == kEmpty) {
      int32_t old = atomicCAS(&keys[h], kEmpty, c);
      if (old == kEmpty || old == c) { atomicAdd(&vals[h], w); return; }
    }
    h = (h + 1u) & mask;
  }
}

// As lds_insert, but gives up after probing every slot once (full table):
// returns false then.
__device__ __forceinline__ bool lds_insert_bounded(int32_t* keys, double* vals, int lg, int32_t c, double w) {
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t h = hslot(c, lg);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    int32_t k = keys[h];
    if (k == c) { atomicAdd(&vals[h], w); return true; }
    if (k == kEmpty) {
      int32_t old = atomicCAS(&keys[h], kEmpty, c);
      if (old == kEmpty || old == c) { atomicAdd(&vals[h], w); return true; }
    }
    h = (h + 1u) & mask;
  }
  return false;
}

// As lds_insert_bounded for a table of any size ts: the home slot is the
// high word of (multiplicative hash of c) * ts, which for ts = 2^lg is
// hslot(c, lg); probing wraps at ts.
__device__ __forceinline__ bool lds_insert_sized(int32_t* keys, double* vals, uint32_t ts, int32_t c, double w) {
  uint32_t h = (uint32_t)(((u64)((uint32_t)c * 0x9E3779B1u) * (u64)ts) >> 32);
  for (uint32_t probe = 0; probe < ts; ++probe) {
    int32_t k = keys[h];
    if (k == c) { atomicAdd(&vals[h], w); return true; }
    if (k == kEmpty) {
      int32_t old = atomicCAS(&keys[h], kEmpty, c);
      if (old == kEmpty || old == c) { atomicAdd(&vals[h], w); return true; }
    }
    h = (h + 1u == ts) ? 0u : h + 1u;
  }
  return false;
}

// ------------------------------------------------ randomized refinement ---
// Counter-based draw for (seed, pass, sweep, vertex, candidate):
// MurmurHash3's 32-bit finalizer mixes the counters into a nonzero
// xorshift32 state (Marsaglia, "Xorshift RNGs", 2003) that takes one step.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return h;
}
__device__ __forceinline__ uint32_t draw32(uint32_t seed, int32_t pass, int32_t sweep, int32_t i, int32_t c) {
  uint32_t x = fmix32((uint32_t)pass * 0x9E3779B9u + (uint32_t)sweep);
  x = fmix32((uint32_t)c ^ x);
  x = fmix32((uint32_t)i ^ x);
  x = fmix32(seed ^ x);
  if (x == 0) x = 0x6D2B79F5u;
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}
// -ln(u), u = (x + 1/2) / 2^32: u = m 2^e with m in [1, 2), ln m = 2 atanh(z)
// summed as the series z + z^3/3 + ... (24 terms, z = (m - 1)/(m + 1) < 1/3);
// plain IEEE operations only, so the value is the same on every device.
__device__ __forceinline__ double neg_ln_unit(uint32_t x) {
  double m = ((double)x + 0.5) * (1.0 / 4294967296.0);
  int32_t e = 0;
  while (m < 1.0) { m *= 2.0; --e; }
  const double z = (m - 1.0) / (m + 1.0), z2 = z * z;
  double s = 0.0, t = z;
#pragma unroll
  for (int32_t k = 0; k < 24; ++k) {
    s += t * (1.0 / (double)(2 * k + 1));
    t *= z2;
  }
  return -((double)e * 0.6931471805599453 + 2.0 * s);
}
// int128 -> double as hi 2^64 + lo (each part converted exactly rounded).
__device__ __forceinline__ double key_to_double(i128 k) {
  const long long hi = (long long)(k >> 64);
  const unsigned long long lo = (unsigned long long)k;
  return (double)hi * 18446744073709551616.0 + (double)lo;
}

// Symmetry check (validate = 2): a multiset hash of the arcs.  For every arc
// (i -> j, weight bits) the check adds H(i, j, w) - H(j, i, w) modulo 2^64,
// for two independent seeds.  A symmetric CSR (every arc matched by its
// reverse with the same weight, duplicates matched in number) sums to zero
// whatever the order; an asymmetric one sums to zero for both seeds only by
// a 2^-128 coincidence (not by construction: an input crafted against these
// public mixers could pass).  H is SplitMix64's finalizer (Steele, Lea,
// Flood 2014) applied twice around the seed.
__device__ __forceinline__ u64 splitmix_fin(u64 x) {
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ __forceinline__ u64 arc_hash(u64 seed, int32_t a, int32_t b, uint32_t wbits) {
  const u64 x = (((u64)(uint32_t)a << 32) | (u64)(uint32_t)b) ^ ((u64)wbits * 0x9E3779B97F4A7C15ull);
  return splitmix_fin(splitmix_fin(x) ^ seed);
}
constexpr u64 kSymSeed0 = 0x243F6A8885A308D3ull, kSymSeed1 = 0x13198A2E03707344ull;
__device__ __forceinline__ void arc_sym(int32_t i, int32_t j, uint32_t wbits, u64& d0, u64& d1) {
  d0 += arc_hash(kSymSeed0, i, j, wbits) - arc_hash(kSymSeed0, j, i, wbits);
  d1 += arc_hash(kSymSeed1, i, j, wbits) - arc_hash(kSymSeed1, j, i, wbits);
}

// Partition hash of a community id for wide rows (Wellons' "lowbias32"
// integer mixer); independent of hslot, which takes the high bits of a
// multiplicative hash.
__device__ __forceinline__ uint32_t wide_part(int32_t c) {
  uint32_t h = (uint32_t)c;
  h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
  return h;
}

// Global-memory table (hubs and giant communities), 16-byte slots.  Inserts
// are atomics performed at L2; a table is read back only by later kernels
// (plain loads after the launch boundary).
// Inserts H[c] += w; returns the slot if this call created the key, else -1.
__device__ __forceinline__ int64_t slot_insert_new(TblSlot* t, int lg, int32_t c, double w) {
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t h = hslot(c, lg);
  while (true) {
    const int32_t old = atomicCAS(&t[h].key, kEmpty, c);
    if (old == kEmpty || old == c) {
      atomicAdd(&t[h].val, w);
      return old == kEmpty ? (int64_t)h : -1;
    }
    h = (h + 1u) & mask;
  }
}

// p[key] += v for every active lane.  Lanes of the wavefront that share the
// key of the first remaining active lane are summed into one atomic (two
// rounds), which takes the load off the address of a giant community; the
// rest add one by one.  Must be reached by the whole wavefront.
template <class T>
__device__ __forceinline__ void atomic_add_keyed(T* p, int32_t key, T v, bool active) {
  u64 rem = __ballot(active);
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    if (!rem) break;
    const int leader = __ffsll((unsigned long long)rem) - 1;
    const int32_t k0 = __shfl(key, leader);
    const bool mine = ((rem >> lane_id()) & 1) && key == k0;
    const u64 m = __ballot(mine);
    const T part = sum_xor<kWave>(mine ? v : T(0));
    if (lane_id() == leader) atomicAdd(&p[k0], part);
    rem &= ~m;
  }
  if ((rem >> lane_id()) & 1) atomicAdd(&p[key], v);
}

// Workgroup-combined keyed adds pv[key] += dv, pu[key] += du.  Threads put
// their entries (any number, at most 2 NT distinct keys per flush) into an
// LDS table of 4 NT slots, where equal keys are summed; the flush adds each
// distinct key once to global memory.  A community shared by many threads
// of the workgroup (the totals of a giant community) so costs one atomic per
// workgroup instead of one per member.  put is per thread; clear and flush
// must be reached by every thread of the workgroup; flush leaves the table
// empty.
template <int NT>
struct KeyedLds {
  static constexpr int kSlots = 4 * NT;
  int32_t key[kSlots];
  double v[kSlots];
  int32_t u[kSlots];
};

template <int NT>
__device__ __forceinline__ void keyed_clear(KeyedLds<NT>& t) {
  for (int s = threadIdx.x; s < KeyedLds<NT>::kSlots; s += NT) {
    t.key[s] = kEmpty;
    t.v[s] = 0.0;
    t.u[s] = 0;
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ void keyed_put(KeyedLds<NT>& t, int32_t key, double dv, int32_t du) {
  constexpr int kLg = __builtin_ctz(KeyedLds<NT>::kSlots);
  constexpr uint32_t mask = KeyedLds<NT>::kSlots - 1;
  static_assert((KeyedLds<NT>::kSlots & mask) == 0, "power-of-two table");
  uint32_t h = hslot(key, kLg);
  while (true) {
    const int32_t k = t.key[h];
    if (k == key) break;
    if (k == kEmpty) {
      const int32_t old = atomicCAS(&t.key[h], kEmpty, key);
      if (old == kEmpty || old == key) break;
    }
    h = (h + 1u) & mask;
  }
  if (dv != 0.0) atomicAdd(&t.v[h], dv);
  if (du != 0) atomicAdd(&t.u[h], du);
}

template <int NT>
__device__ __forceinline__ void keyed_flush(KeyedLds<NT>& t, double* pv, int32_t* pu) {
  __syncthreads();
  for (int s = threadIdx.x; s < KeyedLds<NT>::kSlots; s += NT) {
    const int32_t k = t.key[s];
    if (k != kEmpty) {
      const double v = t.v[s];
      const int32_t u = t.u[s];
      if (v != 0.0) atomicAdd(&pv[k], v);
      if (pu && u != 0) atomicAdd(&pu[k], u);
      t.key[s] = kEmpty;
      t.v[s] = 0.0;
      t.u[s] = 0;
    }
  }
  __syncthreads();
}

// Sub-sweep group of vertex i: MurmurHash3's 32-bit finalizer of i, mod S.
__device__ __forceinline__ int group_of(int64_t i, int S) {
  uint32_t h = (uint32_t)i;
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return (int)(h % (uint32_t)S);
}

__host__ __device__ __forceinline__ int ceil_log2(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

// -------------------------------------------------------- block reductions ---
// Sum over the block (blockDim.x multiple of 64, <= 1024); the result is
// valid in thread 0.  `red` is LDS scratch of >= 16 entries.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = sum_xor<kWave>(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  T s = T(0);
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
  return s;
}

// Sum over the block as block_sum, with the result valid in every thread
// (each thread adds the wavefront sums in the same order, so all agree).
template <class T>
__device__ __forceinline__ T block_allsum(T v, T* red) {
  v = sum_xor<kWave>(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  T s = T(0);
  for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
  return s;
}

__device__ __forceinline__ i128 block_sum_i128(i128 v, i128* red) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += shfl_xor_i128<kWave>(v, o);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  i128 s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
  return s;
}

}  // namespace gvl
