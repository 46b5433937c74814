// Seeded synthetic graph generators.
//
// These build the inputs that both the CPU oracle and the GPU path consume.
// They hold none of the community-detection arithmetic: only random numbers,
// edge lists and CSR assembly.  Every random draw is a pure function of
// (seed, counter) through SplitMix64 (Steele, Lea, Flood 2014), so the graphs
// are identical for any thread count and on any machine.
//
// Output format (all generators): symmetric CSR with int32 offsets[n+1],
// int32 indices[m] (ascending within a row, no duplicates, no self-loops)
// and float weights[m] (integer-valued), the same weight on both directions
// of an undirected edge.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef uint64_t u64;
typedef int64_t i64;

inline u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
// k-th output of a SplitMix64 stream whose state starts at `seed`.
inline u64 draw(u64 seed, u64 k) { return mix64(seed + (k + 1) * 0x9E3779B97F4A7C15ULL); }
inline double unif(u64 seed, u64 k) { return (double)(draw(seed, k) >> 11) * (1.0 / 9007199254740992.0); }
inline u64 stream(u64 seed, u64 id) { return mix64(seed ^ mix64(id + 0x5851F42D4C957F2DULL)); }

struct Edge { int32_t u, v; float w; };

// Seeded Fisher-Yates permutation of [0, n).
std::vector<int32_t> permutation(i64 n, u64 seed) {
  std::vector<int32_t> p(n);
  for (i64 i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (i64 i = n - 1; i > 0; --i) {
    i64 j = (i64)(draw(seed, (u64)i) % (u64)(i + 1));
    std::swap(p[i], p[j]);
  }
  return p;
}

}  // namespace

extern "C" {

typedef struct {
  int64_t n, m;
  int32_t* offsets;
  int32_t* indices;
  float* weights;
  int32_t* truth;  // planted community of each vertex, or NULL
} gen_graph;

void gen_free(gen_graph* g) {
  if (!g) return;
  free(g->offsets); free(g->indices); free(g->weights); free(g->truth);
  memset(g, 0, sizeof(*g));
}

}  // extern "C"

namespace {

// Assemble a symmetric CSR from undirected edges.  Self-loops are dropped,
// both directions are stored, duplicate arcs keep the smallest weight.
int build_csr(i64 n, std::vector<Edge>& edges, gen_graph* out) {
  std::vector<int64_t> deg(n + 1, 0);
  const i64 ne = (i64)edges.size();
  {
    std::vector<std::atomic<int64_t>> cnt(n);
    for (i64 i = 0; i < n; ++i) cnt[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
    for (i64 e = 0; e < ne; ++e) {
      const Edge& x = edges[e];
      if (x.u == x.v) continue;
      cnt[x.u].fetch_add(1, std::memory_order_relaxed);
      cnt[x.v].fetch_add(1, std::memory_order_relaxed);
    }
    for (i64 i = 0; i < n; ++i) deg[i + 1] = deg[i] + cnt[i].load();
  }
  const i64 m0 = deg[n];
  std::vector<int32_t> idx(m0);
  std::vector<float> wt(m0);
  {
    std::vector<std::atomic<int64_t>> cur(n);
    for (i64 i = 0; i < n; ++i) cur[i].store(deg[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
    for (i64 e = 0; e < ne; ++e) {
      const Edge& x = edges[e];
      if (x.u == x.v) continue;
      i64 a = cur[x.u].fetch_add(1, std::memory_order_relaxed);
      idx[a] = x.v; wt[a] = x.w;
      i64 b = cur[x.v].fetch_add(1, std::memory_order_relaxed);
      idx[b] = x.u; wt[b] = x.w;
    }
  }
  std::vector<Edge>().swap(edges);
  // Sort each row by (neighbour, weight) and drop duplicate neighbours.
  std::vector<int64_t> kept(n, 0);
#pragma omp parallel
  {
    std::vector<std::pair<int32_t, float>> row;
#pragma omp for schedule(dynamic, 1024)
    for (i64 i = 0; i < n; ++i) {
      i64 b = deg[i], e = deg[i + 1];
      row.clear();
      for (i64 k = b; k < e; ++k) row.push_back({idx[k], wt[k]});
      std::sort(row.begin(), row.end());
      i64 w = b;
      for (size_t k = 0; k < row.size(); ++k) {
        if (k > 0 && row[k].first == row[k - 1].first) continue;
        idx[w] = row[k].first; wt[w] = row[k].second; ++w;
      }
      kept[i] = w - b;
    }
  }
  i64 m = 0;
  for (i64 i = 0; i < n; ++i) m += kept[i];
  if (m > 2147483647LL) return -1;
  out->n = n; out->m = m;
  out->offsets = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  out->indices = (int32_t*)malloc(sizeof(int32_t) * (m > 0 ? m : 1));
  out->weights = (float*)malloc(sizeof(float) * (m > 0 ? m : 1));
  if (!out->offsets || !out->indices || !out->weights) return -2;
  out->offsets[0] = 0;
  for (i64 i = 0; i < n; ++i) out->offsets[i + 1] = (int32_t)(out->offsets[i] + kept[i]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (i64 i = 0; i < n; ++i) {
    memcpy(out->indices + out->offsets[i], idx.data() + deg[i], sizeof(int32_t) * kept[i]);
    memcpy(out->weights + out->offsets[i], wt.data() + deg[i], sizeof(float) * kept[i]);
  }
  return 0;
}

}  // namespace

extern "C" {

// Planted partition (stochastic block model): `blocks` blocks of
// `block_size` vertices; every unordered pair is an edge with probability
// p_in inside a block and p_out across blocks.  Vertex ids are then
// shuffled by a seeded permutation; truth[] holds each vertex's block.
int gen_planted(int32_t blocks, int32_t block_size, double p_in, double p_out,
                uint64_t seed, gen_graph* out) {
  memset(out, 0, sizeof(*out));
  const i64 n = (i64)blocks * block_size;
  if (n <= 0 || n > 2000000) return -1;
  const u64 s_pair = stream(seed, 1), s_perm = stream(seed, 2);
  std::vector<int64_t> cnt(n + 1, 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 u = 0; u < n; ++u) {
    int64_t c = 0;
    for (i64 v = u + 1; v < n; ++v) {
      double p = (u / block_size == v / block_size) ? p_in : p_out;
      if (unif(s_pair, (u64)(u * n + v)) < p) ++c;
    }
    cnt[u + 1] = c;
  }
  for (i64 u = 0; u < n; ++u) cnt[u + 1] += cnt[u];
  std::vector<int32_t> perm = permutation(n, s_perm);
  std::vector<Edge> edges(cnt[n]);
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 u = 0; u < n; ++u) {
    int64_t k = cnt[u];
    for (i64 v = u + 1; v < n; ++v) {
      double p = (u / block_size == v / block_size) ? p_in : p_out;
      if (unif(s_pair, (u64)(u * n + v)) < p) edges[k++] = {perm[u], perm[v], 1.0f};
    }
  }
  int rc = build_csr(n, edges, out);
  if (rc) return rc;
  out->truth = (int32_t*)malloc(sizeof(int32_t) * n);
  for (i64 u = 0; u < n; ++u) out->truth[perm[u]] = (int32_t)(u / block_size);
  return 0;
}

// R-MAT (Chakrabarti, Zhan, Faloutsos 2004): edge_factor * 2^scale samples,
// each choosing one of four quadrants per level with probabilities
// (a, b, c, 1-a-b-c).  Self-loops and duplicates are removed, the result is
// symmetrised, and vertex ids are shuffled by a seeded permutation.
int gen_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c,
             uint64_t seed, gen_graph* out) {
  memset(out, 0, sizeof(*out));
  if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
  const i64 n = (i64)1 << scale;
  const i64 ne = (i64)edge_factor << scale;
  const u64 s_edge = stream(seed, 11), s_perm = stream(seed, 12);
  const double ab = a + b, abc = a + b + c;
  std::vector<int32_t> perm = permutation(n, s_perm);
  std::vector<Edge> edges(ne);
  const i64 draws_per_edge = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (i64 e = 0; e < ne; ++e) {
    u64 u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      u64 r64 = draw(s_edge, (u64)(e * draws_per_edge + l / 2));
      double r = (double)((l & 1) ? (r64 >> 32) : (r64 & 0xFFFFFFFFULL)) * (1.0 / 4294967296.0);
      int bu, bv;
      if (r < a) { bu = 0; bv = 0; }
      else if (r < ab) { bu = 0; bv = 1; }
      else if (r < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | (u64)bu;
      v = (v << 1) | (u64)bv;
    }
    edges[e] = {perm[u], perm[v], 1.0f};
  }
  return build_csr(n, edges, out);
}

// Road-network-like grid: rows x cols 4-neighbour lattice (row-major ids),
// each lattice edge dropped with probability `drop`; then
// round(diag_frac * #lattice edges) random diagonal shortcuts (a random
// vertex to one of its four diagonal neighbours; out-of-range draws are
// skipped, duplicates merged).  Integer weights uniform in [1, wmax].
int gen_grid(int32_t rows, int32_t cols, double drop, double diag_frac, int32_t wmax,
             uint64_t seed, gen_graph* out) {
  memset(out, 0, sizeof(*out));
  if (rows < 1 || cols < 1 || wmax < 1) return -1;
  const i64 n = (i64)rows * cols;
  const u64 s_drop = stream(seed, 21), s_w = stream(seed, 22), s_diag = stream(seed, 23),
            s_dw = stream(seed, 24);
  const i64 nh = (i64)rows * (cols - 1), nv = (i64)(rows - 1) * cols;
  const i64 nlat = nh + nv;
  std::vector<Edge> edges;
  edges.reserve((size_t)(nlat * (1.0 - drop) * 1.01) + 1024);
  for (i64 k = 0; k < nlat; ++k) {
    if (unif(s_drop, (u64)k) < drop) continue;
    int32_t u, v;
    if (k < nh) { i64 r = k / (cols - 1), cc = k % (cols - 1); u = (int32_t)(r * cols + cc); v = u + 1; }
    else { i64 k2 = k - nh; u = (int32_t)k2; v = (int32_t)(k2 + cols); }
    float w = (float)(1 + (int64_t)(draw(s_w, (u64)k) % (u64)wmax));
    edges.push_back({u, v, w});
  }
  const i64 ndiag = (i64)llround(diag_frac * (double)nlat);
  std::vector<std::pair<std::pair<int32_t, int32_t>, i64>> diag;
  diag.reserve(ndiag);
  for (i64 t = 0; t < ndiag; ++t) {
    i64 v = (i64)(draw(s_diag, (u64)(2 * t)) % (u64)n);
    int dir = (int)(draw(s_diag, (u64)(2 * t + 1)) & 3);
    i64 r = v / cols, cc = v % cols;
    i64 r2 = r + ((dir & 1) ? 1 : -1), c2 = cc + ((dir & 2) ? 1 : -1);
    if (r2 < 0 || r2 >= rows || c2 < 0 || c2 >= cols) continue;
    int32_t a = (int32_t)v, b = (int32_t)(r2 * cols + c2);
    if (a > b) std::swap(a, b);
    diag.push_back({{a, b}, t});
  }
  std::sort(diag.begin(), diag.end());
  for (size_t k = 0; k < diag.size(); ++k) {
    if (k > 0 && diag[k].first == diag[k - 1].first) continue;
    float w = (float)(1 + (int64_t)(draw(s_dw, (u64)diag[k].second) % (u64)wmax));
    edges.push_back({diag[k].first.first, diag[k].first.second, w});
  }
  return build_csr(n, edges, out);
}

// LFR-style benchmark graph (Lancichinetti, Fortunato, Radicchi 2008),
// simplified: degrees from a power law with exponent tau1 on [kmin, kmax],
// with kmin drawn per vertex from the two neighbouring integers whose mix
// gives mean avg_deg exactly; community sizes from a power law with exponent
// tau2 on [cmin, cmax] until they cover n; vertices assigned to communities
// in a shuffled order; each vertex's stubs split into round((1 - mu) k)
// internal (at most its community's size - 1, the rest external) and the
// rest external; stubs paired uniformly at random inside each community
// (internal) and over the whole graph (external), a pair that would make a
// self-loop or repeat an edge going back to be paired again in the next of
// up to 16 rounds (the configuration model with rewiring), so the realised
// mean degree stays close to avg_deg.  Unit weights; truth[] holds the
// planted community.
namespace {
int64_t discrete_powerlaw(u64 s, u64 k, const std::vector<double>& cdf, int64_t lo) {
  const double u = unif(s, k) * cdf.back();
  return lo + (int64_t)(std::lower_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
}
std::vector<double> powerlaw_cdf(int64_t lo, int64_t hi, double tau) {
  std::vector<double> cdf;
  double acc = 0.0;
  for (int64_t k = lo; k <= hi; ++k) { acc += std::pow((double)k, -tau); cdf.push_back(acc); }
  return cdf;
}
double powerlaw_mean(int64_t lo, int64_t hi, double tau) {
  double a = 0.0, b = 0.0;
  for (int64_t k = lo; k <= hi; ++k) { double p = std::pow((double)k, -tau); a += p * k; b += p; }
  return a / b;
}
void shuffle(std::vector<int32_t>& v, u64 s) {
  for (int64_t i = (int64_t)v.size() - 1; i > 0; --i) std::swap(v[i], v[(int64_t)(draw(s, (u64)i) % (u64)(i + 1))]);
}
}  // namespace

namespace {
// Set of undirected edges (a < b) packed into 64-bit keys: open addressing
// with linear probing over a power-of-two table of at least twice the
// number of insertions.
struct EdgeSet {
  std::vector<u64> slot;
  u64 mask;
  explicit EdgeSet(size_t expect) {
    size_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    slot.assign(cap, ~0ull);
    mask = cap - 1;
  }
  // false if the key was already present
  bool insert(u64 key) {
    u64 h = mix64(key) & mask;
    while (slot[h] != ~0ull) {
      if (slot[h] == key) return false;
      h = (h + 1) & mask;
    }
    slot[h] = key;
    return true;
  }
};

// Pairs the stubs uniformly at random.  A pair that would be a self-loop or
// an edge already made goes back; the returned stubs are shuffled and paired
// again, for up to `rounds` rounds.  Stubs still unpaired are dropped.
void pair_stubs(std::vector<int32_t>& stubs, u64 s, EdgeSet& made, std::vector<Edge>& edges,
                int rounds) {
  std::vector<int32_t> back;
  for (int r = 0; r < rounds && stubs.size() >= 2; ++r) {
    shuffle(stubs, stream(s, (u64)r));
    back.clear();
    for (size_t k = 0; k + 1 < stubs.size(); k += 2) {
      int32_t a = stubs[k], b = stubs[k + 1];
      if (a > b) std::swap(a, b);
      if (a == b || !made.insert(((u64)(uint32_t)a << 32) | (u64)(uint32_t)b)) {
        back.push_back(a);
        back.push_back(b);
        continue;
      }
      edges.push_back({a, b, 1.0f});
    }
    if (stubs.size() % 2) back.push_back(stubs.back());
    stubs.swap(back);
  }
}
}  // namespace

extern "C" int gen_lfr(int64_t n, double avg_deg, int64_t kmax, double tau1, double tau2, double mu, int64_t cmin,
                       int64_t cmax, uint64_t seed, gen_graph* out) {
  memset(out, 0, sizeof(*out));
  if (n < 2 || avg_deg <= 0 || kmax < 1 || cmin < 1 || cmax < cmin || mu < 0 || mu > 1) return -1;
  kmax = std::min<int64_t>(kmax, n - 1);
  cmax = std::min<int64_t>(cmax, n);
  cmin = std::min<int64_t>(cmin, cmax);
  const u64 s_deg = stream(seed, 31), s_com = stream(seed, 32), s_ord = stream(seed, 33), s_in = stream(seed, 34),
            s_ex = stream(seed, 35), s_mix = stream(seed, 36);
  // kmin such that mean(kmin) <= avg_deg < mean(kmin + 1); each vertex draws
  // from the kmin + 1 law with probability q, which makes the mean avg_deg
  int64_t kmin = 1;
  while (kmin < kmax && powerlaw_mean(kmin + 1, kmax, tau1) <= avg_deg) ++kmin;
  const double m0 = powerlaw_mean(kmin, kmax, tau1);
  const double m1 = kmin < kmax ? powerlaw_mean(kmin + 1, kmax, tau1) : m0;
  const double q = (m1 > m0 && avg_deg > m0) ? std::min(1.0, (avg_deg - m0) / (m1 - m0)) : 0.0;
  const std::vector<double> dcdf0 = powerlaw_cdf(kmin, kmax, tau1);
  const std::vector<double> dcdf1 = powerlaw_cdf(std::min(kmin + 1, kmax), kmax, tau1);
  std::vector<int64_t> deg(n);
  for (int64_t i = 0; i < n; ++i)
    deg[i] = unif(s_mix, (u64)i) < q ? discrete_powerlaw(s_deg, (u64)i, dcdf1, std::min(kmin + 1, kmax))
                                     : discrete_powerlaw(s_deg, (u64)i, dcdf0, kmin);
  // community sizes
  std::vector<double> ccdf = powerlaw_cdf(cmin, cmax, tau2);
  std::vector<int64_t> csize;
  int64_t covered = 0;
  for (u64 t = 0; covered < n; ++t) {
    int64_t c = discrete_powerlaw(s_com, t, ccdf, cmin);
    if (covered + c > n) c = n - covered;
    csize.push_back(c);
    covered += c;
  }
  // assignment: shuffled vertex order fills communities in turn
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  shuffle(order, s_ord);
  std::vector<int32_t> com(n);
  std::vector<std::vector<int32_t>> members(csize.size());
  int64_t pos = 0;
  for (size_t c = 0; c < csize.size(); ++c)
    for (int64_t k = 0; k < csize[c]; ++k) { com[order[pos]] = (int32_t)c; members[c].push_back(order[pos]); ++pos; }
  std::vector<Edge> edges;
  std::vector<int32_t> ext;
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) total += deg[i];
  EdgeSet made((size_t)(total / 2));
  edges.reserve((size_t)(total / 2 + 16));
  constexpr int kRounds = 16;
  for (size_t c = 0; c < members.size(); ++c) {
    std::vector<int32_t> stubs;
    for (int32_t v : members[c]) {
      int64_t kin = (int64_t)llround((1.0 - mu) * (double)deg[v]);
      kin = std::min<int64_t>(kin, (int64_t)members[c].size() - 1);
      for (int64_t k = 0; k < kin; ++k) stubs.push_back(v);
      for (int64_t k = kin; k < deg[v]; ++k) ext.push_back(v);
    }
    pair_stubs(stubs, stream(s_in, (u64)c), made, edges, kRounds);
  }
  pair_stubs(ext, s_ex, made, edges, kRounds);
  int rc = build_csr(n, edges, out);
  if (rc) return rc;
  out->truth = (int32_t*)malloc(sizeof(int32_t) * n);
  memcpy(out->truth, com.data(), sizeof(int32_t) * n);
  return 0;
}

// Symmetric CSR from an explicit undirected edge list (for small test
// graphs).  Self-loops are kept once, duplicates merged by summing.
int gen_from_edges(int64_t n, int64_t ne, const int32_t* us, const int32_t* vs,
                   const float* ws, gen_graph* out) {
  memset(out, 0, sizeof(*out));
  std::vector<std::vector<std::pair<int32_t, float>>> adj(n);
  for (i64 e = 0; e < ne; ++e) {
    int32_t u = us[e], v = vs[e];
    float w = ws ? ws[e] : 1.0f;
    if (u < 0 || v < 0 || u >= n || v >= n) return -1;
    adj[u].push_back({v, w});
    if (u != v) adj[v].push_back({u, w});
  }
  std::vector<int32_t> off(n + 1, 0), idx;
  std::vector<float> wt;
  for (i64 i = 0; i < n; ++i) {
    auto& r = adj[i];
    std::sort(r.begin(), r.end());
    for (size_t k = 0; k < r.size(); ++k) {
      if (k > 0 && r[k].first == r[k - 1].first) { wt.back() += r[k].second; continue; }
      idx.push_back(r[k].first); wt.push_back(r[k].second);
    }
    off[i + 1] = (int32_t)idx.size();
  }
  out->n = n; out->m = (int64_t)idx.size();
  out->offsets = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
  out->indices = (int32_t*)malloc(sizeof(int32_t) * (idx.size() + 1));
  out->weights = (float*)malloc(sizeof(float) * (wt.size() + 1));
  memcpy(out->offsets, off.data(), sizeof(int32_t) * (n + 1));
  if (!idx.empty()) {
    memcpy(out->indices, idx.data(), sizeof(int32_t) * idx.size());
    memcpy(out->weights, wt.data(), sizeof(float) * wt.size());
  }
  return 0;
}

}  // extern "C"
