// Plain, slow, single-threaded CPU oracle for GVE-Leiden.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
// call this file: it exists so that tests and the benchmark's CPU baseline
// can check the HIP path against an independent implementation.  It shares
// no code, header, table or helper with the GPU library.
//
// What it computes follows the paper (Sahu, "Fast Leiden Algorithm for
// Community Detection in Shared Memory Setting", arXiv:2312.13936):
//   * Eq. 1  modularity                              -> modularity_exact / modularity_fp
//   * Eq. 2  delta-modularity of moving i from d to c  -> gain_fp / gain_key
//   * Alg. 1 the pass loop (leiden)                  -> run_leiden
//   * Alg. 2 local-moving with flag pruning          -> move_seq / move_det
//   * Alg. 3 refinement by constrained merges        -> refine_seq / refine_det
//   * Alg. 4 aggregation into the super-vertex graph -> aggregate
//   * Alg. 5 disconnected-community check            -> disconnected
//   * the Louvain method (louvain = 1): the same pass loop without the
//     refinement, so each pass aggregates the local-moving communities
//     (Sec. 3.2; the paper's comparison of Leiden with Louvain, Sec. 5)
//
// Two modes:
//   mode 0 "seq-async": the paper's algorithm run by a single thread that
//          visits vertices in ascending id order, applying every move at
//          once (Sec. 4.1 asynchronous updates with T = 1).  FP64 gains as
//          the paper's configuration states (Sec. 5.1.2).
//   mode 1 "det-sync": the deterministic synchronous variant (not in the
//          paper): vertices are split into S pseudo-random groups visited in
//          turn; inside a group every active vertex decides from the state at
//          the start of the group and the moves are applied together; ties
//          go to the lowest community id, two adjacent vertices of a group
//          that chose each other's community do not both move, a vertex
//          bouncing between two communities stops (swap and bounce rules in
//          move_det), and every sum and gain is an exact integer (gains are
//          int128 keys).  Used for bit-exact parity.
//
// Readings of points the paper leaves open (all shared with the GPU path by
// specification, not by code):
//   R1  pass 0 starts from singletons; later passes start from the
//       move-based labels of the previous pass (Alg. 1 "use move-based
//       membership"), with community totals summed over members; option
//       refine_based (Sec. 4.1's alternative) starts them from singletons too.
//   R2  global convergence (Alg. 1's test l_i + l_j <= 1 with l_i, l_j
//       counted as iterations performed): local-moving ran one iteration
//       and refinement moved no vertex.
//   R3  |Gamma| = number of distinct refined labels, |Gamma_old| = |V'|;
//       stop when |Gamma| / |V'| > aggregation tolerance (Alg. 1's low-shrink
//       test).  Option shrink_excludes_isolated (not in the paper) leaves the
//       Z vertices of G' without arcs out of both counts,
//       (|Gamma| - Z) / (|V'| - Z), since such vertices can never merge.
//   R4  the result is the flattening of the last refinement.
//   R5  a move is taken only for a strictly positive gain; ties go to the
//       lowest community id; the own community is never a candidate.
//   R6  renumbering = dense rank of the old label in ascending order; the
//       next-pass label of a super-vertex = dense rank of its bound label.
//   R7  neighbours marked unprocessed after a move exclude the vertex itself.
//   R8  resolution gamma multiplies the null-model term of Eq. 1 and Eq. 2.
//   R9  final labels are numbered by first occurrence over v = 0..N-1.
//   R10 no aggregation on the last allowed pass (it cannot change the result).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

typedef int64_t i64;
typedef __int128 i128;

// Deterministic int128 -> double: hi * 2^64 + lo with one rounding in the add.
double i128_to_double(i128 x) {
  i64 hi = (i64)(x >> 64);
  uint64_t lo = (uint64_t)x;
  return (double)hi * 18446744073709551616.0 + (double)lo;
}

struct Graph {
  i64 n = 0;
  std::vector<i64> off;     // n + 1
  std::vector<int32_t> idx; // arcs
  std::vector<double> w;    // arc weights (exact integers when the input is integral)
};

struct PassTrace {
  i64 n = 0, m = 0;
  int32_t iterations = 0;        // local-moving iterations performed
  int32_t converged_first = 0;   // local-moving stopped in its first iteration
  int32_t refine_sweeps = 0;
  i64 communities = 0;           // |Gamma| after refinement
  std::vector<i64> movers;       // per local-moving iteration
  std::vector<i64> refine_movers;
  std::vector<int32_t> bound;    // local-moving labels (C'_B)
  std::vector<int32_t> refined;  // refinement labels (C')
  bool aggregated = false;
  std::vector<int32_t> y_off;    // canonical super-vertex CSR (rows ascending)
  std::vector<int32_t> y_idx;
  std::vector<double> y_w;
};

struct Opts {
  int32_t mode;
  double tolerance, tolerance_drop, aggregation_tolerance;
  int32_t max_iterations, max_passes, refine_sweeps, subsweeps;
  double resolution;
  int32_t trace;
  int32_t louvain = 0;
  int32_t refine_random = 0;  // refinement picks c with probability proportional to its gain
  uint32_t seed = 0;
  int32_t shrink_excludes_isolated = 0;  // R3 variant: vertices without arcs left out of the ratio
  int32_t refine_based = 0;  // next-pass labels from the refinement (Sec. 4.1) instead of local-moving
};

// Sub-sweep group of vertex i: the MurmurHash3 32-bit finalizer of i, mod S
// (a fixed pseudo-random split of the vertices into S groups).
uint32_t fmix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
  return h;
}
int32_t group_of(i64 i, int32_t S) { return (int32_t)(fmix32((uint32_t)i) % (uint32_t)S); }

// Rows longer than this never yield under the swap rule of the synchronous
// local-moving (move_det) and win against shorter ones.
const i64 kSwapRowMax = 128;

// ---------------------------------------------- randomized refinement ---
// The alternative refinement of Sec. 4.1 (Traag's original rule): among the
// targets with a positive gain, vertex i picks c with probability
// proportional to the gain.  Draws are counter-based, one per (seed, pass,
// sweep, vertex, candidate) of the pass graph: MurmurHash3's finalizer
// mixes the counters into a nonzero xorshift32 state (Marsaglia, "Xorshift
// RNGs", 2003) that takes one step, and u = (x + 1/2) / 2^32.  The candidate
// with the largest gain / (-ln u) wins: -ln u / gain is an exponential clock
// of rate gain, and the first of independent clocks to ring is c with
// probability gain_c / sum of gains.
uint32_t draw32(uint32_t seed, int32_t pass, int32_t sweep, i64 i, int32_t c) {
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

// -ln(u) for u = (x + 1/2) / 2^32, with ln written out: u = m 2^e with m in
// [1, 2), ln m = 2 atanh(z) = 2 (z + z^3/3 + ...), z = (m - 1) / (m + 1) < 1/3,
// 24 terms (the tail is below 1e-23).
double neg_ln_unit(uint32_t x) {
  double m = ((double)x + 0.5) * (1.0 / 4294967296.0);
  int32_t e = 0;
  while (m < 1.0) { m *= 2.0; --e; }
  const double z = (m - 1.0) / (m + 1.0), z2 = z * z;
  double s = 0.0, t = z;
  for (int32_t k = 0; k < 24; ++k) {
    s += t * (1.0 / (double)(2 * k + 1));
    t *= z2;
  }
  return -((double)e * 0.6931471805599453 + 2.0 * s);
}

// Selection score of a candidate with a positive gain (key or FP64 gain).
double random_score(double gain, const Opts& o, int32_t pass, int32_t sweep, i64 i, int32_t c) {
  return gain / neg_ln_unit(draw32(o.seed, pass, sweep, i, c));
}

struct Result {
  std::vector<int32_t> membership;
  double q = 0.0;
  int32_t termination = 0;  // 0 converged, 1 low shrink, 2 max passes, 3 empty graph
  std::vector<PassTrace> passes;
};

// ---------------------------------------------------------------- Eq. 1 ---
// Q = sum_c [ sigma_c / 2m - gamma (Sigma_c / 2m)^2 ], with sigma_c the
// weight of arcs inside c (both directions, self-loop once) and Sigma_c the
// total weighted degree of c.
bool all_integral(const Graph& g) {
  for (double x : g.w) if (x != std::floor(x) || x < 0) return false;
  return true;
}

double modularity_exact(const Graph& g, const std::vector<int32_t>& C, double gamma) {
  i64 W = 0, S1 = 0;
  std::vector<i64> tot(g.n, 0);
  for (i64 i = 0; i < g.n; ++i)
    for (i64 e = g.off[i]; e < g.off[i + 1]; ++e) {
      i64 wi = (i64)g.w[e];
      W += wi;
      tot[C[i]] += wi;
      if (C[g.idx[e]] == C[i]) S1 += wi;
    }
  if (W == 0) return 0.0;
  i128 S2 = 0;
  for (i64 c = 0; c < g.n; ++c) S2 += (i128)tot[c] * (i128)tot[c];
  double Wd = (double)W;
  return (double)S1 / Wd - gamma * (i128_to_double(S2) / (Wd * Wd));
}

double modularity_fp(const Graph& g, const std::vector<int32_t>& C, double gamma) {
  double W = 0, S1 = 0;
  std::vector<double> tot(g.n, 0.0);
  for (i64 i = 0; i < g.n; ++i)
    for (i64 e = g.off[i]; e < g.off[i + 1]; ++e) {
      W += g.w[e];
      tot[C[i]] += g.w[e];
      if (C[g.idx[e]] == C[i]) S1 += g.w[e];
    }
  if (W == 0) return 0.0;
  double S2 = 0;
  for (i64 c = 0; c < g.n; ++c) S2 += tot[c] * tot[c];
  return S1 / W - gamma * (S2 / (W * W));
}

double modularity(const Graph& g, const std::vector<int32_t>& C, double gamma) {
  return all_integral(g) ? modularity_exact(g, C, gamma) : modularity_fp(g, C, gamma);
}

// ---------------------------------------------------------------- Eq. 2 ---
// FP64 delta-modularity of moving i from d to c (m = W / 2):
//   dQ = (K_ic - K_id) / m - gamma K_i (K_i + Sigma_c - Sigma_d) / (2 m^2)
double gain_fp(double kic, double kid, double ki, double sc, double sd, double m, double gamma) {
  return (kic - kid) / m - gamma * ki * (ki + sc - sd) / (2.0 * m * m);
}
// Exact integer key with the same sign and order as Eq. 2 for gamma = p / 2^16:
//   dQ = 2 key / (2^16 W^2),  key = 2^16 W (K_ic - K_id) - p K_i (K_i + Sigma_c - Sigma_d).
i128 gain_key(i64 kic, i64 kid, i64 ki, i64 sc, i64 sd, i64 W, i64 p) {
  return (i128)65536 * (i128)W * (i128)(kic - kid) - (i128)p * (i128)ki * (i128)(ki + sc - sd);
}

// The per-vertex community table H of Alg. 2: a dense array indexed by
// community id plus the list of touched ids (the paper's collision-free
// per-thread table, with one thread).
struct Table {
  std::vector<double> val;
  std::vector<char> used;
  std::vector<int32_t> keys;
  explicit Table(i64 n) : val(n, 0.0), used(n, 0) {}
  void add(int32_t c, double w) {
    if (!used[c]) { used[c] = 1; keys.push_back(c); val[c] = 0.0; }
    val[c] += w;
  }
  double get(int32_t c) const { return used[c] ? val[c] : 0.0; }
  void clear() { for (int32_t c : keys) { used[c] = 0; val[c] = 0.0; } keys.clear(); }
};

// scanCommunities / scanBounded (Alg. 2, Alg. 3): accumulate the weight of
// the arcs of i towards each community, skipping i itself, optionally only
// towards vertices with the same bound label.
void scan(Table& H, const Graph& g, const std::vector<int32_t>& C, i64 i,
          const std::vector<int32_t>* bound) {
  for (i64 e = g.off[i]; e < g.off[i + 1]; ++e) {
    int32_t j = g.idx[e];
    if (j == i) continue;
    if (bound && (*bound)[j] != (*bound)[i]) continue;
    H.add(C[j], g.w[e]);
  }
}

struct State {
  std::vector<int32_t> C;   // community of each vertex
  std::vector<double> K;    // weighted degree of each vertex
  std::vector<double> S;    // total weight of each community
  std::vector<i64> size;    // vertices in each community
};

// --------------------------------------------------- Alg. 2, seq-async ---
// Returns the number of iterations performed; *first = converged in the
// first iteration.
int32_t move_seq(const Graph& g, State& st, double tau, const Opts& o, double W,
                 std::vector<i64>* movers, int32_t* first) {
  const i64 n = g.n;
  const double m = W / 2.0, gamma = o.resolution;
  std::vector<char> unprocessed(n, 1);
  Table H(n);
  int32_t it = 0;
  *first = 0;
  for (; it < o.max_iterations; ++it) {
    double dQ = 0.0;
    i64 moved = 0;
    for (i64 i = 0; i < n; ++i) {
      if (!unprocessed[i]) continue;
      unprocessed[i] = 0;
      scan(H, g, st.C, i, nullptr);
      const int32_t d = st.C[i];
      const double kid = H.get(d), ki = st.K[i];
      int32_t best = -1;
      double bg = 0.0;
      for (int32_t c : H.keys) {
        if (c == d) continue;
        double x = gain_fp(H.val[c], kid, ki, st.S[c], st.S[d], m, gamma);
        if (best < 0 || x > bg || (x == bg && c < best)) { best = c; bg = x; }
      }
      H.clear();
      if (best < 0 || !(bg > 0.0)) continue;
      st.S[d] -= ki; st.S[best] += ki;
      st.size[d] -= 1; st.size[best] += 1;
      st.C[i] = best;
      dQ += bg;
      ++moved;
      for (i64 e = g.off[i]; e < g.off[i + 1]; ++e)
        if (g.idx[e] != i) unprocessed[g.idx[e]] = 1;
    }
    if (movers) movers->push_back(moved);
    if (dQ <= tau) { if (it == 0) *first = 1; ++it; break; }
  }
  return it;
}

// ---------------------------------------------------- Alg. 2, det-sync ---
int32_t move_det(const Graph& g, State& st, double tau, const Opts& o, i64 W, i64 p,
                 std::vector<i64>* movers, int32_t* first) {
  const i64 n = g.n;
  const int32_t S = std::max<int32_t>(1, o.subsweeps);
  std::vector<char> unprocessed(n, 1);
  std::vector<int32_t> target(n, -1);
  std::vector<i128> key(n, 0);
  // last move of each vertex: the community it left and the iteration, and
  // the iteration of the move before (bounce rule)
  std::vector<int32_t> left(n, -1), left_it(n, -3), prev_it(n, -3);
  Table H(n);
  int32_t it = 0;
  *first = 0;
  const double denom = 65536.0 * (double)W * (double)W;
  for (; it < o.max_iterations; ++it) {
    i128 sum = 0;
    i64 moved = 0;
    for (int32_t sub = 0; sub < S; ++sub) {
      std::vector<i64> group;
      for (i64 i = 0; i < n; ++i) {
        if (group_of(i, S) != sub) continue;
        target[i] = -1;
        if (!unprocessed[i]) continue;
        unprocessed[i] = 0;
        scan(H, g, st.C, i, nullptr);
        const int32_t d = st.C[i];
        const i64 kid = (i64)H.get(d), ki = (i64)st.K[i];
        int32_t best = -1;
        i128 bk = 0;
        for (int32_t c : H.keys) {
          if (c == d) continue;
          i128 x = gain_key((i64)H.val[c], kid, ki, (i64)st.S[c], (i64)st.S[d], W, p);
          if (best < 0 || x > bk || (x == bk && c < best)) { best = c; bk = x; }
        }
        H.clear();
        if (best < 0 || !(bk > 0)) continue;
        if (st.size[d] == 1 && st.size[best] == 1 && best > d) continue;  // min-label rule
        // Bounce rule: a vertex that moved in each of the two previous
        // iterations does not go straight back to the community it left in
        // the last one (it is cycling with a neighbour of its group).
        if (best == left[i] && left_it[i] == it - 1 && prev_it[i] == it - 2) continue;
        target[i] = best; key[i] = bk;
        group.push_back(i);
      }
      // Swap rule: two adjacent vertices of the group that chose each
      // other's community (i: d -> c while j: c -> d) would trade places and
      // trade back in the next iteration; only one of them moves: the
      // lower id, or the one with more than kSwapRowMax arcs (such rows
      // never yield).  Decided on the state before the group's moves.
      std::vector<i64> go;
      for (i64 i : group) {
        bool yield = false;
        if (g.off[i + 1] - g.off[i] <= kSwapRowMax) {
          const int32_t d = st.C[i], c = target[i];
          for (i64 e = g.off[i]; e < g.off[i + 1] && !yield; ++e) {
            const i64 j = g.idx[e];
            if (j == i || group_of(j, S) != sub || target[j] != d || st.C[j] != c) continue;
            yield = j < i || g.off[j + 1] - g.off[j] > kSwapRowMax;
          }
        }
        if (!yield) go.push_back(i);
      }
      for (i64 i : go) {  // apply the group's moves together
        const int32_t d = st.C[i], c = target[i];
        prev_it[i] = left_it[i];
        left[i] = d;
        left_it[i] = it;
        st.S[d] -= st.K[i]; st.S[c] += st.K[i];
        st.size[d] -= 1; st.size[c] += 1;
        st.C[i] = c;
        sum += key[i];
        ++moved;
      }
      for (i64 i : go)
        for (i64 e = g.off[i]; e < g.off[i + 1]; ++e)
          if (g.idx[e] != i) unprocessed[g.idx[e]] = 1;
    }
    if (movers) movers->push_back(moved);
    const double dq = i128_to_double(sum) * 2.0 / denom;
    if (dq <= tau) { if (it == 0) *first = 1; ++it; break; }
  }
  return it;
}

// --------------------------------------------------- Alg. 3, seq-async ---
// One sweep in ascending order (the paper's single parallel loop with one
// thread); the isolation test is the paper's Sigma'[c] == K'[i].
int32_t refine_seq(const Graph& g, State& st, const std::vector<int32_t>& bound, const Opts& o,
                   double W, int32_t pass, std::vector<i64>* movers) {
  const i64 n = g.n;
  const double m = W / 2.0, gamma = o.resolution;
  Table H(n);
  int32_t sw = 0;
  for (; sw < std::max<int32_t>(1, o.refine_sweeps); ++sw) {
    i64 moved = 0;
    for (i64 i = 0; i < n; ++i) {
      const int32_t d = st.C[i];
      if (st.S[d] != st.K[i]) continue;
      scan(H, g, st.C, i, &bound);
      const double kid = H.get(d), ki = st.K[i];
      int32_t best = -1;
      double bg = 0.0;
      for (int32_t c : H.keys) {
        if (c == d) continue;
        double x = gain_fp(H.val[c], kid, ki, st.S[c], st.S[d], m, gamma);
        if (o.refine_random) {
          if (!(x > 0.0)) continue;
          x = random_score(x, o, pass, sw, i, c);
        }
        if (best < 0 || x > bg || (x == bg && c < best)) { best = c; bg = x; }
      }
      H.clear();
      if (best < 0 || !(bg > 0.0)) continue;
      // atomicCAS(Sigma'[d], K'[i], 0) always succeeds with one thread.
      st.S[d] = 0.0;
      st.S[best] += ki;
      st.size[d] -= 1; st.size[best] += 1;
      st.C[i] = best;
      ++moved;
    }
    if (movers) movers->push_back(moved);
    if (moved == 0) { ++sw; break; }
  }
  return sw;
}

// ---------------------------------------------------- Alg. 3, det-sync ---
// Sweeps until no vertex moves (at most refine_sweeps).  Each sweep visits
// the S vertex groups in turn; inside a group every isolated vertex
// (community of size one) picks its best in-bound target from the state at
// the start of the group, and moves only if no vertex of the group picked
// its own community as a target.
int32_t refine_det(const Graph& g, State& st, const std::vector<int32_t>& bound, const Opts& o,
                   i64 W, i64 p, int32_t pass, std::vector<i64>* movers) {
  const i64 n = g.n;
  const int32_t S = std::max<int32_t>(1, o.subsweeps);
  std::vector<int32_t> target(n, -1);
  std::vector<char> targeted(n, 0);
  Table H(n);
  int32_t sw = 0;
  for (; sw < std::max<int32_t>(1, o.refine_sweeps); ++sw) {
    i64 moved = 0;
    for (int32_t sub = 0; sub < S; ++sub) {
      std::vector<i64> group;
      for (i64 i = 0; i < n; ++i) {
        if (group_of(i, S) != sub) continue;
        target[i] = -1;
        const int32_t d = st.C[i];
        if (st.size[d] != 1 || st.K[i] == 0.0) continue;
        scan(H, g, st.C, i, &bound);
        const i64 kid = (i64)H.get(d), ki = (i64)st.K[i];
        int32_t best = -1;
        i128 bk = 0;
        double bs = 0.0;
        for (int32_t c : H.keys) {
          if (c == d) continue;
          i128 x = gain_key((i64)H.val[c], kid, ki, (i64)st.S[c], (i64)st.S[d], W, p);
          if (o.refine_random) {  // largest score among positive keys, lowest id on ties
            if (!(x > 0)) continue;
            const double s = random_score(i128_to_double(x), o, pass, sw, i, c);
            if (best < 0 || s > bs || (s == bs && c < best)) { best = c; bs = s; bk = x; }
            continue;
          }
          if (best < 0 || x > bk || (x == bk && c < best)) { best = c; bk = x; }
        }
        H.clear();
        if (best < 0 || !(bk > 0)) continue;
        if (st.size[best] == 1 && best > d) continue;  // min-label rule
        target[i] = best;
        group.push_back(i);
      }
      for (i64 i : group) targeted[target[i]] = 1;
      std::vector<i64> go;
      for (i64 i : group)
        if (!targeted[st.C[i]]) go.push_back(i);
      for (i64 i : group) targeted[target[i]] = 0;
      for (i64 i : go) {
        const int32_t d = st.C[i], c = target[i];
        st.S[d] -= st.K[i]; st.S[c] += st.K[i];
        st.size[d] -= 1; st.size[c] += 1;
        st.C[i] = c;
      }
      moved += (i64)go.size();
    }
    if (movers) movers->push_back(moved);
    if (moved == 0) { ++sw; break; }
  }
  return sw;
}

// Dense rank of the labels in use, ascending: out[c] = rank, or -1 if unused.
std::vector<int32_t> dense_rank(const std::vector<int32_t>& labels, i64 space, i64* count) {
  std::vector<char> used(space, 0);
  for (int32_t c : labels) used[c] = 1;
  std::vector<int32_t> r(space, -1);
  int32_t k = 0;
  for (i64 c = 0; c < space; ++c) if (used[c]) r[c] = k++;
  *count = k;
  return r;
}

// ---------------------------------------------------------------- Alg. 4 ---
// Super-vertex graph: row r sums, over every member i of community r and
// every arc (j, w) of i including a self-loop, w into the entry of j's
// community.  `lab` must be dense in [0, nc).  Rows come out sorted.
Graph aggregate(const Graph& g, const std::vector<int32_t>& lab, i64 nc) {
  // community-vertex CSR (countCommunityVertices + exclusiveScan + fill)
  std::vector<i64> coff(nc + 1, 0);
  for (i64 i = 0; i < g.n; ++i) coff[lab[i] + 1] += 1;
  for (i64 c = 0; c < nc; ++c) coff[c + 1] += coff[c];
  std::vector<int32_t> cv(g.n);
  std::vector<i64> cur(coff.begin(), coff.end() - 1);
  for (i64 i = 0; i < g.n; ++i) cv[cur[lab[i]]++] = (int32_t)i;
  Graph y;
  y.n = nc;
  y.off.assign(nc + 1, 0);
  Table H(nc);
  for (i64 c = 0; c < nc; ++c) {
    for (i64 k = coff[c]; k < coff[c + 1]; ++k) {
      i64 i = cv[k];
      for (i64 e = g.off[i]; e < g.off[i + 1]; ++e) H.add(lab[g.idx[e]], g.w[e]);
    }
    std::vector<int32_t> keys = H.keys;
    std::sort(keys.begin(), keys.end());
    for (int32_t d : keys) { y.idx.push_back(d); y.w.push_back(H.val[d]); }
    y.off[c + 1] = (i64)y.idx.size();
    H.clear();
  }
  return y;
}

void init_state(const Graph& g, State& st, const std::vector<int32_t>& start) {
  const i64 n = g.n;
  st.K.assign(n, 0.0);
  for (i64 i = 0; i < n; ++i)
    for (i64 e = g.off[i]; e < g.off[i + 1]; ++e) st.K[i] += g.w[e];
  st.C = start;
  st.S.assign(n, 0.0);
  st.size.assign(n, 0);
  for (i64 i = 0; i < n; ++i) { st.S[st.C[i]] += st.K[i]; st.size[st.C[i]] += 1; }
}

// ---------------------------------------------------------------- Alg. 1 ---
int run_leiden(const Graph& g0, const Opts& o, Result& res) {
  const i64 N = g0.n;
  const bool det = (o.mode == 1);
  double Wd = 0.0;
  i64 Wi = 0;
  for (double x : g0.w) { Wd += x; Wi += (i64)x; }
  i64 p = 0;
  if (det) {
    if (!all_integral(g0)) return -4;
    for (double x : g0.w) if (x > 16777216.0 || x <= 0.0) return -4;
    if (Wi > ((i64)1 << 40)) return -4;
    double pd = o.resolution * 65536.0;
    p = (i64)pd;
    if ((double)p != pd || p < 0 || p > ((i64)1 << 24)) return -5;
  }
  std::vector<int32_t> top(N);
  for (i64 v = 0; v < N; ++v) top[v] = (int32_t)v;
  if (N == 0 || Wd == 0.0) {
    res.membership = top;
    res.q = 0.0;
    res.termination = 3;
    return 0;
  }
  Graph cur = g0;
  std::vector<int32_t> start(N);
  for (i64 v = 0; v < N; ++v) start[v] = (int32_t)v;
  double tau = o.tolerance;
  res.termination = 2;
  std::vector<int32_t> final_refined;  // refined labels of the pass that ended the run
  bool ended = false;
  for (int32_t pass = 0; pass < o.max_passes; ++pass) {
    const i64 n = cur.n;
    State st;
    init_state(cur, st, start);
    PassTrace tr;
    tr.n = n; tr.m = (i64)cur.idx.size();
    int32_t first = 0;
    tr.iterations = det ? move_det(cur, st, tau, o, Wi, p, &tr.movers, &first)
                        : move_seq(cur, st, tau, o, Wd, &tr.movers, &first);
    tr.converged_first = first;
    std::vector<int32_t> bound = st.C;
    if (!o.louvain) {
      // refinement starts from singletons inside the bounds (Alg. 1)
      std::vector<int32_t> ident(n);
      for (i64 i = 0; i < n; ++i) ident[i] = (int32_t)i;
      init_state(cur, st, ident);
      tr.refine_sweeps = det ? refine_det(cur, st, bound, o, Wi, p, pass, &tr.refine_movers)
                             : refine_seq(cur, st, bound, o, Wd, pass, &tr.refine_movers);
    }
    // (the Louvain method aggregates the local-moving communities themselves)
    i64 ncom = 0;
    std::vector<int32_t> rank = dense_rank(st.C, n, &ncom);
    tr.communities = ncom;
    if (o.trace) { tr.bound = bound; tr.refined = st.C; }
    i64 refine_moved = 0;
    for (i64 x : tr.refine_movers) refine_moved += x;
    bool stop = false;
    if (first && refine_moved == 0) { res.termination = 0; stop = true; }
    else {
      // Alg. 1 low shrink: |Gamma| / |Gamma_old| with |Gamma_old| = |V'|.
      // The variant leaves the vertices without arcs (singletons for ever)
      // out of both counts.
      i64 z = 0;
      if (o.shrink_excludes_isolated)
        for (i64 i = 0; i < n; ++i) if (cur.off[i + 1] == cur.off[i]) ++z;
      if (n == z || (double)(ncom - z) / (double)(n - z) > o.aggregation_tolerance) { res.termination = 1; stop = true; }
    }
    if (stop) {
      final_refined = st.C;
      res.passes.push_back(std::move(tr));
      ended = true;
      break;
    }
    std::vector<int32_t> lab(n);
    for (i64 i = 0; i < n; ++i) lab[i] = rank[st.C[i]];
    for (i64 v = 0; v < N; ++v) top[v] = lab[top[v]];
    if (pass + 1 < o.max_passes) {
      Graph y = aggregate(cur, lab, ncom);
      // next-pass labels (Sec. 4.1): move-based, the dense rank of the
      // local-moving label of each super-vertex (Alg. 1); refine-based, the
      // super-vertex's own refined community, i.e. every super-vertex alone
      std::vector<int32_t> nstart(ncom, 0);
      if (o.refine_based) {
        for (i64 c = 0; c < ncom; ++c) nstart[c] = (int32_t)c;
      } else {
        i64 nb = 0;
        std::vector<int32_t> brank = dense_rank(bound, n, &nb);
        for (i64 i = 0; i < n; ++i) nstart[lab[i]] = brank[bound[i]];
      }
      if (o.trace) {
        tr.aggregated = true;
        tr.y_off.resize(y.n + 1);
        for (i64 r = 0; r <= y.n; ++r) tr.y_off[r] = (int32_t)y.off[r];
        tr.y_idx = y.idx;
        tr.y_w = y.w;
      }
      cur = std::move(y);
      start = std::move(nstart);
    }
    res.passes.push_back(std::move(tr));
    tau = tau / o.tolerance_drop;
  }
  if (ended) for (i64 v = 0; v < N; ++v) top[v] = final_refined[top[v]];
  // canonical labels: first occurrence over v = 0..N-1
  std::vector<int32_t> first_id(N, -1);
  int32_t k = 0;
  res.membership.resize(N);
  for (i64 v = 0; v < N; ++v) {
    if (first_id[top[v]] < 0) first_id[top[v]] = k++;
    res.membership[v] = first_id[top[v]];
  }
  res.q = modularity(g0, res.membership, o.resolution);
  return 0;
}

Graph from_csr(i64 n, const int32_t* off, const int32_t* idx, const float* w) {
  Graph g;
  g.n = n;
  g.off.resize(n + 1);
  for (i64 i = 0; i <= n; ++i) g.off[i] = off[i];
  i64 m = g.off[n];
  g.idx.assign(idx, idx + m);
  g.w.resize(m);
  for (i64 e = 0; e < m; ++e) g.w[e] = w ? (double)w[e] : 1.0;
  return g;
}

}  // namespace

extern "C" {

typedef struct {
  int32_t mode;                  // 0 seq-async, 1 det-sync
  double tolerance;              // initial per-iteration tolerance (0.01)
  double tolerance_drop;         // threshold scaling factor (10)
  double aggregation_tolerance;  // 0.8
  int32_t max_iterations;        // 20
  int32_t max_passes;            // 20
  int32_t refine_sweeps;         // seq-async: 1; det-sync: cap on sweeps
  int32_t subsweeps;             // det-sync: pseudo-random vertex groups visited in turn
  double resolution;             // gamma
  int32_t trace;                 // keep per-pass labels and super-vertex CSRs
  int32_t louvain;               // 1: no refinement (the Louvain method)
  int32_t refine_random;         // 1: randomized refinement (gain-proportional choice)
  uint32_t seed;                 // its seed
  int32_t shrink_excludes_isolated;  // 1: low-shrink ratio without the vertices that have no arcs
  int32_t refine_based;          // 1: refine-based next-pass labels (each super-vertex alone)
} oracle_opts;

void oracle_default_opts(oracle_opts* o, int32_t mode) {
  o->mode = mode;
  o->tolerance = 0.01;
  o->tolerance_drop = 10.0;
  o->aggregation_tolerance = 0.8;
  o->max_iterations = 20;
  o->max_passes = 20;
  o->refine_sweeps = mode == 1 ? 20 : 1;
  o->subsweeps = mode == 1 ? 32 : 1;
  o->resolution = 1.0;
  o->trace = 0;
  o->louvain = 0;
  o->refine_random = 0;
  o->seed = 0;
  o->shrink_excludes_isolated = 0;
  o->refine_based = 0;
}

// Runs Leiden; returns an opaque result handle, or NULL with *status set.
void* oracle_leiden(int64_t n, const int32_t* off, const int32_t* idx, const float* w,
                    const oracle_opts* o, int32_t* status) {
  Graph g = from_csr(n, off, idx, w);
  Opts op;
  op.mode = o->mode; op.tolerance = o->tolerance; op.tolerance_drop = o->tolerance_drop;
  op.aggregation_tolerance = o->aggregation_tolerance; op.max_iterations = o->max_iterations;
  op.max_passes = o->max_passes; op.refine_sweeps = o->refine_sweeps; op.subsweeps = o->subsweeps;
  op.resolution = o->resolution; op.trace = o->trace; op.louvain = o->louvain;
  op.refine_random = o->refine_random; op.seed = o->seed;
  op.shrink_excludes_isolated = o->shrink_excludes_isolated;
  op.refine_based = o->refine_based;
  Result* r = new Result();
  int rc = run_leiden(g, op, *r);
  *status = rc;
  if (rc != 0) { delete r; return nullptr; }
  return r;
}

void oracle_free(void* h) { delete (Result*)h; }

double oracle_result(void* h, int32_t* membership, int32_t* passes, int32_t* termination) {
  Result* r = (Result*)h;
  if (membership) memcpy(membership, r->membership.data(), sizeof(int32_t) * r->membership.size());
  if (passes) *passes = (int32_t)r->passes.size();
  if (termination) *termination = r->termination;
  return r->q;
}

// Per-pass summary: sizes, iteration counts, |Gamma|, super-graph size.
int oracle_pass_info(void* h, int32_t pass, int64_t* info /* 8 */) {
  Result* r = (Result*)h;
  if (pass < 0 || pass >= (int32_t)r->passes.size()) return -1;
  const PassTrace& t = r->passes[pass];
  info[0] = t.n; info[1] = t.m; info[2] = t.iterations; info[3] = t.converged_first;
  info[4] = t.refine_sweeps; info[5] = t.communities;
  info[6] = t.aggregated ? (int64_t)t.y_idx.size() : -1;
  info[7] = t.aggregated ? 1 : 0;
  return 0;
}

int oracle_pass_movers(void* h, int32_t pass, int64_t* movers, int64_t* refine_movers) {
  Result* r = (Result*)h;
  if (pass < 0 || pass >= (int32_t)r->passes.size()) return -1;
  const PassTrace& t = r->passes[pass];
  if (movers) memcpy(movers, t.movers.data(), sizeof(int64_t) * t.movers.size());
  if (refine_movers) memcpy(refine_movers, t.refine_movers.data(), sizeof(int64_t) * t.refine_movers.size());
  return 0;
}

// Labels and (if aggregated) the canonical super-vertex CSR of a pass.
int oracle_pass_get(void* h, int32_t pass, int32_t* bound, int32_t* refined, int32_t* y_off,
                    int32_t* y_idx, double* y_w) {
  Result* r = (Result*)h;
  if (pass < 0 || pass >= (int32_t)r->passes.size()) return -1;
  const PassTrace& t = r->passes[pass];
  if (t.bound.empty() && t.n > 0) return -2;  // not traced
  if (bound) memcpy(bound, t.bound.data(), sizeof(int32_t) * t.bound.size());
  if (refined) memcpy(refined, t.refined.data(), sizeof(int32_t) * t.refined.size());
  if (t.aggregated) {
    if (y_off) memcpy(y_off, t.y_off.data(), sizeof(int32_t) * t.y_off.size());
    if (y_idx) memcpy(y_idx, t.y_idx.data(), sizeof(int32_t) * t.y_idx.size());
    if (y_w) memcpy(y_w, t.y_w.data(), sizeof(double) * t.y_w.size());
  }
  return 0;
}

// Eq. 1 on a CSR graph for any membership with labels in [0, n).
double oracle_modularity(int64_t n, const int32_t* off, const int32_t* idx, const float* w,
                         const int32_t* membership, double gamma) {
  Graph g = from_csr(n, off, idx, w);
  std::vector<int32_t> C(membership, membership + n);
  return modularity(g, C, gamma);
}

// Eq. 2 for moving vertex i from its community to community c, FP64.
double oracle_delta_modularity(int64_t n, const int32_t* off, const int32_t* idx, const float* w,
                               const int32_t* membership, int64_t i, int32_t c, double gamma) {
  Graph g = from_csr(n, off, idx, w);
  State st;
  std::vector<int32_t> C(membership, membership + n);
  init_state(g, st, C);
  double W = 0;
  for (double x : g.w) W += x;
  Table H(n);
  scan(H, g, st.C, i, nullptr);
  const int32_t d = st.C[i];
  return gain_fp(H.get(c), H.get(d), st.K[i], st.S[c], st.S[d], W / 2.0, gamma);
}

// The exact integer key of Eq. 2 used by the deterministic mode, for
// gamma = p / 2^16, as its high (signed) and low 64-bit words.
void oracle_gain_key(int64_t kic, int64_t kid, int64_t ki, int64_t sc, int64_t sd, int64_t W, int64_t p,
                     int64_t* hi, uint64_t* lo) {
  const i128 k = gain_key(kic, kid, ki, sc, sd, W, p);
  *hi = (int64_t)(k >> 64);
  *lo = (uint64_t)k;
}

// Alg. 4 on its own: writes the super-vertex CSR for dense labels in
// [0, nc).  Returns the number of arcs; buffers may be NULL to query it.
int64_t oracle_aggregate(int64_t n, const int32_t* off, const int32_t* idx, const float* w,
                         const int32_t* labels, int64_t nc, int32_t* y_off, int32_t* y_idx, double* y_w) {
  Graph g = from_csr(n, off, idx, w);
  std::vector<int32_t> lab(labels, labels + n);
  Graph y = aggregate(g, lab, nc);
  if (y_off) for (int64_t r = 0; r <= nc; ++r) y_off[r] = (int32_t)y.off[r];
  if (y_idx) memcpy(y_idx, y.idx.data(), sizeof(int32_t) * y.idx.size());
  if (y_w) memcpy(y_w, y.w.data(), sizeof(double) * y.w.size());
  return (int64_t)y.idx.size();
}

// Selection score of the randomized refinement for one candidate (exposed
// for the distribution tests).
double oracle_random_score(double gain, uint32_t seed, int32_t pass, int32_t sweep, int64_t i, int32_t c) {
  Opts o{};
  o.seed = seed;
  return random_score(gain, o, pass, sweep, i, c);
}
double oracle_neg_ln_unit(uint32_t x) { return neg_ln_unit(x); }

// Alg. 5: flag[c] = 1 if the vertices of community c are not all reachable
// from one member through vertices of c.  Returns the number flagged.
int64_t oracle_disconnected(int64_t n, const int32_t* off, const int32_t* idx,
                            const int32_t* membership, int32_t* flag) {
  std::vector<i64> size(n, 0);
  for (i64 i = 0; i < n; ++i) size[membership[i]] += 1;
  std::vector<char> vis(n, 0);
  std::vector<int32_t> queue;
  int64_t bad = 0;
  for (i64 c = 0; c < n; ++c) if (flag) flag[c] = 0;
  for (i64 i = 0; i < n; ++i) {
    const int32_t c = membership[i];
    if (size[c] == 0) continue;
    i64 reached = 0;
    queue.clear();
    queue.push_back((int32_t)i);
    vis[i] = 1;
    for (size_t q = 0; q < queue.size(); ++q) {
      int32_t u = queue[q];
      ++reached;
      for (i64 e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = idx[e];
        if (!vis[v] && membership[v] == c) { vis[v] = 1; queue.push_back(v); }
      }
    }
    if (reached < size[c]) { if (flag) flag[c] = 1; ++bad; }
    size[c] = 0;
  }
  return bad;
}

}  // extern "C"
