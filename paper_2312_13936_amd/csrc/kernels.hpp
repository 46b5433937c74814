// Host-side launch interface of the gvl kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gvl {

typedef __int128 i128_t;

constexpr int32_t kEmpty = -1;        // empty hash-table slot
// Work counters and iteration sums are kept in kCntSlots copies indexed by
// workgroup id, so that thousands of workgroups do not serialise on one
// address; the host adds the copies up.
constexpr int kCntSlots = 64;
enum Phase { kMove = 0, kRefine = 1 };  // local-moving (Alg. 2) / refinement (Alg. 3)

// Degree bins (vertex scan) and capacity bins (aggregation rows).  A vertex
// of degree d (or a community whose member arcs total d) goes to the first
// bin with d <= kBinMax[b]; d == 0 is never binned.  Bins 0-4 map a group of
// kBinLanes[b] lanes of one wavefront to each item with an LDS hash table of
// up to 2^8 slots (one to four arcs per lane: more rows in flight than one
// arc per lane); bin 5 maps a 256-thread workgroup with an LDS table.  Bins 6-8 ("wide" rows) map 1, 1 or 2
// workgroups of 1024 threads to a vertex, each with an LDS table of up to
// kWideSlots slots for one partition of the neighbour communities; the
// aggregation uses bins 6-7 (one workgroup per community) and sends
// capacities above kBinMax[kAggLastBin] to the last bin.  The last bin (hubs
// and giant communities) is split by key partitions; only vertex hubs of
// more than kPartMaxDeg arcs use global-memory tables.
constexpr int kNumBins = 10;
constexpr int32_t kBinMax[kNumBins] = {4, 8, 16, 32, 128, 1024, 4096, 8192, 16384, 0x7fffffff};
constexpr int kBinLanes[kNumBins] = {4, 8, 8, 16, 32, 256, 1024, 1024, 2048, 256};
constexpr int kWideBin0 = 6;       // first wide bin
constexpr int kWideClasses = 3;
// bin kWideBin0 + k uses 2^kWideShift[k] partitions of the key space
constexpr int kWideShift[kWideClasses] = {0, 0, 1};
constexpr int kWideMaxParts = 2;
constexpr int kWideSlots = 12288;  // 144 KiB of LDS (keys + FP64 values)
// Aggregation uses bins kWideBin0 .. kAggLastBin (capacities up to 8192 arcs,
// one 1024-thread workgroup and LDS table per community); larger
// capacities take the global-table path.
constexpr int kAggLastBin = 7;
constexpr int kHubBin = kNumBins - 1;

// Bin limits in use: the upper limits of the lane-group bins 0-4 and of the
// workgroup bin 5 are tunable at run time, each at most its compiled
// kBinMax (the kernels of a bin handle any shorter row) and non-decreasing;
// a bin whose limit equals its predecessor's is empty.  Longer bins keep
// kBinMax.  The lowest allowed limit of bin 5 bounds the wide-row work
// arrays of the workspace.
constexpr int kTunedBins = 6;
constexpr int32_t kMinBin5 = 256;
struct BinLimits {
  int32_t v[kNumBins];
};

// Local-moving and refinement visit the vertices in S pseudo-random groups
// (sub-sweeps); the bin lists are laid out group-major so that every
// (group, bin) segment is contiguous.
constexpr int kMaxGroups = 64;
// Fast mode with subsweeps = 0 picks S per input graph: kAutoFewGroups when
// no row has more than kAutoShortRow arcs, else kAutoGroups.  In a fused
// batch a graph with fewer groups than the union puts its group k into
// union group k << shift (shift = log2 of the ratio), so its groups run in
// the same order as alone.
constexpr int kAutoGroups = 32;
constexpr int kAutoFewGroups = 8;
constexpr int32_t kAutoShortRow = 128;
// Synchronous local-moving: rows of more than kSwapRowMax arcs never yield
// under the swap rule and win against shorter rows (a cycle among them is
// stopped by the bounce rule).
constexpr int32_t kSwapRowMax = 128;
// last-move entry of a vertex that has not moved in the pass: no community,
// iterations -3 and -3 (16 bits each); iterations of a pass fit 16 bits
constexpr int32_t kNoLastMove = (int32_t)0xFFFDFFFDu;
constexpr int32_t kMaxIterationsSync = 32767;
static_assert(kSwapRowMax <= kBinMax[4], "rows of the swap rule sit in the lane-group bins or bin 5");

// List layout: for every group its bins 0..kHubBin-1 (group-major), then the
// hub bin of every group, so that all hubs form one region [H0, H0 + H).
struct BinInfo {
  int32_t S;                               // groups (1 for aggregation)
  int32_t count[kMaxGroups][kNumBins];
  int32_t start[kMaxGroups][kNumBins];
  int32_t gstart[kMaxGroups + 1];          // non-hub items of group g: [gstart[g], gend[g])
  int32_t gend[kMaxGroups];
  int32_t H0, H;                           // hub region
  int32_t binned;                          // items with at least one arc
  int32_t maxsize[kNumBins];
};

// Device-side binning counters: counts[g * kNumBins + b], then maxsize[b].
struct BinBuf {
  int32_t counts[kMaxGroups * kNumBins];
  int32_t maxsize[kNumBins];
  int32_t cursors[kMaxGroups * kNumBins];
  int32_t pad;
  // refinement thinning: kept items, their new bin starts, placement cursors
  int32_t kept[kMaxGroups * kNumBins];
  int32_t nstart[kMaxGroups * kNumBins];
  int32_t ncur[kMaxGroups * kNumBins];
};

// Per-graph constants of a fused batch (several graphs in one union graph).
struct GraphParam {
  double inv_m;             // 2 / W
  double gk_scale;          // 2 gamma / W^2
  long long W;              // exact total weight (deterministic mode)
  long long p;              // resolution numerator (deterministic mode)
};

// State read and written by the local-moving / refinement decision kernels.
struct ScanArgs {
  int32_t* C;               // community of each vertex (C')
  const int32_t* CB;        // community bound (C'_B), refinement only
  // synchronous local-moving commits: in the first sweep of a pass every
  // vertex of a later sub-sweep group (of `groups`) is still unprocessed
  // (flag 1), so the commit of group mark_after skips marking those;
  // mark_after = INT32_MAX marks every neighbour
  int32_t mark_after, groups;
  // pass 0, first local-moving sweep, decisions of group ident_after: a
  // vertex of a later sub-sweep group has not moved yet, so C'[j] = j needs
  // no load; -1 = off
  int32_t ident_after;
  int2* CP;                 // refinement: (C'[j], C'_B[j]) side by side, so one load per arc serves the
                            // bound test (the commit keeps .x equal to C')
  double* Sig;              // total weight of each community (Sigma')
  int32_t* size;            // vertices in each community
  const double* K;          // weighted degree of each vertex (K')
  uint8_t* flag;            // local-moving: 1 = unprocessed
  int32_t* target;          // synchronous decisions: chosen community or -1
  int32_t* targeted;        // refinement: stamp of the last group that chose the community as a target
  int32_t stamp;            // refinement: stamp of the current group (unique within a pass, > 0): with
                            // sweep_dev, stamp + *sweep_dev * groups
  const int32_t* sweep_dev; // refinement sweep number in device memory (a replayed sweep reads it
                            // there), or nullptr: the stamp and sweep fields hold the values
  double inv_m;             // 1/m = 2/W
  double gk_scale;          // 2 gamma / W^2
  long long W;              // exact total weight (deterministic mode)
  long long p;              // resolution numerator, gamma = p / 65536 (deterministic mode)
  double* dq;               // fast mode: sum of the gains of the moves made [kCntSlots]
  unsigned long long* dq128;  // deterministic mode: exact int128 sums of move keys [kCntSlots][lo, hi]
  unsigned long long* cnt;  // [kCntSlots][8]: [0] vertices scanned, [1] arcs, [2] candidates,
                            // [3] moves, [4..6] aggregation, [7] arcs scanned by refinement
  unsigned long long* ovf;  // decisions of wide rows and hubs cancelled by a partition table overflow
  // synchronous local-moving (the swap and bounce rules): decisions add
  // their gains to the iteration's sum; a swap-rule candidate (its target
  // stored as -2 - target) also keeps its gain here, which the commit takes
  // back if the move yields (gaink in deterministic mode, else gainf); each
  // vertex's last move (community left; iteration of that move in the low
  // and of the move before in the high 16 bits); the move records the
  // swap rule reads: (community, target, stamp of the iteration and group,
  // 0), written by the decisions of every row longer than kSwapRowMax and
  // of the shorter rows whose target holds a neighbour of the same group,
  // and only read by the commits (stamps are reset every pass); the pass's
  // iteration number in device memory
  double* gainf;
  i128_t* gaink;
  int2* last;
  int4* mv;
  const int32_t* it_dev;
  int32_t grp;              // the group deciding (swap rule)
  const int32_t* gsh;       // fused batches: per-graph group shift (see kAutoFewGroups), or nullptr
  // wide rows: partial bests of the partitions of each vertex of a launch
  // ([vertex][kWideMaxParts]) and the partitions finished per vertex
  double* wd_g;
  i128_t* wd_k;
  int32_t* wd_c;
  int32_t* wd_ok;           // bit 0: eligible (partition 0), bit 1: table overflow
  int32_t* wd_done;         // zero between launches
  int32_t* wd_next;         // task counter of the persistent wide kernel (zero between launches)
  int32_t* wd_exit;         // workgroups finished (zero between launches)
  // fused batches: graph of each vertex, per-graph constants, per-graph
  // summed gains and refinement moves; gid == nullptr for a single graph
  const int32_t* gid;
  const GraphParam* gp;
  double* dqg;              // [G] fast mode
  unsigned long long* dqg128;  // [G][lo, hi] deterministic mode
  unsigned long long* mvg;  // [G] refinement moves
  int32_t commit_grid;      // workgroups per role of a commit launch (at most)
  int32_t sync_moves;       // local-moving records decisions (committed per group) instead of
                            // committing at once: bit 0 rows <= kBinMax[4], bit 1 longer rows
  // randomized refinement (rnd = 1 during refinement sweeps only): draws of
  // (seed, pass, sweep, vertex, candidate) in graph-local ids (vbase: first
  // union id of each graph of a fused batch, else nullptr)
  int32_t rnd;
  uint32_t seed;
  int32_t pass, sweep;
  const int32_t* vbase;
};

// Hub path (vertices with more than kBinMax[kHubBin - 1] arcs, communities
// with more than kBinMax[kAggLastBin] member arcs).  Their arcs are cut into
// chunks of kHubChunk, each pre-aggregated in an LDS table by one workgroup.
// Vertex hubs of more than kPartMaxDeg arcs merge the chunks into the
// hub's global table (Alg. 2 scanCommunities), read back in slices of
// kHubSlice slots by several workgroups; global tables hold
// max(1024, next_pow2(2 min(arcs, |V'|))) slots, allocated in units of 1024.
constexpr int kHubChunk = 2048;
constexpr int kHubGatherLg = 12;      // LDS pre-aggregation table: 4096 slots
constexpr int kHubSlice = 8192;
constexpr int kTblUnit = 1024;
// Vertex hubs of up to kPartMaxDeg arcs, and giant communities of any size
// (Alg. 4 rows, agg_parts), are split instead into P = next_pow2(ceil(deg /
// kPartKeys)) partitions of the neighbour communities (wide_part mod P).  The chunk pass sums each chunk's
// candidates (community, weight) in an LDS table, sorts the distinct ones by
// partition and stores them at the chunk's own arc positions in lbuf / wbuf,
// with the chunk's partition
// offsets in poff; then one workgroup of kPartThreads threads per partition
// reads its runs of every chunk and accumulates them in an LDS table of
// kPartSlots slots (two workgroups per CU).  No global table and no global
// atomic per key are needed, and every arc is read once.
constexpr int32_t kPartKeys = 4096;
constexpr int kPartThreads = 512;
constexpr int kPartSlots = 6144;
constexpr int kPartMaxP = 256;
constexpr int32_t kPartMaxDeg = kPartMaxP * kPartKeys;
__host__ __device__ __forceinline__ bool hub_partitioned(int64_t deg) { return deg <= kPartMaxDeg; }
__host__ __device__ __forceinline__ int32_t hub_parts(int64_t deg) {
  int32_t p = 1;
  while ((int64_t)p * kPartKeys < deg && p < (1 << 24)) p <<= 1;
  return p;
}
// Giant communities of the aggregation are always partitioned, into at most
// kPartMaxP partitions: beyond kPartMaxDeg member arcs a partition's table
// can fill up, and it then emits its share of the row in parts.
__host__ __device__ __forceinline__ int32_t agg_parts(int64_t cap) {
  const int32_t p = hub_parts(cap);
  return p < kPartMaxP ? p : kPartMaxP;
}

// Slot of a global hash table: key and value share one 16-byte slot, so an
// insert (CAS on the key, add on the value) and a read touch one cache line.
struct alignas(16) TblSlot {
  int32_t key;   // kEmpty when free
  int32_t pad;
  double val;
};

struct HubArgs {
  const int32_t* items;       // hub vertex (or giant community) of each hub index p
  const int32_t* chunk_off;   // [H+1] first chunk task of p
  const int32_t* tbl_off;     // [H+1] table offset of p in units of kTblUnit
  const int32_t* slice_off;   // [H+1] first slice task of p
  const int2* chunk_tasks;    // (p, chunk)
  const int2* slice_tasks;    // (p, slice)
  int32_t* active;            // [H] item takes part in this launch
  double* kid;                // [H] weight of a hub's arcs to its own community
  int32_t* done;              // [H] slices finished (last one reduces)
  double* pb_g;               // per slice task: best gain
  i128_t* pb_k;               // per slice task: best exact key
  int32_t* pb_c;              // per slice task: best community
  TblSlot* tbl;               // table region
  int32_t* lbuf;              // partitioned hubs: candidates of each chunk sorted by partition (arc positions)
  double* wbuf;               // their weights (sums: FP64 keeps them exact in det mode)
  uint16_t* poff;             // [chunk task][kPartMaxP + 1] partition offsets inside the chunk
  int32_t* tbl_list;          // occupied slots of each item's table, at the item's table offset
  int32_t* lcnt;              // [H] length of each item's occupied-slot list
  int64_t tbase;              // region offset of the current batch (slots)
  const int32_t* apre;        // aggregation: arc prefix over the community-vertex list
};

// Raw graph description passed to launchers (weights float or double).
struct GraphDesc {
  int64_t n;
  const int32_t* off;
  const int32_t* deg;   // nullptr: plain CSR
  const int32_t* idx;
  const void* w;        // nullptr: unit weights
  bool w_double;
};

// Arguments of the aggregation row kernels (Alg. 4, lines building G'').
struct AggArgs {
  const int32_t* lab;    // renumbered refined label of each vertex (super-vertex id)
  const int32_t* coff;   // community-vertex CSR offsets [ncom + 1]
  const int32_t* cv;     // community-vertex CSR members
  const int32_t* yoff;   // super-vertex row offsets (holey) [ncom + 1]
  int32_t* ydeg;         // filled length of each super-vertex row
  int32_t* yidx;
  void* yw;              // float or double
  bool yw_double;
  unsigned long long* cnt;  // [kCntSlots][8]: [4] vertices, [5] arcs read, [6] arcs written
  int64_t ncom;
};

// ---- scan kernels (k_scan_move.hip, k_scan_refine.hip); one call per group
// `list` is the whole bin list; count/start are the group's bin segments.
// The same launch takes the eligibility snapshot of the group's hubs
// [h0, h1) (h.items indices; an empty range for none) and resets their
// per-decision state, before hub_decide runs on them.
void launch_decide_move(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                        const int32_t* count, const int32_t* start, bool det, int grid_cap, const HubArgs& h,
                        int32_t h0, int32_t h1, int64_t* launches);
void launch_decide_refine(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const int32_t* list,
                          const int32_t* count, const int32_t* start, bool det, int grid_cap, const HubArgs& h,
                          int32_t h0, int32_t h1, int64_t* launches);
// Applies the recorded synchronous decisions of one group in one launch.
// Local-moving: rows of up to kBinMax[4] arcs in tiles (community totals
// through the workgroup-combined table; the movers' rows marked end to end),
// longer rows one workgroup each, hub moves applied in tiles (their targets
// are forgotten by the next group's hub snapshot) and hub rows marked chunk by chunk.
// Refinement: both lists in tiles; vertex i moves only if its own community
// was not chosen as a target by this group (stamp).
struct CommitLaunch {
  const int32_t* l0;   // short rows (local-moving) or every non-hub row (refinement)
  const int32_t* l1;   // long rows (local-moving)
  const int32_t* l2;   // hubs
  int32_t n0, n1, n2;
  int32_t c0, c1;      // chunk tasks of the hubs (local-moving marks)
  int32_t b[5];        // block ranges of the roles: [b[r], b[r+1])
  const int2* chunk_tasks;    // HubArgs::chunk_tasks and items (set by launch_commit)
  const int32_t* hub_items;
};

void launch_commit(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const HubArgs& h, const CommitLaunch& cl,
                   int phase);

// ---- aggregation (k_aggregate.hip)
void launch_agg_rows(hipStream_t st, const GraphDesc& g, const AggArgs& a, const int32_t* list,
                     const int32_t* count, const int32_t* start, int grid_cap, int hub_grid,
                     int64_t* launches);

// ---- hub path (k_hub.hip)
// Per-hub sizes: nchunk, table units and nslice written to chunk_off /
// tbl_off / slice_off[p] (exclusive-scanned by the caller).
void hub_setup(hipStream_t st, const int32_t* off, const int32_t* deg, const int32_t* items, int32_t H,
               int64_t n, int32_t* chunk_off, int32_t* tbl_off, int32_t* slice_off);
void hub_tasks(hipStream_t st, int32_t H, const int32_t* chunk_off, const int32_t* slice_off, int2* chunk_tasks,
               int2* slice_tasks);
// One batch [h0, h1) of one group: gather, own-community weight, evaluation
// (+ commit in fast local-moving); the group's decision launch has taken
// the hubs' eligibility snapshot.
void hub_decide(hipStream_t st, const GraphDesc& g, const ScanArgs& a, const HubArgs& h, int32_t h0, int32_t h1,
                int32_t c0, int32_t c1, int32_t s0, int32_t s1, bool tables, int phase, bool det, int64_t* launches);
// K[i] += sums of the chunks of hub rows (K[i] of hubs zeroed by the caller).
void hub_weights(hipStream_t st, const GraphDesc& g, const HubArgs& h, int32_t c0, int32_t c1, double* K,
                 double* accW, int32_t* flags, int validate);
// Modularity partial sums of hub rows: tot[C[i]] += K part, acc_d[0] (or
// s1g[gid[i]]) += sigma part.
void hub_modularity(hipStream_t st, const GraphDesc& g, const HubArgs& h, int32_t c0, int32_t c1,
                    const int32_t* C, double* tot, double* acc_d, const int32_t* gid = nullptr,
                    double* s1g = nullptr);
// Aggregation of giant communities.
void gagg_setup(hipStream_t st, const int32_t* yoff, const int32_t* items, int32_t H, int32_t* chunk_off,
                int32_t* tbl_off, int32_t* slice_off);
void member_degrees(hipStream_t st, const GraphDesc& g, const int32_t* cv, int64_t n, int32_t* mdeg);
void gagg_rows(hipStream_t st, const GraphDesc& g, const AggArgs& a, const HubArgs& h, int32_t c0, int32_t c1,
               int32_t s0, int32_t s1, int64_t* launches);

// ---- fused batches (k_batch.hip)
enum BatchState : uint8_t { kBatchCont = 0, kBatchEnd = 1, kBatchDone = 2 };
// Device view of a batch of graphs.  vb: vertex bases of all graphs (G + 1);
// ub, uab: vertex and arc bases of the kept graphs in the union.
struct BatchDesc {
  const int32_t* const* off;
  const int32_t* const* idx;
  const float* const* w;     // entries may be nullptr (unit weights)
  const int64_t* n;
  const int64_t* m;
  const int64_t* vb;
  const int64_t* ub;
  const int64_t* uab;
};
// flags[g] |= 1 bad CSR, 2 weight not positive and finite, 4 weight not an
// integer in [1, 2^24]; W[g] += weights.  total = vb[G].
void batch_validate(hipStream_t st, const BatchDesc& d, int32_t G, int64_t total, int32_t* flags, double* W);
// Union CSR of the kept graphs (src[g] = desc index of kept graph g; total =
// ub[G] vertices): uoff[0..total) (uoff[total] set by the caller), uidx,
// uw (float), gid.
void batch_build(hipStream_t st, const BatchDesc& d, const int32_t* src, int32_t G, int64_t total, int32_t* uoff,
                 int32_t* uidx, float* uw, int32_t* gid);
void mask_flags(hipStream_t st, uint8_t* flag, const int32_t* gid, const uint8_t* active, int64_t n);
void graph_nonzero(hipStream_t st, const GraphDesc& g, const int32_t* gid, int32_t* nz);
void gather_at(hipStream_t st, const int32_t* data, const int32_t* pos, int32_t count, int32_t* out);
void gid_next(hipStream_t st, const int32_t* C, const int32_t* newid, const int32_t* gid, const uint8_t* keep,
              int64_t n, int32_t* out);
void lookup_batch(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, const int32_t* newid,
                  const int32_t* gid0, const uint8_t* state, const int32_t* vcur, const int32_t* goff0, bool first);
void batch_outputs(hipStream_t st, const int32_t* canon, int64_t N, const int32_t* gid0, const int32_t* goff0,
                   int32_t* const* out);
void mod_squares_batch(hipStream_t st, const double* tot, int64_t n, const int32_t* cb, int32_t G, double* s2d,
                       unsigned long long* s2u);

// ---- primitives (k_prims.hip)
int scan_tiles(int64_t n);  // number of tiles used by exclusive_scan
// In-place exclusive scan of int32 data[0..n); data[n] receives the total.
// tmp needs scan_tiles(n) + 1 int32 entries.
void exclusive_scan(hipStream_t st, int32_t* data, int64_t n, int32_t* tmp);
void fill_i32(hipStream_t st, int32_t* p, int32_t v, int64_t n);
void fill_u8(hipStream_t st, uint8_t* p, uint8_t v, int64_t n);
void fill_f64(hipStream_t st, double* p, double v, int64_t n);
void fill_slots(hipStream_t st, TblSlot* p, int64_t n);  // empty slots
void fill_u64(hipStream_t st, unsigned long long* p, unsigned long long v, int64_t n);
void iota_i32(hipStream_t st, int32_t* p, int64_t n);
void add_one_i32(hipStream_t st, int32_t* p);  // *p += 1 (a replayable counter step)
void copy_i32(hipStream_t st, int32_t* dst, const int32_t* src, int64_t n);
void pack_labels(hipStream_t st, const int32_t* C, const int32_t* CB, int2* CP, int64_t n);
// Refinement: the items of the bins (segment s = g * kNumBins + b:
// list[cursors[s] .. + counts[s])) still alone in their refined community,
// counted into bb->kept; those of the non-hub bins are then placed from
// bb->nstart into out.
void thin_count(hipStream_t st, const int32_t* list, BinBuf* bb, int S, const int32_t* C, const int32_t* size,
                const double* K);
void thin_scatter(hipStream_t st, const int32_t* list, BinBuf* bb, int S, const int32_t* C, const int32_t* size,
                  const double* K, int32_t* out);
void copy_f64(hipStream_t st, double* dst, const double* src, int64_t n);
void set_size_one(hipStream_t st, int32_t* size, int64_t n);

// K[i] = row sum (self-loop once); *accW += W.  flags[0] |= bad CSR
// (validate only), flags[1] |= weight not an integer in [1, 2^24],
// flags[2] |= weight not positive and finite.
// Rows longer than kBinMax[kHubBin - 1] are skipped (K = 0): the hub path
// adds them (hub_weights).
void vertex_weights(hipStream_t st, const GraphDesc& g, int64_t m, double* K, double* accW,
                    int32_t* flags, int validate);
// Sig[C[i]] += K[i]; size[C[i]] += 1 (Sig, size zeroed by the caller).
void community_totals(hipStream_t st, const int32_t* C, const double* K, double* Sig,
                      int32_t* size, int64_t n);
// Degree binning into S groups: bin_count fills bb->counts / bb->maxsize,
// bin_scatter places item i at bb->cursors[group(i) * kNumBins + bin(i)]++.
// wide = false (aggregation capacities) stops at bin kAggLastBin: larger
// capacities go to the hub bin.
// gid / vbase (fused batches, else nullptr): the group of item i is taken
// from its id inside its own graph, i - vbase[gid[i]]; gsh (nullable): per
// graph, the group is group_of(id, S >> gsh) << gsh.
void bin_count(hipStream_t st, const int32_t* off, const int32_t* deg, int64_t n, int S, bool wide,
               const int32_t* gid, const int32_t* vbase, const int32_t* gsh, const BinLimits& lim, BinBuf* bb);
void bin_scatter(hipStream_t st, const int32_t* off, const int32_t* deg, int64_t n, int S, bool wide,
                 const int32_t* gid, const int32_t* vbase, const int32_t* gsh, const BinLimits& lim, BinBuf* bb,
                 int32_t* list);
// used[c] = 1 for every label c in C[0..n) (used zeroed by the caller);
// with gid / keep only for vertices of graphs g with keep[g].
void mark_used(hipStream_t st, const int32_t* C, int64_t n, int32_t* used, const int32_t* gid = nullptr,
               const uint8_t* keep = nullptr);
// top[v] = newid[C[top[v]]]  (first = 1: top[v] = newid[C[v]]).
void lookup_top(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, const int32_t* newid,
                bool first);
// top[v] = C[top[v]] (or C[v] when first).
void lookup_raw(hipStream_t st, int32_t* top, int64_t N, const int32_t* C, bool first);
// lab[i] = newid[C[i]]; rank[i] = atomic slot in cnt[lab]; cap[lab] += degree(i).
// With gid / keep, vertices of graphs without keep get lab[i] = -1 and are
// skipped by agg_fill and next_labels.
void agg_count(hipStream_t st, const GraphDesc& g, const int32_t* C, const int32_t* newid,
               int32_t* lab, int32_t* rank, int32_t* cnt, int32_t* cap, const int32_t* gid = nullptr,
               const uint8_t* keep = nullptr);
void agg_fill(hipStream_t st, const int32_t* lab, const int32_t* rank, const int32_t* coff, int64_t n,
              int32_t* cv);
// start[lab[i]] = brank[CB[i]] (move-based labels of super-vertices).
// K'[newid[c]] = Sigma'[c] for every used label c of [0, n) (newid: the
// exclusive scan of the used flags, n + 1 entries); K' may not alias Sig.
void next_weights(hipStream_t st, const double* Sig, const int32_t* newid, int64_t n, double* K);
void next_labels(hipStream_t st, const int32_t* lab, const int32_t* CB, const int32_t* brank,
                 int64_t n, int32_t* start);
// Canonical relabelling by first occurrence over v = 0..N-1.
void first_occurrence(hipStream_t st, const int32_t* top, int64_t N, int32_t* first);
void first_flags(hipStream_t st, const int32_t* top, const int32_t* first, int64_t N, int32_t* flags);
void apply_canonical(hipStream_t st, int32_t* top, const int32_t* first, const int32_t* scan, int64_t N);
// Modularity (Eq. 1): S1 = sum of intra-community arc weights (acc_d[0]),
// tot[c] += K_i; then S2 = sum tot[c]^2 (exact int128 into acc_u[0..1] when
// integral, else double into acc_d[1]).  Hub rows are left to hub_modularity.
// gid / s1g (fused batches): S1 per graph into s1g[gid[i]].
void modularity_partial(hipStream_t st, const GraphDesc& g, const int32_t* C, double* tot,
                        double* acc_d, const int32_t* gid = nullptr, double* s1g = nullptr);
void check_offsets(hipStream_t st, const int32_t* off, int64_t n, int64_t m, int32_t* flags);
// acc[0..1] += multiset-hash differences of the arcs (zero for a symmetric
// CSR; offsets already checked).
void symmetry_check(hipStream_t st, const int32_t* off, const int32_t* idx, const float* w, int64_t n,
                    unsigned long long* acc);
// Alg. 5: components of the intra-community arcs (union-find); dis[c] = 1
// and ++cnt[0] for every community c with more than one (comp, root, rep,
// dis: int32[n] scratch / output).
void disconnected_communities(hipStream_t st, const int32_t* off, const int32_t* idx, const int32_t* C, int64_t n,
                              int32_t* comp, int32_t* root, int32_t* rep, int32_t* dis, unsigned long long* cnt);
void modularity_squares(hipStream_t st, const double* tot, int64_t n, bool integral, double* acc_d,
                        unsigned long long* acc_u);

}  // namespace gvl
