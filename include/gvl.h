/*
 * gvl.h -- C ABI of libgvl.so, a GPU (MI355X / gfx950) implementation of the
 * data-parallel hot path of GVE-Leiden (Sahu, arXiv:2312.13936): the
 * per-vertex neighbour-community scan shared by local-moving (Alg. 2) and
 * refinement (Alg. 3), and the aggregation into a super-vertex graph
 * (Alg. 4), driven by the pass loop of Alg. 1.
 *
 * Problem statement (Sec. 3.1-3.2): given an undirected weighted graph G as
 * a symmetric CSR, return a community membership C: V -> Gamma that
 * maximises the modularity of Eq. 1 (with resolution gamma multiplying the
 * null-model term), and the modularity of the returned C.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *     never frees them.  Other pointers are host pointers.
 *   - Work is enqueued on the HIP stream given to gvl_create.  gvl_leiden
 *     returns after the modularity has been copied back to the host.
 *   - Errors are returned as gvl_status codes; nothing is thrown across the
 *     ABI.  On error the membership buffer content is unspecified.
 *   - A context is not thread safe; use one context per host thread.
 *   - The library performs no device allocation on the gvl_leiden path: all
 *     device scratch lives in a caller-provided workspace whose size is
 *     given by gvl_workspace_bytes.
 */
#ifndef GVL_H
#define GVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GVL_OK = 0,
  GVL_E_INVALID_ARG = -1,       /* null pointer, negative size, bad option value */
  GVL_E_BAD_CSR = -2,           /* offsets not monotone / out of range, index out of range */
  GVL_E_NOT_SYMMETRIC = -3,     /* validate = 2: some arc (i, j, w) has no matching reverse arc (j, i, w) */
  GVL_E_NONINTEGER_WEIGHT = -4, /* deterministic mode: weight not an integer in [1, 2^24] or total > 2^40 */
  GVL_E_RESOLUTION = -5,        /* resolution < 0, or (deterministic mode) not p / 65536 with p <= 2^24 */
  GVL_E_WORKSPACE = -6,         /* workspace null or smaller than gvl_workspace_bytes */
  GVL_E_HIP = -8,               /* a HIP runtime call failed */
  GVL_E_BUSY = -9,              /* serving: request not in a state that allows the call */
  GVL_E_BATCH = -10,            /* batch: at least one graph failed (see its status) */
  GVL_E_TABLE_OVERFLOW = -11    /* deterministic mode: a key partition of a wide row or hub held more
                                   distinct neighbour communities than its LDS table (gvl_stats.
                                   table_overflows); the decision could not be computed exactly */
} gvl_status;

enum { GVL_MODE_FAST = 0, GVL_MODE_DET = 1 };

typedef struct gvl_ctx* gvl_ctx_t;

/* Options.  Defaults (gvl_default_options) follow Sec. 4.1 of the paper:
 * tolerance 0.01, tolerance drop 10, aggregation tolerance 0.8, at most 20
 * iterations per local-moving phase; passes are capped at 20. */
typedef struct {
  int32_t mode;                  /* GVL_MODE_FAST: FP64 gains, FP32 super-vertex weights (Sec. 5.1.2),
                                    local-moving schedule chosen by sync_moves;
                                    GVL_MODE_DET: synchronous moves, exact integer gains,
                                    lowest-id ties -- bit-reproducible.  Synchronous local-moving
                                    (both modes) also applies two rules against move cycles: of two
                                    adjacent vertices of a group that chose each other's community,
                                    a row of at most 128 arcs yields to the lower id or the longer
                                    row (swap rule), and a vertex that moved in each of the two
                                    previous iterations does not go straight back to the community
                                    it left in the last one (bounce rule) */
  double tolerance;              /* initial per-iteration tolerance tau (Alg. 2 convergence) */
  double tolerance_drop;         /* threshold scaling: tau /= tolerance_drop after each pass */
  double aggregation_tolerance;  /* Alg. 1 low-shrink test: stop when |Gamma| / |V'| exceeds this,
                                    with |Gamma| the distinct refined labels of the pass and |V'|
                                    the vertices of its graph */
  int32_t max_iterations;        /* cap on local-moving iterations per pass (1 .. 32767) */
  int32_t max_passes;            /* cap on passes */
  int32_t refine_sweeps;         /* cap on synchronous refinement sweeps per pass; sweeps stop
                                    early once one moves no vertex (1 = the single sweep of Alg. 3) */
  int32_t subsweeps;             /* S <= 64: local-moving and refinement visit the vertices in S
                                    pseudo-random groups in turn (sub-sweeps).  0 (fast mode only,
                                    its default): S = 8 if no vertex of the input has more than 128
                                    arcs, else 32 (deterministic mode default: 32) */
  int32_t validate;              /* 0: none; 1: CSR bounds and weight checks on the device (default);
                                    2: also symmetry (Sec. 3.1: the graph is undirected, each edge
                                    stored as two arcs with one weight): a multiset hash of the arcs
                                    (i, j, w) against that of their reverses (j, i, w), one pass over
                                    the arcs; GVL_E_NOT_SYMMETRIC if they differ.  The hash is
                                    probabilistic: an asymmetric input passes with probability
                                    2^-128 unless crafted against its public mixers. */
  int32_t profile;               /* 1: time every kernel class with HIP events (fills gvl_stats ms_*) */
  int32_t debug_trace;           /* 1: keep per-pass labels and super-vertex CSRs for gvl_debug_* */
  int32_t sync_moves;            /* fast mode local-moving: 0 commits every move at once (the
                                    paper's asynchronous updates, Sec. 4.1); bit 0 (rows of <= 128
                                    arcs) and bit 1 (longer rows) instead decide a group on one
                                    snapshot and commit it afterwards (the deterministic schedule with
                                    FP64 gains).  Default 3. */
  int32_t louvain;               /* 1: no refinement -- the super-vertices of each pass are the
                                    local-moving communities, i.e. the Louvain method that Leiden
                                    refines (Sec. 3.2, 3.3); the run stops when local-moving converges
                                    in its first iteration.  Default 0. */
  int32_t refine_random;         /* 1: randomized refinement (Sec. 4.1's alternative to the greedy
                                    one, Traag's original rule): among the in-bound targets with a
                                    positive gain a vertex picks c with probability proportional to
                                    the gain, from counter-based draws of (seed, pass, sweep, vertex,
                                    candidate); deterministic mode stays bit-reproducible for a seed.
                                    Default 0 (greedy). */
  uint32_t seed;                 /* seed of the randomized refinement */
  int32_t shrink_excludes_isolated; /* 1: the low-shrink ratio leaves the Z vertices of G' without
                                    arcs out of both counts, (|Gamma| - Z) / (|V'| - Z) > tolerance
                                    (they can never merge, so counting them ends runs on graphs with
                                    many isolated vertices early).  Not in the paper.  Default 0
                                    (Alg. 1 as printed). */
  int32_t no_graph_replay;       /* 1: launch every kernel from the host.  Default 0: local-moving
                                    iterations and refinement sweeps after the first of a pass are
                                    recorded once into a HIP graph and replayed (same kernels, same
                                    results; the host no longer issues each launch).  Replay is off
                                    while profile = 1. */
  int32_t refine_based;          /* 1: refine-based labels of super-vertices (Sec. 4.1): the next pass
                                    starts with every super-vertex alone in its community, as pass 0
                                    does.  Default 0: move-based, each super-vertex starts in the
                                    local-moving community of its members (Alg. 1). */
} gvl_options;

#define GVL_MAX_PASS_STATS 64

typedef struct {
  int32_t passes;
  int32_t termination;           /* 0 converged, 1 low shrink, 2 max passes, 3 empty graph */
  int64_t num_communities;
  int32_t iterations[GVL_MAX_PASS_STATS];     /* local-moving iterations per pass */
  int32_t refine_sweeps[GVL_MAX_PASS_STATS];  /* refinement sweeps per pass */
  int64_t nv[GVL_MAX_PASS_STATS];             /* |V'| per pass */
  int64_t ne[GVL_MAX_PASS_STATS];             /* arcs of G' per pass */
  int64_t ncom[GVL_MAX_PASS_STATS];           /* |Gamma| after refinement per pass */
  /* device time per phase (profile = 1), milliseconds */
  double ms_move, ms_refine, ms_aggregate, ms_other, ms_total;
  /* algorithmic work counted by the kernels themselves */
  int64_t scan_vertices;   /* vertices scanned by move + refine decision kernels */
  int64_t scan_arcs;       /* arcs read by those kernels */
  int64_t scan_candidates; /* distinct candidate communities evaluated */
  int64_t scan_moves;      /* vertices that changed community */
  int64_t agg_vertices;    /* vertices folded into super-vertices */
  int64_t agg_arcs;        /* arcs read by aggregation */
  int64_t agg_out_arcs;    /* arcs written to super-vertex graphs */
  double ms_scan_kernels;  /* summed duration of scan decision kernels (profile = 1) */
  double ms_agg_kernels;   /* summed duration of the aggregation row kernels (profile = 1) */
  int64_t scan_launches;
  int64_t agg_launches;
  int64_t scan_refine_arcs;      /* part of scan_arcs read by refinement */
  double ms_scan_move_kernels;   /* part of ms_scan_kernels spent in local-moving */
  int64_t graph_launches;        /* iterations and sweeps run as one replayed HIP graph */
  int64_t table_overflows;       /* decisions of wide rows and hubs whose key partition overflowed its
                                    LDS table: the vertex stays put (fast mode); deterministic mode
                                    returns GVL_E_TABLE_OVERFLOW instead */
} gvl_stats;

/* Create a context bound to `device` and to the HIP stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Allocates a few KB of pinned
 * host memory for scalar read-backs. */
gvl_status gvl_create(gvl_ctx_t* ctx, int device, void* hip_stream);
gvl_status gvl_destroy(gvl_ctx_t ctx);

/* Fill `opt` with the defaults for `mode` (32 sub-sweep groups, validation on). */
gvl_status gvl_default_options(gvl_options* opt, int32_t mode);

/* Device workspace needed by gvl_leiden for a graph with n vertices and m
 * arcs (both directions counted).  O(n + m); see the layout in the source. */
gvl_status gvl_workspace_bytes(int64_t n, int64_t m, const gvl_options* opt, size_t* bytes);

/* Leiden community detection (Alg. 1-4; Eq. 1-2).
 *   n, m          vertices and arcs; m = d_offsets[n]; 0 <= m < 2^31.
 *   d_offsets     int32[n+1], d_offsets[0] = 0, non-decreasing.
 *   d_indices     int32[m], neighbours; must describe a symmetric graph
 *                 (each undirected edge stored in both rows, a self-loop
 *                 once).  Rows need not be sorted.
 *   d_weights     float[m] positive weights, or NULL for unit weights.
 *   resolution    gamma >= 0 (1 = modularity of Eq. 1).
 *   d_workspace   device buffer of at least gvl_workspace_bytes bytes.
 *   d_membership  int32[n] output: community of each vertex, numbered by
 *                 first occurrence over v = 0..n-1.
 *   modularity    host double output: Eq. 1 of d_membership.
 *   stats         host output, may be NULL.
 * Deterministic mode additionally requires integer weights in [1, 2^24],
 * total weight <= 2^40 and resolution = p / 65536 with integer p <= 2^24;
 * its results are identical on every run. */
gvl_status gvl_leiden(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_offsets,
                      const int32_t* d_indices, const float* d_weights, double resolution,
                      const gvl_options* opt, void* d_workspace, size_t workspace_bytes,
                      int32_t* d_membership, double* modularity, gvl_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gvl_leiden
 * with its workspace in a device array that the library holds, one copy of
 * GVL_STATIC_WORKSPACE_BYTES (256 MiB) per GPU it runs on, until the
 * process ends.  The caller still provides the input graph and the output
 * membership; arguments and results are those of gvl_leiden.  The call
 * allocates no device memory.
 *   Errors: those of gvl_leiden; GVL_E_WORKSPACE if gvl_workspace_bytes(n,
 *   m, opt) exceeds GVL_STATIC_WORKSPACE_BYTES (e.g. fast mode up to about
 *   330k vertices with 12 arcs each); GVL_E_INVALID_ARG if opt->profile is
 *   set (timing would create HIP events).
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (from several streams or host threads) race and must not be made. */
#define GVL_STATIC_WORKSPACE_BYTES (256u * 1024u * 1024u)
gvl_status gvl_leiden_static(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_offsets,
                             const int32_t* d_indices, const float* d_weights, double resolution,
                             const gvl_options* opt, int32_t* d_membership, double* modularity, gvl_stats* stats);

/* Launch-shape tuning: the degree binning and grid sizes that take the
 * place of the paper's dynamic loop schedule (Sec. 4.1), picked per class of
 * graph by paper_2312_13936_amd/tune.py and kept in a process-wide table.
 * They change which kernel handles a row and how many workgroups a launch
 * uses, never a result.  The table starts from compiled defaults and is
 * loaded once per process, when the first context is created, from
 * $GVL_TUNE_FILE, or (unset) tune.txt next to libgvl.so; "none" skips it.
 * Class of a graph: fused batches GVL_CLASS_BATCH; else n <= 131072
 * GVL_CLASS_SMALL; else m < 6 n GVL_CLASS_LOWDEG; else GVL_CLASS_SKEWED. */
enum { GVL_CLASS_SMALL = 0, GVL_CLASS_LOWDEG = 1, GVL_CLASS_SKEWED = 2, GVL_CLASS_BATCH = 3, GVL_NUM_CLASSES = 4 };
typedef struct {
  int32_t bin_max[6];   /* largest row (arcs, or member arcs of a community) of the lane-group bins 0-4
                           and of the one-workgroup bin 5: non-decreasing, each at most the compiled
                           limit {4, 8, 16, 32, 128, 1024}, bin_max[5] >= 256 (a bin whose limit
                           equals the previous one is empty; its rows go to the next bin) */
  int32_t decide_grid;  /* workgroups per decision launch (at most), 1..65536 */
  int32_t commit_grid;  /* workgroups per commit role (at most), 1..65536 */
  int32_t agg_grid;     /* workgroups per aggregation launch (at most), 1..65536 */
} gvl_tuning;
/* Class of a graph with n vertices and m arcs (fused: 1 for a fused batch). */
gvl_status gvl_graph_class(int64_t n, int64_t m, int32_t fused, int32_t* cls);
gvl_status gvl_get_tuning(int32_t cls, gvl_tuning* t);
/* GVL_E_INVALID_ARG for an unknown class or values outside the limits above;
 * calls running meanwhile keep the values they started with. */
gvl_status gvl_set_tuning(int32_t cls, const gvl_tuning* t);
/* Reads a tune file (lines "<class> b0 b1 b2 b3 b4 b5 decide_grid
 * commit_grid agg_grid", class one of small lowdeg skewed batch, '#'
 * comments); invalid lines are reported on stderr and skipped.
 * GVL_E_INVALID_ARG if the file cannot be opened. */
gvl_status gvl_load_tuning(const char* path);

/* Eq. 1 for a given membership (labels in [0, n)) on the device. */
gvl_status gvl_modularity(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_offsets,
                          const int32_t* d_indices, const float* d_weights,
                          const int32_t* d_membership, double resolution, void* d_workspace,
                          size_t workspace_bytes, double* modularity);

/* Alg. 5 on the device: the number of communities of d_membership (labels
 * in [0, n)) whose members are not all connected by arcs inside the
 * community (the quality check of Sec. 5: Leiden guarantees 0, Louvain does
 * not).  d_flags: optional device int32[n] output, 1 at the label of every
 * disconnected community, else 0.  Workspace: gvl_workspace_bytes(n, m) of
 * the fast mode.  *count receives the number on the host; the call blocks
 * until it is known.  Errors: GVL_E_INVALID_ARG (null count or membership),
 * GVL_E_BAD_CSR (offsets not monotone or not ending at m), GVL_E_WORKSPACE. */
gvl_status gvl_disconnected_communities(gvl_ctx_t ctx, int64_t n, int64_t m, const int32_t* d_offsets,
                                        const int32_t* d_indices, const int32_t* d_membership,
                                        void* d_workspace, size_t workspace_bytes, int32_t* d_flags,
                                        int64_t* count);

/* Measurement aid (not part of Leiden): enqueues on ctx's stream a kernel
 * that sums d_table[d_idx[e]] for e in [0, n_idx) into *d_sink (device,
 * caller-zeroed unsigned 64-bit), four loads in flight per lane, so that
 * the caller can time the device's random-gather rate over an index array
 * (the neighbour-community scan reads one label per arc at the arc's
 * neighbour id, Alg. 2 and Alg. 3).  An index outside [0, n_table) reads
 * entry 0.  Returns without waiting.  Errors: GVL_E_INVALID_ARG (null
 * pointer, n_idx < 0, n_table < 1), GVL_E_HIP. */
gvl_status gvl_gather_probe(gvl_ctx_t ctx, const int32_t* d_idx, int64_t n_idx, const int32_t* d_table,
                            int64_t n_table, unsigned long long* d_sink);

/* Debug export of the last gvl_leiden run made with debug_trace = 1.
 * For pass p: n_out = |V'|, m_out = arcs of the super-vertex graph built in
 * pass p (-1 if the pass did not aggregate).  Host buffers may be NULL.
 * bound/refined: int32[n_out] local-moving and refinement labels.
 * y_off: int32[ncom+1], y_idx: int32[m_out], y_w: double[m_out]: the
 * super-vertex CSR with rows compacted and sorted by neighbour id. */
gvl_status gvl_debug_pass_info(gvl_ctx_t ctx, int32_t pass, int64_t* n_out, int64_t* ncom_out,
                               int64_t* m_out);
gvl_status gvl_debug_export_pass(gvl_ctx_t ctx, int32_t pass, int32_t* bound, int32_t* refined,
                                 int32_t* y_off, int32_t* y_idx, double* y_w);
/* Movers per local-moving iteration / refinement sweep of pass p (debug_trace = 1). */
gvl_status gvl_debug_pass_movers(gvl_ctx_t ctx, int32_t pass, int64_t* movers, int32_t max_it,
                                 int64_t* refine_movers, int32_t max_sw);

/* ------------------------------------------------------------------------
 * Batched and served Leiden (many independent graphs on one GPU).
 *
 * Both run gvl_leiden for every graph on a pool of `lanes` concurrent HIP
 * streams (one host worker thread, one context and one workspace slice per
 * lane), so each graph gets exactly the result it gets alone: bit-identical
 * in deterministic mode, the same algorithm in fast mode.
 * ------------------------------------------------------------------------ */
typedef struct {
  int64_t n, m;                 /* as for gvl_leiden */
  const int32_t* d_offsets;
  const int32_t* d_indices;
  const float* d_weights;       /* NULL: unit weights */
  double resolution;
  int32_t* d_membership;        /* output int32[n] (device, caller-owned) */
} gvl_graph_desc;

/* Device workspace for gvl_leiden_batch: lanes x the largest per-graph
 * workspace. */
gvl_status gvl_batch_workspace_bytes(int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                                     int32_t lanes, size_t* bytes);
/* Leiden on every graph; waits for all.  Work already queued on ctx's stream
 * (e.g. uploads of the inputs) completes before any lane starts.
 * modularities: host double[num_graphs]; statuses: host, nullable.  Returns
 * GVL_E_BATCH if any graph failed, the others are still computed. */
gvl_status gvl_leiden_batch(gvl_ctx_t ctx, int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                            int32_t lanes, void* d_workspace, size_t workspace_bytes, double* modularities,
                            gvl_status* statuses);

/* Fused batch: the graphs run together as one disjoint union, every kernel
 * launch covering all graphs still running, with per-graph gains, stop
 * tests and pass counts (Alg. 1, Alg. 2 per graph); each result is the one
 * gvl_leiden gives for that graph alone (bit-identical in deterministic
 * mode).  Graphs are grouped into runs of < 1.5e9 vertices and arcs; the
 * workspace holds the largest run.  statuses: host gvl_status[num_graphs]
 * (per-graph input errors as gvl_leiden reports them); modularities: host
 * double[num_graphs].  Returns GVL_E_BATCH if any graph failed, the others
 * are still computed; in deterministic mode a partition table overflow in
 * any graph fails the whole call with GVL_E_TABLE_OVERFLOW.  Work already
 * queued on ctx's stream comes first; the call returns when every
 * membership is written. */
gvl_status gvl_fused_workspace_bytes(int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                                     size_t* bytes);
gvl_status gvl_leiden_fused(gvl_ctx_t ctx, int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                            void* d_workspace, size_t workspace_bytes, double* modularities, gvl_status* statuses);

/* Serving with continuous admission.  The caller gives a device arena; a
 * running request holds gvl_workspace_bytes(n, m) of it (rounded up to 256),
 * returned when it completes.  Requests wait in arrival order; a free lane
 * takes the oldest one whose workspace fits in the free arena; one that later
 * requests overtook 64 times is admitted before any other.  The input graph
 * must be fully written (its producing stream synchronised) before
 * submission, and it and the output membership must stay valid until the
 * request is done; the membership is complete once a wait or poll reports
 * GVL_REQ_DONE.  All calls are thread safe.  Errors: GVL_E_INVALID_ARG for a
 * null handle, unknown ticket or bad argument; GVL_E_HIP if a lane cannot be
 * created. */
typedef struct gvl_server* gvl_server_t;
enum { GVL_REQ_PENDING = 0, GVL_REQ_RUNNING = 1, GVL_REQ_DONE = 2, GVL_REQ_CANCELLED = 3 };
typedef struct {
  int32_t state;                /* GVL_REQ_* */
  gvl_status result;            /* status of the run (valid when done) */
  double modularity;
  double latency_ms;            /* submission -> completion (host steady clock) */
  double queue_ms;              /* submission -> start */
} gvl_request_info;
typedef struct {
  int64_t completed, pending, running, max_running;
  size_t arena_bytes, arena_used, arena_peak;
} gvl_server_info;

gvl_status gvl_server_create(gvl_server_t* srv, int device, int32_t lanes, const gvl_options* opt, void* d_arena,
                             size_t arena_bytes);
/* GVL_E_WORKSPACE if the request can never fit into the arena. */
gvl_status gvl_server_submit(gvl_server_t srv, const gvl_graph_desc* graph, uint64_t* ticket);
gvl_status gvl_server_poll(gvl_server_t srv, uint64_t ticket, gvl_request_info* info);
/* Blocks until the request is done or cancelled, or timeout_ms passes
 * (then GVL_E_BUSY with the current state in info); timeout_ms < 0 waits
 * without limit. */
gvl_status gvl_server_wait(gvl_server_t srv, uint64_t ticket, int64_t timeout_ms, gvl_request_info* info);
/* Only a request that is still waiting can be cancelled (else GVL_E_BUSY). */
gvl_status gvl_server_cancel(gvl_server_t srv, uint64_t ticket);
/* Forgets a finished or cancelled request (GVL_E_BUSY while it waits or runs). */
gvl_status gvl_server_release(gvl_server_t srv, uint64_t ticket);
/* Micro-batching: a lane that admits a request of at most max_vertices
 * vertices also takes up to max_batch - 1 further waiting requests of at
 * most that size whose fused workspace fits, and runs them together through
 * gvl_leiden_fused (each result as alone).  max_batch 1 turns it off.
 * Default: 32 requests of at most 262144 vertices. */
gvl_status gvl_server_set_batching(gvl_server_t srv, int32_t max_batch, int64_t max_vertices);
gvl_status gvl_server_stats(gvl_server_t srv, gvl_server_info* info);
/* Finishes running requests, cancels waiting ones, joins the workers. */
gvl_status gvl_server_destroy(gvl_server_t srv);

const char* gvl_status_string(gvl_status s);

#ifdef __cplusplus
}
#endif
#endif /* GVL_H */
