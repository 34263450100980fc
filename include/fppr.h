/*
 * fppr — fully edge-weighted personalized PageRank by Monte Carlo walks on
 * one MI355X (gfx950).
 *
 * Problem (Lin, WWW'19, Definition 1 and Sec. 2.1): for a directed graph
 * G = (V, E, w) with integer weights w(e) >= 1, a termination probability
 * alpha in (0,1) and R walks per source, estimate pi(s,t), the probability
 * that a walk from s ends at t, as count(s,t) / R. A walk moves to an
 * out-neighbour t of its tail u with probability w(u,t) / sum_v w(u,v), then
 * stops there with probability alpha (so it takes at least one step); at a
 * node without out-neighbours it restarts from its head (Sec. 2.1).
 * Algorithm 2 generates the walks; its last phase counts them per
 * (head, tail). The library returns the integer counts; pi_hat = count / R.
 *
 * Exactness: every random number is Philox4x32-10 (Salmon et al., SC'11)
 * keyed by the 64-bit seed (key word 0 = low half) on the counter
 * (walk index i, move index m, source id s, 0); the coin is "stop iff
 * x2 < T(alpha)" with T(alpha) = floor(alpha * 2^32 + 1/2) clamped to
 * [1, 2^32-1]; the weighted pick takes X = floor((x1 * 2^32 + x0) * W / 2^64)
 * and the first out-edge whose inclusive weight prefix exceeds X. Results are
 * therefore a pure function of (graph, alpha, R, seed, source) and do not
 * depend on launch shapes, the hub threshold or which other sources run.
 *
 * Conventions for every call:
 *  - every function returns an fppr_status (0 = FPPR_OK) unless stated;
 *  - pointers documented as "device" are HIP device pointers on the device
 *    that was current when the graph was created; "host" pointers are
 *    ordinary host memory;
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *    device work is enqueued on it and is asynchronous unless stated;
 *  - argument errors are reported synchronously and leave nothing enqueued;
 *    a failed HIP call returns FPPR_DEVICE_ERROR; fppr_last_error() gives a
 *    thread-local description of the last failure;
 *  - no call throws; all handles are opaque; destroy calls accept NULL.
 */
#ifndef FPPR_H
#define FPPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPPR_API __attribute__((visibility("default")))

typedef enum {
  FPPR_OK = 0,
  FPPR_INVALID_ARGUMENT = 1,
  FPPR_OUT_OF_MEMORY = 2,
  FPPR_DEVICE_ERROR = 3,
  FPPR_NOT_READY = 4,  /* poll: request still running */
  FPPR_CAPACITY = 5,   /* submit: admitted later (queued), not an error */
  FPPR_CANCELLED = 6,
  FPPR_INTERNAL = 7
} fppr_status;

enum { FPPR_MEM_HOST = 0, FPPR_MEM_DEVICE = 1 };

/* Walks stop after this many moves even without a terminating coin (never
 * reached in practice for alpha >= 0.01); both the library and any checker
 * apply the same cap. */
#define FPPR_MOVE_CAP 65536u

/* Padding entry of top-k lists shorter than k: (FPPR_NO_NODE, 0). */
#define FPPR_NO_NODE 0xFFFFFFFFu

typedef struct fppr_graph fppr_graph;

/* Graph in CSR form (Sec. 2.1: G = (V, E, w), w(e) > 0; the paper keeps each
 * node's out-neighbour set, Sec. 2.3). Multi-edges and self-loops are
 * allowed; edge order within a row decides which edge a given draw hits, so
 * callers that compare runs keep the same order (canonical: sorted by
 * (dst, w)). */
typedef struct {
  uint32_t n;                  /* nodes, 1 <= n <= 2^32 - 2 */
  uint64_t m;                  /* edges, m < 2^36 */
  const uint64_t* row_offsets; /* [n+1]: 0 = off[0] <= off[1] <= ... <= off[n] = m */
  const uint32_t* col;         /* [m]: destination of each edge, < n */
  const uint32_t* w;           /* [m]: weight of each edge, >= 1 */
  int mem;                     /* FPPR_MEM_HOST: copied at create;
                                  FPPR_MEM_DEVICE: borrowed, the caller keeps the
                                  arrays alive and unchanged in shape until
                                  fppr_graph_destroy */
} fppr_csr;

/* Graph layouts (fppr_graph_opts.layout). All give identical results (the
 * same edge for every draw). The narrow layout reads fewer lines per
 * weighted pick than the wide one. The guide layout reads one 64-byte entry
 * for almost every pick, whatever the degree: each row gets a table indexed
 * by the top bits of the pick's 64-bit draw D, whose entries hold the
 * thresholds ceil(P[j] 2^64 / W) that separate the edges meeting it (the
 * first edge with P[j] > floor(D W / 2^64) is the first with D < that
 * threshold), with child tables over the next bits of D where more than
 * three edges meet one entry; every entry carries the record of the nodes it
 * leads to, so a walk never reads a node's own line. It takes about 64 bytes
 * x (0.7 to 2) per edge plus 8 bytes per edge of thresholds, and 16-byte
 * pool entries; it needs n <= 2^30. The alias and big-move calls need the
 * narrow layout. */
#define FPPR_LAYOUT_AUTO 0u   /* narrow when it fits (max out-degree x max weight
                                 < 2^32), else wide */
#define FPPR_LAYOUT_WIDE 1u   /* always wide */
#define FPPR_LAYOUT_NARROW 2u /* narrow; INVALID_ARGUMENT when it does not fit */
#define FPPR_LAYOUT_GUIDE 3u  /* guide tables; INVALID_ARGUMENT when n > 2^30 */

typedef struct {
  /* Rows with more than hub_threshold out-edges (the large nodes of Sec. 4.1)
   * carry a prefix tree, the integer counterpart of the alias tree
   * (Algorithm 3, Lemma 1): the row is cut into blocks of E edges whose
   * running totals form the next level, F keys to a 128-byte node,
   * recursively; the top level sits in the node's own 128-byte line, so a
   * pick reads the node line, one node per level below the top, and one
   * block of E edges. Wide layout (64-bit prefixes): E = 8, F = 16, up to 14
   * top keys. Narrow layout (32-bit prefixes, for graphs whose row totals
   * fit in 32 bits): E = 16, F = 32, up to 28 top keys. A pick returns
   * exactly the edge a flat search returns, so neither the threshold nor the
   * layout changes results. 0 selects 8 (the fastest on the graphs
   * measured); values below 8 act as 8; UINT32_MAX disables trees (rows of
   * more than E edges are then binary-searched over their blocks). */
  uint32_t hub_threshold;
  /* FPPR_LAYOUT_AUTO, _WIDE, _NARROW or _GUIDE. A narrow graph keeps its
   * layout: a rebuild whose weights push a row total past 2^32 - 1 fails its
   * check (fppr_graph_check) and the graph must be created again. A guide
   * graph is created with room for its child tables plus slack; a rebuild
   * whose new weights need more fails its check the same way. Prefix trees
   * (hub_threshold) do not apply to the guide layout. */
  uint32_t layout;
} fppr_graph_opts;

/* Creates the device graph: validates the CSR (device-side; INVALID_ARGUMENT
 * on n == 0, n > 2^32-2, m >= 2^36, a non-monotone offset array, off[0] != 0,
 * off[n] != m, col >= n, w == 0, a row of 2^27 or more edges), computes the
 * per-row inclusive uint64 weight prefixes, the 128-byte node lines and the
 * prefix trees. Synchronous: returns after the graph is ready. The library
 * allocates its own device arrays (freed by fppr_graph_destroy).
 * opts may be NULL (defaults). */
FPPR_API fppr_status fppr_graph_create(const fppr_csr* csr, const fppr_graph_opts* opts,
                                       void* stream, fppr_graph** out);
FPPR_API fppr_status fppr_graph_destroy(fppr_graph* g);

/* Recomputes every derived array (prefixes, records, prefix trees; the pool if
 * one was built) from the CSR the graph was created from, asynchronously on
 * `stream`, without allocating. For a borrowed CSR whose col/w contents were
 * rewritten in place; row_offsets must be unchanged. Validation failures are
 * recorded on the device and reported by fppr_graph_check. */
FPPR_API fppr_status fppr_graph_rebuild(fppr_graph* g, void* stream);

/* Lays the graph out again for another hub threshold (same meaning as
 * fppr_graph_opts.hub_threshold) and rebuilds the pool if one was built.
 * Results never change. Synchronous; may reallocate the row regions. */
FPPR_API fppr_status fppr_graph_set_hub_threshold(fppr_graph* g, uint32_t hub_threshold, void* stream);

/* Synchronises `stream` and reports a validation failure recorded by
 * fppr_graph_rebuild (INVALID_ARGUMENT) or FPPR_OK. */
FPPR_API fppr_status fppr_graph_check(fppr_graph* g, void* stream);

/* Basic facts of a created graph (host outputs; any pointer may be NULL):
 * n_hubs = rows carrying a prefix tree, n_small = small nodes of the pool
 * (0 without a pool), device_bytes = bytes the library allocated. */
FPPR_API fppr_status fppr_graph_info(const fppr_graph* g, uint32_t* n, uint64_t* m,
                                     uint32_t* n_hubs, uint64_t* n_small, uint64_t* device_bytes);
/* The layout chosen at creation (host output): FPPR_LAYOUT_WIDE,
 * FPPR_LAYOUT_NARROW or FPPR_LAYOUT_GUIDE. */
FPPR_API fppr_status fppr_graph_layout(const fppr_graph* g, uint32_t* layout);

typedef struct {
  uint32_t S;     /* small nodes: 1 <= out-degree <= S (S >= 1) */
  uint32_t L;     /* at most L plain steps per short walk, 1 <= L <= 255 */
  uint32_t K;     /* short walks per small node: power of two in [1, 2^16] */
  double alpha;   /* termination probability; runs that stitch must use the same */
  uint64_t seed;  /* Philox key of the short walks, counter (slot j, step t, node v, 1) */
} fppr_pool_opts;

/* Short-walk pool (Sec. 4.2, "big moves" for small nodes): for every small
 * node v, K walks of at most L plain steps from v, each stopping on its coin
 * (marked terminated), after L steps, or on reaching a node without
 * out-neighbours (both marked active). A stitched run takes, at a small
 * node, slot j = floor(x0 * K / 2^32) of that node's pool: it jumps to the
 * entry's end node, adds its steps, and stops iff the entry is terminated.
 * Owned by the graph; building again replaces it. Asynchronous on `stream`
 * (allocates on first build or when the size grows). */
FPPR_API fppr_status fppr_graph_build_pool(fppr_graph* g, const fppr_pool_opts* opts, void* stream);

/* Copies the pool to host memory in canonical order: small nodes by
 * increasing id, then slot; entry = end | steps << 32 | mark << 48 (mark 1 =
 * terminated). `entries` holds n_small * K values. Synchronous. */
FPPR_API fppr_status fppr_graph_export_pool(const fppr_graph* g, uint64_t* entries, uint64_t count,
                                            void* stream);

/* Alias tables of every row (Sec. 2.2, Algorithm 1; Example 2), in exact
 * integers. For a row of n edges with weights w and total W: P[e] = the
 * switch threshold n w(e) after Algorithm 1's updates, in units of 1/W (so
 * in [0, W]), and alias[e] = the index within the row (0-based) of the edge
 * that slot e passes to. A pick with the 64-bit uniform D takes X =
 * floor(D n W / 2^64), slot i = X div W and keeps i iff X mod W < P[i], else
 * takes alias[i]; each edge is then chosen with probability w / W up to the
 * draw's 2^-64 granularity. Algorithm 1's free choice of x and y is the first
 * of each set in insertion order (FIFO queues seeded in edge order; an edge
 * that drops below W joins the back of the small set).
 * P: device u64[m], alias: device u32[m], both indexed like the CSR's edges;
 * scratch: device u32[2 m] of any contents, used as the two queues. All
 * three are the caller's. Reads the graph's CSR arrays as they are now.
 * Asynchronous on `stream`; INVALID_ARGUMENT for NULL pointers (m > 0). */
FPPR_API fppr_status fppr_graph_alias_tables(const fppr_graph* g, uint64_t* P, uint32_t* alias,
                                             uint32_t* scratch, void* stream);

/* Packs the alias tables into one 16-byte slot per edge for the walks:
 * slots[2e] = P[e], slots[2e + 1] = col[e] | col[a + alias[e]] << 32 (a =
 * the row's first edge), so a pick reads one slot. P, alias: from
 * fppr_graph_alias_tables; slots: device u64[2 m], 16-byte aligned, the
 * caller's. Asynchronous on `stream`; INVALID_ARGUMENT for NULL pointers
 * (m > 0) or a misaligned slots. */
FPPR_API fppr_status fppr_graph_alias_slots(const fppr_graph* g, const uint64_t* P, const uint32_t* alias,
                                            uint64_t* slots, void* stream);

/* One 16-byte record per node for the alias walks: nodes[2v] = the row's
 * first edge, nodes[2v + 1] = W(v) | deg(v) << 32 (row total and out-degree),
 * so a move reads its node in one line. nodes: device u64[2 n], 16-byte
 * aligned, the caller's. Narrow-layout graphs only (W < 2^32).
 * Asynchronous on `stream`; INVALID_ARGUMENT for a wide graph, NULL or a
 * misaligned nodes. */
FPPR_API fppr_status fppr_graph_alias_nodes(const fppr_graph* g, uint64_t* nodes, void* stream);

/* Walks that pick each edge with the alias tables (Sec. 2.2 and Sec. 2.1's
 * walk, Algorithm 2's coin): walk w (w = row * R + i) starts at
 * sources[row] (or node row when sources is NULL, then n_sources must be n);
 * its move m draws Philox4x32-10 on (i, m, s, 0); at a node with d out-edges
 * and total W the move takes X = floor((x1:x0) d W / 2^64), slot = X div W,
 * keeps the slot iff X mod W < P[slot], else alias[slot], then stops iff
 * x2 < T(alpha); a node without out-edges sends the walk back to s; 65,536
 * moves at most. No stitching. endpoints: device u32[n_sources * R] (the end
 * node; 0xFFFFFFFF for a source id >= n); steps: device u32[n_sources * R]
 * or NULL. nodes, slots: what fppr_graph_alias_nodes and
 * fppr_graph_alias_slots built for this graph (other contents give wrong
 * walks, never an out-of-bounds access).
 * Needs a narrow-layout graph (d W < 2^59 keeps X within 64 bits);
 * INVALID_ARGUMENT otherwise, for alpha outside (0, 1), R == 0, NULL
 * pointers or n_sources * R > 2^40. Asynchronous on `stream`. */
FPPR_API fppr_status fppr_run_alias(const fppr_graph* g, const uint64_t* nodes, const uint64_t* slots,
                                    double alpha, uint32_t R, uint64_t seed, const uint32_t* sources,
                                    uint64_t n_sources, uint32_t* endpoints, uint32_t* steps, void* stream);

/* Exact big moves of every small node (Sec. 4.2, Algorithm 4; Lemma 2):
 * for each node v with 1 <= out-degree <= S, the distribution of a walk's
 * first k steps from v (pick by weight, then stop with alpha), as entries
 * end | steps << 32 | mark << 48 (mark 1 = stopped there, 0 = still going)
 * with integer weights in units of 2^-62. A level is expanded while the
 * distinct end nodes reached, plus the frontier and the frozen entries, are
 * fewer than d and the last level reached a new node (Algorithm 4's stop
 * rule), and only if the table cannot pass `cap` entries. Frontier mass at
 * a node without out-edges is frozen as an active outcome of its length.
 * Masses are 62-bit fixed point with a floor after every product: first
 * step floor(w 2^62 / W(v)); an edge (u, t) of frontier mass a carries
 * floor(floor(a C / 2^32) w / W(u)), C = 2^32 - T(alpha); terminated weight
 * floor(a T / 2^32), active floor(a C / 2^32). Zero weights are dropped, and
 * entries are sorted by value.
 * Outputs (device, indexed by node id): counts u32[n] (0 for nodes that are
 * not small), entries u64[n * cap] and weights u64[n * cap] (the inclusive
 * prefix of the entries' weights, so the last is the total), node v's
 * table at [v * cap, v * cap + counts[v]); the rest is left as it was.
 * scratch: device u64[scratch_words] of any contents, at least 8 * cap
 * words; each 8 * cap words serve one node at a time. Needs a narrow-layout
 * graph; INVALID_ARGUMENT otherwise, for alpha outside (0, 1), S or d = 0,
 * cap outside [2 S, 4096], NULL pointers or too little scratch.
 * Asynchronous on `stream`. */
FPPR_API fppr_status fppr_graph_big_moves(const fppr_graph* g, uint32_t S, uint32_t d, uint32_t cap,
                                          double alpha, uint64_t* entries, uint64_t* weights,
                                          uint32_t* counts, uint64_t* scratch, uint64_t scratch_words,
                                          void* stream);

/* Walks of the paper's design (Algorithm 2 with Sec. 2.2's alias picks and
 * Sec. 4.2's big moves): walk w = row * R + i from sources[row] (node row
 * when sources is NULL, then n_sources must be n), move m drawing
 * Philox4x32-10 on (i, m, s, 0). At a node with 1 <= out-degree <= S the
 * move takes the first entry of the node's big-move table whose inclusive
 * weight prefix exceeds floor((x1:x0) * total / 2^64): its end becomes the tail,
 * its steps are added, and a terminated entry ends the walk. At any other
 * node with out-edges it is fppr_run_alias's pick followed by the coin
 * x2 < T(alpha); at a node without out-edges the walk returns to its
 * source and tosses the coin. 65,536 moves at most.
 * slots: from fppr_graph_alias_slots; bm_entries, bm_weights,
 * bm_counts, cap: from fppr_graph_big_moves with the same S (other contents
 * give wrong walks, never an out-of-bounds access). endpoints: device
 * u32[n_sources * R] (0xFFFFFFFF for a source id >= n); steps: device
 * u32[n_sources * R] or NULL. Narrow-layout graphs only; INVALID_ARGUMENT
 * as for fppr_run_alias, or for cap outside [1, 4096]. Asynchronous. */
FPPR_API fppr_status fppr_run_big_moves(const fppr_graph* g, const uint64_t* slots,
                                        const uint64_t* bm_entries, const uint64_t* bm_weights,
                                        const uint32_t* bm_counts, uint32_t cap, uint32_t S, double alpha,
                                        uint32_t R, uint64_t seed, const uint32_t* sources,
                                        uint64_t n_sources, uint32_t* endpoints, uint32_t* steps,
                                        void* stream);

/* T(alpha) = floor(alpha * 2^32 + 1/2) clamped to [1, 2^32-1]: a walk stops
 * after a move iff that move's x2 < T (Algorithm 2's coin "q <= alpha").
 * Returns 0 when alpha is not in (0, 1). */
FPPR_API uint32_t fppr_alpha_threshold(double alpha);

/* Walks per source for the guarantee of Definition 1 (relative error eps for
 * pi >= delta with probability 1 - pf): ceil((2 + 2 eps / 3) ln(2 / pf) /
 * (eps^2 delta)), a Bernstein-bound constant for the Omega(log(1/pf) /
 * (eps^2 delta)) of Sec. 2.1. Returns 0 on invalid input. */
FPPR_API uint64_t fppr_walks_for_guarantee(double eps, double delta, double pf);

enum {
  FPPR_STITCH = 1u,    /* take pool entries at small nodes (needs a pool built
                          with the same alpha) */
  FPPR_COUNTS = 2u,    /* write per-source sparse counts */
  FPPR_DIGESTS = 4u,   /* write per-source digests */
  FPPR_STATS = 8u      /* accumulate walk statistics */
};

typedef struct {
  double alpha;    /* termination probability in (0, 1) */
  uint32_t R;      /* walks per source (omega of Algorithm 2), 1 <= R <= 2^20;
                      FPPR_COUNTS needs R <= 4096 */
  uint64_t seed;   /* Philox key */
  uint32_t topk;   /* k largest counts per source, 0 <= k <= R and k <= 1024 */
  uint32_t flags;  /* FPPR_* bits */
  uint32_t blocks_per_cu; /* walk-launch width: 256-thread workgroups per
                             compute unit, 0 = as many as fit; never changes
                             results */
} fppr_params;

/* Counters accumulated over a run (device memory, 8 x uint64, added to; the
 * caller zeroes them). steps counts edges traversed: restarts and every
 * step of a stitched move included. */
typedef struct {
  uint64_t walks;
  uint64_t moves;          /* Philox-keyed iterations */
  uint64_t steps;
  uint64_t capped;         /* walks stopped by FPPR_MOVE_CAP */
  uint64_t dangling_moves; /* restarts to the head */
  uint64_t plain_moves;    /* weighted picks */
  uint64_t stitched_moves; /* pool entries taken */
  uint64_t probe_log_sum;  /* sum over plain moves of ceil(log2(out-degree)) */
} fppr_stats;

/* Stage timer: HIP events the library records on the run's stream around
 * its walk kernel and its aggregation kernel. Created and owned by the
 * caller through these calls. */
typedef struct fppr_profile fppr_profile;
FPPR_API fppr_status fppr_profile_create(fppr_profile** out);
FPPR_API fppr_status fppr_profile_destroy(fppr_profile* p);
/* Waits for the events of the last run that used `p` and returns the walk
 * and aggregation kernel durations in milliseconds (host outputs). */
FPPR_API fppr_status fppr_profile_read(fppr_profile* p, double* walk_ms, double* aggregate_ms);
/* Splits the walk time of the last single-launch run that used `p`: the walk
 * kernel alone, and the time after it until the coin-only kernel that an
 * all-nodes run launches for the nodes without out-edges has also finished
 * (it runs beside the walk kernel on a stream of the graph's own; 0 when it
 * finished first or was not launched; see fppr_run).
 * Blocked runs report their whole walk-and-count time as walk kernel time;
 * batch runs report 0 coin-only time (their coin-only kernels run on the
 * counting streams and are timed with the aggregation). */
FPPR_API fppr_status fppr_profile_read_walk(fppr_profile* p, double* walk_kernel_ms, double* coin_only_ms);

/* Outputs (all device pointers, caller-owned; NULL = not wanted):
 *  topk       [n_src][k][2] uint32: (t, count) by count descending then t
 *             ascending; rows shorter than k padded with (FPPR_NO_NODE, 0)
 *  counts     [n_src][R][2] uint32: (t, count) sorted by t; entries beyond
 *             n_distinct[s] are zero (needs FPPR_COUNTS)
 *  n_distinct [n_src] uint32: number of distinct endpoints (with counts)
 *  digest     [n_src] uint64: sum mod 2^64 over (t, count) of
 *             fmix64(fmix64(s << 32 | t) ^ (count * 0x9E3779B97F4A7C15)),
 *             fmix64 = MurmurHash3's 64-bit finalizer (needs FPPR_DIGESTS)
 *  endpoints  [n_src][R] uint32: raw endpoint of walk i of source row j at
 *             j * R + i; when given it replaces the workspace's endpoint
 *             buffer
 *  stats      one fppr_stats (needs FPPR_STATS)
 *  profile    host handle of a stage timer, or NULL */
typedef struct {
  uint32_t* topk;
  uint32_t* counts;
  uint32_t* n_distinct;
  uint64_t* digest;
  uint32_t* endpoints;
  fppr_stats* stats;
  fppr_profile* profile;
} fppr_out;

/* Counting and top-k alone (Algorithm 2's last phase: group the walks by
 * (head, tail) and count them; Sec. 1: keep the endpoints some walk
 * reached) over endpoints the caller already has, e.g. those of
 * fppr_run_alias or fppr_run_big_moves: source row j (source id
 * sources[j], or j when sources is NULL, which the digest uses) owns the R
 * walks endpoints[j * R .. j * R + R) (device u32; FPPR_NO_NODE entries are
 * not counted). p gives R, topk and the output flags FPPR_COUNTS /
 * FPPR_DIGESTS (alpha, seed, FPPR_STITCH and FPPR_STATS are not used);
 * outputs as for fppr_run. workspace: device, at least fppr_aggregate_plan
 * bytes (the hash tables of R > 256 without counts). Identical to the
 * counting of fppr_run over the same endpoints. Asynchronous on `stream`. */
FPPR_API fppr_status fppr_aggregate_plan(const fppr_params* p, uint64_t n_sources, uint64_t* workspace_bytes);
FPPR_API fppr_status fppr_aggregate(const fppr_params* p, const uint32_t* endpoints, const uint32_t* sources,
                                    uint64_t n_sources, void* workspace, uint64_t workspace_bytes,
                                    const fppr_out* out, void* stream);

/* Workspace size (bytes, 256-byte aligned device memory) for a run of
 * n_sources sources. Pure host computation. */
FPPR_API fppr_status fppr_plan(const fppr_graph* g, const fppr_params* p, uint64_t n_sources,
                               uint64_t* workspace_bytes);

/* Memory-bounded runs (the bounded injection of Sec. 4.3: only as many walks
 * as memory holds are in flight). The largest block of sources (<=
 * n_sources) whose run fits budget_bytes of workspace (host outputs: the
 * block and its fppr_plan bytes). INVALID_ARGUMENT if not one source fits.
 * Pure host computation. */
FPPR_API fppr_status fppr_plan_block(const fppr_graph* g, const fppr_params* p, uint64_t n_sources,
                                     uint64_t budget_bytes, uint64_t* block_sources,
                                     uint64_t* workspace_bytes);

/* Runs R walks from each source and aggregates them (Algorithm 2).
 * sources: device uint32 [n_sources] (each < n; duplicates allowed), or NULL
 * for all nodes 0..n-1 (then n_sources must equal n). n_sources == 0 is a
 * no-op. workspace: device; with >= fppr_plan(n_sources) bytes one walk launch
 * covers every source; with less (and out->endpoints == NULL) the sources run
 * in blocks of the size fppr_plan_block gives for that many bytes, one walk
 * launch and one counting launch per block, in order. Walk keys do not
 * depend on the blocking, so the results are identical; a profile then
 * reports the whole run as walk time. Asynchronous on `stream`. */
FPPR_API fppr_status fppr_run(fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                              uint64_t n_sources, void* workspace, uint64_t workspace_bytes,
                              const fppr_out* out, void* stream);

/* Size of the device workspace that fppr_run_static uses (per GPU). */
#define FPPR_STATIC_SCRATCH_BYTES (64ull << 20)

/* fppr_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same walks, counting and outputs as fppr_run, with its workspace taken
 * from a fixed device array of FPPR_STATIC_SCRATCH_BYTES inside the library
 * (one per GPU, created when the library's code is loaded on that GPU and
 * kept until the process ends). No hipMalloc, hipFree or other allocation is
 * made. The array's address is looked up on the first call on each device.
 * Runs larger than the array go in blocks of sources as fppr_run does with
 * a small workspace; results are identical to fppr_run's. `out` is the
 * caller's, as for fppr_run; the graph's device must be the current device.
 * INVALID_ARGUMENT as for fppr_run, or when one source needs more workspace
 * than the array holds, or when out->endpoints is given and the whole run
 * does not fit the array. Asynchronous on `stream`.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two host threads) race and give wrong results; calls
 * in sequence on one stream are safe, and each clears what it needs.
 * There is no fppr_run_check for this form: a source id >= n gets no walks,
 * so its row has n_distinct 0 and a top-k of padding entries. */
FPPR_API fppr_status fppr_run_static(fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                                     uint64_t n_sources, const fppr_out* out, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many graphs or source sets in one persistent walk launch.
 * Algorithm 2 runs all walks of all nodes together; a batch extends that to
 * several independent problems of uneven sizes so that small ones do not
 * leave the GPU idle and launch overheads are paid once. Every item keeps
 * its own seed, alpha, R, k and outputs; its results are bit-identical to
 * fppr_run of that item alone (draws depend only on the item's seed and the
 * source, walk and move indices).
 * ---------------------------------------------------------------------- */
typedef struct fppr_batch fppr_batch;

typedef struct {
  fppr_graph* graph;         /* device graph (pool built if FPPR_STITCH) */
  fppr_params params;        /* as for fppr_run */
  const uint32_t* sources;   /* device uint32 [n_sources], or NULL = all nodes */
  uint64_t n_sources;
  fppr_out out;              /* device outputs of this item (profile ignored) */
} fppr_batch_item;

enum {
  FPPR_BATCH_REBUILD = 1u  /* each run of the batch first rebuilds every
                              distinct graph of its items (fppr_graph_rebuild:
                              prefixes, records, trees, pool), on the same
                              stream, so the captured sequence is the whole
                              path */
};

typedef struct {
  uint32_t flags;          /* FPPR_BATCH_* bits */
  uint32_t blocks_per_cu;  /* width of the one walk launch (0 = as many as
                              fit); the items' own blocks_per_cu are ignored */
} fppr_batch_opts;

/* Workspace bytes for a batch (control words, the walk table, one endpoint
 * buffer per item). Pure host computation. */
FPPR_API fppr_status fppr_batch_plan(const fppr_batch_item* items, uint32_t count,
                                     uint64_t* workspace_bytes);

/* Validates every item as fppr_run would, lays out `workspace` (device,
 * >= fppr_batch_plan bytes) and uploads the walk table (synchronous); opts
 * may be NULL (no rebuild, full width). The items' graphs either all have
 * the guide layout or none does (INVALID_ARGUMENT otherwise: one launch runs
 * one walk kernel). Items
 * are ordered by decreasing walk count in the table. The batch keeps a copy
 * of `items`; graphs, sources, outputs and the workspace must outlive it. */
FPPR_API fppr_status fppr_batch_create(const fppr_batch_item* items, uint32_t count,
                                       const fppr_batch_opts* opts, void* workspace,
                                       uint64_t workspace_bytes, fppr_batch** out);

/* Enqueues the batch on `stream`: one persistent walk launch over every
 * item's walks, then each item's counting and top-k. `stats` (device, may be
 * NULL) accumulates over the whole batch; `profile` (may be NULL) times the
 * walk launch and the aggregation launches. */
FPPR_API fppr_status fppr_batch_run(fppr_batch* b, fppr_stats* stats, fppr_profile* profile,
                                    void* stream);

/* Captures fppr_batch_run(b, stats, NULL, stream) into a HIP graph owned by
 * the batch (replacing an earlier capture); fppr_batch_launch replays it on
 * `stream`. The capture records kernels only (counters are cleared by a fill
 * kernel, not a memset). */
FPPR_API fppr_status fppr_batch_capture(fppr_batch* b, fppr_stats* stats, void* stream);
FPPR_API fppr_status fppr_batch_launch(fppr_batch* b, void* stream);

/* Synchronises `stream`; INVALID_ARGUMENT if a batch run met a source id >= n
 * or (FPPR_BATCH_REBUILD) a graph failed its rebuild's validation. */
FPPR_API fppr_status fppr_batch_check(fppr_batch* b, void* stream);

/* The batch's run manifest as JSON (host output): for every item its graph
 * (n, m, layout, hub threshold, tree rows, and the short-walk pool S, L, K,
 * seed, alpha when one is built: the parameters that change a stitched
 * run's results, and that a checker must use), its parameters (alpha, R,
 * seed, top-k, flags), its source count, whether its nodes without
 * out-edges run in the coin-only kernel, its place in the walk table and
 * its counting stream; and the launch width. It records the knobs the
 * autotuner (fppr_autotune) left on each graph before the batch was made
 * (Sec. 4.3's gamma, chosen and then recorded). json: host buffer of `cap`
 * bytes or NULL; *needed (required) gets the length including the final
 * NUL. INVALID_ARGUMENT when json is given and cap < *needed (nothing
 * written). */
FPPR_API fppr_status fppr_batch_manifest(const fppr_batch* b, char* json, size_t cap, size_t* needed);
/* Waits until the batch's last run or replay has finished, then frees the
 * batch (its streams, events and captured graph; not the caller's
 * workspace, graphs or outputs, which may be freed after this returns). */
FPPR_API fppr_status fppr_batch_destroy(fppr_batch* b);

/* ------------------------------------------------------------------------
 * Autotuner. The paper sizes its pipelines from cluster memory and checks the
 * choice by experiment (Sec. 4.3, the gamma analysis; Sec. 5); here the knobs
 * are picked per graph by timed trial runs on a sample of sources:
 *  - hub threshold and walk-launch width, which never change results;
 *  - the short-walk pool (or none), which does: the chosen candidate is
 *    reported so that every other run of that graph, and any checker, uses
 *    the same one.
 * ---------------------------------------------------------------------- */
typedef struct {
  const uint32_t* hub_thresholds;  /* host [n_hub_thresholds] candidates, or NULL
                                      (keep the graph's) */
  uint32_t n_hub_thresholds;
  const uint32_t* blocks_per_cu;   /* host [n_blocks_per_cu] candidates, or NULL
                                      (0 = as many as fit) */
  uint32_t n_blocks_per_cu;
  const fppr_pool_opts* pools;     /* host [n_pools] short-walk candidates (their
                                      alpha is replaced by the run's) */
  uint32_t n_pools;
  uint32_t allow_plain;            /* nonzero: runs without stitching compete too
                                      (always the case when n_pools == 0) */
  uint64_t n_sources;              /* sources of the real run (0 = n), for the
                                      cost estimate */
  uint32_t sample;                 /* trial sources, evenly spread over the
                                      nodes (0 = min(n, 65536)) */
  uint32_t reps;                   /* timed repetitions per trial, best kept
                                      (0 = 3) */
} fppr_tune_space;

typedef struct {
  uint32_t hub_threshold;  /* chosen (the graph is left laid out with it) */
  uint32_t blocks_per_cu;  /* chosen launch width */
  int32_t pool;            /* index of the chosen pool candidate (the graph
                              keeps that pool), or -1 = plain walks (the graph
                              keeps no pool) */
  uint32_t trials;         /* configurations timed */
  double est_ms;           /* estimated run: pool build + walks scaled from the
                              sample to n_sources */
  double plain_est_ms;     /* the same estimate for plain walks at the chosen
                              threshold and width (0 if not timed) */
} fppr_tune_result;

/* Times the candidates (one coordinate at a time: hub threshold with plain
 * walks, then launch width, then the pools) with p's alpha, R and seed; p's
 * flags, topk and blocks_per_cu are ignored. Leaves the graph in the chosen
 * configuration. Synchronous; allocates trial buffers for its own use. */
FPPR_API fppr_status fppr_autotune(fppr_graph* g, const fppr_params* p, const fppr_tune_space* space,
                                   fppr_tune_result* result, void* stream);

/* ------------------------------------------------------------------------
 * Serving. A server keeps one graph (and its pool) resident and answers PPR
 * queries (sources, walk budget R, alpha, seed, k) that arrive over time.
 * Continuous mode: a scheduler thread admits queued queries as slots and
 * device memory free up (each needs n_sources * R * 4 bytes of endpoints plus
 * its outputs), and advances all admitted queries together in walk slices of
 * bounded size; a query that arrives while others run joins the next slice.
 * Algorithm 2's pipelines play the same role (Sec. 4.3: new walks start while
 * earlier ones are in flight, and the in-flight count is bounded by memory).
 * When a query's last walks have run, its counting and top-k go to a second
 * stream and its results are copied to pinned host memory. FIFO mode is the
 * comparison point: one plain launch per query, in arrival order. Draws are
 * keyed by the query's seed, source and walk index only, so a query's result
 * is bit-identical alone, in any mix and in either mode.
 * ---------------------------------------------------------------------- */
typedef struct fppr_server fppr_server;

enum { FPPR_SERVE_CONTINUOUS = 0, FPPR_SERVE_FIFO = 1 };

typedef struct {
  uint32_t mode;           /* FPPR_SERVE_CONTINUOUS or FPPR_SERVE_FIFO */
  uint32_t max_requests;   /* queries in flight at once (slots), 1..4096 */
  uint64_t memory_bytes;   /* device memory for in-flight queries' endpoints
                              and outputs, allocated at create (>= 1 MiB) */
  uint64_t host_bytes;     /* pinned host memory for queued sources and
                              finished results until fppr_server_poll takes
                              them (>= 1 MiB) */
  uint64_t slice_walks;    /* walks per slice in continuous mode (>= 2^16) */
  uint32_t blocks_per_cu;  /* walk-launch width (0 = as many as fit) */
} fppr_server_opts;

typedef struct {
  const uint32_t* sources; /* host [n_sources], each < n; copied by submit */
  uint32_t n_sources;      /* >= 1 */
  uint32_t R;              /* walks per source, 1..2^20 */
  double alpha;            /* in (0, 1); FPPR_STITCH needs the pool's alpha */
  uint64_t seed;           /* Philox key of the query's walks */
  uint32_t topk;           /* 1..1024, <= R */
  uint32_t flags;          /* FPPR_STITCH or 0 */
} fppr_query;

typedef struct {
  uint64_t submit_ns;      /* steady-clock times (ns) of submit, admission */
  uint64_t admit_ns;
  uint64_t done_ns;        /* and of the results reaching host memory */
  uint64_t walks;          /* n_sources * R */
} fppr_query_info;

typedef struct {
  uint64_t submitted, completed, slices, walk_launches;
  uint64_t peak_in_flight;     /* most queries in flight at once */
  uint64_t peak_device_bytes;  /* most device memory held by queries */
  fppr_stats walk_stats;       /* summed over all walk launches */
  uint64_t cancelled;          /* queries cancelled before they completed */
} fppr_server_counters;

/* Latency statistics over completed queries (latency = submit to results in
 * pinned host memory). Percentiles are nearest-rank: p50 is the smallest
 * latency with at least half of the queries at or below it. qps = count /
 * span, span = first submit to last completion of the counted queries. */
typedef struct {
  uint64_t count;
  double p50_ms, p99_ms, mean_ms, max_ms;
  double span_s;
  double qps;
} fppr_latency;

/* Creates the server and its scheduler thread on the current device (the
 * graph's). The graph (and pool) must stay alive and unchanged until
 * fppr_server_destroy. */
FPPR_API fppr_status fppr_server_create(fppr_graph* g, const fppr_server_opts* opts, fppr_server** out);

/* Queues a query (thread-safe, does not block on the GPU) and returns its id.
 * INVALID_ARGUMENT if it is malformed or could never fit the server's memory
 * or pinned budget. */
FPPR_API fppr_status fppr_server_submit(fppr_server* s, const fppr_query* q, uint64_t* id);

/* FPPR_NOT_READY while query `id` runs; FPPR_OK once done: copies its results
 * (host buffers: topk [n_sources][k][2] uint32 as for fppr_run, digest
 * [n_sources] uint64; either may be NULL) and `info`, and forgets the id.
 * fppr_server_wait blocks until done. Both return FPPR_CANCELLED (and forget
 * the id) for a query cancelled by fppr_server_cancel. */
FPPR_API fppr_status fppr_server_poll(fppr_server* s, uint64_t id, uint32_t* topk, uint64_t* digest,
                                      fppr_query_info* info);
FPPR_API fppr_status fppr_server_wait(fppr_server* s, uint64_t id, uint32_t* topk, uint64_t* digest,
                                      fppr_query_info* info);

/* Counters since create (host output; walk_stats synchronises the device). */
FPPR_API fppr_status fppr_server_stats(fppr_server* s, fppr_server_counters* out);

/* Latency statistics (host output) over the queries with id >= first_id
 * that completed since create (0 = all), whether or not their results were
 * taken. The p50/p99 reported beside throughput (Sec. 4.3's in-flight bound
 * makes latency, not only throughput, the server's measure). */
FPPR_API fppr_status fppr_server_latency(fppr_server* s, uint64_t first_id, fppr_latency* out);

/* Cancels query `id` (thread-safe; returns at once). A queued query never
 * reaches the GPU. An admitted one gets no further walk slices; the work
 * already queued for it finishes, and its device memory is freed only after
 * that. A finished query that was not yet taken loses its results. From
 * then on fppr_server_poll / fppr_server_wait of `id` return FPPR_CANCELLED
 * (once the GPU is done with it) and forget the id. INVALID_ARGUMENT for an
 * unknown (or already taken) id. */
FPPR_API fppr_status fppr_server_cancel(fppr_server* s, uint64_t id);

/* Finishes every query already submitted (queued ones included, unless
 * cancelled), stops the thread, frees everything. */
FPPR_API fppr_status fppr_server_destroy(fppr_server* s);

/* Synchronises `stream` and reports whether a run that used `workspace` met
 * a source id >= n (INVALID_ARGUMENT; such a source gets no walks and its
 * endpoints read FPPR_NO_NODE) or FPPR_OK. */
FPPR_API fppr_status fppr_run_check(const void* workspace, void* stream);

/* Thread-local text of the last failure ("" if none). */
FPPR_API const char* fppr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
