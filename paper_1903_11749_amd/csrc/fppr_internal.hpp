// Host-side internals of the library: the graph object and the kernel launch
// entry points of each stage.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/fppr.h"
#include "agg_hash.hpp"
#include "fppr_device.hpp"
#include "guide.hpp"

namespace fppr {

// Error bits written by the validation kernels.
enum : uint32_t {
  kErrOffsets = 1u,
  kErrCol = 2u,
  kErrWeight = 4u,
  kErrDegree = 16u,
  kErrCapacity = 32u,
  kErrNarrow = 64u,  // a row total above 2^32 - 1 in a graph with the narrow layout
  kErrGuide = 128u,  // guide tables: more child entries, tables or levels than the graph holds
};

// Child levels of the guide tables are built one pass each, at most this many.
constexpr uint32_t kGuideLevels = 64;
// Allocation counters of a guide-table build (device memory).
struct GuideCtl {
  unsigned long long next_entry;       // first free entry
  uint32_t pad[30];                    // the two counters in lines of their own
  uint32_t tables[kGuideLevels + 2];   // small child-table slots taken per level
  uint32_t big[kGuideLevels + 2];      // large child-table slots taken per level
};

}  // namespace fppr

struct fppr_graph {
  int device = 0;
  uint32_t n = 0;
  uint64_t m = 0;
  // CSR on the device (borrowed, or owned copies of host input)
  const uint64_t* off = nullptr;
  const uint32_t* col = nullptr;
  const uint32_t* w = nullptr;
  bool owns_csr = false;
  // derived arrays
  fppr::Block* rec = nullptr;       // [n] node lines
  fppr::Block* blocks = nullptr;    // [n_blocks] row regions: tree nodes, leaf blocks
  uint64_t n_blocks = 0;
  uint64_t* region = nullptr;       // [n] first block of each row's region
  uint32_t tree_min = 8;            // rows with more edges carry a prefix tree
  bool narrow = false;              // narrow layout: u32 prefixes (fixed at creation)
  uint32_t n_tree = 0;              // rows with a tree
  bool tagged = false;              // leaf destinations carry class tags (n <= 2^30)
  uint8_t* cls = nullptr;           // [n] class of each node (kTagDangling, kTagSmall or 0)
  uint32_t S_tag = 0;               // small-node bound the tags were made with (0: none)
  // scratch (kept for rebuilds)
  uint32_t* flag = nullptr;         // [n]   per-node u32 input of scans
  uint64_t* scan = nullptr;         // [n]   exclusive scan output
  uint32_t* rows = nullptr;         // [n]   list of long rows
  uint64_t* scan_blocks = nullptr;  // block sums of the scans
  uint32_t* d_err = nullptr;        // [16]  error bits and counters
  // pool
  bool has_pool = false;
  fppr_pool_opts pool_opts{};
  uint32_t pool_T = 0;
  uint32_t K_log2 = 0;
  uint64_t n_small = 0;
  uint64_t* pool = nullptr;          // [n * K]: node v's K entries at v * K (only small nodes' are written)
  // nodes with out-edges and without, each in id order (degrees never change
  // after create, so these are built once)
  uint32_t* live = nullptr;          // [n_live]
  uint32_t* dang = nullptr;          // [n_dang]
  uint64_t n_live = 0, n_dang = 0;
  // side stream of all-nodes runs on graphs with many nodes without
  // out-edges: their coin-only kernel runs there beside the walk kernel
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  std::mutex side_mu;  // keeps each event record and its wait together across host threads
  // guide-table layout (guide.hpp): instead of node lines and row regions
  bool guide = false;
  fppr::guide::Head* ghead = nullptr;      // [n] first entry of each node's table, lg | class << 8
  fppr::guide::Entry* gent = nullptr;      // [g_cap] row tables [0, g_entries1), then child tables
  uint64_t* gT = nullptr;                  // [m] draw thresholds of every edge but a row's last (~0 there)
  uint4* gerec = nullptr;                  // [m] record of every edge's destination: id | tag, base, lg
  uint32_t* gclass = nullptr;              // [n_live] rows by size class (1, 2, 3-4, ..., 33-64, 65-1024, more edges)
  uint64_t gclass_off[10] = {0};           // class c's rows at gclass[gclass_off[c] .. gclass_off[c + 1])
  uint2* gruns = nullptr;                  // [n_runs] (row, first entry) of each run of 16 entries of the longest rows
  uint64_t n_runs = 0;
  uint2* gtiles = nullptr;                 // [n_tiles] (row, tile) of each 1024-edge tile of the longest rows
  uint64_t n_tiles = 0;
  uint64_t* gtile_first = nullptr;         // [rows of that class] first tile of each
  uint64_t* gtsum = nullptr;               // [n_tiles] weight sum, offset within the row, row total
  uint64_t* gtoff = nullptr;
  uint64_t* gttot = nullptr;
  // child tables of alternate levels: g_tcap small ones, then g_tcap_big large ones
  fppr::guide::Pending* gtab[2] = {nullptr, nullptr};
  fppr::GuideCtl* gctl = nullptr;
  uint64_t g_entries1 = 0, g_cap = 0;
  uint32_t g_tcap = 0, g_tcap_big = 0, g_levels = 1;       // deepest level of the last full build
  uint64_t pool_cap = 0;             // u64 words allocated
  uint32_t* small_nodes = nullptr;   // [n] rank -> node
  uint64_t device_bytes = 0;
};

struct fppr_profile {
  // start, walks done, aggregation start, aggregation done, walk kernel done
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace fppr {

void set_error(const std::string& msg);
fppr_status hip_fail(hipError_t e, const char* what);
fppr_status check_params(const fppr_graph* g, const fppr_params* p);
fppr_status check_outputs(const fppr_params* p, const fppr_out* out);
// frees the pool (the graph then has none)
void drop_pool(fppr_graph* g);

// build.hip
hipError_t launch_validate(const fppr_graph* g, hipStream_t s, bool maxima);  // maxima: max degree and weight (layout choice)
// region sizes + scan -> g->region, total blocks at d_err[2..3]
hipError_t launch_region_sizes(fppr_graph* g, hipStream_t s);
// nodes with / without out-edges -> g->live, g->dang; the count of the former
// at d_err[10..11]
hipError_t launch_split_nodes(fppr_graph* g, hipStream_t s);
// prefixes and destinations into leaf blocks, node records
hipError_t launch_leaves(fppr_graph* g, hipStream_t s, bool count_trees);
// class of every node for the destination tags (S: the pool's small-node bound, 0 = none)
hipError_t launch_node_class(fppr_graph* g, uint32_t S, hipStream_t s);
// exclusive scan of u32 input to u64 output; writes the total to *total_dev
hipError_t launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* blocks,
                           uint64_t* total_dev, hipStream_t s);
uint64_t scan_block_count(uint64_t n);

// guide.hip
// table sizes of every node + scan -> g->scan, total at d_err[4..5]
hipError_t launch_guide_sizes(fppr_graph* g, hipStream_t s);
// the rows of size class c (see gclass) to gclass + at; their count at d_err[14..15]
hipError_t launch_guide_class(fppr_graph* g, uint32_t c, uint64_t at, hipStream_t s);
// entry runs of the longest rows: counts and scan (total at d_err[14..15]), then the list
hipError_t launch_guide_runs_count(fppr_graph* g, hipStream_t s);
// 1024-edge tiles of the longest rows: counts and scan (total at d_err[14..15]), then the list
hipError_t launch_guide_tiles_count(fppr_graph* g, hipStream_t s);
hipError_t launch_guide_tiles_fill(fppr_graph* g, hipStream_t s);
hipError_t launch_guide_runs_fill(fppr_graph* g, hipStream_t s);
// heads (bases from g->scan when `bases`, else kept), row tables and the
// first child level's list; children deeper than `levels` are refused
hipError_t launch_guide_build(fppr_graph* g, bool bases, uint32_t levels, hipStream_t s);
// the child tables of one level (2 <= level <= levels)
hipError_t launch_guide_level(fppr_graph* g, uint32_t level, uint32_t levels, hipStream_t s);
hipError_t launch_pool_guide(fppr_graph* g, hipStream_t s);
hipError_t launch_pool_guide_export(const fppr_graph* g, uint64_t* out, hipStream_t s);

// pool.hip
hipError_t launch_small_flags(fppr_graph* g, uint32_t S, hipStream_t s);
hipError_t launch_small_compact(fppr_graph* g, uint32_t S, hipStream_t s);
hipError_t launch_pool(fppr_graph* g, hipStream_t s);
// the pool's entries in canonical order (small nodes by id, then slot; end ids
// without tags) into out[n_small * K]
hipError_t launch_pool_export(const fppr_graph* g, uint64_t* out, hipStream_t s);

// walk.hip
// One descriptor of the walk table: a run of walks on one graph. Ids
// [first, first + count) of the launch map to walk indices walk0 + (id -
// first) of the run; walk index w is walk w % R of source row w / R, and its
// endpoint goes to endpoints[w]. first is a multiple of kWalkChunk.
constexpr uint64_t kWalkChunk = 256;
constexpr uint32_t kSrcBuf = kWalkChunk + 2;  // source ids of one chunk in LDS (rows it spans + 1)
struct WalkDesc {
  const Block* rec;          // node lines
  const Block* blocks;       // row regions
  const uint64_t* pool;      // stitched runs: the graph's pool (node v's entries at v << K_log2;
                             // 16-byte entries in graphs with guide tables)
  const fppr::guide::Head* ghead;   // guide-table graphs: node heads
  const fppr::guide::Entry* gent;   // guide-table graphs: table entries
  uint64_t g_cap;                   // guide-table graphs: entries allocated
  const uint32_t* sources;   // source ids by row, or null for row = node id
  uint32_t* endpoints;
  uint64_t first;
  uint64_t count;
  uint64_t walk0;
  uint64_t R_magic;          // floor((2^64 - 1) / R)
  uint32_t R, n, key0, key1, T, tree_min, K_log2;
  uint32_t S_small;          // stitched runs: small nodes have 1 <= out-degree <= S_small; 0 = plain
  uint32_t flags;            // kDescEpBySource, kDescNarrow, kDescTagged
};
// the endpoint of walk i of source s goes to endpoints[s * R + i] (a run over
// a list of some of the nodes that fills an all-nodes endpoint buffer)
constexpr uint32_t kDescEpBySource = 1;
// the graph has the narrow layout (u32 prefixes, 16-edge leaves, 32-key nodes)
constexpr uint32_t kDescNarrow = 2;
// the graph's leaf destinations and pool entries carry class tags
constexpr uint32_t kDescTagged = 4;
// the graph has the guide-table layout (every descriptor of a table must)
constexpr uint32_t kDescGuide = 8;
// lane_keys: the per-lane-key form of the kernel (for tables whose
// descriptors all read one graph; see same_graph_table)
// descs: the table on the device; host: the same table in host memory (it
// selects the kernel's form: layouts, per-lane keys, inline restarts)
hipError_t launch_walk(const WalkDesc* descs, const WalkDesc* host, uint32_t ndesc, uint64_t total,
                       unsigned long long* ctl, fppr_stats* stats, uint32_t blocks_per_cu, hipStream_t s);
// walk_guide.hip: the walk kernel of tables whose descriptors all have kDescGuide
hipError_t launch_walk_guide(const WalkDesc* descs, const WalkDesc* host, uint32_t ndesc, uint64_t total,
                             unsigned long long* ctl, fppr_stats* stats, uint32_t blocks_per_cu, hipStream_t s);
// 0 when every descriptor's graph is wide, 1 when every one is narrow, 2 mixed
int table_layout(const WalkDesc* h, uint32_t ndesc);
// true when a table (host copy) has more than one descriptor and all of them
// read the same graph arrays
bool same_graph_table(const WalkDesc* h, uint32_t ndesc);
hipError_t launch_set_desc(const WalkDesc& d, WalkDesc* dst, hipStream_t s);
// Walks from the nodes without out-edges of g, R each, under p's seed and
// alpha: every move is a restart at the source (Sec. 2.1), so a walk is its
// sequence of coins and always ends at its source; endpoint of walk i of
// node s -> endpoints[s * R + i]. Statistics as the walk kernel counts them.
hipError_t launch_dangling(const fppr_graph* g, const fppr_params* p, uint32_t* endpoints, fppr_stats* stats,
                           hipStream_t s);
// all-nodes runs split off the walks from nodes without out-edges when those
// are a quarter of the nodes or more (below that the extra source list and
// launch cost more than they save)
inline bool split_dangling(const fppr_graph* g) { return g->n_dang > 0 && g->n_dang * 4 >= g->n; }
// descriptor of walks [walk0, walk0 + count) of a run of `p` on graph g
WalkDesc make_desc(const fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                   uint64_t n_sources, uint32_t* endpoints, uint64_t first, uint64_t walk0,
                   uint64_t count);
hipError_t launch_zero_u64(uint64_t* p, uint64_t count, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s);

// aggregate.hip
struct AggLaunch {
  const uint32_t* endpoints;
  const uint32_t* sources;
  uint64_t n_src;
  uint64_t row0;     // without sources, row r is node row0 + r
  uint32_t R;
  uint32_t k;
  uint32_t* topk;
  uint32_t* counts;
  uint32_t* n_distinct;
  uint64_t* digest;
  uint64_t* table;   // agg_table_bytes of scratch when agg_uses_table (filled here)
  uint32_t H_log2;   // set by launch_aggregate
};
hipError_t launch_aggregate(const AggLaunch& a, hipStream_t s);
AggLaunch make_agg(const fppr_params* p, const uint32_t* endpoints, const uint32_t* sources,
                   uint64_t n_sources, const fppr_out* out);
// sizes of the counting paths and their hash tables: agg_hash.hpp

}  // namespace fppr
