// Batches: several graphs or source sets served by one persistent walk
// launch (the walk table holds one descriptor per item), then each item's
// counting and top-k; optionally captured once into a HIP graph and replayed.
// The per-graph rebuilds in front of the walks and the per-item counting after
// them are independent of each other, so they are spread over four streams
// (the caller's and three of the batch's, forked from and joined back into the
// caller's): the many small kernels of small graphs overlap instead of running
// one after another. Items whose counting uses the shared hash area stay on
// the caller's stream, one after the other.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "batch_layout.hpp"
#include "fppr_internal.hpp"

using namespace fppr;

namespace {

constexpr uint64_t kCtlBytes = kBatchCtlBytes;
constexpr int kLanes = 4;  // the caller's stream + 3 of the batch's

fppr_status invalid(const std::string& msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

uint64_t item_sources(const fppr_batch_item& it) {
  return it.sources ? it.n_sources : it.graph->n;
}

}  // namespace

struct fppr_batch {
  std::vector<fppr_batch_item> items;
  fppr_batch_opts opts{};
  std::vector<fppr_graph*> graphs;    // distinct graphs of the items
  std::vector<WalkDesc> host_table;
  std::vector<uint32_t*> endpoints;   // per item
  unsigned long long* ctl = nullptr;  // in the workspace
  uint64_t* agg_table = nullptr;      // hash tables of items with R > 4096 (shared)
  WalkDesc* table = nullptr;          // in the workspace
  uint64_t total = 0;                 // padded walk ids
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t aux[kLanes - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kLanes - 1] = {};
  hipEvent_t done = nullptr;  // recorded behind every run and replay; destroy waits for it
  std::vector<int> graph_lane, item_lane;  // lane of each graph's rebuild / item's counting
  std::vector<bool> split;                 // all-nodes item: coin-only kernel for nodes without out-edges
  std::vector<BatchRun> runs;              // the walk table (item, first id, walks), largest first
};

namespace {

fppr_status check_items(const fppr_batch_item* items, uint32_t count) {
  if (!items || count == 0) return invalid("batch needs at least one item");
  for (uint32_t k = 0; k < count; ++k) {
    const fppr_batch_item& it = items[k];
    if (!it.graph) return invalid("batch item " + std::to_string(k) + ": graph is NULL");
    // one walk launch serves the whole table, with one kernel per layout family
    if (it.graph->guide != items[0].graph->guide)
      return invalid("batch item " + std::to_string(k) +
                     ": a batch cannot mix graphs with guide tables and graphs with the tree layouts");
    fppr_status st = check_params(it.graph, &it.params);
    if (st != FPPR_OK) return st;
    if (!it.sources && it.n_sources != it.graph->n && it.n_sources != 0)
      return invalid("batch item " + std::to_string(k) + ": sources == NULL needs n_sources == n");
    if ((st = check_outputs(&it.params, &it.out)) != FPPR_OK) return st;
    if (item_sources(it) > (1ull << 40) / it.params.R)
      return invalid("batch item " + std::to_string(k) + ": n_sources * R too large");
  }
  return FPPR_OK;
}

// the shapes batch_layout needs (an all-nodes item over a graph with many
// nodes without out-edges is split: see fppr_batch_create)
std::vector<BatchItemShape> shapes(const fppr_batch_item* items, uint32_t count) {
  std::vector<BatchItemShape> v(count);
  for (uint32_t k = 0; k < count; ++k) {
    const fppr_batch_item& it = items[k];
    v[k].n_rows = item_sources(it);
    v[k].R = it.params.R;
    v[k].counts = (it.params.flags & FPPR_COUNTS) != 0;
    v[k].split = !it.sources && split_dangling(it.graph);
    v[k].n_live = it.graph->n_live;
  }
  return v;
}

void free_batch(fppr_batch* b) {
  if (!b) return;
  // the last run or replay (on the caller's stream) may still read the
  // captured graph and write the workspace the caller frees after this call
  if (b->done) (void)hipEventSynchronize(b->done);
  for (hipStream_t a : b->aux)
    if (a) (void)hipStreamSynchronize(a);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (hipStream_t a : b->aux)
    if (a) (void)hipStreamDestroy(a);
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->done) (void)hipEventDestroy(b->done);
  delete b;
}

// Greedy lanes: each job (largest first) goes to the least loaded lane.
std::vector<int> assign_lanes(const std::vector<uint64_t>& cost, const std::vector<bool>& pinned) {
  std::vector<uint32_t> order(cost.size());
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
  uint64_t load[kLanes] = {};
  std::vector<int> lane(cost.size(), 0);
  for (uint32_t k : order) {
    int best = 0;
    if (!pinned[k])
      for (int l = 1; l < kLanes; ++l)
        if (load[l] < load[best]) best = l;
    lane[k] = best;
    load[best] += cost[k] + 1;
  }
  return lane;
}

// Forks the batch's streams from s (they wait for everything enqueued on s
// so far), or joins them back into s.
hipError_t fork_lanes(fppr_batch* b, hipStream_t s) {
  hipError_t e = hipEventRecord(b->fork, s);
  for (int a = 0; a < kLanes - 1 && e == hipSuccess; ++a) e = hipStreamWaitEvent(b->aux[a], b->fork, 0);
  return e;
}
hipError_t join_lanes(fppr_batch* b, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int a = 0; a < kLanes - 1 && e == hipSuccess; ++a) {
    e = hipEventRecord(b->join[a], b->aux[a]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[a], 0);
  }
  return e;
}

fppr_status enqueue(fppr_batch* b, fppr_stats* stats, fppr_profile* prof, hipStream_t s) {
  auto lane = [&](int l) { return l == 0 ? s : b->aux[l - 1]; };
  hipError_t e;
  if (b->opts.flags & FPPR_BATCH_REBUILD) {
    if ((e = fork_lanes(b, s)) != hipSuccess) return hip_fail(e, "fork streams");
    for (size_t k = 0; k < b->graphs.size(); ++k) {
      const fppr_status st = fppr_graph_rebuild(b->graphs[k], lane(b->graph_lane[k]));
      if (st != FPPR_OK) return st;
    }
    if ((e = join_lanes(b, s)) != hipSuccess) return hip_fail(e, "join streams");
  }
  e = launch_zero_u64(reinterpret_cast<uint64_t*>(b->ctl), kCtlBytes / 8, s);
  if (e != hipSuccess) return hip_fail(e, "zero control words");
  if (prof && (e = hipEventRecord(prof->ev[0], s)) != hipSuccess) return hip_fail(e, "event");
  const uint32_t nt = static_cast<uint32_t>(b->host_table.size());
  e = launch_walk(b->table, b->host_table.data(), nt, b->total, b->ctl, stats, b->opts.blocks_per_cu, s);
  if (e != hipSuccess) return hip_fail(e, "walk kernel");
  if (prof && (e = hipEventRecord(prof->ev[4], s)) != hipSuccess) return hip_fail(e, "event");
  if (prof && (e = hipEventRecord(prof->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
  if (prof && (e = hipEventRecord(prof->ev[2], s)) != hipSuccess) return hip_fail(e, "event");
  if ((e = fork_lanes(b, s)) != hipSuccess) return hip_fail(e, "fork streams");
  for (size_t k = 0; k < b->items.size(); ++k) {
    const fppr_batch_item& it = b->items[k];
    if (b->split[k]) {
      if ((e = launch_dangling(it.graph, &it.params, b->endpoints[k], stats, lane(b->item_lane[k]))) != hipSuccess)
        return hip_fail(e, "dangling walks");
    }
    AggLaunch a = make_agg(&it.params, b->endpoints[k], it.sources, item_sources(it), &it.out);
    a.table = b->agg_table;
    if (a.topk || a.counts || a.digest) {
      if ((e = launch_aggregate(a, lane(b->item_lane[k]))) != hipSuccess) return hip_fail(e, "aggregate kernel");
    }
  }
  if ((e = join_lanes(b, s)) != hipSuccess) return hip_fail(e, "join streams");
  if (prof && (e = hipEventRecord(prof->ev[3], s)) != hipSuccess) return hip_fail(e, "event");
  return FPPR_OK;
}

}  // namespace

extern "C" {

FPPR_API fppr_status fppr_batch_plan(const fppr_batch_item* items, uint32_t count,
                                     uint64_t* workspace_bytes) {
  fppr_status st = check_items(items, count);
  if (st != FPPR_OK) return st;
  if (!workspace_bytes) return invalid("workspace_bytes is NULL");
  *workspace_bytes = batch_layout(shapes(items, count), sizeof(WalkDesc), kWalkChunk).bytes;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_create(const fppr_batch_item* items, uint32_t count,
                                       const fppr_batch_opts* opts, void* workspace,
                                       uint64_t workspace_bytes, fppr_batch** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  uint64_t need = 0;
  fppr_status st = fppr_batch_plan(items, count, &need);
  if (st != FPPR_OK) return st;
  if (!workspace || workspace_bytes < need) return invalid("workspace missing or smaller than fppr_batch_plan");
  if (opts && (opts->flags & ~static_cast<uint32_t>(FPPR_BATCH_REBUILD))) return invalid("unknown batch flag bits");
  auto* b = new fppr_batch();
  b->items.assign(items, items + count);
  if (opts) b->opts = *opts;
  for (uint32_t k = 0; k < count; ++k)
    if (std::find(b->graphs.begin(), b->graphs.end(), items[k].graph) == b->graphs.end())
      b->graphs.push_back(items[k].graph);
  // Largest items first in the walk table, so that small ones fill the tail
  // of the launch. An item over all nodes of its graph walks only from the
  // nodes with out-edges in the walk launch (endpoints placed by source id);
  // the walks from the other nodes only restart at their source and run in a
  // coin-only kernel before the item's counting. Draws and results are
  // unchanged.
  const std::vector<BatchItemShape> sh = shapes(items, count);
  const BatchLayout lay = batch_layout(sh, sizeof(WalkDesc), kWalkChunk);
  char* base = static_cast<char*>(workspace);
  b->ctl = reinterpret_cast<unsigned long long*>(base + lay.ctl);
  b->table = reinterpret_cast<WalkDesc*>(base + lay.table);
  b->agg_table = reinterpret_cast<uint64_t*>(base + lay.agg_table);
  b->endpoints.resize(count);
  b->split.assign(count, false);
  for (uint32_t k = 0; k < count; ++k) {
    b->endpoints[k] = reinterpret_cast<uint32_t*>(base + lay.endpoints[k]);
    b->split[k] = sh[k].split;
  }
  for (const BatchRun& r : lay.runs) {
    const fppr_batch_item& it = items[r.item];
    WalkDesc D = b->split[r.item]
                     ? make_desc(it.graph, &it.params, it.graph->live, it.graph->n_live, b->endpoints[r.item],
                                 r.first, 0, r.count)
                     : make_desc(it.graph, &it.params, it.sources, item_sources(it), b->endpoints[r.item],
                                 r.first, 0, r.count);
    if (b->split[r.item]) D.flags |= kDescEpBySource;
    b->host_table.push_back(D);
  }
  b->total = lay.total;
  b->runs = lay.runs;
  {
    std::vector<uint64_t> gcost(b->graphs.size());
    std::vector<bool> gpin(b->graphs.size(), false);
    for (size_t k = 0; k < b->graphs.size(); ++k) gcost[k] = b->graphs[k]->m + b->graphs[k]->n;
    b->graph_lane = assign_lanes(gcost, gpin);
    std::vector<uint64_t> icost(count);
    std::vector<bool> ipin(count);
    for (uint32_t k = 0; k < count; ++k) {
      icost[k] = item_sources(items[k]) * items[k].params.R;
      ipin[k] = agg_uses_table(items[k].params.R, (items[k].params.flags & FPPR_COUNTS) != 0);
    }
    b->item_lane = assign_lanes(icost, ipin);
  }
  {
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    for (int a = 0; a < kLanes - 1 && e == hipSuccess; ++a) {
      e = hipStreamCreateWithFlags(&b->aux[a], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[a], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "batch streams");
    }
  }
  if (!b->host_table.empty()) {
    hipError_t e = hipMemcpy(b->table, b->host_table.data(), b->host_table.size() * sizeof(WalkDesc),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "upload walk table");
    }
  }
  *out = b;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_run(fppr_batch* b, fppr_stats* stats, fppr_profile* profile,
                                    void* stream) {
  if (!b) return invalid("batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const fppr_status st = enqueue(b, stats, profile, s);
  if (st != FPPR_OK) return st;
  const hipError_t e = hipEventRecord(b->done, s);
  return e == hipSuccess ? FPPR_OK : hip_fail(e, "event");
}

FPPR_API fppr_status fppr_batch_capture(fppr_batch* b, fppr_stats* stats, void* stream) {
  if (!b) return invalid("batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!s) return invalid("capture needs a non-null stream");
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  fppr_status st = enqueue(b, stats, nullptr, s);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (st != FPPR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_launch(fppr_batch* b, void* stream) {
  if (!b) return invalid("batch is NULL");
  if (!b->exec) return invalid("no captured graph (fppr_batch_capture)");
  hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  if ((e = hipEventRecord(b->done, static_cast<hipStream_t>(stream))) != hipSuccess) return hip_fail(e, "event");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_check(fppr_batch* b, void* stream) {
  if (!b) return invalid("batch is NULL");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "sync");
  unsigned long long ctl[2];
  e = hipMemcpy(ctl, b->ctl, sizeof ctl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read batch status");
  if (ctl[1] & 2) return invalid("a walk met guide tables that did not resolve its pick (rebuild the graph)");
  if (ctl[1]) return invalid("a source id was >= n (its walks were skipped)");
  if (b->opts.flags & FPPR_BATCH_REBUILD) {
    for (size_t k = 0; k < b->graphs.size(); ++k) {
      if (fppr_graph_check(b->graphs[k], stream) != FPPR_OK)
        return invalid("graph " + std::to_string(k) + " of the batch failed its rebuild: " + fppr_last_error());
    }
  }
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_manifest(const fppr_batch* b, char* json, size_t cap, size_t* needed) {
  if (!b || !needed) return invalid("batch or needed is NULL");
  std::string j = "{\"launch_blocks_per_cu\": " + std::to_string(b->opts.blocks_per_cu) +
                  ", \"rebuild\": " + ((b->opts.flags & FPPR_BATCH_REBUILD) ? "true" : "false") +
                  ", \"walk_ids\": " + std::to_string(b->total) + ", \"items\": [";
  char num[64];
  auto dbl = [&](double v) {
    std::snprintf(num, sizeof num, "%.17g", v);
    return std::string(num);
  };
  for (size_t k = 0; k < b->items.size(); ++k) {
    const fppr_batch_item& it = b->items[k];
    const fppr_graph* g = it.graph;
    const fppr_params& p = it.params;
    uint64_t first = 0, walks = 0;
    for (const BatchRun& r : b->runs)
      if (r.item == k) {
        first = r.first;
        walks = r.count;
      }
    std::string pool = "null";
    if (g->has_pool)
      pool = "{\"S\": " + std::to_string(g->pool_opts.S) + ", \"L\": " + std::to_string(g->pool_opts.L) +
             ", \"K\": " + std::to_string(g->pool_opts.K) + ", \"seed\": " + std::to_string(g->pool_opts.seed) +
             ", \"alpha\": " + dbl(g->pool_opts.alpha) + ", \"small_nodes\": " + std::to_string(g->n_small) + "}";
    j += std::string(k ? ", " : "") + "{\"item\": " + std::to_string(k) + ", \"graph\": {\"n\": " +
         std::to_string(g->n) + ", \"m\": " + std::to_string(g->m) + ", \"layout\": \"" +
         (g->guide ? "guide" : (g->narrow ? "narrow" : "wide")) + "\", \"hub_threshold\": " + std::to_string(g->tree_min) +
         ", \"tree_rows\": " + std::to_string(g->n_tree) + ", \"pool\": " + pool +
         "}, \"alpha\": " + dbl(p.alpha) + ", \"R\": " + std::to_string(p.R) +
         ", \"seed\": " + std::to_string(p.seed) + ", \"topk\": " + std::to_string(p.topk) +
         ", \"stitch\": " + ((p.flags & FPPR_STITCH) ? "true" : "false") +
         ", \"flags\": " + std::to_string(p.flags) + ", \"sources\": " + std::to_string(item_sources(it)) +
         ", \"all_nodes\": " + (it.sources ? "false" : "true") +
         ", \"coin_only_split\": " + (b->split[k] ? "true" : "false") +
         ", \"first_walk_id\": " + std::to_string(first) + ", \"launch_walks\": " + std::to_string(walks) +
         ", \"counting_stream\": " + std::to_string(b->item_lane[k]) + "}";
  }
  j += "]}";
  *needed = j.size() + 1;
  if (!json) return FPPR_OK;
  if (cap < *needed) return invalid("manifest buffer too small (see *needed)");
  std::memcpy(json, j.c_str(), j.size() + 1);
  return FPPR_OK;
}

FPPR_API fppr_status fppr_batch_destroy(fppr_batch* b) {
  free_batch(b);
  return FPPR_OK;
}

}  // extern "C"
