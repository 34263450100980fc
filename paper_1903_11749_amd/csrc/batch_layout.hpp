// Layout of a batch: where the control words, the walk table, the shared
// counting tables and each item's endpoint buffer sit in the caller's
// workspace, and which runs of walk ids the walk table holds (largest item
// first, each padded to whole chunks). Host code only, shared by
// fppr_batch_plan / fppr_batch_create and a host-side bounds check.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "agg_hash.hpp"

namespace fppr {

struct BatchItemShape {
  uint64_t n_rows;  // source rows of the item (all nodes: n)
  uint32_t R;
  bool counts;      // per-source counts wanted (FPPR_COUNTS)
  bool split;       // all-nodes item: the walk launch takes only the nodes
                    // with out-edges, a coin-only kernel the others
  uint64_t n_live;  // nodes with out-edges (rows of the walk launch when split)
};

struct BatchRun {
  uint32_t item;
  uint64_t first;  // first walk id of the run in the launch (a multiple of the chunk)
  uint64_t count;  // walks
};

struct BatchLayout {
  uint64_t ctl = 0;                      // byte offsets in the workspace
  uint64_t table = 0;
  uint64_t agg_table = 0, agg_bytes = 0; // counting tables shared by the items that use them
  std::vector<uint64_t> endpoints;       // per item: offset and bytes of its endpoint buffer
  std::vector<uint64_t> endpoint_bytes;
  std::vector<BatchRun> runs;            // the walk table, largest item first
  uint64_t total = 0;                    // padded walk ids of the launch
  uint64_t bytes = 0;                    // workspace bytes
};

constexpr uint64_t kBatchAlign = 256;
constexpr uint64_t kBatchCtlBytes = 256;
inline uint64_t batch_align(uint64_t x) { return (x + kBatchAlign - 1) / kBatchAlign * kBatchAlign; }

inline BatchLayout batch_layout(const std::vector<BatchItemShape>& items, uint64_t desc_bytes, uint64_t chunk) {
  BatchLayout L;
  const size_t count = items.size();
  L.ctl = 0;
  L.table = kBatchCtlBytes;
  L.agg_table = L.table + batch_align(count * desc_bytes);
  for (const BatchItemShape& it : items) {  // items count one after the other: one table area serves all
    const uint64_t b = batch_align(agg_table_bytes(it.n_rows, it.R, it.counts));
    if (b > L.agg_bytes) L.agg_bytes = b;
  }
  uint64_t at = L.agg_table + L.agg_bytes;
  L.endpoints.resize(count);
  L.endpoint_bytes.resize(count);
  for (size_t k = 0; k < count; ++k) {
    L.endpoints[k] = at;
    L.endpoint_bytes[k] = batch_align(items[k].n_rows * items[k].R * 4ull);
    at += L.endpoint_bytes[k];
  }
  L.bytes = at;
  std::vector<uint32_t> order(count);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    return items[x].n_rows * items[x].R > items[y].n_rows * items[y].R;
  });
  uint64_t first = 0;
  for (uint32_t k : order) {
    const uint64_t walks = (items[k].split ? items[k].n_live : items[k].n_rows) * items[k].R;
    if (walks == 0) continue;
    L.runs.push_back(BatchRun{k, first, walks});
    first += (walks + chunk - 1) / chunk * chunk;
  }
  L.total = first;
  return L;
}

}  // namespace fppr
