// Alias tables of every row (Sec. 2.2, Algorithm 1; Example 2), and walks
// that pick with them.
//
// For a row of n edges with integer weights w and total W the switch
// probability p(e) = n r(e) is kept as the integer P(e) = n w(e) in units of
// 1/W, so every transfer of Algorithm 1 is exact and no edge is left over
// by rounding. Algorithm 1 leaves the order of its transfers free; here the
// edges below W are filled oldest first by the earliest edge still above W
// (both kept as FIFO queues in edge order), and an edge that falls below W
// while giving joins the back of the fill queue (Example 2's printed tables
// follow from this order). A pick keeps slot i iff U < P(i), else takes
// alias(i).
//
// One thread per row: the loop is a dependent chain (each step may move the
// head of S^l), so a row cannot be split across lanes without changing the
// table. Queue capacities are fixed by construction: an edge enters S^s at
// most once (initially, or when it leaves S^l) and S^l only initially, so
// each queue fits in n slots of the caller's scratch.
#include "alias_row.hpp"
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;

__global__ void k_alias_rows(const uint64_t* __restrict__ off, const uint32_t* __restrict__ w,
                             uint32_t n_rows, uint64_t* __restrict__ P,
                             uint32_t* __restrict__ alias, uint32_t* __restrict__ scratch) {
  const uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  if (v >= n_rows) return;
  const uint64_t a = off[v];
  const uint64_t d = off[v + 1] - a;
  if (d == 0) return;
  alias_row(w + a, d, P + a, alias + a, scratch + 2 * a, scratch + 2 * a + d);
}

// Walks that pick with the alias tables (plain walks of Sec. 2.1: a move
// picks an out-edge, then stops with the coin; a node without out-edges
// sends the walk back to its source). One walk per thread; walk w is walk
// w mod R of source row w div R, its move m draws Philox4x32-10 on (w mod R,
// m, s, 0) as every other walk mode does. The pick: X = high 64 bits of
// (x1:x0) * (d W), slot = X div W, keep the slot iff X mod W < P[slot], else
// take alias[slot]. d W < 2^59 on narrow graphs, so X fits 64 bits. Each
// node is one 16-byte record (row start, total and degree) and each slot one
// 16-byte record (threshold and both destination ids), so a move reads two
// lines.
__global__ void k_walk_alias(const ulonglong2* __restrict__ nodes, const ulonglong2* __restrict__ slots,
                             uint64_t m, uint32_t n,
                             const uint32_t* __restrict__ sources, uint64_t n_src, uint32_t R,
                             uint32_t T, uint32_t k0, uint32_t k1, uint32_t* __restrict__ ep,
                             uint32_t* __restrict__ steps) {
  const uint64_t total = n_src * R;
  for (uint64_t wid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; wid < total;
       wid += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t row = wid / R;
    const uint32_t i = static_cast<uint32_t>(wid - row * R);
    const uint32_t s = sources ? sources[row] : static_cast<uint32_t>(row);
    if (s >= n) {
      ep[wid] = 0xFFFFFFFFu;
      if (steps) steps[wid] = 0;
      continue;
    }
    uint32_t tail = s, len = 0, mv = 0;
    for (;;) {
      const U4 x = philox10(i, mv, s, 0u, k0, k1);
      const ulonglong2 nd = nodes[tail];  // row start, total | degree << 32
      const uint64_t a = nd.x;
      uint64_t d = nd.y >> 32;
      if (a > m || d > m - a) d = 0;  // only with a node table from another graph
      if (d == 0) {
        tail = s;
      } else {
        const uint64_t W = static_cast<uint32_t>(nd.y);
        const uint64_t X = scaled_draw(x.x0, x.x1, d * W);
        uint64_t slot = W ? X / W : 0;
        if (slot >= d) slot = d - 1;  // only with tables or weights changed since the build
        const uint64_t U = X - slot * W;
        const ulonglong2 q = slots[a + slot];  // threshold, own id | alias's id << 32
        const uint32_t t = U < q.x ? static_cast<uint32_t>(q.y) : static_cast<uint32_t>(q.y >> 32);
        tail = t < n ? t : s;
      }
      ++len;
      ++mv;
      if (x.x2 < T || mv == kMoveCap) break;
    }
    ep[wid] = tail;
    if (steps) steps[wid] = len;
  }
}

// node v: {row start, W(v) | deg(v) << 32} (W < 2^32 on narrow graphs)
__global__ void k_alias_nodes(const uint64_t* __restrict__ off, const Block* __restrict__ rec,
                              uint32_t n, ulonglong2* __restrict__ nodes) {
  const uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  if (v >= n) return;
  const uint64_t a = off[v], d = off[v + 1] - a;
  const uint64_t W = d ? (rec[v].key[0] & 0xFFFFFFFFull) : 0;
  nodes[v] = make_ulonglong2(a, W | (d << 32));
}

// slot e of row v: {P[e], col[e] | col[alias[e]] << 32}. One wave per row
// (grid-stride over rows), its lanes striding the row's edges, so a hub's
// slots are written 64 at a time.
constexpr uint32_t kSlotBlocks = 16384;

__global__ void k_alias_slots(const uint64_t* __restrict__ off, const uint32_t* __restrict__ col,
                              uint32_t n_rows, const uint64_t* __restrict__ P,
                              const uint32_t* __restrict__ alias, ulonglong2* __restrict__ slots) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  for (uint64_t v = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 6; v < n_rows;
       v += waves) {
    const uint64_t a = off[v];
    const uint64_t d = off[v + 1] - a;
    for (uint64_t i = lane; i < d; i += 64) {
      uint64_t j = alias[a + i];
      if (j >= d) j = i;
      slots[a + i] = make_ulonglong2(P[a + i], col[a + i] | (static_cast<uint64_t>(col[a + j]) << 32));
    }
  }
}

fppr_status invalid_arg(const char* msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

}  // namespace

}  // namespace fppr

using namespace fppr;

FPPR_API fppr_status fppr_graph_alias_tables(const fppr_graph* g, uint64_t* P, uint32_t* alias,
                                             uint32_t* scratch, void* stream) {
  if (!g) return invalid_arg("graph is NULL");
  if (g->m && (!P || !alias || !scratch)) return invalid_arg("P, alias or scratch is NULL");
  if (g->m == 0) return FPPR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t blocks = static_cast<uint32_t>((g->n + kThreads - 1) / kThreads);
  k_alias_rows<<<blocks, kThreads, 0, s>>>(g->off, g->w, g->n, P, alias, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "alias tables");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_alias_slots(const fppr_graph* g, const uint64_t* P, const uint32_t* alias,
                                            uint64_t* slots, void* stream) {
  if (!g) return invalid_arg("graph is NULL");
  if (g->m && (!P || !alias || !slots)) return invalid_arg("P, alias or slots is NULL");
  if (reinterpret_cast<uintptr_t>(slots) % 16) return invalid_arg("slots must be 16-byte aligned");
  if (g->m == 0) return FPPR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint64_t blocks = (static_cast<uint64_t>(g->n) * 64 + kThreads - 1) / kThreads;
  if (blocks > kSlotBlocks) blocks = kSlotBlocks;
  k_alias_slots<<<static_cast<uint32_t>(blocks), kThreads, 0, s>>>(g->off, g->col, g->n, P, alias,
                                                                    reinterpret_cast<ulonglong2*>(slots));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "alias slots");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_alias_nodes(const fppr_graph* g, uint64_t* nodes, void* stream) {
  if (!g) return invalid_arg("graph is NULL");
  if (!g->narrow) return invalid_arg("alias node records need the narrow layout (32-bit row totals)");
  if (!nodes) return invalid_arg("nodes is NULL");
  if (reinterpret_cast<uintptr_t>(nodes) % 16) return invalid_arg("nodes must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t blocks = static_cast<uint32_t>((g->n + kThreads - 1) / kThreads);
  k_alias_nodes<<<blocks, kThreads, 0, s>>>(g->off, g->rec, g->n, reinterpret_cast<ulonglong2*>(nodes));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "alias nodes");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_run_alias(const fppr_graph* g, const uint64_t* nodes, const uint64_t* slots,
                                    double alpha, uint32_t R, uint64_t seed, const uint32_t* sources,
                                    uint64_t n_sources, uint32_t* endpoints, uint32_t* steps, void* stream) {
  if (!g) return invalid_arg("graph is NULL");
  if (!g->narrow) return invalid_arg("alias walks need a graph with the narrow layout (32-bit row totals)");
  if (!nodes || !slots || !endpoints) return invalid_arg("nodes, slots or endpoints is NULL");
  if (reinterpret_cast<uintptr_t>(slots) % 16 || reinterpret_cast<uintptr_t>(nodes) % 16)
    return invalid_arg("nodes and slots must be 16-byte aligned");
  const uint32_t T = fppr_alpha_threshold(alpha);
  if (T == 0) return invalid_arg("alpha must be in (0, 1)");
  if (R == 0) return invalid_arg("R must be at least 1");
  if (!sources && n_sources != g->n) return invalid_arg("without a source list n_sources must be n");
  if (n_sources == 0) return FPPR_OK;
  if (n_sources > (uint64_t(1) << 40) / R) return invalid_arg("n_sources * R exceeds 2^40");
  const uint64_t total = n_sources * R;
  uint64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_walk_alias<<<static_cast<uint32_t>(blocks), kThreads, 0, s>>>(
      reinterpret_cast<const ulonglong2*>(nodes), reinterpret_cast<const ulonglong2*>(slots), g->m, g->n,
      sources, n_sources, R, T,
      static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), endpoints, steps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "alias walks");
  return FPPR_OK;
}
