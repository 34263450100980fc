// Exact big-move tables of the small nodes (Sec. 4.2, Algorithm 4), one
// thread per node over a bounded set of workspace slots, and walks that take
// them with alias picks elsewhere (the paper's design). The per-node
// expansion, its fixed-point rules and its size cap are in big_moves_node.hpp.
#include "big_moves_node.hpp"
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kBmThreads = 64;

__global__ void k_big_moves(const uint64_t* __restrict__ off, const uint32_t* __restrict__ col,
                            const uint32_t* __restrict__ w, uint32_t n, uint32_t S, uint32_t T,
                            uint32_t d, uint32_t cap, uint64_t* __restrict__ ws, uint64_t slots,
                            uint64_t* __restrict__ entries, uint64_t* __restrict__ weights,
                            uint32_t* __restrict__ counts) {
  const uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  if (t >= slots) return;
  uint64_t* mine = ws + t * 8ull * cap;
  for (uint64_t v = t; v < n; v += slots) {
    const uint64_t deg = off[v + 1] - off[v];
    uint32_t c = 0;
    if (deg >= 1 && deg <= S)
      c = big_moves_node(off, col, w, static_cast<uint32_t>(v), T, d, cap, mine, entries + v * cap,
                         weights + v * cap);
    counts[v] = c;
  }
}

// Walks of the paper's design: at a node with 1 <= out-degree <= S the move
// takes one big move of the node's table (the first entry whose inclusive
// weight prefix exceeds X = high 64 bits of (x1:x0) * total weight, found by
// binary search; a terminated entry ends the walk at its end node, an active
// one continues there); at any other node with out-edges an alias pick with
// the same draw (as in k_walk_alias, one 16-byte slot), then the coin
// x2 < T; a node without out-edges sends the walk back to its source.
// Draws: Philox4x32-10 on (i, m, s, 0).
__global__ void k_walk_bm(const uint64_t* __restrict__ off, const uint32_t* __restrict__ col,
                          const Block* __restrict__ rec, const ulonglong2* __restrict__ slots,
                          const uint64_t* __restrict__ bm_e,
                          const uint64_t* __restrict__ bm_w, const uint32_t* __restrict__ bm_c,
                          uint32_t cap, uint32_t S, uint32_t n, const uint32_t* __restrict__ sources,
                          uint64_t n_src, uint32_t R, uint32_t T, uint32_t k0, uint32_t k1,
                          uint32_t* __restrict__ ep, uint32_t* __restrict__ steps) {
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
    uint32_t tail = s, len = 0, m = 0;
    for (;;) {
      const U4 x = philox10(i, m, s, 0u, k0, k1);
      const uint64_t D = (static_cast<uint64_t>(x.x1) << 32) | x.x0;
      const uint64_t a = off[tail];
      const uint64_t d = off[tail + 1] - a;
      bool stop = x.x2 < T;
      uint32_t c = 0;
      if (d >= 1 && d <= S) {
        c = bm_c[tail];
        if (c > cap) c = 0;  // not a table fppr_graph_big_moves wrote
      }
      if (d == 0) {
        tail = s;
        ++len;
      } else if (c) {
        const uint64_t* te = bm_e + static_cast<uint64_t>(tail) * cap;
        const uint64_t* tw = bm_w + static_cast<uint64_t>(tail) * cap;
        const uint64_t X = __umul64hi(D, tw[c - 1]);
        uint32_t lo = 0, hi = c - 1;  // first inclusive prefix above X
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (tw[mid] > X) hi = mid;
          else lo = mid + 1;
        }
        const uint64_t e = te[lo];
        const uint32_t t = static_cast<uint32_t>(e);
        tail = t < n ? t : s;
        len += static_cast<uint32_t>((e >> 32) & 0xFFFFu);
        stop = ((e >> 48) & 1u) != 0;
      } else {
        const uint64_t W = rec[tail].key[0];
        const uint64_t X = scaled_draw(x.x0, x.x1, d * W);
        uint64_t slot = W ? X / W : 0;
        if (slot >= d) slot = d - 1;
        const uint64_t U = X - slot * W;
        const ulonglong2 q = slots[a + slot];
        const uint32_t t = U < q.x ? static_cast<uint32_t>(q.y) : static_cast<uint32_t>(q.y >> 32);
        tail = t < n ? t : s;
        ++len;
      }
      ++m;
      if (stop || m == kMoveCap) break;
    }
    ep[wid] = tail;
    if (steps) steps[wid] = len;
  }
}

fppr_status bm_invalid(const char* msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

}  // namespace

}  // namespace fppr

using namespace fppr;

FPPR_API fppr_status fppr_graph_big_moves(const fppr_graph* g, uint32_t S, uint32_t d, uint32_t cap,
                                          double alpha, uint64_t* entries, uint64_t* weights,
                                          uint32_t* counts, uint64_t* scratch, uint64_t scratch_words,
                                          void* stream) {
  if (!g) return bm_invalid("graph is NULL");
  if (!g->narrow) return bm_invalid("big-move tables need a graph with the narrow layout (32-bit row totals)");
  if (!entries || !weights || !counts || !scratch) return bm_invalid("an output or the scratch is NULL");
  const uint32_t T = fppr_alpha_threshold(alpha);
  if (T == 0) return bm_invalid("alpha must be in (0, 1)");
  if (S == 0 || d == 0) return bm_invalid("S and d must be at least 1");
  if (cap < 2ull * S || cap > 4096) return bm_invalid("cap must be in [2 S, 4096]");
  uint64_t slots = scratch_words / (8ull * cap);
  if (slots == 0) return bm_invalid("scratch must hold at least 8 * cap words");
  if (slots > g->n) slots = g->n;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t blocks = (slots + kBmThreads - 1) / kBmThreads;
  k_big_moves<<<static_cast<uint32_t>(blocks), kBmThreads, 0, s>>>(g->off, g->col, g->w, g->n, S, T, d,
                                                                    cap, scratch, slots, entries, weights,
                                                                    counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "big-move tables");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_run_big_moves(const fppr_graph* g, const uint64_t* slots,
                                        const uint64_t* bm_entries, const uint64_t* bm_weights,
                                        const uint32_t* bm_counts, uint32_t cap, uint32_t S, double alpha,
                                        uint32_t R, uint64_t seed, const uint32_t* sources,
                                        uint64_t n_sources, uint32_t* endpoints, uint32_t* steps,
                                        void* stream) {
  if (!g) return bm_invalid("graph is NULL");
  if (!g->narrow) return bm_invalid("these walks need a graph with the narrow layout (32-bit row totals)");
  if (!slots || !bm_entries || !bm_weights || !bm_counts || !endpoints)
    return bm_invalid("a table or the endpoints is NULL");
  if (reinterpret_cast<uintptr_t>(slots) % 16) return bm_invalid("slots must be 16-byte aligned");
  const uint32_t T = fppr_alpha_threshold(alpha);
  if (T == 0) return bm_invalid("alpha must be in (0, 1)");
  if (R == 0) return bm_invalid("R must be at least 1");
  if (cap == 0 || cap > 4096) return bm_invalid("cap must be in [1, 4096]");
  if (!sources && n_sources != g->n) return bm_invalid("without a source list n_sources must be n");
  if (n_sources == 0) return FPPR_OK;
  if (n_sources > (uint64_t(1) << 40) / R) return bm_invalid("n_sources * R exceeds 2^40");
  const uint64_t total = n_sources * R;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipStream_t s = static_cast<hipStream_t>(stream);
  k_walk_bm<<<static_cast<uint32_t>(blocks), 256, 0, s>>>(
      g->off, g->col, g->rec, reinterpret_cast<const ulonglong2*>(slots), bm_entries, bm_weights, bm_counts, cap, S, g->n, sources,
      n_sources, R, T, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), endpoints, steps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "big-move walks");
  return FPPR_OK;
}
