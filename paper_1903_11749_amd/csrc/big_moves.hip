// Exact big-move tables of the small nodes (Sec. 4.2, Algorithm 4), one
// thread per node over a bounded set of workspace slots. The per-node
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
