// Alias tables of every row (Sec. 2.2, Algorithm 1; Example 2).
//
// For a row of n edges with integer weights w and total W the switch
// probability p(e) = n r(e) is kept as the integer P(e) = n w(e) in units of
// 1/W, so every update of Algorithm 1 is exact and no edge is left over by
// rounding. "Select any x in S^s and y in S^l" takes the first of each in
// insertion order: both sets are FIFO queues seeded in edge order, and an
// edge whose P drops below W joins the back of S^s (Example 2's printed
// tables follow from this choice). A pick keeps slot i iff U < P(i), else
// takes alias(i).
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
