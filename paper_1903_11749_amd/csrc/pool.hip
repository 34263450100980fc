// Short-walk pool for small nodes (Sec. 4.2, "big moves").
//
// The paper expands, for every small node, the exact distribution of walks of
// up to k steps, each outcome marked terminated or active (Algorithm 4), and
// a walk at a small node draws one outcome (Sec. 4.2, last paragraph). Here a
// small node (1 <= out-degree <= S) keeps K sampled walks of at most L plain
// steps with the same marks, so a walk at a small node takes one pool entry
// with a single 8-byte load. Entry: end | steps << 32 | mark << 48
// (mark 1 = terminated). A pool walk stops on its coin (terminated), after L
// steps, or on arriving at a node without out-neighbours (active: the restart
// to the walk's own head is taken by the walk's next move).
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;

uint32_t grid_for(uint64_t items) {
  uint64_t b = (items + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<uint32_t>(b);
}

__global__ void k_small_flags(const uint64_t* __restrict__ off, uint32_t n, uint32_t S,
                              uint32_t* flag) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t deg = off[u + 1] - off[u];
    flag[u] = (deg >= 1 && deg <= S) ? 1u : 0u;
  }
}

// small_nodes[rank] = u and the stitched node-line table: small nodes point
// at their pool block (absolute address), every other node keeps its plain
// line. Eight lanes copy one 128-byte line, 16 bytes each.
__global__ void k_small_compact(const uint32_t* __restrict__ flag,
                                const uint64_t* __restrict__ rank, const Block* __restrict__ rec,
                                uint32_t n, uint32_t K_log2, uint64_t cap, const uint64_t* pool,
                                uint32_t* __restrict__ small_nodes, Block* __restrict__ rec_st,
                                uint32_t* err) {
  const uint64_t total = static_cast<uint64_t>(n) * 8;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t u = t >> 3;
    const uint32_t part = static_cast<uint32_t>(t & 7);
    ulonglong2 v = reinterpret_cast<const ulonglong2*>(rec + u)[part];
    if (part == 0 && flag[u]) {
      const uint64_t k = rank[u];
      if (k >= cap) {
        atomicOr(err, kErrCapacity);
      } else {
        small_nodes[k] = static_cast<uint32_t>(u);
        // the stitched line carries the address of the node's first entry
        v.x = reinterpret_cast<uint64_t>(pool + (k << K_log2));
        v.y |= kPoolFlag;
      }
    }
    reinterpret_cast<ulonglong2*>(rec_st + u)[part] = v;
  }
}

// One thread per (small node rank, slot j).
__global__ void __launch_bounds__(kThreads) k_pool(GraphView g, const uint32_t* __restrict__ small_nodes,
                                                   uint64_t n_small, uint32_t K_log2, uint32_t L,
                                                   uint32_t T, uint32_t key0, uint32_t key1,
                                                   uint64_t* __restrict__ pool) {
  const uint64_t total = n_small << K_log2;
  for (uint64_t idx = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t j = static_cast<uint32_t>(idx & ((1ull << K_log2) - 1));
    const uint32_t v = small_nodes[idx >> K_log2];
    uint32_t cur = v, steps = 0, mark = 0;
    for (uint32_t t = 0; t < L; ++t) {
      const Block& ln = g.rec[cur];
      const uint64_t od = ln.key[1];
      const uint32_t deg = static_cast<uint32_t>(od & kDegMask);
      if (deg == 0) break;  // arrived at a node without out-edges: stays active
      const U4 x = philox10(j, t, v, 1u, key0, key1);
      const uint64_t X = scaled_draw(x.x0, x.x1, ln.key[0]);
      cur = pick_blocking(g, ln, od >> kRegionShift, deg, X);
      steps += 1;
      if (x.x2 < T) {
        mark = 1;
        break;
      }
    }
    pool[idx] = static_cast<uint64_t>(cur) | (static_cast<uint64_t>(steps) << 32) |
                (static_cast<uint64_t>(mark) << 48);
  }
}

}  // namespace

hipError_t launch_small_flags(fppr_graph* g, uint32_t S, hipStream_t s) {
  hipLaunchKernelGGL(k_small_flags, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, S,
                     g->flag);
  return launch_scan_u32(g->flag, g->scan, g->n, g->scan_blocks,
                         reinterpret_cast<uint64_t*>(g->d_err + 6), s);
}

hipError_t launch_small_compact(fppr_graph* g, uint32_t /*S*/, hipStream_t s) {
  hipLaunchKernelGGL(k_small_compact, dim3(grid_for(static_cast<uint64_t>(g->n) * 8)), dim3(kThreads), 0, s,
                     g->flag, g->scan,
                     g->rec, g->n, g->K_log2, g->n_small, g->pool, g->small_nodes, g->rec_st,
                     g->d_err);
  return hipGetLastError();
}

hipError_t launch_pool(fppr_graph* g, hipStream_t s) {
  const uint64_t total = g->n_small << g->K_log2;
  if (total == 0) return hipSuccess;
  GraphView gv{g->rec, g->blocks, g->tree_min};
  const uint64_t seed = g->pool_opts.seed;
  hipLaunchKernelGGL(k_pool, dim3(grid_for(total)), dim3(kThreads), 0, s, gv, g->small_nodes,
                     g->n_small, g->K_log2, g->pool_opts.L, g->pool_T,
                     static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), g->pool);
  return hipGetLastError();
}

}  // namespace fppr
