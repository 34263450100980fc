// Short-walk pool for small nodes (Sec. 4.2, "big moves").
//
// The paper expands, for every small node, the exact distribution of walks of
// up to k steps, each outcome marked terminated or active (Algorithm 4), and
// a walk at a small node draws one outcome (Sec. 4.2, last paragraph). Here a
// small node (1 <= out-degree <= S) keeps K sampled walks of at most L plain
// steps with the same marks, so a walk at a small node takes one pool entry
// with a single 8-byte load. Entry: end | steps << 32 | mark << 48
// (mark 1 = terminated; in tagged graphs the end id carries its class tag).
// Node v's entries sit at v * K, so a walk that knows v is small (from the
// tag of the edge it arrived over) reads its entry without v's node line.
// A pool walk stops on its coin (terminated), after L steps, or on arriving
// at a node without out-neighbours (active: the restart to the walk's own
// head is taken by the walk's next move).
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

// small_nodes[rank] = u: the small nodes in id order (the pool kernel's work list)
__global__ void k_small_compact(const uint32_t* __restrict__ flag, const uint64_t* __restrict__ rank,
                                uint32_t n, uint64_t cap, uint32_t* __restrict__ small_nodes, uint32_t* err) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (!flag[u]) continue;
    const uint64_t k = rank[u];
    if (k >= cap) atomicOr(err, kErrCapacity);
    else small_nodes[k] = static_cast<uint32_t>(u);
  }
}

// canonical order for export: rank k's entries from node small_nodes[k]'s
// block, end ids without their tags
__global__ void k_pool_export(const uint64_t* __restrict__ pool, const uint32_t* __restrict__ small_nodes,
                              uint64_t n_small, uint32_t K_log2, bool tagged, uint64_t* __restrict__ out) {
  const uint64_t keep = tagged ? ~static_cast<uint64_t>(~kIdMask & 0xFFFFFFFFu) : ~0ull;
  const uint64_t total = n_small << K_log2;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t v = small_nodes[i >> K_log2];
    const uint64_t e = pool[(v << K_log2) + (i & ((1ull << K_log2) - 1))];
    out[i] = e & keep;
  }
}

// The value of the other lane of this lane's aligned pair (DPP quad
// permutation [1, 0, 3, 2]).
__device__ __forceinline__ uint32_t pair_swap(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ uint64_t pair_swap64(uint64_t x) {
  return static_cast<uint64_t>(pair_swap(static_cast<uint32_t>(x))) |
         (static_cast<uint64_t>(pair_swap(static_cast<uint32_t>(x >> 32))) << 32);
}
// keys of q that are <= X: two u64 keys (wide layout) or four u32 keys
// (narrow layout, where X < 2^32)
template <bool kNar>
__device__ __forceinline__ uint32_t count_q(uint4 q, uint64_t X) {
  if (kNar) {
    const uint32_t x = static_cast<uint32_t>(X);
    return (q.x <= x ? 1u : 0u) + (q.y <= x ? 1u : 0u) + (q.z <= x ? 1u : 0u) + (q.w <= x ? 1u : 0u);
  }
  const uint64_t k0 = (static_cast<uint64_t>(q.y) << 32) | q.x;
  const uint64_t k1 = (static_cast<uint64_t>(q.w) << 32) | q.z;
  return (k0 <= X ? 1u : 0u) + (k1 <= X ? 1u : 0u);
}

// A lane pair per (small node rank, slot j): both lanes follow the same pool
// walk, and each reads one half of every 128-byte line it needs (the even
// lane bytes 0..63, the odd lane bytes 64..127), adding the pair's compare
// counts with one DPP swap, so that no lane reads more than 64 bytes of a
// random line. The 64 slots of a small node sit in consecutive pairs, so
// their first steps read the same lines. kNar: the graph's layout.
template <bool kNar>
__global__ void __launch_bounds__(kThreads) k_pool(GraphView g, const uint32_t* __restrict__ small_nodes,
                                                   uint64_t n_small, uint32_t K_log2, uint32_t L,
                                                   uint32_t T, uint32_t key0, uint32_t key1, bool tagged,
                                                   uint64_t* __restrict__ pool) {
  const uint64_t total = n_small << K_log2;
  const uint32_t half = threadIdx.x & 1u;
  const uint64_t stride = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 1;
  for (uint64_t idx = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 1; idx < total;
       idx += stride) {
    const uint32_t j = static_cast<uint32_t>(idx & ((1ull << K_log2) - 1));
    const uint32_t v = small_nodes[idx >> K_log2];
    uint32_t cur = v, tag = 0, steps = 0, mark = 0;
    for (uint32_t t = 0; t < L; ++t) {
      if (tag == kTagDangling) break;  // arrived at a node without out-edges: stays active, no load
      // node line: weight and flags (even lane's first 16 bytes) and top keys
      const uint4* ln = reinterpret_cast<const uint4*>(g.rec + cur) + half * 4;
      const uint4 q0 = ln[0], q1 = ln[1], q2 = ln[2], q3 = ln[3];
      const uint64_t W0 = (static_cast<uint64_t>(q0.y) << 32) | q0.x;
      const uint64_t od0 = (static_cast<uint64_t>(q0.w) << 32) | q0.z;
      const uint64_t Wp = pair_swap64(W0), odp = pair_swap64(od0);
      const uint64_t W = half ? Wp : W0, od = half ? odp : od0;
      const uint32_t deg = static_cast<uint32_t>(od & kDegMask);
      if (deg == 0) break;  // arrived at a node without out-edges: stays active
      const U4 x = philox10(j, t, v, 1u, key0, key1);
      const uint64_t X = scaled_draw(x.x0, x.x1, W);
      const uint64_t region = od >> kRegionShift;
      uint64_t leaf;
      if (deg > g.tree_min) {
        uint32_t c = half ? count_q<kNar>(q0, X) + count_q<kNar>(q1, X) + count_q<kNar>(q2, X) +
                                count_q<kNar>(q3, X)
                          : count_q<kNar>(q1, X) + count_q<kNar>(q2, X) + count_q<kNar>(q3, X);
        c += pair_swap(c);
        uint64_t base = 0, b = c;
        for (uint32_t l = tree_levels(deg, kNar) - 1; l >= 1; --l) {
          const uint4* nd = reinterpret_cast<const uint4*>(g.blocks + region + base + b) + half * 4;
          uint32_t cc = count_q<kNar>(nd[0], X) + count_q<kNar>(nd[1], X) + count_q<kNar>(nd[2], X) +
                        count_q<kNar>(nd[3], X);
          cc += pair_swap(cc);
          base += tree_level_nodes(deg, l, kNar);
          b = (b << node_shift(kNar)) + cc;
        }
        leaf = region + base + b;
      } else {
        uint64_t lo = 0, hi = leaf_blocks(deg, kNar) - 1;
        while (lo < hi) {
          const uint64_t mid = lo + ((hi - lo) >> 1);
          const uint64_t last = kNar ? g.blocks[region + mid].w32[kNarrowLeafEdges - 1]
                                     : g.blocks[region + mid].lf.p[kLeafEdges - 1];
          if (last > X) hi = mid; else lo = mid + 1;
        }
        leaf = region + lo;
      }
      // leaf block: the even lane counts the prefixes (8 or 16), the odd
      // lane holds the destinations
      const uint4* lf = reinterpret_cast<const uint4*>(g.blocks + leaf) + half * 4;
      uint32_t e = 0, dst = 0;
      const uint4 l0 = lf[0], l1 = lf[1], l2 = lf[2], l3 = lf[3];
      if (half == 0) {
        e = count_q<kNar>(l0, X) + count_q<kNar>(l1, X) + count_q<kNar>(l2, X) + count_q<kNar>(l3, X);
      }
      e += pair_swap(e);
      if (half) {
        const uint32_t qi = e >> 2;
        const uint4 w = qi == 0 ? l0 : (qi == 1 ? l1 : (qi == 2 ? l2 : l3));
        const uint32_t k = e & 3u;
        dst = k == 0 ? w.x : (k == 1 ? w.y : (k == 2 ? w.z : w.w));
      }
      dst += pair_swap(dst);
      cur = tagged ? dst & kIdMask : dst;
      tag = tagged ? dst >> kTagShift : 0u;
      steps += 1;
      if (x.x2 < T) {
        mark = 1;
        break;
      }
    }
    if (half == 0)
      pool[(static_cast<uint64_t>(v) << K_log2) + j] = static_cast<uint64_t>(cur | (tag << kTagShift)) |
                                                      (static_cast<uint64_t>(steps) << 32) |
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
  hipLaunchKernelGGL(k_small_compact, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->flag, g->scan, g->n,
                     g->n_small, g->small_nodes, g->d_err);
  return hipGetLastError();
}

hipError_t launch_pool_export(const fppr_graph* g, uint64_t* out, hipStream_t s) {
  const uint64_t total = g->n_small << g->K_log2;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_export, dim3(grid_for(total)), dim3(kThreads), 0, s, g->pool, g->small_nodes,
                     g->n_small, g->K_log2, g->tagged, out);
  return hipGetLastError();
}

hipError_t launch_pool(fppr_graph* g, hipStream_t s) {
  const uint64_t total = g->n_small << g->K_log2;
  if (total == 0) return hipSuccess;
  GraphView gv{g->rec, g->blocks, g->tree_min};
  const uint64_t seed = g->pool_opts.seed;
  if (g->narrow)
    hipLaunchKernelGGL(k_pool<true>, dim3(grid_for(total * 2)), dim3(kThreads), 0, s, gv, g->small_nodes,
                       g->n_small, g->K_log2, g->pool_opts.L, g->pool_T,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), g->tagged, g->pool);
  else
    hipLaunchKernelGGL(k_pool<false>, dim3(grid_for(total * 2)), dim3(kThreads), 0, s, gv, g->small_nodes,
                       g->n_small, g->K_log2, g->pool_opts.L, g->pool_T,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), g->tagged, g->pool);
  return hipGetLastError();
}

}  // namespace fppr
