// Graph ingest: CSR validation, per-row inclusive uint64 weight prefixes laid
// out with the destination ids (class-tagged in graphs of at most 2^30
// nodes) in 128-byte leaf blocks, 128-byte node lines and the rows' prefix
// trees (top level in the node line, 16-ary below), all in one pass over
// the edges.
//
// Routing probability r(s,t) = w(s,t) / sum_v w(s,v) (Sec. 2.1) is realised
// on exact integers: the prefix P of a row is strictly increasing (w >= 1),
// so "first prefix above X" picks edge j for exactly P[j] - P[j-1] of the W
// values of X. Large rows (Sec. 4.1, alias tree) are split recursively into
// groups whose running totals form the next level; descending the tree
// returns the same edge as a flat search (Lemma 1's telescoping product, on
// integers), with one 128-byte node per level.
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kShortRow = 64;  // rows up to this length: one thread each
static_assert(kShortRow / kLeafEdges <= kTopKeys && kShortRow / kNarrowLeafEdges <= kNarrowTopKeys,
              "a short row's tree is its top level alone");

// wave-wide maximum, then one atomic per wave
__device__ __forceinline__ void wave_atomic_max(uint32_t* dst, uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t t = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o, 64));
    v = t > v ? t : v;
  }
  if (__lane_id() == 0 && v) atomicMax(dst, v);
}
// (max_deg / max_w may be NULL: rebuilds keep the layout and skip them)

// Also the largest out-degree (for the layout choice).
__global__ void k_validate_offsets(const uint64_t* __restrict__ off, uint32_t n, uint64_t m,
                                   uint32_t* err, uint32_t* max_deg) {
  uint32_t dmax = 0;
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u], b = off[u + 1];
    uint32_t e = 0;
    if (b < a) e |= kErrOffsets;
    else if (b - a > 0xFFFFFFFFull) e |= kErrDegree;
    else if (b - a > dmax) dmax = static_cast<uint32_t>(b - a);
    if (u == 0 && a != 0) e |= kErrOffsets;
    if (u == n - 1 && b != m) e |= kErrOffsets;
    if (e) atomicOr(err, e);
  }
  if (max_deg) wave_atomic_max(max_deg, dmax);
}

// Also the largest weight (for the layout choice).
__global__ void k_validate_edges(const uint32_t* __restrict__ col, const uint32_t* __restrict__ w,
                                 uint64_t m, uint32_t n, uint32_t* err, uint32_t* max_w) {
  uint32_t e = 0, wmax = 0;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (col[i] >= n) e |= kErrCol;
    const uint32_t wi = w[i];
    if (wi == 0) e |= kErrWeight;
    wmax = wi > wmax ? wi : wmax;
  }
  if (e) atomicOr(err, e);
  if (max_w) wave_atomic_max(max_w, wmax);
}

// Region size (blocks) of every row, the input of the region-offset scan.
__global__ void k_region_sizes(const uint64_t* __restrict__ off, uint32_t n, uint32_t tree_min, bool nar,
                               uint32_t* __restrict__ flag) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t d = off[u + 1] - off[u];
    flag[u] = d <= kMaxDeg ? static_cast<uint32_t>(region_blocks(d, tree_min, nar)) : 0u;
  }
}

// Node line of u without its tree keys (all ~0 until the prefixes fill them in).
__device__ __forceinline__ void write_record(Block* rec, uint64_t u, uint64_t W, uint64_t region,
                                             uint64_t d) {
  const uint64_t od = (region << kRegionShift) | d;
  ulonglong2* dst = reinterpret_cast<ulonglong2*>(rec + u);
  dst[0] = make_ulonglong2(W, od);
#pragma unroll
  for (uint32_t k = 1; k < kNodeKeys / 2; ++k) dst[k] = make_ulonglong2(~0ull, ~0ull);
}

// Destination c of an edge of row u as a leaf stores it: with its class tag
// in tagged graphs. A rebuild validates the CSR on the device without
// waiting, so an id >= n can reach here; it is stored as u itself, so that
// no kernel ever reads a node line past n (the graph's check reports the
// invalid CSR, and its results mean nothing until it is fixed).
__device__ __forceinline__ uint32_t leaf_dest(const uint8_t* __restrict__ cls, uint32_t n, uint32_t c,
                                              uint64_t u) {
  if (c >= n) c = static_cast<uint32_t>(u);
  return cls ? c | (static_cast<uint32_t>(cls[c]) << kTagShift) : c;
}

// Edge j of a row (prefix P, destination c) into its leaf block, by layout;
// slots past the row's end get P = ~0.
__device__ __forceinline__ void put_edge(Block* leaves, uint64_t j, uint64_t P, uint32_t c, bool nar) {
  if (nar) {
    Block& b = leaves[j / kNarrowLeafEdges];
    b.w32[j % kNarrowLeafEdges] = static_cast<uint32_t>(P);
    b.w32[kNarrowLeafEdges + j % kNarrowLeafEdges] = c;
  } else {
    leaves[j / kLeafEdges].lf.p[j % kLeafEdges] = P;
    leaves[j / kLeafEdges].lf.c[j % kLeafEdges] = c;
  }
}
__device__ __forceinline__ void pad_edge(Block* leaves, uint64_t j, bool nar) {
  put_edge(leaves, j, nar ? 0xFFFFFFFFull : ~0ull, 0u, nar);
}
// key k of the top level into the node line, by layout
__device__ __forceinline__ void put_top(Block* line, uint64_t k, uint64_t P, bool nar) {
  if (nar) line->w32[kNarrowTopKey0 + k] = static_cast<uint32_t>(P);
  else line->key[kTopKey0 + k] = P;
}
// slot t of a tree node, by layout
__device__ __forceinline__ void put_key(Block* nd, uint64_t t, uint64_t P, bool nar) {
  if (nar) nd->w32[t] = static_cast<uint32_t>(P);
  else nd->key[t] = P;
}

// Short rows: one thread accumulates its row into its leaf blocks and writes
// its node line (kNar: the graph's layout). Long rows are queued for a block each. Rows with a tree are
// counted when n_tree_rows is given (one atomic per wave; the count depends
// only on the degrees and the threshold, so rebuilds skip it).
template <bool nar>
__global__ void k_leaves_short(const uint64_t* __restrict__ off, const uint32_t* __restrict__ col,
                               const uint32_t* __restrict__ w, const uint64_t* __restrict__ region,
                               const uint8_t* __restrict__ cls, uint32_t n, uint32_t tree_min, uint64_t cap,
                               Block* __restrict__ blk, Block* __restrict__ rec, uint32_t* rows,
                               uint32_t* n_rows, uint32_t* n_tree_rows, uint32_t* err) {
  uint64_t trees = 0;
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u];
    const uint64_t d = off[u + 1] - a;
    const uint64_t r0 = region[u];
    const bool fits = d <= kMaxDeg && r0 + region_blocks(d, tree_min, nar) <= cap;
    // long rows to the queue: one atomic per wave, each lane at its rank
    const bool long_row = fits && d > kShortRow;
    const uint64_t lm = __ballot(long_row);
    if (lm) {
      const int leader = __builtin_ctzll(lm);
      uint32_t base = 0;
      if (static_cast<int>(__lane_id()) == leader) base = atomicAdd(n_rows, static_cast<uint32_t>(__popcll(lm)));
      base = static_cast<uint32_t>(__shfl(static_cast<int>(base), leader, 64));
      if (long_row) rows[base + mask_rank(lm)] = static_cast<uint32_t>(u);
    }
    if (d > kMaxDeg) {
      atomicOr(err, kErrDegree);
      continue;
    }
    trees += d > tree_min ? 1u : 0u;
    if (!fits) {
      atomicOr(err, kErrCapacity);
      continue;
    }
    if (d == 0) {
      write_record(rec, u, 0, r0, 0);
      continue;
    }
    if (long_row) continue;
    Block* leaves = blk + r0 + tree_nodes(d, tree_min, nar);
    // a row this short that has a tree has only its top level (at most 8
    // keys, the leaf blocks' last prefixes): it goes into the node line here
    write_record(rec, u, 0, r0, d);
    const bool tree = d > tree_min;
    const uint64_t E = 1ull << leaf_shift(nar);
    uint64_t acc = 0;
    for (uint64_t j = 0; j < d; ++j) {
      acc += w[a + j];
      put_edge(leaves, j, acc, leaf_dest(cls, n, col[a + j], u), nar);
      if (tree && ((j % E) == E - 1 || j == d - 1)) put_top(rec + u, j / E, acc, nar);
    }
    for (uint64_t j = d; j < leaf_blocks(d, nar) * E; ++j) pad_edge(leaves, j, nar);
    if (nar && acc > 0xFFFFFFFFull) atomicOr(err, kErrNarrow);
    rec[u].key[0] = acc;
  }
  if (n_tree_rows) {
    trees = wave_sum_u64(trees);
    if (__lane_id() == 0 && trees) atomicAdd(n_tree_rows, static_cast<uint32_t>(trees));
  }
}

// Puts prefix P = P[j] of a row with a tree (d edges, L levels, T region tree
// nodes) into every level whose key ends at edge j: key k of level l is
// P[min((k+1) * E * F^(l-1), d) - 1]. The top level goes to the node line
// (whose unused keys are already ~0); at the row's last edge the rest of
// each region level's last node is padded with ~0.
__device__ __forceinline__ void place_tree_key(Block* __restrict__ region_base, Block* __restrict__ line,
                                               uint64_t d, uint32_t L, uint64_t T, uint64_t j, uint64_t P,
                                               bool nar) {
  const bool last = j == d - 1;
  const uint32_t fsh = node_shift(nar);
  const uint64_t F = 1ull << fsh;
  uint64_t span = 1ull << leaf_shift(nar), cum = 0;
  for (uint32_t l = 1; l <= L; ++l, span <<= fsh) {
    if (!last && ((j + 1) & (span - 1)) != 0) return;  // not a key boundary here, nor above
    const uint64_t k = j / span;
    if (l == L) {
      put_top(line, k, P, nar);
    } else {
      cum += tree_level_nodes(d, l, nar);
      Block* nd = region_base + (T - cum) + (k >> fsh);  // levels stored top first
      put_key(nd, k & (F - 1), P, nar);
      if (last)
        for (uint64_t t = (k & (F - 1)) + 1; t < F; ++t) put_key(nd, t, ~0ull, nar);
    }
  }
}

// Long rows: one block per row, scanning tiles of kThreads*4 weights; every
// prefix also goes into the tree levels whose keys end at it.
template <bool nar>
__global__ void __launch_bounds__(kThreads) k_leaves_long(const uint64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ col,
                                                          const uint32_t* __restrict__ w,
                                                          const uint64_t* __restrict__ region,
                                                          const uint8_t* __restrict__ cls, uint32_t n,
                                                          uint32_t tree_min, Block* __restrict__ blk,
                                                          Block* __restrict__ rec,
                                                          const uint32_t* rows,
                                                          const uint32_t* n_rows, uint32_t* err) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint32_t nr = *n_rows;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint32_t u = rows[r];
    const uint64_t a = off[u];
    const uint64_t d = off[u + 1] - a;
    const uint64_t r0 = region[u];
    const uint64_t T = tree_nodes(d, tree_min, nar);
    const bool tree = d > tree_min;
    const uint32_t L = tree ? tree_levels(d, nar) : 0;
    const uint64_t E = 1ull << leaf_shift(nar);
    Block* leaves = blk + r0 + T;
    // the node line before any of its tree keys (the scans' barriers order
    // this write before theirs); its weight comes with the last edge
    if (threadIdx.x == 0) write_record(rec, u, 0, r0, d);
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < d; t0 += kThreads * 4) {
      const uint64_t j0 = t0 + threadIdx.x * 4ull;
      uint64_t v[4];
      uint64_t local = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = j0 + k;
        local += (j < d) ? w[a + j] : 0u;
        v[k] = local;
      }
      uint64_t total;
      const uint64_t excl = block_exclusive_scan_u64<kThreads>(local, lds, &total);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = j0 + k;
        if (j < d) {
          const uint64_t P = carry + excl + v[k];
          put_edge(leaves, j, P, leaf_dest(cls, n, col[a + j], u), nar);
          if (tree) place_tree_key(blk + r0, rec + u, d, L, T, j, P, nar);
          if (j == d - 1) {
            rec[u].key[0] = P;
            if (nar && P > 0xFFFFFFFFull) atomicOr(err, kErrNarrow);
          }
        } else if (j < leaf_blocks(d, nar) * E) {
          pad_edge(leaves, j, nar);
        }
      }
      carry += total;
    }
  }
}

// ---- exclusive scan, u32 -> u64, three phases ----
constexpr int kScanItems = 4;
constexpr uint64_t kScanTile = kThreads * kScanItems;

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in,
                                                          uint64_t n, uint64_t* blocks) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) v += in[base + k];
  uint64_t total;
  block_exclusive_scan_u64<kThreads>(v, lds, &total);
  if (threadIdx.x == 0) blocks[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) k_scan_blocks(uint64_t* blocks, uint64_t nb,
                                                          uint64_t* total_out) {
  __shared__ uint64_t lds[kThreads / 64];
  uint64_t carry = 0;
  for (uint64_t t0 = 0; t0 < nb; t0 += kThreads) {
    const uint64_t i = t0 + threadIdx.x;
    const uint64_t v = i < nb ? blocks[i] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan_u64<kThreads>(v, lds, &total);
    if (i < nb) blocks[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kThreads) k_scan_apply(const uint32_t* __restrict__ in,
                                                         uint64_t n,
                                                         const uint64_t* __restrict__ blocks,
                                                         uint64_t* __restrict__ out) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = local;
    local += (base + k < n) ? in[base + k] : 0u;
  }
  uint64_t total;
  const uint64_t ex = block_exclusive_scan_u64<kThreads>(local, lds, &total) + blocks[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] = ex + v[k];
}

// 1 for nodes with out-edges
__global__ void k_live_flags(const uint64_t* __restrict__ off, uint32_t n, uint32_t* flag) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    flag[v] = off[v + 1] > off[v] ? 1u : 0u;
}

// nodes with out-edges in id order to `live`, the others to `dang`
__global__ void k_split_nodes(const uint32_t* __restrict__ flag, const uint64_t* __restrict__ scan, uint32_t n,
                              uint32_t* live, uint32_t* dang) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (flag[v]) live[scan[v]] = static_cast<uint32_t>(v);
    else dang[v - scan[v]] = static_cast<uint32_t>(v);
  }
}

// class of every node for the destination tags: no out-edges, small under
// the pool's bound S (1 <= out-degree <= S), or neither
__global__ void k_node_class(const uint64_t* __restrict__ off, uint32_t n, uint32_t S, uint8_t* cls) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t d = off[v + 1] - off[v];
    cls[v] = static_cast<uint8_t>(d == 0 ? kTagDangling : (d <= S ? kTagSmall : 0u));
  }
}

uint32_t grid_for(uint64_t items) {
  uint64_t b = (items + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<uint32_t>(b);
}

}  // namespace

uint64_t scan_block_count(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* blocks,
                           uint64_t* total_dev, hipStream_t s) {
  const uint64_t nb = scan_block_count(n);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<uint32_t>(nb)), dim3(kThreads), 0, s, in, n,
                     blocks);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kThreads), 0, s, blocks, nb, total_dev);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<uint32_t>(nb)), dim3(kThreads), 0, s, in, n,
                     blocks, out);
  return hipGetLastError();
}

hipError_t launch_validate(const fppr_graph* g, hipStream_t s, bool maxima) {
  hipLaunchKernelGGL(k_validate_offsets, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n,
                     g->m, g->d_err, maxima ? g->d_err + 12 : nullptr);
  if (g->m)
    hipLaunchKernelGGL(k_validate_edges, dim3(grid_for(g->m)), dim3(kThreads), 0, s, g->col, g->w,
                       g->m, g->n, g->d_err, maxima ? g->d_err + 13 : nullptr);
  return hipGetLastError();
}

hipError_t launch_split_nodes(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_live_flags, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, g->flag);
  hipError_t e = launch_scan_u32(g->flag, g->scan, g->n, g->scan_blocks,
                                 reinterpret_cast<uint64_t*>(g->d_err + 10), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_split_nodes, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->flag, g->scan, g->n,
                     g->live, g->dang);
  return hipGetLastError();
}

hipError_t launch_region_sizes(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_region_sizes, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n,
                     g->tree_min, g->narrow, g->flag);
  return launch_scan_u32(g->flag, g->region, g->n, g->scan_blocks,
                         reinterpret_cast<uint64_t*>(g->d_err + 2), s);
}

template <bool kNar>
void launch_leaves_t(fppr_graph* g, hipStream_t s, bool count_trees) {
  uint32_t* n_long = g->d_err + 1;
  const uint8_t* cls = g->tagged ? g->cls : nullptr;
  hipLaunchKernelGGL(k_leaves_short<kNar>, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->col,
                     g->w, g->region, cls, g->n, g->tree_min, g->n_blocks, g->blocks, g->rec,
                     g->rows, n_long, count_trees ? g->d_err + 9 : nullptr, g->d_err);
  hipLaunchKernelGGL(k_leaves_long<kNar>, dim3(2048), dim3(kThreads), 0, s, g->off, g->col, g->w,
                     g->region, cls, g->n, g->tree_min, g->blocks, g->rec, g->rows, n_long, g->d_err);
}

hipError_t launch_node_class(fppr_graph* g, uint32_t S, hipStream_t s) {
  if (!g->tagged) return hipSuccess;
  hipLaunchKernelGGL(k_node_class, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, S, g->cls);
  g->S_tag = S;
  return hipGetLastError();
}

hipError_t launch_leaves(fppr_graph* g, hipStream_t s, bool count_trees) {
  if (g->narrow) launch_leaves_t<true>(g, s, count_trees);
  else launch_leaves_t<false>(g, s, count_trees);
  return hipGetLastError();
}

}  // namespace fppr
