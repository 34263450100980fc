// Guide-table layout of a graph (guide.hpp): per-node heads, per-edge draw
// thresholds and the tables, built from the CSR in one pass over the rows
// and one short pass per child level; and the short-walk pool of graphs with
// this layout.
//
// Every kernel here keeps its indices inside the arrays it was given even on
// an invalid CSR (a rebuild validates on the device without waiting): ids
// >= n become the row's own node, searches stay inside their row, and child
// tables are only linked once their room is reserved.
#include "fppr_internal.hpp"
#include "guide.hpp"

namespace fppr {

namespace {

using guide::Cand;
using guide::Entry;
using guide::Head;
using guide::Pending;

constexpr int kThreads = 256;
constexpr uint32_t kShortRow = 64;  // rows up to this length: one thread each

uint32_t grid_for(uint64_t items) {
  uint64_t b = (items + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<uint32_t>(b);
}

// thresholds of a row: T(j) for j < d - 1
struct Thr {
  const uint64_t* t;
  __device__ uint64_t operator()(uint32_t j) const { return t[j]; }
};

// candidate c of a row: its destination's record (id with class tag, table, lg)
struct Recs {
  const uint32_t* col;  // the row's destinations
  const Head* head;
  uint32_t n, row;
  __device__ Cand operator()(uint32_t c) const {
    uint32_t v = col[c];
    if (v >= n) v = row;  // invalid CSR: never index past n (the graph's check reports it)
    const Head h = head[v];
    return Cand{v | ((h.meta >> 8) << kTagShift), h.base, h.meta & 0xFFu};
  }
};

// Reserves a child table: nbk entries from the shared counter and a slot in
// the next level's list. ~0u (and the graph's failure bit) when either is
// full or the level limit is reached.
struct Pusher {
  GuideCtl* ctl;
  Pending* out;
  uint64_t cap;
  uint32_t tcap, next_level, max_level;
  uint32_t* err;
  uint64_t off;
  uint32_t row;
  __device__ uint32_t operator()(uint64_t lo, uint64_t hi, uint32_t first, uint32_t last, uint32_t nbk,
                                 uint32_t sh) const {
    if (next_level > max_level) {
      atomicOr(err, kErrGuide);
      return ~0u;
    }
    const unsigned long long base = atomicAdd(&ctl->next_entry, static_cast<unsigned long long>(nbk));
    if (base + nbk > cap) {
      atomicOr(err, kErrGuide);
      return ~0u;
    }
    const uint32_t slot = atomicAdd(&ctl->tables[next_level], 1u);
    if (slot >= tcap) {
      atomicOr(err, kErrGuide);
      return ~0u;
    }
    out[slot] = Pending{lo, hi, off, first, last, row, sh, nbk, static_cast<uint32_t>(base)};
    return static_cast<uint32_t>(base);
  }
};

// entries of each node's row table: 2^table_bits(ceil(log2 d)), none without out-edges
__global__ void k_guide_sizes(const uint64_t* __restrict__ off, uint32_t n, uint32_t* __restrict__ flag) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t d = off[v + 1] - off[v];
    flag[v] = d && d <= kMaxDeg ? 1u << guide::table_bits(guide::ceil_log2(d)) : 0u;
  }
}

// node heads: the table base (from the size scan at creation; degrees never
// change, so rebuilds keep it) and lg | class tag << 8
__global__ void k_guide_heads(const uint64_t* __restrict__ off, const uint64_t* __restrict__ scan,
                              const uint8_t* __restrict__ cls, uint32_t n, Head* __restrict__ head) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t d = off[v + 1] - off[v];
    const uint32_t lg = d && d <= kMaxDeg ? guide::ceil_log2(d) : 0u;
    const uint32_t base = scan ? static_cast<uint32_t>(scan[v]) : head[v].base;
    head[v] = Head{base, lg | (static_cast<uint32_t>(cls[v]) << 8)};
  }
}

__global__ void k_guide_ctl_init(GuideCtl* ctl, uint64_t first_free) {
  for (uint32_t i = threadIdx.x; i < kGuideLevels + 2; i += blockDim.x) ctl->tables[i] = 0;
  if (threadIdx.x == 0) ctl->next_entry = first_free;
}

// Short rows: one thread computes its row's thresholds, then fills its row
// table by one merge of bucket edges and thresholds. Long rows are queued
// for a block each.
__global__ void k_guide_short(const uint64_t* __restrict__ off, const uint32_t* __restrict__ col,
                              const uint32_t* __restrict__ w, const Head* __restrict__ head, uint32_t n,
                              uint64_t* __restrict__ T, Entry* __restrict__ ent, uint32_t* rows, uint32_t* n_rows,
                              GuideCtl* ctl, Pending* out, uint64_t cap, uint32_t tcap, uint32_t max_level,
                              uint32_t* err) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u];
    const uint64_t d = off[u + 1] - a;
    const bool long_row = d > kShortRow && d <= kMaxDeg;
    const uint64_t lm = __ballot(long_row);
    if (lm) {
      const int leader = __builtin_ctzll(lm);
      uint32_t base = 0;
      if (static_cast<int>(__lane_id()) == leader) base = atomicAdd(n_rows, static_cast<uint32_t>(__popcll(lm)));
      base = static_cast<uint32_t>(__shfl(static_cast<int>(base), leader, 64));
      if (long_row) rows[base + mask_rank(lm)] = static_cast<uint32_t>(u);
    }
    if (d == 0 || long_row) continue;
    if (d > kMaxDeg) {
      atomicOr(err, kErrDegree);
      continue;
    }
    uint64_t W = 0;
    for (uint64_t j = 0; j < d; ++j) W += w[a + j];
    if (W == 0) continue;  // zero weights: the validation has reported the CSR
    uint64_t P = 0;
    for (uint64_t j = 0; j + 1 < d; ++j) {
      P += w[a + j];
      T[a + j] = P < W ? guide::threshold(P, W) : ~0ull;
    }
    T[a + d - 1] = ~0ull;
    const Thr th{T + a};
    const Recs rec{col + a, head, n, static_cast<uint32_t>(u)};
    const Pusher push{ctl, out, cap, tcap, 2u, max_level, err, a, static_cast<uint32_t>(u)};
    Entry* row_ent = ent + head[u].base;
    const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
    guide::for_row_buckets(th, static_cast<uint32_t>(d), kb, [&](uint32_t b, uint32_t c0, uint32_t c1) {
      guide::fill_entry(row_ent + b, th, rec, c0, c1, push);
    });
  }
}

// Long rows: one block per row. The row's total, then its prefixes and
// thresholds in tiles of kThreads * 4 edges, then its table entries by
// binary search, one entry per thread.
__global__ void __launch_bounds__(kThreads) k_guide_long(const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ col,
                                                         const uint32_t* __restrict__ w,
                                                         const Head* __restrict__ head, uint32_t n,
                                                         uint64_t* T, Entry* __restrict__ ent,
                                                         const uint32_t* rows, const uint32_t* n_rows,
                                                         GuideCtl* ctl, Pending* out, uint64_t cap, uint32_t tcap,
                                                         uint32_t max_level, uint32_t* err) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint32_t nr = *n_rows;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint32_t u = rows[r];
    const uint64_t a = off[u];
    const uint64_t d = off[u + 1] - a;
    uint64_t part = 0;
    for (uint64_t j = threadIdx.x; j < d; j += kThreads) part += w[a + j];
    uint64_t W = 0;
    block_exclusive_scan_u64<kThreads>(part, lds, &W);
    if (W == 0) continue;  // block-uniform
    uint64_t carry = 0;
    for (uint64_t t0 = 0; t0 < d; t0 += kThreads * 4) {
      const uint64_t j0 = t0 + threadIdx.x * 4ull;
      uint64_t v[4];
      uint64_t local = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = j0 + k;
        local += j < d ? w[a + j] : 0u;
        v[k] = local;
      }
      uint64_t total;
      const uint64_t excl = block_exclusive_scan_u64<kThreads>(local, lds, &total);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t j = j0 + k;
        if (j + 1 < d) {
          const uint64_t P = carry + excl + v[k];
          T[a + j] = P < W ? guide::threshold(P, W) : ~0ull;
        } else if (j + 1 == d) {
          T[a + j] = ~0ull;
        }
      }
      carry += total;
    }
    __syncthreads();  // the row's thresholds, visible to the whole block
    const Thr th{T + a};
    const Recs rec{col + a, head, n, u};
    const Pusher push{ctl, out, cap, tcap, 2u, max_level, err, a, u};
    Entry* row_ent = ent + head[u].base;
    const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
    const uint32_t last = static_cast<uint32_t>(d - 1);
    for (uint32_t b = threadIdx.x; b < (1u << kb); b += kThreads) {
      uint64_t blo, bhi;
      guide::row_bucket(kb, b, &blo, &bhi);
      const uint32_t c0 = guide::containing(th, 0u, last, blo);
      const uint32_t c1 = guide::containing(th, 0u, last, bhi);
      guide::fill_entry(row_ent + b, th, rec, c0, c1, push);
    }
    __syncthreads();  // the next row's scans reuse the LDS words
  }
}

// Child tables of one level: one wave per table, its lanes over the table's
// buckets; tables of the next level go to `out`.
__global__ void __launch_bounds__(kThreads) k_guide_level(const uint32_t* __restrict__ col,
                                                          const Head* __restrict__ head, uint32_t n,
                                                          const uint64_t* __restrict__ T, Entry* __restrict__ ent,
                                                          const Pending* __restrict__ in, Pending* out,
                                                          GuideCtl* ctl, uint32_t level, uint64_t cap,
                                                          uint32_t tcap, uint32_t max_level, uint32_t* err) {
  const uint32_t lane = __lane_id();
  uint32_t count = ctl->tables[level];
  if (count > tcap) count = tcap;
  const uint32_t waves = gridDim.x * (kThreads / 64);
  for (uint32_t t = blockIdx.x * (kThreads / 64) + threadIdx.x / 64; t < count; t += waves) {
    const Pending p = in[t];
    const Thr th{T + p.off};
    const Recs rec{col + p.off, head, n, p.row};
    const Pusher push{ctl, out, cap, tcap, level + 1, max_level, err, p.off, p.row};
    for (uint32_t i = lane; i < p.nbk; i += 64) {
      uint64_t blo, bhi;
      guide::child_bucket(p.origin, p.end, p.sh, i, &blo, &bhi);
      const uint32_t c0 = guide::containing(th, p.a, p.b, blo);
      const uint32_t c1 = guide::containing(th, p.a, p.b, bhi);
      guide::fill_entry(ent + p.base + i, th, rec, c0, c1, push);
    }
  }
}

// The value of the other lane of this lane's aligned pair (DPP quad
// permutation [1, 0, 3, 2]).
__device__ __forceinline__ uint32_t pair_swap(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
}

// Pool walks over guide tables: a lane pair per (small node, slot j), both
// lanes following the same walk; the even lane reads bytes 0..31 of each
// entry and the odd lane bytes 32..47, and one exchange gives both the
// whole entry. Entry (16 bytes) at v * K + j: end id with its class tag,
// end's table, end's lg | steps << 8 | mark << 16 (mark 1 = terminated).
__global__ void __launch_bounds__(kThreads) k_pool_guide(const Head* __restrict__ head,
                                                         const Entry* __restrict__ ent, uint64_t cap,
                                                         const uint32_t* __restrict__ small_nodes, uint64_t n_small,
                                                         uint32_t K_log2, uint32_t L, uint32_t T, uint32_t key0,
                                                         uint32_t key1, uint4* __restrict__ pool) {
  const uint64_t total = n_small << K_log2;
  const uint32_t half = threadIdx.x & 1u;
  const uint64_t stride = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 1;
  for (uint64_t idx = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) >> 1; idx < total;
       idx += stride) {
    const uint32_t j = static_cast<uint32_t>(idx & ((1ull << K_log2) - 1));
    const uint32_t v = small_nodes[idx >> K_log2];
    const Head h = head[v];
    uint32_t cur = v, base = h.base, lg = h.meta & 0xFFu, tag = h.meta >> 8;
    uint32_t steps = 0, mark = 0;
    for (uint32_t t = 0; t < L; ++t) {
      if (tag == kTagDangling) break;  // arrived at a node without out-edges: stays active
      const U4 x = philox10(j, t, v, 1u, key0, key1);
      const uint64_t D = (static_cast<uint64_t>(x.x1) << 32) | x.x0;
      uint64_t e = base + guide::top_bits(D, guide::table_bits(lg));
      for (uint32_t k = 0; k < 64; ++k) {  // at most one entry per level
        if (e >= cap) e = cap - 1;
        const uint4* p = reinterpret_cast<const uint4*>(ent + e) + half * 2;
        const uint4 qa = p[0];
        const uint4 qb = half ? make_uint4(0, 0, 0, 0) : p[1];
        // even lane: lo, hi | L, M; odd lane: R, meta. Both get all of it.
        const uint4 oa = make_uint4(pair_swap(qa.x), pair_swap(qa.y), pair_swap(qa.z), pair_swap(qa.w));
        const uint4 ob = make_uint4(pair_swap(qb.x), pair_swap(qb.y), pair_swap(qb.z), pair_swap(qb.w));
        const uint4 A = half ? oa : qa, B = half ? ob : qb, C = half ? qa : oa;
        const uint64_t lo = (static_cast<uint64_t>(A.y) << 32) | A.x;
        const uint64_t hi = (static_cast<uint64_t>(A.w) << 32) | A.z;
        const uint32_t meta = C.z;
        if (D < lo) {
          cur = B.x;
          base = B.y;
          lg = meta & 0xFFu;
          break;
        }
        if (D >= hi) {
          cur = C.x;
          base = C.y;
          lg = (meta >> 16) & 0xFFu;
          break;
        }
        if (!(meta & guide::kChild)) {
          cur = B.z;
          base = B.w;
          lg = (meta >> 8) & 0xFFu;
          break;
        }
        e = B.w + ((D - lo) >> ((meta >> 8) & 0xFFu));
      }
      tag = cur >> kTagShift;
      cur &= kIdMask;
      steps += 1;
      if (x.x2 < T) {
        mark = 1;
        break;
      }
    }
    if (half == 0)
      pool[(static_cast<uint64_t>(v) << K_log2) + j] =
          make_uint4(cur | (tag << kTagShift), base, lg | (steps << 8) | (mark << 16), 0u);
  }
}

// canonical order for export: rank k's entries from node small_nodes[k]'s
// block, as end | steps << 32 | mark << 48 with plain end ids
__global__ void k_pool_guide_export(const uint4* __restrict__ pool, const uint32_t* __restrict__ small_nodes,
                                    uint64_t n_small, uint32_t K_log2, uint64_t* __restrict__ out) {
  const uint64_t total = n_small << K_log2;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t v = small_nodes[i >> K_log2];
    const uint4 e = pool[(v << K_log2) + (i & ((1ull << K_log2) - 1))];
    out[i] = static_cast<uint64_t>(e.x & kIdMask) | (static_cast<uint64_t>((e.z >> 8) & 0xFFu) << 32) |
             (static_cast<uint64_t>((e.z >> 16) & 1u) << 48);
  }
}

}  // namespace

hipError_t launch_guide_sizes(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_sizes, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, g->flag);
  return launch_scan_u32(g->flag, g->scan, g->n, g->scan_blocks, reinterpret_cast<uint64_t*>(g->d_err + 4), s);
}

hipError_t launch_guide_build(fppr_graph* g, bool bases, uint32_t levels, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_heads, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off,
                     bases ? g->scan : nullptr, g->cls, g->n, g->ghead);
  hipLaunchKernelGGL(k_guide_ctl_init, dim3(1), dim3(64), 0, s, g->gctl, g->g_entries1);
  const uint32_t maxl = levels;
  hipLaunchKernelGGL(k_guide_short, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->col, g->w, g->ghead,
                     g->n, g->gT, g->gent, g->rows, g->d_err + 1, g->gctl, g->gtab[0], g->g_cap, g->g_tcap, maxl,
                     g->d_err);
  hipLaunchKernelGGL(k_guide_long, dim3(2048), dim3(kThreads), 0, s, g->off, g->col, g->w, g->ghead, g->n, g->gT,
                     g->gent, g->rows, g->d_err + 1, g->gctl, g->gtab[0], g->g_cap, g->g_tcap, maxl, g->d_err);
  return hipGetLastError();
}

hipError_t launch_guide_level(fppr_graph* g, uint32_t level, uint32_t levels, hipStream_t s) {
  // level l's tables sit in list (l & 1) (level 2 in list 0)
  const guide::Pending* in = g->gtab[level & 1u ? 1 : 0];
  guide::Pending* out = g->gtab[level & 1u ? 0 : 1];
  hipLaunchKernelGGL(k_guide_level, dim3(1024), dim3(kThreads), 0, s, g->col, g->ghead, g->n, g->gT, g->gent, in,
                     out, g->gctl, level, g->g_cap, g->g_tcap, levels, g->d_err);
  return hipGetLastError();
}

hipError_t launch_pool_guide(fppr_graph* g, hipStream_t s) {
  const uint64_t total = g->n_small << g->K_log2;
  if (total == 0) return hipSuccess;
  const uint64_t seed = g->pool_opts.seed;
  hipLaunchKernelGGL(k_pool_guide, dim3(grid_for(total * 2)), dim3(kThreads), 0, s, g->ghead, g->gent, g->g_cap,
                     g->small_nodes, g->n_small, g->K_log2, g->pool_opts.L, g->pool_T, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32), reinterpret_cast<uint4*>(g->pool));
  return hipGetLastError();
}

hipError_t launch_pool_guide_export(const fppr_graph* g, uint64_t* out, hipStream_t s) {
  const uint64_t total = g->n_small << g->K_log2;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_guide_export, dim3(grid_for(total)), dim3(kThreads), 0, s,
                     reinterpret_cast<const uint4*>(g->pool), g->small_nodes, g->n_small, g->K_log2, out);
  return hipGetLastError();
}

}  // namespace fppr
