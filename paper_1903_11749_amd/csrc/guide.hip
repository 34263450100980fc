// Guide-table layout of a graph (guide.hpp): per-node heads, per-edge draw
// thresholds and the tables, built from the CSR in one pass over the rows
// and one short pass per child level; and the short-walk pool of graphs with
// this layout.
//
// Every kernel here keeps its indices inside the arrays it was given even on
// an invalid CSR (a rebuild validates on the device without waiting): ids
// >= n become the row's own node, searches stay inside their row, and child
// tables are only linked once their room is reserved.
#include <algorithm>

#include "fppr_internal.hpp"
#include "guide.hpp"

namespace fppr {

namespace {

using guide::Cand;
using guide::Entry;
using guide::Head;
using guide::Pending;

constexpr int kThreads = 256;

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

// candidate c of a row: its record from the per-edge record array
struct ERec {
  const uint4* r;  // the row's edge records: id with class tag, table base, lg
  __device__ Cand operator()(uint32_t c) const {
    const uint4 x = r[c];
    return Cand{x.x, x.y, x.z};
  }
};

// record of destination c of row u (ids >= n, only possible in an invalid
// CSR, become u itself: no kernel ever indexes past n)
__device__ __forceinline__ uint4 edge_record(const Head* __restrict__ head, uint32_t n, uint32_t c, uint32_t u) {
  if (c >= n) c = u;
  const Head h = head[c];
  return make_uint4(c | ((h.meta >> 8) << kTagShift), h.base, h.meta & 0xFFu, 0u);
}

// Child-table allocation for a whole wave, called by every lane in
// wave-uniform control flow: each lane with `need` gets a slot in the next
// level's list and nbk entries. A wave takes entries and slots from the
// shared counters in chunks (kEntChunk, kTabChunk) and hands them out from
// its registers, so the counters see one atomic per chunk; the unused rest
// of an entry chunk is never referenced, and unused slots are left with no
// buckets (flush(), at the wave's end). Returns the child's first entry, or
// ~0u (and the graph's failure bit) when the list or the entries are full or
// the level limit is reached.
constexpr uint64_t kEntChunk = 1024;
constexpr uint32_t kTabChunk = 128;
struct Alloc {
  GuideCtl* ctl;
  Pending* out;
  uint64_t cap;
  uint32_t tcap, next_level, max_level;
  uint32_t* err;
  // the wave's chunks (wave-uniform)
  uint64_t e_next = 0, e_end = 0;
  uint64_t t_next = 0, t_end = 0;

  __device__ uint32_t operator()(bool need, uint64_t lo, uint64_t hi, uint32_t first, uint32_t last, uint32_t nbk,
                                 uint32_t sh, uint64_t off, uint32_t row) {
    const uint64_t mask = __ballot(need);
    if (mask == 0) return ~0u;
    const uint64_t v = need ? nbk : 0u;
    const uint64_t inc = wave_inclusive_scan_u64(v);
    const uint64_t total = __shfl(static_cast<unsigned long long>(inc), 63, 64);
    const uint32_t cnt = static_cast<uint32_t>(__popcll(mask));
    const bool open = next_level <= max_level;
    if (!open) {
      if (need) atomicOr(err, kErrGuide);
      return ~0u;
    }
    if (e_next + total > e_end) {
      const uint64_t take = total > kEntChunk ? total : kEntChunk;
      unsigned long long b = 0;
      if (__lane_id() == 0) b = atomicAdd(&ctl->next_entry, static_cast<unsigned long long>(take));
      e_next = __shfl(b, 0, 64);
      e_end = e_next + take;
    }
    if (t_next + cnt > t_end) {
      flush();
      unsigned long long b = 0;
      if (__lane_id() == 0) b = atomicAdd(&ctl->tables[next_level], kTabChunk);
      t_next = __shfl(b, 0, 64);
      t_end = t_next + kTabChunk;  // cnt <= 64 < kTabChunk
    }
    const uint64_t slot = t_next + mask_rank(mask), base = e_next + (inc - v);
    t_next += cnt;
    e_next += total;
    if (!need) return ~0u;
    if (slot >= tcap || base + nbk > cap) {
      atomicOr(err, kErrGuide);
      if (slot < tcap) out[slot] = Pending{0, 0, 0, 0, 0, 0, 0, 0, 0};
      return ~0u;
    }
    out[slot] = Pending{lo, hi, off, first, last, row, sh, nbk, static_cast<uint32_t>(base)};
    return static_cast<uint32_t>(base);
  }
  // the unused slots of the wave's current chunk: no buckets
  __device__ void flush() {
    for (uint64_t t = t_next + __lane_id(); t < t_end && t < tcap; t += 64) out[t] = Pending{0, 0, 0, 0, 0, 0, 0, 0, 0};
    t_next = t_end;
  }
};

// Bounds, candidates and child of one entry, then the entry itself; every
// lane of the wave calls it (for the allocation), `act` marks those with an
// entry to write.
__device__ __forceinline__ void write_entry(Alloc& alloc, bool act, Entry* e, uint32_t c0, uint32_t c1,
                                            uint64_t t0, uint64_t t1, const Cand& L, const Cand& M, const Cand& R,
                                            uint64_t off, uint32_t row) {
  uint64_t lo = 0, hi = 0;
  const uint32_t mc = act ? guide::entry_bounds(c0, c1, t0, t1, &lo, &hi) : 0u;
  uint32_t sh = 0, nbk = 0;
  if (mc) nbk = guide::child_shape(lo, hi, mc, &sh);
  const uint32_t child = alloc(mc != 0, lo, hi, c0 + 1, c1 - 1, nbk, sh, off, row);
  if (act) guide::put_entry(e, lo, hi, mc, L, M, R, child, sh);
}

// entries of each node's row table: 2^table_bits(ceil(log2 d)), none without out-edges
__global__ void k_guide_sizes(const uint64_t* __restrict__ off, uint32_t n, uint32_t* __restrict__ flag) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t d = off[v + 1] - off[v];
    flag[v] = d && d <= kMaxDeg ? 1u << guide::table_bits(guide::ceil_log2(d)) : 0u;
  }
}

// size class of a row: ceil(log2 d) for 1 <= d <= 64 (0..6), 7 above, none without edges
__device__ __forceinline__ uint32_t row_class(uint64_t d) {
  return d == 0 ? ~0u : (d <= 64 ? guide::ceil_log2(d) : 7u);
}
__global__ void k_class_flags(const uint64_t* __restrict__ off, uint32_t n, uint32_t c, uint32_t* __restrict__ flag) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    flag[v] = row_class(off[v + 1] - off[v]) == c ? 1u : 0u;
}
__global__ void k_class_scatter(const uint32_t* __restrict__ flag, const uint64_t* __restrict__ scan, uint32_t n,
                                uint32_t* __restrict__ out) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < n;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (flag[v]) out[scan[v]] = static_cast<uint32_t>(v);
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

__global__ void k_guide_ctl_init(GuideCtl* ctl, uint64_t e1) {
  for (uint32_t i = threadIdx.x; i < kGuideLevels + 2; i += blockDim.x) ctl->tables[i] = 0;
  if (threadIdx.x == 0) ctl->next_entry = e1;
}

// Rows of one size class (2^(CL-1) < d <= 2^CL, d <= 64): a group of 2^CL
// lanes per row. Each lane takes one edge: weight, destination record and,
// after a segmented scan of the group, its prefix and threshold (both
// stored for the child levels); then each of the row's 2^kb <= 2^(CL-1)
// entries is filled by one lane, its candidates found by binary search over
// the group's thresholds and their records taken from the lanes holding
// them, all through lane shuffles.
template <uint32_t CL>
__global__ void __launch_bounds__(kThreads) k_guide_rows(const uint32_t* __restrict__ rows, uint64_t count,
                                                         const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ col,
                                                         const uint32_t* __restrict__ w, const Head* __restrict__ head,
                                                         uint32_t n, uint64_t* __restrict__ T, uint4* __restrict__ erec,
                                                         Entry* __restrict__ ent, Alloc alloc) {
  constexpr uint32_t GL = 1u << CL;
  const uint32_t gi = __lane_id() & (GL - 1);
  const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * kThreads) >> CL;
  const uint64_t first = (static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x) >> CL;
  for (uint64_t r = first; __ballot(r < count) != 0; r += groups) {  // wave-uniform loop
    const bool has = r < count;
    const uint32_t u = has ? rows[r] : 0u;
    const uint64_t a = has ? off[u] : 0;
    const uint32_t d = has ? static_cast<uint32_t>(off[u + 1] - a) : 1u;  // 1 <= d <= GL
    const bool mine = has && gi < d;
    const uint64_t wv = mine ? w[a + gi] : 0u;
    const uint4 rc = mine ? edge_record(head, n, col[a + gi], u) : make_uint4(0, 0, 0, 0);
    uint64_t P = wv;
#pragma unroll
    for (uint32_t o = 1; o < GL; o <<= 1) {
      const uint64_t t = __shfl_up(static_cast<unsigned long long>(P), o, GL);
      if (gi >= o) P += t;
    }
    const uint64_t W = __shfl(static_cast<unsigned long long>(P), static_cast<int>(d - 1), GL);
    const uint64_t Tv = gi + 1 < d ? (P < W ? guide::threshold(P, W) : ~0ull) : ~0ull;
    if (mine) {
      T[a + gi] = Tv;
      erec[a + gi] = rc;
    }
    const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
    const uint32_t nb = 1u << kb;
    uint64_t blo = 0, bhi = 0;
    guide::row_bucket(kb, gi & (nb - 1), &blo, &bhi);
    // candidates holding blo and bhi: the number of thresholds <= each
    uint32_t l0 = 0, h0 = d - 1, l1 = 0, h1 = d - 1;
#pragma unroll
    for (uint32_t it = 0; it <= CL; ++it) {
      const uint32_t m0 = (l0 + h0) >> 1, m1 = (l1 + h1) >> 1;
      const uint64_t t0 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(m0), GL);
      const uint64_t t1 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(m1), GL);
      if (l0 < h0) {
        if (t0 <= blo) l0 = m0 + 1;
        else h0 = m0;
      }
      if (l1 < h1) {
        if (t1 <= bhi) l1 = m1 + 1;
        else h1 = m1;
      }
    }
    const uint32_t c0 = l0, c1 = l1;
    const uint64_t ta = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(c0), GL);
    const uint64_t tb = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(c1 ? c1 - 1 : 0), GL);
    const uint32_t cm = c1 > c0 + 1 ? c0 + 1 : c0;
    Cand L, M, R;
    L.id = __shfl(rc.x, static_cast<int>(c0), GL);
    L.base = __shfl(rc.y, static_cast<int>(c0), GL);
    L.lg = __shfl(rc.z, static_cast<int>(c0), GL);
    M.id = __shfl(rc.x, static_cast<int>(cm), GL);
    M.base = __shfl(rc.y, static_cast<int>(cm), GL);
    M.lg = __shfl(rc.z, static_cast<int>(cm), GL);
    R.id = __shfl(rc.x, static_cast<int>(c1), GL);
    R.base = __shfl(rc.y, static_cast<int>(c1), GL);
    R.lg = __shfl(rc.z, static_cast<int>(c1), GL);
    write_entry(alloc, has && gi < nb, ent + (has ? head[u].base : 0u) + gi, c0, c1, ta, tb, L, M, R, a, u);
  }
  alloc.flush();
}

// Long rows (more than 64 edges): one block per row. The row's total, then
// its prefixes, thresholds and edge records in tiles of kThreads * 4 edges
// (thresholds also staged in LDS for rows of up to kStaged edges), then its
// table entries: each thread takes a run of consecutive entries, finds the
// first one's candidates by binary search and the rest by merging bucket
// edges with thresholds.
constexpr uint32_t kStaged = 4096;
__global__ void __launch_bounds__(kThreads) k_guide_long(const uint32_t* __restrict__ rows, uint64_t count,
                                                         const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ col,
                                                         const uint32_t* __restrict__ w,
                                                         const Head* __restrict__ head, uint32_t n, uint64_t* T,
                                                         uint4* erec, Entry* __restrict__ ent, Alloc alloc) {
  __shared__ uint64_t lds[kThreads / 64];
  __shared__ uint64_t sT[kStaged];
  for (uint64_t r = blockIdx.x; r < count; r += gridDim.x) {
    const uint32_t u = rows[r];
    const uint64_t a = off[u];
    const uint64_t d = off[u + 1] - a;
    const bool staged = d <= kStaged;  // block-uniform
    uint64_t part = 0;
    for (uint64_t j = threadIdx.x; j < d; j += kThreads) part += w[a + j];
    uint64_t W = 0;
    block_exclusive_scan_u64<kThreads>(part, lds, &W);
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
        if (j < d) {
          const uint64_t P = carry + excl + v[k];
          const uint64_t t = j + 1 < d && P < W ? guide::threshold(P, W) : ~0ull;
          T[a + j] = t;
          if (staged) sT[j] = t;
          erec[a + j] = edge_record(head, n, col[a + j], u);
        }
      }
      carry += total;
    }
    __syncthreads();  // the row's thresholds and records, visible to the whole block
    if (W != 0) {  // block-uniform
      const uint64_t* Tg = T + a;
      auto th = [&](uint32_t j) -> uint64_t { return staged ? sT[j] : Tg[j]; };
      const ERec rec{erec + a};
      Entry* row_ent = ent + head[u].base;
      const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
      const uint32_t last = static_cast<uint32_t>(d - 1), nb = 1u << kb;
      const uint32_t run = (nb + kThreads - 1) / kThreads;
      uint32_t c = 0;
      for (uint32_t k = 0; k < run; ++k) {  // block-uniform
        const uint32_t b = threadIdx.x * run + k;
        const bool act = b < nb;
        uint32_t c0 = 0, c1 = 0;
        uint64_t t0 = 0, t1 = 0;
        Cand L{}, M{}, R{};
        if (act) {
          uint64_t blo, bhi;
          guide::row_bucket(kb, b, &blo, &bhi);
          if (k == 0) c = guide::containing(th, 0u, last, blo);
          while (c < last && th(c) <= blo) ++c;
          c0 = c;
          c1 = c0;
          while (c1 < last && th(c1) <= bhi) ++c1;
          if (c1 > c0) {
            t0 = th(c0);
            t1 = th(c1 - 1);
          }
          L = rec(c0);
          R = rec(c1);
          M = c1 > c0 + 1 ? rec(c0 + 1) : L;
          c = c1;
        }
        write_entry(alloc, act, row_ent + (act ? b : 0u), c0, c1, t0, t1, L, M, R, a, u);
      }
    }
    __syncthreads();  // the next row's scans and staging reuse the LDS words
  }
  alloc.flush();
}

// The child tables of one level, one lane per table: its entries in order,
// their candidates by merging bucket edges with the row's thresholds;
// tables of the next level go to the other list. A wave runs until the
// largest table among its lanes is done.
__global__ void __launch_bounds__(kThreads) k_guide_level(const uint64_t* __restrict__ T,
                                                          const uint4* __restrict__ erec, Entry* __restrict__ ent,
                                                          const Pending* __restrict__ in, uint32_t level, Alloc alloc) {
  uint32_t count = alloc.ctl->tables[level];
  if (count > alloc.tcap) count = alloc.tcap;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; __ballot(t < count) != 0;
       t += stride) {  // wave-uniform loop
    Pending p{};
    if (t < count) p = in[t];  // tables that found no room have no buckets
    uint32_t most = p.nbk;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t x = static_cast<uint32_t>(__shfl_xor(static_cast<int>(most), o, 64));
      most = x > most ? x : most;
    }
    const Thr th{T + p.off};
    const ERec rec{erec + p.off};
    uint32_t c = p.a;
    for (uint32_t i = 0; i < most; ++i) {  // wave-uniform
      const bool act = i < p.nbk;
      uint32_t c0 = 0, c1 = 0;
      uint64_t t0 = 0, t1 = 0;
      Cand L{}, M{}, R{};
      if (act) {
        uint64_t blo, bhi;
        guide::child_bucket(p.origin, p.end, p.sh, i, &blo, &bhi);
        while (c < p.b && th(c) <= blo) ++c;
        c0 = c;
        c1 = c0;
        while (c1 < p.b && th(c1) <= bhi) ++c1;
        if (c1 > c0) {
          t0 = th(c0);
          t1 = th(c1 - 1);
        }
        L = rec(c0);
        R = rec(c1);
        M = c1 > c0 + 1 ? rec(c0 + 1) : L;
        c = c1;
      }
      write_entry(alloc, act, ent + (act ? p.base + i : 0u), c0, c1, t0, t1, L, M, R, p.off, p.row);
    }
  }
  alloc.flush();
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

hipError_t launch_guide_class(fppr_graph* g, uint32_t c, uint64_t at, hipStream_t s) {
  hipLaunchKernelGGL(k_class_flags, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, c, g->flag);
  hipError_t e = launch_scan_u32(g->flag, g->scan, g->n, g->scan_blocks, reinterpret_cast<uint64_t*>(g->d_err + 14), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_class_scatter, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->flag, g->scan, g->n,
                     g->gclass + at);
  return hipGetLastError();
}

namespace {
Alloc allocator(fppr_graph* g, uint32_t next_level, uint32_t max_level) {
  const uint32_t list = next_level & 1u ? 1u : 0u;  // level l's tables sit in list (l & 1)
  Alloc a{};
  a.ctl = g->gctl;
  a.out = g->gtab[list];
  a.cap = g->g_cap;
  a.tcap = g->g_tcap;
  a.next_level = next_level;
  a.max_level = max_level;
  a.err = g->d_err;
  return a;
}
template <uint32_t CL>
void launch_rows(fppr_graph* g, const Alloc& p, hipStream_t s) {
  const uint64_t count = g->gclass_off[CL + 1] - g->gclass_off[CL];
  if (!count) return;
  const uint32_t blocks = std::min<uint32_t>(grid_for(count << CL), 2048u);  // few waves: few partial chunks
  hipLaunchKernelGGL(k_guide_rows<CL>, dim3(blocks), dim3(kThreads), 0, s,
                     g->gclass + g->gclass_off[CL], count, g->off, g->col, g->w, g->ghead, g->n, g->gT, g->gerec,
                     g->gent, p);
}
}  // namespace

hipError_t launch_guide_build(fppr_graph* g, bool bases, uint32_t levels, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_heads, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off,
                     bases ? g->scan : nullptr, g->cls, g->n, g->ghead);
  hipLaunchKernelGGL(k_guide_ctl_init, dim3(1), dim3(64), 0, s, g->gctl, g->g_entries1);
  const Alloc p = allocator(g, 2, levels);
  launch_rows<0>(g, p, s);
  launch_rows<1>(g, p, s);
  launch_rows<2>(g, p, s);
  launch_rows<3>(g, p, s);
  launch_rows<4>(g, p, s);
  launch_rows<5>(g, p, s);
  launch_rows<6>(g, p, s);
  const uint64_t nlong = g->gclass_off[8] - g->gclass_off[7];
  if (nlong)
    hipLaunchKernelGGL(k_guide_long, dim3(static_cast<uint32_t>(nlong < 2048 ? nlong : 2048)), dim3(kThreads), 0, s,
                       g->gclass + g->gclass_off[7], nlong, g->off, g->col, g->w, g->ghead, g->n, g->gT, g->gerec,
                       g->gent, p);
  return hipGetLastError();
}

hipError_t launch_guide_level(fppr_graph* g, uint32_t level, uint32_t levels, hipStream_t s) {
  const guide::Pending* in = g->gtab[level & 1u ? 1 : 0];
  hipLaunchKernelGGL(k_guide_level, dim3(2048), dim3(kThreads), 0, s, g->gT, g->gerec, g->gent, in, level,
                     allocator(g, level + 1, levels));
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
