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
// Blocks for a grid-stride kernel over `items` threads' work: no more
// than fit on the device at once (a second round of waves would run with
// the SIMDs partly empty, waiting on loads) and at most `cap`.
template <typename Kernel>
hipError_t resident_grid(Kernel kernel, uint64_t items, uint32_t cap, uint32_t* blocks) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0);
  if (e != hipSuccess) return e;
  const uint32_t fit = static_cast<uint32_t>(std::max(1, per_cu) * std::max(1, cus));
  *blocks = std::min(grid_for(items), std::min(fit, cap));
  return hipSuccess;
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
// level's list and nbk entries. Tables with fewer than kLargeThr thresholds
// between their candidates go to the small list (out[0, tcap)), the others
// to the large list (out[tcap, tcap + tcap_big)), so that a level pass can
// give each list a lane group of its size. A wave takes entries and slots
// from the shared counters in chunks (kEntChunk, kTabChunk) and hands them
// out from its registers, so the counters see one atomic per chunk; the
// unused rest of an entry chunk is never referenced, and unused slots are
// left with no buckets (flush(), at the wave's end). Returns the child's
// first entry, or ~0u (and the graph's failure bit) when its list or the
// entries are full or the level limit is reached.
constexpr uint64_t kEntChunk = 1024;
constexpr uint32_t kTabChunk = 128;
constexpr uint32_t kLargeThr = 8;
// lane 0's value as a wave-uniform (scalar) one; every lane is active here
__device__ __forceinline__ uint64_t first_lane_u64(unsigned long long x) {
  return static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x)))) |
         (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32))))
          << 32);
}
// Inclusive sum over the wave of a 32-bit value by DPP (every lane
// active): within rows of 16 lanes by shifts of 1, 2, 4 and 8 (lanes shifted
// in read 0), then across rows by the broadcasts of lane 15 of each row to
// the next (rows 1 and 3 take it) and of lane 31 (rows 2 and 3 take it).
__device__ __forceinline__ uint32_t wave_inclusive_scan_u32(uint32_t x) {
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, true));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xA, 0xF, false));
  x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xC, 0xF, false));
  return x;
}

// Largest value over the wave (every lane active), wave-uniform: rows of 16
// lanes by DPP (quad swaps, then half-row and row mirrors), then the four
// row results through scalar registers.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  uint32_t y = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
  x = y > x ? y : x;
  y = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x4E, 0xF, 0xF, false));
  x = y > x ? y : x;
  y = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x141, 0xF, 0xF, false));
  x = y > x ? y : x;
  y = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x140, 0xF, 0xF, false));
  x = y > x ? y : x;
  const uint32_t r0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 0));
  const uint32_t r1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 16));
  const uint32_t r2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 32));
  const uint32_t r3 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 48));
  const uint32_t m01 = r0 > r1 ? r0 : r1, m23 = r2 > r3 ? r2 : r3;
  return m01 > m23 ? m01 : m23;
}

struct Alloc {
  GuideCtl* ctl;
  Pending* out;
  uint64_t cap;
  uint32_t tcap, tcap_big, next_level, max_level;
  uint32_t* err;
  // the wave's chunks (wave-uniform)
  uint64_t e_next = 0, e_end = 0;
  uint64_t t_next = 0, t_end = 0;  // small list
  uint64_t b_next = 0, b_end = 0;  // large list

  __device__ uint32_t operator()(bool need, uint64_t lo, uint64_t hi, uint32_t first, uint32_t last, uint32_t nbk,
                                 uint32_t sh, uint64_t off, uint32_t row) {
    const uint64_t mask = __ballot(need);
    if (mask == 0) return ~0u;
    const uint64_t v = need ? nbk : 0u;
    uint64_t inc = 0, total = 0;
    if (__ballot(v >= (1u << 25)) == 0) {  // wave-uniform: the 64 values sum below 2^31
      const uint32_t i32 = wave_inclusive_scan_u32(static_cast<uint32_t>(v));
      inc = i32;
      total = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(i32), 63));
    } else {
      inc = wave_inclusive_scan_u64(v);
      total = first_lane_u64(__shfl(static_cast<unsigned long long>(inc), 63, 64));
    }
    const bool open = next_level <= max_level;
    if (!open) {
      if (need) atomicOr(err, kErrGuide);
      return ~0u;
    }
    if (e_next + total > e_end) {
      const uint64_t take = total > kEntChunk ? total : kEntChunk;
      unsigned long long b = 0;
      if (__lane_id() == 0) b = atomicAdd(&ctl->next_entry, static_cast<unsigned long long>(take));
      e_next = first_lane_u64(b);
      e_end = e_next + first_lane_u64(take);
    }
    const bool large = need && last - first >= kLargeThr;
    const uint64_t ml = __ballot(large), ms = mask & ~ml;
    const uint32_t cs = static_cast<uint32_t>(__popcll(ms)), cl = static_cast<uint32_t>(__popcll(ml));
    if (t_next + cs > t_end) {
      flush_small();
      unsigned long long b = 0;
      if (__lane_id() == 0) b = atomicAdd(&ctl->tables[next_level], kTabChunk);
      t_next = first_lane_u64(b);
      t_end = t_next + kTabChunk;  // cs <= 64 < kTabChunk
    }
    if (b_next + cl > b_end) {
      flush_large();
      unsigned long long b = 0;
      if (__lane_id() == 0) b = atomicAdd(&ctl->big[next_level], kTabChunk);
      b_next = first_lane_u64(b);
      b_end = b_next + kTabChunk;
    }
    const uint64_t slot = large ? b_next + mask_rank(ml) : t_next + mask_rank(ms);
    const uint64_t base = e_next + (inc - v);
    t_next += cs;
    b_next += cl;
    e_next += total;
    if (!need) return ~0u;
    const uint32_t room = large ? tcap_big : tcap;
    Pending* list = large ? out + tcap : out;
    if (slot >= room || base + nbk > cap) {
      atomicOr(err, kErrGuide);
      if (slot < room) list[slot] = Pending{0, 0, 0, 0, 0, 0, 0, 0, 0};
      return ~0u;
    }
    list[slot] = Pending{lo, hi, off, first, last, row, sh, nbk, static_cast<uint32_t>(base)};
    return static_cast<uint32_t>(base);
  }
  // the unused slots of the wave's current chunks: no buckets
  __device__ void flush_small() {
    for (uint64_t t = t_next + __lane_id(); t < t_end && t < tcap; t += 64) out[t] = Pending{0, 0, 0, 0, 0, 0, 0, 0, 0};
    t_next = t_end;
  }
  __device__ void flush_large() {
    for (uint64_t t = b_next + __lane_id(); t < b_end && t < tcap_big; t += 64)
      out[tcap + t] = Pending{0, 0, 0, 0, 0, 0, 0, 0, 0};
    b_next = b_end;
  }
  __device__ void flush() {
    flush_small();
    flush_large();
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

// size class of a row: ceil(log2 d) for 1 <= d <= 64 (0..6), 7 up to kMidMax
// edges, 8 above, none without edges
constexpr uint32_t kMidMax = 1024;
__device__ __forceinline__ uint32_t row_class(uint64_t d) {
  return d == 0 ? ~0u : (d <= 64 ? guide::ceil_log2(d) : (d <= kMidMax ? 7u : 8u));
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
  for (uint32_t i = threadIdx.x; i < kGuideLevels + 2; i += blockDim.x) ctl->tables[i] = ctl->big[i] = 0;
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

// Orders this wave's LDS and global writes before its later reads by
// other lanes of the workgroup (here: of the wave itself).
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// First candidate at or after a whose threshold is above x, by doubling
// steps from a and then binary search (the answer is usually near a).
template <typename Th>
__device__ __forceinline__ uint32_t containing_from(const Th& T, uint32_t a, uint32_t last, uint64_t x) {
  uint32_t lo = a, hi = a, step = 1;
  while (hi < last && T(hi) <= x) {  // every index below hi + 1 is at most x
    lo = hi + 1;
    hi = last - lo > step ? lo + step : last;
    step <<= 1;
  }
  return guide::containing(T, lo, hi, x);
}
// Rows of 65 to kMidMax edges: one wave per row. The row's total and its
// edge records (several edges' loads in flight per lane), then its
// prefixes and thresholds 64 edges at a time (the thresholds also staged in
// the wave's LDS), then its 64 to 512 entries, lane k taking entries k,
// k + 64, ... so that the wave's writes are contiguous: candidates by binary
// search over the staged thresholds and a doubling search from there.
__global__ void __launch_bounds__(kThreads) k_guide_mid(const uint32_t* __restrict__ rows, uint64_t count,
                                                        const uint64_t* __restrict__ off,
                                                        const uint32_t* __restrict__ col,
                                                        const uint32_t* __restrict__ w, const Head* __restrict__ head,
                                                        uint32_t n, uint64_t* T, uint4* erec, Entry* __restrict__ ent,
                                                        Alloc alloc) {
  __shared__ uint64_t sT[kThreads / 64][kMidMax];
  const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
  uint64_t* st = sT[wv];
  const uint64_t waves = static_cast<uint64_t>(gridDim.x) * (kThreads / 64);
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads / 64) + wv; r < count; r += waves) {  // wave-uniform
    const uint32_t u = rows[r];
    const uint64_t a = off[u];
    const uint32_t d = static_cast<uint32_t>(off[u + 1] - a);  // 65 .. kMidMax
    uint64_t part = 0;
#pragma unroll 4
    for (uint32_t j = lane; j < d; j += 64) {
      part += w[a + j];
      erec[a + j] = edge_record(head, n, col[a + j], u);
    }
    const uint64_t W = wave_sum_u64(part);
    uint64_t carry = 0;
    for (uint32_t j0 = 0; j0 < d; j0 += 64) {
      const uint32_t j = j0 + lane;
      const uint64_t x = j < d ? w[a + j] : 0u;
      const uint64_t inc = wave_inclusive_scan_u64(x);
      const uint64_t P = carry + inc;
      carry += __shfl(static_cast<unsigned long long>(inc), 63, 64);
      if (j < d) {
        const uint64_t t = j + 1 < d && P < W ? guide::threshold(P, W) : ~0ull;
        T[a + j] = t;
        st[j] = t;
      }
    }
    group_sync();  // the staged thresholds and the row's records, visible to the wave
    if (W != 0) {  // wave-uniform
      auto th = [&](uint32_t j) -> uint64_t { return st[j]; };
      const ERec rec{erec + a};
      Entry* row_ent = ent + head[u].base;
      const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
      const uint32_t last = d - 1, nb = 1u << kb;  // nb = 64 .. 512
      for (uint32_t b = lane; b < nb; b += 64) {  // wave-uniform: nb is a multiple of 64
        uint64_t blo, bhi;
        guide::row_bucket(kb, b, &blo, &bhi);
        const uint32_t c0 = guide::containing(th, 0u, last, blo);
        const uint32_t c1 = containing_from(th, c0, last, bhi);
        const uint64_t t0 = c1 > c0 ? th(c0) : 0, t1 = c1 > c0 ? th(c1 - 1) : 0;
        const Cand L = rec(c0), R = rec(c1);
        const Cand M = c1 > c0 + 1 ? rec(c0 + 1) : L;
        write_entry(alloc, true, row_ent + b, c0, c1, t0, t1, L, M, R, a, u);
      }
    }
    group_sync();  // the next row's staging reuses the LDS words
  }
  alloc.flush();
}

// Long rows (more than kMidMax edges) are cut into tiles of kTile edges
// (listed at creation: (row, tile)), so that a hub's thresholds spread over
// many blocks: the tiles' weight sums, then each row's running offsets and
// total over its tiles, then each tile's prefixes, thresholds and edge
// records. Their entries come after, from k_guide_runs.
constexpr uint32_t kTile = kThreads * 4;
__device__ __forceinline__ void tile_span(const uint64_t* __restrict__ off, uint2 rt, uint64_t* a, uint64_t* d,
                                          uint64_t* j0, uint64_t* len) {
  *a = off[rt.x];
  *d = off[rt.x + 1] - *a;
  *j0 = static_cast<uint64_t>(rt.y) * kTile;
  *len = *d - *j0 < kTile ? *d - *j0 : kTile;
}

__global__ void __launch_bounds__(kThreads) k_tile_sums(const uint2* __restrict__ tiles, uint64_t count,
                                                        const uint64_t* __restrict__ off,
                                                        const uint32_t* __restrict__ w, uint64_t* __restrict__ tsum) {
  __shared__ uint64_t lds[kThreads / 64];
  for (uint64_t q = blockIdx.x; q < count; q += gridDim.x) {  // block-uniform
    uint64_t a, d, j0, len;
    tile_span(off, tiles[q], &a, &d, &j0, &len);
    uint64_t part = 0;
    for (uint64_t j = threadIdx.x; j < len; j += kThreads) part += w[a + j0 + j];
    uint64_t total = 0;
    block_exclusive_scan_u64<kThreads>(part, lds, &total);
    if (threadIdx.x == 0) tsum[q] = total;
  }
}

// one thread per long row: its tiles' offsets within the row, and the total
__global__ void k_tile_offsets(const uint32_t* __restrict__ rows, uint64_t count, const uint64_t* __restrict__ off,
                               const uint64_t* __restrict__ first, const uint64_t* __restrict__ tsum,
                               uint64_t* __restrict__ toff, uint64_t* __restrict__ ttot) {
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < count;
       r += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t u = rows[r];
    const uint64_t d = off[u + 1] - off[u];
    const uint64_t n = (d + kTile - 1) / kTile, f = first[r];
    uint64_t acc = 0;
    for (uint64_t k = 0; k < n; ++k) {
      toff[f + k] = acc;
      acc += tsum[f + k];
    }
    for (uint64_t k = 0; k < n; ++k) ttot[f + k] = acc;
  }
}

__global__ void __launch_bounds__(kThreads) k_tile_thresholds(const uint2* __restrict__ tiles, uint64_t count,
                                                              const uint64_t* __restrict__ off,
                                                              const uint32_t* __restrict__ col,
                                                              const uint32_t* __restrict__ w,
                                                              const Head* __restrict__ head, uint32_t n,
                                                              const uint64_t* __restrict__ toff,
                                                              const uint64_t* __restrict__ ttot, uint64_t* T,
                                                              uint4* erec) {
  __shared__ uint64_t lds[kThreads / 64];
  for (uint64_t q = blockIdx.x; q < count; q += gridDim.x) {  // block-uniform
    const uint2 rt = tiles[q];
    uint64_t a, d, j0, len;
    tile_span(off, rt, &a, &d, &j0, &len);
    const uint64_t W = ttot[q];
    const uint64_t base = j0 + threadIdx.x * 4ull;
    uint64_t v[4];
    uint64_t local = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t j = base + k;
      local += j < j0 + len ? w[a + j] : 0u;
      v[k] = local;
    }
    uint64_t total;
    const uint64_t excl = block_exclusive_scan_u64<kThreads>(local, lds, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t j = base + k;
      if (j < j0 + len) {
        const uint64_t P = toff[q] + excl + v[k];
        T[a + j] = j + 1 < d && P < W ? guide::threshold(P, W) : ~0ull;
        erec[a + j] = edge_record(head, n, col[a + j], rt.x);
      }
    }
  }
}

// Entries of the long rows: a group of kRun lanes per run of kRun
// consecutive entries of one row (runs listed at creation: (row, first
// entry)), lane k filling entry k, so that a group writes its run's entries
// as one contiguous stretch. The group first narrows, together, the
// candidate range holding the run's draws: each round its 16 lanes read 16
// evenly spaced thresholds of the range at once and keep the part between
// the last one at or below the run's first draw and the first one above its
// last draw, so a row of 2^17 edges takes about four rounds of loads where
// a binary search takes seventeen dependent ones. When at most 32 thresholds
// remain, they sit two per lane and each lane finds its bucket's candidates
// by shuffles; otherwise (light edges crowding the run's draws) each lane
// searches the narrowed range itself.
constexpr uint32_t kRun = 16;
constexpr uint32_t kRunWin = 2 * kRun;
constexpr uint32_t kRunRounds = 6;
__global__ void __launch_bounds__(kThreads) k_guide_runs(const uint2* __restrict__ runs, uint64_t count,
                                                         const uint64_t* __restrict__ off, const Head* __restrict__ head,
                                                         const uint64_t* __restrict__ T, const uint4* __restrict__ erec,
                                                         Entry* __restrict__ ent, Alloc alloc) {
  const uint32_t gi = __lane_id() & (kRun - 1), gb = __lane_id() & ~(kRun - 1);
  const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * kThreads) / kRun;
  // the group's lanes of a wave-wide ballot
  auto group_bits = [&](uint64_t m) { return static_cast<uint32_t>((m >> gb) & ((1u << kRun) - 1)); };
  for (uint64_t q = (blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x) / kRun; __ballot(q < count) != 0;
       q += groups) {  // wave-uniform loop
    bool act = q < count;
    const uint2 rb = act ? runs[q] : make_uint2(0, 0);
    const uint32_t u = rb.x;
    const uint64_t a = act ? off[u] : 0;
    const uint32_t d = act ? static_cast<uint32_t>(off[u + 1] - a) : 1u;
    act = act && d > 1;
    const uint32_t kb = guide::table_bits(guide::ceil_log2(d));
    const uint32_t last = d - 1;
    const Thr th{T + a};
    const ERec rec{erec + a};
    const uint32_t b = rb.y + gi;  // < 2^kb: runs tile the table (2^kb >= 1024 here)
    uint64_t blo = 0, bhi = 0, x0 = 0, x1 = 0, unused = 0;
    guide::row_bucket(kb, b, &blo, &bhi);
    guide::row_bucket(kb, rb.y, &x0, &unused);            // the run's first draw
    guide::row_bucket(kb, rb.y + kRun - 1, &unused, &x1);  // and its last
    // [lo, hi]: holds the candidates of every draw in [x0, x1] (thresholds
    // lo .. hi - 1 remain to be placed)
    uint32_t lo = 0, hi = last;
    bool go = act;  // group-uniform
#pragma unroll 1
    for (uint32_t round = 0; round < kRunRounds; ++round) {
      if (__ballot(go) == 0) break;  // wave-uniform
      const uint32_t span = hi - lo;
      go = go && span > kRunWin;
      // probe i at lo + span (i + 1) / 17: strictly increasing, all below hi
      const uint32_t p = lo + static_cast<uint32_t>(static_cast<uint64_t>(span) * (gi + 1) / (kRun + 1));
      const uint64_t t = go ? th(p) : 0;
      const uint32_t n0 = static_cast<uint32_t>(__popc(group_bits(__ballot(go && t <= x0))));
      const uint32_t n1 = static_cast<uint32_t>(__popc(group_bits(__ballot(go && t <= x1))));
      if (go) {
        // probes below n0 are at or below x0, those from n1 on above x1
        const uint32_t nlo = n0 ? lo + static_cast<uint32_t>(static_cast<uint64_t>(span) * n0 / (kRun + 1)) + 1 : lo;
        const uint32_t nhi =
            n1 < kRun ? lo + static_cast<uint32_t>(static_cast<uint64_t>(span) * (n1 + 1) / (kRun + 1)) : hi;
        go = nlo != lo || nhi != hi;  // no progress: the lanes search from here
        lo = nlo;
        hi = nhi;
      }
    }
    const uint32_t span = hi - lo;
    const bool win = span <= kRunWin;  // group-uniform
    // the remaining thresholds: lo + i in lane i % 16, register i / 16
    const uint64_t wa = act && win && gi < span ? th(lo + gi) : ~0ull;
    const uint64_t wb = act && win && gi + kRun < span ? th(lo + kRun + gi) : ~0ull;
    uint32_t l0 = 0, h0 = win ? span : 0, l1 = 0, h1 = h0;
#pragma unroll
    for (uint32_t it = 0; it < 6; ++it) {  // ranges of at most 33 counts
      const uint32_t m0 = (l0 + h0) >> 1, m1 = (l1 + h1) >> 1;
      const uint64_t y0a = __shfl(static_cast<unsigned long long>(wa), static_cast<int>(m0 & (kRun - 1)), kRun);
      const uint64_t y0b = __shfl(static_cast<unsigned long long>(wb), static_cast<int>(m0 & (kRun - 1)), kRun);
      const uint64_t y1a = __shfl(static_cast<unsigned long long>(wa), static_cast<int>(m1 & (kRun - 1)), kRun);
      const uint64_t y1b = __shfl(static_cast<unsigned long long>(wb), static_cast<int>(m1 & (kRun - 1)), kRun);
      const uint64_t y0 = m0 < kRun ? y0a : y0b, y1 = m1 < kRun ? y1a : y1b;
      if (l0 < h0) {
        if (y0 <= blo) l0 = m0 + 1;
        else h0 = m0;
      }
      if (l1 < h1) {
        if (y1 <= bhi) l1 = m1 + 1;
        else h1 = m1;
      }
    }
    uint32_t c0 = 0, c1 = 0;
    uint64_t t0 = 0, t1 = 0;
    Cand L{}, M{}, R{};
    if (act) {
      if (win) {
        c0 = lo + l0;
        c1 = lo + l1;
      } else {
        c0 = guide::containing(th, lo, hi, blo);
        c1 = containing_from(th, c0, hi, bhi);
      }
      if (c1 > c0) {
        t0 = th(c0);
        t1 = th(c1 - 1);
      }
      L = rec(c0);
      R = rec(c1);
      M = c1 > c0 + 1 ? rec(c0 + 1) : L;
    }
    write_entry(alloc, act, ent + (act ? head[u].base + b : 0u), c0, c1, t0, t1, L, M, R, a, u);
  }
  alloc.flush();
}

// tiles of each long row, and their list (each row's tiles together; the
// first tile of row r at first[r])
__global__ void k_tile_counts(const uint32_t* __restrict__ rows, uint64_t count, const uint64_t* __restrict__ off,
                              uint32_t* __restrict__ flag) {
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < count;
       r += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t u = rows[r];
    flag[r] = static_cast<uint32_t>((off[u + 1] - off[u] + kTile - 1) / kTile);
  }
}
__global__ void k_tile_fill(const uint32_t* __restrict__ rows, uint64_t count, const uint32_t* __restrict__ flag,
                            const uint64_t* __restrict__ scan, uint2* __restrict__ tiles, uint64_t* __restrict__ first) {
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < count;
       r += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    first[r] = scan[r];
    for (uint32_t i = 0; i < flag[r]; ++i) tiles[scan[r] + i] = make_uint2(rows[r], i);
  }
}

// runs of each long row (2^kb / kRun: kb >= 10 there)
__global__ void k_run_counts(const uint32_t* __restrict__ rows, uint64_t count, const uint64_t* __restrict__ off,
                             uint32_t* __restrict__ flag) {
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < count;
       r += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t u = rows[r];
    const uint64_t d = off[u + 1] - off[u];
    flag[r] = (1u << guide::table_bits(guide::ceil_log2(d))) / kRun;
  }
}
__global__ void k_run_fill(const uint32_t* __restrict__ rows, uint64_t count, const uint32_t* __restrict__ flag,
                           const uint64_t* __restrict__ scan, uint2* __restrict__ runs) {
  for (uint64_t r = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; r < count;
       r += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    for (uint32_t i = 0; i < flag[r]; ++i) runs[scan[r] + i] = make_uint2(rows[r], i * kRun);
}

// The child tables of one level, a group of GL lanes per table: 8 for the
// small list (fewer than kLargeThr thresholds between the candidates: about
// six tables in seven, most of 2 to 8 entries), 16 for the large list.
// The group holds the table's thresholds in its lanes when there are fewer
// than GL of them, and each lane fills one entry at a time: candidates by
// binary search over the group's thresholds through lane shuffles (over the
// row's thresholds in memory for larger tables), records from the edge
// records. Tables of the next level go to the other lists.
template <uint32_t GL, bool kLarge>
__global__ void __launch_bounds__(kThreads) k_guide_level(const uint64_t* __restrict__ T,
                                                          const uint4* __restrict__ erec, Entry* __restrict__ ent,
                                                          const Pending* lists, uint32_t level, Alloc alloc) {
  constexpr uint32_t kIters = GL == 8 ? 3u : 4u;  // binary-search steps over at most GL positions
  // not restrict: the loads through it must stay on their side of the
  // barriers below
  const Pending* in = kLarge ? lists + alloc.tcap : lists;
  uint32_t count = kLarge ? alloc.ctl->big[level] : alloc.ctl->tables[level];
  const uint32_t room = kLarge ? alloc.tcap_big : alloc.tcap;
  if (count > room) count = room;
  const uint32_t gi = __lane_id() & (GL - 1);
  const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * kThreads) / GL;
  if (count == 0) return;
  // The part of the group's next table that its loads need (row offset and
  // candidate range, bytes 16..31 of the descriptor) is loaded one iteration
  // ahead; the rest of the descriptor then loads beside the table's
  // thresholds and records. Every load of an iteration is issued on every
  // path (inactive lanes read index 0 and drop the value), so the wait for
  // this table's values below leaves the prefetch in flight.
  static_assert(sizeof(Pending) == 48, "descriptor layout");
  uint64_t t = (blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x) / GL;
  uint4 pn = reinterpret_cast<const uint4*>(in + (t < count ? t : 0))[1];
  bool pn_ok = t < count;
  __builtin_amdgcn_s_waitcnt(0);
  for (; __ballot(t < count) != 0; t += groups) {  // wave-uniform loop
    const uint64_t off = pn_ok ? (static_cast<uint64_t>(pn.y) << 32) | pn.x : 0;
    const uint32_t pa = pn_ok ? pn.z : 0, pb = pn_ok ? pn.w : 0;
    const uint32_t nthr = pb - pa;  // thresholds between the candidates
    // small tables: lane j holds threshold a + j and the record of candidate a + j
    const bool small = nthr < GL;
    const bool tv_ok = gi < nthr && small, rv_ok = gi <= nthr && small;
    const Pending pl = in[pn_ok ? t : 0];
    const uint64_t Tl = T[tv_ok ? off + pa + gi : 0];
    const uint4 Rl = erec[rv_ok ? off + pa + gi : 0];
    // keep the prefetch behind these loads (an empty statement the compiler
    // may not move loads across; it emits nothing)
    __asm__ __volatile__("" ::: "memory");
    const bool was_ok = pn_ok;
    const uint64_t tn = t + groups;
    pn = reinterpret_cast<const uint4*>(in + (tn < count ? tn : 0))[1];
    pn_ok = tn < count;
    __asm__ __volatile__("" ::: "memory");
    // this table's loads complete (vmcnt <= 1: the prefetch may still be in
    // flight; the compiler adds whatever more a use needs)
    __builtin_amdgcn_s_waitcnt(0xF71);
    const Pending p = was_ok ? pl : Pending{};  // tables that found no room have no buckets
    const uint64_t Tv = tv_ok ? Tl : ~0ull;
    const uint4 Rv = rv_ok ? Rl : make_uint4(0, 0, 0, 0);
    const uint32_t most = wave_max_u32((p.nbk + GL - 1) / GL);
    const Thr th{T + p.off};
    const ERec rec{erec + p.off};
    // at least one pass (with no active lane when the wave has no buckets),
    // so that this table's loads are used on every path and stay ahead of
    // the prefetch
    uint32_t k = 0;
    do {  // wave-uniform
      const uint32_t i = k * GL + gi;
      const bool act = i < p.nbk;
      uint64_t blo = 0, bhi = 0;
      if (act) guide::child_bucket(p.origin, p.end, p.sh, i, &blo, &bhi);
      // thresholds <= blo and <= bhi among the group's (every lane shuffles)
      uint32_t l0 = 0, h0 = small ? nthr : 0, l1 = 0, h1 = h0;
#pragma unroll
      for (uint32_t it = 0; it < kIters; ++it) {  // ranges of at most GL positions
        const uint32_t m0 = (l0 + h0) >> 1, m1 = (l1 + h1) >> 1;
        const uint64_t x0 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(m0 & (GL - 1)), GL);
        const uint64_t x1 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(m1 & (GL - 1)), GL);
        if (l0 < h0) {
          if (x0 <= blo) l0 = m0 + 1;
          else h0 = m0;
        }
        if (l1 < h1) {
          if (x1 <= bhi) l1 = m1 + 1;
          else h1 = m1;
        }
      }
      uint32_t j0 = l0, j1 = l1;  // candidates relative to a
      if (act && !small) {
        j0 = guide::containing(th, p.a, p.b, blo) - p.a;
        j1 = guide::containing(th, p.a, p.b, bhi) - p.a;
      }
      const uint32_t jm = j1 > j0 + 1 ? j0 + 1 : j0;
      const uint64_t y0 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>(j0 & (GL - 1)), GL);
      const uint64_t y1 = __shfl(static_cast<unsigned long long>(Tv), static_cast<int>((j1 - 1) & (GL - 1)), GL);
      Cand L{__shfl(Rv.x, static_cast<int>(j0 & (GL - 1)), GL), __shfl(Rv.y, static_cast<int>(j0 & (GL - 1)), GL),
             __shfl(Rv.z, static_cast<int>(j0 & (GL - 1)), GL)};
      Cand M{__shfl(Rv.x, static_cast<int>(jm & (GL - 1)), GL), __shfl(Rv.y, static_cast<int>(jm & (GL - 1)), GL),
             __shfl(Rv.z, static_cast<int>(jm & (GL - 1)), GL)};
      Cand R{__shfl(Rv.x, static_cast<int>(j1 & (GL - 1)), GL), __shfl(Rv.y, static_cast<int>(j1 & (GL - 1)), GL),
             __shfl(Rv.z, static_cast<int>(j1 & (GL - 1)), GL)};
      const uint32_t c0 = p.a + j0, c1 = p.a + j1;
      uint64_t t0 = 0, t1 = 0;
      if (act) {
        if (c1 > c0) {
          t0 = small ? y0 : th(c0);
          t1 = small ? y1 : th(c1 - 1);
        }
        if (!small) {
          L = rec(c0);
          R = rec(c1);
          M = c1 > c0 + 1 ? rec(c0 + 1) : L;
        }
      }
      write_entry(alloc, act, ent + (act ? p.base + i : 0u), c0, c1, t0, t1, L, M, R, p.off, p.row);
    } while (++k < most);
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

hipError_t launch_guide_runs_count(fppr_graph* g, hipStream_t s) {
  const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
  if (!nlong) return hipSuccess;
  hipLaunchKernelGGL(k_run_counts, dim3(grid_for(nlong)), dim3(kThreads), 0, s, g->gclass + g->gclass_off[8], nlong,
                     g->off, g->flag);
  return launch_scan_u32(g->flag, g->scan, nlong, g->scan_blocks, reinterpret_cast<uint64_t*>(g->d_err + 14), s);
}

hipError_t launch_guide_tiles_count(fppr_graph* g, hipStream_t s) {
  const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
  if (!nlong) return hipSuccess;
  hipLaunchKernelGGL(k_tile_counts, dim3(grid_for(nlong)), dim3(kThreads), 0, s, g->gclass + g->gclass_off[8], nlong,
                     g->off, g->flag);
  return launch_scan_u32(g->flag, g->scan, nlong, g->scan_blocks, reinterpret_cast<uint64_t*>(g->d_err + 14), s);
}

hipError_t launch_guide_tiles_fill(fppr_graph* g, hipStream_t s) {
  const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
  if (!nlong) return hipSuccess;
  hipLaunchKernelGGL(k_tile_fill, dim3(grid_for(nlong)), dim3(kThreads), 0, s, g->gclass + g->gclass_off[8], nlong,
                     g->flag, g->scan, g->gtiles, g->gtile_first);
  return hipGetLastError();
}

hipError_t launch_guide_runs_fill(fppr_graph* g, hipStream_t s) {
  const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
  if (!nlong) return hipSuccess;
  hipLaunchKernelGGL(k_run_fill, dim3(grid_for(nlong)), dim3(kThreads), 0, s, g->gclass + g->gclass_off[8], nlong,
                     g->flag, g->scan, g->gruns);
  return hipGetLastError();
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
  a.tcap_big = g->g_tcap_big;
  a.next_level = next_level;
  a.max_level = max_level;
  a.err = g->d_err;
  return a;
}
template <uint32_t CL>
hipError_t launch_rows(fppr_graph* g, const Alloc& p, hipStream_t s) {
  const uint64_t count = g->gclass_off[CL + 1] - g->gclass_off[CL];
  if (!count) return hipSuccess;
  uint32_t blocks = 0;  // few waves: few partial chunks
  const hipError_t e = resident_grid(k_guide_rows<CL>, count << CL, 2048u, &blocks);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_guide_rows<CL>, dim3(blocks), dim3(kThreads), 0, s,
                     g->gclass + g->gclass_off[CL], count, g->off, g->col, g->w, g->ghead, g->n, g->gT, g->gerec,
                     g->gent, p);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_guide_build(fppr_graph* g, bool bases, uint32_t levels, hipStream_t s) {
  hipLaunchKernelGGL(k_guide_heads, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off,
                     bases ? g->scan : nullptr, g->cls, g->n, g->ghead);
  hipLaunchKernelGGL(k_guide_ctl_init, dim3(1), dim3(64), 0, s, g->gctl, g->g_entries1);
  const Alloc p = allocator(g, 2, levels);
  // Rows of more than 1024 edges on the graph's side stream (when it has
  // one: graphs whose all-nodes runs split off the nodes without out-edges),
  // after the heads and counters above and beside the shorter rows on s,
  // which waits for them. No stream of its own: every stream a process
  // creates takes a hardware queue slot, and more of them made the queues
  // the serving streams share. A rebuild recorded into a stream capture
  // keeps everything on s.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return e;
  const bool fork = cs == hipStreamCaptureStatusNone && g->side != nullptr;
  std::unique_lock<std::mutex> lk(g->side_mu, std::defer_lock);
  if (fork) {
    lk.lock();
    e = hipEventRecord(g->fork_ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(g->side, g->fork_ev, 0);
    if (e != hipSuccess) return e;
  }
  hipStream_t s_long = fork ? g->side : s;
  if ((e = launch_rows<0>(g, p, s)) != hipSuccess || (e = launch_rows<1>(g, p, s)) != hipSuccess ||
      (e = launch_rows<2>(g, p, s)) != hipSuccess || (e = launch_rows<3>(g, p, s)) != hipSuccess ||
      (e = launch_rows<4>(g, p, s)) != hipSuccess || (e = launch_rows<5>(g, p, s)) != hipSuccess ||
      (e = launch_rows<6>(g, p, s)) != hipSuccess)
    return e;
  const uint64_t nmid = g->gclass_off[8] - g->gclass_off[7];
  uint32_t mid_blocks = 0;
  if (nmid && (e = resident_grid(k_guide_mid, nmid * 64, 2048u, &mid_blocks)) != hipSuccess) return e;
  if (nmid)
    hipLaunchKernelGGL(k_guide_mid, dim3(mid_blocks), dim3(kThreads), 0, s,
                       g->gclass + g->gclass_off[7], nmid, g->off, g->col, g->w, g->ghead, g->n, g->gT, g->gerec,
                       g->gent, p);
  const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
  if (nlong) {
    hipStream_t t = s_long;
    const uint32_t tb = static_cast<uint32_t>(std::min<uint64_t>(g->n_tiles, 8192));
    hipLaunchKernelGGL(k_tile_sums, dim3(tb), dim3(kThreads), 0, t, g->gtiles, g->n_tiles, g->off, g->w, g->gtsum);
    hipLaunchKernelGGL(k_tile_offsets, dim3(grid_for(nlong)), dim3(kThreads), 0, t, g->gclass + g->gclass_off[8],
                       nlong, g->off, g->gtile_first, g->gtsum, g->gtoff, g->gttot);
    hipLaunchKernelGGL(k_tile_thresholds, dim3(tb), dim3(kThreads), 0, t, g->gtiles, g->n_tiles, g->off, g->col,
                       g->w, g->ghead, g->n, g->gtoff, g->gttot, g->gT, g->gerec);
    uint32_t run_blocks = 0;
    if ((e = resident_grid(k_guide_runs, g->n_runs * kRun, 2048u, &run_blocks)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_guide_runs, dim3(run_blocks), dim3(kThreads), 0, t, g->gruns, g->n_runs, g->off, g->ghead,
                       g->gT, g->gerec, g->gent, p);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (fork) {
    e = hipEventRecord(g->join_ev, g->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, g->join_ev, 0);
  }
  return e;
}

hipError_t launch_guide_level(fppr_graph* g, uint32_t level, uint32_t levels, hipStream_t s) {
  const guide::Pending* in = g->gtab[level & 1u ? 1 : 0];
  const Alloc a = allocator(g, level + 1, levels);
  // the table counts are on the device: as many blocks as fit
  constexpr uint64_t kAll = 2048ull * kThreads;
  uint32_t b8 = 0, b16 = 0;
  hipError_t e = resident_grid(k_guide_level<8, false>, kAll, 2048u, &b8);
  if (e == hipSuccess) e = resident_grid(k_guide_level<16, true>, kAll, 2048u, &b16);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_guide_level<8, false>), dim3(b8), dim3(kThreads), 0, s, g->gT, g->gerec, g->gent, in, level, a);
  hipLaunchKernelGGL((k_guide_level<16, true>), dim3(b16), dim3(kThreads), 0, s, g->gT, g->gerec, g->gent, in, level,
                     a);
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
