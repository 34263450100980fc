// Guide tables for the weighted pick: the guide-table method of inverse-
// transform sampling (Chen and Asau, 1974) turned around so that the table is
// indexed by the draw itself.
//
// The pick of Sec. 2.1 on integers: a row with inclusive weight prefixes
// P[0] < ... < P[d-1] = W takes the 64-bit draw D, forms X = floor(D W / 2^64)
// and returns the first edge j with P[j] > X. Since P[j] is an integer,
// P[j] > floor(D W / 2^64) holds exactly when D < T[j] with
//   T[j] = ceil(P[j] 2^64 / W),
// so edge j owns the draws [T[j-1], T[j]) (T[-1] = 0, T[d-1] = 2^64) and the
// pick becomes a search of D among the row's thresholds T[0..d-2], with no
// need for W at walk time.
//
// A row's table has 2^kb entries (kb = lg - 1 for lg = ceil(log2 d) >= 1,
// else 0), entry b covering the draws whose top kb bits are b. An entry names
// up to three candidates: draws below `lo` go to L, draws at or above `hi` to
// R, the rest to M. When more than three edges meet an entry's draws, M
// points instead to a child table over [lo, hi) that splits it by the draw's
// next bits (bucket i of a child with origin o and shift sh holds the draws
// o + i 2^sh .. o + (i+1) 2^sh - 1), and so on; bucket widths shrink by at
// least one bit per level, so every path ends. Every candidate carries the
// destination's own record (id with its class tag, the first entry of its
// table and its lg), so the walk that arrives there starts its next pick
// from that record with one 64-byte read. The result is exactly the edge the
// flat search returns, for every draw.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FPPR_GUIDE_FN __host__ __device__ __forceinline__
#else
#define FPPR_GUIDE_FN inline
#endif

namespace fppr {
namespace guide {

// One table entry: 64 bytes, so it never straddles a 128-byte line. A walk
// reads it with a lane pair: bytes 0..31 (thresholds, L and M) and 32..47
// (R and the packed lg / shift values).
struct alignas(64) Entry {
  uint64_t lo, hi;
  uint32_t l_id, l_base;
  uint32_t m_id, m_base;  // with kChild: m_base = the child's first entry
  uint32_t r_id, r_base;
  uint32_t meta;          // l_lg | m_lg << 8 | r_lg << 16 | kChild; with kChild m_lg is the child's shift
  uint32_t pad[5];
};
static_assert(sizeof(Entry) == 64, "one half line per entry");
constexpr uint32_t kChild = 1u << 24;

// Per node: the first entry of its table and lg | class tag << 8.
struct Head {
  uint32_t base;
  uint32_t meta;
};

// A child table still to be filled: candidates [a, b] of row `row` (edges
// off .. off + d - 1), draws [origin, end), 2^sh draws per bucket, nbk
// buckets from entry `base`.
struct Pending {
  uint64_t origin, end, off;
  uint32_t a, b, row, sh, nbk, base;
};

FPPR_GUIDE_FN uint32_t clz64(uint64_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return static_cast<uint32_t>(__clzll(static_cast<long long>(x)));
#else
  return static_cast<uint32_t>(__builtin_clzll(x));
#endif
}
FPPR_GUIDE_FN uint32_t bit_length(uint64_t x) { return x ? 64u - clz64(x) : 0u; }
FPPR_GUIDE_FN uint32_t ceil_log2(uint64_t d) { return d <= 1 ? 0u : bit_length(d - 1); }
// table size exponent of a row with lg = ceil(log2 d): 2^kb >= d / 2
FPPR_GUIDE_FN uint32_t table_bits(uint32_t lg) { return lg ? lg - 1 : 0u; }
// entry of the row table that draw D falls in (kb <= 62): its top kb bits
FPPR_GUIDE_FN uint32_t top_bits(uint64_t D, uint32_t kb) {
  return static_cast<uint32_t>((D >> 1) >> (63 - kb));
}

// floor((u1 * 2^64 + u0) / v) for u1 < v, so that the quotient fits in 64
// bits; the remainder to *rem. Knuth's long division (TAOCP vol. 2, 4.3.1,
// Algorithm D) with 32-bit digits: v is normalised so its top bit is set,
// each quotient digit is estimated from the leading digits and corrected at
// most twice.
FPPR_GUIDE_FN uint64_t div128(uint64_t u1, uint64_t u0, uint64_t v, uint64_t* rem) {
  const uint64_t b = 1ull << 32;
  const uint32_t s = clz64(v);
  v <<= s;
  const uint64_t vn1 = v >> 32, vn0 = v & 0xFFFFFFFFull;
  const uint64_t un32 = s ? (u1 << s) | (u0 >> (64 - s)) : u1;
  const uint64_t un10 = u0 << s;
  const uint64_t un1 = un10 >> 32, un0 = un10 & 0xFFFFFFFFull;
  uint64_t q1 = un32 / vn1;
  uint64_t rhat = un32 - q1 * vn1;
  while (q1 >= b || q1 * vn0 > ((rhat << 32) | un1)) {
    q1 -= 1;
    rhat += vn1;
    if (rhat >= b) break;
  }
  const uint64_t un21 = (un32 << 32) + un1 - q1 * v;  // exact: the partial remainder is below v
  uint64_t q0 = un21 / vn1;
  rhat = un21 - q0 * vn1;
  while (q0 >= b || q0 * vn0 > ((rhat << 32) | un0)) {
    q0 -= 1;
    rhat += vn1;
    if (rhat >= b) break;
  }
  if (rem) *rem = ((un21 << 32) + un0 - q0 * v) >> s;
  return (q1 << 32) | q0;
}

// T = ceil(P 2^64 / W) for 1 <= P < W <= 2^63: the first draw that picks an
// edge after the one whose inclusive prefix is P.
FPPR_GUIDE_FN uint64_t threshold(uint64_t P, uint64_t W) {
  uint64_t r = 0;
  const uint64_t q = div128(P, 0, W, &r);
  return q + (r != 0 ? 1u : 0u);
}

// Candidate holding draw x among candidates [a, b] separated by thresholds
// T(a) < ... < T(b-1): a plus the number of those thresholds <= x.
template <class Th>
FPPR_GUIDE_FN uint32_t containing(const Th& T, uint32_t a, uint32_t b, uint64_t x) {
  uint32_t lo = a, hi = b;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (T(mid) <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Layout of the child table over the draws [lo, hi) of an entry whose middle
// holds mc >= 2 candidates: the shift sh is the smallest with fewer than
// 2^ceil(log2 mc) buckets of 2^sh draws; returns the bucket count.
FPPR_GUIDE_FN uint32_t child_shape(uint64_t lo, uint64_t hi, uint32_t mc, uint32_t* sh) {
  const uint64_t span = hi - lo;  // >= mc >= 2: every candidate owns at least one draw
  const uint32_t kc = ceil_log2(mc);
  const uint32_t bl = bit_length(span - 1);
  *sh = bl > kc ? bl - kc : 0u;
  return static_cast<uint32_t>(((span - 1) >> *sh) + 1);
}

// Draws of bucket i of a child table: [o + i 2^sh, min(o + (i+1) 2^sh, end) - 1].
FPPR_GUIDE_FN void child_bucket(uint64_t o, uint64_t end, uint32_t sh, uint32_t i, uint64_t* blo, uint64_t* bhi) {
  *blo = o + (static_cast<uint64_t>(i) << sh);
  const uint64_t room = end - 1 - *blo;
  const uint64_t w = (1ull << sh) - 1;  // sh < 64: a child is narrower than its parent's bucket
  *bhi = *blo + (w < room ? w : room);
}

// Draws of entry b of a row table with 2^kb entries.
FPPR_GUIDE_FN void row_bucket(uint32_t kb, uint32_t b, uint64_t* blo, uint64_t* bhi) {
  if (kb == 0) {
    *blo = 0;
    *bhi = ~0ull;
    return;
  }
  *blo = static_cast<uint64_t>(b) << (64 - kb);
  *bhi = *blo + ((1ull << (64 - kb)) - 1);
}

// Thresholds of the entry whose draws meet candidates c0 .. c1, from
// t0 = T(c0) and t1 = T(c1 - 1) (read only when the entry has more than one
// candidate): returns the number of middle candidates that go to a child
// table (0 when the entry resolves every draw itself).
FPPR_GUIDE_FN uint32_t entry_bounds(uint32_t c0, uint32_t c1, uint64_t t0, uint64_t t1, uint64_t* lo, uint64_t* hi) {
  const uint32_t count = c1 - c0 + 1;
  if (count == 1) {  // every draw to R
    *lo = 0;
    *hi = 0;
    return 0;
  }
  *lo = t0;
  *hi = count == 2 ? t0 : t1;
  return count <= 3 ? 0u : count - 2;
}
template <class Th>
FPPR_GUIDE_FN uint32_t entry_shape(const Th& T, uint32_t c0, uint32_t c1, uint64_t* lo, uint64_t* hi) {
  if (c1 == c0) return entry_bounds(c0, c1, 0, 0, lo, hi);
  return entry_bounds(c0, c1, T(c0), T(c1 - 1), lo, hi);
}

// A candidate's record: destination id (with its class tag), the first
// entry of its table and its lg.
struct Cand {
  uint32_t id, base, lg;
};

// Writes entry e whose draws meet candidates c0 .. c1 (c0 <= c1): bounds lo,
// hi and mc from entry_bounds, L = candidate c0, M = c0 + 1 (when there is
// one), R = c1. With mc > 0 the middle candidates go to the child table at
// entry `child` with shift sh (child_shape); child = ~0u when no room was
// found for it: the entry then sends the middle draws to the first middle
// candidate, and the caller reports the graph as failed.
FPPR_GUIDE_FN void put_entry(Entry* e, uint64_t lo, uint64_t hi, uint32_t mc, const Cand& L, const Cand& M,
                             const Cand& R, uint32_t child, uint32_t sh) {
  Entry x{};
  x.lo = lo;
  x.hi = hi;
  x.l_id = L.id;
  x.l_base = L.base;
  x.r_id = R.id;
  x.r_base = R.base;
  x.m_id = M.id;
  x.m_base = M.base;
  x.meta = L.lg | (M.lg << 8) | (R.lg << 16);
  if (mc && child != ~0u) {
    x.m_id = 0;
    x.m_base = child;
    x.meta = L.lg | (sh << 8) | (R.lg << 16) | kChild;
  }
  *e = x;
}

// An entry from thresholds T(j) and candidate records rec(c) read through
// accessors; push(lo, hi, first, last, nbk, sh) lays out the child table of
// the middle candidates first..last when there is one and returns its first
// entry (or ~0u).
template <class Th, class Rec, class Push>
FPPR_GUIDE_FN void fill_entry(Entry* e, const Th& T, const Rec& rec, uint32_t c0, uint32_t c1, Push&& push) {
  uint64_t lo = 0, hi = 0;
  const uint32_t mc = entry_shape(T, c0, c1, &lo, &hi);
  const Cand L = rec(c0), R = rec(c1);
  const Cand M = c1 - c0 >= 2 ? rec(c0 + 1) : L;
  uint32_t sh = 0, child = ~0u;
  if (mc) {
    const uint32_t nbk = child_shape(lo, hi, mc, &sh);
    child = push(lo, hi, c0 + 1, c1 - 1, nbk, sh);
  }
  put_entry(e, lo, hi, mc, L, M, R, child, sh);
}

// Candidates c0 .. c1 of every entry of a row table (2^kb entries, d >= 1
// edges), in entry order by one merge of bucket edges and thresholds:
// fn(b, c0, c1) for b = 0 .. 2^kb - 1. O(d + 2^kb) threshold reads.
template <class Th, class Fn>
FPPR_GUIDE_FN void for_row_buckets(const Th& T, uint32_t d, uint32_t kb, Fn&& fn) {
  uint32_t c = 0;
  for (uint32_t b = 0; b < (1u << kb); ++b) {
    uint64_t blo, bhi;
    row_bucket(kb, b, &blo, &bhi);
    while (c + 1 < d && T(c) <= blo) ++c;
    uint32_t c1 = c;
    while (c1 + 1 < d && T(c1) <= bhi) ++c1;
    fn(b, c, c1);
  }
}

// The pick of draw D at a node with record (base, lg): follows entries (and
// child tables) until one resolves; ent(i) reads entry i. Returns the chosen
// candidate's record and the number of entries read.
template <class Ent>
FPPR_GUIDE_FN Cand pick(const Ent& ent, uint32_t base, uint32_t lg, uint64_t D, uint32_t* reads) {
  uint32_t i = base + top_bits(D, table_bits(lg));
  for (uint32_t k = 1;; ++k) {
    const Entry& x = ent(i);
    if (D < x.lo) {
      *reads = k;
      return Cand{x.l_id, x.l_base, x.meta & 0xFFu};
    }
    if (D >= x.hi) {
      *reads = k;
      return Cand{x.r_id, x.r_base, (x.meta >> 16) & 0xFFu};
    }
    if (!(x.meta & kChild)) {
      *reads = k;
      return Cand{x.m_id, x.m_base, (x.meta >> 8) & 0xFFu};
    }
    i = x.m_base + static_cast<uint32_t>((D - x.lo) >> ((x.meta >> 8) & 0xFFu));
  }
}

}  // namespace guide
}  // namespace fppr
