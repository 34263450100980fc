// Device building blocks shared by the kernels of this library: the
// counter-based generator, the node record format, the integer weighted pick
// and wave helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fppr {

// ---------------------------------------------------------------------------
// Node line: 128 bytes per node (one memory line, read by one dependent
// load), laid out as a Block:
//   key[0]: total weight W of the row
//   key[1]: (first block of the row's region << 28) | flags
//   bytes 16..127: the top level of the row's prefix tree (~0 past its end
//           and in rows without a tree): up to 14 u64 keys (wide layout) or
//           up to 28 u32 keys (narrow layout)
// flags: bits 0..26 out-degree; bit 27 is set by the walk kernel in its own
// registers for a small node of a stitched run (never stored).
// ---------------------------------------------------------------------------
constexpr uint32_t kRegionShift = 28;
constexpr uint64_t kDegMask = (1u << 27) - 1;
constexpr uint64_t kPoolFlag = 1u << 27;
constexpr uint64_t kMaxDeg = kDegMask;           // rows up to 2^27 - 1 edges
constexpr uint64_t kMaxEdges = 1ull << 36;
constexpr uint32_t kMoveCap = 65536u;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// Destination tags. In graphs of at most 2^30 nodes every destination id
// stored in a leaf block (and every pool entry's end node) carries its node's
// class in bits 30..31, so a walk that arrives over an edge knows, without
// reading the node's line, that the node has no out-edges (the move restarts
// at the head) or is a small node of the pool (a stitched run reads the pool
// entry directly). Larger graphs store plain ids (tag 0 everywhere).
constexpr uint32_t kTagShift = 30;
constexpr uint32_t kIdMask = (1u << kTagShift) - 1;
constexpr uint32_t kTagDangling = 1;  // no out-edges
constexpr uint32_t kTagSmall = 2;     // 1 <= out-degree <= the pool's S
constexpr uint64_t kMaxTaggedNodes = 1ull << kTagShift;

// ---------------------------------------------------------------------------
// Row regions. Every row owns a run of 128-byte blocks (one memory line):
//   [prefix-tree nodes below the top level, top first][leaf blocks]
// A graph has one of two layouts, fixed when it is created:
//   wide:   leaf block b holds edges 8b .. 8b+7 of the row: their inclusive
//           weight prefixes P (8 x u64) and destination ids (8 x u32); a
//           tree node holds 16 u64 keys; the node line up to 14 top keys.
//   narrow: every row's total weight fits in 32 bits (checked at creation
//           as max out-degree x max weight < 2^32, and by every rebuild), so
//           prefixes are u32: leaf block b holds edges 16b .. 16b+15 (16 x
//           u32 prefixes, then 16 x u32 ids); a tree node holds 32 u32 keys;
//           the node line up to 28 top keys. Twice the fan-out per line.
// Slots past the row's end hold P = ~0. A pick that knows its leaf block
// reads one line.
// Prefix tree (integer form of the alias tree, Sec. 4.1 and Algorithm 3: the
// row is cut into groups whose total weights form the next level,
// recursively, and a pick walks from the top down to one group): rows with
// more than the tree threshold of edges carry it. Level 1 has one key per
// leaf block, level l one key per F keys of level l-1 (F = 16 or 32 keys a
// node); key k of level l is P[min((k+1) * E * F^(l-1), d) - 1] (E = 8 or 16
// edges a leaf). The top level L is the first with at most 14 (28) keys and
// sits in the node line; every level below it is stored as nodes of F keys
// (128 bytes; unused keys ~0). Taking the first key > X at every level and
// then the first prefix > X in the leaf returns exactly the edge a flat
// search over P returns.
// ---------------------------------------------------------------------------
constexpr uint32_t kLeafEdges = 8;        // wide layout
constexpr uint32_t kNodeKeys = 16;
constexpr uint32_t kTopKeys = 14;
constexpr uint32_t kTopKey0 = 2;          // first u64 word of the top keys
constexpr uint32_t kNarrowLeafEdges = 16; // narrow layout
constexpr uint32_t kNarrowNodeKeys = 32;
constexpr uint32_t kNarrowTopKeys = 28;
constexpr uint32_t kNarrowTopKey0 = 4;    // first u32 word of the top keys

struct LeafBlock {
  uint64_t p[kLeafEdges];  // inclusive prefixes (~0 past the row's end)
  uint32_t c[kLeafEdges];  // destination ids
  uint32_t pad[kLeafEdges];
};
union alignas(128) Block {
  uint64_t key[kNodeKeys];  // wide tree node or node line
  LeafBlock lf;             // wide leaf block
  uint32_t w32[32];         // narrow: tree node keys, or leaf prefixes [0, 16) and ids [16, 32)
};
static_assert(sizeof(Block) == 128, "one memory line per block");

// log2 of the edges per leaf block, log2 of the keys per tree node, and the
// top keys a node line holds, by layout
__host__ __device__ __forceinline__ uint32_t leaf_shift(bool nar) { return nar ? 4u : 3u; }
__host__ __device__ __forceinline__ uint32_t node_shift(bool nar) { return nar ? 5u : 4u; }
__host__ __device__ __forceinline__ uint32_t top_keys(bool nar) { return nar ? kNarrowTopKeys : kTopKeys; }

__host__ __device__ __forceinline__ uint64_t leaf_blocks(uint64_t d, bool nar) {
  return (d + (1ull << leaf_shift(nar)) - 1) >> leaf_shift(nar);
}
// levels of the tree of a row with d edges, the top level included: level 1
// has one key per leaf block, each level F times fewer (rounded up)
__host__ __device__ __forceinline__ uint32_t tree_levels(uint64_t d, bool nar) {
  uint32_t L = 1;
  uint64_t keys = leaf_blocks(d, nar);
  while (keys > top_keys(nar)) {
    ++L;
    keys = (keys + (1ull << node_shift(nar)) - 1) >> node_shift(nar);
  }
  return L;
}
// nodes of level l >= 1: ceil(d / (E * F^l))
__host__ __device__ __forceinline__ uint64_t tree_level_nodes(uint64_t d, uint32_t l, bool nar) {
  const uint32_t sh = leaf_shift(nar) + node_shift(nar) * l;
  return (d + (1ull << sh) - 1) >> sh;
}
// tree nodes a row keeps in its region: every level below the top (0 when
// it has no tree, or its tree is the top level alone)
__host__ __device__ __forceinline__ uint64_t tree_nodes(uint64_t d, uint32_t tree_min, bool nar) {
  if (d <= tree_min) return 0;
  const uint32_t L = tree_levels(d, nar);
  uint64_t t = 0;
  for (uint32_t l = 1; l < L; ++l) t += tree_level_nodes(d, l, nar);
  return t;
}
__host__ __device__ __forceinline__ uint64_t region_blocks(uint64_t d, uint32_t tree_min, bool nar) {
  return d ? tree_nodes(d, tree_min, nar) + leaf_blocks(d, nar) : 0;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, key bumped by
// the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // 32x32 -> 64-bit products: one v_mad_u64_u32 each
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = static_cast<uint32_t>(p1);
    c2 = n2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// X uniform on [0, W): high 64 bits of the 128-bit product (x1:x0) * W.
__device__ __forceinline__ uint64_t scaled_draw(uint32_t x0, uint32_t x1, uint64_t W) {
  return __umul64hi((static_cast<uint64_t>(x1) << 32) | x0, W);
}

// High 64 bits of a 64 x 64-bit product.
__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return static_cast<uint64_t>((static_cast<unsigned __int128>(a) * b) >> 64);
#endif
}

// Source row q = w div R of walk index w (and *rem = w mod R), with R_magic =
// floor((2^64 - 1) / R): the estimate mulhi(w, R_magic) is q or q - 1.
__host__ __device__ __forceinline__ uint64_t walk_row(uint64_t w, uint32_t R, uint64_t R_magic, uint64_t* rem) {
  uint64_t q = mulhi64(w, R_magic);
  uint64_t r = w - q * R;
  if (r >= R) {
    q += 1;
    r -= R;
  }
  *rem = r;
  return q;
}

// Descriptor of walk id c in a table sorted by first id: the last one whose
// first id is <= c (first(0) = 0 <= c). first(k) reads descriptor k's first id.
template <typename First>
__host__ __device__ __forceinline__ uint32_t desc_of(uint64_t c, uint32_t ndesc, First&& first) {
  uint32_t lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (first(mid) <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct GraphView {
  const Block* __restrict__ rec;     // node lines (plain table)
  const Block* __restrict__ blocks;  // row regions
  uint32_t tree_min;                 // rows with deg > tree_min (>= 8) have a tree
};

__device__ __forceinline__ uint32_t ceil_log2_u32(uint32_t d) {
  return d <= 1 ? 0u : 32u - __clz(d - 1u);
}

// 64-bit MurmurHash3 finalizer; the per-source digest adds
// fmix64(fmix64(s << 32 | t) ^ (count * 0x9E3779B97F4A7C15)) over (t, count).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}
__device__ __forceinline__ uint64_t digest_term(uint32_t s, uint32_t t, uint32_t c) {
  return fmix64(fmix64((static_cast<uint64_t>(s) << 32) | t) ^
                (static_cast<uint64_t>(c) * 0x9E3779B97F4A7C15ull));
}

// rank of this lane among the lanes set in mask (lanes below it)
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  unsigned long long x = v;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_inclusive_scan_u64(uint64_t v) {
  unsigned long long x = v;
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(x, o, 64);
    if (lane >= static_cast<uint32_t>(o)) x += t;
  }
  return x;
}

// Exclusive scan over a block of kThreads threads (multiple of 64). `lds`
// holds kThreads/64 values. Returns the exclusive prefix; *total gets the
// block sum. Contains barriers: every thread of the block must call it.
template <int kThreads>
__device__ __forceinline__ uint64_t block_exclusive_scan_u64(uint64_t v, uint64_t* lds,
                                                             uint64_t* total) {
  constexpr int kWaves = kThreads / 64;
  const uint32_t lane = __lane_id();
  const uint32_t wave = threadIdx.x / 64;
  const uint64_t inc = wave_inclusive_scan_u64(v);
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  uint64_t before = 0, sum = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint64_t t = lds[i];
    if (i < static_cast<int>(wave)) before += t;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return before + inc - v;
}

}  // namespace fppr
