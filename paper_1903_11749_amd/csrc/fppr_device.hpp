// Device building blocks shared by the kernels of this library: the
// counter-based generator, the integer weighted pick and wave helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fppr {

// ---------------------------------------------------------------------------
// Node records (16 bytes, one per node, read with one 128-bit load):
//   x,y  : low/high words of the row's total weight W (plain record), or of
//          the pool base index (stitched record of a small node)
//   z,w  : low/high words of  (row offset << 24) | code
// code: 0 -> no out-edges; 1..0x7FFFFF -> out-degree; 0x800000 | h -> hub h;
//       0xFFFFFF -> small node served by the pool (stitched table only).
// ---------------------------------------------------------------------------
constexpr uint32_t kCodeBits = 24;
constexpr uint32_t kCodeMask = 0xFFFFFFu;
constexpr uint32_t kHubFlag = 0x800000u;
constexpr uint32_t kMaxPlainDeg = 0x7FFFFFu;
constexpr uint32_t kMaxHubs = 0x7FFFFFu;   // hub ids 0 .. kMaxHubs-1
constexpr uint32_t kPoolCode = 0xFFFFFFu;
constexpr uint32_t kMoveCap = 65536u;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

struct HubEntry {  // 16 bytes
  uint32_t deg;
  uint32_t nchunks;
  uint64_t tl_off;  // first entry of this hub in the top-level table
};

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
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// X uniform on [0, W): high 64 bits of the 128-bit product (x1:x0) * W.
__device__ __forceinline__ uint64_t scaled_draw(uint32_t x0, uint32_t x1, uint64_t W) {
  return __umul64hi((static_cast<uint64_t>(x1) << 32) | x0, W);
}

// First index j in [lo, hi] of P with P[j] > X, given P[hi] > X.
__device__ __forceinline__ uint64_t upper_bound(const uint64_t* __restrict__ P, uint64_t lo,
                                                uint64_t hi, uint64_t X) {
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (P[mid] > X) hi = mid; else lo = mid + 1;
  }
  return lo;
}

struct GraphView {
  const uint4* __restrict__ rec;       // plain records
  const uint64_t* __restrict__ P;      // inclusive row prefixes
  const uint32_t* __restrict__ col;
  const HubEntry* __restrict__ hubs;
  const uint64_t* __restrict__ TL;     // hub top-level tables
  uint32_t chunk_log2;
};

// Edge index (global, into col) chosen by draw X at a node with record
// fields (off, code), code != 0 and code != kPoolCode.
__device__ __forceinline__ uint64_t pick_edge(const GraphView& g, uint64_t off, uint32_t code,
                                              uint64_t X) {
  if (code & kHubFlag) {
    const HubEntry h = g.hubs[code & ~kHubFlag];
    const uint64_t c = upper_bound(g.TL + h.tl_off, 0, h.nchunks - 1, X);
    const uint64_t lo = c << g.chunk_log2;
    uint64_t hi = lo + (1ull << g.chunk_log2) - 1;
    if (hi > h.deg - 1) hi = h.deg - 1;
    return off + upper_bound(g.P + off, lo, hi, X);
  }
  return off + upper_bound(g.P + off, 0, code - 1, X);
}

__device__ __forceinline__ uint64_t rec_w(uint4 r) {
  return (static_cast<uint64_t>(r.y) << 32) | r.x;
}
__device__ __forceinline__ uint64_t rec_od(uint4 r) {
  return (static_cast<uint64_t>(r.w) << 32) | r.z;
}

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
  return fmix64(fmix64((static_cast<uint64_t>(s) << 32) | t) ^ (static_cast<uint64_t>(c) * 0x9E3779B97F4A7C15ull));
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

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
