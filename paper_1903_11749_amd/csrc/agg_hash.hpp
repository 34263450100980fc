// Index arithmetic of the large-budget counting kernel (k_aggregate_big):
// the LDS hash table's home slot and probe stride, the global spill table's
// home slot, the count histogram's bin and the visiting order of a pass over
// a global table. Plain integer code, compiled for the device and for the
// host, so that a host build can run the same index sequences against
// exact-size buffers with bounds checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fppr {

constexpr uint32_t kAggWaveMaxR = 256;   // largest R of the one-wave-per-source path
constexpr uint32_t kAggMaxR = 4096;      // largest R with counts (the LDS tile sort)
constexpr uint32_t kMaxR = 1u << 20;     // largest R (hash path above kAggMaxR: no counts)
constexpr uint32_t kAggBigGroups = 512;  // blocks (and hash tables) of the hash path

// Counting without per-source counts and R > kAggWaveMaxR takes the hash path,
// which needs agg_table_bytes of scratch: log2 of the slots per global table
// (at least twice R, so a table is at most half full), the tables (= blocks)
// used, and the bytes (0 when the path is not taken).
inline bool agg_uses_table(uint32_t R, bool counts) { return R > kAggWaveMaxR && !counts; }
inline uint32_t agg_table_log2(uint32_t R) {
  uint32_t l = 1;
  while ((1ull << l) < 2ull * R) ++l;
  return l;
}
inline uint32_t agg_table_groups(uint64_t n_src, uint32_t R) {
  const uint64_t slot_bytes = 8ull << agg_table_log2(R);
  uint64_t g = (1ull << 30) / slot_bytes;  // about 1 GiB of tables at most
  if (g > kAggBigGroups) g = kAggBigGroups;
  if (g < 64) g = 64;
  if (g > n_src) g = n_src;
  return static_cast<uint32_t>(g ? g : 1);
}
inline uint64_t agg_table_bytes(uint64_t n_src, uint32_t R, bool counts) {
  if (!agg_uses_table(R, counts) || n_src == 0) return 0;
  return static_cast<uint64_t>(agg_table_groups(n_src, R)) << (agg_table_log2(R) + 3);
}

namespace agg {

constexpr int kBigThreads = 1024;              // threads of a counting block
constexpr uint32_t kLdsLog2 = 14;
constexpr uint32_t kLdsSlots = 1u << kLdsLog2; // LDS table: keys + counts, 128 KB
constexpr uint32_t kLdsProbes = 8;             // probes before an endpoint spills
constexpr uint32_t kHistBins = 2048;           // histogram of min(count, 2047)
constexpr uint32_t kCandCap = 2048;            // candidates sorted in LDS
constexpr uint64_t kEmpty = 0xFFFFFFFF00000000ull;  // empty global slot

// LDS table: home slot and odd probe stride of node t (double hashing)
__host__ __device__ inline uint32_t lds_home(uint32_t t) { return (t * 0x9E3779B1u) >> (32 - kLdsLog2); }
__host__ __device__ inline uint32_t lds_stride(uint32_t t) {
  return ((t * 0x85EBCA6Bu) >> (32 - kLdsLog2)) | 1u;
}
__host__ __device__ inline uint32_t lds_next(uint32_t h, uint32_t stride) { return (h + stride) & (kLdsSlots - 1); }

// global table of 2^log2 slots (1 <= log2 <= 31): home slot of t, then
// linear probing
__host__ __device__ inline uint32_t table_home(uint32_t t, uint32_t log2) { return (t * 0x9E3779B1u) >> (32 - log2); }
__host__ __device__ inline uint32_t table_next(uint32_t h, uint32_t log2) { return (h + 1) & ((1u << log2) - 1); }

__host__ __device__ inline uint32_t hist_bin(uint32_t c) { return c < kHistBins - 1 ? c : kHistBins - 1; }

// A pass of thread `tid` over a table of H slots read two slots (16 bytes)
// at a time: index j of the n4 = H / 2 pairs. Rounds of four loads in flight
// first (quad(j) reads pairs j, j + T, j + 2T, j + 3T, T = kBigThreads), then
// single pairs (one(j)).
template <typename Quad, typename One>
__host__ __device__ inline void pass_pairs(uint32_t tid, uint32_t H, Quad&& quad, One&& one) {
  const uint32_t n4 = H / 2;
  uint32_t j = tid;
  for (; j + 3 * kBigThreads < n4; j += 4 * kBigThreads) quad(j);
  for (; j < n4; j += kBigThreads) one(j);
}

}  // namespace agg
}  // namespace fppr
