// Endpoint counting and top-k (Algorithm 2, last phase: group terminated
// walks by (head, tail) and count; Sec. 1: keep only endpoints that some walk
// reached). pi_hat(s, t) = count(s, t) / R is left to the caller.
//
// A block handles a tile of sources whose endpoint segments fit in LDS
// together (segment length padded to a power of two Rp >= 16). Each segment
// is sorted with a bitonic network in LDS, run heads are ranked by a block
// scan, and the runs give the sparse (t, count) list in increasing t. The
// ranking order for top-k is (count desc, t asc), obtained by sorting the
// 64-bit keys (~count << 32 | t) ascending.
#include "agg_hash.hpp"
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kTile = kAggMaxR;        // endpoints per tile
constexpr uint32_t kPer = kTile / kThreads;  // consecutive elements per thread
constexpr uint32_t kMinSeg = kPer;
constexpr uint32_t kMaxSegs = kTile / kMinSeg;
constexpr uint32_t kPad = 0xFFFFFFFFu;

template <typename T>
__device__ __forceinline__ void bitonic_segments(T* key, uint32_t Rp) {
  for (uint32_t k = 2; k <= Rp; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t idx = threadIdx.x; idx < kTile; idx += kThreads) {
        const uint32_t p = idx ^ j;
        if (p > idx) {
          const T a = key[idx], b = key[p];
          // every segment ends ascending: the final merge (k == Rp) must not
          // take its direction from the segment index bit
          const bool up = (k == Rp) || (idx & k) == 0;
          if ((a > b) == up) {
            key[idx] = b;
            key[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_aggregate(AggLaunch a, uint32_t Rp) {
  __shared__ uint32_t key[kTile];
  __shared__ uint32_t pos[kTile];
  __shared__ uint64_t rk[kTile];
  __shared__ uint32_t seg_base[kMaxSegs + 1];
  __shared__ uint32_t seg_end[kMaxSegs];  // endpoints of the segment that are not FPPR_NO_NODE
  __shared__ unsigned long long dig[kMaxSegs];
  __shared__ uint64_t scan_lds[kThreads / 64];

  const uint32_t spt = kTile / Rp;  // sources per tile
  const uint64_t tiles = (a.n_src + spt - 1) / spt;
  const uint32_t R = a.R;

  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t s0 = tile * spt;
    const uint32_t ns = static_cast<uint32_t>((a.n_src - s0) < spt ? (a.n_src - s0) : spt);

    // load the segments, padding to Rp
    for (uint32_t idx = threadIdx.x; idx < kTile; idx += kThreads) {
      const uint32_t seg = idx / Rp, j = idx % Rp;
      key[idx] = (seg < ns && j < R) ? a.endpoints[(s0 + seg) * R + j] : kPad;
    }
    if (threadIdx.x < kMaxSegs) dig[threadIdx.x] = 0;
    __syncthreads();
    bitonic_segments<uint32_t>(key, Rp);

    // run heads; each thread owns kPer consecutive elements (a segment start
    // is always the first element of some thread's range since Rp >= kPer)
    const uint32_t e0 = threadIdx.x * kPer;
    uint32_t heads = 0;
    uint32_t hmask = 0;
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint32_t idx = e0 + q;
      const uint32_t v = key[idx];
      const bool h = v != kPad && ((idx % Rp) == 0 || key[idx - 1] != v);
      // the last endpoint before the padding (FPPR_NO_NODE sorts last) ends
      // the last run
      if (v != kPad && ((idx % Rp) == Rp - 1 || key[idx + 1] == kPad)) seg_end[idx / Rp] = idx % Rp + 1;
      hmask |= (h ? 1u : 0u) << q;
      heads += h ? 1u : 0u;
    }
    uint64_t total;
    const uint32_t excl = static_cast<uint32_t>(block_exclusive_scan_u64<kThreads>(heads, scan_lds, &total));
    if ((e0 % Rp) == 0) seg_base[e0 / Rp] = excl;
    if (threadIdx.x == 0) seg_base[kTile / Rp] = static_cast<uint32_t>(total);
    __syncthreads();
    {
      const uint32_t seg = e0 / Rp;
      uint32_t r = excl - seg_base[seg];
#pragma unroll
      for (uint32_t q = 0; q < kPer; ++q)
        if (hmask & (1u << q)) pos[seg * Rp + (r++)] = (e0 + q) % Rp;
    }
    __syncthreads();

    // runs -> counts, digest, ranking keys
    for (uint32_t idx = threadIdx.x; idx < kTile; idx += kThreads) {
      const uint32_t seg = idx / Rp, r = idx % Rp;
      const uint32_t nd = seg_base[seg + 1] - seg_base[seg];
      uint64_t rkey = ~0ull;
      if (seg < ns) {
        const uint64_t row = s0 + seg;
        if (r < nd) {
          const uint32_t p = pos[idx];
          const uint32_t t = key[seg * Rp + p];
          const uint32_t c = ((r + 1 < nd) ? pos[idx + 1] : seg_end[seg]) - p;
          rkey = (static_cast<uint64_t>(~c) << 32) | t;
          if (a.counts) {
            a.counts[(row * R + r) * 2] = t;
            a.counts[(row * R + r) * 2 + 1] = c;
          }
          if (a.digest) {
            const uint32_t src = a.sources ? a.sources[row] : static_cast<uint32_t>(a.row0 + row);
            atomicAdd(&dig[seg], static_cast<unsigned long long>(digest_term(src, t, c)));
          }
        } else if (a.counts && r < R) {
          a.counts[(row * R + r) * 2] = 0;
          a.counts[(row * R + r) * 2 + 1] = 0;
        }
        if (r == 0 && a.n_distinct) a.n_distinct[row] = nd;
      }
      rk[idx] = rkey;
    }
    __syncthreads();
    if (a.digest && threadIdx.x < ns) a.digest[s0 + threadIdx.x] = dig[threadIdx.x];

    if (a.topk && a.k) {
      bitonic_segments<uint64_t>(rk, Rp);
      for (uint32_t idx = threadIdx.x; idx < ns * a.k; idx += kThreads) {
        const uint32_t seg = idx / a.k, q = idx % a.k;
        const uint64_t v = rk[seg * Rp + q];
        uint32_t t = kNoNode, c = 0;
        if (v != ~0ull) {
          t = static_cast<uint32_t>(v);
          c = ~static_cast<uint32_t>(v >> 32);
        }
        a.topk[((s0 + seg) * a.k + q) * 2] = t;
        a.topk[((s0 + seg) * a.k + q) * 2 + 1] = c;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// R <= 256: one wave per source, E = ceil(R/64) endpoints per lane (element
// index idx = e * 64 + lane), sorted across the wave by lane exchanges; the
// runs of equal endpoints found by ballots give counts and digests, and the
// top-k positions are handed out by ballots too (no second sort).
// ---------------------------------------------------------------------------
// The value of lane (this lane ^ j), j a power of two below 64 (a constant
// once the sort's loops are unrolled): DPP within rows of 16 lanes for
// j = 1, 2, 4, 8, a swizzle within 32 lanes for j = 16, a permute for 32.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, uint32_t j) {
  const int x = static_cast<int>(v);
  switch (j) {
    case 1: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
    case 2: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
    case 4: {  // half-row mirror (i -> 7 - i), then quad reverse (i -> i ^ 3): i -> i ^ 4
      const int m = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);
      return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, false));
    }
    case 8: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));  // row rotate by 8
    case 16: return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(x, 0x401F));  // xor 16 within 32 lanes
    default: return static_cast<uint32_t>(__shfl_xor(x, static_cast<int>(j), 64));
  }
}

// Bitonic sort of the wave's 64 * E values ascending in element order
// (idx = e * 64 + lane). Every compare-exchange runs one way (the lower
// index keeps the minimum): during merge level k the blocks that the network
// orders descending hold their values complemented (~x reverses the unsigned
// order), so the exchange direction depends only on j, a mask per j instead
// of one per (k, j, register). Changing the complemented blocks from one
// level to the next is one XOR per register.
template <int E>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[E]) {
  const uint32_t lane = __lane_id();
  constexpr uint32_t N = 64 * E;
  uint32_t flip[E];
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) flip[e] = 0;
#pragma unroll
  for (uint32_t k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t want = ((e * 64 + lane) & k) ? ~0u : 0u;
      v[e] ^= flip[e] ^ want;
      flip[e] = want;
    }
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {  // partner in another register of the same lane
        const uint32_t je = j / 64;
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const uint32_t pe = e ^ je;
          if (pe > e) {
            const uint32_t x = v[e], y = v[pe];
            v[e] = x < y ? x : y;
            v[pe] = x < y ? y : x;
          }
        }
      } else {  // partner in lane ^ j of the same register
        const bool lower = (lane & j) == 0;  // this lane holds the lower index
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const uint32_t other = xor_lane(v[e], j);
          v[e] = lower ? (v[e] < other ? v[e] : other) : (v[e] > other ? v[e] : other);
        }
      }
    }
  }
  // the last level (k = N) complements nothing: flip is 0 here
}

// Largest value over the wave (every lane active): rows of 16 lanes by DPP,
// then the four row results through scalar registers. Wave-uniform result.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (uint32_t j = 1; j < 16; j <<= 1) {
    const uint32_t y = xor_lane(x, j);
    x = y > x ? y : x;
  }
  const uint32_t r0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 0));
  const uint32_t r1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 16));
  const uint32_t r2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 32));
  const uint32_t r3 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 48));
  const uint32_t m01 = r0 > r1 ? r0 : r1, m23 = r2 > r3 ? r2 : r3;
  return m01 > m23 ? m01 : m23;
}

template <int E>
__global__ void __launch_bounds__(kThreads) k_aggregate_wave(AggLaunch a) {
  const uint32_t lane = __lane_id();
  const uint32_t wv = threadIdx.x / 64;
  const uint32_t R = a.R;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (kThreads / 64);
  for (uint64_t row = blockIdx.x * static_cast<uint64_t>(kThreads / 64) + wv; row < a.n_src;
       row += nwaves) {
    uint32_t v[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t idx = e * 64 + lane;
      v[e] = idx < R ? a.endpoints[row * R + idx] : kPad;
    }
    const uint32_t src = a.sources ? a.sources[row] : static_cast<uint32_t>(a.row0 + row);
    // endpoints that are not FPPR_NO_NODE: they sort first, and the last
    // run ends where they end
    uint32_t nvalid = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) nvalid += static_cast<uint32_t>(__popcll(__ballot(v[e] != kPad)));
    // Every walk of the source ended at the same node (always the case for a
    // source without out-edges, whose walks restart at it until they stop):
    // one distinct endpoint with count R, no sorting.
    {
      const uint32_t t0 = static_cast<uint32_t>(__shfl(static_cast<int>(v[0]), 0, 64));
      bool same = true;
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) same = same && (e * 64 + lane >= R || v[e] == t0);
      if (__ballot(!same) == 0) {
        const uint32_t nd = t0 != kPad ? 1u : 0u;
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const uint32_t idx = e * 64 + lane;
          if (a.counts && idx < R) {
            const bool head = idx < nd;
            a.counts[(row * R + idx) * 2] = head ? t0 : 0u;
            a.counts[(row * R + idx) * 2 + 1] = head ? R : 0u;
          }
        }
        if (lane == 0) {
          if (a.n_distinct) a.n_distinct[row] = nd;
          if (a.digest) a.digest[row] = nd ? digest_term(src, t0, R) : 0ull;
        }
        if (a.topk) {
          for (uint32_t q = lane; q < a.k; q += 64) {
            const bool head = q < nd;
            a.topk[(row * a.k + q) * 2] = head ? t0 : kNoNode;
            a.topk[(row * a.k + q) * 2 + 1] = head ? R : 0u;
          }
        }
        continue;
      }
    }
    wave_bitonic<E>(v);

    // run heads: first element of each group of equal endpoints
    uint64_t hm[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      uint32_t prev = static_cast<uint32_t>(__shfl_up(static_cast<int>(v[e]), 1, 64));
      if (e > 0) {
        const uint32_t wrap = static_cast<uint32_t>(__shfl(static_cast<int>(v[e - 1]), 63, 64));
        if (lane == 0) prev = wrap;
      }
      const bool first = (e == 0 && lane == 0);
      hm[e] = __ballot(v[e] != kPad && (first || prev != v[e]));
    }
    uint32_t nd = 0;
    uint32_t before[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      before[e] = nd;
      nd += static_cast<uint32_t>(__popcll(hm[e]));
    }
    uint64_t dig = 0;
    uint32_t cnt[E];  // size of the run this element heads, 0 elsewhere
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t idx = e * 64 + lane;
      cnt[e] = 0;
      if ((hm[e] >> lane) & 1ull) {
        const uint32_t rank = before[e] + mask_rank(hm[e]);
        // next head after idx, or the end of the valid endpoints
        const uint64_t above = lane == 63 ? 0ull : (hm[e] & (~0ull << (lane + 1)));
        uint32_t nxt = nvalid;
        if (above) {
          nxt = e * 64 + static_cast<uint32_t>(__builtin_ctzll(above));
        } else {
#pragma unroll
          for (uint32_t e2 = E - 1; e2 > e; --e2)
            if (hm[e2]) nxt = e2 * 64 + static_cast<uint32_t>(__builtin_ctzll(hm[e2]));
        }
        const uint32_t c = nxt - idx;
        cnt[e] = c;
        if (a.counts) {
          a.counts[(row * R + rank) * 2] = v[e];
          a.counts[(row * R + rank) * 2 + 1] = c;
        }
        if (a.digest) dig += digest_term(src, v[e], c);
      }
      if (a.counts && idx >= nd && idx < R) {
        a.counts[(row * R + idx) * 2] = 0;
        a.counts[(row * R + idx) * 2 + 1] = 0;
      }
    }
    if (a.n_distinct && lane == 0) a.n_distinct[row] = nd;
    if (a.digest) {
      dig = wave_sum_u64(dig);
      if (lane == 0) a.digest[row] = dig;
    }
    if (a.topk && a.k) {
      // Ranking by (count desc, t asc) without a second sort: the run heads
      // already stand in increasing t (element order), so the runs of the
      // largest count take the first positions in element order, those of
      // the next largest count the following ones, and so on until k
      // positions are taken. One pass per distinct count value (at most
      // about sqrt(2R) of them, a handful in practice).
      uint32_t pos[E];
      uint32_t mx = 0;
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) {
        pos[e] = ~0u;
        mx = cnt[e] > mx ? cnt[e] : mx;
      }
      uint32_t cur = wave_max_u32(mx), base = 0;  // wave-uniform
      while (cur != 0 && base < a.k) {
        uint32_t below = 0;  // largest count under cur held by this lane
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const bool here = cnt[e] == cur;
          const uint64_t m = __ballot(here);
          if (here) pos[e] = base + mask_rank(m);
          base += static_cast<uint32_t>(__popcll(m));
          if (cnt[e] < cur && cnt[e] > below) below = cnt[e];
        }
        cur = wave_max_u32(below);
      }
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) {
        if (pos[e] < a.k) {
          a.topk[(row * a.k + pos[e]) * 2] = v[e];
          a.topk[(row * a.k + pos[e]) * 2 + 1] = cnt[e];
        }
        const uint32_t q = e * 64 + lane;
        if (q >= nd && q < a.k) {
          a.topk[(row * a.k + q) * 2] = kNoNode;
          a.topk[(row * a.k + q) * 2 + 1] = 0u;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// R > kAggMaxR (large walk budgets, up to 2^20 per source): one 1024-thread
// block per source at a time, the only block on its compute unit. Walks from
// one source pile up on a few nearby nodes, so counting starts in a
// 16384-slot hash table in LDS (128 KB), where contended atomics are cheap.
// An endpoint that finds no LDS slot within 8 probes goes to an
// open-addressing hash table in global memory (one 8-byte slot = t << 32 |
// count, empty = kEmpty, at most half full); later steps visit the LDS
// entries and, when something spilled, the global table. A pass over the
// entries gives the digest, the number of distinct endpoints
// and a histogram of min(count, 2047); a block scan of the histogram from the
// top gives the count threshold of the k-th entry. The entries at or above it
// are sorted in LDS by (count desc, t asc) when at most 2048; otherwise an
// exact radix select over the 64-bit ranking keys finds the k-th key first.
// The last pass over a global table also empties it for the next source.
// ---------------------------------------------------------------------------
using agg::kBigThreads;
using agg::kCandCap;
using agg::kEmpty;
using agg::kHistBins;
using agg::kLdsProbes;
using agg::kLdsSlots;

// loads that see other threads' atomics (served by L2, not the CU's cache)
__device__ __forceinline__ uint64_t load_l2(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Makes the block's table writes (atomics, plain stores) visible to its later
// plain loads: only this block touches its table, so release and acquire at
// workgroup scope around the barrier are enough.
__device__ __forceinline__ void table_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ranking key: larger = earlier in the top-k (count desc, then t asc)
__device__ __forceinline__ uint64_t rank_key(uint64_t e) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(e)) << 32) | static_cast<uint32_t>(~(e >> 32));
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* lds) {
  v = wave_sum_u64(v);
  const uint32_t wave = threadIdx.x / 64;
  __syncthreads();
  if (__lane_id() == 0) lds[wave] = v;
  __syncthreads();
  uint64_t t = 0;
  for (uint32_t i = 0; i < kBigThreads / 64; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// One pass of the block over its table (H >= 2 slots), two slots per 16-byte
// load, four loads in flight per thread; f(entry) sees every occupied slot.
// kReset empties the table behind the pass.
template <bool kReset, typename F>
__device__ __forceinline__ void table_pass(uint64_t* tab, uint32_t H, F&& f) {
  uint4* t4 = reinterpret_cast<uint4*>(tab);
  const uint4 empty2 = make_uint4(0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu);  // two kEmpty slots
  auto visit = [&](const uint4& v) {
    const uint64_t e0 = (static_cast<uint64_t>(v.y) << 32) | v.x;
    const uint64_t e1 = (static_cast<uint64_t>(v.w) << 32) | v.z;
    if (e0 != kEmpty) f(e0);
    if (e1 != kEmpty) f(e1);
  };
  agg::pass_pairs(
      threadIdx.x, H,
      [&](uint32_t j) {
        uint4 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) v[u] = t4[j + u * kBigThreads];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
          visit(v[u]);
          if (kReset) t4[j + u * kBigThreads] = empty2;
        }
      },
      [&](uint32_t j) {
        const uint4 v = t4[j];
        visit(v);
        if (kReset) t4[j] = empty2;
      });
}

// Adds one walk ending at t to the table, starting from slot h whose value
// was read as cur.
__device__ __forceinline__ void table_insert(uint64_t* tab, uint32_t log2, uint32_t t, uint32_t c, uint32_t h,
                                             uint64_t cur) {
  for (;;) {
    if (cur != kEmpty) {
      if ((cur >> 32) == t) {
        atomicAdd(reinterpret_cast<unsigned long long*>(tab + h), static_cast<unsigned long long>(c));
        return;
      }
      h = agg::table_next(h, log2);
      cur = load_l2(tab + h);
      continue;
    }
    const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(tab + h),
                                   static_cast<unsigned long long>(kEmpty),
                                   static_cast<unsigned long long>((static_cast<uint64_t>(t) << 32) | c));
    if (old == kEmpty) return;
    cur = old;  // taken meanwhile: look at what is there now
  }
}

static_assert(kLdsSlots % (4 * kBigThreads) == 0, "whole flush rounds");

// Counts t in the LDS table (keys lk, counts lc; empty key kNoNode); false if
// no slot was free within kLdsProbes probes. Double hashing (an odd stride
// from a second hash) keeps probe windows from running into each other.
__device__ __forceinline__ bool lds_insert(uint32_t* lk, uint32_t* lc, uint32_t t) {
  uint32_t h = agg::lds_home(t);
  const uint32_t step = agg::lds_stride(t);
  for (uint32_t p = 0; p < kLdsProbes; ++p) {
    uint32_t k = lk[h];
    if (k == kNoNode) {
      k = atomicCAS(&lk[h], kNoNode, t);
      if (k == kNoNode) k = t;
    }
    if (k == t) {
      atomicAdd(&lc[h], 1u);
      return true;
    }
    h = agg::lds_next(h, step);
  }
  return false;
}

// Adds c[u] walks ending at t[u] to the global table for the live ones of four
// keys: each first claims its home slot optimistically, all four claims in
// flight together; a key that meets another key there probes on alone.
__device__ __forceinline__ void table_insert4(uint64_t* tab, uint32_t log2, const uint32_t (&t)[4],
                                              const uint32_t (&c)[4], const bool (&live)[4]) {
  uint32_t h[4];
  uint64_t old[4];
#pragma unroll
  for (uint32_t u = 0; u < 4; ++u) {
    h[u] = agg::table_home(t[u], log2);
    old[u] = live[u] ? atomicCAS(reinterpret_cast<unsigned long long*>(tab + h[u]),
                                 static_cast<unsigned long long>(kEmpty),
                                 static_cast<unsigned long long>((static_cast<uint64_t>(t[u]) << 32) | c[u]))
                     : kEmpty;
  }
#pragma unroll
  for (uint32_t u = 0; u < 4; ++u)
    if (live[u] && old[u] != kEmpty) table_insert(tab, log2, t[u], c[u], h[u], old[u]);
}

__global__ void __launch_bounds__(kBigThreads) k_aggregate_big(AggLaunch a) {
  __shared__ uint32_t lk[kLdsSlots];
  __shared__ uint32_t lc[kLdsSlots];
  __shared__ uint32_t hist[kHistBins];
  __shared__ uint64_t cand[kCandCap];
  __shared__ uint64_t red[kBigThreads / 64];
  __shared__ uint64_t s_key;      // threshold key (radix path)
  __shared__ uint32_t s_cstar, s_cand, s_n, s_digit, s_rem, s_spill;
  const uint32_t tid = threadIdx.x;
  const uint32_t H = 1u << a.H_log2;
  uint64_t* tab = a.table + (static_cast<uint64_t>(blockIdx.x) << a.H_log2);
  const uint32_t R = a.R;

  for (uint64_t row = blockIdx.x; row < a.n_src; row += gridDim.x) {
    const uint32_t src = a.sources ? a.sources[row] : static_cast<uint32_t>(a.row0 + row);
    const uint32_t* ep = a.endpoints + row * R;
    // 1. count: LDS first, the global table for what does not fit there
    for (uint32_t i = tid; i < kLdsSlots; i += kBigThreads) {
      lk[i] = kNoNode;
      lc[i] = 0;
    }
    for (uint32_t b = tid; b < kHistBins; b += kBigThreads) hist[b] = 0;
    if (tid == 0) s_spill = 0;
    __syncthreads();
    bool spilled = false;
    for (uint32_t i0 = tid; i0 < R; i0 += 4 * kBigThreads) {
      uint32_t t[4];
      const uint32_t one[4] = {1u, 1u, 1u, 1u};
      bool g[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * kBigThreads;
        t[u] = i < R ? ep[i] : kNoNode;  // kNoNode: a source that got no walks
      }
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        g[u] = t[u] != kNoNode && !lds_insert(lk, lc, t[u]);
        spilled |= g[u];
      }
      if (g[0] || g[1] || g[2] || g[3]) table_insert4(tab, a.H_log2, t, one, g);
    }
    if (spilled) s_spill = 1;
    table_sync();
    // A key is in exactly one of the tables: LDS slots only ever go from
    // empty to a key, so a key whose probe window was full stays out of LDS.
    const bool spill = s_spill != 0;
    auto each_lds = [&](auto&& f) {
      for (uint32_t i = tid; i < kLdsSlots; i += kBigThreads) {
        const uint32_t k = lk[i];
        if (k != kNoNode) f((static_cast<uint64_t>(k) << 32) | lc[i]);
      }
    };
    // every entry once
    auto each = [&](auto&& f) {
      each_lds(f);
      if (spill) table_pass<false>(tab, H, f);
    };

    // 2. digest, distinct endpoints, count histogram
    uint64_t dg = 0, nd = 0;
    each([&](uint64_t e) {
      const uint32_t t = static_cast<uint32_t>(e >> 32), c = static_cast<uint32_t>(e);
      dg += digest_term(src, t, c);
      ++nd;
      atomicAdd(&hist[agg::hist_bin(c)], 1u);
    });
    dg = block_sum_u64(dg, red);
    nd = block_sum_u64(nd, red);
    if (tid == 0) {
      if (a.digest) a.digest[row] = dg;
      if (a.n_distinct) a.n_distinct[row] = static_cast<uint32_t>(nd);
    }
    const uint32_t need = (a.topk && a.k) ? static_cast<uint32_t>(nd < a.k ? nd : a.k) : 0u;

    // 3. threshold: the highest bin b with #(bin >= b) >= need. Thread j owns
    // bins 2047 - 2j and 2046 - 2j.
    int mode = 0;  // 0: nothing to select, 1: collect c >= cstar, 2: collect key >= s_key
    if (need) {
      const uint32_t bh = kHistBins - 1 - 2 * tid, bl = bh - 1;
      const uint32_t vh = hist[bh], vl = hist[bl];
      uint64_t tot;
      const uint64_t above = block_exclusive_scan_u64<kBigThreads>(vh + vl, red, &tot);
      if (above < need && above + vh >= need) {
        s_cstar = bh;
        s_cand = static_cast<uint32_t>(above + vh);
      } else if (above + vh < need && above + vh + vl >= need) {
        s_cstar = bl;
        s_cand = static_cast<uint32_t>(above + vh + vl);
      }
      __syncthreads();
      mode = s_cand <= kCandCap ? 1 : 2;
    }
    const uint32_t cstar = need ? s_cstar : 0u;

    if (mode == 2) {
      // exact radix select of the need-th largest ranking key among c >= cstar
      uint64_t prefix = 0;
      uint32_t rem = need;
      for (int shift = 56; shift >= 0; shift -= 8) {
        for (uint32_t b = tid; b < 256; b += kBigThreads) hist[b] = 0;
        __syncthreads();
        each([&](uint64_t e) {
          if (static_cast<uint32_t>(e) < cstar) return;
          const uint64_t key = rank_key(e);
          if (shift == 56 || (key >> (shift + 8)) == (prefix >> (shift + 8)))
            atomicAdd(&hist[(key >> shift) & 255u], 1u);
        });
        __syncthreads();
        const uint32_t v = tid < 256 ? hist[255 - tid] : 0u;
        uint64_t tot;
        const uint64_t above = block_exclusive_scan_u64<kBigThreads>(v, red, &tot);
        if (tid < 256 && above < rem && above + v >= rem) {
          s_digit = 255 - tid;
          s_rem = rem - static_cast<uint32_t>(above);
        }
        __syncthreads();
        prefix |= static_cast<uint64_t>(s_digit) << shift;
        rem = s_rem;
        __syncthreads();
      }
      if (tid == 0) s_key = prefix;
    }
    if (tid == 0) s_n = 0;
    __syncthreads();

    // 4. collect the selected entries (and empty the global table)
    const uint64_t kmin = mode == 2 ? s_key : 0ull;
    auto collect = [&](uint64_t e) {
      bool take = false;
      if (mode == 1) take = static_cast<uint32_t>(e) >= cstar;
      else if (mode == 2) take = rank_key(e) >= kmin;
      if (take) cand[atomicAdd(&s_n, 1u)] = rank_key(e);
    };
    each_lds(collect);
    if (spill) table_pass<true>(tab, H, collect);
    __syncthreads();

    // 5. sort the candidates (descending) and write the top-k row
    if (a.topk && a.k) {
      const uint32_t nc = s_n;
      uint32_t P = 2;
      while (P < nc) P <<= 1;
      for (uint32_t i = nc + tid; i < P; i += kBigThreads) cand[i] = 0;
      __syncthreads();
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t idx = tid; idx < P; idx += kBigThreads) {
            const uint32_t q = idx ^ j;
            if (q > idx) {
              const uint64_t x = cand[idx], y = cand[q];
              const bool desc = (idx & k) == 0;
              if ((x < y) == desc) {
                cand[idx] = y;
                cand[q] = x;
              }
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t q = tid; q < a.k; q += kBigThreads) {
        uint32_t t = kNoNode, c = 0;
        if (q < need) {
          const uint64_t v = cand[q];
          t = ~static_cast<uint32_t>(v);
          c = static_cast<uint32_t>(v >> 32);
        }
        a.topk[(row * a.k + q) * 2] = t;
        a.topk[(row * a.k + q) * 2 + 1] = c;
      }
    }
    table_sync();  // the emptied table is seen by the next row's probes
  }
}

}  // namespace

hipError_t launch_aggregate(const AggLaunch& a, hipStream_t s) {
  if (a.n_src == 0) return hipSuccess;
  if (agg_uses_table(a.R, a.counts != nullptr)) {
    if (!a.table) return hipErrorInvalidValue;
    AggLaunch b = a;
    b.H_log2 = agg_table_log2(a.R);
    const uint32_t groups = agg_table_groups(a.n_src, a.R);
    hipError_t e = launch_fill_u64(b.table, static_cast<uint64_t>(groups) << b.H_log2, kEmpty, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_aggregate_big, dim3(groups), dim3(kBigThreads), 0, s, b);
    return hipGetLastError();
  }
  if (a.R <= 256) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    uint64_t blocks = static_cast<uint64_t>(cus) * 16;
    const uint64_t need = (a.n_src + 3) / 4;
    if (blocks > need) blocks = need;
    const dim3 grid(static_cast<uint32_t>(blocks)), block(kThreads);
    if (a.R <= 64) hipLaunchKernelGGL(k_aggregate_wave<1>, grid, block, 0, s, a);
    else if (a.R <= 128) hipLaunchKernelGGL(k_aggregate_wave<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_aggregate_wave<4>, grid, block, 0, s, a);
    return hipGetLastError();
  }
  uint32_t Rp = kMinSeg;
  while (Rp < a.R) Rp <<= 1;
  const uint32_t spt = kTile / Rp;
  const uint64_t tiles = (a.n_src + spt - 1) / spt;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  uint64_t blocks = static_cast<uint64_t>(cus) * 8;
  if (blocks > tiles) blocks = tiles;
  hipLaunchKernelGGL(k_aggregate, dim3(static_cast<uint32_t>(blocks)), dim3(kThreads), 0, s, a, Rp);
  return hipGetLastError();
}

}  // namespace fppr
