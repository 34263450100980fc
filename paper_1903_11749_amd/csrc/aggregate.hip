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
          const uint32_t c = ((r + 1 < nd) ? pos[idx + 1] : R) - p;
          rkey = (static_cast<uint64_t>(~c) << 32) | t;
          if (a.counts) {
            a.counts[(row * R + r) * 2] = t;
            a.counts[(row * R + r) * 2 + 1] = c;
          }
          if (a.digest) {
            const uint32_t src = a.sources ? a.sources[row] : static_cast<uint32_t>(row);
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
// index idx = e * 64 + lane), sorted across the wave with shuffles.
// ---------------------------------------------------------------------------
template <int E>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[E]) {
  const uint32_t lane = __lane_id();
  constexpr uint32_t N = 64 * E;
#pragma unroll
  for (uint32_t k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {  // partner in another register of the same lane
        const uint32_t je = j / 64;
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const uint32_t pe = e ^ je;
          if (pe > e) {
            const bool up = (((e * 64 + lane) & k) == 0);
            const uint32_t a = v[e], b = v[pe];
            const bool sw = (a > b) == up;
            v[e] = sw ? b : a;
            v[pe] = sw ? a : b;
          }
        }
      } else {  // partner in lane ^ j of the same register
#pragma unroll
        for (uint32_t e = 0; e < E; ++e) {
          const uint32_t idx = e * 64 + lane;
          const uint32_t other = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v[e]), static_cast<int>(j), 64));
          const bool up = (idx & k) == 0;
          const bool lower = (lane & j) == 0;  // this lane holds the lower index
          const bool take_min = (lower == up);
          v[e] = take_min ? (v[e] < other ? v[e] : other) : (v[e] > other ? v[e] : other);
        }
      }
    }
  }
}

template <int E>
__global__ void __launch_bounds__(kThreads) k_aggregate_wave(AggLaunch a) {
  constexpr uint32_t N = 64 * E;
  __shared__ uint32_t run_t[kThreads / 64][N];
  __shared__ uint32_t run_key[kThreads / 64][N];
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
    const uint32_t src = a.sources ? a.sources[row] : static_cast<uint32_t>(row);
    uint64_t dig = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t idx = e * 64 + lane;
      if ((hm[e] >> lane) & 1ull) {
        const uint32_t rank = before[e] + mask_rank(hm[e]);
        // next head after idx, or R (end of the valid endpoints)
        const uint64_t above = lane == 63 ? 0ull : (hm[e] & (~0ull << (lane + 1)));
        uint32_t nxt = R;
        if (above) {
          nxt = e * 64 + static_cast<uint32_t>(__builtin_ctzll(above));
        } else {
#pragma unroll
          for (uint32_t e2 = E - 1; e2 > e; --e2)
            if (hm[e2]) nxt = e2 * 64 + static_cast<uint32_t>(__builtin_ctzll(hm[e2]));
        }
        const uint32_t c = nxt - idx;
        if (a.counts) {
          a.counts[(row * R + rank) * 2] = v[e];
          a.counts[(row * R + rank) * 2 + 1] = c;
        }
        if (a.digest) dig += digest_term(src, v[e], c);
        run_t[wv][rank] = v[e];
        // ranking key: count descending, then rank (= node id) ascending
        run_key[wv][rank] = ((N - c) << 8) | rank;
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
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      uint32_t kv[E];
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) {
        const uint32_t idx = e * 64 + lane;
        kv[e] = idx < nd ? run_key[wv][idx] : 0xFFFFFFFFu;
      }
      wave_bitonic<E>(kv);
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) {
        const uint32_t q = e * 64 + lane;
        if (q < a.k) {
          uint32_t t = kNoNode, c = 0;
          if (q < nd) {
            t = run_t[wv][kv[e] & 0xFFu];
            c = N - (kv[e] >> 8);
          }
          a.topk[(row * a.k + q) * 2] = t;
          a.topk[(row * a.k + q) * 2 + 1] = c;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

}  // namespace

hipError_t launch_aggregate(const AggLaunch& a, hipStream_t s) {
  if (a.n_src == 0) return hipSuccess;
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
