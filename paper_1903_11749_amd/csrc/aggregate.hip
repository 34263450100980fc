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

}  // namespace

hipError_t launch_aggregate(const AggLaunch& a, hipStream_t s) {
  if (a.n_src == 0) return hipSuccess;
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
