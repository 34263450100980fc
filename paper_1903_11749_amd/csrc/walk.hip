// The walk kernel: R walks from each source (Algorithm 2, Sec. 2.1).
//
// Algorithm 2 extends every active path by one step per round and starts a
// new batch of gamma walks per node once the previous batch has moved
// (parallel pipelines, Fig. 2, Sec. 4.3). On the GPU the same effect comes
// without rounds: a persistent grid of 64-lane waves, one walk per lane in
// registers; a lane whose walk terminated takes the next walk id at once
// (ballot + mbcnt over the idle lanes, one atomic per wave per chunk of
// ids), so the number of walks in flight stays at the lane count.
//
// One move (integer only):
//   x = Philox4x32-10(key = seed, counter = (i, m, s, 0))
//   node without out-edges: tail = s (restart from the head, Sec. 2.1)
//   small node (stitched runs): take pool entry floor(x0 * K / 2^32)
//   otherwise: X = floor((x1:x0) * W / 2^64), first edge with prefix > X
//   stop iff x2 < T (or the stitched entry is terminated), or m hits the cap
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
constexpr uint64_t kChunk = 256;  // walk ids claimed per wave at a time

struct WalkArgs {
  GraphView g;
  const uint4* __restrict__ rec;  // plain or stitched records
  const uint32_t* __restrict__ sources;
  uint64_t total;  // n_src * R
  uint32_t R;
  uint64_t R_magic;
  uint32_t n;
  uint32_t key0, key1, T;
  const uint64_t* __restrict__ pool;
  uint32_t K_log2;
  uint32_t* __restrict__ endpoints;
  unsigned long long* work_counter;  // [0] next id, [1] invalid-source flag
  fppr_stats* stats;
};

template <bool kStitch, bool kStats>
__global__ void __launch_bounds__(kThreads) k_walk(WalkArgs a) {
  const uint32_t lane = __lane_id();
  bool active = false;
  uint64_t g = 0;
  uint32_t s = 0, i = 0, m = 0, tail = 0, len = 0;
  uint64_t cur = 0, end = 0;  // wave-uniform chunk of walk ids
  bool exhausted = false;
  uint64_t st_moves = 0, st_steps = 0;
  uint32_t st_walks = 0, st_capped = 0, st_dang = 0, st_plain = 0, st_stitch = 0, st_log = 0;

  for (;;) {
    // ---- refill idle lanes from the wave's chunk of walk ids ----
    uint64_t idle = __ballot(!active);
    while (idle != 0 && !exhausted) {
      if (cur >= end) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(a.work_counter, static_cast<unsigned long long>(kChunk));
        c = __shfl(c, 0, 64);
        if (c >= a.total) {
          exhausted = true;
          break;
        }
        cur = c;
        end = (c + kChunk < a.total) ? c + kChunk : a.total;
      }
      const uint64_t avail = end - cur;
      const uint32_t nidle = static_cast<uint32_t>(__popcll(idle));
      const uint32_t take = avail < nidle ? static_cast<uint32_t>(avail) : nidle;
      if (!active) {
        const uint32_t r = mask_rank(idle);
        if (r < take) {
          g = cur + r;
          uint64_t q = __umul64hi(g, a.R_magic);
          uint64_t rem = g - q * a.R;
          if (rem >= a.R) {
            q += 1;
            rem -= a.R;
          }
          s = a.sources ? a.sources[q] : static_cast<uint32_t>(q);
          i = static_cast<uint32_t>(rem);
          tail = s;
          m = 0;
          len = 0;
          active = true;
          if (s >= a.n) {  // invalid source: no walk, recorded for the caller
            a.endpoints[g] = kNoNode;
            atomicOr(a.work_counter + 1, 1ull);
            active = false;
          }
        }
      }
      cur += take;
      idle = __ballot(!active);
    }
    if (__ballot(active) == 0) break;

    // ---- one move ----
    if (active) {
      const U4 x = philox10(i, m, s, 0u, a.key0, a.key1);
      const uint4 r = a.rec[tail];
      const uint64_t od = rec_od(r);
      const uint32_t code = static_cast<uint32_t>(od) & kCodeMask;
      bool stop;
      if (code == 0) {
        tail = s;
        len += 1;
        stop = x.x2 < a.T;
        if (kStats) ++st_dang;
      } else if (kStitch && code == kPoolCode) {
        const uint64_t slot = (static_cast<uint64_t>(x.x0) << a.K_log2) >> 32;
        const uint64_t e = a.pool[rec_w(r) + slot];
        tail = static_cast<uint32_t>(e);
        len += static_cast<uint32_t>(e >> 32) & 0xFFFFu;
        stop = ((e >> 48) & 1u) != 0;
        if (kStats) ++st_stitch;
      } else {
        const uint64_t X = scaled_draw(x.x0, x.x1, rec_w(r));
        const uint64_t e = pick_edge(a.g, od >> kCodeBits, code, X);
        tail = a.g.col[e];
        len += 1;
        stop = x.x2 < a.T;
        if (kStats) {
          ++st_plain;
          const uint32_t deg = (code & kHubFlag) ? a.g.hubs[code & ~kHubFlag].deg : code;
          st_log += ceil_log2_u32(deg);
        }
      }
      m += 1;
      if (!stop && m == kMoveCap) {
        stop = true;
        if (kStats) ++st_capped;
      }
      if (stop) {
        a.endpoints[g] = tail;
        active = false;
        if (kStats) {
          ++st_walks;
          st_moves += m;
          st_steps += len;
        }
      }
    }
  }

  if (kStats) {
    const uint64_t v[8] = {st_walks, st_moves, st_steps, st_capped,
                           st_dang, st_plain, st_stitch, st_log};
    unsigned long long* out = reinterpret_cast<unsigned long long*>(a.stats);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t t = wave_sum_u64(v[k]);
      if (lane == 0 && t) atomicAdd(out + k, static_cast<unsigned long long>(t));
    }
  }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t count, uint64_t value) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = value;
}

template <bool kStitch, bool kStats>
hipError_t launch_walk_t(const WalkArgs& a, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk<kStitch, kStats>, kThreads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  uint64_t blocks = static_cast<uint64_t>(cus) * per_cu;
  const uint64_t need = (a.total + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_walk<kStitch, kStats>), dim3(static_cast<uint32_t>(blocks)), dim3(kThreads),
                     0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u64(uint64_t* p, uint64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  uint64_t b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<uint32_t>(b)), dim3(256), 0, s, p, count, 0ull);
  return hipGetLastError();
}

hipError_t launch_walk(const fppr_graph* g, const WalkLaunch& w, hipStream_t s) {
  WalkArgs a{};
  a.g = GraphView{g->rec, g->P, g->col, g->hubs, g->TL, g->chunk_log2};
  a.rec = w.rec;
  a.sources = w.sources;
  a.total = w.n_src * w.R;
  a.R = w.R;
  a.R_magic = w.R_magic;
  a.n = g->n;
  a.key0 = w.key0;
  a.key1 = w.key1;
  a.T = w.T;
  a.pool = w.pool;
  a.K_log2 = w.K_log2;
  a.endpoints = w.endpoints;
  a.work_counter = w.work_counter;
  a.stats = w.stats;
  if (a.total == 0) return hipSuccess;
  if (w.stitch) return w.stats ? launch_walk_t<true, true>(a, s) : launch_walk_t<true, false>(a, s);
  return w.stats ? launch_walk_t<false, true>(a, s) : launch_walk_t<false, false>(a, s);
}

}  // namespace fppr
