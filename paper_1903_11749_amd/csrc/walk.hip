// The walk kernel: R walks from each source (Algorithm 2, Sec. 2.1).
//
// Algorithm 2 extends every active path by one step per round and starts a
// new batch of gamma walks per node once the previous batch has moved
// (parallel pipelines, Fig. 2, Sec. 4.3). On the GPU the same effect comes
// without rounds: a persistent grid of 64-lane waves, one walk per lane in
// registers; a lane whose walk terminated takes the next walk id at once
// (ballot + mbcnt over the idle lanes, one atomic per wave per chunk of ids).
//
// Each lane runs its walk as a small state machine that needs exactly one
// dependent load per loop iteration (node record, one 128-byte tree node, one
// 128-byte leaf block of prefixes and destinations, or one pool entry). Tree
// nodes and leaf blocks are read by lane pairs, 64 bytes per lane: on gfx950
// random 128-byte lines stream at full rate only when each lane takes at most
// half a line (a lane reading a whole line of its own runs 3.7x slower). Lanes therefore
// advance independently: an iteration costs one memory latency, not the
// longest move in the wave. The head's record stays in registers, so the
// restart from a node without out-edges (Sec. 2.1) costs no load at all.
//
// One move (integer only):
//   x = Philox4x32-10(key = seed, counter = (i, m, s, 0))
//   node without out-edges: tail = s
//   small node (stitched runs): pool entry floor(x0 * K / 2^32) of the node
//   otherwise: X = floor((x1:x0) * W / 2^64), first edge with prefix > X
//   stop iff x2 < T (or the stitched entry is terminated), or m hits the cap
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
constexpr uint64_t kChunk = 256;          // walk ids claimed per wave at a time
constexpr uint32_t kInlineRestarts = 8;   // restarts handled per iteration

enum : uint32_t {
  kIdle = 0,
  kSrcRec = 1,  // load the head's record (kept in registers)
  kRec = 2,     // load the tail's record
  kTree = 3,    // load one prefix-tree node (128 bytes)
  kBsearch = 4, // load one leaf block's last prefix (rows without a tree, > 8 edges)
  kLeaf = 5,    // load one leaf block: 8 prefixes and their destinations
  kPool = 6,    // load one pool entry
  kCont = 7,    // no load: continue restarts at the head
};

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

struct Lane {
  // walk
  uint64_t g;
  uint32_t s, i, m, len, tail;
  // head record
  uint64_t sW, s_od;
  // current move
  uint32_t ph;
  uint64_t X;     // draw, or the pool entry index
  uint64_t off;   // first block of the row's region
  uint32_t deg, x2;
  // search state (blocks relative to the region): tree descent (lvl; lo =
  // node within the level, hi = first node of the level) or candidate leaf
  // blocks [lo, hi]; a leaf load reads block hi + lo
  uint32_t lvl;
  uint32_t lo;
  uint32_t hi;
  // statistics (restart moves = moves - picks - stitched; walks counted per
  // wave); 32-bit per lane, flushed to the global counters before overflow
  uint32_t st_moves, st_steps, st_plain, st_stitch, st_log;
};

// Orders this wave's LDS writes before its later LDS reads (the wave's own
// lanes only; no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value of the other lane of this lane's aligned pair (DPP quad
// permutation [1, 0, 3, 2]).
__device__ __forceinline__ uint32_t swap_pair(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
}

template <bool kStitch, bool kStats>
__global__ void __launch_bounds__(kThreads) k_walk(WalkArgs a) {
  __shared__ uint64_t sh_blk[kThreads / 64][64];
  __shared__ uint64_t sh_x[kThreads / 64][64];
  __shared__ uint32_t sh_res[kThreads / 64][64];
  const uint32_t lane = __lane_id();
  const uint32_t wv = threadIdx.x / 64;
  Lane L{};
  L.ph = kIdle;
  uint64_t cur = 0, end = 0;  // wave-uniform chunk of walk ids (scalar registers)
  bool exhausted = false;
  uint64_t walks = 0;         // walks started by this wave

  for (;;) {
    // ---- refill idle lanes from the wave's chunk of walk ids ----
    uint64_t idle = __ballot(L.ph == kIdle);
    while (idle != 0 && !exhausted) {
      if (cur >= end) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(a.work_counter, static_cast<unsigned long long>(kChunk));
        c = static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(c))) |
            (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(c >> 32))) << 32);
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
      if (L.ph == kIdle) {
        const uint32_t r = mask_rank(idle);
        if (r < take) {
          L.g = cur + r;
          uint64_t q = __umul64hi(L.g, a.R_magic);
          uint64_t rem = L.g - q * a.R;
          if (rem >= a.R) {
            q += 1;
            rem -= a.R;
          }
          L.s = a.sources ? a.sources[q] : static_cast<uint32_t>(q);
          L.i = static_cast<uint32_t>(rem);
          L.tail = L.s;
          L.m = 0;
          L.len = 0;
          L.ph = kSrcRec;
          if (L.s >= a.n) {  // invalid source: no walk, recorded for the caller
            a.endpoints[L.g] = kNoNode;
            atomicOr(a.work_counter + 1, 1ull);
            if (kStats) atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats->walks), ~0ull);
            L.ph = kIdle;
          }
        }
      }
      cur += take;
      walks += take;
      idle = __ballot(L.ph == kIdle);
    }
    if (__ballot(L.ph != kIdle) == 0) break;

    // ---- this iteration's loads ----
    // Records, pool entries and probes are one small load per lane. Tree nodes
    // and leaf blocks are whole 128-byte lines: lanes load them cooperatively,
    // 8 lanes x 16 bytes per line, the line of lane 8r + g by group g in round
    // r, so every load instruction touches 8 lines instead of 64.
    const uint32_t ph = L.ph;
    uint64_t v0 = 0, v1 = 0;
    if (ph == kSrcRec || ph == kRec) {
      const uint4 r = a.rec[L.tail];
      v0 = rec_w(r);
      v1 = rec_od(r);
    } else if (ph == kBsearch) {
      v0 = a.g.blocks[L.off + L.lo + ((L.hi - L.lo) >> 1)].lf.p[kLeafEdges - 1];
    } else if (kStitch && ph == kPool) {
      v0 = a.pool[L.X];
    }
    const bool want_line = (ph == kTree || ph == kLeaf);
    const uint64_t line_mask = __ballot(want_line);
    const uint64_t leaf_mask = __ballot(ph == kLeaf);
    uint32_t line_res = 0;  // tree: keys <= X in the node; leaf: destination
    if (line_mask) {
      // Owners publish their line and draw in the wave's LDS table. Lane pairs
      // load lines: in round r the pair p reads the line of lane 32 r + p, the
      // even lane its first 64 bytes (tree keys 0..7, or the leaf's 8
      // prefixes), the odd lane the rest (keys 8..15, or the 8 destinations).
      sh_blk[wv][lane] = want_line ? L.off + L.hi + L.lo : 0;
      sh_x[wv][lane] = L.X;
      wave_sync();
      const uint32_t half = lane & 1u, pair = lane >> 1;
      const uint4* base = reinterpret_cast<const uint4*>(a.g.blocks);
      uint4 q[2][4];
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t owner = 32 * r + pair;
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) q[r][k] = make_uint4(0, 0, 0, 0);
        if ((line_mask >> owner) & 1ull) {
          const uint4* src = base + sh_blk[wv][owner] * 8 + half * 4;
#pragma unroll
          for (uint32_t k = 0; k < 4; ++k) q[r][k] = src[k];
        }
      }
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        if (((line_mask >> (32 * r)) & 0xFFFFFFFFull) == 0) continue;
        const uint32_t owner = 32 * r + pair;
        const uint64_t xo = sh_x[wv][owner];
        const bool leaf = (leaf_mask >> owner) & 1ull;
        uint32_t cnt = 0;
        if (!leaf || half == 0) {
#pragma unroll
          for (uint32_t k = 0; k < 4; ++k) {
            const uint64_t k0 = (static_cast<uint64_t>(q[r][k].y) << 32) | q[r][k].x;
            const uint64_t k1 = (static_cast<uint64_t>(q[r][k].w) << 32) | q[r][k].z;
            cnt += (k0 <= xo ? 1u : 0u) + (k1 <= xo ? 1u : 0u);
          }
        }
        cnt += swap_pair(cnt);  // both lanes of the pair hold the total
        if (leaf) {  // destination j = cnt: word j of the odd lane's 8 ids
          if (half == 1) {
            const uint4 w = (cnt < 4) ? q[r][0] : q[r][1];
            const uint32_t jw = cnt & 3u;
            sh_res[wv][owner] = jw == 0 ? w.x : (jw == 1 ? w.y : (jw == 2 ? w.z : w.w));
          }
        } else if (half == 0) {
          sh_res[wv][owner] = cnt;
        }
      }
      wave_sync();
      line_res = sh_res[wv][lane];
      wave_sync();
    }

    // ---- consume: a finished step, a new move to start, or a search step ----
    bool begin = false, step = false, coin = false;
    uint64_t bw = L.sW, bod = L.s_od;  // record of the move to start
    if (ph == kSrcRec || ph == kRec) {
      if (ph == kSrcRec) {
        L.sW = v0;
        L.s_od = v1;
      }
      bw = v0;
      bod = v1;
      begin = true;
    } else if (ph == kTree) {
      L.hi += static_cast<uint32_t>(tree_level_nodes(L.deg, L.lvl));
      L.lo = L.lo * kNodeKeys + line_res;
      if (--L.lvl == 0) {  // leaves start right after the tree: block hi + lo
        L.lo += L.hi;
        L.hi = 0;
        L.ph = kLeaf;
      }
    } else if (ph == kBsearch) {  // over leaf blocks: their last prefixes
      const uint32_t mid = L.lo + ((L.hi - L.lo) >> 1);
      if (v0 > L.X) L.hi = mid; else L.lo = mid + 1;
      if (L.lo == L.hi) {
        L.hi = 0;
        L.ph = kLeaf;
      }
    } else if (ph == kLeaf) {
      L.tail = line_res;
      L.len += 1;
      step = true;
      coin = L.x2 < a.T;
    } else if (kStitch && ph == kPool) {
      const uint64_t e = v0;
      L.tail = static_cast<uint32_t>(e);
      L.len += static_cast<uint32_t>(e >> 32) & 0xFFFFu;
      if (kStats) ++L.st_stitch;
      step = true;
      coin = ((e >> 48) & 1u) != 0;
    } else if (ph == kCont) {
      begin = true;
    }

    bool done = false, capped = false;
    if (step) {
      L.m += 1;
      if (coin || L.m == kMoveCap) {
        done = true;
        capped = !coin;
      } else if (L.tail == L.s) {
        begin = true;  // back at the head: its record is in registers
      } else {
        L.ph = kRec;
      }
    }

    // ---- start a move at the tail with record (bw, bod) ----
    if (begin) {
      for (uint32_t restarts = 0;; ++restarts) {
        const U4 x = philox10(L.i, L.m, L.s, 0u, a.key0, a.key1);
        const uint32_t d = static_cast<uint32_t>(bod & kDegMask);
        if (d == 0) {  // no out-edges: back to the head, then the coin
          L.tail = L.s;
          L.len += 1;
          L.m += 1;
          const bool cn = x.x2 < a.T;
          if (cn || L.m == kMoveCap) {
            done = true;
            capped = !cn;
            break;
          }
          bw = L.sW;
          bod = L.s_od;
          if (restarts + 1 >= kInlineRestarts) {
            L.ph = kCont;
            break;
          }
          continue;
        }
        if (kStitch && (bod & kPoolFlag)) {
          L.X = bw + ((static_cast<uint64_t>(x.x0) << a.K_log2) >> 32);
          L.ph = kPool;
          break;
        }
        L.X = scaled_draw(x.x0, x.x1, bw);
        L.x2 = x.x2;
        L.off = bod >> kRegionShift;  // first block of the row's region
        L.deg = d;
        if (kStats) {
          ++L.st_plain;
          L.st_log += ceil_log2_u32(d);
        }
        L.lo = 0;
        L.hi = 0;
        if (d > a.g.tree_min) {
          L.lvl = tree_levels(d);  // lo: node within the level, hi: first node of the level
          L.ph = kTree;
        } else if (d > kLeafEdges) {
          L.hi = static_cast<uint32_t>(leaf_blocks(d)) - 1;  // candidate leaf blocks [lo, hi]
          L.ph = kBsearch;
        } else {
          L.ph = kLeaf;  // the one leaf block
        }
        break;
      }
    }

    // ---- a terminated walk writes its endpoint and frees the lane ----
    if (done) {
      a.endpoints[L.g] = L.tail;
      L.ph = kIdle;
      if (kStats) {
        L.st_moves += L.m;
        L.st_steps += L.len;
        if (capped) atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats->capped), 1ull);
        // one walk adds at most 2^16 moves and 2^24 steps: flush well before 2^32
        if ((L.st_steps | L.st_moves | L.st_log) >= 0x40000000u) {
          unsigned long long* out = reinterpret_cast<unsigned long long*>(a.stats);
          atomicAdd(out + 1, static_cast<unsigned long long>(L.st_moves));
          atomicAdd(out + 2, static_cast<unsigned long long>(L.st_steps));
          atomicAdd(out + 4, static_cast<unsigned long long>(L.st_moves - L.st_plain - L.st_stitch));
          atomicAdd(out + 5, static_cast<unsigned long long>(L.st_plain));
          atomicAdd(out + 6, static_cast<unsigned long long>(L.st_stitch));
          atomicAdd(out + 7, static_cast<unsigned long long>(L.st_log));
          L.st_moves = L.st_steps = L.st_plain = L.st_stitch = L.st_log = 0;
        }
      }
    }
  }

  if (kStats) {
    // fppr_stats order: walks, moves, steps, capped, dangling, plain, stitched, log
    const uint64_t dang = static_cast<uint64_t>(L.st_moves) - L.st_plain - L.st_stitch;
    const uint64_t vals[6] = {L.st_moves, L.st_steps, dang, L.st_plain, L.st_stitch, L.st_log};
    const int slot[6] = {1, 2, 4, 5, 6, 7};
    unsigned long long* out = reinterpret_cast<unsigned long long*>(a.stats);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint64_t t = wave_sum_u64(vals[k]);
      if (lane == 0 && t) atomicAdd(out + slot[k], static_cast<unsigned long long>(t));
    }
    if (lane == 0 && walks) atomicAdd(out, static_cast<unsigned long long>(walks));
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
  a.g = GraphView{g->rec, g->blocks, g->tree_min};
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
