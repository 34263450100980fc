// The walk kernel: R walks from each source (Algorithm 2, Sec. 2.1).
//
// Algorithm 2 extends every active path by one step per round and starts a
// new batch of gamma walks per node once the previous batch has moved
// (parallel pipelines, Fig. 2, Sec. 4.3). On the GPU the same effect comes
// without rounds: a persistent grid of 64-lane waves, one walk per lane in
// registers; a lane whose walk terminated takes the next walk id at once
// (ballot + mbcnt over the idle lanes, one atomic per wave per chunk of ids).
//
// Work comes from a table of descriptors. Each covers a run of walks on one
// graph with its own seed, coin threshold, walks per source, sources and
// endpoint buffer; its ids are padded to whole chunks so a chunk never mixes
// descriptors. A plain run is a one-entry table; a batch of graphs or source
// sets, or the slices of many queries, are longer tables served by the same
// launch. Draws depend only on (seed, source, walk, move), never on the table.
// A wave serves one descriptor at a time, so all of its values sit in scalar
// registers; a wave that claims a chunk of another descriptor lets its running
// walks finish before it switches. When every descriptor of the table reads
// the same graph (the slices of many queries), a second form of the kernel
// keeps each walk's Philox key and coin threshold in its lane instead, and
// waves switch descriptors without waiting.
//
// Each lane runs its walk as a small state machine that needs exactly one
// dependent load per loop iteration (a 128-byte node line, one 128-byte tree
// node, one 128-byte leaf block of prefixes and destinations, or one pool
// entry). Lines are read by lane pairs, 64 bytes per lane: on gfx950 random
// 128-byte lines stream at full rate only when each lane takes at most half a
// line (a lane reading a whole line of its own runs 3.7x slower). A node
// line brings the top level of the row's prefix tree with it; the pair hands
// its keys to the owner through LDS, so a pick at a row with a tree starts one
// level down. The head's weight and flags stay in registers, so the restart
// from a node without out-edges (Sec. 2.1) costs no load at all.
//
// One move (integer only):
//   x = Philox4x32-10(key = seed, counter = (i, m, s, 0))
//   node without out-edges: tail = s
//   small node (stitched runs): pool entry floor(x0 * K / 2^32) of the node
//   otherwise: X = floor((x1:x0) * W / 2^64), first edge with prefix > X
//   stop iff x2 < T (or the stitched entry is terminated), or m hits the cap
// In graphs of at most 2^30 nodes every destination a leaf block or a pool
// entry holds carries its node's class, so a move at a node without
// out-edges needs no load and a stitched move reads only its pool entry
// (node v's entries sit at v * K); only picks read the tail's node line.
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
using fppr::kSrcBuf;
// Restarts at the head handled inline per loop iteration: 4 in general
// (2..16 measured), 1 for tables of all-nodes runs whose nodes without
// out-edges went to the coin-only kernel: restarts are rare there, and a
// loop that cannot repeat costs less.

enum : uint32_t {
  kIdle = 0,
  kSrcRec = 1,  // load the head's node line (weight and flags kept in registers)
  kRec = 2,     // load the tail's node line
  kTree = 3,    // load one prefix-tree node (128 bytes)
  kBsearch = 4, // load one leaf block's last prefix (rows without a tree, > 8 edges)
  kLeaf = 5,    // load one leaf block: 8 prefixes and their destinations
  kPool = 6,    // load one pool entry
  kCont = 7,    // no load: continue restarts at the head
};

struct WalkTable {
  const WalkDesc* __restrict__ descs;
  uint32_t ndesc;
  uint64_t total;                    // ids over all descriptors (padded)
  unsigned long long* ctl;           // [0] next id, [1] invalid-source flag
  fppr_stats* stats;
};

struct Lane {
  // walk
  uint32_t* ep;  // endpoint slot
  uint32_t s, i, m, len, tail;
  // head record
  uint64_t sW, s_od;
  // the walk's key and coin threshold (per-lane form of the kernel only)
  uint32_t k0, k1, T;
  // current move
  uint32_t ph;
  uint64_t X;     // draw, or the address of the pool entry
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

__device__ __forceinline__ uint32_t sread(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Loads through global-address-space pointers: addresses handed around as
// integers (through LDS) would otherwise become flat loads, which also count
// against the LDS counter.
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
typedef const U32x4 __attribute__((address_space(1)))* GlobalV4;
typedef const uint64_t __attribute__((address_space(1)))* GlobalU64;
typedef const uint32_t __attribute__((address_space(1)))* GlobalU32;
// 16 bytes at addr + 16 k
__device__ __forceinline__ uint4 gload16(uint64_t addr, uint32_t k) {
  const U32x4 v = ((GlobalV4)addr)[k];
  return make_uint4(v.x, v.y, v.z, v.w);
}

// word j (0..3) of v, without branches
__device__ __forceinline__ uint32_t word_of(uint4 v, uint32_t j) {
  const uint32_t a = (j & 1u) ? v.y : v.x;
  const uint32_t b = (j & 1u) ? v.w : v.z;
  return (j & 2u) ? b : a;
}

// keys of q that are <= X: two u64 keys (wide layout) or four u32 keys
// (narrow layout, where X < 2^32); `nar` is wave-uniform
__device__ __forceinline__ uint32_t count_q(uint4 q, uint64_t X, bool nar) {
  if (nar) {
    const uint32_t x = static_cast<uint32_t>(X);
    return (q.x <= x ? 1u : 0u) + (q.y <= x ? 1u : 0u) + (q.z <= x ? 1u : 0u) + (q.w <= x ? 1u : 0u);
  }
  const uint64_t k0 = (static_cast<uint64_t>(q.y) << 32) | q.x;
  const uint64_t k1 = (static_cast<uint64_t>(q.w) << 32) | q.z;
  return (k0 <= X ? 1u : 0u) + (k1 <= X ? 1u : 0u);
}
__device__ __forceinline__ uint64_t sread64(uint64_t x) {
  return static_cast<uint64_t>(sread(static_cast<uint32_t>(x))) |
         (static_cast<uint64_t>(sread(static_cast<uint32_t>(x >> 32))) << 32);
}

// kLayout: 0 = every descriptor's graph is wide, 1 = every one is narrow,
// 2 = mixed (read per descriptor). kInlineRestarts: see above.
template <bool kStats, bool kLaneKeys, int kLayout, uint32_t kInlineRestarts>
__global__ void __launch_bounds__(kThreads) k_walk(WalkTable t) {
  __shared__ uint64_t sh_line[kThreads / 64][64];
  __shared__ uint64_t sh_x[kThreads / 64][64];
  __shared__ uint32_t sh_res[kThreads / 64][64];
  __shared__ uint32_t sh_src[kThreads / 64][kSrcBuf];  // the current chunk's source ids
  __shared__ uint4 sh_top[kThreads / 64][64][kTopKeys / 2];  // top tree keys of each lane's node line
  const uint32_t lane = __lane_id();
  const uint32_t wv = threadIdx.x / 64;
  Lane L{};
  L.ph = kIdle;
  // the wave's current chunk [cur, end) of descriptor d and that descriptor's
  // values (all wave-uniform)
  constexpr uint64_t kNoChunk = ~0ull;
  uint64_t cur = 0, end = 0, pend = kNoChunk;
  uint32_t d = ~0u, pend_d = 0;
  bool exhausted = false;
  uint64_t walks = 0;  // walks started by this wave
  const Block* rec = nullptr;
  const Block* blocks = nullptr;
  const uint64_t* pool = nullptr;
  const uint32_t* sources = nullptr;
  uint32_t* endpoints = nullptr;
  uint64_t first = 0, walk0 = 0, R_magic = 0, src_q0 = 0;
  uint32_t R = 1, n = 0, T = 0, key0 = 0, key1 = 0, tree_min = 0, K_log2 = 0, S_small = 0, dflags = 0;

  for (;;) {
    // ---- refill idle lanes from the wave's chunk of walk ids ----
    uint64_t idle = __ballot(L.ph == kIdle);
    while (idle != 0 && !exhausted) {
      if (cur >= end) {
        uint64_t c;
        uint32_t dn;
        if (pend != kNoChunk) {
          c = pend;
          dn = pend_d;
        } else {
          unsigned long long a = 0;
          if (lane == 0) a = atomicAdd(t.ctl, static_cast<unsigned long long>(kWalkChunk));
          c = sread64(a);
          if (c >= t.total) {
            exhausted = true;
            break;
          }
          // descriptor holding chunk c: the last one with first <= c
          dn = sread(desc_of(c, t.ndesc, [&](uint32_t k) { return t.descs[k].first; }));
        }
        if (dn != d) {
          const WalkDesc& Dn = t.descs[dn];
          const bool same_graph = kLaneKeys && d != ~0u && Dn.rec == rec && Dn.blocks == blocks &&
                                  Dn.tree_min == tree_min && Dn.K_log2 == K_log2 && Dn.pool == pool &&
                                  Dn.S_small == S_small;
          if (!same_graph && __ballot(L.ph != kIdle) != 0) {  // finish the running walks first
            pend = c;
            pend_d = dn;
            break;
          }
          d = dn;
          const WalkDesc& D = t.descs[d];
          rec = D.rec;
          blocks = D.blocks;
          pool = D.pool;
          S_small = D.S_small;
          sources = D.sources;
          endpoints = D.endpoints;
          first = D.first;
          walk0 = D.walk0;
          R_magic = D.R_magic;
          R = D.R;
          n = D.n;
          T = D.T;
          key0 = D.key0;
          key1 = D.key1;
          tree_min = D.tree_min;
          K_log2 = D.K_log2;
          dflags = D.flags;
          end = first + D.count;  // limit of the descriptor, clipped below
        } else {
          end = t.descs[d].first + t.descs[d].count;
        }
        pend = kNoChunk;
        cur = c;
        if (c + kWalkChunk < end) end = c + kWalkChunk;
        if (sources) {
          // the chunk's source rows [q_lo, q_hi] to LDS in one coalesced load,
          // so that refills read source ids without waiting on memory
          uint64_t rm;
          const uint64_t q_lo = walk_row(walk0 + (cur - first), R, R_magic, &rm);
          const uint64_t q_hi = walk_row(walk0 + (end - 1 - first), R, R_magic, &rm);
          const uint32_t rows = static_cast<uint32_t>(q_hi - q_lo + 1);  // <= kSrcBuf
          for (uint32_t j = lane; j < rows; j += 64) sh_src[wv][j] = sources[q_lo + j];
          src_q0 = q_lo;
          wave_sync();
        }
      }
      const uint64_t avail = end - cur;
      const uint32_t nidle = static_cast<uint32_t>(__popcll(idle));
      const uint32_t take = avail < nidle ? static_cast<uint32_t>(avail) : nidle;
      if (L.ph == kIdle) {
        const uint32_t r = mask_rank(idle);
        if (r < take) {
          const uint64_t w = walk0 + (cur + r - first);  // walk index within its run
          uint64_t rem;
          const uint64_t q = walk_row(w, R, R_magic, &rem);
          L.s = sources ? sh_src[wv][q - src_q0] : static_cast<uint32_t>(q);
          L.i = static_cast<uint32_t>(rem);
          if (kLaneKeys) {
            L.k0 = key0;
            L.k1 = key1;
            L.T = T;
          }
          L.ep = (dflags & kDescEpBySource) ? endpoints + static_cast<uint64_t>(L.s) * R + rem : endpoints + w;
          L.tail = L.s;
          L.m = 0;
          L.len = 0;
          L.ph = kSrcRec;
          if (L.s >= n) {  // invalid source: no walk, recorded for the caller
            if (!(dflags & kDescEpBySource)) *L.ep = kNoNode;
            atomicOr(t.ctl + 1, 1ull);
            if (kStats) atomicAdd(reinterpret_cast<unsigned long long*>(&t.stats->walks), ~0ull);
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
    // Pool entries and probes are one small load per lane. Node lines, tree
    // nodes and leaf blocks are whole 128-byte lines loaded by lane pairs.
    const uint32_t ph = L.ph;
    // the graph's layout (wave-uniform; a constant unless the table mixes layouts)
    const bool nar = kLayout == 2 ? (dflags & kDescNarrow) != 0 : kLayout == 1;
    const bool rec_line = (ph == kSrcRec || ph == kRec);
    // vb and vp are read only by the lanes that load them: no lane writes
    // them otherwise, since a write to a destination of a load in flight in
    // other lanes would wait for that load before the line loads below
    uint32_t vb32;  // narrow layout
    uint64_t vb64, vp;
    if (ph == kBsearch) {
      const uint64_t lb = reinterpret_cast<uint64_t>(blocks + L.off + L.lo + ((L.hi - L.lo) >> 1));
      if (nar) vb32 = ((GlobalU32)lb)[kNarrowLeafEdges - 1];
      else vb64 = ((GlobalU64)lb)[kLeafEdges - 1];
    } else if (ph == kPool) {
      vp = *(GlobalU64)L.X;
    }
    // an empty statement loads may not be moved across (it emits nothing):
    // these loads stay ahead of the line loads, all in flight together
    __asm__ __volatile__("" ::: "memory");
    uint64_t v0 = 0, v1 = 0;
    const bool want_line = rec_line || ph == kTree || ph == kLeaf;
    const uint64_t line_mask = __ballot(want_line);
    const uint64_t leaf_mask = __ballot(ph == kLeaf);
    const uint64_t rec_mask = __ballot(rec_line);
    uint32_t line_res = 0;  // tree: keys <= X in the node; leaf: destination
    if (line_mask) {
      // Owners publish their line and draw in the wave's LDS table. Lane pairs
      // load lines: in round r the pair p reads the line of lane 32 r + p, the
      // even lane its first 64 bytes (tree keys 0..7, the leaf's 8 prefixes,
      // or the node line's weight, flags and top keys 0..5), the odd lane the
      // rest (keys 8..15, the 8 destinations, or top keys 6..13).
      sh_line[wv][lane] = !want_line ? 0
                          : rec_line ? reinterpret_cast<uint64_t>(rec + L.tail)
                                     : reinterpret_cast<uint64_t>(blocks + L.off + L.hi + L.lo);
      sh_x[wv][lane] = L.X;
      wave_sync();
      const uint32_t half = lane & 1u, pair = lane >> 1;
      uint4 q[2][4];
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t owner = 32 * r + pair;
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) q[r][k] = make_uint4(0, 0, 0, 0);
        if ((line_mask >> owner) & 1ull) {
          const uint64_t src = sh_line[wv][owner] + half * 64;
#pragma unroll
          for (uint32_t k = 0; k < 4; ++k) q[r][k] = gload16(src, k);
        }
      }
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        if (((line_mask >> (32 * r)) & 0xFFFFFFFFull) == 0) continue;
        const uint32_t owner = 32 * r + pair;
        if ((rec_mask >> owner) & 1ull) {  // node line: weight and flags, top keys to the owner
          uint4* top = sh_top[wv][owner];
          if (half == 0) {
            sh_x[wv][owner] = (static_cast<uint64_t>(q[r][0].y) << 32) | q[r][0].x;
            sh_line[wv][owner] = (static_cast<uint64_t>(q[r][0].w) << 32) | q[r][0].z;
            top[0] = q[r][1];
            top[1] = q[r][2];
            top[2] = q[r][3];
          } else {
            top[3] = q[r][0];
            top[4] = q[r][1];
            top[5] = q[r][2];
            top[6] = q[r][3];
          }
          continue;
        }
        const uint64_t xo = sh_x[wv][owner];
        const bool leaf = (leaf_mask >> owner) & 1ull;
        uint32_t cnt = 0;
        if (!leaf || half == 0) {
#pragma unroll
          for (uint32_t k = 0; k < 4; ++k) cnt += count_q(q[r][k], xo, nar);
        }
        cnt += swap_pair(cnt);  // both lanes of the pair hold the total
        if (leaf) {  // destination j = cnt: word j of the odd lane's 8 (16) ids
          if (half == 1) {  // selects of values (an indexed pick would put q in scratch)
            const uint32_t jw = cnt & 3u, qi = cnt >> 2;
            const uint32_t w0 = word_of(q[r][0], jw), w1 = word_of(q[r][1], jw);
            if (!nar) {
              sh_res[wv][owner] = (qi & 1u) ? w1 : w0;
            } else {
              const uint32_t w2 = word_of(q[r][2], jw), w3 = word_of(q[r][3], jw);
              const uint32_t lo2 = (qi & 1u) ? w1 : w0;
              const uint32_t hi2 = (qi & 1u) ? w3 : w2;
              sh_res[wv][owner] = (qi & 2u) ? hi2 : lo2;
            }
          }
        } else if (half == 0) {
          sh_res[wv][owner] = cnt;
        }
      }
      wave_sync();
      line_res = sh_res[wv][lane];
      if (rec_line) {
        v0 = sh_x[wv][lane];
        v1 = sh_line[wv][lane];
      }
      wave_sync();
    }

    // ---- consume: a finished step, a new move to start, or a search step ----
    bool begin = false, step = false, coin = false;
    uint32_t tag = 0;                  // class tag of the node a step arrived at
    const bool tagged = (dflags & kDescTagged) != 0;
    uint64_t bw = L.sW, bod = L.s_od;  // record of the move to start
    if (ph == kSrcRec || ph == kRec) {
      // a small node of a stitched run (1 <= out-degree <= S_small) is marked
      // in the register copy of its flags
      const uint32_t dg = static_cast<uint32_t>(v1 & kDegMask);
      if (dg - 1u < S_small) v1 |= kPoolFlag;
      if (ph == kSrcRec) {
        L.sW = v0;
        L.s_od = v1;
      }
      bw = v0;
      bod = v1;
      begin = true;
    } else if (ph == kTree) {
      L.hi += static_cast<uint32_t>(tree_level_nodes(L.deg, L.lvl, nar));
      L.lo = (L.lo << node_shift(nar)) + line_res;
      if (--L.lvl == 0) {  // leaves start right after the tree: block hi + lo
        L.lo += L.hi;
        L.hi = 0;
        L.ph = kLeaf;
      }
    } else if (ph == kBsearch) {  // over leaf blocks: their last prefixes
      const uint32_t mid = L.lo + ((L.hi - L.lo) >> 1);
      const uint64_t vb = nar ? static_cast<uint64_t>(vb32) : vb64;
      if (vb > L.X) L.hi = mid; else L.lo = mid + 1;
      if (L.lo == L.hi) {
        L.hi = 0;
        L.ph = kLeaf;
      }
    } else if (ph == kLeaf) {
      L.tail = tagged ? line_res & kIdMask : line_res;
      tag = tagged ? line_res >> kTagShift : 0u;
      L.len += 1;
      step = true;
      coin = L.x2 < (kLaneKeys ? L.T : T);
    } else if (ph == kPool) {
      const uint64_t e = vp;
      const uint32_t end = static_cast<uint32_t>(e);
      L.tail = tagged ? end & kIdMask : end;
      tag = tagged ? end >> kTagShift : 0u;
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
        begin = true;  // back at the head: its weight and flags are in registers
      } else if (tag == kTagDangling) {
        begin = true;  // no out-edges (known from the edge's tag): the move restarts, no load
        bw = 0;
        bod = 0;
      } else if (tag == kTagSmall && S_small) {
        begin = true;  // small node of the pool (known from the tag): the move reads its entry directly
        bw = 0;
        bod = kPoolFlag | 1u;
      } else {
        L.ph = kRec;
      }
    }

    // ---- start a move at the tail with weight bw and flags bod ----
    if (begin) {
      bool fresh = rec_line;  // the node line was loaded this iteration: its top keys are in LDS
      for (uint32_t restarts = 0;; ++restarts) {
        const U4 x = kLaneKeys ? philox10(L.i, L.m, L.s, 0u, L.k0, L.k1)
                               : philox10(L.i, L.m, L.s, 0u, key0, key1);
        const uint32_t dg = static_cast<uint32_t>(bod & kDegMask);
        if (dg == 0) {  // no out-edges: back to the head, then the coin
          L.tail = L.s;
          L.len += 1;
          L.m += 1;
          const bool cn = x.x2 < (kLaneKeys ? L.T : T);
          if (cn || L.m == kMoveCap) {
            done = true;
            capped = !cn;
            break;
          }
          bw = L.sW;
          bod = L.s_od;
          fresh = false;
          if (restarts + 1 >= kInlineRestarts) {
            L.ph = kCont;
            break;
          }
          continue;
        }
        if (bod & kPoolFlag) {  // small node: entry floor(x0 K / 2^32) of its K at tail * K
          const uint64_t slot = (static_cast<uint64_t>(x.x0) << K_log2) >> 32;
          L.X = reinterpret_cast<uint64_t>(pool + ((static_cast<uint64_t>(L.tail) << K_log2) + slot));
          L.ph = kPool;
          break;
        }
        if (dg > tree_min && !fresh) {  // the head's top keys: load its line again (same draw)
          L.ph = kRec;
          break;
        }
        L.X = scaled_draw(x.x0, x.x1, bw);
        L.x2 = x.x2;
        L.off = bod >> kRegionShift;  // first block of the row's region
        L.deg = dg;
        if (kStats) {
          ++L.st_plain;
          L.st_log += ceil_log2_u32(dg);
        }
        L.lo = 0;
        L.hi = 0;
        if (dg > tree_min) {
          // top level from the node line; lo: node within the next level (or
          // the leaf block), hi: first node of that level
          uint32_t c = 0;
#pragma unroll
          for (uint32_t k = 0; k < kTopKeys / 2; ++k) c += count_q(sh_top[wv][lane][k], L.X, nar);
          L.lo = c;
          const uint32_t lv = tree_levels(dg, nar);
          if (lv == 1) {
            L.ph = kLeaf;
          } else {
            L.lvl = lv - 1;
            L.ph = kTree;
          }
        } else if (dg > (1u << leaf_shift(nar))) {
          L.hi = static_cast<uint32_t>(leaf_blocks(dg, nar)) - 1;  // candidate leaf blocks [lo, hi]
          L.ph = kBsearch;
        } else {
          L.ph = kLeaf;  // the one leaf block
        }
        break;
      }
    }

    // ---- a terminated walk writes its endpoint and frees the lane ----
    if (done) {
      *L.ep = L.tail;
      L.ph = kIdle;
      if (kStats) {
        L.st_moves += L.m;
        L.st_steps += L.len;
        if (capped) atomicAdd(reinterpret_cast<unsigned long long*>(&t.stats->capped), 1ull);
        // one walk adds at most 2^16 moves and 2^24 steps: flush well before 2^32
        if ((L.st_steps | L.st_moves | L.st_log) >= 0x40000000u) {
          unsigned long long* out = reinterpret_cast<unsigned long long*>(t.stats);
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
    unsigned long long* out = reinterpret_cast<unsigned long long*>(t.stats);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint64_t v = wave_sum_u64(vals[k]);
      if (lane == 0 && v) atomicAdd(out + slot[k], static_cast<unsigned long long>(v));
    }
    if (lane == 0 && walks) atomicAdd(out, static_cast<unsigned long long>(walks));
  }
}

// Walks from nodes without out-edges. Such a walk restarts at its source on
// every move, so it ends there whatever its coins: the endpoints are written
// as whole rows, each wave taking row after row with its lanes on
// consecutive walk slots. The coins only decide the statistics (moves and
// capped walks); when those are wanted, each thread then draws the coins of
// a contiguous range of walks, one move per loop iteration, so a wave's
// lanes stay busy until their whole range is done.
template <bool kStats>
__global__ void __launch_bounds__(kThreads) k_dangling(const uint32_t* __restrict__ dang, uint64_t n_dang,
                                                       uint32_t R, uint64_t R_magic, uint32_t T, uint32_t key0,
                                                       uint32_t key1, uint32_t* __restrict__ endpoints,
                                                       fppr_stats* stats) {
  const uint32_t lane = __lane_id();
  const uint64_t waves = static_cast<uint64_t>(gridDim.x) * (kThreads / 64);
  for (uint64_t q = static_cast<uint64_t>(blockIdx.x) * (kThreads / 64) + threadIdx.x / 64; q < n_dang;
       q += waves) {
    const uint32_t s = dang[q];
    uint32_t* row = endpoints + static_cast<uint64_t>(s) * R;
    for (uint32_t i = lane; i < R; i += 64) row[i] = s;
  }
  if (!kStats) return;

  const uint64_t total = n_dang * R;
  const uint64_t threads = static_cast<uint64_t>(gridDim.x) * kThreads;
  const uint64_t per = (total + threads - 1) / threads;
  const uint64_t w0 = (static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x) * per;
  uint64_t left = w0 < total ? (total - w0 < per ? total - w0 : per) : 0;
  const uint64_t walks = left;
  uint64_t q = 0;
  uint32_t i = 0, s = 0, s_next = 0, m = 0;
  if (left) {
    uint64_t rem;
    q = walk_row(w0, R, R_magic, &rem);
    i = static_cast<uint32_t>(rem);
    s = dang[q];
    if (left > R - i) s_next = dang[q + 1];  // the range continues into the next row
  }
  uint64_t moves = 0, capped = 0;
  while (__ballot(left != 0) != 0) {
    if (left) {
      const U4 x = philox10(i, m, s, 0u, key0, key1);
      m += 1;
      const bool coin = x.x2 < T;
      if (coin || m == kMoveCap) {
        moves += m;
        capped += coin ? 0u : 1u;
        m = 0;
        left -= 1;
        if (++i == R) {  // next row: its source was loaded a row ago
          i = 0;
          q += 1;
          s = s_next;
          if (left > R) s_next = dang[q + 1];
        }
      }
    }
  }
  // fppr_stats order: walks, moves, steps, capped, dangling, plain, stitched, log
  unsigned long long* out = reinterpret_cast<unsigned long long*>(stats);
  const uint64_t vw = wave_sum_u64(walks), vm = wave_sum_u64(moves), vc = wave_sum_u64(capped);
  if (lane == 0) {
    if (vw) atomicAdd(out + 0, static_cast<unsigned long long>(vw));
    if (vm) {
      atomicAdd(out + 1, static_cast<unsigned long long>(vm));
      atomicAdd(out + 2, static_cast<unsigned long long>(vm));
      atomicAdd(out + 4, static_cast<unsigned long long>(vm));
    }
    if (vc) atomicAdd(out + 3, static_cast<unsigned long long>(vc));
  }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t count, uint64_t value) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = value;
}

__global__ void k_set_desc(WalkDesc d, WalkDesc* dst) {
  if (threadIdx.x == 0) *dst = d;
}

template <bool kStats, bool kLaneKeys, int kLayout, uint32_t kRestarts>
hipError_t launch_walk_t(const WalkTable& t, uint32_t blocks_per_cu, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk<kStats, kLaneKeys, kLayout, kRestarts>,
                                                   kThreads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  if (blocks_per_cu && static_cast<int>(blocks_per_cu) < per_cu) per_cu = static_cast<int>(blocks_per_cu);
  uint64_t blocks = static_cast<uint64_t>(cus) * per_cu;
  const uint64_t need = (t.total + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_walk<kStats, kLaneKeys, kLayout, kRestarts>), dim3(static_cast<uint32_t>(blocks)),
                     dim3(kThreads), 0, s, t);
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

hipError_t launch_dangling(const fppr_graph* g, const fppr_params* p, uint32_t* endpoints, fppr_stats* stats,
                           hipStream_t s) {
  if (g->n_dang == 0) return hipSuccess;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  e = stats ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dangling<true>, kThreads, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dangling<false>, kThreads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  uint64_t blocks = static_cast<uint64_t>(cus) * per_cu;
  const uint64_t total = g->n_dang * p->R;
  const uint64_t need = (total + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need;
  const uint32_t T = fppr_alpha_threshold(p->alpha);
  const uint32_t k0 = static_cast<uint32_t>(p->seed), k1 = static_cast<uint32_t>(p->seed >> 32);
  if (stats)
    hipLaunchKernelGGL(k_dangling<true>, dim3(static_cast<uint32_t>(blocks)), dim3(kThreads), 0, s, g->dang,
                       g->n_dang, p->R, ~0ull / p->R, T, k0, k1, endpoints, stats);
  else
    hipLaunchKernelGGL(k_dangling<false>, dim3(static_cast<uint32_t>(blocks)), dim3(kThreads), 0, s, g->dang,
                       g->n_dang, p->R, ~0ull / p->R, T, k0, k1, endpoints, stats);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  uint64_t b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill_u64, dim3(static_cast<uint32_t>(b)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_set_desc(const WalkDesc& d, WalkDesc* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, s, d, dst);
  return hipGetLastError();
}

int table_layout(const WalkDesc* h, uint32_t ndesc) {
  bool nar = false, wide = false;
  for (uint32_t k = 0; k < ndesc; ++k) ((h[k].flags & kDescNarrow) ? nar : wide) = true;
  return nar && wide ? 2 : (nar ? 1 : 0);
}

namespace {
template <int kLayout, uint32_t kR>
hipError_t launch_plain(const WalkTable& t, bool stats, uint32_t b, hipStream_t s) {
  return stats ? launch_walk_t<true, false, kLayout, kR>(t, b, s) : launch_walk_t<false, false, kLayout, kR>(t, b, s);
}
}  // namespace

hipError_t launch_walk(const WalkDesc* descs, const WalkDesc* host, uint32_t ndesc, uint64_t total,
                       unsigned long long* ctl, fppr_stats* stats, uint32_t blocks_per_cu, hipStream_t s) {
  if (total == 0 || ndesc == 0) return hipSuccess;
  uint32_t guides = 0;
  for (uint32_t k = 0; k < ndesc; ++k) guides += (host[k].flags & kDescGuide) ? 1u : 0u;
  if (guides == ndesc) return launch_walk_guide(descs, host, ndesc, total, ctl, stats, blocks_per_cu, s);
  if (guides) return hipErrorInvalidValue;  // one table cannot mix guide tables with the tree layouts
  WalkTable t{descs, ndesc, total, ctl, stats};
  const uint32_t b = blocks_per_cu;
  const int layout = table_layout(host, ndesc);
  if (same_graph_table(host, ndesc)) {  // one graph, so one layout; per-lane keys
    if (layout == 1) return stats ? launch_walk_t<true, true, 1, 4>(t, b, s) : launch_walk_t<false, true, 1, 4>(t, b, s);
    return stats ? launch_walk_t<true, true, 0, 4>(t, b, s) : launch_walk_t<false, true, 0, 4>(t, b, s);
  }
  bool split_only = true;  // every descriptor runs the nodes with out-edges of an all-nodes run
  for (uint32_t k = 0; k < ndesc; ++k) split_only = split_only && (host[k].flags & kDescEpBySource);
  const bool st = stats != nullptr;
  if (split_only) {
    if (layout == 0) return launch_plain<0, 1>(t, st, b, s);
    if (layout == 1) return launch_plain<1, 1>(t, st, b, s);
    return launch_plain<2, 1>(t, st, b, s);
  }
  if (layout == 0) return launch_plain<0, 4>(t, st, b, s);
  if (layout == 1) return launch_plain<1, 4>(t, st, b, s);
  return launch_plain<2, 4>(t, st, b, s);
}

bool same_graph_table(const WalkDesc* h, uint32_t ndesc) {
  for (uint32_t k = 1; k < ndesc; ++k)
    if (h[k].rec != h[0].rec || h[k].blocks != h[0].blocks || h[k].tree_min != h[0].tree_min ||
        h[k].K_log2 != h[0].K_log2 || h[k].pool != h[0].pool || h[k].S_small != h[0].S_small ||
        h[k].ghead != h[0].ghead || h[k].gent != h[0].gent)
      return false;
  return ndesc > 1;
}

}  // namespace fppr
