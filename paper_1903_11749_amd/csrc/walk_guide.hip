// The walk kernel of graphs with the guide-table layout (guide.hpp): the
// same walks as the kernel of the tree layouts (Algorithm 2, Sec. 2.1; the
// same draws, the same edges), with one 64-byte entry read per weighted pick
// for almost every draw.
//
// A persistent grid of 64-lane waves keeps one walk per lane; a lane whose
// walk ended takes the next walk id at once (ballot + mbcnt over the idle
// lanes, one atomic per wave per chunk of ids), from a table of descriptors
// served as by the other walk kernel. A walk always knows the record of the
// node it is at (the first entry of its table, its lg and class): entries
// and pool entries carry the record of every node they lead to, and the
// head's record is read once when the walk starts. So every loop iteration
// needs at most one dependent load per lane:
//   kHead   the head's 8-byte record (once per walk)
//   kEntry  one table entry (64 bytes, read by a lane pair, 32 + 16 bytes)
//   kPool   one 16-byte pool entry (a stitched move)
// and a move at a node without out-edges (known from its class) needs none.
//
// One move (integer only):
//   x = Philox4x32-10(key = seed, counter = (i, m, s, 0))
//   node without out-edges: tail = s
//   small node (stitched runs): pool entry floor(x0 * K / 2^32) of the node
//   otherwise: draw D = x1:x0, entry base + top bits of D, then its L, M or R
//     (or a child entry), which is the first edge with prefix > floor(D W / 2^64)
//   stop iff x2 < T (or the stitched entry is terminated), or m hits the cap
#include "fppr_internal.hpp"
#include "guide.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;

enum : uint32_t {
  kIdle = 0,
  kHead = 1,   // load the head's record
  kEntry = 2,  // load a table entry
  kPool = 3,   // load a pool entry
  kCont = 4,   // no load: continue restarts at the head
};
constexpr uint32_t kResChild = 0xFFFFFFFFu;  // an entry's result: descend to a child entry

struct WalkTable {
  const WalkDesc* __restrict__ descs;
  uint32_t ndesc;
  uint64_t total;
  unsigned long long* ctl;  // [0] next id, [1] bit 0: a source id >= n, bit 1: a pick left unresolved
  fppr_stats* stats;
};

struct Lane {
  uint32_t* ep;
  uint32_t s, i, m, len;
  uint32_t tail, tbase, tlg, ttag;  // the node the walk is at: id, table, lg, class
  uint32_t sbase, slg, stag;        // the head's record
  uint32_t k0, k1, T;               // per-lane form only
  uint32_t ph;
  uint64_t X;  // the pick's draw D, or the pool entry's address
  uint32_t x2;
  uint32_t ent, hops;  // entry to read next; child entries read by this pick
  uint32_t st_moves, st_steps, st_plain, st_stitch, st_log;
};

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
__device__ __forceinline__ uint64_t sread64(uint64_t x) {
  return static_cast<uint64_t>(sread(static_cast<uint32_t>(x))) |
         (static_cast<uint64_t>(sread(static_cast<uint32_t>(x >> 32))) << 32);
}

typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
typedef const U32x4 __attribute__((address_space(1)))* GlobalV4;
typedef const uint64_t __attribute__((address_space(1)))* GlobalU64;
__device__ __forceinline__ uint4 gload16(uint64_t addr, uint32_t k) {
  const U32x4 v = ((GlobalV4)addr)[k];
  return make_uint4(v.x, v.y, v.z, v.w);
}
// The three used words of a 16-byte pool entry: a load with no dead
// destination register, which the compiler would otherwise reuse at once
// and so wait for the load there (before the iteration's other loads are
// issued).
typedef uint32_t U32x2 __attribute__((ext_vector_type(2)));
typedef const U32x2 __attribute__((address_space(1)))* GlobalV2;
__device__ __forceinline__ uint2 gload8(uint64_t addr) {
  const U32x2 v = *((GlobalV2)addr);
  return make_uint2(v.x, v.y);
}
typedef uint32_t U32x3 __attribute__((ext_vector_type(3)));
typedef const U32x3 __attribute__((address_space(1)))* GlobalV3;
__device__ __forceinline__ uint3 gload12(uint64_t addr) {
  const U32x3 v = *((GlobalV3)addr);
  return make_uint3(v.x, v.y, v.z);
}

template <bool kStats, bool kLaneKeys, uint32_t kInlineRestarts>
__global__ void __launch_bounds__(kThreads) k_walk_guide(WalkTable t) {
  __shared__ uint64_t sh_addr[kThreads / 64][64];
  __shared__ uint64_t sh_x[kThreads / 64][64];
  __shared__ uint32_t sh_r0[kThreads / 64][64];
  __shared__ uint32_t sh_r1[kThreads / 64][64];
  __shared__ uint32_t sh_r2[kThreads / 64][64];
  __shared__ uint32_t sh_src[kThreads / 64][kSrcBuf];
  const uint32_t lane = __lane_id();
  const uint32_t wv = threadIdx.x / 64;
  Lane L{};
  L.ph = kIdle;
  constexpr uint64_t kNoChunk = ~0ull;
  uint64_t cur = 0, end = 0, pend = kNoChunk;
  uint32_t d = ~0u, pend_d = 0;
  bool exhausted = false;
  uint64_t walks = 0;
  const guide::Head* head = nullptr;
  const guide::Entry* gent = nullptr;
  const uint4* pool = nullptr;
  const uint32_t* sources = nullptr;
  uint32_t* endpoints = nullptr;
  uint64_t first = 0, walk0 = 0, R_magic = 0, src_q0 = 0, cap = 1;
  uint32_t R = 1, n = 0, T = 0, key0 = 0, key1 = 0, K_log2 = 0, S_small = 0, dflags = 0;

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
          dn = sread(desc_of(c, t.ndesc, [&](uint32_t k) { return t.descs[k].first; }));
        }
        if (dn != d) {
          const WalkDesc& Dn = t.descs[dn];
          const bool same_graph = kLaneKeys && d != ~0u && Dn.ghead == head && Dn.gent == gent &&
                                  Dn.K_log2 == K_log2 && reinterpret_cast<const uint4*>(Dn.pool) == pool &&
                                  Dn.S_small == S_small;
          if (!same_graph && __ballot(L.ph != kIdle) != 0) {  // finish the running walks first
            pend = c;
            pend_d = dn;
            break;
          }
          d = dn;
          const WalkDesc& D = t.descs[d];
          head = D.ghead;
          gent = D.gent;
          cap = D.g_cap;
          pool = reinterpret_cast<const uint4*>(D.pool);
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
          K_log2 = D.K_log2;
          dflags = D.flags;
          end = first + D.count;
        } else {
          end = t.descs[d].first + t.descs[d].count;
        }
        pend = kNoChunk;
        cur = c;
        if (c + kWalkChunk < end) end = c + kWalkChunk;
        if (sources) {
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
          const uint64_t w = walk0 + (cur + r - first);
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
          L.ph = kHead;
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
    const uint32_t ph = L.ph;
    // read only by the lanes that load them (no zeroing for the others: a
    // write to a destination of a load in flight in other lanes would wait
    // for that load before the iteration's entry loads are issued)
    uint2 hv;
    uint3 pv;
    if (ph == kHead) {
      hv = gload8(reinterpret_cast<uint64_t>(head + L.s));
    } else if (ph == kPool) {
      pv = gload12(L.X);
    }
    // an empty statement loads may not be moved across (it emits nothing):
    // these loads stay ahead of the entry loads, all in flight together
    __asm__ __volatile__("" ::: "memory");
    const uint64_t ent_mask = __ballot(ph == kEntry);
    uint32_t r0 = 0, r1 = 0, r2 = 0;
    if (ent_mask) {
      // Owners publish their entry and draw; in round r the pair p reads the
      // entry of lane 32 r + p, the even lane bytes 0..31 (thresholds, L, M),
      // the odd lane bytes 32..47 (R and the lg values).
      uint32_t e = L.ent;
      if (e >= cap) e = static_cast<uint32_t>(cap - 1);
      sh_addr[wv][lane] = ph == kEntry ? reinterpret_cast<uint64_t>(gent + e) : 0;
      sh_x[wv][lane] = L.X;
      wave_sync();
      const uint32_t half = lane & 1u, pair = lane >> 1;
      uint4 qa[2], qb[2];
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t owner = 32 * r + pair;
        qa[r] = make_uint4(0, 0, 0, 0);
        qb[r] = make_uint4(0, 0, 0, 0);
        if ((ent_mask >> owner) & 1ull) {
          const uint64_t src = sh_addr[wv][owner] + half * 32;
          qa[r] = gload16(src, 0);
          if (!half) qb[r] = gload16(src, 1);
        }
      }
#pragma unroll
      for (uint32_t r = 0; r < 2; ++r) {
        if (((ent_mask >> (32 * r)) & 0xFFFFFFFFull) == 0) continue;  // wave-uniform
        const uint32_t owner = 32 * r + pair;
        const bool active = (ent_mask >> owner) & 1ull;
        const uint64_t D = sh_x[wv][owner];
        const uint64_t lo = (static_cast<uint64_t>(qa[r].y) << 32) | qa[r].x;
        const uint64_t hi = (static_cast<uint64_t>(qa[r].w) << 32) | qa[r].z;
        const uint32_t sel = D < lo ? 0u : (D >= hi ? 2u : 1u);  // meaningful on the even lane
        const uint32_t got = swap_pair(half ? qa[r].z : sel);    // even lane: meta; odd lane: sel
        if (active) {
          if (!half) {
            if (sel != 2u) {
              const uint32_t meta = got;
              const uint32_t id = sel == 0u ? qb[r].x : qb[r].z;
              const uint32_t base = sel == 0u ? qb[r].y : qb[r].w;
              const uint32_t lgv = (meta >> (sel * 8u)) & 0xFFu;
              if (sel == 1u && (meta & guide::kChild)) {
                sh_r0[wv][owner] = base + static_cast<uint32_t>((D - lo) >> lgv);
                sh_r2[wv][owner] = kResChild;
              } else {
                sh_r0[wv][owner] = id;
                sh_r1[wv][owner] = base;
                sh_r2[wv][owner] = lgv;
              }
            }
          } else if (got == 2u) {
            sh_r0[wv][owner] = qa[r].x;
            sh_r1[wv][owner] = qa[r].y;
            sh_r2[wv][owner] = (qa[r].z >> 16) & 0xFFu;
          }
        }
      }
      wave_sync();
      r0 = sh_r0[wv][lane];
      r1 = sh_r1[wv][lane];
      r2 = sh_r2[wv][lane];
      wave_sync();
    }

    // ---- consume: a finished step, a new move to start, or a child entry ----
    bool begin = false, step = false, coin = false, done = false, capped = false;
    if (ph == kHead) {
      L.sbase = hv.x;
      L.slg = hv.y & 0xFFu;
      L.stag = hv.y >> 8;
      L.tbase = L.sbase;
      L.tlg = L.slg;
      L.ttag = L.stag;
      begin = true;
    } else if (ph == kEntry) {
      if (r2 == kResChild) {
        // every child narrows the draws by a bit at least: a pick that reads
        // 64 of them met tables that do not resolve (reported, walk ended)
        if (++L.hops < 64) {
          L.ent = r0;
        } else {
          atomicOr(t.ctl + 1, 2ull);
          done = true;
        }
      } else {
        L.tail = r0 & kIdMask;
        L.ttag = r0 >> kTagShift;
        L.tbase = r1;
        L.tlg = r2;
        L.len += 1;
        step = true;
        coin = L.x2 < (kLaneKeys ? L.T : T);
      }
    } else if (ph == kPool) {
      L.tail = pv.x & kIdMask;
      L.ttag = pv.x >> kTagShift;
      L.tbase = pv.y;
      L.tlg = pv.z & 0xFFu;
      L.len += (pv.z >> 8) & 0xFFu;
      if (kStats) ++L.st_stitch;
      step = true;
      coin = ((pv.z >> 16) & 1u) != 0;
    } else if (ph == kCont) {
      begin = true;
    }

    if (step) {
      L.m += 1;
      if (coin || L.m == kMoveCap) {
        done = true;
        capped = !coin;
      } else {
        begin = true;
      }
    }

    // ---- start a move at the tail ----
    if (begin) {
      for (uint32_t restarts = 0;; ++restarts) {
        const U4 x = kLaneKeys ? philox10(L.i, L.m, L.s, 0u, L.k0, L.k1)
                               : philox10(L.i, L.m, L.s, 0u, key0, key1);
        if (L.ttag == kTagDangling) {  // no out-edges: back to the head, then the coin
          L.tail = L.s;
          L.tbase = L.sbase;
          L.tlg = L.slg;
          L.ttag = L.stag;
          L.len += 1;
          L.m += 1;
          const bool cn = x.x2 < (kLaneKeys ? L.T : T);
          if (cn || L.m == kMoveCap) {
            done = true;
            capped = !cn;
            break;
          }
          if (restarts + 1 >= kInlineRestarts) {
            L.ph = kCont;
            break;
          }
          continue;
        }
        if (L.ttag == kTagSmall && S_small) {  // small node: entry floor(x0 K / 2^32) of its K at tail * K
          const uint64_t slot = (static_cast<uint64_t>(x.x0) << K_log2) >> 32;
          L.X = reinterpret_cast<uint64_t>(pool + ((static_cast<uint64_t>(L.tail) << K_log2) + slot));
          L.ph = kPool;
          break;
        }
        const uint64_t D = (static_cast<uint64_t>(x.x1) << 32) | x.x0;
        L.X = D;
        L.x2 = x.x2;
        L.ent = L.tbase + guide::top_bits(D, guide::table_bits(L.tlg));
        L.hops = 0;
        if (kStats) {
          ++L.st_plain;
          L.st_log += L.tlg;
        }
        L.ph = kEntry;
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

template <bool kStats, bool kLaneKeys, uint32_t kRestarts>
hipError_t launch_t(const WalkTable& t, uint32_t blocks_per_cu, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_guide<kStats, kLaneKeys, kRestarts>, kThreads,
                                                   0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  if (blocks_per_cu && static_cast<int>(blocks_per_cu) < per_cu) per_cu = static_cast<int>(blocks_per_cu);
  uint64_t blocks = static_cast<uint64_t>(cus) * per_cu;
  const uint64_t need = (t.total + kThreads - 1) / kThreads;
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_walk_guide<kStats, kLaneKeys, kRestarts>), dim3(static_cast<uint32_t>(blocks)),
                     dim3(kThreads), 0, s, t);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_walk_guide(const WalkDesc* descs, const WalkDesc* host, uint32_t ndesc, uint64_t total,
                             unsigned long long* ctl, fppr_stats* stats, uint32_t blocks_per_cu, hipStream_t s) {
  if (total == 0 || ndesc == 0) return hipSuccess;
  WalkTable t{descs, ndesc, total, ctl, stats};
  const uint32_t b = blocks_per_cu;
  const bool st = stats != nullptr;
  if (same_graph_table(host, ndesc))
    return st ? launch_t<true, true, 4>(t, b, s) : launch_t<false, true, 4>(t, b, s);
  bool split_only = true;  // every descriptor runs the nodes with out-edges of an all-nodes run
  for (uint32_t k = 0; k < ndesc; ++k) split_only = split_only && (host[k].flags & kDescEpBySource);
  if (split_only) return st ? launch_t<true, false, 1>(t, b, s) : launch_t<false, false, 1>(t, b, s);
  return st ? launch_t<true, false, 4>(t, b, s) : launch_t<false, false, 4>(t, b, s);
}

}  // namespace fppr
