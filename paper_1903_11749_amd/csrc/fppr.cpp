// C-ABI of the library: graph lifetime, pool, planning and runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "fppr_internal.hpp"

namespace fppr {

namespace {
thread_local std::string g_last_error;

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Run workspace: [0, 256) control words, [256, 512) the walk descriptor,
// then the endpoint buffer.
constexpr uint64_t kCtlBytes = 256;
constexpr uint64_t kDescBytes = 256;
static_assert(sizeof(WalkDesc) <= kDescBytes, "descriptor slot");

template <typename T>
hipError_t dmalloc(T** p, uint64_t count, uint64_t* acc) {
  uint64_t bytes = align_up(count * sizeof(T));
  if (bytes == 0) bytes = kAlign;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e == hipSuccess) {
    *p = static_cast<T*>(q);
    if (acc) *acc += bytes;
  }
  return e;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(const_cast<void*>(static_cast<const void*>(p)));
  p = nullptr;
}

void free_graph(fppr_graph* g) {
  if (!g) return;
  int prev = -1;
  if (hipGetDevice(&prev) == hipSuccess && prev != g->device) (void)hipSetDevice(g->device);
  if (g->owns_csr) {
    dfree(g->off);
    dfree(g->col);
    dfree(g->w);
  }
  dfree(g->rec);
  dfree(g->blocks);
  dfree(g->region);
  dfree(g->flag);
  dfree(g->scan);
  dfree(g->rows);
  dfree(g->scan_blocks);
  dfree(g->d_err);
  dfree(g->pool);
  dfree(g->small_nodes);
  dfree(g->cls);
  dfree(g->live);
  dfree(g->dang);
  dfree(g->ghead);
  dfree(g->gent);
  dfree(g->gT);
  dfree(g->gerec);
  dfree(g->gclass);
  dfree(g->gruns);
  dfree(g->gtiles);
  dfree(g->gtile_first);
  dfree(g->gtsum);
  dfree(g->gtoff);
  dfree(g->gttot);
  dfree(g->gtab[0]);
  dfree(g->gtab[1]);
  dfree(g->gctl);
  if (g->side) (void)hipStreamDestroy(g->side);
  if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
  if (g->join_ev) (void)hipEventDestroy(g->join_ev);
  if (prev >= 0 && prev != g->device) (void)hipSetDevice(prev);
  delete g;
}

std::string err_bits(uint32_t e) {
  std::string s;
  if (e & kErrOffsets) s += " row_offsets not monotone / off[0] != 0 / off[n] != m;";
  if (e & kErrCol) s += " col >= n;";
  if (e & kErrWeight) s += " weight == 0;";
  if (e & kErrDegree) s += " a row has 2^27 or more edges;";
  if (e & kErrCapacity) s += " pool table overflow (graph changed shape);";
  if (e & kErrNarrow) s += " a row's total weight exceeds 2^32 - 1 in a graph created with 32-bit prefixes (recreate it);";
  if (e & kErrGuide) s += " the guide tables need more room than the graph was created with (recreate it);";
  return s;
}

fppr_status invalid(const std::string& msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

// Host-visible copy of the control words of d_err.
struct Ctl {
  uint32_t err;
  uint32_t n_rows;
  uint64_t blocks;
  uint64_t small;
  uint32_t n_tree;
  uint64_t live;
  uint32_t max_deg, max_w;
};

hipError_t read_ctl(const fppr_graph* g, hipStream_t s, Ctl* c) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  uint32_t raw[16];
  e = hipMemcpy(raw, g->d_err, sizeof raw, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  c->err = raw[0];
  c->n_rows = raw[1];
  std::memcpy(&c->blocks, raw + 2, 8);
  std::memcpy(&c->small, raw + 6, 8);
  c->n_tree = raw[9];
  std::memcpy(&c->live, raw + 10, 8);
  c->max_deg = raw[12];
  c->max_w = raw[13];
  return hipSuccess;
}

hipError_t zero_ctl(fppr_graph* g, hipStream_t s) {
  return launch_zero_u64(reinterpret_cast<uint64_t*>(g->d_err), 8, s);
}

// region offsets, leaf blocks + records, prefix trees (no host sync; the
// region scan reproduces the block count of the first build when row_offsets
// are unchanged, and the kernels refuse to write past it otherwise)
hipError_t derive(fppr_graph* g, hipStream_t s) {
  hipError_t e;
  if (g->guide) {
    // levels beyond the first build's depth + 2 are refused (and reported)
    const uint32_t levels = std::min<uint32_t>(g->g_levels + 2, kGuideLevels);
    if ((e = launch_guide_build(g, false, levels, s)) != hipSuccess) return e;
    for (uint32_t l = 2; l <= levels; ++l)
      if ((e = launch_guide_level(g, l, levels, s)) != hipSuccess) return e;
    return hipSuccess;
  }
  if ((e = launch_region_sizes(g, s)) != hipSuccess) return e;
  return launch_leaves(g, s, false);  // the tree-row count is unchanged
}

// Guide tables at creation: sizes and bases, then the build level by level,
// reading back each level's table count; when entries or table lists run out
// the build starts again with room for what the counters asked for.
fppr_status create_guide(fppr_graph* g, hipStream_t s);

fppr_status create_guide(fppr_graph* g, hipStream_t s) {
  using guide::Entry;
  using guide::Pending;
  uint64_t* acc = &g->device_bytes;
  hipError_t e;
  if ((e = launch_guide_sizes(g, s)) != hipSuccess) return hip_fail(e, "guide table sizes");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  uint64_t e1 = 0;
  if ((e = hipMemcpy(&e1, g->d_err + 4, 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "read sizes");
  if (e1 >= (1ull << 32)) return invalid("layout GUIDE needs fewer than 2^32 row-table entries");
  g->g_entries1 = e1;
  if ((e = dmalloc(&g->ghead, g->n, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide heads)");
  if ((e = dmalloc(&g->gT, g->m, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide thresholds)");
  if ((e = dmalloc(&g->gerec, g->m, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(edge records)");
  if ((e = dmalloc(&g->gctl, 1, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide counters)");
  // rows by size class (degrees never change: built once). The table bases
  // sit in g->scan until the build below reads them, so the class lists are
  // made first, in a scratch list of their own.
  if ((e = dmalloc(&g->gclass, g->n, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(row classes)");
  {
    uint64_t* bases = nullptr;  // the table bases, kept while the class scans reuse g->scan
    if ((e = dmalloc(&bases, g->n, nullptr)) != hipSuccess) return hip_fail(e, "hipMalloc(scratch)");
    e = hipMemcpyAsync(bases, g->scan, g->n * 8, hipMemcpyDeviceToDevice, s);
    uint64_t at = 0;
    for (uint32_t c = 0; c < 9 && e == hipSuccess; ++c) {
      g->gclass_off[c] = at;
      e = launch_guide_class(g, c, at, s);
      uint64_t cnt = 0;
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess) e = hipMemcpy(&cnt, g->d_err + 14, 8, hipMemcpyDeviceToHost);
      at += cnt;
    }
    g->gclass_off[9] = at;
    // runs of entries of the longest rows
    uint64_t runs = 0;
    if (e == hipSuccess) e = launch_guide_runs_count(g, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && g->gclass_off[9] > g->gclass_off[8])
      e = hipMemcpy(&runs, g->d_err + 14, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = dmalloc(&g->gruns, runs ? runs : 1, acc);
    if (e == hipSuccess) e = launch_guide_runs_fill(g, s);
    g->n_runs = runs;
    // tiles of the longest rows
    uint64_t tiles = 0;
    const uint64_t nlong = g->gclass_off[9] - g->gclass_off[8];
    if (e == hipSuccess) e = launch_guide_tiles_count(g, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && nlong) e = hipMemcpy(&tiles, g->d_err + 14, 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = dmalloc(&g->gtiles, tiles ? tiles : 1, acc);
    if (e == hipSuccess) e = dmalloc(&g->gtile_first, nlong ? nlong : 1, acc);
    if (e == hipSuccess) e = dmalloc(&g->gtsum, tiles ? tiles : 1, acc);
    if (e == hipSuccess) e = dmalloc(&g->gtoff, tiles ? tiles : 1, acc);
    if (e == hipSuccess) e = dmalloc(&g->gttot, tiles ? tiles : 1, acc);
    if (e == hipSuccess) e = launch_guide_tiles_fill(g, s);
    g->n_tiles = tiles;
    if (e == hipSuccess) e = hipMemcpyAsync(g->scan, bases, g->n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(bases);
    if (e != hipSuccess) return hip_fail(e, "row classes");
  }
  const uint64_t kMaxCap = (1ull << 32) - 1;  // entry indices are 32-bit
  // The first pass has room for the row tables only: the child tables'
  // entries are counted, not written, and the second pass allocates what
  // was counted plus an eighth for rebuilds whose weights crowd more
  // (child tables took 1.5x the row tables' entries at R-MAT scale 24).
  // Graphs with no crowded entries are done in one pass.
  uint64_t cap = std::min(kMaxCap, e1 + (1u << 20));
  // 0.19 child tables per row-table entry at scale 24, about one in seven
  // of them large
  uint64_t tcap = e1 / 4 + (1u << 16), tcap_big = e1 / 16 + (1u << 16);
  for (int attempt = 0;; ++attempt) {
    if (attempt == 6) return invalid("guide tables did not fit after several attempts");
    if ((e = dmalloc(&g->gent, cap, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide entries)");
    if ((e = dmalloc(&g->gtab[0], tcap + tcap_big, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide tables)");
    if ((e = dmalloc(&g->gtab[1], tcap + tcap_big, acc)) != hipSuccess) return hip_fail(e, "hipMalloc(guide tables)");
    g->g_cap = cap;
    g->g_tcap = static_cast<uint32_t>(tcap);
    g->g_tcap_big = static_cast<uint32_t>(tcap_big);
    if ((e = zero_ctl(g, s)) != hipSuccess) return hip_fail(e, "zero control words");
    if ((e = launch_guide_build(g, true, kGuideLevels, s)) != hipSuccess) return hip_fail(e, "guide tables");
    uint32_t depth = 1;
    GuideCtl h{};
    for (uint32_t l = 2; l <= kGuideLevels; ++l) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
      if ((e = hipMemcpy(&h, g->gctl, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "read");
      if ((h.tables[l] == 0 && h.big[l] == 0) || h.tables[l] > tcap || h.big[l] > tcap_big || h.next_entry > cap)
        break;
      if ((e = launch_guide_level(g, l, kGuideLevels, s)) != hipSuccess) return hip_fail(e, "guide level");
      depth = l;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
    if ((e = hipMemcpy(&h, g->gctl, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "read");
    uint32_t err = 0;
    if ((e = hipMemcpy(&err, g->d_err, 4, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "read");
    uint64_t most = 0, most_big = 0;
    for (uint32_t l = 0; l < kGuideLevels + 2; ++l) {
      most = std::max<uint64_t>(most, h.tables[l]);
      most_big = std::max<uint64_t>(most_big, h.big[l]);
    }
    const bool lists_full = most > tcap || most_big > tcap_big;
    const bool full = h.next_entry > cap || lists_full;
    if (!full) {
      if (err & kErrGuide) return invalid("guide tables need more than 64 levels");
      if (err) return invalid("graph build failed:" + err_bits(err));
      g->g_levels = depth;
      return FPPR_OK;
    }
    g->device_bytes -= align_up(cap * sizeof(Entry)) + 2 * align_up((tcap + tcap_big) * sizeof(Pending));
    dfree(g->gent);
    dfree(g->gtab[0]);
    dfree(g->gtab[1]);
    if (cap == kMaxCap && h.next_entry > cap) return invalid("layout GUIDE needs fewer than 2^32 table entries");
    // the counters ran on past the room: every table that was asked for is
    // counted, though the children of those that did not fit are not (a
    // lower bound, so a deep graph may take another pass); lists that ran
    // out grow as well
    if (lists_full) {
      if (most > tcap) tcap = std::max(tcap * 2, most + most / 4);
      if (most_big > tcap_big) tcap_big = std::max(tcap_big * 2, most_big + most_big / 4);
      if (tcap + tcap_big >= (1ull << 32)) return invalid("layout GUIDE needs fewer than 2^32 child tables per level");
      cap = std::min(kMaxCap, std::max<uint64_t>(cap, h.next_entry + h.next_entry / 4));
    } else {
      cap = std::min<uint64_t>(kMaxCap, h.next_entry + h.next_entry / 8 + (1u << 20));
    }
  }
}

uint32_t log2_exact(uint32_t v) {
  uint32_t l = 0;
  while ((1u << l) < v) ++l;
  return l;
}

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

void drop_pool(fppr_graph* g) {
  if (!g->pool) return;
  (void)hipDeviceSynchronize();
  g->device_bytes -= align_up(g->pool_cap * 8);
  dfree(g->pool);
  g->pool_cap = 0;
  g->has_pool = false;
  g->n_small = 0;
}

fppr_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? FPPR_OUT_OF_MEMORY : FPPR_DEVICE_ERROR;
}

WalkDesc make_desc(const fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                   uint64_t n_sources, uint32_t* endpoints, uint64_t first, uint64_t walk0,
                   uint64_t count) {
  (void)n_sources;
  const bool stitch = (p->flags & FPPR_STITCH) != 0;
  WalkDesc D{};
  D.rec = g->rec;
  D.blocks = g->blocks;
  D.ghead = g->ghead;
  D.gent = g->gent;
  D.g_cap = g->g_cap;
  D.pool = stitch ? g->pool : nullptr;
  D.S_small = stitch ? g->pool_opts.S : 0u;
  D.sources = sources;
  D.endpoints = endpoints;
  D.first = first;
  D.count = count;
  D.walk0 = walk0;
  D.R_magic = ~0ull / p->R;
  D.R = p->R;
  D.n = g->n;
  D.key0 = static_cast<uint32_t>(p->seed);
  D.key1 = static_cast<uint32_t>(p->seed >> 32);
  D.T = fppr_alpha_threshold(p->alpha);
  D.tree_min = g->tree_min;
  D.K_log2 = stitch ? g->K_log2 : 0;
  D.flags = (g->narrow ? kDescNarrow : 0u) | (g->tagged ? kDescTagged : 0u) | (g->guide ? kDescGuide : 0u);
  return D;
}

AggLaunch make_agg(const fppr_params* p, const uint32_t* endpoints, const uint32_t* sources,
                   uint64_t n_sources, const fppr_out* out) {
  AggLaunch a{};
  a.endpoints = endpoints;
  a.sources = sources;
  a.n_src = n_sources;
  a.R = p->R;
  a.k = p->topk;
  a.topk = p->topk ? out->topk : nullptr;
  a.counts = (p->flags & FPPR_COUNTS) ? out->counts : nullptr;
  a.n_distinct = (p->flags & FPPR_COUNTS) ? out->n_distinct : nullptr;
  a.digest = (p->flags & FPPR_DIGESTS) ? out->digest : nullptr;
  return a;
}

fppr_status check_outputs(const fppr_params* p, const fppr_out* out) {
  if (!out) {
    set_error("out is NULL");
    return FPPR_INVALID_ARGUMENT;
  }
  std::string msg;
  if (p->topk && !out->topk) msg = "topk > 0 needs out->topk";
  else if ((p->flags & FPPR_COUNTS) && (!out->counts || !out->n_distinct))
    msg = "FPPR_COUNTS needs out->counts and out->n_distinct";
  else if ((p->flags & FPPR_DIGESTS) && !out->digest) msg = "FPPR_DIGESTS needs out->digest";
  if (msg.empty()) return FPPR_OK;
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

}  // namespace fppr

using namespace fppr;

extern "C" {

FPPR_API const char* fppr_last_error(void) { return g_last_error.c_str(); }

FPPR_API uint32_t fppr_alpha_threshold(double alpha) {
  if (!(alpha > 0.0 && alpha < 1.0)) return 0;
  double t = std::floor(alpha * 4294967296.0 + 0.5);
  if (t < 1.0) t = 1.0;
  if (t > 4294967295.0) t = 4294967295.0;
  return static_cast<uint32_t>(t);
}

FPPR_API uint64_t fppr_walks_for_guarantee(double eps, double delta, double pf) {
  if (!(eps > 0.0) || !(delta > 0.0 && delta <= 1.0) || !(pf > 0.0 && pf < 1.0)) return 0;
  const double r = std::ceil((2.0 + 2.0 * eps / 3.0) * std::log(2.0 / pf) / (eps * eps * delta));
  if (!(r < 1.8e19)) return 0;
  return static_cast<uint64_t>(r);
}

FPPR_API fppr_status fppr_graph_create(const fppr_csr* csr, const fppr_graph_opts* opts,
                                       void* stream, fppr_graph** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  if (!csr) return invalid("csr is NULL");
  if (csr->n == 0 || csr->n > 0xFFFFFFFEu) return invalid("n must be in [1, 2^32-2]");
  if (csr->m >= kMaxEdges) return invalid("m must be below 2^36");
  if (!csr->row_offsets) return invalid("row_offsets is NULL");
  if (csr->m && (!csr->col || !csr->w)) return invalid("col or w is NULL");
  if (csr->mem != FPPR_MEM_HOST && csr->mem != FPPR_MEM_DEVICE) return invalid("mem must be HOST or DEVICE");
  uint32_t H = kLeafEdges;
  if (opts && opts->hub_threshold) H = opts->hub_threshold;
  if (H < kLeafEdges) H = kLeafEdges;
  const uint32_t layout = opts ? opts->layout : FPPR_LAYOUT_AUTO;
  if (layout != FPPR_LAYOUT_AUTO && layout != FPPR_LAYOUT_WIDE && layout != FPPR_LAYOUT_NARROW &&
      layout != FPPR_LAYOUT_GUIDE)
    return invalid("layout must be AUTO, WIDE, NARROW or GUIDE");
  if (layout == FPPR_LAYOUT_GUIDE && csr->n > kMaxTaggedNodes) return invalid("layout GUIDE needs n <= 2^30");
  hipStream_t s = static_cast<hipStream_t>(stream);

  fppr_graph* g = new fppr_graph();
  g->n = csr->n;
  g->m = csr->m;
  g->tree_min = H;
  g->tagged = csr->n <= kMaxTaggedNodes;
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipGetDevice");
  }
  const uint64_t n = g->n, m = g->m;
  uint64_t* acc = &g->device_bytes;
#define FPPR_TRY(expr, what)        \
  do {                              \
    hipError_t e_ = (expr);         \
    if (e_ != hipSuccess) {         \
      fppr_status st_ = hip_fail(e_, what); \
      free_graph(g);                \
      return st_;                   \
    }                               \
  } while (0)

  if (csr->mem == FPPR_MEM_HOST) {
    uint64_t* off = nullptr;
    uint32_t *col = nullptr, *w = nullptr;
    g->owns_csr = true;
    FPPR_TRY(dmalloc(&off, n + 1, acc), "hipMalloc(row_offsets)");
    g->off = off;
    FPPR_TRY(dmalloc(&col, m, acc), "hipMalloc(col)");
    g->col = col;
    FPPR_TRY(dmalloc(&w, m, acc), "hipMalloc(w)");
    g->w = w;
    FPPR_TRY(hipMemcpyAsync(off, csr->row_offsets, (n + 1) * 8, hipMemcpyHostToDevice, s), "copy offsets");
    if (m) {
      FPPR_TRY(hipMemcpyAsync(col, csr->col, m * 4, hipMemcpyHostToDevice, s), "copy col");
      FPPR_TRY(hipMemcpyAsync(w, csr->w, m * 4, hipMemcpyHostToDevice, s), "copy w");
    }
  } else {
    g->off = csr->row_offsets;
    g->col = csr->col;
    g->w = csr->w;
  }
  if (layout != FPPR_LAYOUT_GUIDE) {
    FPPR_TRY(dmalloc(&g->rec, n, acc), "hipMalloc(rec)");
    FPPR_TRY(dmalloc(&g->region, n, acc), "hipMalloc(region)");
  }
  FPPR_TRY(dmalloc(&g->flag, n, acc), "hipMalloc(flag)");
  FPPR_TRY(dmalloc(&g->scan, n, acc), "hipMalloc(scan)");
  FPPR_TRY(dmalloc(&g->rows, n, acc), "hipMalloc(rows)");
  FPPR_TRY(dmalloc(&g->scan_blocks, scan_block_count(n) + 1, acc), "hipMalloc(scan blocks)");
  FPPR_TRY(dmalloc(&g->d_err, 16, acc), "hipMalloc(ctl)");

  FPPR_TRY(zero_ctl(g, s), "zero control words");
  FPPR_TRY(launch_validate(g, s, true), "validate");
  Ctl c{};
  FPPR_TRY(read_ctl(g, s, &c), "read validation");
  if (c.err) {
    std::string msg = "invalid CSR:" + err_bits(c.err);
    free_graph(g);
    return invalid(msg);
  }
  // narrow layout: every row total surely fits in 32 bits
  const bool fits = static_cast<uint64_t>(c.max_deg) * c.max_w <= 0xFFFFFFFFull;
  if (layout == FPPR_LAYOUT_NARROW && !fits) {
    free_graph(g);
    return invalid("layout NARROW needs max out-degree x max weight < 2^32");
  }
  g->narrow = layout == FPPR_LAYOUT_NARROW || (layout == FPPR_LAYOUT_AUTO && fits);
  g->guide = layout == FPPR_LAYOUT_GUIDE;
  FPPR_TRY(dmalloc(&g->live, n, acc), "hipMalloc(live nodes)");
  FPPR_TRY(dmalloc(&g->dang, n, acc), "hipMalloc(dangling nodes)");
  FPPR_TRY(launch_split_nodes(g, s), "split nodes");
  if (!g->guide) FPPR_TRY(launch_region_sizes(g, s), "region sizes");
  FPPR_TRY(read_ctl(g, s, &c), "read region sizes");
  g->n_live = c.live;
  g->n_dang = n - c.live;
  if (split_dangling(g)) {
    FPPR_TRY(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking), "hipStreamCreate(side)");
    FPPR_TRY(hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming), "hipEventCreate(fork)");
    FPPR_TRY(hipEventCreateWithFlags(&g->join_ev, hipEventDisableTiming), "hipEventCreate(join)");
  }
  if (g->tagged) {
    FPPR_TRY(dmalloc(&g->cls, n, acc), "hipMalloc(node classes)");
    FPPR_TRY(launch_node_class(g, 0, s), "node classes");
  }
  if (g->guide) {
    const fppr_status st = create_guide(g, s);
    if (st != FPPR_OK) {
      free_graph(g);
      return st;
    }
  } else {
    g->n_blocks = c.blocks;
    FPPR_TRY(dmalloc(&g->blocks, g->n_blocks, acc), "hipMalloc(blocks)");
    FPPR_TRY(launch_leaves(g, s, true), "leaf blocks");
  }
  FPPR_TRY(read_ctl(g, s, &c), "read build status");
  if (c.err) {
    std::string msg = "graph build failed:" + err_bits(c.err);
    free_graph(g);
    return invalid(msg);
  }
#undef FPPR_TRY
  g->n_tree = c.n_tree;
  *out = g;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_destroy(fppr_graph* g) {
  if (!g) return FPPR_OK;
  (void)hipDeviceSynchronize();
  free_graph(g);
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_info(const fppr_graph* g, uint32_t* n, uint64_t* m,
                                     uint32_t* n_hubs, uint64_t* n_small, uint64_t* device_bytes) {
  if (!g) return invalid("graph is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (n_hubs) *n_hubs = g->n_tree;
  if (n_small) *n_small = g->has_pool ? g->n_small : 0;
  if (device_bytes) *device_bytes = g->device_bytes;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_layout(const fppr_graph* g, uint32_t* layout) {
  if (!g || !layout) return invalid("graph or layout is NULL");
  *layout = g->guide ? FPPR_LAYOUT_GUIDE : (g->narrow ? FPPR_LAYOUT_NARROW : FPPR_LAYOUT_WIDE);
  return FPPR_OK;
}

static fppr_status pool_kernels(fppr_graph* g, hipStream_t s) {
  hipError_t e;
  if ((e = launch_small_flags(g, g->pool_opts.S, s)) != hipSuccess) return hip_fail(e, "small flags");
  if ((e = launch_small_compact(g, g->pool_opts.S, s)) != hipSuccess) return hip_fail(e, "small compact");
  if ((e = g->guide ? launch_pool_guide(g, s) : launch_pool(g, s)) != hipSuccess) return hip_fail(e, "pool");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_build_pool(fppr_graph* g, const fppr_pool_opts* o, void* stream) {
  if (!g || !o) return invalid("graph or opts is NULL");
  if (o->S < 1) return invalid("S must be >= 1");
  if (o->L < 1 || o->L > 255) return invalid("L must be in [1, 255]");
  if (!is_pow2(o->K) || o->K > 65536) return invalid("K must be a power of two in [1, 2^16]");
  const uint32_t T = fppr_alpha_threshold(o->alpha);
  if (!T) return invalid("alpha must be in (0, 1)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  uint64_t n_small = g->n_small;
  const bool retag = g->tagged && g->S_tag != o->S;
  if (!g->has_pool || g->pool_opts.S != o->S || retag) {
    if ((e = launch_small_flags(g, o->S, s)) != hipSuccess) return hip_fail(e, "small flags");
    Ctl c{};
    if ((e = read_ctl(g, s, &c)) != hipSuccess) return hip_fail(e, "read small count");
    if (c.err) return invalid("graph failed its last validation:" + err_bits(c.err));
    n_small = c.small;
  }
  // node-indexed: node v's K entries at v * K, so a walk that arrives at a
  // small node over a tagged edge finds its entry without the node's line
  // (entries of 16 bytes with guide tables: the end node's record rides along)
  const uint64_t need = static_cast<uint64_t>(g->n) * o->K * (g->guide ? 2u : 1u);
  if (!g->small_nodes) {
    if ((e = dmalloc(&g->small_nodes, g->n, &g->device_bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(small nodes)");
  }
  if (need > g->pool_cap || !g->pool) {
    if (g->pool) {
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
      g->device_bytes -= align_up(g->pool_cap * 8);
      dfree(g->pool);
      g->pool_cap = 0;
    }
    if ((e = dmalloc(&g->pool, need, &g->device_bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(pool)");
    g->pool_cap = need;
  }
  g->pool_opts = *o;
  g->pool_T = T;
  g->K_log2 = log2_exact(o->K);
  g->n_small = n_small;
  g->has_pool = true;
  if (retag) {  // the leaves' small-node tags follow the pool's S (the leaf kernels count long rows from 0)
    if ((e = zero_ctl(g, s)) != hipSuccess) return hip_fail(e, "zero control words");
    if ((e = launch_node_class(g, o->S, s)) != hipSuccess) return hip_fail(e, "node classes");
    if ((e = derive(g, s)) != hipSuccess) return hip_fail(e, "leaf blocks");
  }
  return pool_kernels(g, s);
}

FPPR_API fppr_status fppr_graph_export_pool(const fppr_graph* g, uint64_t* entries, uint64_t count,
                                            void* stream) {
  if (!g || !entries) return invalid("graph or entries is NULL");
  if (!g->has_pool) return invalid("no pool built");
  const uint64_t total = g->n_small * g->pool_opts.K;
  if (count < total) return invalid("entries too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!total) return FPPR_OK;
  uint64_t* tmp = nullptr;  // the canonical order, gathered from the node-indexed pool
  hipError_t e = hipMalloc(&tmp, total * 8);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(pool export)");
  e = g->guide ? launch_pool_guide_export(g, tmp, s) : launch_pool_export(g, tmp, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(entries, tmp, total * 8, hipMemcpyDeviceToHost);
  (void)hipFree(tmp);
  if (e != hipSuccess) return hip_fail(e, "export pool");
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_rebuild(fppr_graph* g, void* stream) {
  if (!g) return invalid("graph is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if ((e = zero_ctl(g, s)) != hipSuccess) return hip_fail(e, "zero control words");
  if ((e = launch_validate(g, s, false)) != hipSuccess) return hip_fail(e, "validate");
  if ((e = derive(g, s)) != hipSuccess) return hip_fail(e, "derive");
  if (g->has_pool) return pool_kernels(g, s);
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_set_hub_threshold(fppr_graph* g, uint32_t hub_threshold, void* stream) {
  if (!g) return invalid("graph is NULL");
  uint32_t H = hub_threshold ? hub_threshold : kLeafEdges;
  if (H < kLeafEdges) H = kLeafEdges;
  if (H == g->tree_min) return FPPR_OK;
  if (g->guide) {  // guide tables have no prefix trees: nothing to lay out again
    g->tree_min = H;
    return FPPR_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  g->tree_min = H;
  if ((e = zero_ctl(g, s)) != hipSuccess) return hip_fail(e, "zero control words");
  if ((e = launch_region_sizes(g, s)) != hipSuccess) return hip_fail(e, "region sizes");
  Ctl c{};
  if ((e = read_ctl(g, s, &c)) != hipSuccess) return hip_fail(e, "read region sizes");
  if (c.blocks != g->n_blocks) {
    g->device_bytes -= align_up(g->n_blocks * sizeof(Block));
    dfree(g->blocks);
    g->n_blocks = 0;
    if ((e = dmalloc(&g->blocks, c.blocks, &g->device_bytes)) != hipSuccess) return hip_fail(e, "hipMalloc(blocks)");
    g->n_blocks = c.blocks;
  }
  if ((e = launch_leaves(g, s, true)) != hipSuccess) return hip_fail(e, "leaf blocks");
  if ((e = read_ctl(g, s, &c)) != hipSuccess) return hip_fail(e, "read build status");
  if (c.err) return invalid("graph build failed:" + err_bits(c.err));
  g->n_tree = c.n_tree;
  if (g->has_pool) {
    fppr_status st = pool_kernels(g, s);
    if (st != FPPR_OK) return st;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  }
  return FPPR_OK;
}

FPPR_API fppr_status fppr_graph_check(fppr_graph* g, void* stream) {
  if (!g) return invalid("graph is NULL");
  Ctl c{};
  hipError_t e = read_ctl(g, static_cast<hipStream_t>(stream), &c);
  if (e != hipSuccess) return hip_fail(e, "read control words");
  if (c.err) return invalid("graph rebuild failed:" + err_bits(c.err));
  return FPPR_OK;
}

}  // extern "C"

fppr_status fppr::check_params(const fppr_graph* g, const fppr_params* p) {
  if (!g || !p) return invalid("graph or params is NULL");
  if (!fppr_alpha_threshold(p->alpha)) return invalid("alpha must be in (0, 1)");
  if (p->R < 1 || p->R > kMaxR) return invalid("R must be in [1, 2^20]");
  if ((p->flags & FPPR_COUNTS) && p->R > kAggMaxR) return invalid("FPPR_COUNTS needs R <= 4096");
  if (p->topk > p->R || p->topk > 1024) return invalid("topk must be <= R and <= 1024");
  if (p->flags & ~(FPPR_STITCH | FPPR_COUNTS | FPPR_DIGESTS | FPPR_STATS)) return invalid("unknown flag bits");
  if (p->flags & FPPR_STITCH) {
    if (!g->has_pool) return invalid("FPPR_STITCH needs a pool (fppr_graph_build_pool)");
    if (g->pool_T != fppr_alpha_threshold(p->alpha)) return invalid("pool was built for another alpha");
  }
  return FPPR_OK;
}

extern "C" {

FPPR_API fppr_status fppr_plan(const fppr_graph* g, const fppr_params* p, uint64_t n_sources,
                               uint64_t* workspace_bytes) {
  fppr_status st = check_params(g, p);
  if (st != FPPR_OK) return st;
  if (!workspace_bytes) return invalid("workspace_bytes is NULL");
  *workspace_bytes = kCtlBytes + kDescBytes + align_up(n_sources * p->R * 4ull) +
                     agg_table_bytes(n_sources, p->R, (p->flags & FPPR_COUNTS) != 0);
  return FPPR_OK;
}

FPPR_API fppr_status fppr_plan_block(const fppr_graph* g, const fppr_params* p, uint64_t n_sources,
                                     uint64_t budget_bytes, uint64_t* block_sources,
                                     uint64_t* workspace_bytes) {
  fppr_status st = check_params(g, p);
  if (st != FPPR_OK) return st;
  if (!block_sources || !workspace_bytes) return invalid("block_sources or workspace_bytes is NULL");
  uint64_t need = 0;
  fppr_plan(g, p, 1, &need);
  if (n_sources == 0 || need > budget_bytes) return invalid("not even one source fits the budget");
  // the plan grows with the block: the largest block that fits, by bisection
  uint64_t lo = 1, hi = n_sources;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    fppr_plan(g, p, mid, &need);
    if (need <= budget_bytes) lo = mid; else hi = mid - 1;
  }
  fppr_plan(g, p, lo, &need);
  *block_sources = lo;
  *workspace_bytes = need;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_run(fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                              uint64_t n_sources, void* workspace, uint64_t workspace_bytes,
                              const fppr_out* out, void* stream) {
  fppr_status st = check_params(g, p);
  if (st != FPPR_OK) return st;
  if (!out) return invalid("out is NULL");
  if (!sources && n_sources != g->n) return invalid("sources == NULL needs n_sources == n");
  if (n_sources == 0) return FPPR_OK;
  if (n_sources > (1ull << 40) / p->R) return invalid("n_sources * R too large");
  if (!workspace) return invalid("workspace is NULL");
  if ((st = check_outputs(p, out)) != FPPR_OK) return st;
  if ((p->flags & FPPR_STATS) && !out->stats) return invalid("FPPR_STATS needs out->stats");
  uint64_t need = 0, block = n_sources;
  fppr_plan(g, p, n_sources, &need);
  if (workspace_bytes < need) {  // memory-bounded run: blocks of sources that fit
    if (out->endpoints) return invalid("workspace smaller than fppr_plan (a blocked run needs out->endpoints == NULL)");
    if (fppr_plan_block(g, p, n_sources, workspace_bytes, &block, &need) != FPPR_OK)
      return invalid("workspace smaller than fppr_plan of one source");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* ctl = static_cast<unsigned long long*>(workspace);
  auto* desc = reinterpret_cast<WalkDesc*>(static_cast<char*>(workspace) + kCtlBytes);
  uint32_t* ws_ep = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) + kCtlBytes + kDescBytes);
  uint64_t* table = reinterpret_cast<uint64_t*>(static_cast<char*>(workspace) + kCtlBytes + kDescBytes +
                                                align_up(block * p->R * 4ull));
  const bool blocked = block < n_sources;
  fppr_stats* stats = (p->flags & FPPR_STATS) ? out->stats : nullptr;
  fppr_profile* prof = out->profile;
  hipError_t e = launch_zero_u64(reinterpret_cast<uint64_t*>(ctl), kCtlBytes / 8, s);
  if (e != hipSuccess) return hip_fail(e, "zero control words");
  if (prof && (e = hipEventRecord(prof->ev[0], s)) != hipSuccess) return hip_fail(e, "event");
  for (uint64_t r0 = 0; r0 < n_sources; r0 += block) {
    const uint64_t nb = std::min(block, n_sources - r0);
    // walk ids stay global (walk0 = r0 R): the kernel writes endpoints[w], so
    // the block buffer is addressed through a pointer moved back by r0 R
    uint32_t* ep_base = out->endpoints ? out->endpoints
                                       : reinterpret_cast<uint32_t*>(reinterpret_cast<uintptr_t>(ws_ep) -
                                                                     r0 * p->R * 4ull);
    if (r0 > 0 && (e = launch_zero_u64(reinterpret_cast<uint64_t*>(ctl), 1, s)) != hipSuccess)
      return hip_fail(e, "zero walk counter");  // the invalid-source flag accumulates
    // All nodes in one launch: the walk kernel takes the nodes with out-edges
    // and a coin-only kernel the others (their walks only restart at the
    // source and always end there); draws and results are those of one
    // launch over every node. The coin-only kernel (arithmetic only, few
    // registers, no LDS) runs on the graph's side stream, in the wave slots
    // the memory-bound walk kernel leaves free.
    const bool split = !sources && !blocked && split_dangling(g);
    WalkDesc D = split ? make_desc(g, p, g->live, g->n_live, ep_base, 0, 0, g->n_live * p->R)
                       : make_desc(g, p, sources, n_sources, ep_base, 0, r0 * p->R, nb * p->R);
    if (split) D.flags |= kDescEpBySource;
    if ((e = launch_set_desc(D, desc, s)) != hipSuccess) return hip_fail(e, "walk descriptor");
    const uint64_t total = (D.count + kWalkChunk - 1) / kWalkChunk * kWalkChunk;
    if (split) {  // the side stream starts after everything queued on `s` so far
      std::lock_guard<std::mutex> lk(g->side_mu);
      if ((e = hipEventRecord(g->fork_ev, s)) != hipSuccess) return hip_fail(e, "fork event");
      if ((e = hipStreamWaitEvent(g->side, g->fork_ev, 0)) != hipSuccess) return hip_fail(e, "fork wait");
    }
    if (total && (e = launch_walk(desc, &D, 1, total, ctl, stats, p->blocks_per_cu, s)) != hipSuccess)
      return hip_fail(e, "walk kernel");
    if (prof && !blocked && (e = hipEventRecord(prof->ev[4], s)) != hipSuccess) return hip_fail(e, "event");
    if (split) {
      std::lock_guard<std::mutex> lk(g->side_mu);
      if ((e = launch_dangling(g, p, ep_base, stats, g->side)) != hipSuccess) return hip_fail(e, "dangling walks");
      if ((e = hipEventRecord(g->join_ev, g->side)) != hipSuccess) return hip_fail(e, "join event");
      if ((e = hipStreamWaitEvent(s, g->join_ev, 0)) != hipSuccess) return hip_fail(e, "join wait");
    }
    if (prof && !blocked && (e = hipEventRecord(prof->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
    AggLaunch a = make_agg(p, out->endpoints ? out->endpoints + r0 * p->R : ws_ep, sources ? sources + r0 : nullptr,
                           nb, out);
    a.row0 = sources ? 0 : r0;
    if (a.topk) a.topk += r0 * a.k * 2;
    if (a.counts) a.counts += r0 * p->R * 2;
    if (a.n_distinct) a.n_distinct += r0;
    if (a.digest) a.digest += r0;
    a.table = table;
    if (prof && !blocked && (e = hipEventRecord(prof->ev[2], s)) != hipSuccess) return hip_fail(e, "event");
    if (a.topk || a.counts || a.digest) {
      if ((e = launch_aggregate(a, s)) != hipSuccess) return hip_fail(e, "aggregate kernel");
    }
  }
  if (prof && blocked) {  // blocked runs: the walk time covers every block's walks and counting
    if ((e = hipEventRecord(prof->ev[4], s)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventRecord(prof->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventRecord(prof->ev[2], s)) != hipSuccess) return hip_fail(e, "event");
  }
  if (prof && (e = hipEventRecord(prof->ev[3], s)) != hipSuccess) return hip_fail(e, "event");
  return FPPR_OK;
}

}  // extern "C"

// Workspace of fppr_run_static: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends. Host code never passes
// the array's name to a kernel or a copy (on the host it is only a stand-in
// for the symbol); it uses the device address hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[FPPR_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's copy of `scratch` (looked up on the
// first call on that device)
fppr_status static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return invalid("device index out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static workspace)");
    if (!ptr) return invalid("hipGetSymbolAddress returned no address for the static workspace");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FPPR_OK;
}
}  // namespace

extern "C" {

FPPR_API fppr_status fppr_run_static(fppr_graph* g, const fppr_params* p, const uint32_t* sources,
                                     uint64_t n_sources, const fppr_out* out, void* stream) {
  fppr_status st = check_params(g, p);
  if (st != FPPR_OK) return st;
  if (!out) return invalid("out is NULL");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != g->device) return invalid("fppr_run_static: the graph's device must be the current device");
  uint64_t one = 0, all = 0;
  fppr_plan(g, p, 1, &one);
  fppr_plan(g, p, n_sources, &all);
  if (one > FPPR_STATIC_SCRATCH_BYTES)
    return invalid("fppr_run_static: one source needs " + std::to_string(one) +
                   " bytes of workspace, above the static workspace of " +
                   std::to_string(FPPR_STATIC_SCRATCH_BYTES) + " bytes");
  if (out->endpoints && all > FPPR_STATIC_SCRATCH_BYTES)
    return invalid("fppr_run_static: with out->endpoints the whole run (" + std::to_string(all) +
                   " bytes) must fit the static workspace of " + std::to_string(FPPR_STATIC_SCRATCH_BYTES) +
                   " bytes");
  void* ws = nullptr;
  if ((st = static_scratch(dev, &ws)) != FPPR_OK) return st;
  return fppr_run(g, p, sources, n_sources, ws, FPPR_STATIC_SCRATCH_BYTES, out, stream);
}

namespace {
// the parameters counting uses (no graph): R, k and the output flags
fppr_status check_count_params(const fppr_params* p) {
  if (!p) return invalid("params is NULL");
  if (p->R < 1 || p->R > kMaxR) return invalid("R must be in [1, 2^20]");
  if ((p->flags & FPPR_COUNTS) && p->R > kAggMaxR) return invalid("FPPR_COUNTS needs R <= 4096");
  if (p->topk > p->R || p->topk > 1024) return invalid("topk must be <= R and <= 1024");
  if (p->flags & ~(FPPR_STITCH | FPPR_COUNTS | FPPR_DIGESTS | FPPR_STATS)) return invalid("unknown flag bits");
  return FPPR_OK;
}
}  // namespace

FPPR_API fppr_status fppr_aggregate_plan(const fppr_params* p, uint64_t n_sources, uint64_t* workspace_bytes) {
  fppr_status st = check_count_params(p);
  if (st != FPPR_OK) return st;
  if (!workspace_bytes) return invalid("workspace_bytes is NULL");
  *workspace_bytes = std::max<uint64_t>(kAlign, agg_table_bytes(n_sources, p->R, (p->flags & FPPR_COUNTS) != 0));
  return FPPR_OK;
}

FPPR_API fppr_status fppr_aggregate(const fppr_params* p, const uint32_t* endpoints, const uint32_t* sources,
                                    uint64_t n_sources, void* workspace, uint64_t workspace_bytes,
                                    const fppr_out* out, void* stream) {
  fppr_status st = check_count_params(p);
  if (st != FPPR_OK) return st;
  if ((st = check_outputs(p, out)) != FPPR_OK) return st;
  if (n_sources == 0) return FPPR_OK;
  if (!endpoints) return invalid("endpoints is NULL");
  if (n_sources > (1ull << 40) / p->R) return invalid("n_sources * R too large");
  uint64_t need = 0;
  fppr_aggregate_plan(p, n_sources, &need);
  if (!workspace || workspace_bytes < need) return invalid("workspace missing or smaller than fppr_aggregate_plan");
  AggLaunch a = make_agg(p, endpoints, sources, n_sources, out);
  a.table = static_cast<uint64_t*>(workspace);
  if (!(a.topk || a.counts || a.digest)) return FPPR_OK;
  const hipError_t e = launch_aggregate(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FPPR_OK : hip_fail(e, "aggregate kernel");
}

FPPR_API fppr_status fppr_profile_create(fppr_profile** out) {
  if (!out) return invalid("out is NULL");
  auto* p = new fppr_profile();
  for (auto& e : p->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      fppr_profile_destroy(p);
      return hip_fail(r, "hipEventCreate");
    }
  }
  *out = p;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_profile_destroy(fppr_profile* p) {
  if (!p) return FPPR_OK;
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_profile_read(fppr_profile* p, double* walk_ms, double* aggregate_ms) {
  if (!p) return invalid("profile is NULL");
  hipError_t e = hipEventSynchronize(p->ev[3]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  float a = 0.f, b = 0.f;
  if ((e = hipEventElapsedTime(&a, p->ev[0], p->ev[1])) != hipSuccess) return hip_fail(e, "elapsed");
  if ((e = hipEventElapsedTime(&b, p->ev[2], p->ev[3])) != hipSuccess) return hip_fail(e, "elapsed");
  if (walk_ms) *walk_ms = a;
  if (aggregate_ms) *aggregate_ms = b;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_profile_read_walk(fppr_profile* p, double* walk_kernel_ms, double* coin_only_ms) {
  if (!p) return invalid("profile is NULL");
  hipError_t e = hipEventSynchronize(p->ev[3]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  float a = 0.f, b = 0.f;
  if ((e = hipEventElapsedTime(&a, p->ev[0], p->ev[4])) != hipSuccess) return hip_fail(e, "elapsed");
  if ((e = hipEventElapsedTime(&b, p->ev[4], p->ev[1])) != hipSuccess) return hip_fail(e, "elapsed");
  if (walk_kernel_ms) *walk_kernel_ms = a;
  if (coin_only_ms) *coin_only_ms = b;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_run_check(const void* workspace, void* stream) {
  if (!workspace) return invalid("workspace is NULL");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "sync");
  unsigned long long ctl[2];
  e = hipMemcpy(ctl, workspace, sizeof ctl, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read run status");
  if (ctl[1] & 2) return invalid("a walk met guide tables that did not resolve its pick (rebuild the graph)");
  if (ctl[1]) return invalid("a source id was >= n (its walks were skipped)");
  return FPPR_OK;
}

}  // extern "C"
