// Host build of the index arithmetic of two device paths, run against
// exact-size buffers with a bounds check on every access (and built with
// AddressSanitizer by tests/test_host_index_paths.py):
//
//  batch   the batch's workspace layout (batch_layout.hpp, the code
//          fppr_batch_create uses), then every walk id of the launch as the
//          walk kernel maps it (desc_of, walk_row: the kernel's own helpers):
//          its descriptor, the chunk's window of source rows in LDS, the
//          source id and the endpoint slot; the coin-only kernel's rows and
//          per-thread ranges; each item's counting extents. Every endpoint
//          slot of every item must be written exactly once.
//  agg     the large-budget counting kernel's hash paths, one block per row,
//          its threads taken one after the other: LDS table with double
//          hashing, spills to the global table, passes over the global
//          table, histogram threshold, candidate collection and radix select
//          (agg_hash.hpp, the kernel's own index functions). Results are
//          compared with a plain count and sort.
//
// Input (binary): see main(). Prints "ok" or the first violation and exits 1.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "agg_hash.hpp"
#include "batch_layout.hpp"
#include "fppr_internal.hpp"

using namespace fppr;

namespace {

[[noreturn]] void fail(const std::string& what) {
  printf("VIOLATION: %s\n", what.c_str());
  fflush(stdout);
  exit(1);
}

template <typename T>
struct Buf {  // exact-size buffer; every access is checked
  std::vector<T> v;
  const char* name;
  Buf(size_t n, T x, const char* nm) : v(n, x), name(nm) {}
  T& at(uint64_t i) {
    if (i >= v.size()) fail(std::string(name) + ": index " + std::to_string(i) + " >= " + std::to_string(v.size()));
    return v[i];
  }
};

FILE* g_in = nullptr;
uint64_t rd64() {
  uint64_t x;
  if (fread(&x, 8, 1, g_in) != 1) fail("short input");
  return x;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
struct Item {
  uint64_t n, R, counts, all;
  std::vector<uint32_t> src;   // explicit sources (may hold ids >= n)
  std::vector<uint32_t> live, dang;
};

void check_batch(const std::vector<Item>& items, const std::vector<uint64_t>& thread_counts) {
  const uint32_t count = static_cast<uint32_t>(items.size());
  std::vector<BatchItemShape> sh(count);
  for (uint32_t k = 0; k < count; ++k) {
    const Item& it = items[k];
    sh[k].n_rows = it.all ? it.n : it.src.size();
    sh[k].R = static_cast<uint32_t>(it.R);
    sh[k].counts = it.counts != 0;
    const uint64_t nd = it.dang.size();
    sh[k].split = it.all && nd > 0 && nd * 4 >= it.n;  // split_dangling
    sh[k].n_live = it.live.size();
  }
  const BatchLayout L = batch_layout(sh, sizeof(WalkDesc), kWalkChunk);
  // regions in order, disjoint, inside the workspace
  if (L.table < L.ctl + kBatchCtlBytes) fail("table overlaps control words");
  if (L.agg_table < L.table + count * sizeof(WalkDesc)) fail("walk table overlaps the counting tables");
  uint64_t at = L.agg_table + L.agg_bytes;
  for (uint32_t k = 0; k < count; ++k) {
    if (L.endpoints[k] < at) fail("endpoint buffer " + std::to_string(k) + " overlaps");
    if (L.endpoints[k] % 256) fail("endpoint buffer misaligned");
    if (L.endpoint_bytes[k] < sh[k].n_rows * sh[k].R * 4) fail("endpoint buffer too small");
    at = L.endpoints[k] + L.endpoint_bytes[k];
  }
  if (at > L.bytes) fail("endpoint buffers past the workspace");
  // the walk table
  uint64_t prev_end = 0;
  for (const BatchRun& r : L.runs) {
    if (r.first % kWalkChunk) fail("run does not start on a chunk");
    if (r.first < prev_end) fail("runs overlap");
    prev_end = r.first + (r.count + kWalkChunk - 1) / kWalkChunk * kWalkChunk;
  }
  if (prev_end != L.total) fail("total != end of the last run");
  const uint32_t nr = static_cast<uint32_t>(L.runs.size());
  // endpoint slots written per item
  std::vector<Buf<uint8_t>> wrote;
  for (uint32_t k = 0; k < count; ++k) wrote.emplace_back(L.endpoint_bytes[k] / 4, 0, "endpoint slots");
  const uint64_t n_chunks = L.total / kWalkChunk;
  const bool every = n_chunks <= (1ull << 16);
  std::vector<uint64_t> chunks;
  if (every) {
    for (uint64_t c = 0; c < L.total; c += kWalkChunk) chunks.push_back(c);
  } else {  // the first and last two chunks of every run and an odd stride through the launch
    for (const BatchRun& r : L.runs) {
      const uint64_t nc = (r.count + kWalkChunk - 1) / kWalkChunk;
      for (uint64_t j : {uint64_t{0}, uint64_t{1}, nc - 2, nc - 1})
        if (j < nc) chunks.push_back(r.first + j * kWalkChunk);
    }
    for (uint64_t j = 0; j < n_chunks; j += 1021) chunks.push_back(j * kWalkChunk);
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
  }
  for (uint64_t c : chunks) {
    const uint32_t d = desc_of(c, nr, [&](uint32_t j) { return L.runs.at(j).first; });
    const BatchRun& r = L.runs.at(d);
    const Item& it = items[r.item];
    const BatchItemShape& s = sh[r.item];
    const uint32_t R = s.R;
    const uint64_t R_magic = ~0ull / R;
    const uint64_t first = r.first, walk0 = 0;
    if (c < first) fail("chunk before its run");
    uint64_t end = first + r.count;
    if (c >= end) fail("chunk starts past its run's walks");
    if (c + kWalkChunk < end) end = c + kWalkChunk;
    const bool by_src = s.split;
    const bool has_src = s.split || !it.all;
    const std::vector<uint32_t>& rows_src = s.split ? it.live : it.src;
    uint64_t q_lo = 0, rows = 0, rm;
    if (has_src) {
      q_lo = walk_row(walk0 + (c - first), R, R_magic, &rm);
      const uint64_t q_hi = walk_row(walk0 + (end - 1 - first), R, R_magic, &rm);
      rows = q_hi - q_lo + 1;
      if (rows > kSrcBuf) fail("a chunk spans more source rows than the LDS window holds");
      for (uint64_t j = 0; j < rows; ++j)
        if (q_lo + j >= rows_src.size()) fail("source row past the source list");
    }
    for (uint64_t id = c; id < end; ++id) {
      const uint64_t w = walk0 + (id - first);
      uint64_t rem;
      const uint64_t q = walk_row(w, R, R_magic, &rem);
      if (rem >= R || q * R + rem != w) fail("walk_row");
      uint64_t src;
      if (has_src) {
        if (q < q_lo || q - q_lo >= rows) fail("row outside the chunk's LDS window");
        src = rows_src.at(q);
      } else {
        src = q;
      }
      const bool valid = src < it.n;
      if (!valid && by_src) fail("a split run met an invalid source");
      if (by_src) {
        wrote[r.item].at(src * R + rem) += 1;
      } else {
        wrote[r.item].at(w) += 1;  // endpoint (or the no-node mark for an invalid source)
      }
    }
  }
  // the coin-only kernel of split items: whole rows, then per-thread ranges
  for (uint32_t k = 0; k < count; ++k) {
    if (!sh[k].split) continue;
    const Item& it = items[k];
    const uint32_t R = sh[k].R;
    const uint64_t n_dang = it.dang.size();
    for (uint64_t q = 0; q < n_dang; q += every ? 1 : 97)
      for (uint32_t i = 0; i < R; ++i) wrote[k].at(static_cast<uint64_t>(it.dang.at(q)) * R + i) += 1;
    const uint64_t total = n_dang * R;
    const uint64_t R_magic = ~0ull / R;
    for (uint64_t threads : thread_counts) {
      const uint64_t per = (total + threads - 1) / threads;
      uint64_t seen = 0;
      for (uint64_t t = 0; t < threads; ++t) {
        const uint64_t w0 = t * per;
        uint64_t left = w0 < total ? (total - w0 < per ? total - w0 : per) : 0;
        if (!left) continue;
        uint64_t rem;
        uint64_t q = walk_row(w0, R, R_magic, &rem);
        uint32_t i = static_cast<uint32_t>(rem);
        (void)it.dang.at(q);
        if (left > R - i) (void)it.dang.at(q + 1);
        while (left) {  // row by row (the coins do not move indices)
          const uint64_t in_row = R - i;  // walks of the range left in row q
          if (left <= in_row) {
            seen += left;
            left = 0;
            break;
          }
          seen += in_row;  // the last walk of row q wraps into row q + 1
          left -= in_row;
          i = 0;
          q += 1;
          (void)it.dang.at(q);  // its source, loaded a row earlier
          if (left > R) (void)it.dang.at(q + 1);
        }
      }
      if (seen != total) fail("coin-only ranges do not cover the walks");
    }
  }
  for (uint32_t k = 0; k < count; ++k) {
    const uint64_t slots = sh[k].n_rows * sh[k].R;
    for (uint64_t i = 0; i < wrote[k].v.size(); ++i)
      if (every ? wrote[k].v[i] != (i < slots ? 1 : 0) : (wrote[k].v[i] > 1 || (i >= slots && wrote[k].v[i])))
        fail("item " + std::to_string(k) + ": endpoint slot " + std::to_string(i) + " written " +
             std::to_string(wrote[k].v[i]) + " times");
    // counting: reads n_rows * R endpoints; the hash path's tables
    if (agg_uses_table(sh[k].R, sh[k].counts) && sh[k].n_rows) {
      const uint64_t need = static_cast<uint64_t>(agg_table_groups(sh[k].n_rows, sh[k].R))
                            << (agg_table_log2(sh[k].R) + 3);
      if (need > L.agg_bytes) fail("counting tables past their area");
    }
  }
}

// ---------------------------------------------------------------------------
// large-budget counting (one block per row, threads in sequence)
// ---------------------------------------------------------------------------
uint64_t rank_key(uint64_t e) {  // larger = earlier (count desc, then t asc)
  return (static_cast<uint64_t>(static_cast<uint32_t>(e)) << 32) | static_cast<uint32_t>(~(e >> 32));
}

void table_add(Buf<uint64_t>& tab, uint64_t base, uint32_t log2, uint32_t t, uint32_t c) {
  uint32_t h = agg::table_home(t, log2);
  for (uint32_t probes = 0;; ++probes) {
    if (probes > (1u << log2)) fail("global table full");
    uint64_t& e = tab.at(base + h);
    if (e == agg::kEmpty) {
      e = (static_cast<uint64_t>(t) << 32) | c;
      return;
    }
    if ((e >> 32) == t) {
      e += c;
      return;
    }
    h = agg::table_next(h, log2);
  }
}

void check_agg_row(const std::vector<uint32_t>& ep_in, uint32_t k, uint32_t groups, uint32_t block) {
  const uint32_t R = static_cast<uint32_t>(ep_in.size());
  const uint32_t log2 = agg_table_log2(R);
  const uint32_t H = 1u << log2;
  const uint32_t T = agg::kBigThreads;
  Buf<uint32_t> ep(R, 0, "endpoints");
  for (uint32_t i = 0; i < R; ++i) ep.v[i] = ep_in[i];
  Buf<uint64_t> tab(static_cast<uint64_t>(groups) << log2, agg::kEmpty, "global table");
  const uint64_t base = static_cast<uint64_t>(block) << log2;
  Buf<uint32_t> lk(agg::kLdsSlots, kNoNode, "LDS keys"), lc(agg::kLdsSlots, 0, "LDS counts");
  Buf<uint32_t> hist(agg::kHistBins, 0, "histogram");
  Buf<uint64_t> cand(agg::kCandCap, 0, "candidates");
  // 1. count: LDS first, the global table for what does not fit there
  bool spill = false;
  for (uint32_t tid = 0; tid < T; ++tid) {
    for (uint32_t i0 = tid; i0 < R; i0 += 4 * T) {
      for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t i = i0 + u * T;
        const uint32_t t = i < R ? ep.at(i) : kNoNode;
        if (t == kNoNode) continue;
        uint32_t h = agg::lds_home(t);
        const uint32_t st = agg::lds_stride(t);
        bool done = false;
        for (uint32_t p = 0; p < agg::kLdsProbes && !done; ++p) {
          uint32_t& key = lk.at(h);
          if (key == kNoNode) key = t;
          if (key == t) {
            lc.at(h) += 1;
            done = true;
          }
          h = agg::lds_next(h, st);
        }
        if (!done) {
          spill = true;
          table_add(tab, base, log2, t, 1);
        }
      }
    }
  }
  std::vector<uint64_t> entries;  // what each pass sees
  auto each = [&](bool reset) {
    entries.clear();
    for (uint32_t tid = 0; tid < T; ++tid)
      for (uint32_t i = tid; i < agg::kLdsSlots; i += T)
        if (lk.at(i) != kNoNode) entries.push_back((static_cast<uint64_t>(lk.at(i)) << 32) | lc.at(i));
    if (!spill) return;
    for (uint32_t tid = 0; tid < T; ++tid) {
      auto pair = [&](uint32_t j) {
        for (uint32_t s = 0; s < 2; ++s) {
          uint64_t& e = tab.at(base + 2ull * j + s);
          if (e != agg::kEmpty) entries.push_back(e);
          if (reset) e = agg::kEmpty;
        }
      };
      agg::pass_pairs(
          tid, H, [&](uint32_t j) { for (uint32_t u = 0; u < 4; ++u) pair(j + u * T); }, pair);
    }
  };
  // 2. distinct endpoints and the histogram
  each(false);
  const uint64_t nd = entries.size();
  for (uint64_t e : entries) hist.at(agg::hist_bin(static_cast<uint32_t>(e))) += 1;
  // the plain count
  std::map<uint32_t, uint32_t> want;
  for (uint32_t i = 0; i < R; ++i)
    if (ep_in[i] != kNoNode) ++want[ep_in[i]];
  if (nd != want.size()) fail("distinct endpoints differ from the plain count");
  for (uint64_t e : entries)
    if (want.at(static_cast<uint32_t>(e >> 32)) != static_cast<uint32_t>(e)) fail("count differs");
  const uint32_t need = static_cast<uint32_t>(nd < k ? nd : k);
  // 3. threshold: thread j owns bins 2047 - 2j and 2046 - 2j
  int mode = 0;
  uint32_t cstar = 0, ncand = 0, setters = 0;
  if (need) {
    uint64_t above = 0;
    for (uint32_t tid = 0; tid < T; ++tid) {
      const uint32_t bh = agg::kHistBins - 1 - 2 * tid, bl = bh - 1;
      const uint32_t vh = hist.at(bh), vl = hist.at(bl);
      if (above < need && above + vh >= need) {
        cstar = bh;
        ncand = static_cast<uint32_t>(above + vh);
        ++setters;
      } else if (above + vh < need && above + vh + vl >= need) {
        cstar = bl;
        ncand = static_cast<uint32_t>(above + vh + vl);
        ++setters;
      }
      above += vh + vl;
    }
    if (setters != 1) fail("threshold set by " + std::to_string(setters) + " threads");
    mode = ncand <= agg::kCandCap ? 1 : 2;
  }
  uint64_t kmin = 0;
  if (mode == 2) {  // radix select of the need-th largest key among c >= cstar
    uint64_t prefix = 0;
    uint32_t rem = need;
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (uint32_t b = 0; b < 256; ++b) hist.at(b) = 0;
      for (uint64_t e : entries) {
        if (static_cast<uint32_t>(e) < cstar) continue;
        const uint64_t key = rank_key(e);
        if (shift == 56 || (key >> (shift + 8)) == (prefix >> (shift + 8))) hist.at((key >> shift) & 255u) += 1;
      }
      uint64_t above = 0;
      uint32_t digit = 256, nrem = 0;
      for (uint32_t tid = 0; tid < 256; ++tid) {
        const uint32_t v = hist.at(255 - tid);
        if (above < rem && above + v >= rem) {
          digit = 255 - tid;
          nrem = rem - static_cast<uint32_t>(above);
        }
        above += v;
      }
      if (digit == 256) fail("radix select found no digit");
      prefix |= static_cast<uint64_t>(digit) << shift;
      rem = nrem;
    }
    kmin = prefix;
  }
  // 4. collect (and empty the global table)
  uint32_t ns = 0;
  auto collect = [&](uint64_t e) {
    bool take = false;
    if (mode == 1) take = static_cast<uint32_t>(e) >= cstar;
    else if (mode == 2) take = rank_key(e) >= kmin;
    if (take) cand.at(ns++) = rank_key(e);
  };
  each(true);
  for (uint64_t e : entries) collect(e);
  for (uint64_t i = 0; i < tab.v.size(); ++i)
    if (tab.v[i] != agg::kEmpty) fail("global table not emptied by the last pass");
  // 5. sort and the top-k row
  if (need) {
    uint32_t P = 2;
    while (P < ns) P <<= 1;
    for (uint32_t i = ns; i < P; ++i) cand.at(i) = 0;
    std::vector<uint64_t> sorted(cand.v.begin(), cand.v.begin() + P);
    std::sort(sorted.begin(), sorted.end(), std::greater<uint64_t>());
    std::vector<std::pair<uint32_t, uint32_t>> ref;  // (count, t)
    for (auto& kv : want) ref.push_back({kv.second, kv.first});
    std::sort(ref.begin(), ref.end(), [](auto a, auto b) { return a.first != b.first ? a.first > b.first : a.second < b.second; });
    for (uint32_t q = 0; q < need; ++q) {
      const uint32_t t = ~static_cast<uint32_t>(sorted[q]), c = static_cast<uint32_t>(sorted[q] >> 32);
      if (t != ref[q].second || c != ref[q].first) fail("top-k entry " + std::to_string(q) + " differs");
    }
  }
}

}  // namespace

// Input: u64 kind. kind 1 (batch): u64 n_threads_counts, those u64 counts,
// u64 items, per item: u64 n, R, counts, all, n_src, n_src u32 (padded to 8
// bytes), n u8 dangling flags (padded to 8 bytes). kind 2 (agg): u64 rows,
// per row: u64 R, k, groups, block, then R u32 (padded to 8 bytes).
int main(int argc, char** argv) {
  if (argc != 2) fail("usage: host_index_paths <input>");
  g_in = fopen(argv[1], "rb");
  if (!g_in) fail("cannot open input");
  while (true) {
    uint64_t kind;
    if (fread(&kind, 8, 1, g_in) != 1) break;
    if (kind == 1) {
      std::vector<uint64_t> tc(rd64());
      for (auto& x : tc) x = rd64();
      std::vector<Item> items(rd64());
      for (Item& it : items) {
        it.n = rd64();
        it.R = rd64();
        it.counts = rd64();
        it.all = rd64();
        it.src.resize(rd64());
        if (!it.src.empty() && fread(it.src.data(), 4, it.src.size(), g_in) != it.src.size()) fail("short input");
        if (it.src.size() & 1) fseek(g_in, 4, SEEK_CUR);
        std::vector<uint8_t> dflag(it.n);
        if (it.n && fread(dflag.data(), 1, it.n, g_in) != it.n) fail("short input");
        if (it.n % 8) fseek(g_in, 8 - it.n % 8, SEEK_CUR);
        for (uint32_t v = 0; v < it.n; ++v) (dflag[v] ? it.dang : it.live).push_back(v);
      }
      check_batch(items, tc);
    } else if (kind == 2) {
      const uint64_t rows = rd64();
      for (uint64_t r = 0; r < rows; ++r) {
        const uint32_t R = static_cast<uint32_t>(rd64()), k = static_cast<uint32_t>(rd64());
        const uint32_t groups = static_cast<uint32_t>(rd64()), block = static_cast<uint32_t>(rd64());
        std::vector<uint32_t> ep(R);
        if (fread(ep.data(), 4, R, g_in) != R) fail("short input");
        if (R & 1) fseek(g_in, 4, SEEK_CUR);
        check_agg_row(ep, k, groups, block);
      }
    } else {
      fail("unknown input kind");
    }
  }
  printf("ok\n");
  return 0;
}
