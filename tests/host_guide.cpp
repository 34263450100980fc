// Host build of the guide-table routines (paper_1903_11749_amd/csrc/guide.hpp),
// the code the device kernels run, checked against plain definitions:
//
//  thresholds  reads pairs (P, W) and prints ceil(P 2^64 / W) for each, for
//              the caller to compare with exact integer arithmetic;
//  rows        reads rows of integer weights, builds each row's table and
//              child tables with containing + fill_entry (level by level, as the device
//              build does), then picks with pick() for many draws of every
//              row (random ones, every threshold and its neighbours, every
//              bucket edge) and compares each with the flat search "first
//              prefix above floor(D W / 2^64)". Every table access is bounds
//              checked. Prints entries, levels and mean reads per pick.
//
// Input (binary, little endian) on stdin:
//   thresholds: u64 mode=1, u64 count, then count x (u64 P, u64 W)
//   rows:       u64 mode=2, u64 rows, u64 draws per row, u64 seed, then per
//               row u64 d and d x u32 weights (>= 1)
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <deque>
#include <string>
#include <vector>

#include "guide.hpp"

using namespace fppr::guide;

namespace {

[[noreturn]] void fail(const std::string& what) {
  printf("VIOLATION: %s\n", what.c_str());
  fflush(stdout);
  exit(1);
}

uint64_t rd() {
  uint64_t v = 0;
  if (fread(&v, 8, 1, stdin) != 1) fail("short input");
  return v;
}

uint64_t splitmix(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// first edge whose inclusive prefix exceeds floor(D W / 2^64)
uint32_t flat_pick(const std::vector<uint64_t>& P, uint64_t D) {
  const uint64_t W = P.back();
  const uint64_t X = static_cast<uint64_t>((static_cast<unsigned __int128>(D) * W) >> 64);
  uint32_t lo = 0, hi = static_cast<uint32_t>(P.size()) - 1;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (P[mid] > X) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

int rows_mode() {
  const uint64_t nrows = rd(), draws = rd();
  uint64_t seed = rd();
  uint64_t entries_total = 0, reads_total = 0, picks_total = 0;
  uint32_t max_level = 0;
  for (uint64_t r = 0; r < nrows; ++r) {
    const uint64_t d = rd();
    if (d == 0 || d >= (1ull << 27)) fail("row length out of range");
    std::vector<uint64_t> P(d);
    uint64_t acc = 0;
    for (uint64_t j = 0; j < d; ++j) {
      uint32_t w = 0;
      if (fread(&w, 4, 1, stdin) != 1) fail("short row");
      if (w == 0) fail("zero weight");
      acc += w;
      P[j] = acc;
    }
    const uint64_t W = acc;
    std::vector<uint64_t> T(d > 1 ? d - 1 : 0);
    for (uint64_t j = 0; j + 1 < d; ++j) {
      T[j] = threshold(P[j], W);
      if (j && T[j] <= T[j - 1]) fail("thresholds not increasing");
    }
    auto Tf = [&](uint32_t j) -> uint64_t {
      if (j >= T.size()) fail("threshold index " + std::to_string(j) + " out of range");
      return T[j];
    };
    // candidate c's record: the edge index itself as the id
    auto rec = [&](uint32_t c) -> Cand {
      if (c >= d) fail("candidate out of range");
      return Cand{c, 0u, 0u};
    };
    const uint32_t lg = ceil_log2(d), kb = table_bits(lg);
    std::vector<Entry> ent(static_cast<size_t>(1) << kb);
    std::vector<uint32_t> level_of(ent.size(), 1);
    std::deque<std::pair<Pending, uint32_t>> todo;  // child tables with their level
    uint32_t cur_level = 1;
    auto push = [&](uint64_t lo, uint64_t hi, uint32_t first, uint32_t last, uint32_t nbk, uint32_t sh) -> uint32_t {
      if (last < first || last - first + 1 < 2) fail("child with fewer than two candidates");
      if (nbk < 2 || nbk > 2 * (last - first + 1)) fail("child bucket count out of range");
      const uint32_t base = static_cast<uint32_t>(ent.size());
      ent.resize(ent.size() + nbk);
      level_of.resize(ent.size(), cur_level + 1);
      Pending p{lo, hi, 0, first, last, static_cast<uint32_t>(r), sh, nbk, base};
      todo.push_back({p, cur_level + 1});
      return base;
    };
    // level 1 by the merge the short-row kernel uses, each entry's
    // candidates also found by the binary search the other kernels use
    for_row_buckets(Tf, static_cast<uint32_t>(d), kb, [&](uint32_t b, uint32_t c0, uint32_t c1) {
      uint64_t blo, bhi;
      row_bucket(kb, b, &blo, &bhi);
      if (c0 != containing(Tf, 0u, static_cast<uint32_t>(d - 1), blo) ||
          c1 != containing(Tf, 0u, static_cast<uint32_t>(d - 1), bhi))
        fail("merge and binary search disagree");
      Entry e{};  // push() may grow the table: fill a copy
      fill_entry(&e, Tf, rec, c0, c1, push);
      ent[b] = e;
    });
    while (!todo.empty()) {
      const Pending p = todo.front().first;
      cur_level = todo.front().second;
      todo.pop_front();
      if (cur_level > 64) fail("more than 64 levels");
      if (cur_level > max_level) max_level = cur_level;
      for (uint32_t i = 0; i < p.nbk; ++i) {
        uint64_t blo, bhi;
        child_bucket(p.origin, p.end, p.sh, i, &blo, &bhi);
        if (blo < p.origin || bhi >= p.end || bhi < blo) fail("child bucket outside its table");
        Entry e{};
        const uint32_t c0 = containing(Tf, p.a, p.b, blo), c1 = containing(Tf, p.a, p.b, bhi);
        if (c1 < c0) fail("empty bucket");
        fill_entry(&e, Tf, rec, c0, c1, push);
        ent[p.base + i] = e;
      }
    }
    entries_total += ent.size();
    auto entf = [&](uint32_t i) -> const Entry& {
      if (i >= ent.size()) fail("entry index out of range");
      return ent[i];
    };
    auto check = [&](uint64_t D) {
      uint32_t reads = 0;
      const Cand c = pick(entf, 0u, lg, D, &reads);
      const uint32_t want = flat_pick(P, D);
      if (c.id != want)
        fail("row " + std::to_string(r) + " d " + std::to_string(d) + " draw " + std::to_string(D) + ": guide " +
             std::to_string(c.id) + ", flat " + std::to_string(want));
      reads_total += reads;
      picks_total += 1;
    };
    for (uint64_t k = 0; k < draws; ++k) check(splitmix(&seed));
    check(0);
    check(~0ull);
    for (uint64_t j = 0; j + 1 < d; ++j) {
      check(T[j]);
      check(T[j] - 1);
      if (T[j] != ~0ull) check(T[j] + 1);
    }
    if (kb)
      for (uint64_t b = 1; b < (1ull << kb); ++b) {
        check((b << (64 - kb)) - 1);
        check(b << (64 - kb));
      }
  }
  printf("ok entries %llu levels %u reads_per_pick %.4f\n", static_cast<unsigned long long>(entries_total),
         max_level, picks_total ? static_cast<double>(reads_total) / picks_total : 0.0);
  return 0;
}

int thresholds_mode() {
  const uint64_t count = rd();
  for (uint64_t k = 0; k < count; ++k) {
    const uint64_t P = rd(), W = rd();
    if (!(P >= 1 && P < W && W <= (1ull << 63))) fail("threshold input out of range");
    const uint64_t t = threshold(P, W);
    fwrite(&t, 8, 1, stdout);
  }
  return 0;
}

}  // namespace

int main() {
  const uint64_t mode = rd();
  if (mode == 1) return thresholds_mode();
  if (mode == 2) return rows_mode();
  fail("unknown mode");
}
