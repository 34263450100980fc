// One row's alias table (Sec. 2.2, Algorithm 1) in exact integers: P[e] =
// n w(e) in units of 1/W, then Algorithm 1's updates with FIFO queues for
// the small and large sets (seeded in edge order; an edge that drops below W
// joins the back of the small set). small and large each hold d entries:
// an edge enters the small set at most once and the large set only at the
// start. Callable from a kernel (one thread per row) and from host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fppr {

__host__ __device__ inline void alias_row(const uint32_t* w, uint64_t d, uint64_t* P,
                                          uint32_t* alias, uint32_t* small, uint32_t* large) {
  uint64_t W = 0;
  for (uint64_t i = 0; i < d; ++i) W += w[i];
  uint64_t ns = 0, nl = 0;
  for (uint64_t i = 0; i < d; ++i) {
    const uint64_t p = d * w[i];
    P[i] = p;
    alias[i] = static_cast<uint32_t>(i);
    if (p < W) small[ns++] = static_cast<uint32_t>(i);
    else if (p > W) large[nl++] = static_cast<uint32_t>(i);
  }
  // The head of the large set keeps its threshold in a register until it
  // leaves the set (the same arithmetic; no memory round trip per step).
  uint64_t hs = 0, hl = 0, py = 0;
  bool held = false;
  while (hl < nl && hs < ns) {
    const uint32_t x = small[hs++];
    const uint32_t y = large[hl];
    if (!held) {
      py = P[y];
      held = true;
    }
    alias[x] = y;
    py -= W - P[x];
    if (py <= W) {
      P[y] = py;
      held = false;
      ++hl;
      if (py < W) small[ns++] = y;
    }
  }
  if (held) P[large[hl]] = py;
}

}  // namespace fppr
