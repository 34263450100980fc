// Exact big moves of one small node (Sec. 4.2, Algorithm 4; Lemma 2) in
// 62-bit fixed point, with a size cap.
//
// For a small node v: the distribution of the first k steps of a walk from v
// (pick an out-edge by weight, then stop with alpha = T / 2^32), split into
// terminated outcomes (stopped at t after j steps) and active ones (still
// going at t after j steps), expanded level by level:
//   F  the frontier: mass that has just arrived at a node (by node),
//   B  every arrival (by node and step), terminated weight = alpha x mass,
//   Z  frontier mass at a node without out-edges, frozen as an active
//      outcome of its own length (the walk's restart target is not v's).
// A level is expanded while (distinct nodes in B) + |F| + |Z| < d and the
// previous level reached a new node (Algorithm 4's stop rule), and only if
// the table cannot pass `cap` entries afterwards (the current entries plus
// two per out-edge of the frontier). Masses are units of 2^-62 with a floor
// after every product: first step floor(w 2^62 / W(v)); an edge (u, t) of a
// frontier entry of mass a carries floor(floor(a C / 2^32) w / W(u)) with C =
// 2^32 - T; terminated weight floor(a T / 2^32), active floor(a C / 2^32).
// Sums are exact, so the result does not depend on visiting order. Output:
// entries t | j << 32 | mark << 48 (mark 1 = terminated), zero weights
// dropped, sorted by entry, with the inclusive prefix of their weights
// (strictly increasing, so a pick is a binary search).
//
// Row totals must fit 32 bits (the narrow layout's bound), which keeps every
// product below 2^94 and every division a 96-by-32-bit one. Plain integer
// code, callable from a kernel (one thread per node) and from the host.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fppr {

constexpr uint64_t kBmOne = 1ull << 62;

// high 64 bits of a * b, from 32-bit limbs
__host__ __device__ inline uint64_t bm_mulhi(uint64_t a, uint64_t b) {
  const uint64_t a0 = static_cast<uint32_t>(a), a1 = a >> 32;
  const uint64_t b0 = static_cast<uint32_t>(b), b1 = b >> 32;
  const uint64_t p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
  const uint64_t mid = (p00 >> 32) + static_cast<uint32_t>(p01) + static_cast<uint32_t>(p10);
  return p11 + (p01 >> 32) + (p10 >> 32) + (mid >> 32);
}

// floor(a b / 2^32) for a <= 2^62, b < 2^32
__host__ __device__ inline uint64_t bm_mul_shr32(uint64_t a, uint32_t b) {
  const uint64_t lo = a * b, hi = bm_mulhi(a, b);
  return (hi << 32) | (lo >> 32);
}

// floor(a b / W) for a <= 2^62, 1 <= b <= W < 2^32 (quotient <= a)
__host__ __device__ inline uint64_t bm_mul_div(uint64_t a, uint32_t b, uint32_t W) {
  const uint64_t lo = a * b, hi = bm_mulhi(a, b);  // a b = hi:lo < 2^94
  uint64_t r = hi % W;
  uint64_t t = (r << 32) | (lo >> 32);
  const uint64_t q1 = t / W;
  r = t % W;
  t = (r << 32) | (lo & 0xFFFFFFFFull);
  return (q1 << 32) + t / W;
}

// adds mass to key in (k, m)[0, n), appending if absent; false when full
__host__ __device__ inline bool bm_add(uint64_t* k, uint64_t* m, uint32_t& n, uint32_t cap,
                                       uint64_t key, uint64_t mass) {
  for (uint32_t i = 0; i < n; ++i)
    if (k[i] == key) {
      m[i] += mass;
      return true;
    }
  if (n >= cap) return false;
  k[n] = key;
  m[n] = mass;
  ++n;
  return true;
}

// Workspace of one node: 8 arrays of cap words (B, F, F', Z keys and masses).
// Returns the number of entries written to out_e / out_w (entries and
// inclusive weight prefixes, at most cap), or
// 0xFFFFFFFF if a set outgrew cap (cannot happen when cap >= 2 deg(v)).
__host__ __device__ inline uint32_t big_moves_node(const uint64_t* off, const uint32_t* col,
                                                   const uint32_t* w, uint32_t v, uint32_t T,
                                                   uint32_t d, uint32_t cap, uint64_t* ws,
                                                   uint64_t* out_e, uint64_t* out_w) {
  uint64_t *bk = ws, *bm = ws + cap, *fk = ws + 2 * cap, *fm = ws + 3 * cap;
  uint64_t *gk = ws + 4 * cap, *gm = ws + 5 * cap, *zk = ws + 6 * cap, *zm = ws + 7 * cap;
  const uint32_t C = static_cast<uint32_t>((1ull << 32) - T);
  uint32_t nb = 0, nf = 0, nz = 0, nbt = 0;
  const uint64_t a0 = off[v], d0 = off[v + 1] - a0;
  uint32_t Wv = 0;
  for (uint64_t e = 0; e < d0; ++e) Wv += w[a0 + e];
  for (uint64_t e = 0; e < d0; ++e)
    if (!bm_add(fk, fm, nf, cap, col[a0 + e], bm_mul_div(kBmOne, w[a0 + e], Wv))) return 0xFFFFFFFFu;
  for (uint32_t i = 0; i < nf; ++i)
    if (!bm_add(bk, bm, nb, cap, fk[i] | (1ull << 32), fm[i])) return 0xFFFFFFFFu;
  nbt = nf;
  uint32_t j = 1, prev = 0;
  while (nbt + nf + nz < d && prev < nbt) {
    uint64_t out_edges = 0;
    for (uint32_t i = 0; i < nf; ++i) out_edges += off[fk[i] + 1] - off[fk[i]];
    if (nb + nf + nz + 2 * out_edges > cap) break;
    prev = nbt;
    uint32_t ng = 0;
    for (uint32_t i = 0; i < nf; ++i) {
      const uint32_t u = static_cast<uint32_t>(fk[i]);
      const uint64_t a = off[u], du = off[u + 1] - a;
      if (du == 0) {
        if (!bm_add(zk, zm, nz, cap, u | (static_cast<uint64_t>(j) << 32), fm[i])) return 0xFFFFFFFFu;
        continue;
      }
      uint32_t Wu = 0;
      for (uint64_t e = 0; e < du; ++e) Wu += w[a + e];
      const uint64_t c = bm_mul_shr32(fm[i], C);
      for (uint64_t e = 0; e < du; ++e)
        if (!bm_add(gk, gm, ng, cap, col[a + e], bm_mul_div(c, w[a + e], Wu))) return 0xFFFFFFFFu;
    }
    ++j;
    for (uint32_t i = 0; i < ng; ++i) {
      bool seen = false;
      for (uint32_t q = 0; q < nb; ++q) seen |= static_cast<uint32_t>(bk[q]) == static_cast<uint32_t>(gk[i]);
      if (!seen) ++nbt;
      if (!bm_add(bk, bm, nb, cap, gk[i] | (static_cast<uint64_t>(j) << 32), gm[i])) return 0xFFFFFFFFu;
    }
    for (uint32_t i = 0; i < ng; ++i) {
      fk[i] = gk[i];
      fm[i] = gm[i];
    }
    nf = ng;
  }
  // the table: terminated arrivals, the active frontier, frozen entries
  uint32_t n = 0;
  auto put = [&](uint64_t e, uint64_t q) {
    if (q == 0 || n >= cap) return;
    uint32_t p = n++;
    while (p > 0 && out_e[p - 1] > e) {  // insertion by entry
      out_e[p] = out_e[p - 1];
      out_w[p] = out_w[p - 1];
      --p;
    }
    out_e[p] = e;
    out_w[p] = q;
  };
  for (uint32_t i = 0; i < nb; ++i) put(bk[i] | (1ull << 48), bm_mul_shr32(bm[i], T));
  for (uint32_t i = 0; i < nf; ++i) put(fk[i] | (static_cast<uint64_t>(j) << 32), bm_mul_shr32(fm[i], C));
  for (uint32_t i = 0; i < nz; ++i) put(zk[i], bm_mul_shr32(zm[i], C));
  for (uint32_t i = 1; i < n; ++i) out_w[i] += out_w[i - 1];  // inclusive prefix
  return n;
}

}  // namespace fppr
