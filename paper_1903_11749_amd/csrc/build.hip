// Graph ingest: CSR validation, per-row inclusive uint64 weight prefixes,
// 16-byte node records and hub top-level tables.
//
// Routing probability r(s,t) = w(s,t) / sum_v w(s,v) (Sec. 2.1) is realised
// on exact integers: the prefix P of a row is strictly increasing (w >= 1),
// so "first prefix above X" picks edge j for exactly P[j] - P[j-1] of the W
// values of X. Large rows (Sec. 4.1, alias tree) get a top-level table of
// every chunk-th prefix; searching it first and then one chunk returns the
// same edge as a flat search (Lemma 1's telescoping product, on integers).
#include "fppr_internal.hpp"

namespace fppr {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kShortRow = 64;  // rows up to this length: one thread each

__global__ void k_validate_offsets(const uint64_t* __restrict__ off, uint32_t n, uint64_t m,
                                   uint32_t* err) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u], b = off[u + 1];
    uint32_t e = 0;
    if (b < a) e |= kErrOffsets;
    else if (b - a > 0xFFFFFFFFull) e |= kErrDegree;
    if (u == 0 && a != 0) e |= kErrOffsets;
    if (u == n - 1 && b != m) e |= kErrOffsets;
    if (e) atomicOr(err, e);
  }
}

__global__ void k_validate_edges(const uint32_t* __restrict__ col, const uint32_t* __restrict__ w,
                                 uint64_t m, uint32_t n, uint32_t* err) {
  uint32_t e = 0;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (col[i] >= n) e |= kErrCol;
    if (w[i] == 0) e |= kErrWeight;
  }
  if (e) atomicOr(err, e);
}

// Short rows: one thread accumulates its row. Long rows are queued.
__global__ void k_prefix_short(const uint64_t* __restrict__ off, const uint32_t* __restrict__ w,
                               uint64_t* __restrict__ P, uint32_t n, uint32_t* rows,
                               uint32_t* n_rows) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u], b = off[u + 1];
    if (b <= a) continue;
    if (b - a > kShortRow) {
      rows[atomicAdd(n_rows, 1u)] = static_cast<uint32_t>(u);
      continue;
    }
    uint64_t acc = 0;
    for (uint64_t e = a; e < b; ++e) {
      acc += w[e];
      P[e] = acc;
    }
  }
}

// Long rows: one block per row, scanning tiles of kThreads*4 weights.
__global__ void __launch_bounds__(kThreads) k_prefix_long(const uint64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ w,
                                                          uint64_t* __restrict__ P,
                                                          const uint32_t* rows,
                                                          const uint32_t* n_rows) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint32_t nr = *n_rows;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const uint32_t u = rows[r];
    const uint64_t a = off[u], b = off[u + 1];
    uint64_t carry = 0;
    for (uint64_t t0 = a; t0 < b; t0 += kThreads * 4) {
      const uint64_t e0 = t0 + threadIdx.x * 4ull;
      uint64_t v[4];
      uint64_t local = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t e = e0 + k;
        local += (e < b) ? w[e] : 0u;
        v[k] = local;
      }
      uint64_t total;
      const uint64_t excl = block_exclusive_scan_u64<kThreads>(local, lds, &total);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint64_t e = e0 + k;
        if (e < b) P[e] = carry + excl + v[k];
      }
      carry += total;
    }
  }
}

__device__ __forceinline__ bool is_hub(uint64_t deg, uint32_t H) {
  return deg > H || deg > kMaxPlainDeg;
}

__global__ void k_hub_flags(const uint64_t* __restrict__ off, uint32_t n, uint32_t H,
                            uint32_t* flag) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    flag[u] = is_hub(off[u + 1] - off[u], H) ? 1u : 0u;
  }
}

__global__ void k_hub_chunks(const uint64_t* __restrict__ off, uint32_t n, uint32_t H,
                             uint32_t chunk_log2, uint32_t* flag) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t deg = off[u + 1] - off[u];
    flag[u] = is_hub(deg, H)
                  ? static_cast<uint32_t>((deg + (1ull << chunk_log2) - 1) >> chunk_log2)
                  : 0u;
  }
}

// Records, hub entries and top-level tables. hub_id = exclusive scan of hub
// flags, tl = exclusive scan of chunk counts; capacities guard rebuilds.
__global__ void k_records(const uint64_t* __restrict__ off, const uint64_t* __restrict__ P,
                          uint32_t n, uint32_t H, uint32_t chunk_log2,
                          const uint64_t* __restrict__ hub_id, const uint64_t* __restrict__ tl,
                          uint32_t hub_cap, uint64_t tl_cap, uint4* __restrict__ rec,
                          HubEntry* __restrict__ hubs, uint64_t* __restrict__ TL, uint32_t* err) {
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < n;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t a = off[u];
    const uint64_t deg = off[u + 1] - a;
    uint64_t W = 0;
    uint32_t code = 0;
    if (deg > 0) {
      W = P[a + deg - 1];
      if (is_hub(deg, H)) {
        const uint64_t h = hub_id[u];
        const uint64_t nch = (deg + (1ull << chunk_log2) - 1) >> chunk_log2;
        const uint64_t t0 = tl[u];
        if (h >= hub_cap || h >= kMaxHubs || t0 + nch > tl_cap) {
          atomicOr(err, kErrHubs);
          continue;
        }
        code = kHubFlag | static_cast<uint32_t>(h);
        hubs[h] = HubEntry{static_cast<uint32_t>(deg), static_cast<uint32_t>(nch), t0};
        for (uint64_t c = 0; c < nch; ++c) {
          uint64_t last = ((c + 1) << chunk_log2) - 1;
          if (last > deg - 1) last = deg - 1;
          TL[t0 + c] = P[a + last];
        }
      } else {
        code = static_cast<uint32_t>(deg);
      }
    }
    const uint64_t od = (a << kCodeBits) | code;
    rec[u] = make_uint4(static_cast<uint32_t>(W), static_cast<uint32_t>(W >> 32),
                        static_cast<uint32_t>(od), static_cast<uint32_t>(od >> 32));
  }
}

// ---- exclusive scan, u32 -> u64, three phases ----
constexpr int kScanItems = 4;
constexpr uint64_t kScanTile = kThreads * kScanItems;

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ in,
                                                          uint64_t n, uint64_t* blocks) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) v += in[base + k];
  uint64_t total;
  block_exclusive_scan_u64<kThreads>(v, lds, &total);
  if (threadIdx.x == 0) blocks[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) k_scan_blocks(uint64_t* blocks, uint64_t nb,
                                                          uint64_t* total_out) {
  __shared__ uint64_t lds[kThreads / 64];
  uint64_t carry = 0;
  for (uint64_t t0 = 0; t0 < nb; t0 += kThreads) {
    const uint64_t i = t0 + threadIdx.x;
    const uint64_t v = i < nb ? blocks[i] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan_u64<kThreads>(v, lds, &total);
    if (i < nb) blocks[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void __launch_bounds__(kThreads) k_scan_apply(const uint32_t* __restrict__ in,
                                                         uint64_t n,
                                                         const uint64_t* __restrict__ blocks,
                                                         uint64_t* __restrict__ out) {
  __shared__ uint64_t lds[kThreads / 64];
  const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = local;
    local += (base + k < n) ? in[base + k] : 0u;
  }
  uint64_t total;
  const uint64_t ex = block_exclusive_scan_u64<kThreads>(local, lds, &total) + blocks[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] = ex + v[k];
}

uint32_t grid_for(uint64_t items) {
  uint64_t b = (items + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<uint32_t>(b);
}

}  // namespace

uint64_t scan_block_count(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* blocks,
                           uint64_t* total_dev, hipStream_t s) {
  const uint64_t nb = scan_block_count(n);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<uint32_t>(nb)), dim3(kThreads), 0, s, in, n,
                     blocks);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kThreads), 0, s, blocks, nb, total_dev);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<uint32_t>(nb)), dim3(kThreads), 0, s, in, n,
                     blocks, out);
  return hipGetLastError();
}

hipError_t launch_validate(const fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_offsets, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n,
                     g->m, g->d_err);
  if (g->m)
    hipLaunchKernelGGL(k_validate_edges, dim3(grid_for(g->m)), dim3(kThreads), 0, s, g->col, g->w,
                       g->m, g->n, g->d_err);
  return hipGetLastError();
}

hipError_t launch_row_prefix(fppr_graph* g, hipStream_t s) {
  if (g->m == 0) return hipSuccess;
  uint32_t* n_rows = g->d_err + 1;
  hipLaunchKernelGGL(k_prefix_short, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->w,
                     g->P, g->n, g->rows, n_rows);
  hipLaunchKernelGGL(k_prefix_long, dim3(2048), dim3(kThreads), 0, s, g->off, g->w, g->P, g->rows,
                     n_rows);
  return hipGetLastError();
}

hipError_t launch_hub_flags(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_hub_flags, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, g->H,
                     g->flag);
  return launch_scan_u32(g->flag, g->scan, g->n, g->scan_blocks,
                         reinterpret_cast<uint64_t*>(g->d_err + 2), s);
}

hipError_t launch_hub_chunks(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_hub_chunks, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->n, g->H,
                     g->chunk_log2, g->flag);
  return launch_scan_u32(g->flag, g->scan2, g->n, g->scan_blocks,
                         reinterpret_cast<uint64_t*>(g->d_err + 4), s);
}

hipError_t launch_records(fppr_graph* g, hipStream_t s) {
  hipLaunchKernelGGL(k_records, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->off, g->P, g->n,
                     g->H, g->chunk_log2, g->scan, g->scan2, g->n_hub, g->n_tl, g->rec, g->hubs,
                     g->TL, g->d_err);
  return hipGetLastError();
}

}  // namespace fppr
