// Autotuner: picks a graph's hub threshold, walk-launch width and short-walk
// pool by timing trial runs on a sample of its sources. The paper sizes its
// per-round injection from memory and validates the choice by experiment
// (Sec. 4.3 and Sec. 5); on one GPU the knobs that matter are the layout of
// large rows, the launch width and whether stitching pays for its pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fppr_internal.hpp"

using namespace fppr;

namespace {

fppr_status invalid(const std::string& msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

// Device buffers of the trial runs, freed on scope exit.
struct TrialBuffers {
  uint32_t* sources = nullptr;
  uint32_t* endpoints = nullptr;
  unsigned long long* ctl = nullptr;
  WalkDesc* desc = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~TrialBuffers() {
    (void)hipDeviceSynchronize();
    if (sources) (void)hipFree(sources);
    if (endpoints) (void)hipFree(endpoints);
    if (ctl) (void)hipFree(ctl);
    if (desc) (void)hipFree(desc);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

struct Trial {
  fppr_graph* g;
  fppr_params p;
  TrialBuffers* buf;
  uint64_t n_sample;
  uint32_t reps;
  hipStream_t s;
  uint32_t count = 0;

  // best-of-reps walk time (ms) of the sample
  fppr_status walk_ms(bool stitch, uint32_t blocks_per_cu, double* ms) {
    fppr_params q = p;
    q.flags = stitch ? FPPR_STITCH : 0u;
    const WalkDesc D = make_desc(g, &q, buf->sources, n_sample, buf->endpoints, 0, 0, n_sample * q.R);
    const uint64_t total = (D.count + kWalkChunk - 1) / kWalkChunk * kWalkChunk;
    hipError_t e = launch_set_desc(D, buf->desc, s);
    if (e != hipSuccess) return hip_fail(e, "walk descriptor");
    double best = 1e300;
    for (uint32_t r = 0; r <= reps; ++r) {  // first pass warms caches, not timed
      if ((e = launch_zero_u64(reinterpret_cast<uint64_t*>(buf->ctl), 2, s)) != hipSuccess)
        return hip_fail(e, "zero control words");
      if ((e = hipEventRecord(buf->ev[0], s)) != hipSuccess) return hip_fail(e, "event");
      if ((e = launch_walk(buf->desc, &D, 1, total, buf->ctl, nullptr, blocks_per_cu, s)) != hipSuccess)
        return hip_fail(e, "walk kernel");
      if ((e = hipEventRecord(buf->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventSynchronize(buf->ev[1])) != hipSuccess) return hip_fail(e, "event sync");
      float t = 0.f;
      if ((e = hipEventElapsedTime(&t, buf->ev[0], buf->ev[1])) != hipSuccess) return hip_fail(e, "elapsed");
      if (r > 0) best = std::min(best, static_cast<double>(t));
    }
    ++count;
    *ms = best;
    return FPPR_OK;
  }

  // best-of-reps pool build time (ms); the pool is left built
  fppr_status pool_ms(const fppr_pool_opts& o, double* ms) {
    fppr_status st = fppr_graph_build_pool(g, &o, s);  // allocates if needed
    if (st != FPPR_OK) return st;
    double best = 1e300;
    for (uint32_t r = 0; r < reps; ++r) {
      hipError_t e = hipEventRecord(buf->ev[0], s);
      if (e != hipSuccess) return hip_fail(e, "event");
      if ((st = fppr_graph_build_pool(g, &o, s)) != FPPR_OK) return st;
      if ((e = hipEventRecord(buf->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventSynchronize(buf->ev[1])) != hipSuccess) return hip_fail(e, "event sync");
      float t = 0.f;
      if ((e = hipEventElapsedTime(&t, buf->ev[0], buf->ev[1])) != hipSuccess) return hip_fail(e, "elapsed");
      best = std::min(best, static_cast<double>(t));
    }
    *ms = best;
    return FPPR_OK;
  }
};

}  // namespace

extern "C" {

FPPR_API fppr_status fppr_autotune(fppr_graph* g, const fppr_params* p, const fppr_tune_space* sp,
                                   fppr_tune_result* res, void* stream) {
  if (!g || !p || !sp || !res) return invalid("graph, params, space or result is NULL");
  fppr_params base = *p;
  base.flags = 0;
  base.topk = 0;
  base.blocks_per_cu = 0;
  fppr_status st = check_params(g, &base);
  if (st != FPPR_OK) return st;
  if (sp->n_hub_thresholds && !sp->hub_thresholds) return invalid("hub_thresholds is NULL");
  if (sp->n_blocks_per_cu && !sp->blocks_per_cu) return invalid("blocks_per_cu is NULL");
  if (sp->n_pools && !sp->pools) return invalid("pools is NULL");
  for (uint32_t k = 0; k < sp->n_pools; ++k) {
    const fppr_pool_opts& o = sp->pools[k];
    if (o.S < 1 || o.L < 1 || o.L > 255 || !o.K || (o.K & (o.K - 1)) || o.K > 65536)
      return invalid("pool candidate " + std::to_string(k) + " is invalid");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t n = g->n;
  const uint64_t n_sample = sp->sample ? std::min<uint64_t>(sp->sample, n) : std::min<uint64_t>(n, 65536);
  const uint64_t n_sources = sp->n_sources ? sp->n_sources : n;
  const double scale = static_cast<double>(n_sources) / static_cast<double>(n_sample);

  TrialBuffers buf;
  hipError_t e;
  if ((e = hipMalloc(&buf.sources, n_sample * 4)) != hipSuccess) return hip_fail(e, "hipMalloc(sample)");
  if ((e = hipMalloc(&buf.endpoints, n_sample * base.R * 4ull)) != hipSuccess)
    return hip_fail(e, "hipMalloc(trial endpoints)");
  if ((e = hipMalloc(&buf.ctl, 256)) != hipSuccess) return hip_fail(e, "hipMalloc(ctl)");
  if ((e = hipMalloc(&buf.desc, sizeof(WalkDesc))) != hipSuccess) return hip_fail(e, "hipMalloc(desc)");
  for (hipEvent_t& ev : buf.ev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  {
    // evenly spread sample: row j -> floor(j * n / n_sample)
    std::vector<uint32_t> h(n_sample);
    for (uint64_t j = 0; j < n_sample; ++j) h[j] = static_cast<uint32_t>(j * n / n_sample);
    if ((e = hipMemcpy(buf.sources, h.data(), n_sample * 4, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "upload sample");
  }
  Trial tr{g, base, &buf, n_sample, sp->reps ? sp->reps : 3u, s};

  // 1. hub threshold, plain walks at full width
  uint32_t best_h = g->tree_min;
  double best = 1e300;
  if (sp->n_hub_thresholds) {
    for (uint32_t k = 0; k < sp->n_hub_thresholds; ++k) {
      if ((st = fppr_graph_set_hub_threshold(g, sp->hub_thresholds[k], s)) != FPPR_OK) return st;
      double ms = 0;
      if ((st = tr.walk_ms(false, 0, &ms)) != FPPR_OK) return st;
      if (ms < best) {
        best = ms;
        best_h = g->tree_min;
      }
    }
    if ((st = fppr_graph_set_hub_threshold(g, best_h, s)) != FPPR_OK) return st;
  } else if ((st = tr.walk_ms(false, 0, &best)) != FPPR_OK) {
    return st;
  }

  // 2. launch width, plain walks
  uint32_t best_b = 0;
  double best_plain = best;
  for (uint32_t k = 0; k < sp->n_blocks_per_cu; ++k) {
    const uint32_t b = sp->blocks_per_cu[k];
    if (b == 0) continue;  // the full width was timed in step 1
    double ms = 0;
    if ((st = tr.walk_ms(false, b, &ms)) != FPPR_OK) return st;
    if (ms < best_plain) {
      best_plain = ms;
      best_b = b;
    }
  }

  // 3. pools: build time plus stitched walks
  int32_t best_pool = -1;
  double best_cost = (sp->allow_plain || sp->n_pools == 0) ? best_plain * scale : 1e300;
  for (uint32_t k = 0; k < sp->n_pools; ++k) {
    fppr_pool_opts o = sp->pools[k];
    o.alpha = base.alpha;
    double build = 0, ms = 0;
    if ((st = tr.pool_ms(o, &build)) != FPPR_OK) return st;
    if ((st = tr.walk_ms(true, best_b, &ms)) != FPPR_OK) return st;
    const double cost = build + ms * scale;
    if (cost < best_cost) {
      best_cost = cost;
      best_pool = static_cast<int32_t>(k);
    }
  }
  if (best_pool < 0) {
    drop_pool(g);
  } else if (static_cast<uint32_t>(best_pool) + 1 != sp->n_pools) {
    fppr_pool_opts o = sp->pools[best_pool];
    o.alpha = base.alpha;
    if ((st = fppr_graph_build_pool(g, &o, s)) != FPPR_OK) return st;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "sync");
  res->hub_threshold = best_h;
  res->blocks_per_cu = best_b;
  res->pool = best_pool;
  res->trials = tr.count;
  res->est_ms = best_cost;
  res->plain_est_ms = best_plain * scale;
  return FPPR_OK;
}

}  // extern "C"
