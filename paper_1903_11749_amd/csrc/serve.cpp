// Serving: a resident graph answers PPR queries that arrive over time.
//
// Continuous mode. A scheduler thread admits queued queries in arrival order
// while slots and device memory allow (first-fit arena over one allocation
// made at create). Every admitted query owns its sources, endpoint buffer and
// outputs. The thread issues walk slices on the walk stream: one walk launch
// over a table that gives each admitted query with walks left a share of the
// slice (half in equal shares, the rest in admission order), so a query that
// arrives while others run joins at the next slice. Walk ids of a query are
// scheduled in order across slices; the walk index, not the slice, keys the
// draws. Slices alternate between two walk streams, so the next slice starts
// on the compute units that the current slice's longest walks leave idle (a
// launch otherwise ends with ~0.5 ms in which only its last walks run). After
// the slice holding a query's last walks, its counting and top-k
// run on the aggregation stream (waiting on that slice's event), the results
// are copied to pinned host memory and an event marks the query done. At most
// two slices are in flight, so the host builds the next table while the GPU
// runs the current one. This is the pipelined injection of Algorithm 2 (Sec.
// 4.3: new walks start while earlier ones are in flight, bounded by memory),
// applied to a stream of queries.
//
// FIFO mode (the comparison point): each admitted query is one plain walk
// launch over all its walks followed by its counting, all on one stream, in
// arrival order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fppr_internal.hpp"

using namespace fppr;

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kRing = 3;                 // slice tables: in flight + being built
constexpr size_t kMaxSlicesInFlight = 2;
constexpr uint64_t kCtlBytes = 256;

uint64_t now_ns() {
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now().time_since_epoch())
                                   .count());
}

fppr_status invalid(const std::string& msg) {
  set_error(msg);
  return FPPR_INVALID_ARGUMENT;
}

// First-fit allocator of offsets in one preallocated range; 256-byte
// granules; frees coalesce with their neighbours.
class Arena {
 public:
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    used_ -= bytes;
    uint64_t start = off, len = bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }
  uint64_t peak() const { return peak_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0, peak_ = 0;
};

enum class St { kQueued, kActive, kAggregating, kDone, kCancelled };

struct Req {
  uint64_t id = 0;
  fppr_params p{};
  uint32_t n = 0;
  uint64_t walks = 0, next = 0;  // walks scheduled so far: [0, next)
  uint64_t dev_off = 0, dev_bytes = 0, host_off = 0, host_bytes = 0;
  uint32_t* d_src = nullptr;
  uint32_t* d_ep = nullptr;
  uint32_t* d_topk = nullptr;
  uint64_t* d_digest = nullptr;
  uint32_t* h_src = nullptr;
  uint32_t* h_topk = nullptr;
  uint64_t* h_digest = nullptr;
  hipEvent_t done = nullptr;
  fppr_query_info info{};
  St st = St::kQueued;
  bool cancel = false;  // set by fppr_server_cancel while the query is on the GPU
};

// submit and completion times of a finished query, for the latency statistics
struct Done {
  uint64_t id, submit_ns, done_ns;
};

// device: sources | endpoints | top-k | digests
uint64_t dev_bytes_of(uint64_t n, uint64_t R, uint64_t k) {
  return align_up(n * 4) + align_up(n * R * 4) + align_up(n * k * 8) + align_up(n * 8);
}
// pinned host: sources | top-k | digests
uint64_t host_bytes_of(uint64_t n, uint64_t k) { return align_up(n * 4) + align_up(n * k * 8) + align_up(n * 8); }

}  // namespace

struct fppr_server {
  fppr_graph* g = nullptr;
  fppr_server_opts o{};
  int device = 0;
  char* dev_base = nullptr;
  char* host_base = nullptr;
  Arena dev_arena, host_arena;
  uint64_t* agg_table = nullptr;  // hash tables of R > 4096 counting (one stream uses them)
  fppr_stats* d_stats = nullptr;
  hipStream_t walk_s = nullptr, agg_s = nullptr;
  hipStream_t walk2_s = nullptr;  // continuous mode: slices alternate between walk_s and walk2_s
  hipStream_t up_s = nullptr;     // continuous mode: source uploads
  hipEvent_t up_ev = nullptr;     // recorded after the latest upload
  WalkDesc* h_tab[kRing] = {};
  WalkDesc* d_tab[kRing] = {};
  unsigned long long* d_ctl[kRing] = {};
  hipEvent_t ev[kRing] = {};
  bool ring_busy[kRing] = {};

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queued;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  uint64_t in_flight = 0;
  bool stop = false;
  bool failed = false;
  std::string error;
  fppr_server_counters st{};
  std::vector<Done> finished;  // every completed query since create, in completion order
  std::thread thr;
};

namespace {

bool fail(fppr_server* S, hipError_t e, const char* what) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->failed = true;
  S->error = std::string(what) + ": " + hipGetErrorString(e);
  S->cv_done.notify_all();
  return false;
}

bool enqueue_aggregate(fppr_server* S, Req* r, hipStream_t s) {
  fppr_out out{};
  out.topk = r->d_topk;
  out.digest = r->d_digest;
  AggLaunch a = make_agg(&r->p, r->d_ep, r->d_src, r->n, &out);
  a.table = S->agg_table;
  hipError_t e = launch_aggregate(a, s);
  if (e != hipSuccess) return fail(S, e, "aggregate kernel");
  const uint64_t k = r->p.topk;
  if ((e = hipMemcpyAsync(r->h_topk, r->d_topk, r->n * k * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(S, e, "copy top-k");
  if ((e = hipMemcpyAsync(r->h_digest, r->d_digest, r->n * 8ull, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(S, e, "copy digests");
  if ((e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming)) != hipSuccess) return fail(S, e, "event");
  if ((e = hipEventRecord(r->done, s)) != hipSuccess) return fail(S, e, "event record");
  r->st = St::kAggregating;
  return true;
}

// A cancelled query still on the GPU: no counting; an event behind what is
// already queued for it (the caller made agg_s wait for the slices in flight)
// frees its memory once the kernels that use it have finished.
bool enqueue_retire(fppr_server* S, Req* r, hipStream_t s) {
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming)) != hipSuccess) return fail(S, e, "event");
  if ((e = hipEventRecord(r->done, s)) != hipSuccess) return fail(S, e, "event record");
  r->st = St::kAggregating;
  return true;
}

// Launches one walk table held in ring slot `slot` (host copy filled) on
// stream ws.
bool launch_slot(fppr_server* S, int slot, uint32_t nd, uint64_t total, hipStream_t ws) {
  hipError_t e;
  if ((e = hipMemcpyAsync(S->d_tab[slot], S->h_tab[slot], nd * sizeof(WalkDesc), hipMemcpyHostToDevice,
                          ws)) != hipSuccess)
    return fail(S, e, "upload walk table");
  if ((e = launch_zero_u64(reinterpret_cast<uint64_t*>(S->d_ctl[slot]), kCtlBytes / 8, ws)) != hipSuccess)
    return fail(S, e, "zero control words");
  if ((e = launch_walk(S->d_tab[slot], S->h_tab[slot], nd, total, S->d_ctl[slot], S->d_stats, S->o.blocks_per_cu,
                       ws)) != hipSuccess)
    return fail(S, e, "walk kernel");
  if ((e = hipEventRecord(S->ev[slot], ws)) != hipSuccess) return fail(S, e, "event record");
  S->ring_busy[slot] = true;
  std::lock_guard<std::mutex> lk(S->mu);
  ++S->st.walk_launches;
  return true;
}

void loop(fppr_server* S) {
  if (hipSetDevice(S->device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->failed = true;
    S->error = "hipSetDevice in the scheduler thread";
    S->cv_done.notify_all();
    return;
  }
  const bool fifo = S->o.mode == FPPR_SERVE_FIFO;
  std::deque<Req*> active;       // admitted, walks left to schedule (admission order)
  std::deque<Req*> aggregating;  // done events pending (stream order)
  std::deque<int> slices;        // ring slots in flight (launch order)
  int ring = 0;
  uint64_t slice_no = 0;
  std::vector<uint64_t> take;

  for (;;) {
    bool progress = false;
    // 1. slices that finished free their ring slots
    while (!slices.empty() && hipEventQuery(S->ev[slices.front()]) == hipSuccess) {
      S->ring_busy[slices.front()] = false;
      slices.pop_front();
      progress = true;
    }
    // 2. finished queries
    while (!aggregating.empty()) {
      Req* r = aggregating.front();
      if (hipEventQuery(r->done) != hipSuccess) break;
      (void)hipEventDestroy(r->done);
      r->done = nullptr;
      aggregating.pop_front();
      std::lock_guard<std::mutex> lk(S->mu);
      r->info.done_ns = now_ns();
      S->dev_arena.release(r->dev_off, r->dev_bytes);
      --S->in_flight;
      if (r->cancel) {  // results not wanted: the pinned staging goes too
        S->host_arena.release(r->host_off, r->host_bytes);
        r->st = St::kCancelled;
        ++S->st.cancelled;
      } else {
        r->st = St::kDone;
        ++S->st.completed;
        S->finished.push_back(Done{r->id, r->info.submit_ns, r->info.done_ns});
      }
      S->cv_done.notify_all();
      progress = true;
    }
    // 3. admission: arrival order, while a slot and device memory are free
    std::vector<Req*> admitted;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      while (!S->queued.empty() && S->in_flight < S->o.max_requests) {
        Req* r = S->queued.front();
        uint64_t off = 0;
        if (!S->dev_arena.alloc(r->dev_bytes, &off)) break;  // the head waits for memory
        S->queued.pop_front();
        r->dev_off = off;
        char* base = S->dev_base + off;
        r->d_src = reinterpret_cast<uint32_t*>(base);
        base += align_up(r->n * 4ull);
        r->d_ep = reinterpret_cast<uint32_t*>(base);
        base += align_up(r->n * static_cast<uint64_t>(r->p.R) * 4);
        r->d_topk = reinterpret_cast<uint32_t*>(base);
        base += align_up(r->n * static_cast<uint64_t>(r->p.topk) * 8);
        r->d_digest = reinterpret_cast<uint64_t*>(base);
        r->info.admit_ns = now_ns();
        r->st = St::kActive;
        ++S->in_flight;
        S->st.peak_in_flight = std::max<uint64_t>(S->st.peak_in_flight, S->in_flight);
        S->st.peak_device_bytes = S->dev_arena.peak();
        admitted.push_back(r);
      }
    }
    for (Req* r : admitted) {
      hipError_t e = hipMemcpyAsync(r->d_src, r->h_src, r->n * 4ull, hipMemcpyHostToDevice,
                                    fifo ? S->walk_s : S->up_s);
      if (e == hipSuccess && !fifo) e = hipEventRecord(S->up_ev, S->up_s);
      if (e != hipSuccess) {
        fail(S, e, "upload sources");
        return;
      }
      progress = true;
      if (!fifo) {
        active.push_back(r);
        continue;
      }
      // FIFO: one plain launch over all the query's walks, then its counting
      const int slot = ring;
      ring = (ring + 1) % kRing;
      if (S->ring_busy[slot]) {  // the oldest slice in flight
        if ((e = hipEventSynchronize(S->ev[slot])) != hipSuccess) {
          fail(S, e, "event sync");
          return;
        }
        S->ring_busy[slot] = false;
        slices.pop_front();
      }
      S->h_tab[slot][0] = make_desc(S->g, &r->p, r->d_src, r->n, r->d_ep, 0, 0, r->walks);
      r->next = r->walks;
      const uint64_t total = (r->walks + kWalkChunk - 1) / kWalkChunk * kWalkChunk;
      if (!launch_slot(S, slot, 1, total, S->walk_s)) return;
      slices.push_back(slot);
      if (!enqueue_aggregate(S, r, S->walk_s)) return;
      aggregating.push_back(r);
      std::lock_guard<std::mutex> lk(S->mu);
      ++S->st.slices;
    }
    // 4a. cancelled admitted queries get no more walks; their memory is freed
    // once the slices in flight (which may hold their walks) have finished
    {
      std::vector<Req*> gone;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = active.begin(); it != active.end();) {
          if ((*it)->cancel) {
            gone.push_back(*it);
            it = active.erase(it);
          } else {
            ++it;
          }
        }
      }
      if (!gone.empty()) {
        for (int x : slices) {
          if (hipStreamWaitEvent(S->agg_s, S->ev[x], 0) != hipSuccess) {
            fail(S, hipErrorUnknown, "stream wait");
            return;
          }
        }
        for (Req* r : gone) {
          if (!enqueue_retire(S, r, S->agg_s)) return;
          aggregating.push_back(r);
        }
        progress = true;
      }
    }
    // 4. continuous: the next slice over every admitted query with walks left
    if (!fifo && !active.empty() && slices.size() < kMaxSlicesInFlight) {
      const int slot = ring;
      ring = (ring + 1) % kRing;
      if (S->ring_busy[slot]) {  // cannot happen with 2 in flight and 3 slots
        if (hipEventSynchronize(S->ev[slot]) != hipSuccess) {
          fail(S, hipErrorUnknown, "ring");
          return;
        }
        S->ring_busy[slot] = false;
      }
      // half of the slice in equal shares (a small query finishes in one
      // slice), the rest to the oldest queries first (the head keeps at least
      // half the rate, which bounds the tail latency)
      const uint64_t na = active.size();
      uint64_t budget = S->o.slice_walks;
      uint64_t fair = budget / 2 / na / kWalkChunk * kWalkChunk;
      if (fair < kWalkChunk) fair = kWalkChunk;
      take.assign(na, 0);
      for (uint64_t i = 0; i < na && budget; ++i) {
        const uint64_t left = active[i]->walks - active[i]->next;
        take[i] = std::min({left, fair, budget});
        budget -= take[i];
      }
      for (uint64_t i = 0; i < na && budget; ++i) {
        const uint64_t more = std::min(active[i]->walks - active[i]->next - take[i], budget);
        take[i] += more;
        budget -= more;
      }
      uint32_t nd = 0;
      uint64_t first = 0;
      for (uint64_t i = 0; i < na; ++i) {
        if (!take[i]) continue;
        Req* r = active[i];
        S->h_tab[slot][nd++] = make_desc(S->g, &r->p, r->d_src, r->n, r->d_ep, first, r->next, take[i]);
        first += (take[i] + kWalkChunk - 1) / kWalkChunk * kWalkChunk;
        r->next += take[i];
      }
      // Slices alternate between two streams: the next slice's blocks start
      // on the compute units that the current slice's last walks leave idle.
      hipStream_t ws = (slice_no++ & 1) ? S->walk2_s : S->walk_s;
      if (hipStreamWaitEvent(ws, S->up_ev, 0) != hipSuccess) {
        fail(S, hipErrorUnknown, "wait for source uploads");
        return;
      }
      if (!launch_slot(S, slot, nd, first, ws)) return;
      slices.push_back(slot);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->st.slices;
      }
      bool waited = false;
      for (auto it = active.begin(); it != active.end();) {
        Req* r = *it;
        if (r->next < r->walks) {
          ++it;
          continue;
        }
        if (!waited) {
          // every slice still in flight (this one and at most one before it,
          // on the other stream) may hold walks of the finished queries
          for (int x : slices) {
            hipError_t e = hipStreamWaitEvent(S->agg_s, S->ev[x], 0);
            if (e != hipSuccess) {
              fail(S, e, "stream wait");
              return;
            }
          }
          waited = true;
        }
        if (!enqueue_aggregate(S, r, S->agg_s)) return;
        aggregating.push_back(r);
        it = active.erase(it);
      }
      progress = true;
    }
    // 5. idle: wait for a submission or a little GPU progress
    if (!progress) {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop && S->queued.empty() && active.empty() && aggregating.empty() && slices.empty()) break;
      const bool gpu_busy = !aggregating.empty() || !slices.empty();
      S->cv_work.wait_for(lk, std::chrono::microseconds(gpu_busy ? 20 : 2000));
    }
  }
}

void free_server(fppr_server* S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : S->reqs) {
    if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    delete kv.second;
  }
  for (int i = 0; i < kRing; ++i) {
    if (S->h_tab[i]) (void)hipHostFree(S->h_tab[i]);
    if (S->d_tab[i]) (void)hipFree(S->d_tab[i]);
    if (S->d_ctl[i]) (void)hipFree(S->d_ctl[i]);
    if (S->ev[i]) (void)hipEventDestroy(S->ev[i]);
  }
  if (S->dev_base) (void)hipFree(S->dev_base);
  if (S->host_base) (void)hipHostFree(S->host_base);
  if (S->agg_table) (void)hipFree(S->agg_table);
  if (S->d_stats) (void)hipFree(S->d_stats);
  if (S->walk_s) (void)hipStreamDestroy(S->walk_s);
  if (S->walk2_s) (void)hipStreamDestroy(S->walk2_s);
  if (S->up_s) (void)hipStreamDestroy(S->up_s);
  if (S->up_ev) (void)hipEventDestroy(S->up_ev);
  if (S->agg_s) (void)hipStreamDestroy(S->agg_s);
  delete S;
}

// poll / wait of a cancelled query: FPPR_CANCELLED, and the id is forgotten
fppr_status forget_cancelled(fppr_server* S, Req* r) {
  S->reqs.erase(r->id);
  delete r;
  set_error("query was cancelled");
  return FPPR_CANCELLED;
}

fppr_status take_result(fppr_server* S, Req* r, uint32_t* topk, uint64_t* digest, fppr_query_info* info) {
  if (topk) std::memcpy(topk, r->h_topk, r->n * static_cast<uint64_t>(r->p.topk) * 8);
  if (digest) std::memcpy(digest, r->h_digest, r->n * 8ull);
  if (info) *info = r->info;
  S->host_arena.release(r->host_off, r->host_bytes);
  S->reqs.erase(r->id);
  delete r;
  return FPPR_OK;
}

}  // namespace

extern "C" {

FPPR_API fppr_status fppr_server_create(fppr_graph* g, const fppr_server_opts* opts, fppr_server** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  if (!g || !opts) return invalid("graph or opts is NULL");
  const fppr_server_opts& o = *opts;
  if (o.mode != FPPR_SERVE_CONTINUOUS && o.mode != FPPR_SERVE_FIFO) return invalid("unknown mode");
  if (o.max_requests < 1 || o.max_requests > 4096) return invalid("max_requests must be in [1, 4096]");
  if (o.memory_bytes < (1u << 20) || o.host_bytes < (1u << 20)) return invalid("memory budgets must be >= 1 MiB");
  if (o.mode == FPPR_SERVE_CONTINUOUS && o.slice_walks < (1u << 16)) return invalid("slice_walks must be >= 2^16");
  auto* S = new fppr_server();
  S->g = g;
  S->o = o;
  hipError_t e = hipGetDevice(&S->device);
#define FPPR_SERVE_TRY(expr, what)          \
  do {                                      \
    if ((e = (expr)) != hipSuccess) {       \
      fppr_status st_ = hip_fail(e, what);  \
      free_server(S);                       \
      return st_;                           \
    }                                       \
  } while (0)
  FPPR_SERVE_TRY(e, "hipGetDevice");
  FPPR_SERVE_TRY(hipMalloc(&S->dev_base, align_up(o.memory_bytes)), "hipMalloc(server memory)");
  FPPR_SERVE_TRY(hipHostMalloc(&S->host_base, align_up(o.host_bytes), hipHostMallocDefault), "hipHostMalloc");
  FPPR_SERVE_TRY(hipMalloc(&S->agg_table, std::max<uint64_t>(agg_table_bytes(kAggBigGroups, kMaxR, false), 256)),
                 "hipMalloc(counting tables)");
  FPPR_SERVE_TRY(hipMalloc(&S->d_stats, sizeof(fppr_stats)), "hipMalloc(stats)");
  FPPR_SERVE_TRY(hipMemset(S->d_stats, 0, sizeof(fppr_stats)), "zero stats");
  FPPR_SERVE_TRY(hipStreamCreateWithFlags(&S->walk_s, hipStreamNonBlocking), "stream");
  FPPR_SERVE_TRY(hipStreamCreateWithFlags(&S->walk2_s, hipStreamNonBlocking), "stream");
  FPPR_SERVE_TRY(hipStreamCreateWithFlags(&S->up_s, hipStreamNonBlocking), "stream");
  FPPR_SERVE_TRY(hipEventCreateWithFlags(&S->up_ev, hipEventDisableTiming), "event");
  FPPR_SERVE_TRY(hipEventRecord(S->up_ev, S->up_s), "event record");
  FPPR_SERVE_TRY(hipStreamCreateWithFlags(&S->agg_s, hipStreamNonBlocking), "stream");
  for (int i = 0; i < kRing; ++i) {
    FPPR_SERVE_TRY(hipHostMalloc(&S->h_tab[i], o.max_requests * sizeof(WalkDesc), hipHostMallocDefault),
                   "hipHostMalloc(walk table)");
    FPPR_SERVE_TRY(hipMalloc(&S->d_tab[i], o.max_requests * sizeof(WalkDesc)), "hipMalloc(walk table)");
    FPPR_SERVE_TRY(hipMalloc(&S->d_ctl[i], kCtlBytes), "hipMalloc(control words)");
    FPPR_SERVE_TRY(hipEventCreateWithFlags(&S->ev[i], hipEventDisableTiming), "event");
  }
#undef FPPR_SERVE_TRY
  S->dev_arena.reset(align_up(o.memory_bytes));
  S->host_arena.reset(align_up(o.host_bytes));
  S->thr = std::thread(loop, S);
  *out = S;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_server_submit(fppr_server* S, const fppr_query* q, uint64_t* id) {
  if (!S || !q || !id) return invalid("server, query or id is NULL");
  if (!q->sources || q->n_sources < 1) return invalid("a query needs at least one source");
  fppr_params p{};
  p.alpha = q->alpha;
  p.R = q->R;
  p.seed = q->seed;
  p.topk = q->topk;
  p.flags = (q->flags & FPPR_STITCH) | FPPR_DIGESTS;
  p.blocks_per_cu = S->o.blocks_per_cu;
  if (q->flags & ~static_cast<uint32_t>(FPPR_STITCH)) return invalid("query flags: only FPPR_STITCH");
  if (q->topk < 1) return invalid("topk must be >= 1");
  fppr_status st = check_params(S->g, &p);
  if (st != FPPR_OK) return st;
  for (uint32_t i = 0; i < q->n_sources; ++i)
    if (q->sources[i] >= S->g->n) return invalid("source id >= n");
  const uint64_t n = q->n_sources;
  const uint64_t dev = dev_bytes_of(n, p.R, p.topk), host = host_bytes_of(n, p.topk);
  if (dev > align_up(S->o.memory_bytes)) return invalid("query needs more device memory than the server has");
  if (host > align_up(S->o.host_bytes)) return invalid("query needs more pinned memory than the server has");
  auto* r = new Req();
  r->p = p;
  r->n = q->n_sources;
  r->walks = n * p.R;
  r->dev_bytes = dev;
  r->host_bytes = host;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->failed) {
      delete r;
      set_error(S->error);
      return FPPR_DEVICE_ERROR;
    }
    if (S->stop) {
      delete r;
      return invalid("server is shutting down");
    }
    uint64_t off = 0;
    if (!S->host_arena.alloc(host, &off)) {
      delete r;
      set_error("pinned staging full: poll finished queries, then submit again");
      return FPPR_CAPACITY;
    }
    r->host_off = off;
    char* base = S->host_base + off;
    r->h_src = reinterpret_cast<uint32_t*>(base);
    base += align_up(n * 4);
    r->h_topk = reinterpret_cast<uint32_t*>(base);
    base += align_up(n * p.topk * 8);
    r->h_digest = reinterpret_cast<uint64_t*>(base);
    std::memcpy(r->h_src, q->sources, n * 4);
    r->id = S->next_id++;
    r->info.submit_ns = now_ns();
    r->info.walks = r->walks;
    S->reqs[r->id] = r;
    S->queued.push_back(r);
    ++S->st.submitted;
    *id = r->id;
  }
  S->cv_work.notify_one();
  return FPPR_OK;
}

FPPR_API fppr_status fppr_server_poll(fppr_server* S, uint64_t id, uint32_t* topk, uint64_t* digest,
                                      fppr_query_info* info) {
  if (!S) return invalid("server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return invalid("unknown query id");
  if (it->second->st == St::kCancelled) return forget_cancelled(S, it->second);
  if (it->second->st != St::kDone) {
    if (S->failed) {
      set_error(S->error);
      return FPPR_DEVICE_ERROR;
    }
    return FPPR_NOT_READY;
  }
  return take_result(S, it->second, topk, digest, info);
}

FPPR_API fppr_status fppr_server_wait(fppr_server* S, uint64_t id, uint32_t* topk, uint64_t* digest,
                                      fppr_query_info* info) {
  if (!S) return invalid("server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return invalid("unknown query id");
    if (it->second->st == St::kDone) return take_result(S, it->second, topk, digest, info);
    if (it->second->st == St::kCancelled) return forget_cancelled(S, it->second);
    if (S->failed) {
      set_error(S->error);
      return FPPR_DEVICE_ERROR;
    }
    S->cv_done.wait(lk);
  }
}

FPPR_API fppr_status fppr_server_stats(fppr_server* S, fppr_server_counters* out) {
  if (!S || !out) return invalid("server or out is NULL");
  fppr_stats ws{};
  hipError_t e = hipMemcpy(&ws, S->d_stats, sizeof ws, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read server stats");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->walk_stats = ws;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_server_cancel(fppr_server* S, uint64_t id) {
  if (!S) return invalid("server is NULL");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return invalid("unknown query id");
    Req* r = it->second;
    switch (r->st) {
      case St::kQueued:  // never admitted: nothing on the GPU
        S->queued.erase(std::find(S->queued.begin(), S->queued.end(), r));
        S->host_arena.release(r->host_off, r->host_bytes);
        r->st = St::kCancelled;
        ++S->st.cancelled;
        break;
      case St::kDone:  // finished but not taken: its results are dropped
        S->host_arena.release(r->host_off, r->host_bytes);
        r->st = St::kCancelled;
        break;
      case St::kActive:
      case St::kAggregating:
        r->cancel = true;  // the scheduler stops its walks and frees it when the GPU is done with it
        break;
      case St::kCancelled:
        break;
    }
  }
  S->cv_work.notify_all();
  S->cv_done.notify_all();
  return FPPR_OK;
}

FPPR_API fppr_status fppr_server_latency(fppr_server* S, uint64_t first_id, fppr_latency* out) {
  if (!S || !out) return invalid("server or out is NULL");
  std::vector<uint64_t> lat;
  uint64_t t0 = ~0ull, t1 = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    lat.reserve(S->finished.size());
    for (const Done& d : S->finished) {
      if (d.id < first_id) continue;
      lat.push_back(d.done_ns - d.submit_ns);
      t0 = std::min(t0, d.submit_ns);
      t1 = std::max(t1, d.done_ns);
    }
  }
  *out = fppr_latency{};
  out->count = lat.size();
  if (lat.empty()) return FPPR_OK;
  std::sort(lat.begin(), lat.end());
  // nearest-rank percentile: the smallest latency with at least q of the queries at or below it
  auto pct = [&](double q) {
    uint64_t r = static_cast<uint64_t>(std::ceil(q * static_cast<double>(lat.size())));
    if (r < 1) r = 1;
    return static_cast<double>(lat[r - 1]) * 1e-6;
  };
  double sum = 0.0;
  for (uint64_t v : lat) sum += static_cast<double>(v);
  out->p50_ms = pct(0.50);
  out->p99_ms = pct(0.99);
  out->mean_ms = sum / static_cast<double>(lat.size()) * 1e-6;
  out->max_ms = static_cast<double>(lat.back()) * 1e-6;
  out->span_s = static_cast<double>(t1 - t0) * 1e-9;
  out->qps = out->span_s > 0 ? static_cast<double>(lat.size()) / out->span_s : 0.0;
  return FPPR_OK;
}

FPPR_API fppr_status fppr_server_destroy(fppr_server* S) {
  if (!S) return FPPR_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->thr.joinable()) S->thr.join();
  const bool failed = S->failed;
  const std::string err = S->error;
  free_server(S);
  if (failed) {
    set_error(err);
    return FPPR_DEVICE_ERROR;
  }
  return FPPR_OK;
}

}  // extern "C"
