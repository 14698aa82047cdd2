// Request server: admits independent solves of mixed dimensions, sizes and
// widths into a caller-provided HBM arena and runs them concurrently.
//
// Every request gets a resident hierarchy for its parameters (reused by later
// requests with bitwise-identical parameters, created inside the arena when
// the budget allows, idle ones evicted least-recently-used when it does not)
// and one of `max_slots` execution slots, each a HIP stream of its own. A
// slot runs the request's whole solve — FP64 right-hand sides of every level
// to BFP, FMG, the finest iterate back to FP64 into the caller's buffer — as
// one replay of a HIP graph captured once per resident hierarchy (the
// request's buffers reach the graph through a small device table of
// pointers, copied in before the replay), so a request costs the host two
// calls instead of a hundred launches; it then records an event. Polling
// checks events without blocking, frees finished
// slots and admits queued requests in arrival order (continuous batching:
// requests join as slots and memory free up, and the work of all running
// slots overlaps on the device). Each result is the same, bit for bit, as
// the solve run alone: every request owns its blocks and every operation is
// exact.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"

using namespace bfpk;

namespace {

struct Resident {
  mg_params prm;
  mg_hierarchy* h = nullptr;
  size_t off = 0, size = 0;
  const double** table = nullptr;   // device: rhs[0..L-1], x_out
  hipGraphExec_t graph = nullptr;
  bool busy = false;
  uint64_t last_use = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  const double** staging = nullptr;   // pinned host copy of a request's table
  int res = -1;
  uint64_t ticket = 0;
  bool busy = false;
};

constexpr size_t kTableBytes = 256;   // MG_MAX_LEVELS + 1 pointers, rounded up

void drop(Resident& r) {
  if (r.graph) hipGraphExecDestroy(r.graph);
  r.graph = nullptr;
  mg_hierarchy_destroy(r.h);
  r.h = nullptr;
}

struct Queued {
  uint64_t ticket;
  mg_request req;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Default executor threshold of the server's hierarchies: 2D grids up to
// 255^2 and 3D grids up to 31^3 run entirely inside one recorded program.
// Measured on MI355X with the serving trace: throughput is bounded by kernel
// dispatch rather than by compute when each request issues ~100 launches,
// so running more levels in one workgroup per request (fewer launches,
// longer single-request latency) keeps up with 2000 requests/s where the
// 4096-point default falls behind.
constexpr int64_t kServerExecPoints = 70000;

}  // namespace

struct mg_server {
  mg_server_cfg cfg;
  int64_t exec_points = 0;
  char* arena = nullptr;
  size_t bytes = 0;
  std::vector<Resident> pool;
  std::vector<std::pair<size_t, size_t>> free_ranges;   // (offset, size), sorted
  std::vector<Slot> slots;
  std::deque<Queued> queue;
  std::unordered_map<uint64_t, mg_result> finished;
  std::unordered_map<uint64_t, int> running;            // ticket -> slot
  uint64_t next_ticket = 1, clock = 0;

  ~mg_server() {
    for (Slot& s : slots) {
      if (s.stream) hipStreamSynchronize(s.stream);
      if (s.start) hipEventDestroy(s.start);
      if (s.done) hipEventDestroy(s.done);
      if (s.stream) hipStreamDestroy(s.stream);
      if (s.staging) hipHostFree(s.staging);
    }
    for (Resident& r : pool) drop(r);
  }

  // capture the whole solve of a resident hierarchy, reading the request's
  // buffers from its table
  int capture(Resident& r, hipStream_t s) {
    hipGraph_t g = nullptr;
    int rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
    if (rc) return rc;
    const int L = r.prm.L;
    for (int j = 1; j <= L && !rc; ++j) rc = set_rhs_table(r.h, j, r.table, j - 1, s);
    if (!rc) rc = mg_fmg(r.h, s);
    bfp_vec x;
    if (!rc) rc = mg_get_vec(r.h, L, 0, &x);
    if (!rc) rc = to_f64_impl(&x, nullptr, (double* const*)r.table, L, s);
    const int rc_end = hip_check(hipStreamEndCapture(s, &g), "graph capture");
    if (!rc) rc = rc_end;
    if (!rc) rc = hip_check(hipGraphInstantiate(&r.graph, g, nullptr, nullptr, 0), "graph instantiate");
    if (g) hipGraphDestroy(g);
    return rc;
  }

  // first-fit allocation of `size` bytes of the arena; false when no range fits
  bool alloc(size_t size, size_t* off) {
    for (size_t i = 0; i < free_ranges.size(); ++i) {
      if (free_ranges[i].second >= size) {
        *off = free_ranges[i].first;
        free_ranges[i].first += size;
        free_ranges[i].second -= size;
        if (!free_ranges[i].second) free_ranges.erase(free_ranges.begin() + i);
        return true;
      }
    }
    return false;
  }

  void release(size_t off, size_t size) {
    free_ranges.emplace_back(off, size);
    std::sort(free_ranges.begin(), free_ranges.end());
    std::vector<std::pair<size_t, size_t>> merged;
    for (auto& r : free_ranges) {
      if (!merged.empty() && merged.back().first + merged.back().second == r.first)
        merged.back().second += r.second;
      else
        merged.push_back(r);
    }
    free_ranges.swap(merged);
  }

  // an idle resident hierarchy for these parameters: reused, created, or
  // created after evicting idle ones (least recently used first); -1 when
  // the arena cannot hold it now
  int resident_for(const mg_params& p, hipStream_t s, int* rc) {
    const int64_t exec_points = this->exec_points;
    *rc = BFP_OK;
    for (size_t i = 0; i < pool.size(); ++i)
      if (!pool[i].busy && !std::memcmp(&pool[i].prm, &p, sizeof p)) return (int)i;
    size_t hb0 = 0;
    if ((*rc = hierarchy_bytes_ex(&p, exec_points, &hb0))) return -1;
    const size_t hb = align256(hb0);
    const size_t need = hb + kTableBytes;
    if (hb == 0 || need > bytes) {
      *rc = fail(BFP_ENOMEM, "a request needs %zu bytes of the %zu-byte arena", need, bytes);
      return -1;
    }
    size_t off;
    while (!alloc(need, &off)) {
      int victim = -1;
      for (size_t i = 0; i < pool.size(); ++i)
        if (!pool[i].busy && (victim < 0 || pool[i].last_use < pool[victim].last_use))
          victim = (int)i;
      if (victim < 0) return -1;   // everything resident is running: wait
      drop(pool[victim]);
      release(pool[victim].off, pool[victim].size);
      pool.erase(pool.begin() + victim);
      for (Slot& sl : slots)
        if (sl.busy && sl.res > victim) --sl.res;
    }
    Resident r;
    r.prm = p;
    r.off = off;
    r.size = need;
    r.table = (const double**)(arena + off + hb);
    if ((*rc = hierarchy_create_ex(&p, arena + off, hb, s, exec_points, &r.h)) ||
        (*rc = capture(r, s))) {
      if (r.h) drop(r);
      release(off, need);
      return -1;
    }
    pool.push_back(r);
    return (int)pool.size() - 1;
  }

  int launch(Slot& sl, int res, const Queued& q) {
    Resident& R = pool[res];
    const int L = R.prm.L;
    // the slot is idle, so its staging copy of the previous table was consumed
    for (int j = 0; j < L; ++j) sl.staging[j] = q.req.rhs_dev[j];
    sl.staging[L] = q.req.x_out_dev;
    int rc = hip_check(hipMemcpyAsync(R.table, sl.staging, (L + 1) * sizeof(double*),
                                      hipMemcpyHostToDevice, sl.stream), "request table");
    if (!rc) rc = hip_check(hipEventRecord(sl.start, sl.stream), "request start event");
    if (!rc) rc = hip_check(hipGraphLaunch(R.graph, sl.stream), "request graph");
    if (!rc) rc = hip_check(hipEventRecord(sl.done, sl.stream), "request done event");
    if (rc) return rc;
    R.busy = true;
    R.last_use = ++clock;
    sl.busy = true;
    sl.res = res;
    sl.ticket = q.ticket;
    running[q.ticket] = (int)(&sl - slots.data());
    return BFP_OK;
  }

  // retire finished slots, then admit queued requests in arrival order
  int progress() {
    for (Slot& sl : slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.done);
      if (e == hipErrorNotReady) continue;
      mg_result r{};
      r.status = e == hipSuccess ? BFP_OK : BFP_EHIP;
      float ms = 0.f;
      if (e == hipSuccess) hipEventElapsedTime(&ms, sl.start, sl.done);
      r.gpu_ms = ms;
      finished[sl.ticket] = r;
      running.erase(sl.ticket);
      pool[sl.res].busy = false;
      sl.busy = false;
      sl.res = -1;
    }
    while (!queue.empty()) {
      int free_slot = -1;
      for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i].busy) { free_slot = (int)i; break; }
      if (free_slot < 0) break;
      Slot& sl = slots[free_slot];
      int rc;
      const int res = resident_for(queue.front().req.prm, sl.stream, &rc);
      if (rc) {   // cannot ever run: report it and drop it
        mg_result r{};
        r.status = rc;
        finished[queue.front().ticket] = r;
        queue.pop_front();
        continue;
      }
      if (res < 0) break;   // memory busy: wait for running requests
      if ((rc = launch(sl, res, queue.front()))) return rc;
      queue.pop_front();
    }
    return BFP_OK;
  }
};

extern "C" {

int mg_server_create(const mg_server_cfg* cfg, void* arena_dev, size_t bytes, mg_server** out) {
  if (!cfg || !arena_dev || !out) return fail(BFP_EINVAL, "NULL argument");
  if ((uintptr_t)arena_dev % 256) return fail(BFP_EINVAL, "arena must be 256-byte aligned");
  if (cfg->max_slots < 1 || cfg->max_slots > 64) return fail(BFP_EINVAL, "max_slots must be in 1..64");
  if (cfg->max_queue < 1) return fail(BFP_EINVAL, "max_queue must be >= 1");
  mg_server* s = new (std::nothrow) mg_server();
  if (!s) return fail(BFP_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->exec_points = cfg->exec_max_points > 0 ? cfg->exec_max_points : kServerExecPoints;
  s->arena = static_cast<char*>(arena_dev);
  s->bytes = bytes & ~(size_t)255;
  s->free_ranges.emplace_back(0, s->bytes);
  s->slots.resize(cfg->max_slots);
  for (Slot& sl : s->slots) {
    int rc = hip_check(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking), "slot stream");
    if (!rc) rc = hip_check(hipEventCreate(&sl.start), "slot event");
    if (!rc) rc = hip_check(hipEventCreate(&sl.done), "slot event");
    if (!rc) rc = hip_check(hipHostMalloc((void**)&sl.staging, kTableBytes, hipHostMallocDefault),
                            "slot staging");
    if (rc) { delete s; return rc; }
  }
  *out = s;
  return BFP_OK;
}

int mg_server_submit(mg_server* s, const mg_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(BFP_EINVAL, "NULL argument");
  int rc = params_ok(&req->prm);
  if (rc) return rc;
  if (!req->x_out_dev) return fail(BFP_EINVAL, "x_out_dev is NULL");
  for (int j = 1; j <= req->prm.L; ++j)
    if (!req->rhs_dev[j - 1]) return fail(BFP_EINVAL, "rhs_dev[%d] is NULL", j - 1);
  if ((int64_t)s->queue.size() >= s->cfg.max_queue) return fail(BFP_EBUSY, "request queue is full");
  Queued q;
  q.ticket = s->next_ticket++;
  q.req = *req;
  s->queue.push_back(q);
  *ticket = q.ticket;
  return s->progress();
}

int mg_server_poll(mg_server* s, uint64_t ticket, mg_result* out) {
  if (!s || !out) return fail(BFP_EINVAL, "NULL argument");
  int rc = s->progress();
  if (rc) return rc;
  auto it = s->finished.find(ticket);
  if (it != s->finished.end()) {
    *out = it->second;
    s->finished.erase(it);
    return out->status == BFP_OK ? BFP_OK : out->status;
  }
  if (s->running.count(ticket)) return BFP_PENDING;
  for (const Queued& q : s->queue)
    if (q.ticket == ticket) return BFP_PENDING;
  return fail(BFP_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
}

int mg_server_collect(mg_server* s, uint64_t* tickets, mg_result* results, int cap, int* count) {
  if (!s || !count || (cap > 0 && (!tickets || !results))) return fail(BFP_EINVAL, "NULL argument");
  int rc = s->progress();
  if (rc) return rc;
  int k = 0;
  for (auto it = s->finished.begin(); it != s->finished.end() && k < cap;) {
    tickets[k] = it->first;
    results[k] = it->second;
    ++k;
    it = s->finished.erase(it);
  }
  *count = k;
  return BFP_OK;
}

int mg_server_stats(const mg_server* s, int* queued, int* running, size_t* resident_bytes) {
  if (!s) return fail(BFP_EINVAL, "NULL server");
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = (int)s->running.size();
  if (resident_bytes) {
    size_t b = 0;
    for (const Resident& r : s->pool) b += r.size;
    *resident_bytes = b;
  }
  return BFP_OK;
}

int mg_server_destroy(mg_server* s) {
  delete s;
  return BFP_OK;
}

}  // extern "C"
