// server.h - continuous-batching solve server (host runtime, C++).
//
// Requests (grid, boundary pairs, precision, a DEVICE field solved in place)
// are queued in arrival order.  A worker thread admits the request at the
// head of the queue as soon as an execution slot (a HIP stream) is free and
// its HBM fits the budget next to what is already held, and enqueues its
// solve on that slot's stream at once, so requests that arrive while others
// run overlap with them on the device.  Completion is observed through one
// event per slot.
//
// Ordering with the caller: server_submit records an event on the caller's
// (producer) stream; the slot's stream waits for it before the solve, so the
// solve sees every write the caller enqueued on that stream before the call.
//
// Plans are immutable tables (twiddles, eigenvalue shifts, operator rows),
// cached by problem geometry and shared by every request of that geometry,
// FP64 or refined: a refined solve runs on the refinement workspace of the
// slot it was admitted to (FP64 copy of f, FP32 correction, status block),
// grown to the largest refined request the slot has run.
//
// HBM budget: the fields of the running requests plus everything the server
// itself holds on the device (slot workspaces, cached plans' tables, buffers
// and plans waiting to be freed) stay within the budget whenever more than
// one request runs; a request that fits the budget alone is always admitted
// once the device is idle.  A device free waits for the whole device, so the
// server frees memory (grown-out workspaces, evicted plans) only when no
// request is in flight.
//
// The mutex guards the queue, the request table and the counters; plan
// creation, workspace allocation and the enqueueing of a solve run outside
// it, so submissions and waits never stall behind them.
//
// Included by poisson.hip (uses its error reporting, plan internals and the
// refined-solve driver).
#pragma once
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct ServerRequest {
  long long id = 0;
  int dims[3] = {0, 0, 0};
  double dx = 0, dy = 0;
  std::vector<double> dz;
  int bc[3] = {0, 0, 0};
  int precision = POISSON_FP64;
  double tol = 1e-10;
  int max_iters = 4;
  double* field = nullptr;
  hipEvent_t ready = nullptr;   // recorded on the producer stream at submission
  size_t points = 0;
  size_t field_bytes = 0;       // 8 B per point, held while running
  int state = 0;                // 0 queued, 1 admitted, 2 done
  int status = POISSON_OK;
  int iters = 0;
  double rel = 0.0;
  int plan_hit = 0;
  std::string msg;
  std::string key;
  poisson_plan* plan = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct CachedPlan {
  poisson_plan* plan = nullptr;
  int users = 0;
  double last_used = 0;
};

// Plans hold only geometry-dependent tables: precision is not in the key.
std::string plan_key(const ServerRequest& r) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
  put(r.dims, sizeof(r.dims));
  put(&r.dx, sizeof(double));
  put(&r.dy, sizeof(double));
  put(r.bc, sizeof(r.bc));
  put(r.dz.data(), r.dz.size() * sizeof(double));
  return k;
}

struct ServerSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  long long req = -1;
  int state = 0;                // 0 free, 1 being prepared, 2 running
  // refinement workspace
  double* f64 = nullptr;
  float* e32 = nullptr;
  double* stats = nullptr;
  double* stats_host = nullptr;
  size_t points = 0;            // capacity of f64 / e32
};

size_t slot_work_bytes(size_t points) {
  return points * (sizeof(double) + sizeof(float)) + REFINE_STAT_SLOTS * sizeof(double);
}

}  // namespace

struct poisson_server {
  int device = 0;
  size_t budget = 0;
  size_t inflight = 0;          // fields of the admitted requests
  size_t held = 0;              // device memory of the server: workspaces, plan tables, retired
  size_t peak = 0;              // largest inflight + held after an admission
  int max_plans = 64;
  std::vector<ServerSlot> slots;
  std::vector<std::pair<void*, size_t>> retired;       // device buffers to free when idle
  std::vector<poisson_plan*> retired_plans;            // evicted plans to destroy when idle
  std::vector<hipEvent_t> event_pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<long long> queue;
  std::unordered_map<long long, ServerRequest> reqs;
  std::map<std::string, CachedPlan> cache;             // worker thread only
  long long next_id = 0;
  int running = 0;                                     // admitted and not yet done
  bool stop = false;
  long long hits = 0, misses = 0;
  int nplans = 0;                                      // cached plans + evicted ones not yet freed
  std::thread worker;
};

// The cached plan for request r, or a new one (worker thread, no lock held).
// *table_bytes receives the tables of a newly created plan (0 on a hit).
static poisson_plan* server_acquire(poisson_server* S, ServerRequest& r, size_t* table_bytes,
                                    std::vector<poisson_plan*>& evicted) {
  *table_bytes = 0;
  auto it = S->cache.find(r.key);
  if (it != S->cache.end()) {
    ++it->second.users;
    it->second.last_used = now_s();
    r.plan_hit = 1;
    return it->second.plan;
  }
  // evict idle plans beyond the cache size, least recently used first
  while ((int)S->cache.size() >= S->max_plans) {
    auto best = S->cache.end();
    for (auto c = S->cache.begin(); c != S->cache.end(); ++c)
      if (c->second.users == 0 && (best == S->cache.end() || c->second.last_used < best->second.last_used))
        best = c;
    if (best == S->cache.end()) break;   // all in use: grow past the limit
    evicted.push_back(best->second.plan);
    S->cache.erase(best);
  }
  poisson_plan* p = plan_create(r.dims[0], r.dims[1], r.dims[2], r.dx, r.dy, r.dz.data(), r.bc[0],
                                r.bc[1], r.bc[2]);
  if (!p) return nullptr;
  S->cache[r.key] = CachedPlan{p, 1, now_s()};
  *table_bytes = p->tab_bytes;
  return p;
}

static void server_release(poisson_server* S, const ServerRequest& r) {
  auto it = S->cache.find(r.key);
  if (it != S->cache.end() && it->second.plan == r.plan && it->second.users > 0) {
    --it->second.users;
    it->second.last_used = now_s();
  }
}

static void server_finish(poisson_server* S, ServerRequest& r, int status, const char* msg) {
  r.state = 2;
  r.status = status;
  if (msg) r.msg = msg;
  r.t_done = now_s();
  if (r.ready) {
    S->event_pool.push_back(r.ready);
    r.ready = nullptr;
  }
  S->cv_done.notify_all();
}

// Grow slot s's refinement workspace to `points` (worker thread, no lock
// held).  The replaced buffers go to `retired`.
static int slot_grow(ServerSlot& s, size_t points, std::vector<std::pair<void*, size_t>>& retired) {
  if (!s.stats_host &&
      hipHostMalloc(&s.stats_host, REFINE_STAT_SLOTS * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    s.stats_host = nullptr;
    return fail(POISSON_ENOMEM, "refinement status block (host)");
  }
  if (!s.stats && hipMalloc(&s.stats, REFINE_STAT_SLOTS * sizeof(double)) != hipSuccess) {
    s.stats = nullptr;
    return fail(POISSON_ENOMEM, "refinement status block");
  }
  if (s.points >= points) return POISSON_OK;
  double* f = nullptr;
  float* e = nullptr;
  if (hipMalloc(&f, points * sizeof(double)) != hipSuccess) return fail(POISSON_ENOMEM, "refinement workspace of %zu points", points);
  if (hipMalloc(&e, points * sizeof(float)) != hipSuccess) {
    retired.push_back({f, points * sizeof(double)});
    return fail(POISSON_ENOMEM, "refinement workspace of %zu points", points);
  }
  if (s.f64) retired.push_back({s.f64, s.points * sizeof(double)});
  if (s.e32) retired.push_back({s.e32, s.points * sizeof(float)});
  s.f64 = f;
  s.e32 = e;
  s.points = points;
  return POISSON_OK;
}

// Enqueue request r on slot s (worker thread, no lock held).
static int server_launch(poisson_server* S, ServerSlot& slot, ServerRequest& r) {
  if (r.ready) HIP_TRY(hipStreamWaitEvent(slot.stream, r.ready, 0));
  int rc;
  if (r.precision == POISSON_FP32_REFINED) {
    const RefineWork W{slot.f64, slot.e32, slot.stats, r.tol, r.max_iters};
    if ((rc = run_refined(r.plan, W, r.field, slot.stream))) return rc;
    HIP_TRY(hipMemcpyAsync(slot.stats_host, slot.stats, REFINE_PARTIALS * sizeof(double),
                           hipMemcpyDeviceToHost, slot.stream));
  } else if ((rc = solve_typed<double>(r.plan, r.field, slot.stream))) {
    return rc;
  }
  HIP_TRY(hipEventRecord(slot.done, slot.stream));
  return POISSON_OK;
}

static void server_loop(poisson_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progress = false;
    // completions
    for (ServerSlot& slot : S->slots) {
      if (slot.state != 2) continue;
      const hipError_t q = hipEventQuery(slot.done);
      if (q == hipErrorNotReady) continue;
      ServerRequest& r = S->reqs.at(slot.req);
      int status = q == hipSuccess ? POISSON_OK : POISSON_EHIP;
      r.iters = 1;
      if (status == POISSON_OK && r.precision == POISSON_FP32_REFINED) {
        const bool conv = refine_status_decode(slot.stats_host, r.max_iters, &r.iters, &r.rel);
        if (!conv) status = POISSON_ENOTCONVERGED;
      }
      server_release(S, r);
      S->inflight -= r.field_bytes;
      slot.req = -1;
      slot.state = 0;
      --S->running;
      server_finish(S, r, status, q == hipSuccess ? nullptr : hipGetErrorString(q));
      progress = true;
    }
    // memory waiting to be freed, once nothing is in flight (a free waits
    // for the device)
    if (S->running == 0 && (!S->retired.empty() || !S->retired_plans.empty())) {
      std::vector<std::pair<void*, size_t>> bufs;
      std::vector<poisson_plan*> plans;
      bufs.swap(S->retired);
      plans.swap(S->retired_plans);
      lk.unlock();
      size_t freed = 0;
      for (auto& b : bufs) {
        (void)hipFree(b.first);
        freed += b.second;
      }
      for (poisson_plan* p : plans) {
        freed += p->tab_bytes;
        plan_destroy(p);
      }
      lk.lock();
      S->held -= freed;
      S->nplans = (int)S->cache.size();
      progress = true;
    }
    // admission of the request at the head of the queue
    if (!S->queue.empty()) {
      ServerSlot* slot = nullptr;
      for (ServerSlot& s : S->slots)
        if (s.state == 0) { slot = &s; break; }
      ServerRequest& r = S->reqs.at(S->queue.front());
      // a grown workspace is new memory: the replaced one is freed only
      // once the device is idle
      size_t growth = 0;
      if (slot && r.precision == POISSON_FP32_REFINED && r.points > slot->points)
        growth = r.points * (sizeof(double) + sizeof(float)) +
                 (slot->stats ? 0 : REFINE_STAT_SLOTS * sizeof(double));
      const bool fits = slot && S->inflight + S->held + r.field_bytes + growth <= S->budget;
      if (slot && (fits || S->running == 0)) {
        S->queue.pop_front();
        progress = true;
        slot->state = 1;
        slot->req = r.id;
        r.state = 1;
        S->inflight += r.field_bytes;
        ++S->running;
        // admitted over budget on an idle device: release the other slots'
        // workspaces first
        if (!fits)
          for (ServerSlot& s : S->slots)
            if (&s != slot && s.state == 0 && s.f64) {
              S->retired.push_back({s.f64, s.points * sizeof(double)});
              S->retired.push_back({s.e32, s.points * sizeof(float)});
              s.f64 = nullptr;
              s.e32 = nullptr;
              s.points = 0;
            }
        lk.unlock();
        // nothing else runs when an over-budget request is admitted: free now
        std::vector<std::pair<void*, size_t>> retired_now;
        size_t freed = 0;
        if (!fits) {
          std::lock_guard<std::mutex> g(S->mu);
          retired_now.swap(S->retired);
        }
        for (auto& b : retired_now) {
          (void)hipFree(b.first);
          freed += b.second;
        }
        size_t tables = 0;
        std::vector<poisson_plan*> evicted;
        std::vector<std::pair<void*, size_t>> grown_out;
        int rc = POISSON_OK;
        r.plan = server_acquire(S, r, &tables, evicted);
        if (!r.plan) rc = g_err ? g_err : POISSON_EHIP;
        const size_t before = slot->stats ? slot_work_bytes(slot->points) : 0;
        if (!rc && r.precision == POISSON_FP32_REFINED) rc = slot_grow(*slot, r.points, grown_out);
        const size_t after = slot->stats ? slot_work_bytes(slot->points) : 0;
        const double t_start = now_s();
        if (!rc) rc = server_launch(S, *slot, r);
        const std::string msg = rc ? std::string(g_msg) : std::string();
        lk.lock();
        S->held = S->held - freed + tables + (after - before);
        for (auto& b : grown_out) S->retired.push_back(b);   // still counted in held
        size_t grown_bytes = 0;
        for (auto& b : grown_out) grown_bytes += b.second;
        S->held += grown_bytes;
        for (poisson_plan* p : evicted) S->retired_plans.push_back(p);   // tables still counted
        S->nplans = (int)(S->cache.size() + S->retired_plans.size());
        if (r.plan_hit) ++S->hits;
        else if (r.plan) ++S->misses;
        r.t_start = t_start;
        if (rc) {
          if (r.plan) server_release(S, r);
          S->inflight -= r.field_bytes;
          slot->req = -1;
          slot->state = 0;
          --S->running;
          server_finish(S, r, rc, msg.c_str());
        } else {
          slot->state = 2;
          S->peak = std::max(S->peak, S->inflight + S->held);
        }
        continue;
      }
    }
    if (S->stop && S->queue.empty() && S->running == 0) break;
    if (!progress) {
      if (S->running > 0) {
        // poll the slots' events again shortly
        S->cv_work.wait_for(lk, std::chrono::microseconds(20));
      } else if (!S->stop) {
        S->cv_work.wait(lk);
      }
    }
  }
}

extern "C" poisson_server* server_create(int slots, size_t hbm_budget, int max_plans) {
  if (slots < 1 || slots > 64) { fail(POISSON_EINVAL, "slots must be in [1, 64]"); return nullptr; }
  if (max_plans < 1) { fail(POISSON_EINVAL, "max_plans must be >= 1"); return nullptr; }
  poisson_server* S = new poisson_server();
  if (hipGetDevice(&S->device) != hipSuccess) { fail(POISSON_EHIP, "hipGetDevice failed"); delete S; return nullptr; }
  if (hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { fail(POISSON_EHIP, "hipMemGetInfo failed"); delete S; return nullptr; }
    hbm_budget = free_b / 10 * 8;
  }
  S->budget = hbm_budget;
  S->max_plans = max_plans;
  S->slots.resize(slots);
  for (ServerSlot& s : S->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      fail(POISSON_EHIP, "stream/event creation failed");
      for (ServerSlot& t : S->slots) {
        if (t.stream) (void)hipStreamDestroy(t.stream);
        if (t.done) (void)hipEventDestroy(t.done);
      }
      delete S;
      return nullptr;
    }
  }
  S->worker = std::thread(server_loop, S);
  return S;
}

extern "C" long long server_submit(poisson_server* S, int nx, int ny, int nz, double dx, double dy,
                                   const double* dz, int bc_x, int bc_y, int bc_z, int precision,
                                   double tol, int max_iters, double* field, hipStream_t producer) {
  if (!S || !dz || !field) return fail(POISSON_EINVAL, "null argument");
  if (int rc = misaligned(field, "field")) return rc;
  if (nx < 1 || ny < 1 || nz < 1) return fail(POISSON_EINVAL, "sizes must be >= 1");
  if (precision != POISSON_FP64 && precision != POISSON_FP32_REFINED)
    return fail(POISSON_EINVAL, "unknown precision mode %d", precision);
  if (precision == POISSON_FP32_REFINED) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(POISSON_EINVAL, "tol must be finite and > 0");
    if (max_iters < 1 || max_iters > REFINE_MAX_SWEEPS)
      return fail(POISSON_EINVAL, "max_iters must be in [1, %d]", REFINE_MAX_SWEEPS);
  }
  ServerRequest r;
  r.dims[0] = nx; r.dims[1] = ny; r.dims[2] = nz;
  r.dx = dx; r.dy = dy;
  r.dz.assign(dz, dz + nz);
  r.bc[0] = bc_x; r.bc[1] = bc_y; r.bc[2] = bc_z;
  r.precision = precision;
  r.tol = tol;
  r.max_iters = max_iters;
  r.field = field;
  r.key = plan_key(r);
  r.points = (size_t)nx * ny * nz;
  r.field_bytes = r.points * sizeof(double);
  const size_t alone = r.field_bytes + (precision == POISSON_FP32_REFINED ? slot_work_bytes(r.points) : 0);
  if (alone > S->budget)
    return fail(POISSON_EUNSUPPORTED, "request needs %zu B of HBM, over the budget of %zu B", alone,
                S->budget);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(POISSON_EINVAL, "server is shutting down");
    if (!S->event_pool.empty()) {
      r.ready = S->event_pool.back();
      S->event_pool.pop_back();
    }
  }
  if (!r.ready && hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
    return fail(POISSON_EHIP, "event creation failed");
  if (hipEventRecord(r.ready, producer) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->event_pool.push_back(r.ready);
    return fail(POISSON_EHIP, "hipEventRecord on the producer stream failed");
  }
  r.t_submit = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  r.id = S->next_id++;
  const long long id = r.id;
  S->reqs.emplace(id, std::move(r));
  S->queue.push_back(id);
  S->cv_work.notify_one();
  return id;
}

extern "C" int server_wait(poisson_server* S, long long id, poisson_request_info* info) {
  if (!S) return fail(POISSON_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return fail(POISSON_EINVAL, "unknown request %lld", id);
  ServerRequest& r = it->second;   // element references survive rehashing, iterators do not
  S->cv_done.wait(lk, [&] { return r.state == 2; });
  if (info) {
    info->status = r.status;
    info->iters = r.iters;
    info->plan_cached = r.plan_hit;
    info->last_update_rel = r.rel;
    info->submit_s = r.t_submit;
    info->start_s = r.t_start;
    info->done_s = r.t_done;
    info->points = (long long)r.points;
  }
  const int status = r.status;
  if (status && status != POISSON_ENOTCONVERGED)
    fail(status, "request %lld: %s", id, r.msg.c_str());
  S->reqs.erase(id);
  return status;
}

extern "C" int server_stats(poisson_server* S, long long* plan_hits, long long* plan_misses,
                            int* plans_resident, size_t* budget) {
  if (!S) return fail(POISSON_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (plan_hits) *plan_hits = S->hits;
  if (plan_misses) *plan_misses = S->misses;
  if (plans_resident) *plans_resident = S->nplans;
  if (budget) *budget = S->budget;
  return POISSON_OK;
}

extern "C" int server_usage(poisson_server* S, size_t* held_bytes, size_t* peak_bytes) {
  if (!S) return fail(POISSON_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (held_bytes) *held_bytes = S->held;
  if (peak_bytes) *peak_bytes = S->peak;
  return POISSON_OK;
}

extern "C" void server_destroy(poisson_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->cache) plan_destroy(kv.second.plan);
  for (poisson_plan* p : S->retired_plans) plan_destroy(p);
  for (auto& b : S->retired) (void)hipFree(b.first);
  for (ServerSlot& s : S->slots) {
    if (s.f64) (void)hipFree(s.f64);
    if (s.e32) (void)hipFree(s.e32);
    if (s.stats) (void)hipFree(s.stats);
    if (s.stats_host) (void)hipHostFree(s.stats_host);
    (void)hipStreamDestroy(s.stream);
    (void)hipEventDestroy(s.done);
  }
  for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
  for (auto& kv : S->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  delete S;
}
