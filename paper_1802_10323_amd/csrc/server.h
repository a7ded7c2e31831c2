// server.h - continuous-batching solve server (host runtime, C++).
//
// Requests (grid, boundary pairs, precision, a DEVICE field solved in place)
// are queued in arrival order.  A worker thread admits the request at the
// head of the queue as soon as an execution slot (a HIP stream) is free and
// the HBM its solve holds (field, plus the refinement workspace of an
// FP32 + refinement solve) fits the budget next to the requests in flight;
// the admitted solve is enqueued on that slot's stream at once, so requests
// that arrive while others run overlap with them on the device.  Completion
// is observed through one event per slot.  Plans (device tables and
// twiddles) are kept in a cache keyed by the problem and reused: an FP64
// plan only reads its tables and is shared by concurrent requests; a
// refined plan serves one request at a time (the cache holds as many copies
// as are in use at once) and runs on the refinement workspace of the slot
// it was admitted to, so a cached plan holds only its small tables.
//
// Included by poisson.hip (uses its error reporting and plan internals).
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
  size_t footprint = 0;
  int state = 0;            // 0 queued, 1 running, 2 done
  int status = POISSON_OK;
  int iters = 0;
  double rel = 0.0;
  int plan_hit = 0;
  std::string msg;
  poisson_plan* plan = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct CachedPlan {
  poisson_plan* plan = nullptr;
  int users = 0;
  double last_used = 0;
};

std::string plan_key(const ServerRequest& r) {
  std::string k;
  auto put = [&](const void* p, size_t n) { k.append(reinterpret_cast<const char*>(p), n); };
  put(r.dims, sizeof(r.dims));
  put(&r.dx, sizeof(double));
  put(&r.dy, sizeof(double));
  put(r.bc, sizeof(r.bc));
  put(&r.precision, sizeof(int));
  put(r.dz.data(), r.dz.size() * sizeof(double));
  return k;
}

}  // namespace

struct poisson_server {
  int device = 0;
  size_t budget = 0;
  size_t inflight = 0;
  int max_plans = 64;
  int nplans = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<long long> slot_req;
  // refinement workspace of each slot (FP64 f and FP32 residual), grown to
  // the largest refined request it has run; replaced buffers are released
  // only at destruction, so serving never frees device memory (a free waits
  // for the whole device)
  std::vector<double*> ws_f64;
  std::vector<float*> ws_e32;
  std::vector<size_t> ws_points;
  std::vector<void*> retired;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<long long> queue;
  std::unordered_map<long long, ServerRequest> reqs;
  std::map<std::string, std::vector<CachedPlan>> cache;
  long long next_id = 0;
  int running = 0;
  bool stop = false;
  long long hits = 0, misses = 0;
  std::thread worker;
};

// A plan for request r from the cache (or a new one); nullptr on failure.
static poisson_plan* server_acquire(poisson_server* S, ServerRequest& r) {
  const std::string key = plan_key(r);
  std::vector<CachedPlan>& v = S->cache[key];
  for (CachedPlan& c : v) {
    if (r.precision == POISSON_FP64 || c.users == 0) {
      ++c.users;
      c.last_used = now_s();
      r.plan_hit = 1;
      ++S->hits;
      return c.plan;
    }
  }
  // evict idle plans beyond the cache size (least recently used first)
  while (S->nplans >= S->max_plans) {
    std::map<std::string, std::vector<CachedPlan>>::iterator best_it = S->cache.end();
    size_t best_i = 0;
    double best_t = 1e300;
    for (auto it = S->cache.begin(); it != S->cache.end(); ++it)
      for (size_t i = 0; i < it->second.size(); ++i)
        if (it->second[i].users == 0 && it->second[i].last_used < best_t) {
          best_t = it->second[i].last_used;
          best_it = it;
          best_i = i;
        }
    if (best_it == S->cache.end()) break;   // all in use: grow past the limit
    plan_destroy(best_it->second[best_i].plan);
    best_it->second.erase(best_it->second.begin() + (long)best_i);
    --S->nplans;
  }
  ++S->misses;
  poisson_plan* p = plan_create(r.dims[0], r.dims[1], r.dims[2], r.dx, r.dy, r.dz.data(), r.bc[0],
                                r.bc[1], r.bc[2]);
  if (!p) return nullptr;
  std::vector<CachedPlan>& w = S->cache[key];   // (eviction may have rehashed nothing: std::map)
  w.push_back(CachedPlan{p, 1, now_s()});
  ++S->nplans;
  return p;
}

static void server_release(poisson_server* S, ServerRequest& r) {
  auto it = S->cache.find(plan_key(r));
  if (it == S->cache.end()) return;
  for (CachedPlan& c : it->second)
    if (c.plan == r.plan && c.users > 0) {
      --c.users;
      c.last_used = now_s();
      return;
    }
}

static void server_finish(poisson_server* S, ServerRequest& r, int status, const char* msg) {
  r.state = 2;
  r.status = status;
  if (msg) r.msg = msg;
  r.t_done = now_s();
  S->cv_done.notify_all();
}

static void server_loop(poisson_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progress = false;
    // completions
    for (size_t s = 0; s < S->streams.size(); ++s) {
      const long long id = S->slot_req[s];
      if (id < 0) continue;
      const hipError_t q = hipEventQuery(S->events[s]);
      if (q == hipErrorNotReady) continue;
      ServerRequest& r = S->reqs[id];
      int status = q == hipSuccess ? POISSON_OK : POISSON_EHIP;
      if (status == POISSON_OK && r.precision == POISSON_FP32_REFINED) {
        status = solve_status(r.plan, &r.iters, &r.rel);
      } else {
        r.iters = 1;
      }
      server_release(S, r);
      S->inflight -= r.footprint;
      S->slot_req[s] = -1;
      --S->running;
      server_finish(S, r, status, q == hipSuccess ? nullptr : hipGetErrorString(q));
      progress = true;
    }
    // admissions, in arrival order
    while (!S->queue.empty()) {
      int slot = -1;
      for (size_t s = 0; s < S->streams.size(); ++s)
        if (S->slot_req[s] < 0) { slot = (int)s; break; }
      if (slot < 0) break;
      ServerRequest& r = S->reqs[S->queue.front()];
      if (S->inflight > 0 && S->inflight + r.footprint > S->budget) break;
      S->queue.pop_front();
      progress = true;
      r.plan = server_acquire(S, r);
      if (!r.plan) {
        server_finish(S, r, g_err ? g_err : POISSON_EHIP, g_msg);
        continue;
      }
      if (r.precision == POISSON_FP32_REFINED) {
        const size_t N = (size_t)r.dims[0] * r.dims[1] * r.dims[2];
        int rc = POISSON_OK;
        if (S->ws_points[slot] < N) {
          double* f = nullptr;
          float* e = nullptr;
          if (hipMalloc(&f, N * sizeof(double)) != hipSuccess ||
              hipMalloc(&e, N * sizeof(float)) != hipSuccess) {
            if (f) S->retired.push_back(f);
            rc = fail(POISSON_ENOMEM, "refinement workspace of %zu points", N);
          } else {
            if (S->ws_f64[slot]) S->retired.push_back(S->ws_f64[slot]);
            if (S->ws_e32[slot]) S->retired.push_back(S->ws_e32[slot]);
            S->ws_f64[slot] = f;
            S->ws_e32[slot] = e;
            S->ws_points[slot] = N;
          }
        }
        if (!rc) rc = plan_refine_on(r.plan, r.tol, r.max_iters, S->ws_f64[slot], S->ws_e32[slot]);
        if (rc) { server_release(S, r); server_finish(S, r, rc, g_msg); continue; }
      }
      r.t_start = now_s();
      int rc = solve(r.plan, r.field, S->streams[slot]);
      if (!rc && hipEventRecord(S->events[slot], S->streams[slot]) != hipSuccess)
        rc = fail(POISSON_EHIP, "hipEventRecord failed");
      if (rc) { server_release(S, r); server_finish(S, r, rc, g_msg); continue; }
      r.state = 1;
      S->slot_req[slot] = r.id;
      S->inflight += r.footprint;
      ++S->running;
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
  for (int s = 0; s < slots; ++s) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      fail(POISSON_EHIP, "stream/event creation failed");
      for (auto x : S->streams) (void)hipStreamDestroy(x);
      for (auto x : S->events) (void)hipEventDestroy(x);
      delete S;
      return nullptr;
    }
    S->streams.push_back(st);
    S->events.push_back(ev);
    S->slot_req.push_back(-1);
    S->ws_f64.push_back(nullptr);
    S->ws_e32.push_back(nullptr);
    S->ws_points.push_back(0);
  }
  S->worker = std::thread(server_loop, S);
  return S;
}

extern "C" long long server_submit(poisson_server* S, int nx, int ny, int nz, double dx, double dy,
                                   const double* dz, int bc_x, int bc_y, int bc_z, int precision,
                                   double tol, int max_iters, double* field) {
  if (!S || !dz || !field) return fail(POISSON_EINVAL, "null argument");
  if (nx < 1 || ny < 1 || nz < 1) return fail(POISSON_EINVAL, "sizes must be >= 1");
  if (precision != POISSON_FP64 && precision != POISSON_FP32_REFINED)
    return fail(POISSON_EINVAL, "unknown precision mode %d", precision);
  ServerRequest r;
  r.dims[0] = nx; r.dims[1] = ny; r.dims[2] = nz;
  r.dx = dx; r.dy = dy;
  r.dz.assign(dz, dz + nz);
  r.bc[0] = bc_x; r.bc[1] = bc_y; r.bc[2] = bc_z;
  r.precision = precision;
  r.tol = tol;
  r.max_iters = max_iters;
  r.field = field;
  const size_t N = (size_t)nx * ny * nz;
  r.footprint = N * sizeof(double) +
                (precision == POISSON_FP32_REFINED ? N * (sizeof(double) + sizeof(float)) : 0);
  r.t_submit = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(POISSON_EINVAL, "server is shutting down");
  if (r.footprint > S->budget)
    return fail(POISSON_EUNSUPPORTED, "request needs %zu B of HBM, over the budget of %zu B",
                r.footprint, S->budget);
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
  S->cv_done.wait(lk, [&] { return S->reqs[id].state == 2; });
  ServerRequest& r = S->reqs[id];
  if (info) {
    info->status = r.status;
    info->iters = r.iters;
    info->plan_cached = r.plan_hit;
    info->last_update_rel = r.rel;
    info->submit_s = r.t_submit;
    info->start_s = r.t_start;
    info->done_s = r.t_done;
    info->points = (long long)r.dims[0] * r.dims[1] * r.dims[2];
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

extern "C" void server_destroy(poisson_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->cache)
    for (CachedPlan& c : kv.second) plan_destroy(c.plan);
  for (double* f : S->ws_f64) if (f) (void)hipFree(f);
  for (float* e : S->ws_e32) if (e) (void)hipFree(e);
  for (void* x : S->retired) (void)hipFree(x);
  for (auto x : S->streams) (void)hipStreamDestroy(x);
  for (auto x : S->events) (void)hipEventDestroy(x);
  delete S;
}
