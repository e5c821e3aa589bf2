// Serving runtime of the HPM library: independent solves in flight on one device at once.
//
// One first-in-first-out queue of requests; "slots" host worker threads, each with its own HIP
// stream; plans kept resident between requests and reused by problem. The request at the head
// of the queue is admitted by whichever worker is free once its estimated memory fits the
// budget. Workers run the same create/rebuild/execute steps as the plan API, so a request's
// result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hpm_internal.h"

namespace hpm {
namespace {

constexpr int kMaxSlots = 16;

struct Request {
  uint64_t ticket = 0;
  hpm_problem prob{};
  int64_t n = 0;
  const void *x = nullptr, *y = nullptr, *z = nullptr, *m = nullptr;
  void *phi = nullptr, *ax = nullptr, *ay = nullptr, *az = nullptr;
  size_t estimate = 0;
  bool done = false;
  hpm_status status = HPM_OK;
  std::string msg;
  int slot = -1;
  double submit_ms = 0, start_ms = 0, done_ms = 0;
  size_t plan_bytes = 0;
};

// A resident plan. "key" is the problem it was made for; "bytes" its measured device memory
// (0 until it has served a request).
struct Pooled {
  std::unique_ptr<hpm_plan_s> plan;
  hpm_problem key{};
  size_t bytes = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

bool same_problem(const hpm_problem& a, const hpm_problem& b) {
  return std::memcmp(&a, &b, sizeof(hpm_problem)) == 0;
}

}  // namespace
}  // namespace hpm

using namespace hpm;

struct hpm_server_s {
  int device = 0;
  int slots = 1;
  size_t budget = 0;  // 0: no limit
  std::chrono::steady_clock::time_point t0;
  std::vector<hipStream_t> streams;

  std::mutex mu;
  std::condition_variable cv_work;  // workers: a request arrived, memory or a plan was freed, stop
  std::condition_variable cv_done;  // callers of wait: a request finished
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  std::list<Pooled> pool;
  size_t held = 0;  // sum of pooled plans' bytes plus the reservations of running requests
  size_t peak_held = 0;
  int running = 0;
  uint64_t next_ticket = 1, clock = 0;
  int64_t submitted = 0, completed = 0, failed = 0, created = 0, released = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }

  void worker(int slot);
  // Under the lock: admits the head of the queue if it fits. On success returns the request with
  // its pool entry (created busy if none was idle) and the bytes reserved for it; plans released
  // to make room are moved to "evicted" (their device memory is freed by the caller, unlocked).
  bool admit(std::shared_ptr<Request>& r, std::list<Pooled>::iterator& entry, size_t& reserved,
             std::vector<std::unique_ptr<hpm_plan_s>>& evicted);
  void finish(const std::shared_ptr<Request>& r, hpm_status st, const std::string& msg);
};

bool hpm_server_s::admit(std::shared_ptr<Request>& r, std::list<Pooled>::iterator& entry,
                         size_t& reserved, std::vector<std::unique_ptr<hpm_plan_s>>& evicted) {
  const std::shared_ptr<Request> head = queue.front();
  // the idle plan of the same problem that needs the least growth
  auto cand = pool.end();
  size_t idle_other = 0;
  for (auto it = pool.begin(); it != pool.end(); ++it) {
    if (it->busy) continue;
    if (same_problem(it->key, head->prob) && (cand == pool.end() || it->bytes > cand->bytes))
      cand = it;
    idle_other += it->bytes;
  }
  if (cand != pool.end()) idle_other -= cand->bytes;
  const size_t have = cand == pool.end() ? 0 : cand->bytes;
  const size_t growth = head->estimate > have ? head->estimate - have : 0;
  if (budget && held + growth > budget) {
    if (held - idle_other + growth > budget) {  // releasing every idle plan would not be enough
      if (running > 0) return false;            // wait for a running request to finish
      r = head;                                 // it can never fit: fail it
      queue.pop_front();
      r->status = HPM_ERR_NO_MEMORY;
      r->msg = "request needs an estimated " + std::to_string(head->estimate) +
               " bytes of device memory; the server's budget is " + std::to_string(budget);
      return true;  // entry stays pool.end()
    }
    while (held + growth > budget) {  // release idle plans, least recently used first
      auto lru = pool.end();
      for (auto it = pool.begin(); it != pool.end(); ++it)
        if (!it->busy && it != cand && (lru == pool.end() || it->last_use < lru->last_use)) lru = it;
      held -= lru->bytes;
      evicted.push_back(std::move(lru->plan));
      pool.erase(lru);
      released += 1;
    }
  }
  if (cand == pool.end()) {
    pool.emplace_back();
    cand = std::prev(pool.end());
    cand->key = head->prob;
  }
  cand->busy = true;
  entry = cand;
  reserved = growth;
  held += growth;
  peak_held = std::max(peak_held, held);
  r = head;
  queue.pop_front();
  return true;
}

void hpm_server_s::finish(const std::shared_ptr<Request>& r, hpm_status st, const std::string& msg) {
  r->status = st;
  r->msg = msg;
  r->done = true;
  r->done_ms = now_ms();
  completed += 1;
  if (st != HPM_OK) failed += 1;
}

void hpm_server_s::worker(int slot) {
  (void)hipSetDevice(device);
  hipStream_t s = streams[size_t(slot)];
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    std::shared_ptr<Request> r;
    auto entry = pool.end();
    size_t reserved = 0;
    std::vector<std::unique_ptr<hpm_plan_s>> evicted;
    cv_work.wait(lk, [&] {
      if (queue.empty()) return stop;
      return admit(r, entry, reserved, evicted);
    });
    if (!r) return;  // stopped with an empty queue
    if (!queue.empty()) cv_work.notify_one();  // another idle worker may take the next request
    if (entry == pool.end()) {  // failed at admission
      finish(r, r->status, r->msg);
      lk.unlock();
      evicted.clear();
      lk.lock();
      cv_done.notify_all();
      cv_work.notify_all();
      continue;
    }
    running += 1;
    r->slot = slot;
    r->start_ms = now_ms();
    std::unique_ptr<hpm_plan_s> plan = std::move(entry->plan);
    // the plan may hold its own bytes, this request's reservation and the budget still free
    const size_t cap = budget ? entry->bytes + reserved + (budget > held ? budget - held : 0) : 0;
    lk.unlock();

    evicted.clear();  // frees the released plans' device memory before this request allocates
    const bool fresh = !plan;
    std::string msg;
    const hpm_status st = guarded([&] {
      if (fresh) {
        plan.reset(new hpm_plan_s());
        plan->p.byte_cap = cap;
        create_plan(plan->p, &r->prob, r->n, r->x, r->y, r->z, s);
      } else {
        plan->p.byte_cap = cap;
        rebuild_plan(plan->p, r->n, r->x, r->y, r->z, s);
      }
      execute_plan(plan->p, r->m, r->phi, r->ax, r->ay, r->az, s);
      HPM_HIP(hipStreamSynchronize(s));
    });
    if (st != HPM_OK) msg = hpm_last_error();
    // a plan whose creation failed is dropped, and so is any plan after a device error; a plan
    // whose rebuild was refused (positions out of the box) is rebuilt by its next request
    const bool keep = plan && !(fresh && st != HPM_OK) && st != HPM_ERR_DEVICE;
    const size_t bytes = plan ? plan->p.device_bytes() : 0;

    lk.lock();
    running -= 1;
    held -= reserved + entry->bytes;
    if (keep) {
      entry->plan = std::move(plan);
      entry->bytes = bytes;
      entry->busy = false;
      entry->last_use = ++clock;
      held += bytes;
      if (fresh) created += 1;
    } else {
      pool.erase(entry);
    }
    peak_held = std::max(peak_held, held);
    r->plan_bytes = bytes;
    finish(r, st, msg);
    cv_done.notify_all();
    cv_work.notify_all();
    if (plan) {  // not kept: free it without the lock
      lk.unlock();
      plan.reset();
      lk.lock();
    }
  }
}

namespace {

void fill_info(const Request& r, hpm_request_info* info) {
  if (!info) return;
  info->status = r.status;
  info->slot = r.slot;
  info->n = r.n;
  info->submit_ms = r.submit_ms;
  info->start_ms = r.start_ms;
  info->done_ms = r.done_ms;
  info->plan_bytes = int64_t(r.plan_bytes);
  info->estimate_bytes = int64_t(r.estimate);
}

// Reports a finished request and releases its ticket (the caller holds the lock).
hpm_status report(hpm_server_s* sv, std::unordered_map<uint64_t, std::shared_ptr<Request>>::iterator it,
                  hpm_request_info* info) {
  std::shared_ptr<Request> r = it->second;
  sv->tickets.erase(it);
  fill_info(*r, info);
  if (r->status != HPM_OK) set_last_error(r->msg);
  return r->status;
}

}  // namespace

extern "C" {

hpm_status hpm_server_create(const hpm_server_config* cfg, hpm_server** out) {
  if (out) *out = nullptr;
  hpm_server_s* sv = nullptr;
  hpm_status st = guarded([&] {
    if (!out || !cfg) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    if (cfg->abi != HPM_ABI_VERSION) fail(HPM_ERR_INVALID_ARG, "config.abi != HPM_ABI_VERSION");
    if (cfg->slots < 1 || cfg->slots > kMaxSlots) fail(HPM_ERR_INVALID_ARG, "slots must be 1..16");
    if (cfg->hbm_budget < 0) fail(HPM_ERR_INVALID_ARG, "hbm_budget must be >= 0");
    for (int k = 0; k < 4; ++k)
      if (cfg->reserved[k] != 0) fail(HPM_ERR_INVALID_ARG, "config.reserved must be 0");
    sv = new hpm_server_s();
    sv->slots = cfg->slots;
    sv->budget = size_t(cfg->hbm_budget);
    sv->t0 = std::chrono::steady_clock::now();
    HPM_HIP(hipGetDevice(&sv->device));
    for (int k = 0; k < sv->slots; ++k) {
      hipStream_t s = nullptr;
      HPM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      sv->streams.push_back(s);
    }
    for (int k = 0; k < sv->slots; ++k) sv->workers.emplace_back([sv, k] { sv->worker(k); });
  });
  if (st != HPM_OK) {
    if (sv) {
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
      }
      sv->cv_work.notify_all();
      for (auto& t : sv->workers) t.join();
      for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
      delete sv;
    }
    return st;
  }
  *out = sv;
  return HPM_OK;
}

hpm_status hpm_server_submit(hpm_server* server, const hpm_problem* problem, int64_t n,
                             const void* x, const void* y, const void* z, const void* m,
                             void* phi, void* ax, void* ay, void* az, uint64_t* ticket) {
  return guarded([&] {
    if (!server || !ticket) fail(HPM_ERR_INVALID_ARG, "NULL argument");
    check_problem(problem);
    check_size(problem, n);
    if (!x || !y || !z || !m || !phi || !ax || !ay || !az)
      fail(HPM_ERR_INVALID_ARG, "array pointer is NULL");
    auto r = std::make_shared<Request>();
    r->prob = *problem;
    r->n = n;
    r->x = x, r->y = y, r->z = z, r->m = m;
    r->phi = phi, r->ax = ax, r->ay = ay, r->az = az;
    r->estimate = plan_bytes_estimate(*problem, n);
    {
      std::lock_guard<std::mutex> lk(server->mu);
      if (server->stop) fail(HPM_ERR_INVALID_ARG, "server is shutting down");
      r->ticket = server->next_ticket++;
      r->submit_ms = server->now_ms();
      server->tickets.emplace(r->ticket, r);
      server->queue.push_back(r);
      server->submitted += 1;
      *ticket = r->ticket;
    }
    server->cv_work.notify_one();
  });
}

hpm_status hpm_server_poll(hpm_server* server, uint64_t ticket, hpm_request_info* info) {
  if (!server) {
    set_last_error("server is NULL");
    return HPM_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(server->mu);
  auto it = server->tickets.find(ticket);
  if (it == server->tickets.end()) {
    set_last_error("unknown or already reported ticket");
    return HPM_ERR_INVALID_ARG;
  }
  if (!it->second->done) return HPM_ERR_NOT_READY;
  return report(server, it, info);
}

hpm_status hpm_server_wait(hpm_server* server, uint64_t ticket, hpm_request_info* info) {
  if (!server) {
    set_last_error("server is NULL");
    return HPM_ERR_INVALID_ARG;
  }
  std::unique_lock<std::mutex> lk(server->mu);
  auto it = server->tickets.find(ticket);
  if (it == server->tickets.end()) {
    set_last_error("unknown or already reported ticket");
    return HPM_ERR_INVALID_ARG;
  }
  std::shared_ptr<Request> r = it->second;
  server->cv_done.wait(lk, [&] { return r->done; });
  it = server->tickets.find(ticket);
  if (it == server->tickets.end()) {  // reported meanwhile by another thread
    set_last_error("ticket reported by another call");
    return HPM_ERR_INVALID_ARG;
  }
  return report(server, it, info);
}

hpm_status hpm_server_run_batch(hpm_server* server, int32_t count, const hpm_problem* problems,
                                const int64_t* n, const void* const* x, const void* const* y,
                                const void* const* z, const void* const* m, void* const* phi,
                                void* const* ax, void* const* ay, void* const* az,
                                int32_t* status) {
  std::vector<uint64_t> tk;
  std::vector<hpm_status> st;
  hpm_status first = guarded([&] {
    if (!server) fail(HPM_ERR_INVALID_ARG, "server is NULL");
    if (count < 0) fail(HPM_ERR_INVALID_ARG, "count must be >= 0");
    if (count > 0 && (!problems || !n || !x || !y || !z || !m || !phi || !ax || !ay || !az))
      fail(HPM_ERR_INVALID_ARG, "NULL array");
  });
  if (first != HPM_OK) return first;
  std::vector<int> order(static_cast<size_t>(count));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  tk.assign(size_t(count), 0);
  st.assign(size_t(count), HPM_OK);
  std::vector<bool> queued(static_cast<size_t>(count), false);
  for (int i : order) {
    st[size_t(i)] = hpm_server_submit(server, &problems[i], n[i], x[i], y[i], z[i], m[i], phi[i],
                                      ax[i], ay[i], az[i], &tk[size_t(i)]);
    queued[size_t(i)] = st[size_t(i)] == HPM_OK;
  }
  for (int i : order)
    if (queued[size_t(i)]) st[size_t(i)] = hpm_server_wait(server, tk[size_t(i)], nullptr);
  hpm_status ret = HPM_OK;
  for (int i = 0; i < count; ++i) {
    if (status) status[i] = st[size_t(i)];
    if (ret == HPM_OK && st[size_t(i)] != HPM_OK) ret = st[size_t(i)];
  }
  return ret;
}

hpm_status hpm_server_stats_get(hpm_server* server, hpm_server_stats* stats) {
  if (!server || !stats) {
    set_last_error("NULL argument");
    return HPM_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(server->mu);
  *stats = hpm_server_stats{};
  stats->submitted = server->submitted;
  stats->completed = server->completed;
  stats->failed = server->failed;
  stats->queued = int32_t(server->queue.size());
  stats->running = server->running;
  stats->plans = int64_t(server->pool.size());
  stats->held_bytes = int64_t(server->held);
  stats->peak_held_bytes = int64_t(server->peak_held);
  stats->plans_created = server->created;
  stats->plans_released = server->released;
  return HPM_OK;
}

void hpm_server_destroy(hpm_server* server) {
  if (!server) return;
  {
    std::lock_guard<std::mutex> lk(server->mu);
    server->stop = true;
  }
  server->cv_work.notify_all();
  for (auto& t : server->workers) t.join();  // workers leave once the queue is empty
  server->pool.clear();
  for (hipStream_t s : server->streams) (void)hipStreamDestroy(s);
  delete server;
}

}  // extern "C"
