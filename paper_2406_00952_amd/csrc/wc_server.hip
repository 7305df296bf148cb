// Serving: a queue of whole solves run by worker threads, one HIP stream each, with
// admission by the plans' HBM footprint and a cache of idle plans for reuse.
//
// Scheduling.  Requests start in submission order.  The head of the queue starts when a
// worker is free and either an idle plan of the same shape exists (same sizes, method,
// precision and restart: it is retargeted to the new problem without allocating) or the
// plans held by running requests plus the head's footprint fit the budget (idle plans
// are freed, oldest first, to make room).  A running request keeps its plan until it is
// done; the plan then goes to the idle cache, still counted against the budget.
//
// Concurrency happens on the device: every worker enqueues its solve's kernels on its
// own stream, so small and large solves overlap and a new request does not wait for the
// ones in flight.  The solve itself is the library's ordinary wc_solve, so results do not
// depend on what else runs (every reduction has a fixed order).

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wc.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Key {
  wc_problem prob{};
  wc_opts opts{};
  std::vector<double> aface;

  bool operator==(const Key &o) const {
    const wc_problem &a = prob, &b = o.prob;
    const bool pe = a.dims == b.dims && a.M == b.M && a.n == b.n && a.T == b.T &&
                    a.theta == b.theta && a.gamma == b.gamma && a.zeta == b.zeta &&
                    a.s2_remedy == b.s2_remedy;
    const wc_opts &c = opts, &d = o.opts;
    const bool oe = c.method == d.method && c.precision == d.precision && c.tol == d.tol &&
                    c.maxit == d.maxit && c.restart == d.restart && c.flexible == d.flexible &&
                    c.mg_max_cycles == d.mg_max_cycles && c.mg_tol == d.mg_tol &&
                    c.graphs == d.graphs && c.lowrank == d.lowrank;
    return pe && oe && aface == o.aface;
  }

  // same device footprint and buffers: a plan for one can be retargeted to the other
  bool same_shape(const Key &o) const {
    return prob.dims == o.prob.dims && prob.M == o.prob.M && prob.n == o.prob.n &&
           opts.method == o.opts.method && opts.precision == o.opts.precision &&
           opts.restart == o.opts.restart && opts.flexible == o.opts.flexible &&
           opts.lowrank == o.opts.lowrank && aface.empty() == o.aface.empty();
  }
};

enum ReqState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Req {
  Key key;
  const double *f = nullptr, *g = nullptr, *y0 = nullptr;
  double *y = nullptr, *p = nullptr, *u = nullptr;
  size_t bytes = 0;
  int state = QUEUED;
  wc_info info{};
  Clock::time_point t_submit, t_start, t_end;
};

struct IdlePlan {
  Key key;
  wc_plan *plan;
  size_t bytes;
};

}  // namespace

struct wc_server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next = 1;
  std::list<IdlePlan> idle;  // oldest first
  size_t in_use = 0;         // footprints of running requests' plans and of idle plans
  bool stop = false;
  std::vector<std::thread> workers;

  size_t idle_bytes() const {
    size_t b = 0;
    for (const auto &i : idle) b += i.bytes;
    return b;
  }

  bool idle_match(const Key &k) const {
    for (const auto &i : idle)
      if (i.key.same_shape(k)) return true;
    return false;
  }

  // called with mu held
  bool can_start() const {
    if (queue.empty()) return false;
    const Req &r = reqs.at(queue.front());
    if (idle_match(r.key)) return true;
    return in_use - idle_bytes() + r.bytes <= budget;
  }

  void worker();
};

void wc_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  if (hipStreamCreate(&stream) != hipSuccess) stream = nullptr;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] { return stop || can_start(); });
    if (stop) break;
    const uint64_t id = queue.front();
    queue.pop_front();
    Req &r = reqs.at(id);
    // an idle plan for the same problem, else one of the same shape to retarget
    wc_plan *plan = nullptr;
    bool exact = false;
    for (int pass = 0; pass < 2 && !plan; ++pass)
      for (auto it = idle.begin(); it != idle.end(); ++it)
        if (pass == 0 ? it->key == r.key : it->key.same_shape(r.key)) {
          plan = it->plan;
          exact = pass == 0;
          idle.erase(it);
          break;
        }
    std::vector<wc_plan *> evict;
    if (!plan) {
      while (in_use + r.bytes > budget && !idle.empty()) {
        evict.push_back(idle.front().plan);
        in_use -= idle.front().bytes;
        idle.pop_front();
      }
      in_use += r.bytes;
    }
    r.state = RUNNING;
    r.t_start = Clock::now();
    lk.unlock();
    for (wc_plan *e : evict) (void)wc_plan_destroy(e);
    wc_status st = WC_OK;
    wc_problem pr = r.key.prob;
    pr.a_face_host = r.key.aface.empty() ? nullptr : r.key.aface.data();
    if (!stream) {
      st = WC_E_HIP;
    } else if (!plan) {
      st = wc_plan_create(&pr, &r.key.opts, stream, &plan);
    } else {
      st = wc_plan_set_stream(plan, stream);
      if (st == WC_OK && !exact) st = wc_plan_retarget(plan, &pr, &r.key.opts);
    }
    wc_info info{};
    if (st == WC_OK) st = wc_solve(plan, r.f, r.g, r.y0, r.y, r.p, r.u, &info);
    info.status = st;
    lk.lock();
    r.info = info;
    r.t_end = Clock::now();
    r.state = DONE;
    if (plan) idle.push_back({r.key, plan, r.bytes});
    else in_use -= r.bytes;
    cv.notify_all();
  }
  lk.unlock();
  if (stream) (void)hipStreamDestroy(stream);
}

extern "C" {

wc_status wc_server_create(size_t hbm_budget, int max_concurrency, wc_server **out) {
  if (!out) return WC_E_ARG;
  *out = nullptr;
  if (max_concurrency < 1 || max_concurrency > 64) return WC_E_ARG;
  wc_server *s = new (std::nothrow) wc_server();
  if (!s) return WC_E_NOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return WC_E_HIP;
  }
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return WC_E_HIP;
    }
    hbm_budget = fr / 10 * 9;
  }
  s->budget = hbm_budget;
  for (int i = 0; i < max_concurrency; ++i) s->workers.emplace_back([s] { s->worker(); });
  *out = s;
  return WC_OK;
}

wc_status wc_server_destroy(wc_server *s) {
  if (!s) return WC_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (uint64_t id : s->queue) {
      Req &r = s->reqs.at(id);
      r.state = DONE;
      r.info.status = WC_E_CANCELLED;
      r.t_end = Clock::now();
    }
    s->queue.clear();
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->workers) t.join();
  for (auto &i : s->idle) (void)wc_plan_destroy(i.plan);
  delete s;
  return WC_OK;
}

wc_status wc_server_submit(wc_server *s, const wc_problem *prob, const wc_opts *opts,
                           const double *f, const double *g, const double *y0, double *y,
                           double *p, double *u, uint64_t *ticket) {
  if (!s || !prob || !opts || !f || !g || !y0 || !y || !p || !ticket) return WC_E_ARG;
  const size_t bytes = wc_plan_footprint_bytes(prob, opts);
  if (bytes == 0) return WC_E_ARG;
  if (bytes > s->budget) return WC_E_ADMISSION;
  Req r;
  r.key.prob = *prob;
  r.key.prob.a_face_host = nullptr;
  r.key.opts = *opts;
  if (prob->a_face_host) {
    const size_t nf = prob->dims == 1 ? (size_t)prob->M + 1 : 2 * (size_t)prob->M * (prob->M + 1);
    r.key.aface.assign(prob->a_face_host, prob->a_face_host + nf);
  }
  r.f = f; r.g = g; r.y0 = y0; r.y = y; r.p = p; r.u = u;
  r.bytes = bytes;
  r.t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return WC_E_CANCELLED;
    const uint64_t id = s->next++;
    s->reqs.emplace(id, std::move(r));
    s->queue.push_back(id);
    *ticket = id;
  }
  s->cv.notify_all();
  return WC_OK;
}

wc_status wc_server_poll(wc_server *s, uint64_t ticket, int *done, wc_info *info) {
  if (!s || !done) return WC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return WC_E_ARG;
  *done = it->second.state == DONE ? 1 : 0;
  if (*done && info) *info = it->second.info;
  return WC_OK;
}

wc_status wc_server_wait(wc_server *s, uint64_t ticket, wc_info *info, double *queue_ms,
                         double *total_ms) {
  if (!s) return WC_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return WC_E_ARG;
  const Req &r = it->second;  // element references survive rehashing, iterators do not
  s->cv.wait(lk, [&] { return r.state == DONE; });
  if (info) *info = r.info;
  const bool started = r.t_start.time_since_epoch().count() != 0;
  if (queue_ms)
    *queue_ms = started ? std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count() : 0.0;
  if (total_ms) *total_ms = std::chrono::duration<double, std::milli>(r.t_end - r.t_submit).count();
  s->reqs.erase(ticket);
  return WC_OK;
}

wc_status wc_server_cancel(wc_server *s, uint64_t ticket) {
  if (!s) return WC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.state != QUEUED) return WC_E_ARG;
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == ticket) {
      s->queue.erase(q);
      break;
    }
  it->second.state = DONE;
  it->second.info.status = WC_E_CANCELLED;
  it->second.t_end = Clock::now();
  s->cv.notify_all();
  return WC_OK;
}

size_t wc_server_bytes_in_use(wc_server *s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->in_use;
}

}  // extern "C"
