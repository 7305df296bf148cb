// Serving: requests admitted by the HBM footprint of their plans, run with iteration-level
// continuous batching where the batched preconditioner kernels apply and as whole solves on
// worker threads otherwise, with a cache of idle plans for reuse.
//
// Continuous batching.  GMRES(k)-P_S requests in the standard form on 2D grids with a = 1
// (n and M + 1 in {64, ..., 512}) go to one batcher thread that runs a lockstep engine:
// every round advances each active solve by one Krylov step, applying the preconditioner of
// all of them in one launch per pass, and synchronises once.  Queued requests join at the
// next round boundary as soon as memory allows (up to 32 active), finished ones leave at
// the round in which they converge, so a request never waits for a batch to drain.
//
// Whole solves.  Other requests (1D, variable a, MINRES, the low-rank form, other sizes)
// run wc_solve on worker threads, one HIP stream each, so they overlap on the device with
// each other and with the batcher.
//
// Admission.  Each queue starts its requests in submission order.  The head of a queue
// starts when an idle plan of the same shape exists (same sizes, method, precision and
// restart: it is retargeted to the new problem without allocating) or the plans held by
// running requests plus the head's footprint fit the budget (idle plans are freed, oldest
// first, to make room).  A running request keeps its plan until it is done; the plan then
// goes to the idle cache, still counted against the budget.
//
// Results do not depend on what else runs: every reduction has a fixed order and each
// batched kernel's work units read and write one instance only, so a request gives the same
// bits alone and in any mix (on the same path).

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wc_internal.h"

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
                    a.s2_remedy == b.s2_remedy && a.disc == b.disc && a.bc == b.bc &&
                    a.kappa == b.kappa;
    const wc_opts &c = opts, &d = o.opts;
    const bool oe = c.method == d.method && c.precision == d.precision && c.tol == d.tol &&
                    c.maxit == d.maxit && c.restart == d.restart && c.flexible == d.flexible &&
                    c.mg_max_cycles == d.mg_max_cycles && c.mg_tol == d.mg_tol &&
                    c.graphs == d.graphs && c.lowrank == d.lowrank;
    return pe && oe && aface == o.aface;
  }

  // same device footprint and buffers: a plan for one can be retargeted to the other (the
  // preconditioner's path, which zeta == pi or not decides at equal sizes, must match too)
  bool same_shape(const Key &o) const {
    const bool pi_a = std::fabs(prob.zeta - M_PI) <= 1e-12;
    const bool pi_b = std::fabs(o.prob.zeta - M_PI) <= 1e-12;
    return prob.dims == o.prob.dims && prob.M == o.prob.M && prob.n == o.prob.n &&
           prob.disc == o.prob.disc && prob.bc == o.prob.bc && pi_a == pi_b &&
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
  bool batched = false;  // served by the lockstep engine
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
  std::deque<uint64_t> queue;   // whole solves (workers)
  std::deque<uint64_t> bqueue;  // continuously batched solves (batcher)
  std::thread batcher;
  uint64_t n_batched = 0;       // requests that ran in the lockstep engine
  int max_lanes = 0;            // largest number of solves active in one round
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
  bool can_start(const std::deque<uint64_t> &q) const {
    if (q.empty()) return false;
    const Req &r = reqs.at(q.front());
    if (idle_match(r.key)) return true;
    return in_use - idle_bytes() + r.bytes <= budget;
  }

  // called with mu held: pops the head of q and picks its plan (an idle one for the same
  // problem, else one of the same shape to retarget, else none: memory is reserved and
  // idle plans to free are returned in evict)
  uint64_t take(std::deque<uint64_t> &q, wc_plan **plan, bool *exact,
                std::vector<wc_plan *> &evict) {
    const uint64_t id = q.front();
    q.pop_front();
    Req &r = reqs.at(id);
    *plan = nullptr;
    *exact = false;
    for (int pass = 0; pass < 2 && !*plan; ++pass)
      for (auto it = idle.begin(); it != idle.end(); ++it)
        if (pass == 0 ? it->key == r.key : it->key.same_shape(r.key)) {
          *plan = it->plan;
          *exact = pass == 0;
          idle.erase(it);
          break;
        }
    if (!*plan) {
      while (in_use + r.bytes > budget && !idle.empty()) {
        evict.push_back(idle.front().plan);
        in_use -= idle.front().bytes;
        idle.pop_front();
      }
      in_use += r.bytes;
    }
    r.state = RUNNING;
    r.t_start = Clock::now();
    return id;
  }

  // without mu: a plan for request r on stream (created, or retargeted unless exact)
  static wc_status prepare(Req &r, wc_plan **plan, bool exact, hipStream_t stream) {
    wc_problem pr = r.key.prob;
    pr.a_face_host = r.key.aface.empty() ? nullptr : r.key.aface.data();
    if (!stream) return WC_E_HIP;
    if (!*plan) return wc_plan_create(&pr, &r.key.opts, stream, plan);
    wc_status st = wc_plan_set_stream(*plan, stream);
    if (st == WC_OK && !exact) st = wc_plan_retarget(*plan, &pr, &r.key.opts);
    return st;
  }

  // with mu held: request id finished with info; its plan (or reservation) is released
  void finish(uint64_t id, wc_plan *plan, const wc_info &info) {
    Req &r = reqs.at(id);
    r.info = info;
    r.t_end = Clock::now();
    r.state = DONE;
    if (plan) idle.push_back({r.key, plan, r.bytes});
    else in_use -= r.bytes;
  }

  void worker();
  void batch_loop();
};

void wc_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  if (hipStreamCreate(&stream) != hipSuccess) stream = nullptr;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] { return stop || can_start(queue); });
    if (stop) break;
    wc_plan *plan = nullptr;
    bool exact = false;
    std::vector<wc_plan *> evict;
    const uint64_t id = take(queue, &plan, &exact, evict);
    Req &r = reqs.at(id);
    lk.unlock();
    for (wc_plan *e : evict) (void)wc_plan_destroy(e);
    wc_status st = prepare(r, &plan, exact, stream);
    wc_info info{};
    if (st == WC_OK) st = wc_solve(plan, r.f, r.g, r.y0, r.y, r.p, r.u, &info);
    info.status = st;
    lk.lock();
    finish(id, plan, info);
    cv.notify_all();
  }
  lk.unlock();
  if (stream) (void)hipStreamDestroy(stream);
}

void wc_server::batch_loop() {
  (void)hipSetDevice(device);
  hipStream_t stream = nullptr;
  if (hipStreamCreate(&stream) != hipSuccess) stream = nullptr;
  LockstepEngine *eng = stream ? wc::lockstep_create(stream) : nullptr;
  std::unordered_map<uint64_t, wc_plan *> lane_plans;  // the engine's solves and their plans
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    const int active = eng ? wc::lockstep_active(eng) : 0;
    cv.wait(lk, [&] { return stop || active > 0 || can_start(bqueue); });
    if (stop && active == 0) break;
    // admission at this round boundary
    struct Adm {
      uint64_t id;
      Req *req;  // element pointers of the map stay valid; the request is RUNNING
      wc_plan *plan;
      bool exact;
    };
    std::vector<Adm> adm;
    std::vector<wc_plan *> evict;
    while (!stop && active + (int)adm.size() < wc::kBatchMax && can_start(bqueue)) {
      Adm a{};
      a.id = take(bqueue, &a.plan, &a.exact, evict);
      a.req = &reqs.at(a.id);
      adm.push_back(a);
    }
    lk.unlock();
    for (wc_plan *e : evict) (void)wc_plan_destroy(e);
    std::vector<wc::LockstepDone> done;
    for (Adm &a : adm) {
      Req &r = *a.req;
      wc_status st = eng ? prepare(r, &a.plan, a.exact, stream) : WC_E_HIP;
      if (st == WC_OK &&
          wc::lockstep_add(eng, a.plan, r.f, r.g, r.y0, r.y, r.p, r.u, a.id) != hipSuccess)
        st = WC_E_HIP;
      if (st != WC_OK) {
        wc_info info{};
        info.status = st;
        done.push_back({a.id, a.plan, info});
      } else {
        lane_plans[a.id] = a.plan;
      }
    }
    const int lanes = eng ? wc::lockstep_active(eng) : 0;
    hipError_t e = hipSuccess;
    if (lanes > 0) e = wc::lockstep_round(eng, done);
    if (e != hipSuccess) {  // the engine's state is unusable: fail its solves, start afresh
      (void)hipGetLastError();
      wc::lockstep_destroy(eng);
      for (auto &kv : lane_plans) (void)wc_plan_destroy(kv.second);
      lk.lock();
      for (const wc::LockstepDone &d : done)
        if (!lane_plans.count(d.tag)) finish(d.tag, d.plan, d.info);
      for (auto &kv : lane_plans) {
        wc_info info{};
        info.status = WC_E_HIP;
        finish(kv.first, nullptr, info);
      }
      lane_plans.clear();
      eng = wc::lockstep_create(stream);
      cv.notify_all();
      continue;
    }
    lk.lock();
    if (lanes > max_lanes) max_lanes = lanes;
    for (const wc::LockstepDone &d : done) {
      finish(d.tag, d.plan, d.info);
      lane_plans.erase(d.tag);
      ++n_batched;
    }
    if (!done.empty()) cv.notify_all();
  }
  lk.unlock();
  wc::lockstep_destroy(eng);
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
  s->batcher = std::thread([s] { s->batch_loop(); });
  *out = s;
  return WC_OK;
}

wc_status wc_server_destroy(wc_server *s) {
  if (!s) return WC_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto *q : {&s->queue, &s->bqueue}) {
      for (uint64_t id : *q) {
        Req &r = s->reqs.at(id);
        r.state = DONE;
        r.info.status = WC_E_CANCELLED;
        r.t_end = Clock::now();
      }
      q->clear();
    }
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->workers) t.join();
  if (s->batcher.joinable()) s->batcher.join();  // finishes the solves it is running
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
    const bool batched = wc::lockstep_eligible(prob, opts);
    r.batched = batched;
    s->reqs.emplace(id, std::move(r));
    (batched ? s->bqueue : s->queue).push_back(id);
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
  for (auto *qq : {&s->queue, &s->bqueue})
    for (auto q = qq->begin(); q != qq->end(); ++q)
      if (*q == ticket) {
        qq->erase(q);
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

wc_status wc_server_stats(wc_server *s, uint64_t *batched, int *max_active) {
  if (!s) return WC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batched) *batched = s->n_batched;
  if (max_active) *max_active = s->max_lanes;
  return WC_OK;
}

}  // extern "C"
