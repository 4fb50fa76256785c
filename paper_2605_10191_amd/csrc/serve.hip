// Continuous-batching solve server.
//
// A scheduler thread owns the context's stream while serving.  Each cycle it
//   1. admits queued requests in arrival order while a column slot is free
//      and the device bytes their Krylov bases need fit the budget (a request
//      that does not fit waits; one larger than the whole budget is refused
//      at submission), running their bounds and plan;
//   2. groups the running solves by operator pattern and precision; each
//      group filters the current Lanczos vector of all its members as one
//      multi-column recurrence on the group's stream, then every member takes
//      its own Lanczos step (reorthogonalization, convergence check,
//      extraction) on its own stream, the members of the round side by side
//      on a pool of host threads;
//   3. retires the members that finished, which frees their slots and bytes
//      for the next admissions.
// Requests thus join and leave a running batch between Lanczos iterations,
// and a request's result does not depend on which others share its batch
// beyond the rounding of the batched filter.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.hpp"
#include "solve_run.hpp"

struct polfed_req {
  polfed_ctx* ctx = nullptr;
  const polfed_op* op = nullptr;
  polfed_params p{};
  const double* x0 = nullptr;
  double *evals = nullptr, *evecs = nullptr, *resid = nullptr;
  size_t footprint = 0;     // device bytes reserved at admission
  size_t held = 0;          // bytes reserved now (admission plus grants)
  size_t held_max = 0;      // the most ever reserved
  size_t prepaid = 0;       // part of footprint learned from an eviction
  polfed_ctx* own = nullptr;  // the request's context (own stream) while admitted
  hipEvent_t ready = nullptr;  // on own's stream: v_k written, w free
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::mutex m;
  std::condition_variable cv;
  bool done = false;
  polfed_status status = POLFED_OK;
  std::string err;
  int n_found = 0;
  polfed_report rep{};
  std::unique_ptr<polfed::SolveRun> run;
};

namespace polfed {

struct Server {
  polfed_ctx* ctx = nullptr;
  size_t budget = 0, used = 0;
  int max_cols = 0;
  std::mutex m;
  std::condition_variable cv;
  std::deque<polfed_req*> pending;
  std::vector<polfed_req*> active;
  bool stop = false;
  std::thread th;
  struct Group {
    BatchFilter bf;
  };
  std::map<std::string, Group> groups;
  // one child context (own stream) per chain pattern for the groups' filter
  // recurrences, so that groups of different patterns overlap on the device
  std::map<std::string, polfed_ctx*> children;
  polfed_ctx* child_for(const polfed_req* r);
  // host threads that advance the members of a round side by side
  std::vector<std::thread> pool;
  std::mutex pm;
  std::condition_variable pcv, pdone;
  std::deque<std::function<void()>> jobs;
  int busy = 0;
  bool pool_stop = false;
  void start_pool(int n);
  void run_all(std::vector<std::function<void()>>& work);
  ~Server();
  void loop();
  void admit();
  void complete(polfed_req* r, polfed_status st, const std::string& err);
  void evict(polfed_req* r);
  bool take(polfed_req* r, size_t bytes);
  void give(polfed_req* r, size_t bytes);
};

static std::string pattern_of(const polfed_op* op) {
  const bool batchable = op->model == Model::Chain && !op->pattern_key.empty() &&
                         op->split_nseg > 0;
  return batchable ? op->pattern_key : std::string("other");
}

static polfed_ctx* new_child(const polfed_ctx* parent) {
  auto c = std::make_unique<polfed_ctx>();
  c->device = parent->device;
  c->n_cu = parent->n_cu;
  HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  c->own_stream = true;
  HIPC(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  return c.release();
}

static void delete_child(polfed_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  (void)hipStreamDestroy(c->stream);
  (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

polfed_ctx* Server::child_for(const polfed_req* r) {
  const std::string key = pattern_of(r->op);
  auto it = children.find(key);
  if (it != children.end()) return it->second;
  return children[key] = new_child(ctx);
}

void Server::start_pool(int n) {
  for (int i = 0; i < n; ++i)
    pool.emplace_back([this] {
      (void)hipSetDevice(ctx->device);
      for (;;) {
        std::function<void()> job;
        {
          std::unique_lock<std::mutex> lk(pm);
          pcv.wait(lk, [&] { return pool_stop || !jobs.empty(); });
          if (pool_stop && jobs.empty()) return;
          job = std::move(jobs.front());
          jobs.pop_front();
        }
        job();  // catches its own errors
        std::lock_guard<std::mutex> lk(pm);
        if (--busy == 0) pdone.notify_all();
      }
    });
}

// Runs the jobs on the pool and waits for all of them.
void Server::run_all(std::vector<std::function<void()>>& work) {
  if (work.empty()) return;
  if (pool.empty() || work.size() == 1) {
    for (auto& f : work) f();
    return;
  }
  std::unique_lock<std::mutex> lk(pm);
  busy += (int)work.size();
  for (auto& f : work) jobs.push_back(std::move(f));
  pcv.notify_all();
  pdone.wait(lk, [&] { return busy == 0; });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(pm);
    pool_stop = true;
  }
  pcv.notify_all();
  for (auto& t : pool) t.join();
  for (auto& kv : children) delete_child(kv.second);
}

static std::string group_key(const polfed_req* r) {
  const polfed_op* op = r->op;
  const bool batchable = op->model == Model::Chain && !op->pattern_key.empty() &&
                         op->split_nseg > 0;
  // operators that cannot share a recurrence each form their own group
  std::string k = batchable ? op->pattern_key : "op:" + std::to_string((uintptr_t)op) + ":" +
                                                    std::to_string((uintptr_t)r);
  return k + (r->run->fp32 ? "|f32" : "|f64");
}

// The request's own context and event, after its solve is gone.
static void release_own(polfed_req* r) {
  if (r->ready) {
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
  }
  delete_child(r->own);
  r->own = nullptr;
}

// Hands an admitted request back to its caller.  Everything the server keeps
// of it (its place among the active solves, its share of the budget, the
// solve and its device memory) is released first: once done is set, the
// caller may destroy the request at any moment, so marking it done, under
// its lock and with the waiters notified before the lock is released, is the
// server's last access to it.
void Server::complete(polfed_req* r, polfed_status st, const std::string& err) {
  std::unique_ptr<SolveRun> run = std::move(r->run);
  polfed_report rep = run ? run->R : polfed_report{};
  if (run) rep.mem_peak = (double)run->tally.peak;
  rep.mem_reserved = (double)r->held_max;
  run.reset();
  release_own(r);
  {
    std::lock_guard<std::mutex> lk(m);
    active.erase(std::remove(active.begin(), active.end(), r), active.end());
    used -= r->held;
    r->held = 0;
  }
  std::lock_guard<std::mutex> lk(r->m);
  r->status = st;
  r->err = err;
  r->rep = rep;
  r->t_done = now_seconds();
  r->rep.t_queue = r->t_admit > 0 ? r->t_admit - r->t_submit : 0;
  r->rep.t_latency = r->t_done - r->t_submit;
  r->done = true;
  r->cv.notify_all();
}

// Grants a running solve more of the budget (false: not available now).
bool Server::take(polfed_req* r, size_t bytes) {
  std::lock_guard<std::mutex> lk(m);
  if (used + bytes > budget) return false;
  used += bytes;
  r->held += bytes;
  r->held_max = std::max(r->held_max, r->held);
  return true;
}

void Server::give(polfed_req* r, size_t bytes) {
  std::lock_guard<std::mutex> lk(m);
  bytes = std::min(bytes, r->held);
  used -= bytes;
  r->held -= bytes;
}

// Every running solve waits for bytes that only a finishing solve could
// free: the latest admitted one is stopped, its memory returned, and it goes
// back to the head of the queue reserving what it has learned it needs (or
// fails if that exceeds the whole budget).  Its solve restarts from x0 when
// it is admitted again.
void Server::evict(polfed_req* r) {
  const size_t need = r->held + r->run->want;
  r->run.reset();
  release_own(r);
  {
    std::lock_guard<std::mutex> lk(m);
    active.erase(std::remove(active.begin(), active.end(), r), active.end());
    used -= r->held;
    r->held = 0;
    if (need <= budget) {
      r->prepaid += need - std::min(need, r->footprint);
      r->footprint = std::max(r->footprint, need);
      pending.push_front(r);
      return;
    }
  }
  complete(r, POLFED_ERR_OOM,
           "serve: the solve needs " + std::to_string(need) +
               " device bytes as its Krylov space grew, more than the whole budget of " +
               std::to_string(budget));
}

// Admission in arrival order: stop at the first request that does not fit,
// so a large request is not overtaken for ever by smaller ones.
void Server::admit() {
  for (;;) {
    polfed_req* r = nullptr;
    {
      std::lock_guard<std::mutex> lk(m);
      if (pending.empty() || (int)active.size() >= max_cols) return;
      if (used + pending.front()->footprint > budget) return;
      r = pending.front();
      pending.pop_front();
      used += r->footprint;
      r->held = r->footprint;
      r->held_max = std::max(r->held_max, r->held);
    }
    r->t_admit = now_seconds();
    try {
      (void)child_for(r);  // the pattern's stream for its group filter
      r->own = new_child(ctx);
      HIPC(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
      polfed_ctx* cc = r->own;
      // the start vector was written on the caller's stream
      hipEvent_t ready;
      HIPC(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      HIPC(hipEventRecord(ready, ctx->stream));
      HIPC(hipStreamWaitEvent(cc->stream, ready, 0));
      HIPC(hipEventDestroy(ready));
      r->run.reset(new SolveRun());
      r->run->granted = r->prepaid;
      r->run->take = [this, r](size_t b) { return take(r, b); };
      r->run->give = [this, r](size_t b) { give(r, b); };
      TallyScope ts(&r->run->tally);
      r->run->setup(cc, r->op, r->p, r->x0, r->evals, r->evecs, r->resid, &r->n_found);
      HIPC(hipEventRecord(r->ready, cc->stream));  // v_0 written
      std::lock_guard<std::mutex> lk(m);
      active.push_back(r);
    } catch (const Error& e) {
      complete(r, e.code, e.what());
    } catch (const std::exception& e) {
      complete(r, POLFED_ERR_INVALID, e.what());
    }
  }
}

void Server::loop() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(m);
      cv.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
      if (stop && pending.empty() && active.empty()) return;
    }
    // API calls waiting for the context go first
    while (ctx->api_waiting.load() > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    std::lock_guard<std::mutex> ctx_lk(ctx->mu);
    admit();
    // current groups
    // a solve waiting for budget takes no filter step this round
    std::map<std::string, std::vector<polfed_req*>> by_key;
    std::vector<polfed_req*> waiting;
    for (auto* r : active) {
      if (r->run->blocked())
        waiting.push_back(r);
      else
        by_key[group_key(r)].push_back(r);
    }
    for (auto it = groups.begin(); it != groups.end();)
      it = by_key.count(it->first) ? std::next(it) : groups.erase(it);
    // every group's filter application is launched before any member is
    // advanced: advancing reads a member's Lanczos coefficients back and so
    // waits for its group's filter, which would otherwise keep the groups'
    // recurrences from running side by side on their streams
    std::vector<std::pair<Group*, const std::vector<polfed_req*>*>> launched;
    for (auto& kv : by_key) {
      std::vector<SolveRun*> runs;
      for (auto* r : kv.second) runs.push_back(r->run.get());
      Group& g = groups[kv.first];
      try {
        if (runs.size() == 1 && kv.first.rfind("op:", 0) == 0) {
          // a solve of its own: the filter on the request's stream
          TallyScope ts(&runs[0]->tally);
          runs[0]->filter_self();
        } else {
          // the group's recurrence on the pattern's stream, after every
          // member's v_k is written (on its own stream), and every member's
          // Lanczos step after the recurrence has written its w
          polfed_ctx* gc = child_for(kv.second[0]);
          for (auto* r : kv.second) HIPC(hipStreamWaitEvent(gc->stream, r->ready, 0));
          // rebuilt whenever a member joined or left (a new solve may reuse
          // a finished one's address, so members are compared by uid)
          if (!g.bf.same_members(runs)) g.bf.form(gc, runs);
          g.bf.run();
          hipEvent_t fe;
          HIPC(hipEventCreateWithFlags(&fe, hipEventDisableTiming));
          HIPC(hipEventRecord(fe, gc->stream));
          for (auto* r : kv.second) HIPC(hipStreamWaitEvent(r->own->stream, fe, 0));
          HIPC(hipEventDestroy(fe));
        }
      } catch (const Error& e) {
        g.bf.forget();
        for (auto* r : kv.second) complete(r, e.code, e.what());
        continue;
      }
      launched.push_back({&g, &kv.second});
    }
    // every member of the launched groups takes its Lanczos step
    // (reorthogonalization on its own stream, then the periodic check and
    // extraction, which wait for that stream only) on the host thread pool
    std::vector<polfed_req*> adv;
    for (auto& gm : launched) adv.insert(adv.end(), gm.second->begin(), gm.second->end());
    std::vector<std::pair<polfed_status, std::string>> outcome(adv.size());
    std::vector<char> finished(adv.size(), 0);
    std::vector<std::function<void()>> work;
    for (size_t i = 0; i < adv.size(); ++i)
      work.push_back([&, i] {
        polfed_req* r = adv[i];
        try {
          TallyScope ts(&r->run->tally);
          r->run->advance();
          HIPC(hipEventRecord(r->ready, r->own->stream));  // v_{k+1} written
          if (r->run->done) {
            finished[i] = 1;
            outcome[i] = {r->run->status, ""};
          }
        } catch (const Error& e) {
          finished[i] = 1;
          outcome[i] = {e.code, e.what()};
        } catch (const std::exception& e) {
          finished[i] = 1;
          outcome[i] = {POLFED_ERR_INVALID, e.what()};
        }
      });
    run_all(work);
    {
      size_t i = 0;
      for (auto& gm : launched) {
        Group& g = *gm.first;
        bool drained = false;
        for (size_t q = 0; q < gm.second->size(); ++q, ++i) {
          if (!finished[i]) continue;
          if (!drained) {
            g.bf.drain();  // the filter timings of the leaving members
            drained = true;
          }
          polfed_report& R = adv[i]->run->R;
          R.filter_GBps = R.t_filter > 0 ? R.filter_bytes / R.t_filter / 1e9 : 0;
          complete(adv[i], outcome[i].first, outcome[i].second);
        }
      }
    }
    // solves waiting for budget: granted now if others have released bytes
    bool progress = !launched.empty();
    for (auto* r : waiting) {
      try {
        TallyScope ts(&r->run->tally);
        r->run->resume();
        if (!r->run->blocked()) progress = true;
        if (r->run->done) complete(r, r->run->status, "");
      } catch (const Error& e) {
        complete(r, e.code, e.what());
        progress = true;
      } catch (const std::exception& e) {
        complete(r, POLFED_ERR_INVALID, e.what());
        progress = true;
      }
    }
    if (!progress && !waiting.empty()) {
      polfed_req* last = nullptr;
      for (auto* r : waiting)
        if (r->run && r->run->blocked() && (!last || r->t_admit > last->t_admit)) last = r;
      if (last) evict(last);
    }
  }
}

polfed_status serve_start(polfed_ctx* ctx, size_t budget, int max_cols) {
  REQUIRE(!ctx->server, "serving already started on this context");
  REQUIRE(budget > 0, "serve: need a positive HBM budget");
  REQUIRE(max_cols >= 1, "serve: need max_cols >= 1");
  auto* s = new Server();
  s->ctx = ctx;
  s->budget = budget;
  s->max_cols = max_cols;
  ctx->server = s;
  s->start_pool(std::min(8, std::max(1, max_cols)));
  s->th = std::thread([s] { s->loop(); });
  return POLFED_OK;
}

polfed_status serve_submit(polfed_ctx* ctx, const polfed_op* op, const polfed_params* p,
                           const double* x0, double* evals, double* evecs, double* resid,
                           polfed_req** out) {
  REQUIRE(ctx->server, "serve: call polfed_serve_start first");
  REQUIRE(op && op->ctx == ctx, "serve: operator missing or from another context");
  REQUIRE(p && x0 && evals && evecs && resid && out, "serve: null argument");
  REQUIRE(p->n_ev >= 1 && p->n_ev <= op->D, "serve: need 1 <= n_ev <= D");
  REQUIRE(p->precision == POLFED_FP64 || p->precision == POLFED_FP32 ||
              p->precision == POLFED_PRECISION_AUTO,
          "serve: bad precision");
  REQUIRE(p->block_size <= 1, "serve: block Lanczos (block_size > 1) runs through polfed_solve only");
  Server* s = ctx->server;
  // device bytes of the request; an automatic precision is resolved at
  // admission, so it reserves the larger of the two
  size_t fp = 0;
  for (const int prec : {POLFED_FP64, POLFED_FP32}) {
    if (p->precision != prec && p->precision != POLFED_PRECISION_AUTO) continue;
    polfed_params q = *p;
    q.precision = prec;
    const size_t tb = prec == POLFED_FP32 ? 4 : 8;
    fp = std::max(fp, SolveRun::footprint(op, q) + 4 * (size_t)op->D * tb);
  }
  if (fp > s->budget)
    fail(POLFED_ERR_REJECTED, "serve: request needs " + std::to_string(fp) +
                                  " device bytes, more than the whole budget of " +
                                  std::to_string(s->budget));
  auto* r = new polfed_req();
  r->ctx = ctx;
  r->op = op;
  r->p = *p;
  r->x0 = x0;
  r->evals = evals;
  r->evecs = evecs;
  r->resid = resid;
  r->footprint = fp;
  // the server's loop enqueues for many groups: a filter application is one
  // graph replay unless the caller asked for direct launches
  if (r->p.graph == 0) r->p.graph = 1;
  r->t_submit = now_seconds();
  {
    std::lock_guard<std::mutex> lk(s->m);
    REQUIRE(!s->stop, "serve: server is stopping");
    s->pending.push_back(r);
  }
  s->cv.notify_all();
  *out = r;
  return POLFED_OK;
}

polfed_status req_poll(polfed_req* r, int* done) {
  REQUIRE(r && done, "null request");
  std::lock_guard<std::mutex> lk(r->m);
  *done = r->done ? 1 : 0;
  return POLFED_OK;
}

polfed_status req_wait(polfed_req* r, int* n_found, polfed_report* rep) {
  REQUIRE(r, "null request");
  std::unique_lock<std::mutex> lk(r->m);
  r->cv.wait(lk, [&] { return r->done; });
  if (n_found) *n_found = r->n_found;
  if (rep) *rep = r->rep;
  if (r->status < 0) fail(r->status, r->err);
  return r->status;
}

polfed_status req_destroy(polfed_req* r) {
  if (!r) return POLFED_OK;
  {
    std::lock_guard<std::mutex> lk(r->m);
    if (!r->done) fail(POLFED_ERR_BUSY, "request still running; wait for it first");
  }
  delete r;
  return POLFED_OK;
}

// Finishes every submitted request, then ends the scheduler thread.
polfed_status serve_stop(polfed_ctx* ctx) {
  Server* s = ctx->server;
  if (!s) return POLFED_OK;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  ctx->server = nullptr;
  delete s;
  return POLFED_OK;
}

}  // namespace polfed
