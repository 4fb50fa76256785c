// Continuous-batching solve server.
//
// A scheduler thread owns the context's stream while serving.  Each cycle it
//   1. admits queued requests in arrival order while a column slot is free
//      and the device bytes their Krylov bases need fit the budget (a request
//      that does not fit waits; one larger than the whole budget is refused
//      at submission), running their bounds and plan;
//   2. groups the running solves by operator pattern and precision; each
//      group filters the current Lanczos vector of all its members as one
//      multi-column recurrence, then every member takes its own Lanczos step
//      (reorthogonalization, convergence check, extraction);
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
  // one child context (own stream) per chain pattern, so that groups of
  // different patterns overlap on the device
  std::map<std::string, polfed_ctx*> children;
  polfed_ctx* child_for(const polfed_req* r);
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

polfed_ctx* Server::child_for(const polfed_req* r) {
  const std::string key = pattern_of(r->op);
  auto it = children.find(key);
  if (it != children.end()) return it->second;
  auto c = std::make_unique<polfed_ctx>();
  c->device = ctx->device;
  c->n_cu = ctx->n_cu;
  HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  c->own_stream = true;
  HIPC(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  return children[key] = c.release();
}

Server::~Server() {
  for (auto& kv : children) {
    polfed_ctx* c = kv.second;
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
    (void)hipStreamDestroy(c->cap_stream);
    delete c;
  }
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
      polfed_ctx* cc = child_for(r);
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
          TallyScope ts(&runs[0]->tally);
          runs[0]->filter_self();
        } else {
          // rebuilt whenever a member joined or left (a new solve may reuse
          // a finished one's address, so members are compared by uid)
          if (!g.bf.same_members(runs)) g.bf.form(runs[0]->ctx, runs);
          g.bf.run();
        }
      } catch (const Error& e) {
        g.bf.forget();
        for (auto* r : kv.second) complete(r, e.code, e.what());
        continue;
      }
      launched.push_back({&g, &kv.second});
    }
    for (auto& gm : launched) {
      Group& g = *gm.first;
      std::vector<std::pair<polfed_req*, std::pair<polfed_status, std::string>>> fin;
      for (auto* r : *gm.second) {
        try {
          TallyScope ts(&r->run->tally);
          r->run->advance();
          if (r->run->done) fin.push_back({r, {r->run->status, ""}});
        } catch (const Error& e) {
          fin.push_back({r, {e.code, e.what()}});
        } catch (const std::exception& e) {
          fin.push_back({r, {POLFED_ERR_INVALID, e.what()}});
        }
      }
      if (!fin.empty()) {
        g.bf.drain();  // the filter timings of the leaving members
        for (auto& f : fin) {
          polfed_report& R = f.first->run->R;
          R.filter_GBps = R.t_filter > 0 ? R.filter_bytes / R.t_filter / 1e9 : 0;
          complete(f.first, f.second.first, f.second.second);
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
