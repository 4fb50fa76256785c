// Continuous-batching solve server.
//
// A scheduler thread admits requests and hands out rounds of work:
//   1. it admits queued requests in arrival order while a column slot is
//      free and the device bytes their Krylov bases need fit the budget (a
//      request that does not fit waits; one larger than the whole budget is
//      refused at submission), running their bounds and plan;
//   2. it groups the running solves by operator pattern and precision; a
//      round of a group filters the current Lanczos vector of all its
//      members as one multi-column recurrence, then every member takes its
//      Lanczos step (reorthogonalization, convergence check, extraction),
//      all on the group's one stream.  Rounds run as jobs on a pool of host
//      threads, each group's next round as soon as its last one ended, so
//      groups proceed at their own pace: a group of short chains (short
//      filters, many rounds per second) is not held to the pace of a group
//      of long chains.  One stream per group keeps the groups on separate
//      hardware queues where the device has enough of them;
//   3. it retires the members that finished, which frees their slots and
//      bytes for the next admissions.
// Requests thus join and leave a running batch between Lanczos iterations,
// and a request's result does not depend on which others share its batch
// beyond the rounding of the batched filter.
//
// Locking: the scheduler thread takes the context lock (ctx->mu) for
// admissions and the start of rounds only.  Rounds hold ctx->serve_mu
// shared; library calls that may use or change an operator take it
// exclusively (after ctx->mu, so no new round starts meanwhile) and so run
// between rounds, while calls that only build new objects do not wait for
// rounds at all.  Two rounds in flight never share an operator (an
// operator's lazily tuned kernel choices are not guarded otherwise), and a
// request whose operator is in a round in flight waits to be admitted.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <shared_mutex>
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
  // on the stream of the request's last work (its set-up or its group's
  // last round): v_k written, w free
  hipEvent_t ready = nullptr;
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
  std::mutex m;  // pending, active, used, done_rounds, kick, stop
  std::condition_variable cv;
  std::deque<polfed_req*> pending;
  std::vector<polfed_req*> active;
  bool stop = false;
  bool kick = false;  // a request arrived
  std::thread th;
  // The solves of one operator pattern and precision; its recurrence runs on
  // the group's own stream.  Touched by the scheduler thread while no round
  // of the group is in flight, and by the round's job while one is.
  struct Group {
    BatchFilter bf;
    polfed_ctx* gc = nullptr;
    bool busy = false;
  };
  std::map<std::string, std::unique_ptr<Group>> groups;
  // streams of groups that ended, for the next new group: a group's stream
  // lives until the server stops, since events recorded on it (a member's
  // ready event, its timing events) can outlive the group when the member
  // moves on to another group
  std::vector<polfed_ctx*> spare_ctx;
  // a round that ended, with the members that finished in it
  struct Done {
    Group* g = nullptr;
    std::vector<polfed_req*> members;
    std::vector<char> finished;
    std::vector<std::pair<polfed_status, std::string>> outcome;
  };
  std::deque<Done> done_rounds;
  // scheduler thread only
  int in_flight = 0;                             // rounds
  std::set<const polfed_req*> busy_reqs;         // members of rounds in flight
  std::map<const polfed_op*, int> busy_ops;      // their operators
  // host seconds spent in the server's phases (printed at the end with
  // POLFED_VERBOSE): admission set-up, group formation, filter launch,
  // member steps; and counts of rounds and formations
  std::atomic<int64_t> t_setup_us{0}, t_form_us{0}, t_run_us{0}, t_adv_us{0};
  std::atomic<int64_t> n_rounds{0}, n_forms{0};
  // host threads that run the rounds
  std::vector<std::thread> pool;
  std::mutex pm;
  std::condition_variable pcv;
  std::deque<std::function<void()>> jobs;
  bool pool_stop = false;
  void start_pool(int n);
  void post(std::function<void()> job);
  ~Server();
  void loop();
  void admit();
  void round(Group* g, const std::string& key, std::vector<polfed_req*> members);
  void settle(Done& d);
  void complete(polfed_req* r, polfed_status st, const std::string& err);
  void evict(polfed_req* r);
  bool take(polfed_req* r, size_t bytes);
  void give(polfed_req* r, size_t bytes);
};

static polfed_ctx* new_child(const polfed_ctx* parent) {
  auto c = std::make_unique<polfed_ctx>();
  c->device = parent->device;
  c->n_cu = parent->n_cu;
  HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  c->own_stream = true;
  HIPC(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  register_stream(c->device, c->stream);
  return c.release();
}

static void delete_child(polfed_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->ws) b.release();
  unregister_stream(c->device, c->stream);
  (void)hipStreamDestroy(c->stream);
  (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

void Server::start_pool(int n) {
  for (int i = 0; i < n; ++i)
    pool.emplace_back([this] {
      (void)hipSetDevice(ctx->device);
      g_no_capture = true;
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
      }
    });
}

void Server::post(std::function<void()> job) {
  {
    std::lock_guard<std::mutex> lk(pm);
    jobs.push_back(std::move(job));
  }
  pcv.notify_one();
}

Server::~Server() {
  if (verbose())
    std::fprintf(stderr,
                 "[polfed] server: %lld rounds, %lld formations; host s: set-up %.2f, "
                 "formation %.2f, filter launch %.2f, member steps %.2f\n",
                 (long long)n_rounds.load(), (long long)n_forms.load(), 1e-6 * t_setup_us.load(),
                 1e-6 * t_form_us.load(), 1e-6 * t_run_us.load(), 1e-6 * t_adv_us.load());
  {
    std::lock_guard<std::mutex> lk(pm);
    pool_stop = true;
  }
  pcv.notify_all();
  for (auto& t : pool) t.join();
  // every request has finished: the groups' events go before their streams
  for (auto& kv : groups) {
    kv.second->bf.forget();
    delete_child(kv.second->gc);
  }
  for (polfed_ctx* c : spare_ctx) delete_child(c);
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

// The request's event, after its solve is gone.
static void release_own(polfed_req* r) {
  if (r->ready) {
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
  }
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
// so a large request is not overtaken for ever by smaller ones (nor while
// its operator is in a round in flight: setting up a solve may tune it).
void Server::admit() {
  for (;;) {
    polfed_req* r = nullptr;
    {
      std::lock_guard<std::mutex> lk(m);
      if (pending.empty() || (int)active.size() >= max_cols) return;
      if (used + pending.front()->footprint > budget) return;
      if (busy_ops.count(pending.front()->op)) return;
      r = pending.front();
      pending.pop_front();
      used += r->footprint;
      r->held = r->footprint;
      r->held_max = std::max(r->held_max, r->held);
    }
    r->t_admit = now_seconds();
    try {
      HIPC(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
      // the set-up (bounds, plan, v_0) on the context's stream, where the
      // caller wrote the start vector; the rounds run on the group's stream
      polfed_ctx* cc = ctx;
      r->run.reset(new SolveRun());
      r->run->granted = r->prepaid;
      r->run->take = [this, r](size_t b) { return take(r, b); };
      r->run->give = [this, r](size_t b) { give(r, b); };
      TallyScope ts(&r->run->tally);
      const double t0 = now_seconds();
      r->run->setup(cc, r->op, r->p, r->x0, r->evals, r->evecs, r->resid, &r->n_found);
      HIPC(hipEventRecord(r->ready, cc->stream));  // v_0 written
      t_setup_us += (int64_t)(1e6 * (now_seconds() - t0));
      std::lock_guard<std::mutex> lk(m);
      active.push_back(r);
    } catch (const Error& e) {
      complete(r, e.code, e.what());
    } catch (const std::exception& e) {
      complete(r, POLFED_ERR_INVALID, e.what());
    }
  }
}

// One round of a group, on a pool thread: the filter application for every
// member, then each member's Lanczos step.  Members that finish are handed
// to the scheduler thread, which retires them.
void Server::round(Group* g, const std::string& key, std::vector<polfed_req*> members) {
  Done d;
  d.g = g;
  d.members = std::move(members);
  const size_t n = d.members.size();
  d.finished.assign(n, 0);
  d.outcome.resize(n);
  {
    std::shared_lock<std::shared_mutex> sl(ctx->serve_mu);
    std::vector<SolveRun*> runs;
    for (auto* r : d.members) runs.push_back(r->run.get());
    bool filtered = false;
    try {
      // every member's work runs on the group's stream (one hardware queue
      // per group, so the groups do not wait for each other), after its
      // last work elsewhere (set-up, or a round of another group)
      for (auto* r : d.members) {
        HIPC(hipStreamWaitEvent(g->gc->stream, r->ready, 0));
        r->run->ctx = g->gc;
      }
      if (n == 1 && key.rfind("op:", 0) == 0) {
        // a solve of its own: the single-column filter
        TallyScope ts(&runs[0]->tally);
        runs[0]->filter_self();
      } else {
        // rebuilt whenever a member joined or left (a new solve may reuse a
        // finished one's address, so members are compared by uid)
        const double t0 = now_seconds();
        if (!g->bf.same_members(runs)) {
          g->bf.form(g->gc, runs);
          ++n_forms;
        }
        const double t1 = now_seconds();
        g->bf.run();
        t_form_us += (int64_t)(1e6 * (t1 - t0));
        t_run_us += (int64_t)(1e6 * (now_seconds() - t1));
      }
      filtered = true;
    } catch (const Error& e) {
      g->bf.forget();
      for (size_t i = 0; i < n; ++i) d.outcome[i] = {e.code, e.what()};
    } catch (const std::exception& e) {
      g->bf.forget();
      for (size_t i = 0; i < n; ++i) d.outcome[i] = {POLFED_ERR_INVALID, e.what()};
    }
    if (!filtered) {
      d.finished.assign(n, 1);
    } else {
      bool leaving = false;
      const double t0 = now_seconds();
      for (size_t i = 0; i < n; ++i) {
        polfed_req* r = d.members[i];
        try {
          TallyScope ts(&r->run->tally);
          r->run->advance();
          HIPC(hipEventRecord(r->ready, g->gc->stream));  // v_{k+1} written
          if (r->run->done) {
            d.finished[i] = 1;
            d.outcome[i] = {r->run->status, ""};
          }
        } catch (const Error& e) {
          d.finished[i] = 1;
          d.outcome[i] = {e.code, e.what()};
        } catch (const std::exception& e) {
          d.finished[i] = 1;
          d.outcome[i] = {POLFED_ERR_INVALID, e.what()};
        }
        // a member leaves the group when it finished, waits for bytes, or
        // changed precision (an FP32 run restarted in FP64)
        if (d.finished[i] || r->run->blocked() || group_key(r) != key) leaving = true;
      }
      t_adv_us += (int64_t)(1e6 * (now_seconds() - t0));
      ++n_rounds;
      if (leaving) {
        // the filter timings of this group's past rounds, while every
        // member they name is alive
        try {
          g->bf.drain();
        } catch (const std::exception&) {
          g->bf.forget();
        }
      }
      for (size_t i = 0; i < n; ++i)
        if (d.finished[i]) {
          polfed_report& R = d.members[i]->run->R;
          R.filter_GBps = R.t_filter > 0 ? R.filter_bytes / R.t_filter / 1e9 : 0;
        }
    }
  }
  {
    std::lock_guard<std::mutex> lk(m);
    done_rounds.push_back(std::move(d));
  }
  cv.notify_all();
}

// A round that ended: its group and operators are free again, and its
// finished members are retired.
void Server::settle(Done& d) {
  d.g->busy = false;
  --in_flight;
  for (auto* r : d.members) {
    busy_reqs.erase(r);
    auto it = busy_ops.find(r->op);
    if (--it->second == 0) busy_ops.erase(it);
  }
  for (size_t i = 0; i < d.members.size(); ++i)
    if (d.finished[i]) complete(d.members[i], d.outcome[i].first, d.outcome[i].second);
}

void Server::loop() {
  (void)hipSetDevice(ctx->device);
  g_no_capture = true;
  for (;;) {
    std::deque<Done> ended;
    {
      std::unique_lock<std::mutex> lk(m);
      // wakes when a round ends or a request arrives; with no round in
      // flight, at once while there is work to decide on
      cv.wait(lk, [&] {
        return !done_rounds.empty() || kick ||
               (in_flight == 0 && (stop || !pending.empty() || !active.empty()));
      });
      if (stop && pending.empty() && active.empty() && in_flight == 0 && done_rounds.empty())
        return;
      ended.swap(done_rounds);
      kick = false;
    }
    for (auto& d : ended) settle(d);
    // API calls waiting for the context go first
    while (ctx->api_waiting.load() > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    std::lock_guard<std::mutex> ctx_lk(ctx->mu);
    admit();
    // the solves not in a round in flight, by group; a solve waiting for
    // budget takes no filter step
    std::vector<polfed_req*> act;
    {
      std::lock_guard<std::mutex> lk(m);
      act = active;
    }
    std::map<std::string, std::vector<polfed_req*>> by_key;
    std::vector<polfed_req*> waiting;
    for (auto* r : act) {
      if (busy_reqs.count(r)) continue;
      if (r->run->blocked())
        waiting.push_back(r);
      else
        by_key[group_key(r)].push_back(r);
    }
    for (auto it = groups.begin(); it != groups.end();) {
      if (!it->second->busy && !by_key.count(it->first)) {
        it->second->bf.forget();
        spare_ctx.push_back(it->second->gc);
        it = groups.erase(it);
      } else {
        ++it;
      }
    }
    bool launched = false;
    for (auto& kv : by_key) {
      std::unique_ptr<Group>& gp = groups[kv.first];
      if (!gp) {
        gp.reset(new Group());
        if (!spare_ctx.empty()) {
          gp->gc = spare_ctx.back();
          spare_ctx.pop_back();
        } else {
          gp->gc = new_child(ctx);
        }
      }
      if (gp->busy) continue;  // the new members join its next round
      bool clash = false;
      for (auto* r : kv.second) clash = clash || busy_ops.count(r->op) > 0;
      if (clash) continue;  // after the round that uses the operator
      gp->busy = true;
      ++in_flight;
      for (auto* r : kv.second) {
        busy_reqs.insert(r);
        ++busy_ops[r->op];
      }
      Group* g = gp.get();
      std::string key = kv.first;
      std::vector<polfed_req*> mem = kv.second;
      post([this, g, key, mem]() { round(g, key, mem); });
      launched = true;
    }
    // solves waiting for budget: granted now if others have released bytes
    bool progress = launched || in_flight > 0;
    for (auto* r : waiting) {
      try {
        TallyScope ts(&r->run->tally);
        // on this thread's stream, after the solve's last work (its group
        // may have ended and handed its stream to another group); the next
        // round of the solve waits for what resume queues here
        HIPC(hipStreamWaitEvent(ctx->stream, r->ready, 0));
        r->run->ctx = ctx;
        r->run->resume();
        HIPC(hipEventRecord(r->ready, ctx->stream));
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
    // every running solve waits for bytes that no round in flight can free
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
  // the server's threads capture no graphs: filter steps launch directly
  r->p.graph = 2;
  r->t_submit = now_seconds();
  {
    std::lock_guard<std::mutex> lk(s->m);
    REQUIRE(!s->stop, "serve: server is stopping");
    s->pending.push_back(r);
    s->kick = true;
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
