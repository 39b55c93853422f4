// Request loop of the library (mspcg_server_*): resident gauge fields,
// admission in arrival order by device footprint, and two ways of running
// the admitted requests:
//
//   continuous batching (default): one engine per request shape (field,
//   Mobius parameters, tiling, solver parameters), each a handle with an
//   open continuous-batching session of a fixed number of RHS slots
//   (mspcg_cb_*) driven by a thread of its own on its own HIP stream.  A
//   request's right-hand sides queue at their shape's engine and enter its
//   slots as earlier ones finish, between iteration pairs, while the others
//   keep iterating; engines of different shapes run concurrently.
//
//   per-request contexts: one resident solver context per shape and one
//   worker thread with its own stream per admitted request, which runs the
//   request as one batched solve (mspcg_solve_batch_device).
//
// Built on the public C ABI only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "mspcg.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// a resident solver context (per-request mode): one handle with its
// workspaces, sharing the gauge field of its field's handle
struct Ctx {
  mspcg_t h = nullptr;
  std::string key;
  int64_t bytes = 0;   // device bytes accounted to it (allocated or reserved)
  bool busy = false;
  uint64_t last_use = 0;
  Ctx() = default;
  Ctx(const Ctx&) = delete;
  Ctx& operator=(const Ctx&) = delete;
  ~Ctx() {
    if (h) (void)mspcg_destroy(h);
  }
};

struct Req {
  mspcg_request r;
  std::vector<mspcg_stats> st;
  mspcg_status status = MSPCG_OK;
  std::string err;
  double t_submit = 0, t_end = 0;
  bool done = false;
  Ctx* ctx = nullptr;
  int remaining = 0;   // continuous batching: right-hand sides not finished
};

struct Field {
  mspcg_t h = nullptr;
  int32_t dims[4];
  int64_t bytes = 0;
};

std::string key_of(const mspcg_request& r, bool with_solver) {
  char buf[512];
  int n = std::snprintf(buf, sizeof(buf), "%d|%d|%a|%a|%a|%a|%d,%d,%d,%d", r.field, r.Ls, r.b, r.c, r.M5, r.mf,
                        r.sub[0], r.sub[1], r.sub[2], r.sub[3]);
  if (with_solver) {
    const mspcg_solver_params& p = r.solver;
    std::snprintf(buf + n, sizeof(buf) - (size_t)n, "|%a|%d|%d|%d|%d|%a|%d|%d", p.tol, p.maxiter, p.inner_iters,
                  (int)p.inner_prec, (int)p.outer_prec, p.reliable_delta, p.beta_rule, p.use_precond);
  }
  return buf;
}

// a right-hand side of a request (continuous batching)
struct Job {
  Req* q = nullptr;
  int i = 0;
};

}  // namespace

struct mspcg_server;

namespace {

// one request shape with an open continuous-batching session
struct Engine {
  mspcg_server* s = nullptr;
  mspcg_t h = nullptr;
  std::string key;
  int64_t bytes = 0;
  int slots = 0;
  int64_t per = 0;         // reals of one right-hand side (2 x 12 x Ls x V/2)
  std::deque<Job> queue;   // waiting for a slot (under the server's mutex)
  int in_slots = 0;        // jobs in slots (under the server's mutex)
  bool stop = false;
  uint64_t last_use = 0;
  std::condition_variable cv;
  std::thread th;
  bool idle() const { return queue.empty() && in_slots == 0; }
  void run();
};

}  // namespace

struct mspcg_server {
  int device = 0;
  int64_t budget = 0;
  int max_inflight = 1;
  int mode = 1;      // 1: continuous batching, 0: per-request contexts
  int slots = 8;     // RHS slots of a continuous-batching engine
  // contexts launch eagerly unless enabled: while a capture is open, device-
  // wide synchronization by any other thread of the process fails, and the
  // caller's threads are not the server's to restrict
  int graphs = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Field> fields;
  std::list<std::unique_ptr<Ctx>> ctxs;
  std::list<std::unique_ptr<Engine>> engines;
  std::vector<std::unique_ptr<Engine>> retired;   // stopping; joined outside the lock
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::deque<Req*> waiting;   // submitted, not admitted
  std::deque<Req*> ready;     // per-request mode: admitted, not yet picked up by a worker
  std::vector<std::thread> workers;

  int64_t next_ticket = 1;
  int64_t used = 0, peak = 0, completed = 0, evictions = 0;
  int inflight = 0, peak_inflight = 0;
  uint64_t tick = 0;
  bool stop = false;

  // ---------------------------------------------------------------- under mu
  void complete(Req* q, mspcg_status st, const std::string& err) {
    q->status = st;
    q->err = err;
    q->t_end = now_ms();
    q->done = true;
    ++completed;
    cv_done.notify_all();
  }

  // free the least recently used idle context or engine other than `keep`
  bool evict_one(const void* keep) {
    auto victim = ctxs.end();
    for (auto it = ctxs.begin(); it != ctxs.end(); ++it) {
      const Ctx* c = it->get();
      if (c->busy || c == keep) continue;
      if (victim == ctxs.end() || c->last_use < (*victim)->last_use) victim = it;
    }
    auto ev = engines.end();
    for (auto it = engines.begin(); it != engines.end(); ++it) {
      const Engine* e = it->get();
      if (!e->idle() || e == keep) continue;
      if (ev == engines.end() || e->last_use < (*ev)->last_use) ev = it;
    }
    const bool take_ctx = victim != ctxs.end() &&
                          (ev == engines.end() || (*victim)->last_use <= (*ev)->last_use);
    if (take_ctx) {
      used -= (*victim)->bytes;
      ctxs.erase(victim);
    } else if (ev != engines.end()) {
      used -= (*ev)->bytes;
      (*ev)->stop = true;
      (*ev)->cv.notify_all();
      retired.push_back(std::move(*ev));
      engines.erase(ev);
    } else {
      return false;
    }
    ++evictions;
    return true;
  }

  // a handle for the request's shape sharing its field's gauge links
  mspcg_t new_handle(const mspcg_request& r, mspcg_status& st, std::string& err) {
    const Field& f = fields[(size_t)r.field];
    mspcg_t h = nullptr;
    st = mspcg_create(&h, f.dims, device);
    if (st == MSPCG_OK) st = mspcg_share_gauge(h, f.h);
    if (st == MSPCG_OK) st = mspcg_set_graphs(h, graphs);
    if (st == MSPCG_OK) st = mspcg_set_mobius(h, r.Ls, r.b, r.c, r.M5, r.mf);
    const bool tiled = r.sub[0] > 0 || r.sub[1] > 0 || r.sub[2] > 0 || r.sub[3] > 0;
    if (st == MSPCG_OK && tiled) st = mspcg_set_subdomains(h, r.sub);
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      if (h) (void)mspcg_destroy(h);
      return nullptr;
    }
    return h;
  }

  // a context for the request's key: an idle resident one, else a new one
  Ctx* context_for(Req* q, mspcg_status& st, std::string& err) {
    const std::string key = key_of(q->r, false);
    Ctx* best = nullptr;
    for (auto& c : ctxs)
      if (!c->busy && c->key == key && (!best || c->bytes > best->bytes)) best = c.get();
    if (best) return best;
    std::unique_ptr<Ctx> c(new Ctx());
    c->key = key;
    c->h = new_handle(q->r, st, err);
    if (!c->h) return nullptr;
    int64_t est = 0, alloc = 0;
    st = mspcg_footprint(c->h, 1, &est, &alloc);
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      return nullptr;
    }
    c->bytes = alloc;
    used += alloc;
    peak = std::max(peak, used);
    ctxs.push_back(std::move(c));
    return ctxs.back().get();
  }

  // continuous batching: the engine of the request's shape, created when
  // the budget allows; nullptr with st == OK means "wait for memory"
  Engine* engine_for(Req* q, mspcg_status& st, std::string& err) {
    const std::string key = key_of(q->r, true);
    for (auto& e : engines)
      if (e->key == key) return e.get();
    int active = 0;
    for (auto& e : engines) active += !e->idle();
    mspcg_t h = new_handle(q->r, st, err);
    if (!h) return nullptr;
    // An engine opens with as many of the server's slots as the budget
    // holds (at least one): a large volume runs fewer right-hand sides at
    // a time, and a request with more right-hand sides than slots runs them
    // in turn.
    int n = slots;
    int64_t est = 0, alloc = 0;
    st = mspcg_set_solver(h, &q->r.solver);
    if (st == MSPCG_OK) st = mspcg_footprint(h, n, &est, &alloc);
    while (st == MSPCG_OK && active < max_inflight && used + est > budget && evict_one(nullptr)) {
    }
    while (st == MSPCG_OK && n > 1 && used + est > budget) st = mspcg_footprint(h, --n, &est, &alloc);
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      (void)mspcg_destroy(h);
      return nullptr;
    }
    if (used + est > budget || active >= max_inflight) {
      (void)mspcg_destroy(h);
      bool busy = active > 0;
      for (auto& c : ctxs) busy |= c->busy;
      if (!busy) {   // it does not fit even alone
        st = MSPCG_ERR_OOM;
        err = "an engine of one slot needs " + std::to_string(est) +
              " bytes beyond the resident fields; the budget leaves " + std::to_string(budget - used);
      }
      return nullptr;
    }
    st = mspcg_cb_open(h, n, nullptr);
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      (void)mspcg_destroy(h);
      return nullptr;
    }
    std::unique_ptr<Engine> e(new Engine());
    e->s = this;
    e->h = h;
    e->key = key;
    e->bytes = est;
    e->slots = n;
    const Field& f = fields[(size_t)q->r.field];
    e->per = (int64_t)q->r.Ls * ((int64_t)f.dims[0] * f.dims[1] * f.dims[2] * f.dims[3] / 2) * 24;
    used += est;
    peak = std::max(peak, used);
    Engine* ep = e.get();
    engines.push_back(std::move(e));
    ep->th = std::thread([ep] { ep->run(); });
    return ep;
  }

  // admit waiting requests in arrival order while slots and memory allow
  void dispatch() {
    while (!waiting.empty()) {
      Req* q = waiting.front();
      mspcg_status st = MSPCG_OK;
      std::string err;
      if (mode == 1) {
        Engine* e = engine_for(q, st, err);
        if (!e) {
          if (st == MSPCG_OK) break;   // wait for memory or an engine to go idle
          waiting.pop_front();
          complete(q, st, err);
          continue;
        }
        waiting.pop_front();
        q->remaining = q->r.nrhs;
        for (int i = 0; i < q->r.nrhs; ++i) e->queue.push_back(Job{q, i});
        e->last_use = ++tick;
        ++inflight;
        peak_inflight = std::max(peak_inflight, inflight);
        e->cv.notify_all();
        continue;
      }
      if (inflight >= max_inflight) break;
      Ctx* c = context_for(q, st, err);
      if (!c) {
        waiting.pop_front();
        complete(q, st, err);
        continue;
      }
      int64_t est = 0, alloc = 0;
      st = mspcg_set_solver(c->h, &q->r.solver);
      if (st == MSPCG_OK) st = mspcg_footprint(c->h, q->r.nrhs, &est, &alloc);
      if (st != MSPCG_OK) {
        waiting.pop_front();
        complete(q, st, mspcg_last_error());
        continue;
      }
      const int64_t need = std::max<int64_t>(0, est - c->bytes);
      while (used + need > budget && evict_one(c)) {
      }
      if (used + need > budget) {
        if (inflight == 0) {   // it does not fit even alone
          waiting.pop_front();
          complete(q, MSPCG_ERR_OOM, "request needs " + std::to_string(est) + " bytes beyond the resident fields; " +
                                         "the budget leaves " + std::to_string(budget - (used - c->bytes)));
          continue;
        }
        break;   // wait for running requests to free memory
      }
      used += need;
      c->bytes += need;
      peak = std::max(peak, used);
      c->busy = true;
      q->ctx = c;
      waiting.pop_front();
      ready.push_back(q);
      ++inflight;
      peak_inflight = std::max(peak_inflight, inflight);
      cv_work.notify_one();
    }
  }

  // join stopped engines (without the lock: they take it while stopping)
  void reap() {
    std::vector<std::unique_ptr<Engine>> r;
    {
      std::lock_guard<std::mutex> lk(mu);
      r.swap(retired);
    }
    for (auto& e : r)
      if (e->th.joinable()) e->th.join();
  }

  // ---------------------------------------------------------------- per-request workers
  void worker() {
    for (;;) {
      Req* q = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !ready.empty(); });
        if (ready.empty()) return;   // stop
        q = ready.front();
        ready.pop_front();
      }
      Ctx* c = q->ctx;
      mspcg_status st = mspcg_solve_batch_device(c->h, q->r.nrhs, q->r.src, q->r.x, nullptr, nullptr, q->st.data());
      std::string err;
      if (st != MSPCG_OK) err = mspcg_last_error();
      int64_t est = 0, alloc = 0;
      const bool have = mspcg_footprint(c->h, 1, &est, &alloc) == MSPCG_OK;
      std::lock_guard<std::mutex> lk(mu);
      if (have) {
        used += alloc - c->bytes;
        c->bytes = alloc;
      }
      c->busy = false;
      c->last_use = ++tick;
      --inflight;
      complete(q, st, err);
      dispatch();
    }
  }
};

namespace {

// status of a request from those of its right-hand sides
mspcg_status merge_status(mspcg_status a, mspcg_status b) {
  if (a == MSPCG_ERR_BREAKDOWN || b == MSPCG_ERR_BREAKDOWN) return MSPCG_ERR_BREAKDOWN;
  if (a < 0) return a;
  if (b < 0) return b;
  if (a == MSPCG_NOT_CONVERGED || b == MSPCG_NOT_CONVERGED) return MSPCG_NOT_CONVERGED;
  return MSPCG_OK;
}

// The engine's thread: move queued right-hand sides into free slots, run a
// step (joins, one iteration pair, finished slots write x), hand finished
// right-hand sides back to their requests.  Only this thread uses the handle.
void Engine::run() {
  mspcg_server& S = *s;
  std::vector<Job> slot_job((size_t)slots);
  for (;;) {
    std::vector<Job> take;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || in_slots > 0; });
      if (stop && idle()) break;
      int free_slots = slots - in_slots;
      while (free_slots > 0 && !queue.empty()) {
        take.push_back(queue.front());
        queue.pop_front();
        --free_slots;
        ++in_slots;
      }
    }
    std::vector<std::pair<Job, mspcg_status>> failed;
    std::string err;
    for (const Job& j : take) {
      int32_t slot = -1;
      const mspcg_status st = mspcg_cb_submit(h, j.q->r.src + (int64_t)j.i * per, j.q->r.x + (int64_t)j.i * per, &slot);
      if (st != MSPCG_OK || slot < 0) {
        err = mspcg_last_error();
        failed.push_back({j, st == MSPCG_OK ? MSPCG_ERR_HIP : st});
      } else {
        slot_job[(size_t)slot] = j;
      }
    }
    int32_t running = 0, pending = 0;
    mspcg_status st = mspcg_cb_step(h, &running, &pending);
    std::vector<std::pair<Job, mspcg_stats>> finished;
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      for (int i = 0; i < slots; ++i)
        if (slot_job[(size_t)i].q) {
          failed.push_back({slot_job[(size_t)i], st});
          slot_job[(size_t)i] = Job();
        }
      (void)mspcg_cb_close(h);              // start over with an empty session
      (void)mspcg_cb_open(h, slots, nullptr);
    } else {
      for (int i = 0; i < slots; ++i) {
        if (!slot_job[(size_t)i].q) continue;
        int32_t done = 0;
        mspcg_stats sts;
        if (mspcg_cb_poll(h, i, &done, &sts) == MSPCG_OK && done) {
          finished.push_back({slot_job[(size_t)i], sts});
          slot_job[(size_t)i] = Job();
        }
      }
    }
    if (failed.empty() && finished.empty()) continue;
    std::lock_guard<std::mutex> lk(S.mu);
    auto retire_job = [&](const Job& j, const mspcg_stats& sts, mspcg_status js) {
      Req* q = j.q;
      q->st[(size_t)j.i] = sts;
      q->status = merge_status(q->status, js);   // the worst outcome of its right-hand sides
      if (js < 0 && js != MSPCG_ERR_BREAKDOWN && q->err.empty()) q->err = err;
      --in_slots;
      if (--q->remaining == 0) {
        --S.inflight;
        const mspcg_status qs = q->status;
        const std::string qe = q->err;
        S.complete(q, qs, qe);
      }
    };
    for (auto& jf : finished) retire_job(jf.first, jf.second, (mspcg_status)jf.second.status);
    for (auto& jf : failed) {
      mspcg_stats z;
      std::memset(&z, 0, sizeof(z));
      z.status = jf.second;
      retire_job(jf.first, z, jf.second);
    }
    last_use = ++S.tick;
    if (idle()) S.dispatch();   // an idle engine may make room for waiting shapes
  }
  (void)mspcg_cb_close(h);
  (void)mspcg_destroy(h);
  h = nullptr;
}

template <typename F> mspcg_status srv_guard(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    mspcg::set_last_error("host allocation failed");
    return MSPCG_ERR_OOM;
  } catch (const std::exception& e) {
    mspcg::set_last_error(e.what());
    return MSPCG_ERR_HIP;
  }
}

mspcg_status fail(mspcg_status st, const char* msg) {
  mspcg::set_last_error(msg);
  return st;
}

}  // namespace

extern "C" {

mspcg_status mspcg_server_create(mspcg_server_t* out, int32_t device, int64_t hbm_budget, int32_t max_inflight) {
  return srv_guard([&]() -> mspcg_status {
    if (!out) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (device < 0 || hbm_budget <= 0 || max_inflight < 1 || max_inflight > 64)
      return fail(MSPCG_ERR_INVALID_ARG, "device >= 0, budget > 0 and 1 <= max_inflight <= 64 required");
    std::unique_ptr<mspcg_server> s(new mspcg_server());
    s->device = device;
    s->budget = hbm_budget;
    s->max_inflight = max_inflight;
    mspcg_server* p = s.get();
    for (int i = 0; i < max_inflight; ++i) s->workers.emplace_back([p] { p->worker(); });
    *out = s.release();
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_destroy(mspcg_server_t s) {
  return srv_guard([&]() -> mspcg_status {
    if (!s) return MSPCG_OK;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait(lk, [&] { return s->waiting.empty() && s->ready.empty() && s->inflight == 0; });
      s->stop = true;
      for (auto& e : s->engines) {
        e->stop = true;
        e->cv.notify_all();
        s->retired.push_back(std::move(e));
      }
      s->engines.clear();
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    s->reap();
    s->ctxs.clear();
    for (auto& f : s->fields) (void)mspcg_destroy(f.h);
    delete s;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_add_field(mspcg_server_t s, const int32_t dims[4], const double* U, int32_t* field) {
  return srv_guard([&]() -> mspcg_status {
    if (!s || !dims || !U || !field) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    Field f;
    for (int m = 0; m < 4; ++m) f.dims[m] = dims[m];
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    f.bytes = V * 4 * 10 * (16 + 8 + 4);   // FP64, FP32 and FP16 link layouts (9 entries padded to 10)
    std::lock_guard<std::mutex> lk(s->mu);
    while (s->used + f.bytes > s->budget && s->evict_one(nullptr)) {
    }
    if (s->used + f.bytes > s->budget) return fail(MSPCG_ERR_OOM, "gauge field does not fit the HBM budget");
    mspcg_status st = mspcg_create(&f.h, f.dims, s->device);
    if (st == MSPCG_OK) st = mspcg_load_gauge(f.h, U);
    if (st != MSPCG_OK) {
      const std::string err = mspcg_last_error();
      if (f.h) (void)mspcg_destroy(f.h);
      return fail(st, err.c_str());
    }
    s->used += f.bytes;
    s->peak = std::max(s->peak, s->used);
    s->fields.push_back(f);
    *field = (int32_t)s->fields.size() - 1;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_submit(mspcg_server_t s, const mspcg_request* r, int64_t* ticket) {
  return srv_guard([&]() -> mspcg_status {
    if (!s || !r || !ticket || !r->src || !r->x) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    if (r->nrhs < 1 || r->nrhs > 1024) return fail(MSPCG_ERR_INVALID_ARG, "nrhs must be in [1, 1024]");
    s->reap();
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->field < 0 || (size_t)r->field >= s->fields.size()) return fail(MSPCG_ERR_INVALID_ARG, "unknown field");
    std::unique_ptr<Req> q(new Req());
    q->r = *r;
    q->st.resize((size_t)r->nrhs);
    q->t_submit = now_ms();
    const int64_t t = s->next_ticket++;
    Req* qp = q.get();
    s->reqs[t] = std::move(q);
    s->waiting.push_back(qp);
    s->dispatch();
    *ticket = t;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_poll(mspcg_server_t s, int64_t ticket, int32_t* done) {
  return srv_guard([&]() -> mspcg_status {
    if (!s || !done) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MSPCG_ERR_INVALID_ARG, "unknown ticket");
    *done = it->second->done ? 1 : 0;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_wait(mspcg_server_t s, int64_t ticket, mspcg_stats* st, double* latency_ms) {
  return srv_guard([&]() -> mspcg_status {
    if (!s) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(MSPCG_ERR_INVALID_ARG, "unknown ticket");
    Req* q = it->second.get();
    s->cv_done.wait(lk, [&] { return q->done; });
    if (st) std::memcpy(st, q->st.data(), q->st.size() * sizeof(mspcg_stats));
    if (latency_ms) *latency_ms = q->t_end - q->t_submit;
    const mspcg_status r = q->status;
    const std::string err = q->err;
    s->reqs.erase(it);
    lk.unlock();
    s->reap();
    if (r != MSPCG_OK) mspcg::set_last_error(err.c_str());
    return r;
  });
}

mspcg_status mspcg_server_set_graphs(mspcg_server_t s, int32_t on) {
  return srv_guard([&]() -> mspcg_status {
    if (!s) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->engines.empty()) return fail(MSPCG_ERR_INVALID_ARG, "engines are running; set graphs before the first request");
    s->graphs = on != 0 ? 1 : 0;
    for (auto& c : s->ctxs) (void)mspcg_set_graphs(c->h, s->graphs);
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_set_mode(mspcg_server_t s, int32_t mode, int32_t slots) {
  return srv_guard([&]() -> mspcg_status {
    if (!s) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    if ((mode != 0 && mode != 1) || slots < 1 || slots > 1024)
      return fail(MSPCG_ERR_INVALID_ARG, "mode 0 or 1 and 1 <= slots <= 1024 required");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->inflight > 0 || !s->waiting.empty()) return fail(MSPCG_ERR_INVALID_ARG, "requests are in flight");
    for (auto& e : s->engines) {   // idle engines of the old setting go
      s->used -= e->bytes;
      e->stop = true;
      e->cv.notify_all();
      s->retired.push_back(std::move(e));
    }
    s->engines.clear();
    s->mode = mode;
    s->slots = slots;
    return MSPCG_OK;
  });
}

mspcg_status mspcg_server_info(mspcg_server_t s, mspcg_server_stats* info) {
  return srv_guard([&]() -> mspcg_status {
    if (!s || !info) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    info->budget = s->budget;
    info->bytes_in_use = s->used;
    info->bytes_peak = s->peak;
    info->inflight = s->inflight;
    info->waiting = (int32_t)s->waiting.size();
    info->peak_inflight = s->peak_inflight;
    info->contexts = (int32_t)(s->ctxs.size() + s->engines.size());
    info->completed = s->completed;
    info->evictions = s->evictions;
    return MSPCG_OK;
  });
}

}  // extern "C"
