// Request loop of the library (mspcg_server_*): resident gauge fields,
// resident solver contexts keyed by (field, Mobius parameters, tiling),
// admission in arrival order by device footprint, and one worker thread with
// its own HIP stream per request in flight, so that admitted requests run
// concurrently on the device.  Built on the public C ABI only.
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

// a resident solver context: one handle with its workspaces, sharing the
// gauge field of its field's handle
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
};

struct Field {
  mspcg_t h = nullptr;
  int32_t dims[4];
  int64_t bytes = 0;
};

std::string key_of(const mspcg_request& r) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%d|%d|%a|%a|%a|%a|%d,%d,%d,%d", r.field, r.Ls, r.b, r.c, r.M5, r.mf, r.sub[0],
                r.sub[1], r.sub[2], r.sub[3]);
  return buf;
}

}  // namespace

struct mspcg_server {
  int device = 0;
  int64_t budget = 0;
  int max_inflight = 1;
  // contexts launch eagerly unless enabled: while a capture is open, device-
  // wide synchronization by any other thread of the process fails, and the
  // caller's threads are not the server's to restrict
  int graphs = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Field> fields;
  std::list<std::unique_ptr<Ctx>> ctxs;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::deque<Req*> waiting;   // submitted, not admitted
  std::deque<Req*> ready;     // admitted, not yet picked up by a worker
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

  // free the least recently used idle context other than `keep`
  bool evict_one(const Ctx* keep) {
    auto victim = ctxs.end();
    for (auto it = ctxs.begin(); it != ctxs.end(); ++it) {
      const Ctx* c = it->get();
      if (c->busy || c == keep) continue;
      if (victim == ctxs.end() || c->last_use < (*victim)->last_use) victim = it;
    }
    if (victim == ctxs.end()) return false;
    used -= (*victim)->bytes;
    ctxs.erase(victim);
    ++evictions;
    return true;
  }

  // a context for the request's key: an idle resident one, else a new one
  Ctx* context_for(Req* q, mspcg_status& st, std::string& err) {
    const std::string key = key_of(q->r);
    Ctx* best = nullptr;
    for (auto& c : ctxs)
      if (!c->busy && c->key == key && (!best || c->bytes > best->bytes)) best = c.get();
    if (best) return best;
    const Field& f = fields[(size_t)q->r.field];
    std::unique_ptr<Ctx> c(new Ctx());
    c->key = key;
    st = mspcg_create(&c->h, f.dims, device);
    if (st == MSPCG_OK) st = mspcg_share_gauge(c->h, f.h);
    if (st == MSPCG_OK) st = mspcg_set_graphs(c->h, graphs);
    if (st == MSPCG_OK) st = mspcg_set_mobius(c->h, q->r.Ls, q->r.b, q->r.c, q->r.M5, q->r.mf);
    const bool tiled = q->r.sub[0] > 0 || q->r.sub[1] > 0 || q->r.sub[2] > 0 || q->r.sub[3] > 0;
    if (st == MSPCG_OK && tiled) st = mspcg_set_subdomains(c->h, q->r.sub);
    if (st != MSPCG_OK) {
      err = mspcg_last_error();
      return nullptr;
    }
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

  // admit waiting requests in arrival order while slots and memory allow
  void dispatch() {
    while (!waiting.empty() && inflight < max_inflight) {
      Req* q = waiting.front();
      mspcg_status st = MSPCG_OK;
      std::string err;
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

  // ---------------------------------------------------------------- workers
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
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
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
    if (r != MSPCG_OK) mspcg::set_last_error(err.c_str());
    return r;
  });
}

mspcg_status mspcg_server_set_graphs(mspcg_server_t s, int32_t on) {
  return srv_guard([&]() -> mspcg_status {
    if (!s) return fail(MSPCG_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs = on != 0 ? 1 : 0;
    for (auto& c : s->ctxs) (void)mspcg_set_graphs(c->h, s->graphs);
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
    info->contexts = (int32_t)s->ctxs.size();
    info->completed = s->completed;
    info->evictions = s->evictions;
    return MSPCG_OK;
  });
}

}  // extern "C"
