// Serving loop: media stay resident after their setup phase; a worker thread
// admits solve requests by HBM budget and advances every right-hand side in
// flight through the batch engine (continuous batching, one engine and one
// stream per model family so that 2D and 3D work overlaps on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "mcmg.h"
#include "runtime.h"

using namespace mcmg;

namespace {

using Clock = std::chrono::steady_clock;

double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

struct Medium {
  Ctx* c = nullptr;
  size_t base_bytes = 0;                    // handle bytes (includes its own workspace)
  size_t slot_bytes = 0;                    // one extra workspace
  Slot own;                                 // the handle's own workspace
  std::vector<Slot*> idle;                  // workspaces not in use
  std::vector<std::unique_ptr<Slot>> extra; // allocated extra workspaces
  int engine = -1;
};

struct Request {
  uint64_t id = 0;
  int medium = 0, nrhs = 0, maxit = 0;
  double tol = 0;
  std::vector<const double*> f;
  std::vector<double*> u;
  Clock::time_point t_submit, t_admit;
  std::vector<Work> works;
  int remaining = 0;
  mcmg_completion comp{};
};

}  // namespace

struct mcmg_server_s {
  mcmg_server_opts opts{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  // shared with callers (guarded by mu)
  std::vector<std::unique_ptr<Medium>> media;
  std::deque<std::unique_ptr<Request>> queue;
  std::deque<mcmg_completion> done;
  size_t bytes_media = 0, bytes_slots = 0, bytes_peak = 0;
  int n_slots = 0, inflight = 0, inflight_peak = 0, queued = 0, completed = 0;
  long long ticks = 0, rebuilds = 0;
  bool stop = false;
  mcmg_status err = MCMG_OK;
  std::string err_msg;
  uint64_t next_id = 1;
  // worker only
  std::deque<std::unique_ptr<Request>> pending;
  std::vector<std::unique_ptr<Request>> active;
  std::vector<std::unique_ptr<Engine>> engines;
  std::thread worker;

  void note_bytes() {
    bytes_peak = std::max(bytes_peak, bytes_media + bytes_slots);
  }
  void run();
  mcmg_status admit();
  mcmg_status tick();
  void fail_all(mcmg_status st);
};

namespace {

// Releases one idle extra workspace of any medium other than `keep`.
bool release_one(mcmg_server_s* S, int keep) {
  std::vector<Medium*> ms;
  {
    std::lock_guard<std::mutex> g(S->mu);   // callers may append media meanwhile
    for (auto& m : S->media) ms.push_back(m.get());
  }
  for (size_t i = 0; i < ms.size(); ++i) {
    if ((int)i == keep) continue;
    Medium& M = *ms[i];
    for (size_t k = 0; k < M.idle.size(); ++k) {
      Slot* sl = M.idle[k];
      if (sl == &M.own) continue;
      M.idle.erase(M.idle.begin() + k);
      const size_t b = sl->bytes;
      M.c->free_slot(*sl);
      for (size_t q = 0; q < M.extra.size(); ++q)
        if (M.extra[q].get() == sl) { M.extra.erase(M.extra.begin() + q); break; }
      std::lock_guard<std::mutex> g(S->mu);
      S->bytes_slots -= b;
      S->n_slots--;
      return true;
    }
  }
  return false;
}

}  // namespace

mcmg_status mcmg_server_s::admit() {
  while (!pending.empty()) {
    Request& R = *pending.front();
    Medium* M;
    {
      std::lock_guard<std::mutex> g(mu);
      M = media[R.medium].get();
    }
    int now_inflight;
    {
      std::lock_guard<std::mutex> g(mu);
      now_inflight = inflight;
    }
    if (opts.max_inflight > 0 && now_inflight + R.nrhs > opts.max_inflight) break;
    const int need = R.nrhs - (int)M->idle.size();
    if (need > 0) {
      const size_t bytes = (size_t)need * M->slot_bytes;
      bool fits;
      while (true) {
        {
          std::lock_guard<std::mutex> g(mu);
          fits = bytes_media + bytes_slots + bytes <= opts.hbm_budget;
        }
        if (fits || !release_one(this, R.medium)) break;
      }
      if (!fits) break;   // wait for in-flight work to finish
      for (int k = 0; k < need; ++k) {
        auto sl = std::make_unique<Slot>();
        mcmg_status st = M->c->alloc_slot(*sl);
        if (st != MCMG_OK) {
          if (now_inflight > 0) return MCMG_OK;   // retry once memory frees up
          return st;
        }
        {
          std::lock_guard<std::mutex> g(mu);
          bytes_slots += sl->bytes;
          n_slots++;
          note_bytes();
        }
        M->idle.push_back(sl.get());
        M->extra.push_back(std::move(sl));
      }
    }
    if (M->engine < 0) {
      for (size_t e = 0; e < engines.size() && M->engine < 0; ++e)
        if (engines[e]->compatible(M->c, nullptr)) M->engine = (int)e;
      if (M->engine < 0) {
        auto eng = std::make_unique<Engine>();
        eng->use_graphs = opts.graphs != 0;
        mcmg_status st = eng->open(M->c);
        if (st != MCMG_OK) return st;
        engines.push_back(std::move(eng));
        M->engine = (int)engines.size() - 1;
      }
    }
    Engine& E = *engines[M->engine];
    R.works.resize(R.nrhs);
    for (int i = 0; i < R.nrhs; ++i) {
      Work& w = R.works[i];
      w.c = M->c;
      w.slot = M->idle.back();
      M->idle.pop_back();
      w.f = R.f[i];
      w.u = R.u[i];
      w.tol = R.tol;
      w.maxit = R.maxit;
      w.tag = (uint64_t)(uintptr_t)&R;
      mcmg_status st = E.add(&w);
      if (st != MCMG_OK) return st;
    }
    R.remaining = R.nrhs;
    R.t_admit = Clock::now();
    R.comp.req_id = R.id;
    R.comp.nrhs = R.nrhs;
    R.comp.status = MCMG_OK;
    R.comp.queue_s = secs(R.t_submit, R.t_admit);
    {
      std::lock_guard<std::mutex> g(mu);
      inflight += R.nrhs;
      inflight_peak = std::max(inflight_peak, inflight);
      queued--;
    }
    active.push_back(std::move(pending.front()));
    pending.pop_front();
  }
  return MCMG_OK;
}

mcmg_status mcmg_server_s::tick() {
  std::vector<Engine*> go;
  for (auto& e : engines)
    if (e->live() > 0) go.push_back(e.get());
  for (Engine* e : go) {
    mcmg_status st = e->issue();
    if (st != MCMG_OK) return st;
  }
  std::vector<Work*> fin;
  for (Engine* e : go) {
    mcmg_status st = e->complete(&fin);
    if (st != MCMG_OK) return st;
  }
  const Clock::time_point now = Clock::now();
  std::vector<mcmg_completion> out;
  for (Work* w : fin) {
    Request& R = *(Request*)(uintptr_t)w->tag;
    Medium* M;
    {
      std::lock_guard<std::mutex> g(mu);
      M = media[R.medium].get();
    }
    M->idle.push_back(w->slot);
    R.comp.iters_total += w->its;
    R.comp.iters_max = std::max(R.comp.iters_max, w->its);
    R.comp.relres_max = std::max(R.comp.relres_max, w->relres);
    if (w->status < 0 && R.comp.status >= 0) R.comp.status = w->status;
    else if (R.comp.status >= 0 && w->status > R.comp.status) R.comp.status = w->status;
    if (--R.remaining == 0) {
      R.comp.latency_s = secs(R.t_submit, now);
      out.push_back(R.comp);
    }
  }
  for (Engine* e : go) e->drop_done();
  if (!fin.empty())
    active.erase(std::remove_if(active.begin(), active.end(),
                                [](const std::unique_ptr<Request>& r) { return r->remaining == 0; }),
                 active.end());
  std::lock_guard<std::mutex> g(mu);
  ticks += (long long)go.size();
  rebuilds = 0;
  for (auto& e : engines) rebuilds += e->rebuilds;
  inflight -= (int)fin.size();
  for (auto& c : out) done.push_back(c);
  completed += (int)out.size();
  if (!out.empty()) cv_done.notify_all();
  return MCMG_OK;
}

void mcmg_server_s::fail_all(mcmg_status st) {
  std::lock_guard<std::mutex> g(mu);
  err = st;
  err_msg = mcmg_last_error();
  const Clock::time_point now = Clock::now();
  auto drain = [&](std::unique_ptr<Request>& r) {
    mcmg_completion c = r->comp;
    c.req_id = r->id;
    c.nrhs = r->nrhs;
    c.status = st;
    c.latency_s = secs(r->t_submit, now);
    done.push_back(c);
  };
  for (auto& r : active) drain(r);
  for (auto& r : pending) drain(r);
  for (auto& r : queue) drain(r);
  queue.clear();
  cv_done.notify_all();
}

void mcmg_server_s::run() {
  (void)hipSetDevice(device);
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      auto idle = [&] {
        if (stop) return false;
        if (!queue.empty()) return false;
        for (auto& e : engines)
          if (e->live() > 0) return false;
        return true;
      };
      // nothing in flight and nothing new: sleep until a submit or stop
      while (idle() && pending.empty()) cv_work.wait(lk);
      if (stop) return;
      while (!queue.empty()) {
        pending.push_back(std::move(queue.front()));
        queue.pop_front();
      }
    }
    mcmg_status st = admit();
    if (st == MCMG_OK) {
      bool any = false;
      for (auto& e : engines) any |= e->live() > 0;
      if (any) {
        st = tick();
      } else if (!pending.empty()) {
        // nothing in flight and the head request still does not fit (media
        // added after it was queued): it completes alone with E_BUDGET
        std::unique_ptr<Request> r = std::move(pending.front());
        pending.pop_front();
        mcmg_completion c{};
        c.req_id = r->id;
        c.nrhs = r->nrhs;
        c.status = MCMG_E_BUDGET;
        c.latency_s = secs(r->t_submit, Clock::now());
        std::lock_guard<std::mutex> g(mu);
        queued--;
        done.push_back(c);
        completed++;
        cv_done.notify_all();
      }
    }
    if (st != MCMG_OK) {
      fail_all(st);
      std::unique_lock<std::mutex> lk(mu);
      while (!stop) cv_work.wait(lk);
      return;
    }
  }
}

extern "C" {

mcmg_status mcmg_server_create(const mcmg_server_opts* opts, mcmg_server* out) {
  if (!opts || !out) return fail(MCMG_E_ARG, "null argument");
  if (opts->hbm_budget == 0) return fail(MCMG_E_ARG, "zero HBM budget");
  if (opts->max_inflight < 0) return fail(MCMG_E_ARG, "negative max_inflight");
  auto S = std::make_unique<mcmg_server_s>();
  S->opts = *opts;
  if (hipGetDevice(&S->device) != hipSuccess) return fail(MCMG_E_HIP, "no device");
  mcmg_server_s* p = S.get();
  try {
    S->worker = std::thread([p] { p->run(); });
  } catch (...) {
    return fail(MCMG_E_ARG, "worker thread creation failed");
  }
  *out = S.release();
  return MCMG_OK;
}

mcmg_status mcmg_server_add_handle(mcmg_server s, mcmg_handle h, int* medium_id) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  if (!s || !medium_id) { mcmg_destroy(h); return fail(MCMG_E_ARG, "null argument"); }
  Ctx* c = (Ctx*)h;
  if (hipStreamSynchronize(c->stream) != hipSuccess) { mcmg_destroy(h); return fail(MCMG_E_HIP, "stream sync"); }
  auto M = std::make_unique<Medium>();
  M->c = c;
  M->base_bytes = mcmg_device_bytes(h);
  M->slot_bytes = c->slot_bytes();
  M->own = c->current_slot();
  M->idle.push_back(&M->own);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->bytes_media + s->bytes_slots + M->base_bytes > s->opts.hbm_budget) {
    mcmg_destroy(h);
    return fail(MCMG_E_BUDGET, "medium (%zu bytes) does not fit the HBM budget", M->base_bytes);
  }
  s->bytes_media += M->base_bytes;
  s->note_bytes();
  s->media.push_back(std::move(M));
  *medium_id = (int)s->media.size() - 1;
  return MCMG_OK;
}

mcmg_status mcmg_server_add_medium(mcmg_server s, const double* c, mcmg_grid grid, double omega,
                                   double h, mcmg_pml pml, mcmg_weights w, const mcmg_opts* opt,
                                   int* medium_id) {
  if (!s || !medium_id) return fail(MCMG_E_ARG, "null argument");
  mcmg_opts o{};
  if (opt) o = *opt;
  o.stream = nullptr;
  mcmg_handle hd = nullptr;
  mcmg_status st = mcmg_setup(c, grid, omega, h, pml, w, &o, &hd);
  if (st != MCMG_OK) return st;
  return mcmg_server_add_handle(s, hd, medium_id);
}

mcmg_status mcmg_server_submit(mcmg_server s, int medium_id, const double* const* f,
                               double* const* u, int nrhs, double tol, int maxit,
                               uint64_t* req_id) {
  if (!s || !f || !u || !req_id) return fail(MCMG_E_ARG, "null argument");
  if (nrhs < 1) return fail(MCMG_E_ARG, "nrhs must be >= 1");
  if (!(tol > 0) || maxit < 0) return fail(MCMG_E_ARG, "bad tol/maxit");
  for (int i = 0; i < nrhs; ++i)
    if (!f[i] || !u[i]) return fail(MCMG_E_ARG, "null f/u %d", i);
  auto R = std::make_unique<Request>();
  R->medium = medium_id;
  R->nrhs = nrhs;
  R->tol = tol;
  R->maxit = maxit;
  R->f.assign(f, f + nrhs);
  R->u.assign(u, u + nrhs);
  std::lock_guard<std::mutex> g(s->mu);
  if (s->err != MCMG_OK) return fail(s->err, "server stopped: %s", s->err_msg.c_str());
  if (medium_id < 0 || medium_id >= (int)s->media.size()) return fail(MCMG_E_ARG, "unknown medium %d", medium_id);
  const Medium& M = *s->media[medium_id];
  if (s->opts.max_inflight > 0 && nrhs > s->opts.max_inflight)
    return fail(MCMG_E_BUDGET, "nrhs %d exceeds max_inflight %d", nrhs, s->opts.max_inflight);
  if (s->bytes_media + (size_t)(nrhs - 1) * M.slot_bytes > s->opts.hbm_budget)
    return fail(MCMG_E_BUDGET, "request of %d rhs can never fit the HBM budget", nrhs);
  R->id = s->next_id++;
  R->t_submit = Clock::now();
  *req_id = R->id;
  s->queued++;
  s->queue.push_back(std::move(R));
  s->cv_work.notify_one();
  return MCMG_OK;
}

mcmg_status mcmg_server_poll(mcmg_server s, mcmg_completion* out, int max, int* n, int wait_ms) {
  if (!s || !n || (max > 0 && !out)) return fail(MCMG_E_ARG, "null argument");
  *n = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0 && s->err == MCMG_OK)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty() || s->err != MCMG_OK; });
  while (*n < max && !s->done.empty()) {
    out[(*n)++] = s->done.front();
    s->done.pop_front();
  }
  if (s->err != MCMG_OK) return fail(s->err, "server stopped: %s", s->err_msg.c_str());
  return MCMG_OK;
}

mcmg_status mcmg_server_get_stats(mcmg_server s, mcmg_server_stats* out) {
  if (!s || !out) return fail(MCMG_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  out->bytes_in_use = s->bytes_media + s->bytes_slots;
  out->bytes_peak = s->bytes_peak;
  out->media = (int)s->media.size();
  out->slots = s->n_slots;
  out->inflight = s->inflight;
  out->queued = s->queued;
  out->completed = s->completed;
  out->inflight_peak = s->inflight_peak;
  out->ticks = s->ticks;
  out->rebuilds = s->rebuilds;
  return MCMG_OK;
}

void mcmg_server_destroy(mcmg_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->engines.clear();   // synchronises their streams
  for (auto& M : s->media) {
    for (auto& sl : M->extra) M->c->free_slot(*sl);
    mcmg_destroy((mcmg_handle)M->c);
  }
  delete s;
}

}  // extern "C"
