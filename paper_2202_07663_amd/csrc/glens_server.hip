// Continuous-batching fit server: gl_server_create / gl_submit / gl_poll / gl_server_destroy.
//
// Requests (one lens system + fit options each) wait in a FIFO queue. A scheduler thread
// owns one HIP stream and loops over ticks:
//   1. admit queued requests (FIFO) while an active slot is free and the device memory of
//      the request (inputs, work space, fit state) fits in the HBM budget;
//   2. advance every active system by up to steps_per_tick Adam steps; systems with the
//      same kernel configuration (mass model, shapelet order, PSF size) share one launch
//      per kernel, so work of systems that arrived at different times overlaps on the GPU;
//   3. retire systems that reached their step budget: evaluate log L, pick the best
//      particle, record the result with its timestamps, free its memory.
// Admission also keeps the active systems' sub-pixel work per step near what fills the GPU
// (fill_subpixels): large systems then run close to first-come-first-served, which keeps
// latency low, while small systems are batched into shared launches.
// A system's arithmetic (work split, summation orders, random starts) depends only on its
// own request, so its result is the same whether it runs alone or in a mix.
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "glens_fit.h"
#include "glens_host.h"

namespace glens {

static uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return uint64_t(ts.tv_sec) * 1000000000ull + uint64_t(ts.tv_nsec);
}

struct Request {
  uint64_t ticket = 0;
  ModelCfg cfg;
  std::vector<float> psf, obs;
  gl_model_desc desc;  // host pointers re-pointed at psf / obs
  FitParams fp;
  std::vector<Prior> priors;
  size_t bytes = 0;
  double work = 0.0;  // sub-pixel evaluations per step
  uint64_t t_submit = 0;
};

struct Active {
  std::unique_ptr<Request> req;
  SystemData sys;
  Workspace ws;
  FitBuffers fb;
  int tiles = 1;
  uint64_t t_admit = 0;
  int failed = GL_OK;  // first error of a launch on this system; it then retires with it
};

static double request_work(const ModelCfg& c, int P) {
  return double(P) * c.H * c.W * c.k * c.k;
}

static size_t request_bytes(const ModelCfg& c, int P) {
  const int HW = c.H * c.W;
  const size_t psf_tab = c.K <= kMfmaMaxK ? size_t(2) * c.K * 64 * 16 * sizeof(uint16_t) : 0;
  return sizeof(float) * (2 * c.K * c.K + HW) + psf_tab +
         workspace_bytes(P, acc_rows_upto(P, HW), HW, c.d, true, beta_per_particle(c)) +
         fit_buffers_bytes(P, c.d);
}

}  // namespace glens

using namespace glens;

struct gl_server {
  gl_server_opts opts;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::unique_ptr<Request>> queue;
  std::map<uint64_t, gl_fit_result> done;
  std::map<uint64_t, int> pending;  // ticket -> 1 while queued or active
  uint64_t next_ticket = 1;
  bool closing = false;
  std::thread th;
  hipStream_t stream = nullptr;
  // stats (guarded by mu)
  gl_server_stats st{};
  std::vector<std::unique_ptr<Active>> active;  // scheduler thread only
  double active_work = 0.0;                      // scheduler thread only
};

static void finish(gl_server* s, Active& a, const gl_fit_result& r) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->done[a.req->ticket] = r;
  s->pending.erase(a.req->ticket);
  s->st.completed++;
  s->st.hbm_in_use -= a.req->bytes;
  if (r.status != GL_OK) {
    s->st.failed++;
    s->st.last_error = r.status;
  }
}

static gl_fit_result error_result(const Active& a, int rc) {
  gl_fit_result r;
  std::memset(&r, 0, sizeof(r));
  r.status = rc;
  r.d = a.req->cfg.d;
  r.best = -1;
  r.t_submit = a.req->t_submit;
  r.t_admit = a.t_admit;
  r.t_done = now_ns();
  return r;
}

static void release(Active& a) {
  fit_buffers_free(a.fb);
  workspace_free(a.ws);
  system_free(a.sys);
}

static int admit(gl_server* s, std::unique_ptr<Request> rq) {
  auto a = std::make_unique<Active>();
  a->t_admit = now_ns();
  const ModelCfg& c = rq->cfg;
  const int HW = c.H * c.W;
  a->tiles = choose_tiles(rq->fp.P, HW);
  int rc = system_upload(&rq->desc, c, a->sys);
  if (!rc) rc = workspace_reserve(a->ws, rq->fp.P, a->tiles, HW, c.d, true, beta_per_particle(c));
  if (!rc) rc = fit_buffers_alloc(a->fb, rq->fp.P, c.d, rq->priors.data());
  a->req = std::move(rq);
  if (!rc) {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.nsys = 1;
    g.sys[0] = make_sys(a->sys, a->ws, a->req->fp.P, a->tiles);
    attach_fit(g.sys[0], a->fb, a->req->fp, a->ws);
    rc = launch_fit_init(g, s->stream);
  }
  if (rc) {  // retired at once with the error; the stream has no work of it in flight
    s->active_work -= a->req->work;
    if (hipStreamSynchronize(s->stream) != hipSuccess) rc = GL_E_DEVICE;
    const gl_fit_result r = error_result(*a, rc);
    release(*a);
    finish(s, *a, r);
    return rc;
  }
  s->active.push_back(std::move(a));
  return GL_OK;
}

// Systems grouped by kernel configuration; each group runs `mode` and, for mode 2, Adam. A
// group whose launches fail marks its systems (they retire with the error at the end of the
// tick); the other groups go on.
static int run_grouped(gl_server* s, std::vector<Active*>& sys, int mode) {
  int first_rc = GL_OK;
  std::map<std::pair<int, int>, std::vector<Active*>> by_key;
  for (Active* a : sys) by_key[{subpix_key(a->req->cfg), a->req->cfg.K}].push_back(a);
  for (auto& kv : by_key) {
    auto& list = kv.second;
    for (size_t i0 = 0; i0 < list.size(); i0 += kMaxGroup) {
      Group g;
      std::memset(&g, 0, sizeof(g));
      g.nsys = int(std::min<size_t>(kMaxGroup, list.size() - i0));
      for (int i = 0; i < g.nsys; ++i) {
        Active* a = list[i0 + i];
        g.sys[i] = make_sys(a->sys, a->ws, a->req->fp.P, a->tiles);
        attach_fit(g.sys[i], a->fb, a->req->fp, a->ws);
      }
      int rc = run_group(g, kv.first.first, kv.first.second, mode, s->stream);
      if (!rc && mode == 2) rc = launch_adam(g, s->stream);
      if (!rc && mode == 1) rc = launch_logpost(g, s->stream);
      if (rc) {
        for (int i = 0; i < g.nsys; ++i)
          if (list[i0 + i]->failed == GL_OK) list[i0 + i]->failed = rc;
        if (first_rc == GL_OK) first_rc = rc;
      }
    }
  }
  return first_rc;
}

static void tick(gl_server* s) {
  // 1. admission
  while (true) {
    std::unique_ptr<Request> rq;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty() || int(s->active.size()) >= s->opts.max_systems) break;
      if (s->st.hbm_in_use + s->queue.front()->bytes > s->opts.hbm_budget_bytes) break;
      if (!s->active.empty() && s->active_work + s->queue.front()->work > s->opts.fill_subpixels)
        break;
      rq = std::move(s->queue.front());
      s->queue.pop_front();
      s->st.hbm_in_use += rq->bytes;
      s->st.hbm_peak = std::max(s->st.hbm_peak, s->st.hbm_in_use);
      s->st.admitted++;
      s->st.queued = int(s->queue.size());
    }
    s->active_work += rq->work;
    admit(s, std::move(rq));  // a failure retires the request with its status
  }
  if (s->active.empty()) return;
  // 2. advance every active system by up to steps_per_tick steps
  for (int k = 0; k < s->opts.steps_per_tick; ++k) {
    std::vector<Active*> run;
    for (auto& a : s->active)
      if (a->failed == GL_OK && a->req->fp.step < a->req->fp.K) run.push_back(a.get());
    if (run.empty()) break;
    run_grouped(s, run, 2);
    for (Active* a : run)
      if (a->failed == GL_OK) a->req->fp.step++;
  }
  // 3. retire finished and failed systems
  auto done = [](const Active& a) { return a.failed != GL_OK || a.req->fp.step >= a.req->fp.K; };
  std::vector<Active*> fin;
  for (auto& a : s->active)
    if (a->failed == GL_OK && a->req->fp.step >= a->req->fp.K) fin.push_back(a.get());
  if (!fin.empty()) run_grouped(s, fin, 1);
  if (hipStreamSynchronize(s->stream) != hipSuccess) {
    (void)hipGetLastError();
    for (auto& a : s->active)
      if (a->failed == GL_OK) a->failed = GL_E_DEVICE;
  }
  for (auto& ap : s->active) {
    Active* a = ap.get();
    if (!done(*a)) continue;
    s->active_work -= a->req->work;
    gl_fit_result r;
    if (a->failed != GL_OK) {
      r = error_result(*a, a->failed);
    } else {
      std::memset(&r, 0, sizeof(r));
      int rc = fit_result_from_device(a->fb, a->ws, a->req->fp.P, a->req->cfg, s->stream, &r);
      if (rc) r.status = rc;
      r.t_submit = a->req->t_submit;
      r.t_admit = a->t_admit;
      r.t_done = now_ns();
    }
    release(*a);
    finish(s, *a, r);
  }
  s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                 [&](const std::unique_ptr<Active>& a) { return done(*a); }),
                  s->active.end());
  std::lock_guard<std::mutex> lk(s->mu);
  s->st.ticks++;
  s->st.active = int(s->active.size());
}

static void scheduler(gl_server* s) {
  (void)hipSetDevice(s->device);
  while (true) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->closing || !s->queue.empty() || !s->active.empty(); });
      if (s->closing && s->queue.empty() && s->active.empty()) break;
    }
    tick(s);
  }
}

extern "C" {

int gl_server_create(const gl_server_opts* o, gl_server** out) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!o) return set_error(GL_E_INVALID, "opts is NULL");
  if (o->max_systems < 1) return set_error(GL_E_INVALID, "max_systems must be >= 1");
  if (o->steps_per_tick < 1) return set_error(GL_E_INVALID, "steps_per_tick must be >= 1");
  if (o->hbm_budget_bytes == 0) return set_error(GL_E_INVALID, "hbm_budget_bytes must be > 0");
  gl_server* s = new (std::nothrow) gl_server();
  if (!s) return set_error(GL_E_NOMEM, "host allocation failed");
  s->opts = *o;
  if (!(s->opts.fill_subpixels > 0.0)) s->opts.fill_subpixels = 6e7;
  if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess) {
    delete s;
    return set_error(GL_E_DEVICE, "cannot create the server stream");
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return GL_OK;
}

int gl_server_destroy(gl_server* s) {
  clear_error();
  if (!s) return GL_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
  }
  s->cv.notify_all();
  s->th.join();
  (void)hipStreamDestroy(s->stream);
  delete s;
  return GL_OK;
}

int gl_submit(gl_server* s, const gl_model_desc* desc, const gl_fit_opts* o, uint64_t* ticket) {
  clear_error();
  if (!s || !ticket) return set_error(GL_E_INVALID, "NULL argument");
  auto rq = std::make_unique<Request>();
  int rc = validate_desc(desc, &rq->cfg);
  if (rc) return rc;
  if (!desc->obs) return set_error(GL_E_INVALID, "obs is NULL");
  if ((rc = validate_fit_opts(o, rq->cfg.d, rq->priors))) return rc;
  const ModelCfg& c = rq->cfg;
  rq->psf.assign(desc->psf, desc->psf + c.K * c.K);
  rq->obs.assign(desc->obs, desc->obs + c.H * c.W);
  rq->desc = *desc;
  rq->desc.psf = rq->psf.data();
  rq->desc.obs = rq->obs.data();
  rq->fp = fit_params(o);
  rq->bytes = request_bytes(c, o->P);
  rq->work = request_work(c, o->P);
  if (rq->bytes > s->opts.hbm_budget_bytes)
    return set_error(GL_E_BUDGET, "request needs %zu bytes, budget is %zu", rq->bytes,
                     s->opts.hbm_budget_bytes);
  rq->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) return set_error(GL_E_CLOSED, "server is shutting down");
    rq->ticket = s->next_ticket++;
    *ticket = rq->ticket;
    s->pending[rq->ticket] = 1;
    s->queue.push_back(std::move(rq));
    s->st.submitted++;
    s->st.queued = int(s->queue.size());
  }
  s->cv.notify_all();
  return GL_OK;
}

int gl_poll(gl_server* s, uint64_t ticket, gl_fit_result* out) {
  clear_error();
  if (!s || !out) return set_error(GL_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    *out = it->second;
    s->done.erase(it);
    return GL_OK;
  }
  if (s->pending.count(ticket)) return GL_PENDING;
  return set_error(GL_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
}

int gl_server_get_stats(gl_server* s, gl_server_stats* out) {
  clear_error();
  if (!s || !out) return set_error(GL_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return GL_OK;
}

}  // extern "C"
