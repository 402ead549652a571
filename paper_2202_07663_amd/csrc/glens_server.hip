// Continuous-batching fit server: gl_server_create / gl_submit / gl_poll / gl_server_destroy.
//
// Requests (one lens system + fit options each) wait in a FIFO queue. A scheduler thread
// owns one HIP stream and keeps the GPU fed with ticks; it never waits on the stream as a
// whole:
//   1. admit queued requests (FIFO) while an active slot is free, the device memory of the
//      request (inputs, work space, fit state) fits in the HBM budget, and the active
//      systems' sub-pixel work per step stays near what fills the GPU (fill_subpixels).
//      Admission takes a device block from a pool of blocks released by finished systems
//      (device memory is allocated only when no cached block fits), writes the system's
//      inputs into pinned staging memory and enqueues their copy, then the start draws;
//   2. enqueue a tick: every running system advances by steps_per_tick Adam steps, systems
//      with the same kernel configuration (mass model, lens light, shapelet order, PSF size)
//      sharing one launch per kernel, so work of systems that arrived at different times
//      overlaps on the GPU; systems that reach their step budget then get their log L pass,
//      the best-particle selection on the device and an asynchronous copy of that result to
//      pinned host memory; an event marks the end of the tick;
//   3. reap finished ticks (event queries): their systems' results are recorded with their
//      timestamps and their blocks and staging go back to the pools. At most two ticks are
//      in flight: the host prepares tick t + 1 while the GPU runs tick t.
// A system's arithmetic (work split, summation orders, random starts) depends only on its
// own request, so its result is the same whether it runs alone or in a mix, and equal to
// gl_fit's on the same request.
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
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

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Device blocks cached across systems (scheduler thread only). Sizes are rounded up to
// sixteenths of the next power of two, so that requests of similar size reuse each other's
// blocks; a cached block serves a request of up to twice its class.
class DevicePool {
 public:
  static size_t size_class(size_t b) {
    size_t p = 1;
    while (p < b) p <<= 1;
    const size_t step = std::max<size_t>(p / 16, 256);
    return (b + step - 1) / step * step;
  }
  // A block of at least `bytes` (its size in *got), from the cache or hipMalloc.
  int take(size_t bytes, char** out, size_t* got) {
    const size_t cls = size_class(bytes);
    auto it = free_.lower_bound(cls);
    if (it != free_.end() && it->first <= 2 * cls) {
      *out = it->second;
      *got = it->first;
      cached_ -= it->first;
      free_.erase(it);
      return GL_OK;
    }
    char* p = nullptr;
    GL_HIP(hipMalloc(&p, cls));
    *out = p;
    *got = cls;
    return GL_OK;
  }
  void give(char* p, size_t bytes) {
    free_.emplace(bytes, p);
    cached_ += bytes;
  }
  size_t cached() const { return cached_; }
  // Free cached blocks, largest first, until at most `keep` bytes stay cached.
  void trim(size_t keep) {
    while (cached_ > keep && !free_.empty()) {
      auto it = std::prev(free_.end());
      (void)hipFree(it->second);
      cached_ -= it->first;
      free_.erase(it);
    }
  }
  ~DevicePool() { trim(0); }

 private:
  std::multimap<size_t, char*> free_;
  size_t cached_ = 0;
};

// Pinned host buffers for uploads (scheduler thread only), kept for reuse.
class PinnedPool {
 public:
  int take(size_t bytes, char** out, size_t* got) {
    const size_t cls = DevicePool::size_class(bytes);
    auto it = free_.lower_bound(cls);
    if (it != free_.end() && it->first <= 2 * cls) {
      *out = it->second;
      *got = it->first;
      free_.erase(it);
      return GL_OK;
    }
    void* p = nullptr;
    GL_HIP(hipHostMalloc(&p, cls, hipHostMallocDefault));
    *out = static_cast<char*>(p);
    *got = cls;
    return GL_OK;
  }
  void give(char* p, size_t bytes) { free_.emplace(bytes, p); }
  ~PinnedPool() {
    for (auto& kv : free_) (void)hipHostFree(kv.second);
  }

 private:
  std::multimap<size_t, char*> free_;
};

struct Request {
  uint64_t ticket = 0;
  ModelCfg cfg;
  std::vector<float> psf, obs;
  gl_model_desc desc;  // host pointers re-pointed at psf / obs
  FitParams fp;
  std::vector<Prior> priors;
  size_t bytes = 0;   // device block (pool size class)
  double work = 0.0;  // sub-pixel evaluations per step
  uint64_t t_submit = 0;
};

enum SysState { RUNNING, RETIRING };

struct Active {
  std::unique_ptr<Request> req;
  SystemData sys;
  Workspace ws;
  FitBuffers fb;
  FitOut* out_dev = nullptr;   // in the block
  FitOut* out_host = nullptr;  // pinned
  char* block = nullptr;
  size_t block_bytes = 0;
  int tiles = 1;
  uint64_t t_admit = 0;
  SysState state = RUNNING;
  bool done = false;
  int failed = GL_OK;  // first error of a launch on this system; it then retires with it
};

struct Staged {
  char* p;
  size_t bytes;
};

// One enqueued tick: its end event, the systems whose results it delivers, and the staging
// buffers whose copies it covers.
struct Tick {
  hipEvent_t ev = nullptr;
  std::vector<Active*> retiring;
  std::vector<Staged> staging;
};

static void layout_sizes(const ModelCfg& c, int P, size_t* sys_b, size_t* ws_b, size_t* fb_b) {
  const int HW = c.H * c.W, KK = c.K * c.K;
  const size_t tab = c.K <= kMfmaMaxK ? sizeof(uint16_t) * size_t(2) * c.K * 64 * 16 : 0;
  *sys_b = 2 * al256(sizeof(float) * KK) + al256(tab) + al256(sizeof(float) * HW);
  *ws_b = workspace_bytes(P, acc_rows_upto(P, HW), HW, c.d, true, beta_per_particle(c));
  *fb_b = fit_buffers_bytes(P, c.d);
}

static size_t request_bytes(const ModelCfg& c, int P) {
  size_t a, b, f;
  layout_sizes(c, P, &a, &b, &f);
  return DevicePool::size_class(a + b + f + al256(sizeof(FitOut)));
}

static double request_work(const ModelCfg& c, int P) {
  return double(P) * c.H * c.W * c.k * c.k;
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
  gl_server_stats st{};  // guarded by mu
  // scheduler thread only
  std::vector<std::unique_ptr<Active>> active;
  double active_work = 0.0;  // of the running systems
  DevicePool pool;
  PinnedPool pinned;
  std::deque<Tick> inflight;
  std::vector<Staged> staged;  // uploads enqueued since the last tick's event
  std::vector<hipEvent_t> spare_events;
  FitOut* out_host = nullptr;  // pinned, max_systems slots
  std::vector<int> free_slots;
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

// The system's memory back to the pools (its GPU work is complete, or ordered on the
// server's stream before any later use of the block).
static void release(gl_server* s, Active& a) {
  if (a.block) s->pool.give(a.block, a.block_bytes);
  a.block = nullptr;
  if (a.out_host) s->free_slots.push_back(int(a.out_host - s->out_host));
  a.out_host = nullptr;
}

static hipEvent_t get_event(gl_server* s) {
  if (!s->spare_events.empty()) {
    hipEvent_t e = s->spare_events.back();
    s->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

static int admit(gl_server* s, std::unique_ptr<Request> rq) {
  auto a = std::make_unique<Active>();
  a->t_admit = now_ns();
  a->req = std::move(rq);
  const Request& r = *a->req;
  const ModelCfg& c = r.cfg;
  const int HW = c.H * c.W, P = r.fp.P;
  a->tiles = choose_tiles(P, HW);
  size_t sys_b, ws_b, fb_b;
  layout_sizes(c, P, &sys_b, &ws_b, &fb_b);
  // the budget covers the active blocks (this one included) and the cache
  {
    size_t in_use;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      in_use = s->st.hbm_in_use;
    }
    const size_t room = s->opts.hbm_budget_bytes - std::min(s->opts.hbm_budget_bytes, in_use);
    if (s->pool.cached() > room) s->pool.trim(room);
  }
  int rc = s->pool.take(r.bytes, &a->block, &a->block_bytes);
  if (!rc && s->free_slots.empty()) rc = set_error(GL_E_DEVICE, "no result slot");
  if (!rc) {
    a->out_host = s->out_host + s->free_slots.back();
    s->free_slots.pop_back();
    std::vector<uint8_t> img;
    int sx = 0;
    system_image(&r.desc, c, img, &sx);
    system_bind(a->sys, c, a->block, img.size(), 1, sx);
    workspace_layout(a->ws, a->block + sys_b, P, acc_rows_upto(P, HW), HW, c.d, true,
                     beta_per_particle(c));
    fit_buffers_layout(a->fb, a->block + sys_b + ws_b, P, c.d);
    a->out_dev = reinterpret_cast<FitOut*>(a->block + sys_b + ws_b + fb_b);
    const size_t pri_b = sizeof(Prior) * c.d;
    Staged stg{nullptr, 0};
    rc = s->pinned.take(img.size() + pri_b, &stg.p, &stg.bytes);
    if (!rc) {
      std::memcpy(stg.p, img.data(), img.size());
      std::memcpy(stg.p + img.size(), r.priors.data(), pri_b);
      const hipError_t e1 =
          hipMemcpyAsync(a->block, stg.p, img.size(), hipMemcpyHostToDevice, s->stream);
      const hipError_t e2 = hipMemcpyAsync(a->fb.prior, stg.p + img.size(), pri_b,
                                           hipMemcpyHostToDevice, s->stream);
      s->staged.push_back(stg);  // given back when the next tick's event completes
      if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        rc = set_error(GL_E_DEVICE, "input upload failed");
      }
    }
  }
  if (!rc) {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.nsys = 1;
    g.sys[0] = make_sys(a->sys, a->ws, P, a->tiles);
    attach_fit(g.sys[0], a->fb, a->req->fp, a->ws);
    rc = launch_fit_init(g, s->stream);
  }
  if (rc) {
    // nothing of it runs later; copies already enqueued into its block are ordered on the
    // stream before any reuse of the block
    const gl_fit_result res = error_result(*a, rc);
    release(s, *a);
    finish(s, *a, res);
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.active = int(s->active.size());
    return rc;
  }
  s->active_work += r.work;
  s->active.push_back(std::move(a));
  return GL_OK;
}

// Systems grouped by kernel configuration; each group runs `mode` (2: one Adam step; 1: the
// log L pass, the log posterior and the best-particle selection). A group whose launches
// fail marks its systems (they retire with the error); the other groups go on.
static void run_grouped(gl_server* s, const std::vector<Active*>& sys, int mode) {
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
        g.sys[i].fit_out = a->out_dev;
      }
      int rc = run_group(g, kv.first.first, kv.first.second, mode, s->stream);
      if (!rc && mode == 2) rc = launch_adam(g, s->stream);
      if (!rc && mode == 1) rc = launch_logpost(g, s->stream);
      if (!rc && mode == 1) rc = launch_fit_best(g, s->stream);
      if (rc)
        for (int i = 0; i < g.nsys; ++i)
          if (list[i0 + i]->failed == GL_OK) list[i0 + i]->failed = rc;
    }
  }
}

// Retire the systems of the oldest in-flight tick once it has completed (wait: block on it).
static bool reap_one(gl_server* s, bool wait) {
  if (s->inflight.empty()) return false;
  Tick& t = s->inflight.front();
  const hipError_t e = wait ? hipEventSynchronize(t.ev) : hipEventQuery(t.ev);
  if (e == hipErrorNotReady) return false;
  const bool device_ok = e == hipSuccess;
  if (!device_ok) (void)hipGetLastError();
  for (Active* a : t.retiring) {
    gl_fit_result r;
    if (a->failed != GL_OK || !device_ok) {
      r = error_result(*a, a->failed != GL_OK ? a->failed : GL_E_DEVICE);
    } else {
      std::memset(&r, 0, sizeof(r));
      fit_result_from_out(*a->out_host, a->req->cfg, &r);
      r.t_submit = a->req->t_submit;
      r.t_admit = a->t_admit;
      r.t_done = now_ns();
    }
    release(s, *a);
    finish(s, *a, r);
    a->done = true;
  }
  for (const Staged& st : t.staging) s->pinned.give(st.p, st.bytes);
  s->spare_events.push_back(t.ev);
  s->inflight.pop_front();
  s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                 [](const std::unique_ptr<Active>& a) { return a->done; }),
                  s->active.end());
  std::lock_guard<std::mutex> lk(s->mu);
  s->st.active = int(s->active.size());
  return true;
}

// Enqueue one tick of the running systems, then its end event.
static void enqueue_tick(gl_server* s) {
  std::vector<Active*> running;
  for (auto& a : s->active)
    if (a->state == RUNNING) running.push_back(a.get());
  for (int k = 0; k < s->opts.steps_per_tick; ++k) {
    std::vector<Active*> run;
    for (Active* a : running)
      if (a->failed == GL_OK && a->req->fp.step < a->req->fp.K) run.push_back(a);
    if (run.empty()) break;
    run_grouped(s, run, 2);
    for (Active* a : run)
      if (a->failed == GL_OK) a->req->fp.step++;
  }
  Tick t;
  std::vector<Active*> fin;
  for (Active* a : running) {
    if (a->failed == GL_OK && a->req->fp.step < a->req->fp.K) continue;
    if (a->failed == GL_OK) fin.push_back(a);
    a->state = RETIRING;
    s->active_work -= a->req->work;
    t.retiring.push_back(a);
  }
  if (!fin.empty()) run_grouped(s, fin, 1);
  for (Active* a : fin)
    if (a->failed == GL_OK &&
        hipMemcpyAsync(a->out_host, a->out_dev, sizeof(FitOut), hipMemcpyDeviceToHost,
                       s->stream) != hipSuccess) {
      (void)hipGetLastError();
      a->failed = GL_E_DEVICE;
    }
  t.staging.swap(s->staged);
  t.ev = get_event(s);
  if (!t.ev || hipEventRecord(t.ev, s->stream) != hipSuccess) {
    // no event to track this tick: finish it here, and mark it with a fresh event if one can
    // be made (otherwise its systems retire with a device error)
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s->stream);
    if (!t.ev) t.ev = get_event(s);
    if (!t.ev || hipEventRecord(t.ev, s->stream) != hipSuccess) {
      (void)hipGetLastError();
      for (Active* a : t.retiring)
        if (a->failed == GL_OK) a->failed = GL_E_DEVICE;
      if (!t.ev) {  // retire without an event
        for (Active* a : t.retiring) {
          const gl_fit_result r = error_result(*a, a->failed);
          release(s, *a);
          finish(s, *a, r);
          a->done = true;
        }
        for (const Staged& st : t.staging) s->pinned.give(st.p, st.bytes);
        return;
      }
    }
  }
  s->inflight.push_back(std::move(t));
}

static void scheduler(gl_server* s) {
  (void)hipSetDevice(s->device);
  while (true) {
    while (reap_one(s, false)) {
    }
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                   [](const std::unique_ptr<Active>& a) { return a->done; }),
                    s->active.end());
    bool have_queue;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->closing && s->queue.empty() && s->active.empty() && s->inflight.empty()) break;
      if (s->queue.empty() && s->active.empty() && s->inflight.empty()) {
        s->cv.wait(lk, [&] { return s->closing || !s->queue.empty(); });
        continue;
      }
      have_queue = !s->queue.empty();
    }
    // admission (FIFO) under the slot, budget and fill limits
    while (have_queue) {
      std::unique_ptr<Request> rq;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->queue.empty() || int(s->active.size()) >= s->opts.max_systems) break;
        if (s->st.hbm_in_use + s->queue.front()->bytes > s->opts.hbm_budget_bytes) break;
        if (s->active_work > 0.0 &&
            s->active_work + s->queue.front()->work > s->opts.fill_subpixels)
          break;
        rq = std::move(s->queue.front());
        s->queue.pop_front();
        s->st.hbm_in_use += rq->bytes;
        s->st.hbm_peak = std::max(s->st.hbm_peak, s->st.hbm_in_use);
        s->st.admitted++;
        s->st.queued = int(s->queue.size());
      }
      admit(s, std::move(rq));  // a failure retires the request with its status
    }
    bool any_running = false;
    for (auto& a : s->active) any_running = any_running || a->state == RUNNING;
    if (any_running) {
      enqueue_tick(s);
      std::lock_guard<std::mutex> lk(s->mu);
      s->st.ticks++;
      s->st.active = int(s->active.size());
    }
    // at most two ticks in flight; with nothing to enqueue, wait for the oldest
    if (s->inflight.size() >= 2 || (!any_running && !s->inflight.empty())) reap_one(s, true);
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
  void* slots = nullptr;
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc(&slots, sizeof(FitOut) * size_t(o->max_systems), hipHostMallocDefault) !=
          hipSuccess) {
    (void)hipGetLastError();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return set_error(GL_E_DEVICE, "cannot create the server stream or result slots");
  }
  s->out_host = static_cast<FitOut*>(slots);
  for (int i = o->max_systems - 1; i >= 0; --i) s->free_slots.push_back(i);
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
  (void)hipStreamSynchronize(s->stream);
  for (const Staged& st : s->staged) s->pinned.give(st.p, st.bytes);
  for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
  (void)hipHostFree(s->out_host);
  (void)hipStreamDestroy(s->stream);
  delete s;  // the pools free their blocks
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
