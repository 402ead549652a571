// Fixed-budget multi-start fit (Sec. 2.2 bijectors and Jacobian-corrected prior, Sec. 2.3
// multi-start gradient descent with Adam): kernels and the gl_fit* C ABI.
//
// One Adam step of one system = the gl_loglik_grad pipeline evaluated at theta = g(z)
// (the prologue applies the bijector) + adam_kernel, which forms
//   d f / d z = -( d logL/d theta * g'(z) + d log p~ / d z ),  f = -(log L + log p~),
// and updates (z, m, v) with the learning rate lr0 -> lr1 linear over K steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "glens_device.h"
#include "glens_fit.h"
#include "glens_fit_device.h"
#include "glens_host.h"

namespace glens {

__global__ void __launch_bounds__(256) fit_init_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int idx = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (idx >= s.P * s.d) return;
  const int p = idx / s.d, j = idx - p * s.d;
  s.z[idx] = draw_start(s.prior[j], s.seed_lo, s.seed_hi, p, j);
  s.mom1[idx] = 0.f;
  s.mom2[idx] = 0.f;
}

__global__ void __launch_bounds__(256) adam_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int idx = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (idx >= s.P * s.d) return;
  const int p = idx / s.d, j = idx - p * s.d;
  if (!isfinite(s.logl[p])) return;  // a non-finite particle stays where it is
  const float z = s.z[idx];
  float dlp, dth;
  log_prior_z(s.prior[j], z, s.theta_out[idx], dlp, dth);
  const float gz = -(s.grad[idx] * dth + dlp);
  const float b1 = s.beta1, b2 = s.beta2;
  const float m = b1 * s.mom1[idx] + (1.0f - b1) * gz;
  const float v = b2 * s.mom2[idx] + (1.0f - b2) * gz * gz;
  const int t = s.step + 1;
  const float mhat = m / (1.0f - powf(b1, float(t)));
  const float vhat = v / (1.0f - powf(b2, float(t)));
  const float lr = s.lr0 + (s.lr1 - s.lr0) * float(min(s.step, s.nsteps)) / float(s.nsteps);
  s.mom1[idx] = m;
  s.mom2[idx] = v;
  s.z[idx] = z - lr * mhat / (sqrtf(vhat) + s.eps_adam);
}

// log posterior in unconstrained space of each particle: log L + sum_j log p~(z_j).
__global__ void __launch_bounds__(64) logpost_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int p = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (p >= s.P) return;
  double lp = 0.0;
  for (int j = 0; j < s.d; ++j) {
    float dlp, dth;
    lp += log_prior_z(s.prior[j], s.z[(size_t)p * s.d + j], s.theta_out[(size_t)p * s.d + j],
                      dlp, dth);
  }
  const double v = s.logl[p] + lp;
  s.logpost[p] = isfinite(v) ? v : -INFINITY;
}

// One 256-lane block per system: the particle with the largest finite log posterior (ties
// to the lowest index, as fit_result_from_device picks it) and its values, into s.fit_out.
__global__ void __launch_bounds__(256) fit_best_kernel(Group g) {
  __shared__ double sv[256];
  __shared__ int sb[256];
  const SysDesc& s = g.sys[find_sys(g, blockIdx.x)];
  const int t = threadIdx.x;
  double bv = 0.0;
  int bi = -1;
  for (int p = t; p < s.P; p += blockDim.x) {  // increasing p: a tie keeps the lower index
    const double v = s.logpost[p];
    if (isfinite(v) && (bi < 0 || v > bv)) {
      bv = v;
      bi = p;
    }
  }
  sv[t] = bv;
  sb[t] = bi;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) {
      const int j = sb[t + off];
      if (j >= 0 && (sb[t] < 0 || sv[t + off] > sv[t] || (sv[t + off] == sv[t] && j < sb[t]))) {
        sv[t] = sv[t + off];
        sb[t] = j;
      }
    }
    __syncthreads();
  }
  FitOut* o = s.fit_out;
  const int best = sb[0];
  if (t == 0) {
    o->best = best;
    o->logpost = best >= 0 ? sv[0] : -INFINITY;
    o->logl = best >= 0 ? s.logl[best] : -INFINITY;
    o->chi2 = best >= 0 ? s.chi2[best] : INFINITY;
  }
  if (best >= 0)
    for (int j = t; j < s.d; j += blockDim.x) {
      o->theta[j] = s.theta_out[(size_t)best * s.d + j];
      o->z[j] = s.z[(size_t)best * s.d + j];
    }
}

static int launch_elem(void (*k)(Group), Group& g, int per_sys_threads_fn(const SysDesc&),
                       int threads, hipStream_t st) {
  int b = 0;
  for (int i = 0; i < g.nsys; ++i) {
    g.block0[i] = b;
    b += (per_sys_threads_fn(g.sys[i]) + threads - 1) / threads;
  }
  g.block0[g.nsys] = b;
  if (b == 0) return GL_OK;
  hipLaunchKernelGGL(k, dim3(b), dim3(threads), 0, st, g);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GL_OK : set_error(GL_E_DEVICE, "launch: %s", hipGetErrorString(e));
}

static int n_elems(const SysDesc& s) { return s.P * s.d; }
static int n_parts(const SysDesc& s) { return s.P; }

int launch_fit_init(Group& g, hipStream_t st) { return launch_elem(fit_init_kernel, g, n_elems, 256, st); }
int launch_adam(Group& g, hipStream_t st) { return launch_elem(adam_kernel, g, n_elems, 256, st); }
int launch_logpost(Group& g, hipStream_t st) { return launch_elem(logpost_kernel, g, n_parts, 64, st); }
static int one_block(const SysDesc&) { return 256; }
int launch_fit_best(Group& g, hipStream_t st) { return launch_elem(fit_best_kernel, g, one_block, 256, st); }

void fit_result_from_out(const FitOut& o, const ModelCfg& c, gl_fit_result* out) {
  out->d = c.d;
  out->best = o.best;
  if (o.best < 0) {
    out->status = GL_E_NUMERIC;
    return;
  }
  out->status = GL_OK;
  std::memcpy(out->theta_best, o.theta, sizeof(float) * c.d);
  std::memcpy(out->z_best, o.z, sizeof(float) * c.d);
  out->logl_best = o.logl;
  out->logpost_best = o.logpost;
  const int dof = c.H * c.W - c.d;
  out->chi2nu = dof > 0 ? o.chi2 / dof : o.chi2;
}

// ------------------------------------------------------------------------------------------
// host helpers
// ------------------------------------------------------------------------------------------
int validate_fit_opts(const gl_fit_opts* o, int d, std::vector<Prior>& pri) {
  if (!o) return set_error(GL_E_INVALID, "opts is NULL");
  if (o->P < 1) return set_error(GL_E_INVALID, "P must be >= 1");
  if (o->K < 1) return set_error(GL_E_INVALID, "K must be >= 1");
  if (!(std::isfinite(o->lr0) && std::isfinite(o->lr1) && o->lr0 >= 0.f && o->lr1 >= 0.f))
    return set_error(GL_E_INVALID, "learning rates must be finite and >= 0");
  const bool dflt = o->beta1 == 0.f && o->beta2 == 0.f && o->eps == 0.f;
  if (!dflt && !(o->beta1 >= 0.f && o->beta1 < 1.f && o->beta2 >= 0.f && o->beta2 < 1.f && o->eps > 0.f))
    return set_error(GL_E_INVALID, "Adam constants out of range");
  if (!o->priors) return set_error(GL_E_INVALID, "priors is NULL");
  pri.resize(d);
  for (int j = 0; j < d; ++j) {
    const gl_prior& p = o->priors[j];
    Prior& q = pri[j];
    q.family = p.family;
    q.mu = p.mu;
    q.sigma = p.sigma;
    q.lo = p.lo;
    q.hi = p.hi;
    const double ls2pi = 0.5 * std::log(2.0 * M_PI);
    switch (p.family) {
      case GL_PRIOR_NORMAL:
      case GL_PRIOR_LOGNORMAL:
        if (!(p.sigma > 0.f) || !std::isfinite(p.mu))
          return set_error(GL_E_INVALID, "prior %d: sigma must be > 0", j);
        q.logc = float(-std::log(double(p.sigma)) - ls2pi);
        break;
      case GL_PRIOR_TRUNCNORMAL: {
        if (!(p.sigma > 0.f) || !(p.lo < p.hi))
          return set_error(GL_E_INVALID, "prior %d: need sigma > 0 and lo < hi", j);
        const double a = (double(p.lo) - p.mu) / p.sigma, b = (double(p.hi) - p.mu) / p.sigma;
        const double Z = 0.5 * std::erfc(-b / std::sqrt(2.0)) - 0.5 * std::erfc(-a / std::sqrt(2.0));
        if (!(Z > 0.0)) return set_error(GL_E_INVALID, "prior %d: empty truncation", j);
        // log p(theta) + log|J| = -r^2/2 - log sigma - log sqrt(2 pi) - log Z + log(hi - lo)
        //                         + log s + log(1 - s)
        q.logc = float(-std::log(double(p.sigma)) - ls2pi - std::log(Z) +
                       std::log(double(p.hi) - p.lo));
        break;
      }
      case GL_PRIOR_UNIFORM:
        if (!(p.lo < p.hi)) return set_error(GL_E_INVALID, "prior %d: need lo < hi", j);
        q.logc = 0.f;
        break;
      default:
        return set_error(GL_E_INVALID, "prior %d: unknown family %d", j, p.family);
    }
  }
  return GL_OK;
}


FitParams fit_params(const gl_fit_opts* o) {
  FitParams f;
  f.P = o->P;
  f.K = o->K;
  f.step = 0;
  f.lr0 = o->lr0;
  f.lr1 = o->lr1;
  if (!(o->beta1 == 0.f && o->beta2 == 0.f && o->eps == 0.f)) {
    f.beta1 = o->beta1;
    f.beta2 = o->beta2;
    f.eps = o->eps;
  }
  f.seed = o->seed;
  return f;
}

static size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

size_t fit_buffers_bytes(int P, int d) {
  return 3 * a256(sizeof(float) * size_t(P) * d) + a256(sizeof(Prior) * d) +
         2 * a256(sizeof(double) * P);
}

void fit_buffers_layout(FitBuffers& fb, char* base, int P, int d) {
  fb.P = P;
  fb.d = d;
  fb.bytes = fit_buffers_bytes(P, d);
  fb.base = base;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += a256(b);
    return p;
  };
  fb.z = reinterpret_cast<float*>(take(sizeof(float) * size_t(P) * d));
  fb.m = reinterpret_cast<float*>(take(sizeof(float) * size_t(P) * d));
  fb.v = reinterpret_cast<float*>(take(sizeof(float) * size_t(P) * d));
  fb.prior = reinterpret_cast<Prior*>(take(sizeof(Prior) * d));
  fb.logpost = reinterpret_cast<double*>(take(sizeof(double) * P));
  fb.chi2 = reinterpret_cast<double*>(take(sizeof(double) * P));
}

int fit_buffers_alloc(FitBuffers& fb, int P, int d, const Prior* host_priors) {
  char* base = nullptr;
  GL_HIP(hipMalloc(&base, fit_buffers_bytes(P, d)));
  fit_buffers_layout(fb, base, P, d);
  fb.owned = true;
  GL_HIP(hipMemcpy(fb.prior, host_priors, sizeof(Prior) * d, hipMemcpyHostToDevice));
  return GL_OK;
}

void fit_buffers_free(FitBuffers& fb) {
  if (fb.owned && fb.base) (void)hipFree(fb.base);
  fb = FitBuffers();
}

void attach_fit(SysDesc& s, const FitBuffers& fb, const FitParams& fp, const Workspace& ws) {
  s.theta = nullptr;
  s.z = fb.z;
  s.prior = fb.prior;
  s.theta_out = ws.theta;
  s.mom1 = fb.m;
  s.mom2 = fb.v;
  s.logpost = fb.logpost;
  s.chi2 = fb.chi2;
  s.logl = ws.logl;
  s.grad = ws.grad;
  s.step = fp.step;
  s.nsteps = fp.K;
  s.lr0 = fp.lr0;
  s.lr1 = fp.lr1;
  s.beta1 = fp.beta1;
  s.beta2 = fp.beta2;
  s.eps_adam = fp.eps;
  s.seed_lo = uint32_t(fp.seed);
  s.seed_hi = uint32_t(fp.seed >> 32);
}

int fit_result_from_device(const FitBuffers& fb, const Workspace& ws, int P, const ModelCfg& c,
                           hipStream_t st, gl_fit_result* out) {
  std::vector<double> lp(P), c2(P);
  GL_HIP(hipMemcpyAsync(lp.data(), fb.logpost, sizeof(double) * P, hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(c2.data(), fb.chi2, sizeof(double) * P, hipMemcpyDeviceToHost, st));
  GL_HIP(hipStreamSynchronize(st));
  int best = -1;
  for (int p = 0; p < P; ++p)
    if (std::isfinite(lp[p]) && (best < 0 || lp[p] > lp[best])) best = p;
  out->d = c.d;
  out->best = best;
  if (best < 0) {
    out->status = GL_E_NUMERIC;
    return set_error(GL_E_NUMERIC, "no particle has a finite log posterior");
  }
  double ll = 0.0;
  GL_HIP(hipMemcpyAsync(out->theta_best, ws.theta + size_t(best) * c.d, sizeof(float) * c.d,
                        hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(out->z_best, fb.z + size_t(best) * c.d, sizeof(float) * c.d,
                        hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(&ll, ws.logl + best, sizeof(double), hipMemcpyDeviceToHost, st));
  GL_HIP(hipStreamSynchronize(st));
  out->status = GL_OK;
  out->logl_best = ll;
  out->logpost_best = lp[best];
  const int dof = c.H * c.W - c.d;
  out->chi2nu = dof > 0 ? c2[best] / dof : c2[best];
  return GL_OK;
}

}  // namespace glens

using namespace glens;

struct gl_fit_state {
  gl_model* model = nullptr;
  FitBuffers fb;
  FitParams fp;
};

// The model's work space at this fit's size with the fit buffers (a likelihood call on the
// same model between two fit calls may have regrown it).
static int fit_reserve(gl_fit_state* st) {
  gl_model* m = st->model;
  const ModelCfg& c = m->sys.cfg;
  const int HW = c.H * c.W;
  return workspace_reserve(m->ws, st->fp.P, choose_tiles(st->fp.P, HW), HW, c.d, true,
                           beta_per_particle(c));
}

static SysDesc fit_sys(gl_fit_state* st) {
  gl_model* m = st->model;
  const int tiles = choose_tiles(st->fp.P, m->sys.cfg.H * m->sys.cfg.W);
  SysDesc s = make_sys(m->sys, m->ws, st->fp.P, tiles);
  attach_fit(s, st->fb, st->fp, m->ws);
  return s;
}

extern "C" {

int gl_fit_state_create(gl_model* m, const gl_fit_opts* o, gl_fit_state** out, void* stream) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!m) return set_error(GL_E_INVALID, "model is NULL");
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  std::vector<Prior> pri;
  int rc = validate_fit_opts(o, m->sys.cfg.d, pri);
  if (rc) return rc;
  gl_fit_state* st = new (std::nothrow) gl_fit_state();
  if (!st) return set_error(GL_E_NOMEM, "host allocation failed");
  st->model = m;
  st->fp = fit_params(o);
  const ModelCfg& c = m->sys.cfg;
  rc = workspace_reserve(m->ws, o->P, choose_tiles(o->P, c.H * c.W), c.H * c.W, c.d, true,
                         beta_per_particle(c));
  if (!rc) rc = fit_buffers_alloc(st->fb, o->P, c.d, pri.data());
  if (rc) {
    fit_buffers_free(st->fb);
    delete st;
    return rc;
  }
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = fit_sys(st);
  rc = launch_fit_init(g, (hipStream_t)stream);
  if (rc) {
    fit_buffers_free(st->fb);
    delete st;
    return rc;
  }
  *out = st;
  return GL_OK;
}

int gl_fit_state_destroy(gl_fit_state* st) {
  clear_error();
  if (!st) return GL_OK;
  (void)hipDeviceSynchronize();
  fit_buffers_free(st->fb);
  delete st;
  return GL_OK;
}

int gl_fit_state_step(gl_fit_state* st, int n, void* stream) {
  clear_error();
  if (!st) return set_error(GL_E_INVALID, "state is NULL");
  if (n < 0) return set_error(GL_E_INVALID, "n must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const ModelCfg& c = st->model->sys.cfg;
  if (n > 0) {
    int rc = fit_reserve(st);
    if (rc) return rc;
  }
  for (int i = 0; i < n; ++i) {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.nsys = 1;
    g.sys[0] = fit_sys(st);
    int rc = run_group(g, subpix_key(c), c.K, 2, s);
    if (!rc) rc = launch_adam(g, s);
    if (rc) return rc;
    st->fp.step++;
  }
  return GL_OK;
}

int gl_fit_state_load(gl_fit_state* st, const float* z, const float* m, const float* v, int step,
                      void* stream) {
  clear_error();
  if (!st) return set_error(GL_E_INVALID, "state is NULL");
  if (step < 0) return set_error(GL_E_INVALID, "step must be >= 0");
  int rc;
  if ((rc = check_device_ptr(z, "z")) || (rc = check_device_ptr(m, "m")) ||
      (rc = check_device_ptr(v, "v")))
    return rc;
  const size_t b = sizeof(float) * size_t(st->fp.P) * st->fb.d;
  hipStream_t s = (hipStream_t)stream;
  GL_HIP(hipMemcpyAsync(st->fb.z, z, b, hipMemcpyDeviceToDevice, s));
  GL_HIP(hipMemcpyAsync(st->fb.m, m, b, hipMemcpyDeviceToDevice, s));
  GL_HIP(hipMemcpyAsync(st->fb.v, v, b, hipMemcpyDeviceToDevice, s));
  st->fp.step = step;
  return GL_OK;
}

int gl_fit_state_store(gl_fit_state* st, float* z, float* m, float* v, int* step, void* stream) {
  clear_error();
  if (!st) return set_error(GL_E_INVALID, "state is NULL");
  const size_t b = sizeof(float) * size_t(st->fp.P) * st->fb.d;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (z && (rc = check_device_ptr(z, "z"))) return rc;
  if (m && (rc = check_device_ptr(m, "m"))) return rc;
  if (v && (rc = check_device_ptr(v, "v"))) return rc;
  if (z) GL_HIP(hipMemcpyAsync(z, st->fb.z, b, hipMemcpyDeviceToDevice, s));
  if (m) GL_HIP(hipMemcpyAsync(m, st->fb.m, b, hipMemcpyDeviceToDevice, s));
  if (v) GL_HIP(hipMemcpyAsync(v, st->fb.v, b, hipMemcpyDeviceToDevice, s));
  if (step) *step = st->fp.step;
  return GL_OK;
}

int gl_fit_state_result(gl_fit_state* st, gl_fit_result* out, void* stream) {
  clear_error();
  if (!st || !out) return set_error(GL_E_INVALID, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const ModelCfg& c = st->model->sys.cfg;
  int rc = fit_reserve(st);
  if (rc) return rc;
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = fit_sys(st);
  rc = run_group(g, subpix_key(c), c.K, 1, s);
  if (!rc) rc = launch_logpost(g, s);
  if (rc) return rc;
  return fit_result_from_device(st->fb, st->model->ws, st->fp.P, c, s, out);
}

int gl_fit(gl_model* m, const gl_fit_opts* o, gl_fit_result* out, void* stream) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  gl_fit_state* st = nullptr;
  int rc = gl_fit_state_create(m, o, &st, stream);
  if (rc) return rc;
  rc = gl_fit_state_step(st, o->K, stream);
  if (!rc) rc = gl_fit_state_result(st, out, stream);
  const std::string err = rc ? std::string(gl_last_error()) : std::string();
  gl_fit_state_destroy(st);
  if (rc) set_error(rc, "%s", err.c_str());
  return rc;
}

}  // extern "C"
