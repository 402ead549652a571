// Variational inference with a multivariate normal surrogate (Sec. 2.4): the gl_vi* C ABI.
//
// q = N(mu, Sigma) in unconstrained space, Sigma = L L^T with L from the Cholesky bijector:
// the n_c = d(d+1)/2 values v fill the lower triangle of L row by row (entry i(i+1)/2 + j
// is L_ij) and the diagonal is exponentiated. The ELBO loss E_q[log q - log p~(I, z)] is
// minimised by Adam over x = (mu, v). Each iteration:
//   draw     one block per sample s: eps_s ~ N(0, I) (Philox, counter (s, j, k, tag)),
//            z_s = mu + L eps_s, rounded to FP32 for the likelihood pipeline, and the
//            pipeline's decode of it (prologue) in the same kernel;
//   pipeline log L and d log L / d theta at g(z_s) for every sample in one batched launch;
//   grad     one block per sample: the pipeline's finalize, then f_s = -log p~(z_s | I) and
//            grad f_s (prior, bijector) in the same kernel;
//   reduce   one block per chunk of kViChunk samples (staged in LDS): per entry of x the
//            chunk's sum (in sample order, FP64) of (grad f)_i or (grad f)_i eps_j over its
//            samples with a finite objective, and the chunk's sum of f and sample count;
//   update   one lane per entry of x: the chunks' sums added in chunk order give the
//            pathwise gradient estimate (mean over the samples with a finite objective) of
//              mu_i: E[(grad f)_i],  L_ij (i > j): E[(grad f)_i eps_j],
//              v_ii = log L_ii: L_ii E[(grad f)_i eps_i] - 1,
//            then Adam at the iteration's learning rate. x is double-buffered so that every
//            lane reads the iteration's old state; lane 0 also records the loss
//            E[f] - sum_i log L_ii - (d/2)(1 + log 2 pi).
// With the score-function estimator (the form the paper prints, eq. elbo-grad: the mean over
// the samples of (log q(z) - log p~(I, z)) grad log q(z), grad at fixed z) the last two
// stages are instead:
//   reduce   per chunk: w_s = log q(z_s) - log p~(I, z_s) = f_s - |eps_s|^2 / 2
//            - sum_i log L_ii - (d/2) log 2 pi, and the chunk's sums of w_s eps_s (one per
//            mu entry) and w_s eps_si eps_sj (i >= j), then its sum of f, count and sum of w;
//   update   one block: the chunks' sums added in chunk order give a = sum w eps and the
//            lower triangle of B = sum w eps eps^T; with grad log q = (L^-T eps, the lower
//            triangle of L^-T eps eps^T, diagonal L_ii (..)_ii - 1) the estimate is
//            L^-T a / n for mu, (L^-T B)_ij / n for i > j and L_ii (L^-T B)_ii / n -
//            sum w / n for v_ii; each column of L^-T B is one back substitution with L^T
//            (rows i >= j only), in LDS; then Adam on every entry.
// The learning rate rises from 0 to lr_max as lr_max (1 - (1 - k / warmup)^2) over the
// first `warmup` iterations (the paper: 0 -> 1e-3 over 500), then stays at lr_max, or, when
// a final rate is given, falls geometrically to it on the last iteration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "glens_device.h"
#include "glens_fit.h"
#include "glens_fit_device.h"
#include "glens_host.h"
#include "glens_particle.h"

namespace glens {

constexpr int kViThreads = 64;
constexpr int kViChunk = 32;  // samples per block of the reduction
constexpr uint32_t kViDrawTag = 0x76690000u;
constexpr uint32_t kViSampleTag = 0x76697371u;
constexpr double kLog2Pi = 1.8378770664093453;  // log(2 pi)

struct ViArgs {
  int n, d, nc, k;
  float lr;
  float beta1, beta2, adam_eps;
  double bc1, bc2;     // Adam's bias corrections 1 - beta^(k + 1) of this iteration
  const Prior* prior;
  const double* x;     // [d + nc] current (mu, v)
  double* x_new;       // [d + nc] next (mu, v)
  double* m;           // [d + nc] Adam moments
  double* s;
  double* eps;         // [n][d] this iteration's draws
  float* z32;          // [n][d] samples for the pipeline
  float* g;            // [n][d] grad f
  double* f;           // [n] f, NaN when not finite
  const double* logl;  // pipeline outputs
  const float* grad;
  const float* theta;
  double* loss;        // [K] loss history
  double* part;        // [chunks][d + nc + 2] per-chunk sums, then the chunk's sum of f and count
  uint32_t seed_lo, seed_hi;
};

// Row and column of entry q of x: (q, -1) for mu_q, else the lower-triangle position of
// v_(q - d) (row-major: r = i(i+1)/2 + j).
__device__ __forceinline__ void vi_entry(int q, int d, int& i, int& j) {
  if (q < d) {
    i = q;
    j = -1;
    return;
  }
  const int r = q - d;
  i = int((sqrt(8.0 * r + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= r) ++i;
  while (i * (i + 1) / 2 > r) --i;
  j = r - i * (i + 1) / 2;
}

__device__ __forceinline__ double chol_entry(const double* v, int i, int j) {
  const double e = v[i * (i + 1) / 2 + j];
  return i == j ? exp(e) : e;
}

// z = mu + L eps for one sample (block), eps drawn with tag `tag` at iteration `k`. The
// factor is first copied to LDS (its diagonal exponentiated there): each lane's row then
// reads it without an L2 round trip per entry.
__device__ __forceinline__ void draw_sample(const double* mu, const double* v, int d, int s,
                                            int k, uint32_t tag, uint32_t seed_lo,
                                            uint32_t seed_hi, double* s_eps, double* eps_out,
                                            float* z32_out, double* z64_out) {
  __shared__ double s_l[kMaxParams * (kMaxParams + 1) / 2];
  const int nc = d * (d + 1) / 2;
  for (int q = threadIdx.x; q < nc; q += kViThreads) s_l[q] = v[q];
  for (int j = threadIdx.x; j < d; j += kViThreads) {
    uint32_t w[4] = {uint32_t(s), uint32_t(j), uint32_t(k), tag};
    philox4x32_10(w, seed_lo, seed_hi);
    const double u1 = u01(w[0], w[1]), u2 = u01(w[2], w[3]);
    const double e = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    s_eps[j] = e;
    if (eps_out) eps_out[size_t(s) * d + j] = e;
  }
  __syncthreads();  // the raw factor is in LDS
  for (int i = threadIdx.x; i < d; i += kViThreads) {
    const int q = i * (i + 1) / 2 + i;
    s_l[q] = exp(s_l[q]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += kViThreads) {
    double zi = mu[i];
    const double* li = s_l + i * (i + 1) / 2;
    for (int j = 0; j <= i; ++j) zi += li[j] * s_eps[j];
    if (z32_out) z32_out[size_t(s) * d + i] = float(zi);
    if (z64_out) z64_out[size_t(s) * d + i] = zi;
  }
}

// This iteration's draw of sample s = blockIdx.x, then the pipeline's decode of it
// (prologue): one launch instead of two.
__global__ void __launch_bounds__(kViThreads) vi_draw_decode_kernel(SysDesc s, ViArgs a) {
  __shared__ double s_eps[kMaxParams];
  draw_sample(a.x, a.x + a.d, a.d, blockIdx.x, a.k, kViDrawTag, a.seed_lo, a.seed_hi, s_eps,
              a.eps, a.z32, nullptr);
  __syncthreads();  // this sample's z is written
  prologue_particle(s, blockIdx.x);
}

// f = -log p~(z | I) and its gradient for one sample (terms summed in parameter order).
__device__ __forceinline__ void sample_objective(const ViArgs& a) {
  __shared__ double s_t[kMaxParams];
  __shared__ int s_bad;
  const int c = blockIdx.x;
  const size_t row = size_t(c) * a.d;
  int bad_lane = 0;
  for (int j = threadIdx.x; j < a.d; j += kViThreads) {
    float dlp, dth;
    s_t[j] = log_prior_z(a.prior[j], a.z32[row + j], a.theta[row + j], dlp, dth);
    const float gj = -(a.grad[row + j] * dth + dlp);
    a.g[row + j] = gj;
    bad_lane |= !isfinite(gj);
  }
  const int bad_any = __any(bad_lane);
  __syncthreads();
  if (threadIdx.x == 0) {
    double lp = a.logl[c];
    for (int j = 0; j < a.d; ++j) lp += s_t[j];
    s_bad = bad_any || !isfinite(lp);
    a.f[c] = s_bad ? NAN : -lp;
  }
}

// The pipeline's finalize (log L and its gradient) for sample blockIdx.x, then f and its
// gradient: one launch instead of two.
__global__ void __launch_bounds__(kViThreads) vi_finalize_objective_kernel(SysDesc s, ViArgs a) {
  finalize_particle(s, blockIdx.x);
  __syncthreads();  // this sample's log L and gradient are written
  sample_objective(a);
}

// Per-chunk sums of the gradient estimate's terms (one block per kViChunk samples).
__global__ void __launch_bounds__(256) vi_reduce_kernel(ViArgs a) {
  __shared__ double s_g[kViChunk][kMaxParams], s_e[kViChunk][kMaxParams];
  const int d = a.d, nx = a.d + a.nc;
  const int s0 = blockIdx.x * kViChunk, ns = min(kViChunk, a.n - s0);
  for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
    const int t = idx / d, j = idx - t * d;
    const size_t o = size_t(s0 + t) * d + j;
    const bool ok = isfinite(a.f[s0 + t]);  // a sample without a finite objective adds 0
    s_g[t][j] = ok ? double(a.g[o]) : 0.0;
    s_e[t][j] = ok ? a.eps[o] : 0.0;
  }
  __syncthreads();
  double* out = a.part + size_t(blockIdx.x) * (nx + 2);
  for (int q = threadIdx.x; q < nx; q += blockDim.x) {
    int i, j;
    vi_entry(q, d, i, j);
    double sum = 0.0;
    if (j < 0) {
      for (int t = 0; t < ns; ++t) sum += s_g[t][i];
    } else {
      for (int t = 0; t < ns; ++t) sum += s_g[t][i] * s_e[t][j];
    }
    out[q] = sum;
  }
  if (threadIdx.x == 0) {
    double fsum = 0.0;
    int nok = 0;
#pragma unroll 8
    for (int t = 0; t < ns; ++t) {
      const double fs = a.f[s0 + t];
      if (!isfinite(fs)) continue;
      ++nok;
      fsum += fs;
    }
    out[nx] = fsum;
    out[nx + 1] = nok;
  }
}

// Adam on entry q of x with gradient estimate gq.
__device__ __forceinline__ void vi_adam_entry(const ViArgs& a, int q, double gq) {
  const double mq = a.beta1 * a.m[q] + (1.0 - a.beta1) * gq;
  const double sq = a.beta2 * a.s[q] + (1.0 - a.beta2) * gq * gq;
  a.m[q] = mq;
  a.s[q] = sq;
  const double mhat = mq / a.bc1;
  const double shat = sq / a.bc2;
  a.x_new[q] = a.x[q] - a.lr * mhat / (sqrt(shat) + a.adam_eps);
}

// Gradient estimate and Adam update of one entry of x (and the loss, lane 0), from the
// chunks' sums.
__global__ void __launch_bounds__(256) vi_update_kernel(ViArgs a, int chunks) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int d = a.d, nx = a.d + a.nc;
  if (q >= nx) return;
  const double* v = a.x + d;
  int i, j;
  vi_entry(q, d, i, j);
  double sum = 0.0, fsum = 0.0, nokd = 0.0;
#pragma unroll 8
  for (int c = 0; c < chunks; ++c) {  // in chunk order (unrolled: the loads go out together)
    const double* pc = a.part + size_t(c) * (nx + 2);
    sum += pc[q];
    fsum += pc[nx];
    nokd += pc[nx + 1];
  }
  const int nok = int(nokd);
  if (nok == 0) {  // no usable sample: keep the state
    a.x_new[q] = a.x[q];
    if (q == 0) a.loss[a.k] = NAN;
    return;
  }
  double gq = sum / nok;
  if (j == i) gq = exp(v[i * (i + 1) / 2 + i]) * gq - 1.0;
  if (q == 0) {
    double logdet = 0.0;
    for (int t = 0; t < d; ++t) logdet += v[t * (t + 1) / 2 + t];
    a.loss[a.k] = fsum / nok - logdet - 0.5 * d * (1.0 + kLog2Pi);
  }
  vi_adam_entry(a, q, gq);
}

// Score-function estimator, per-chunk sums (one block per kViChunk samples): entry q < d
// gets sum w eps_q, entry (i, j) of v gets sum w eps_i eps_j; then the chunk's sum of f,
// count and sum of w. Samples without a finite objective add 0 everywhere.
__global__ void __launch_bounds__(256) vi_reduce_score_kernel(ViArgs a) {
  __shared__ double s_e[kViChunk][kMaxParams];
  __shared__ double s_w[kViChunk];
  const int d = a.d, nx = a.d + a.nc;
  const int s0 = blockIdx.x * kViChunk, ns = min(kViChunk, a.n - s0);
  for (int idx = threadIdx.x; idx < ns * d; idx += blockDim.x) {
    const int t = idx / d, j = idx - t * d;
    s_e[t][j] = a.eps[size_t(s0 + t) * d + j];
  }
  __syncthreads();
  if (threadIdx.x < ns) {
    const int t = threadIdx.x;
    const double fs = a.f[s0 + t];
    double e2 = 0.0, logdet = 0.0;
    for (int j = 0; j < d; ++j) e2 += s_e[t][j] * s_e[t][j];
    for (int i = 0; i < d; ++i) logdet += a.x[d + i * (i + 1) / 2 + i];
    s_w[t] = isfinite(fs) ? fs - 0.5 * e2 - logdet - 0.5 * d * kLog2Pi : 0.0;
  }
  __syncthreads();
  double* out = a.part + size_t(blockIdx.x) * (nx + 3);
  for (int q = threadIdx.x; q < nx; q += blockDim.x) {
    int i, j;
    vi_entry(q, d, i, j);
    double sum = 0.0;
    if (j < 0) {
      for (int t = 0; t < ns; ++t) sum += s_w[t] * s_e[t][i];
    } else {
      for (int t = 0; t < ns; ++t) sum += s_w[t] * s_e[t][i] * s_e[t][j];
    }
    out[q] = sum;
  }
  if (threadIdx.x == 0) {
    double fsum = 0.0, wsum = 0.0;
    int nok = 0;
    for (int t = 0; t < ns; ++t) {
      const double fs = a.f[s0 + t];
      if (!isfinite(fs)) continue;
      ++nok;
      fsum += fs;
      wsum += s_w[t];
    }
    out[nx] = fsum;
    out[nx + 1] = nok;
    out[nx + 2] = wsum;
  }
}

// Score-function estimator, one block: chunk sums, the back substitutions with L^T, the
// estimate and Adam on every entry. Dynamic LDS: L packed [nc] (diagonal exponentiated) and
// X [d][d + 1]: column j < d holds rows i >= j of B then of L^-T B, column d holds a then
// L^-T a.
__global__ void __launch_bounds__(256) vi_update_score_kernel(ViArgs a, int chunks) {
  extern __shared__ double s_dyn[];
  __shared__ double s_tot[3];
  const int d = a.d, nc = a.nc, nx = d + nc, ld = d + 1;
  double* s_l = s_dyn;
  double* X = s_dyn + nc;
  const double* v = a.x + d;
  for (int q = threadIdx.x; q < nc; q += blockDim.x) s_l[q] = v[q];
  // chunk sums in chunk order
  for (int q = threadIdx.x; q < nx + 3; q += blockDim.x) {
    double sum = 0.0;
    for (int c = 0; c < chunks; ++c) sum += a.part[size_t(c) * (nx + 3) + q];
    if (q < d) {
      X[q * ld + d] = sum;
    } else if (q < nx) {
      int i, j;
      vi_entry(q, d, i, j);
      X[i * ld + j] = sum;
    } else {
      s_tot[q - nx] = sum;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const int q = i * (i + 1) / 2 + i;
    s_l[q] = exp(s_l[q]);
  }
  __syncthreads();
  // column t: solve L^T x = b from the last row up (rows >= t for the columns of B)
  for (int t = threadIdx.x; t <= d; t += blockDim.x) {
    const int lo = t < d ? t : 0;
    for (int i = d - 1; i >= lo; --i) {
      double x = X[i * ld + t];
      for (int k = i + 1; k < d; ++k) x -= s_l[k * (k + 1) / 2 + i] * X[k * ld + t];
      X[i * ld + t] = x / s_l[i * (i + 1) / 2 + i];
    }
  }
  __syncthreads();
  const double fsum = s_tot[0], nokd = s_tot[1], wsum = s_tot[2];
  const int nok = int(nokd);
  for (int q = threadIdx.x; q < nx; q += blockDim.x) {
    if (nok == 0) {  // no usable sample: keep the state
      a.x_new[q] = a.x[q];
      if (q == 0) a.loss[a.k] = NAN;
      continue;
    }
    int i, j;
    vi_entry(q, d, i, j);
    double gq;
    if (j < 0) {
      gq = X[i * ld + d] / nok;
    } else if (j < i) {
      gq = X[i * ld + j] / nok;
    } else {
      gq = s_l[i * (i + 1) / 2 + i] * X[i * ld + i] / nok - wsum / nok;
    }
    if (q == 0) {
      double logdet = 0.0;
      for (int t = 0; t < d; ++t) logdet += v[t * (t + 1) / 2 + t];
      a.loss[a.k] = fsum / nok - logdet - 0.5 * d * (1.0 + kLog2Pi);
    }
    vi_adam_entry(a, q, gq);
  }
}

// Draws from the surrogate: z_s = mu + L eps_s (FP64), counter (s, j, 0, tag).
__global__ void __launch_bounds__(kViThreads) vi_sample_kernel(ViArgs a, double* z) {
  __shared__ double s_eps[kMaxParams];
  draw_sample(a.x, a.x + a.d, a.d, blockIdx.x, 0, kViSampleTag, a.seed_lo, a.seed_hi, s_eps,
              nullptr, nullptr, z);
}

// Dense L (lower, [d][d]) and Sigma = L L^T ([d][d]); either may be NULL.
__global__ void __launch_bounds__(256) vi_dense_kernel(const double* x, int d, double* chol,
                                                       double* cov) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d * d) return;
  const int i = q / d, j = q - i * d;
  const double* v = x + d;
  if (chol) chol[q] = j <= i ? chol_entry(v, i, j) : 0.0;
  if (cov) {
    double c = 0.0;
    const int kmax = i < j ? i : j;
    for (int k = 0; k <= kmax; ++k) c += chol_entry(v, i, k) * chol_entry(v, j, k);
    cov[q] = c;
  }
}

}  // namespace glens

using namespace glens;


struct gl_vi {
  gl_model* model = nullptr;
  int n = 0, d = 0, nc = 0, K = 0, k = 0, cur = 0, warmup = 0;
  float lr_max = 0.f, lr_final = 0.f;
  int estimator = GL_VI_PATHWISE;
  char* base = nullptr;
  double* x[2] = {nullptr, nullptr};
  ViArgs a{};
  FitBuffers fb;  // holds the priors
};

static int vi_check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GL_OK : set_error(GL_E_DEVICE, "launch: %s", hipGetErrorString(e));
}

static float vi_learning_rate(const gl_vi* v, int k) {
  if (k < v->warmup) {
    const double frac = 1.0 - double(k) / v->warmup;
    return float(v->lr_max * (1.0 - frac * frac));
  }
  const int span = v->K - 1 - v->warmup;
  if (v->lr_final <= 0.f || span <= 0) return v->lr_max;
  const double t = std::min(1.0, double(k - v->warmup) / span);
  return float(double(v->lr_max) * std::pow(double(v->lr_final) / v->lr_max, t));
}

static int vi_iteration(gl_vi* v, hipStream_t st) {
  gl_model* m = v->model;
  const ModelCfg& c = m->sys.cfg;
  const int tiles = choose_tiles(v->n, c.H * c.W);
  int rc = workspace_reserve(m->ws, v->n, tiles, c.H * c.W, c.d, true, beta_per_particle(c));
  if (rc) return rc;
  ViArgs& a = v->a;
  a.k = v->k;
  a.lr = vi_learning_rate(v, v->k);
  a.bc1 = 1.0 - std::pow(double(a.beta1), double(v->k + 1));
  a.bc2 = 1.0 - std::pow(double(a.beta2), double(v->k + 1));
  a.x = v->x[v->cur];
  a.x_new = v->x[1 - v->cur];
  a.logl = m->ws.logl;
  a.grad = m->ws.grad;
  a.theta = m->ws.theta;
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = make_sys(m->sys, m->ws, v->n, tiles);
  g.sys[0].theta = nullptr;
  g.sys[0].z = a.z32;
  g.sys[0].prior = v->fb.prior;
  g.sys[0].theta_out = m->ws.theta;
  g.sys[0].logl = m->ws.logl;
  g.sys[0].grad = m->ws.grad;
  g.sys[0].mode = 2;
  // draw + decode, the pipeline without its first and last stages, finalize + objective
  hipLaunchKernelGGL(vi_draw_decode_kernel, dim3(v->n), dim3(kViThreads), 0, st, g.sys[0], a);
  if ((rc = vi_check_launch())) return rc;
  if ((rc = run_group(g, subpix_key(c), c.K, 2, st, nullptr, false, false))) return rc;
  hipLaunchKernelGGL(vi_finalize_objective_kernel, dim3(v->n), dim3(kViThreads), 0, st,
                     g.sys[0], a);
  if ((rc = vi_check_launch())) return rc;
  const int nx = v->d + v->nc, chunks = (v->n + kViChunk - 1) / kViChunk;
  if (v->estimator == GL_VI_SCORE) {
    const size_t lds = sizeof(double) * (size_t(v->nc) + size_t(v->d) * (v->d + 1));
    hipLaunchKernelGGL(vi_reduce_score_kernel, dim3(chunks), dim3(256), 0, st, a);
    if ((rc = vi_check_launch())) return rc;
    hipLaunchKernelGGL(vi_update_score_kernel, dim3(1), dim3(256), lds, st, a, chunks);
    if ((rc = vi_check_launch())) return rc;
  } else {
    hipLaunchKernelGGL(vi_reduce_kernel, dim3(chunks), dim3(256), 0, st, a);
    if ((rc = vi_check_launch())) return rc;
    hipLaunchKernelGGL(vi_update_kernel, dim3((nx + 255) / 256), dim3(256), 0, st, a, chunks);
    if ((rc = vi_check_launch())) return rc;
  }
  v->cur = 1 - v->cur;
  v->k++;
  return GL_OK;
}

extern "C" {

int gl_vi_create(gl_model* m, const gl_vi_opts* o, const double* mu0, gl_vi** out,
                 void* stream) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!m || !o || !mu0) return set_error(GL_E_INVALID, "NULL argument");
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  if (o->n_samples < 1 || o->K < 1 || o->lr_warmup < 0)
    return set_error(GL_E_INVALID, "need n_samples >= 1, K >= 1, lr_warmup >= 0");
  if (!(o->lr_max >= 0.f) || !std::isfinite(o->lr_max))
    return set_error(GL_E_INVALID, "lr_max must be finite and >= 0");
  if (!(o->lr_final >= 0.f) || !std::isfinite(o->lr_final) ||
      (o->lr_final > 0.f && !(o->lr_max > 0.f)))
    return set_error(GL_E_INVALID, "lr_final must be finite and >= 0 (> 0 needs lr_max > 0)");
  if (!(o->init_sd > 0.f) || !std::isfinite(o->init_sd))
    return set_error(GL_E_INVALID, "init_sd must be > 0");
  if (o->estimator != GL_VI_PATHWISE && o->estimator != GL_VI_SCORE)
    return set_error(GL_E_INVALID, "estimator must be GL_VI_PATHWISE or GL_VI_SCORE");
  const ModelCfg& c = m->sys.cfg;
  const int d = c.d, nc = d * (d + 1) / 2, n = o->n_samples, nx = d + nc;
  gl_fit_opts fo;
  std::memset(&fo, 0, sizeof(fo));
  fo.P = n;
  fo.K = 1;
  fo.priors = o->priors;
  std::vector<Prior> pri;
  int rc = validate_fit_opts(&fo, d, pri);
  if (rc) return rc;
  if ((rc = check_device_ptr(mu0, "mu0"))) return rc;
  gl_vi* v = new (std::nothrow) gl_vi();
  if (!v) return set_error(GL_E_NOMEM, "host allocation failed");
  v->model = m;
  v->n = n;
  v->d = d;
  v->nc = nc;
  v->K = o->K;
  v->warmup = o->lr_warmup;
  v->lr_max = o->lr_max;
  v->lr_final = o->lr_final;
  v->estimator = o->estimator;
  hipStream_t st = (hipStream_t)stream;
  rc = workspace_reserve(m->ws, n, choose_tiles(n, c.H * c.W), c.H * c.W, d, true,
                         beta_per_particle(c));
  if (!rc) rc = fit_buffers_alloc(v->fb, n, d, pri.data());
  const size_t nd = size_t(n) * d;
  const size_t npart = size_t((n + kViChunk - 1) / kViChunk) * (nx + 3);
  const size_t bytes = sizeof(double) * (4 * size_t(nx) + nd + n + o->K + npart) +
                       sizeof(float) * 2 * nd + 256 * 12;
  if (!rc && hipMalloc(&v->base, bytes) != hipSuccess) rc = set_error(GL_E_NOMEM, "hipMalloc failed");
  if (rc) {
    fit_buffers_free(v->fb);
    delete v;
    return rc;
  }
  char* q = v->base;
  auto take = [&](size_t b) {
    char* r = q;
    q += (b + 255) & ~size_t(255);
    return r;
  };
  v->x[0] = reinterpret_cast<double*>(take(sizeof(double) * nx));
  v->x[1] = reinterpret_cast<double*>(take(sizeof(double) * nx));
  ViArgs& a = v->a;
  a.n = n;
  a.d = d;
  a.nc = nc;
  a.prior = v->fb.prior;
  a.m = reinterpret_cast<double*>(take(sizeof(double) * nx));
  a.s = reinterpret_cast<double*>(take(sizeof(double) * nx));
  a.eps = reinterpret_cast<double*>(take(sizeof(double) * nd));
  a.f = reinterpret_cast<double*>(take(sizeof(double) * n));
  a.loss = reinterpret_cast<double*>(take(sizeof(double) * o->K));
  a.part = reinterpret_cast<double*>(take(sizeof(double) * npart));
  a.z32 = reinterpret_cast<float*>(take(sizeof(float) * nd));
  a.g = reinterpret_cast<float*>(take(sizeof(float) * nd));
  const bool defaults = o->beta1 == 0.f && o->beta2 == 0.f && o->eps == 0.f;
  a.beta1 = defaults ? 0.9f : o->beta1;
  a.beta2 = defaults ? 0.999f : o->beta2;
  a.adam_eps = defaults ? 1e-8f : o->eps;
  a.seed_lo = uint32_t(o->seed);
  a.seed_hi = uint32_t(o->seed >> 32);
  // x = (mu0, v) with L = init_sd I: v_ii = log(init_sd), off-diagonal 0; moments 0
  std::vector<double> x0(nx, 0.0);
  for (int i = 0; i < d; ++i) x0[d + i * (i + 1) / 2 + i] = std::log(double(o->init_sd));
  std::vector<double> zero(nx, 0.0), nan_loss(o->K, NAN);
  bool ok = hipMemcpy(v->x[0] + d, x0.data() + d, sizeof(double) * nc, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.m, zero.data(), sizeof(double) * nx, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.s, zero.data(), sizeof(double) * nx, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.loss, nan_loss.data(), sizeof(double) * o->K, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpyAsync(v->x[0], mu0, sizeof(double) * d, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (!ok) {
    (void)hipFree(v->base);
    fit_buffers_free(v->fb);
    delete v;
    return set_error(GL_E_DEVICE, "upload failed");
  }
  *out = v;
  return GL_OK;
}

int gl_vi_destroy(gl_vi* v) {
  clear_error();
  if (!v) return GL_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(v->base);
  fit_buffers_free(v->fb);
  delete v;
  return GL_OK;
}

int gl_vi_step(gl_vi* v, int n, void* stream) {
  clear_error();
  if (!v) return set_error(GL_E_INVALID, "state is NULL");
  if (n < 0 || v->k + n > v->K)
    return set_error(GL_E_INVALID, "%d iterations requested, %d left", n, v->K - v->k);
  for (int i = 0; i < n; ++i) {
    int rc = vi_iteration(v, (hipStream_t)stream);
    if (rc) return rc;
  }
  return GL_OK;
}

int gl_vi_get(gl_vi* v, double* mu, double* chol, double* cov, void* stream) {
  clear_error();
  if (!v) return set_error(GL_E_INVALID, "state is NULL");
  int rc;
  if ((mu && (rc = check_device_ptr(mu, "mu"))) || (chol && (rc = check_device_ptr(chol, "chol"))) ||
      (cov && (rc = check_device_ptr(cov, "cov"))))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const double* x = v->x[v->cur];
  if (mu) GL_HIP(hipMemcpyAsync(mu, x, sizeof(double) * v->d, hipMemcpyDeviceToDevice, st));
  if (chol || cov) {
    const int dd = v->d * v->d;
    hipLaunchKernelGGL(vi_dense_kernel, dim3((dd + 255) / 256), dim3(256), 0, st, x, v->d, chol,
                       cov);
    if ((rc = vi_check_launch())) return rc;
  }
  return GL_OK;
}

int gl_vi_sample(gl_vi* v, int n, uint64_t seed, double* z, void* stream) {
  clear_error();
  if (!v) return set_error(GL_E_INVALID, "state is NULL");
  if (n < 0) return set_error(GL_E_INVALID, "n must be >= 0");
  if (n == 0) return GL_OK;
  int rc = check_device_ptr(z, "z");
  if (rc) return rc;
  ViArgs a = v->a;
  a.x = v->x[v->cur];
  a.seed_lo = uint32_t(seed);
  a.seed_hi = uint32_t(seed >> 32);
  hipLaunchKernelGGL(vi_sample_kernel, dim3(n), dim3(kViThreads), 0, (hipStream_t)stream, a, z);
  return vi_check_launch();
}

int gl_vi_get_state(gl_vi* v, double* x, double* m, double* s, int* k, double* loss,
                    void* stream) {
  clear_error();
  if (!v) return set_error(GL_E_INVALID, "state is NULL");
  int rc;
  if ((x && (rc = check_device_ptr(x, "x"))) || (m && (rc = check_device_ptr(m, "m"))) ||
      (s && (rc = check_device_ptr(s, "s"))) || (loss && (rc = check_device_ptr(loss, "loss"))))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t b = sizeof(double) * (v->d + v->nc);
  if (x) GL_HIP(hipMemcpyAsync(x, v->x[v->cur], b, hipMemcpyDeviceToDevice, st));
  if (m) GL_HIP(hipMemcpyAsync(m, v->a.m, b, hipMemcpyDeviceToDevice, st));
  if (s) GL_HIP(hipMemcpyAsync(s, v->a.s, b, hipMemcpyDeviceToDevice, st));
  if (loss) GL_HIP(hipMemcpyAsync(loss, v->a.loss, sizeof(double) * v->K, hipMemcpyDeviceToDevice, st));
  if (k) *k = v->k;
  return GL_OK;
}

int gl_vi_set_state(gl_vi* v, const double* x, const double* m, const double* s, int k,
                    void* stream) {
  clear_error();
  if (!v) return set_error(GL_E_INVALID, "state is NULL");
  if (k < 0 || k > v->K) return set_error(GL_E_INVALID, "k must be in [0, K]");
  int rc;
  if ((rc = check_device_ptr(x, "x")) || (rc = check_device_ptr(m, "m")) ||
      (rc = check_device_ptr(s, "s")))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t b = sizeof(double) * (v->d + v->nc);
  GL_HIP(hipMemcpyAsync(v->x[v->cur], x, b, hipMemcpyDeviceToDevice, st));
  GL_HIP(hipMemcpyAsync(v->a.m, m, b, hipMemcpyDeviceToDevice, st));
  GL_HIP(hipMemcpyAsync(v->a.s, s, b, hipMemcpyDeviceToDevice, st));
  v->k = k;
  return GL_OK;
}

}  // extern "C"
