// Preconditioned Hamiltonian Monte Carlo over many chains (Sec. 2.5): the gl_hmc* C ABI.
//
// Target: log p~(z | I) = log L(g(z)) + log p~(z) in unconstrained space (Sec. 2.2), with
// the gradient from the likelihood pipeline plus the prior / bijector terms. Each chain
// runs, per trajectory:
//   p ~ N(0, M);  half kick, then L drifts z += eps M^-1 p separated by full kicks, and a
//   final half kick (leapfrog);  accept with probability min(1, e^(H0 - H1)),
//   H = -log p~(z | I) + p^T M^-1 p / 2.
// M^-1 = S is given by its lower Cholesky factor S = C C^T (the paper takes M as the inverse
// of the variational covariance, so C is that covariance's factor): p = C^-T n with
// n ~ N(0, I), p^T S p / 2 = |C^T p|^2 / 2 and the drift applies C (C^T p).
// During the first adapt_frac of burn-in the step size follows Hoffman & Gelman's dual
// averaging towards target_accept (the paper uses 0.75 over the first 80% of burn-in); it
// is then fixed at the averaged value. With mass adaptation (not in the paper), M^-1 is
// re-estimated inside the same adaptation window from the chains' positions over three
// windows of trajectories, each twice as long as the one before, between an initial buffer
// (15% of the window) and a terminal one (10%), the estimate of each replacing the factor
// and restarting the step-size averaging. Every chain is one particle of the likelihood launch,
// so a leapfrog step costs one batched gradient call over all chains; the pipeline's last
// stage (finalize), the kick and drift and the next step's decode (prologue) run fused in
// one per-chain kernel, so that a step after the first launches the sub-pixel forward pass,
// the PSF pass, the sub-pixel adjoint and that kernel. The per-chain kernels run one 64-lane
// block per chain with the chain's d <= 68 coordinates in LDS. The trajectory counter lives
// in device memory, so a trajectory's launches do not change between trajectories.
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

constexpr int kHmcThreads = 64;

struct HmcArgs {
  int C, d;
  int n_burn, n_adapt;
  float target;
  float eps_fixed;     // > 0: use this step size instead of the adapted one
  const Prior* prior;
  const float* chol;   // [d][d] row-major lower factor of M^-1
  const float* chol_it;// [d][d] row-major (chol^-1)^T, upper triangular
  int* traj;           // index of the current trajectory (device scalar)
  double* z;           // [C][d] position (unconstrained), FP64 so that many small drifts
                       // accumulate without rounding (posterior widths can be ~1e-6 of |z|)
  float* z32;          // [C][d] FP32 copy of z read by the likelihood pipeline
  float* p;            // [C][d] momentum
  float* g;            // [C][d] d log p~(z | I) / dz
  double* lp;          // [C] log p~(z | I)
  double* zs;          // [C][d] trajectory start
  float* gs;
  double* lps;
  double* k0;          // [C] kinetic energy at the start
  int* bad;            // [C] a non-finite log posterior was met along the trajectory
  const double* logl;  // [C] from the likelihood pipeline
  const float* grad;   // [C][d] d log L / d theta from the pipeline
  const float* theta;  // [C][d] g(z) from the prologue
  float* eps;          // adapted step size (device scalar)
  double* da;          // dual averaging: mu, h, log_eps_bar, m
  float* accept;       // [C] acceptance probability of the last trajectory
  double* stats;       // sum of the chain-mean acceptance over sampled trajectories, count
  float* samples;      // [n_samples][C][d] physical parameters
  uint32_t seed_lo, seed_hi;
  // trajectory-length adaptation (ChEES)
  int adapt_len;       // 1: adapt T during the first n_adapt trajectories
  float u;             // jitter of the current trajectory (t = u T)
  float* T;            // trajectory length (device scalar)
  double* la;          // log T, Adam second moment, update count, averaged log T
  double* zbar;        // [2][d] chain means of the starts and of the proposals
  double* cg;          // [C] ChEES gradient term of each chain
  // mass adaptation
  double* mom;         // moments of the current window: [0] count, [1 + i] sum of
                       // (z - zref)_i, [1 + d + i d + j] sum of (z - zref)_i (z - zref)_j
  double* zref;        // [d] shift of those sums (chain 0's position at the window start),
                       // so that they hold deviations of the posterior's width, not of |z|
};

__device__ __forceinline__ float step_size(const HmcArgs& a) {
  return a.eps_fixed > 0.f ? a.eps_fixed : *a.eps;
}

// Copies the d x d factor m to LDS (the per-chain products read every entry in dependent
// chains, where LDS reads wait far less than L2 ones); the caller synchronises the block.
__device__ __forceinline__ void stage_factor(const float* m, int d, float* s_m) {
  for (int q = threadIdx.x; q < d * d; q += kHmcThreads) s_m[q] = m[q];
}

// v = chol^T x for one chain (chol, x in LDS, v to LDS); lanes own output coordinates.
__device__ __forceinline__ void chol_t_times(const float* chol, int d, const float* x, float* v) {
  for (int j = threadIdx.x; j < d; j += kHmcThreads) {
    float s = 0.f;
#pragma unroll 4
    for (int i = j; i < d; ++i) s += chol[i * d + j] * x[i];
    v[j] = s;
  }
}

// p += scale eps g (scale 0: no kick); then, if drift, z += eps chol (chol^T p). p is
// mirrored in s_p. One block per chain; the caller has synchronised the block.
__device__ __forceinline__ void kick_drift(const HmcArgs& a, const float* s_g, float scale,
                                           int drift, float* s_p, float* s_v) {
  const int c = blockIdx.x;
  const float eps = step_size(a);
  const size_t row = size_t(c) * a.d;
  if (scale != 0.f) {
    for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
      const float pn = a.p[row + j] + scale * eps * s_g[j];
      a.p[row + j] = pn;
      s_p[j] = pn;
    }
  }
  if (!drift) return;
  __shared__ float s_chol[kMaxParams * kMaxParams];
  stage_factor(a.chol, a.d, s_chol);
  __syncthreads();
  chol_t_times(s_chol, a.d, s_p, s_v);
  __syncthreads();
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    float s = 0.f;
#pragma unroll 4
    for (int i = 0; i <= j; ++i) s += s_chol[j * a.d + i] * s_v[i];
    const double zn = a.z[row + j] + double(eps) * s;
    a.z[row + j] = zn;
    a.z32[row + j] = float(zn);
  }
}

// log p~(z | I) and its gradient from the pipeline outputs (terms summed in parameter
// order by lane 0), then the kick and drift of the leapfrog step.
__device__ __forceinline__ void grad_move(const HmcArgs& a, float scale, int drift) {
  __shared__ double s_t[kMaxParams];
  __shared__ float s_g[kMaxParams], s_p[kMaxParams], s_v[kMaxParams];
  __shared__ int s_bad;
  const int c = blockIdx.x;
  const size_t row = size_t(c) * a.d;
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    float dlp, dth;
    s_t[j] = log_prior_z(a.prior[j], a.z32[row + j], a.theta[row + j], dlp, dth);
    s_g[j] = a.grad[row + j] * dth + dlp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lp = a.logl[c];
    for (int j = 0; j < a.d; ++j) lp += s_t[j];
    const int bad = !isfinite(lp);
    if (bad) {
      lp = -INFINITY;
      a.bad[c] = 1;
    }
    a.lp[c] = lp;
    s_bad = bad;
  }
  __syncthreads();
  const int bad = s_bad;
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    if (bad) s_g[j] = 0.f;
    a.g[row + j] = s_g[j];
  }
  kick_drift(a, s_g, scale, drift, s_p, s_v);
}

// One block per chain: the pipeline's finalize (log L and its gradient), log p~ and its
// gradient, the kick and, with a drift, the decode of the new position for the next step's
// pipeline (prologue), which then starts at the sub-pixel forward pass. Two launches fewer
// per leapfrog step than finalize, kick/drift and prologue apart, with the same arithmetic.
__global__ void __launch_bounds__(kHmcThreads) hmc_finalize_move_kernel(SysDesc s, HmcArgs a,
                                                                        float scale, int drift) {
  finalize_particle(s, blockIdx.x);
  __syncthreads();  // this chain's log L and gradient are written
  grad_move(a, scale, drift);
  if (!drift) return;
  __syncthreads();  // this chain's new position is written
  prologue_particle(s, blockIdx.x);
}

// New momentum p = chol^-T n, saved trajectory start and kinetic energy |n|^2 / 2, then the
// first half kick and drift.
__global__ void __launch_bounds__(kHmcThreads) hmc_begin_kernel(HmcArgs a) {
  __shared__ float s_n[kMaxParams], s_g[kMaxParams], s_p[kMaxParams], s_v[kMaxParams];
  __shared__ float s_cit[kMaxParams * kMaxParams];
  const int c = blockIdx.x;
  const int traj = *a.traj;
  const size_t row = size_t(c) * a.d;
  stage_factor(a.chol_it, a.d, s_cit);
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    uint32_t w[4] = {uint32_t(c), uint32_t(j), uint32_t(traj), 0x6d6f6d65u};
    philox4x32_10(w, a.seed_lo, a.seed_hi);
    const double u1 = u01(w[0], w[1]), u2 = u01(w[2], w[3]);
    s_n[j] = float(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    a.zs[row + j] = a.z[row + j];
    s_g[j] = a.gs[row + j] = a.g[row + j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.d; i += kHmcThreads) {
    float s = 0.f;
    for (int j = i; j < a.d; ++j) s += s_cit[i * a.d + j] * s_n[j];
    a.p[row + i] = s;
  }
  if (threadIdx.x == 0) {
    double k = 0.0;
    for (int j = 0; j < a.d; ++j) k += 0.5 * double(s_n[j]) * s_n[j];
    a.k0[c] = k;
    a.lps[c] = a.lp[c];
    a.bad[c] = 0;
  }
  __syncthreads();
  kick_drift(a, s_g, 0.5f, 1, s_p, s_v);
}

// Chain means of the trajectory starts and of the proposals (one lane per parameter, chains
// in order), for the ChEES gradient.
__global__ void __launch_bounds__(kHmcThreads) hmc_mean_kernel(HmcArgs a) {
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    double m0 = 0.0, m1 = 0.0;
    for (int c = 0; c < a.C; ++c) {
      m0 += a.zs[size_t(c) * a.d + j];
      m1 += a.z[size_t(c) * a.d + j];
    }
    a.zbar[j] = m0 / a.C;
    a.zbar[a.d + j] = m1 / a.C;
  }
}

// Metropolis accept / reject and the sample record.
__global__ void __launch_bounds__(kHmcThreads) hmc_finish_kernel(HmcArgs a) {
  __shared__ float s_p[kMaxParams], s_v[kMaxParams];
  __shared__ double s_w[kMaxParams];
  __shared__ int s_keep;
  const int c = blockIdx.x;
  const int traj = *a.traj;
  const size_t row = size_t(c) * a.d;
  __shared__ float s_chol[kMaxParams * kMaxParams];
  stage_factor(a.chol, a.d, s_chol);
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) s_p[j] = a.p[row + j];
  __syncthreads();
  chol_t_times(s_chol, a.d, s_p, s_v);
  __syncthreads();
  const bool chees = a.adapt_len && traj < a.n_adapt;
  if (chees) {  // per coordinate: (z' - zbar')_j (M^-1 p')_j, M^-1 p' = chol (chol^T p')
    for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
      float v = 0.f;
      for (int i = 0; i <= j; ++i) v += s_chol[j * a.d + i] * s_v[i];
      s_w[j] = (a.z[row + j] - a.zbar[a.d + j]) * double(v);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double k1 = 0.0;
    for (int j = 0; j < a.d; ++j) k1 += 0.5 * double(s_v[j]) * s_v[j];
    if (chees) {  // (|z' - zbar'|^2 - |z - zbar|^2) ((z' - zbar') . M^-1 p') u
      double d1 = 0.0, d0 = 0.0, dot = 0.0;
      for (int j = 0; j < a.d; ++j) {
        const double e1 = a.z[row + j] - a.zbar[a.d + j], e0 = a.zs[row + j] - a.zbar[j];
        d1 += e1 * e1;
        d0 += e0 * e0;
        dot += s_w[j];
      }
      const double gc = (d1 - d0) * dot * a.u;
      a.cg[c] = isfinite(gc) ? gc : 0.0;
    }
    const double h0 = -a.lps[c] + a.k0[c], h1 = -a.lp[c] + k1;
    double acc = exp(fmin(0.0, h0 - h1));
    if (a.bad[c] || !isfinite(h1) || !isfinite(acc)) acc = 0.0;
    uint32_t w[4] = {uint32_t(c), 0xffffffffu, uint32_t(traj), 0x61636370u};
    philox4x32_10(w, a.seed_lo, a.seed_hi);
    const int keep = u01(w[0], w[1]) < acc;
    if (!keep) a.lp[c] = a.lps[c];
    a.accept[c] = float(acc);
    s_keep = keep;
  }
  __syncthreads();
  const int keep = s_keep;
  float* out = a.samples && traj >= a.n_burn ? a.samples + (size_t(traj - a.n_burn) * a.C + c) * a.d
                                             : nullptr;
  for (int j = threadIdx.x; j < a.d; j += kHmcThreads) {
    if (!keep) {
      const double zj = a.zs[row + j];
      a.z[row + j] = zj;
      a.z32[row + j] = float(zj);
      a.g[row + j] = a.gs[row + j];
    }
    if (out) out[j] = bijector_fwd(a.prior[j], a.z32[row + j]);
  }
}

// Step-size adaptation (one lane, after every chain's accept): dual averaging on the
// chain-mean acceptance probability; then the trajectory counter advances.
__global__ void hmc_adapt_kernel(HmcArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int traj = *a.traj;
  double mean = 0.0;
  for (int c = 0; c < a.C; ++c) mean += a.accept[c];
  mean /= a.C;
  if (traj < a.n_adapt) {
    const double t0 = 10.0, gamma = 0.05, kappa = 0.75;
    const double m = a.da[3] + 1.0;
    const double w = 1.0 / (m + t0);
    const double h = (1.0 - w) * a.da[1] + w * (a.target - mean);
    // kept within e^+-40 of mu so that a run of rejections cannot underflow eps to zero
    const double log_eps = fmin(fmax(a.da[0] - sqrt(m) / gamma * h, a.da[0] - 40.0), a.da[0] + 40.0);
    const double eta = pow(m, -kappa);
    a.da[1] = h;
    a.da[2] = eta * log_eps + (1.0 - eta) * a.da[2];
    a.da[3] = m;
    *a.eps = float(traj + 1 == a.n_adapt ? exp(a.da[2]) : exp(log_eps));
  }
  if (a.adapt_len && traj < a.n_adapt) {
    // ChEES: acceptance-weighted mean gradient w.r.t. T, then Adam (beta1 = 0, beta2 =
    // 0.95, rate 0.025) ascending in log T; the averaged log T uses the weights m^-kappa
    // A chain with acceptance probability 0 has weight 0: it is left out, so that a far
    // (rejected) proposal cannot turn the sum into 0 x inf.
    double num = 0.0, den = 0.0;
    for (int c = 0; c < a.C; ++c) {
      if (!(a.accept[c] > 0.f)) continue;
      num += double(a.accept[c]) * a.cg[c];
      den += a.accept[c];
    }
    const double g = den > 0.0 ? num / den * exp(a.la[0]) : 0.0;
    if (den > 0.0 && isfinite(g * g)) {
      const double m = a.la[2] + 1.0;
      const double v = 0.95 * a.la[1] + 0.05 * g * g;
      const double vhat = v / (1.0 - pow(0.95, m));
      const double logT = a.la[0] + 0.025 * g / (sqrt(vhat) + 1e-8);
      const double eta = pow(m, -0.75);
      a.la[0] = logT;
      a.la[1] = v;
      a.la[2] = m;
      a.la[3] = eta * logT + (1.0 - eta) * a.la[3];
    }
    *a.T = float(traj + 1 == a.n_adapt ? exp(a.la[3]) : exp(a.la[0]));
  }
  if (traj >= a.n_burn) {
    a.stats[0] += mean;
    a.stats[1] += 1.0;
  }
  *a.traj = traj + 1;
}

// Mass adaptation: clear the window's moments and take chain 0's position as their shift.
__global__ void __launch_bounds__(256) hmc_window_start_kernel(HmcArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < 1 + a.d + a.d * a.d) a.mom[q] = 0.0;
  if (q < a.d) a.zref[q] = a.z[q];
}

// Mass adaptation: add the chains' positions after this trajectory's accept to the window's
// moments (one lane per entry, chains in order).
__global__ void __launch_bounds__(256) hmc_moments_kernel(HmcArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.d * a.d) return;
  const int i = q / a.d, j = q - i * a.d;
  const double ri = a.zref[i], rj = a.zref[j];
  double s = 0.0, s1 = 0.0;
  for (int c = 0; c < a.C; ++c) {
    const double ei = a.z[size_t(c) * a.d + i] - ri;
    s += ei * (a.z[size_t(c) * a.d + j] - rj);
    s1 += ei;
  }
  a.mom[1 + a.d + q] += s;
  if (j == 0) a.mom[1 + i] += s1;
  if (q == 0) a.mom[0] += a.C;
}

// Starts drawn from the prior when the caller gives none.
__global__ void __launch_bounds__(256) hmc_start_kernel(HmcArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.C * a.d) return;
  const int c = i / a.d, j = i - c * a.d;
  const float z = draw_start(a.prior[j], a.seed_lo ^ 0x5eedu, a.seed_hi, c, j);
  a.z[i] = z;
  a.z32[i] = z;
}

// FP32 copy of caller-supplied positions.
__global__ void __launch_bounds__(256) hmc_round_kernel(HmcArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.C * a.d) a.z32[i] = float(a.z[i]);
}

}  // namespace glens

using namespace glens;


struct gl_hmc {
  gl_model* model = nullptr;
  int C = 0, d = 0, L = 1, n_burn = 0, n_samples = 0, n_adapt = 0, done = 0;
  int max_leapfrog = 1000;
  long long leapfrogs = 0;  // leapfrog steps run by gl_hmc_run
  float T_fixed = 0.f, eps_fixed = 0.f;  // cached once adaptation has ended
  float T0 = 0.f, eps0 = 0.f;            // the values before the first update
  // mass adaptation: window k takes the positions after trajectories [win[k], win[k + 1])
  std::vector<int> win;
  int mass_updates = 0;
  float* chol_d = nullptr;
  float* chol_it_d = nullptr;
  bool pc_ready = false;  // the chains' particle constants are those of their current z
  float* te_host = nullptr;  // pinned: (T, eps) after trajectory j's update, in slot j & 1
  hipEvent_t te_ev[2] = {nullptr, nullptr};  // the copies into each slot
  float target = 0.75f;
  uint64_t seed = 0;
  char* base = nullptr;
  HmcArgs a{};
  FitBuffers fb;  // holds the priors (and unused fit arrays)
};

static void hmc_free(gl_hmc* h) {
  if (h->base) (void)hipFree(h->base);
  if (h->te_host) (void)hipHostFree(h->te_host);
  for (hipEvent_t e : h->te_ev)
    if (e) (void)hipEventDestroy(e);
  fit_buffers_free(h->fb);
  delete h;
}

static int hmc_launch1(void (*k)(HmcArgs), const HmcArgs& a, int n, int threads, hipStream_t st) {
  hipLaunchKernelGGL(k, dim3((n + threads - 1) / threads), dim3(threads), 0, st, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GL_OK : set_error(GL_E_DEVICE, "launch: %s", hipGetErrorString(e));
}


// Lower Cholesky factor of the symmetric matrix s [d][d] (row-major, double); false unless
// positive definite.
static bool cholesky(std::vector<double>& s, int d) {
  for (int j = 0; j < d; ++j) {
    double diag = s[j * d + j];
    for (int k = 0; k < j; ++k) diag -= s[j * d + k] * s[j * d + k];
    if (!(diag > 0.0) || !std::isfinite(diag)) return false;
    const double ljj = std::sqrt(diag);
    s[j * d + j] = ljj;
    for (int i = j + 1; i < d; ++i) {
      double v = s[i * d + j];
      for (int k = 0; k < j; ++k) v -= s[i * d + k] * s[j * d + k];
      s[i * d + j] = v / ljj;
    }
    for (int k = j + 1; k < d; ++k) s[j * d + k] = 0.0;
  }
  return true;
}

// Transposed inverse of the lower-triangular l [d][d] (upper triangular result).
static std::vector<double> inverse_transpose_lower(const std::vector<double>& l, int d) {
  std::vector<double> inv(size_t(d) * d, 0.0);  // inv = l^-1, lower triangular
  for (int c = 0; c < d; ++c) {  // solve l x = e_c by forward substitution
    for (int i = c; i < d; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= l[i * d + k] * inv[k * d + c];
      inv[i * d + c] = v / l[i * d + i];
    }
  }
  std::vector<double> t(size_t(d) * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) t[i * d + j] = inv[j * d + i];
  return t;
}

// Window boundaries of the mass adaptation over n_adapt trajectories: an initial buffer of
// 15%, three windows in the ratio 1 : 2 : 4, a terminal buffer of 10% (no windows when the
// middle part is under 7 trajectories).
static std::vector<int> mass_windows(int n_adapt) {
  const int b0 = int(0.15 * n_adapt), b1 = int(0.10 * n_adapt);
  const int span = n_adapt - b0 - b1;
  if (span < 7) return {};
  return {b0, b0 + span / 7, b0 + (3 * span) / 7, b0 + span};
}

// End of a mass-adaptation window: M^-1 from the window's moments (the sample covariance
// with its off-diagonal entries shrunk by n / (n + 5) towards its diagonal), factored on the
// host; the step-size averaging restarts from the current step size. The factor is kept
// when the estimate is not positive definite (e.g. a coordinate that never moved).
static int hmc_update_mass(gl_hmc* h, hipStream_t st) {
  const int d = h->d;
  const size_t nm = 1 + size_t(d) + size_t(d) * d;
  std::vector<double> mom(nm);
  float eps = 0.f;
  GL_HIP(hipMemcpyAsync(mom.data(), h->a.mom, sizeof(double) * nm, hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(&eps, h->a.eps, sizeof(float), hipMemcpyDeviceToHost, st));
  GL_HIP(hipStreamSynchronize(st));
  const double n = mom[0];
  if (!(n >= 2.0)) return GL_OK;
  std::vector<double> S(size_t(d) * d);
  const double shrink = n / (n + 5.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double mi = mom[1 + i] / n, mj = mom[1 + j] / n;
      const double cv = (mom[1 + d + size_t(i) * d + j] - n * mi * mj) / (n - 1.0);
      S[size_t(i) * d + j] = i == j ? cv : shrink * cv;
    }
  if (!cholesky(S, d)) return GL_OK;
  const std::vector<double> SIT = inverse_transpose_lower(S, d);
  const std::vector<float> chol(S.begin(), S.end()), chol_it(SIT.begin(), SIT.end());
  const double da0[4] = {std::log(10.0 * double(eps)), 0.0, 0.0, 0.0};
  GL_HIP(hipMemcpyAsync(h->chol_d, chol.data(), sizeof(float) * d * d, hipMemcpyHostToDevice, st));
  GL_HIP(hipMemcpyAsync(h->chol_it_d, chol_it.data(), sizeof(float) * d * d,
                        hipMemcpyHostToDevice, st));
  GL_HIP(hipMemcpyAsync(h->a.da, da0, sizeof(da0), hipMemcpyHostToDevice, st));
  GL_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
  h->mass_updates++;
  return GL_OK;
}

// log p~(z | I) and its gradient at the chains' current positions, then a leapfrog kick
// of scale eps (scale 0: none) and, if drift, a drift.
static int hmc_gradient(gl_hmc* h, float scale, int drift, hipStream_t st) {
  gl_model* m = h->model;
  const ModelCfg& c = m->sys.cfg;
  const int tiles = choose_tiles(h->C, c.H * c.W);
  // Another call on the model may have regrown its workspace: reserve and re-read.
  const PConst* pc_before = m->ws.pc;
  int rc = workspace_reserve(m->ws, h->C, tiles, c.H * c.W, c.d, true, beta_per_particle(c));
  if (rc) return rc;
  if (m->ws.pc != pc_before) h->pc_ready = false;
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = make_sys(m->sys, m->ws, h->C, tiles);
  g.sys[0].theta = nullptr;
  g.sys[0].z = h->a.z32;
  g.sys[0].prior = h->fb.prior;
  g.sys[0].theta_out = m->ws.theta;
  g.sys[0].logl = m->ws.logl;
  g.sys[0].grad = m->ws.grad;
  h->a.logl = m->ws.logl;
  h->a.grad = m->ws.grad;
  h->a.theta = m->ws.theta;
  // the previous step's fused kernel decoded the current positions unless pc_ready is false
  rc = run_group(g, subpix_key(c), c.K, 2, st, nullptr, !h->pc_ready, false);
  h->pc_ready = false;
  if (rc) return rc;
  hipLaunchKernelGGL(hmc_finalize_move_kernel, dim3(h->C), dim3(kHmcThreads), 0, st, g.sys[0],
                     h->a, scale, drift);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GL_E_DEVICE, "launch: %s", hipGetErrorString(e));
  h->pc_ready = drift != 0;
  return GL_OK;
}

// van der Corput sequence in base 2: the jitter of trajectory k (k >= 1).
static double halton2(long long k) {
  double f = 1.0, r = 0.0;
  while (k > 0) {
    f *= 0.5;
    r += f * double(k & 1);
    k >>= 1;
  }
  return r;
}

static int hmc_trajectory(gl_hmc* h, hipStream_t st) {
  HmcArgs& a = h->a;
  int L = h->L;
  if (a.adapt_len) {
    // L = ceil(u T / eps) with the jitter u shared by all chains. T and eps adapt on the
    // device; trajectory k takes them as they stood after trajectory k - 2's update (the
    // initial values for k < 2). Each update is copied to pinned memory behind it, so the
    // host waits only for a trajectory that is over while the next one is already queued,
    // and the stream never drains between trajectories.
    float T = h->T_fixed, eps = h->eps_fixed;
    if (!(T > 0.f)) {
      const int j = std::min(h->done - 2, h->n_adapt - 1);  // the last update that counts
      if (j < 0) {
        T = h->T0;
        eps = h->eps0;
      } else {
        const int slot = j & 1;
        GL_HIP(hipEventSynchronize(h->te_ev[slot]));
        T = h->te_host[2 * slot];
        eps = h->te_host[2 * slot + 1];
        if (j == h->n_adapt - 1) {  // the final values
          h->T_fixed = T;
          h->eps_fixed = eps;
        }
      }
    }
    const double u = halton2(h->done + 1);
    a.u = float(u);
    const double steps = std::ceil(u * double(T) / double(eps));
    L = int(std::min(double(h->max_leapfrog), std::max(1.0, std::isfinite(steps) ? steps : 1.0)));
  }
  h->leapfrogs += L;
  h->pc_ready = false;  // the first half step drifts the positions
  int rc = hmc_launch1(hmc_begin_kernel, a, a.C * kHmcThreads, kHmcThreads, st);
  for (int l = 0; !rc && l < L; ++l)
    rc = hmc_gradient(h, l + 1 < L ? 1.0f : 0.5f, l + 1 < L, st);
  if (!rc && a.adapt_len && h->done < h->n_adapt)
    rc = hmc_launch1(hmc_mean_kernel, a, kHmcThreads, kHmcThreads, st);
  if (!rc) rc = hmc_launch1(hmc_finish_kernel, a, a.C * kHmcThreads, kHmcThreads, st);
  if (!rc) rc = hmc_launch1(hmc_adapt_kernel, a, 1, 64, st);
  for (size_t k = 0; !rc && k + 1 < h->win.size(); ++k) {
    if (h->done < h->win[k] || h->done >= h->win[k + 1]) continue;
    if (h->done == h->win[k])
      rc = hmc_launch1(hmc_window_start_kernel, a, 1 + a.d + a.d * a.d, 256, st);
    if (!rc) rc = hmc_launch1(hmc_moments_kernel, a, a.d * a.d, 256, st);
    if (!rc && h->done + 1 == h->win[k + 1]) rc = hmc_update_mass(h, st);
  }
  if (!rc && a.adapt_len && h->done < h->n_adapt) {  // this trajectory updated T and eps
    const int slot = h->done & 1;
    GL_HIP(hipMemcpyAsync(h->te_host + 2 * slot, a.T, sizeof(float), hipMemcpyDeviceToHost, st));
    GL_HIP(hipMemcpyAsync(h->te_host + 2 * slot + 1, a.eps, sizeof(float), hipMemcpyDeviceToHost,
                          st));
    GL_HIP(hipEventRecord(h->te_ev[slot], st));
  }
  if (!rc) h->done++;
  return rc;
}

extern "C" {

int gl_hmc_create(gl_model* m, const gl_hmc_opts* o, const double* z0, gl_hmc** out,
                  void* stream) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!m || !o) return set_error(GL_E_INVALID, "NULL argument");
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  if (o->chains < 1 || o->n_leapfrog < 1 || o->n_burn < 0 || o->n_samples < 0)
    return set_error(GL_E_INVALID, "need chains >= 1, n_leapfrog >= 1, n_burn, n_samples >= 0");
  if (!(o->step_size > 0.f) || !std::isfinite(o->step_size))
    return set_error(GL_E_INVALID, "step_size must be > 0");
  if (!(o->target_accept > 0.f && o->target_accept < 1.f))
    return set_error(GL_E_INVALID, "target_accept must be in (0, 1)");
  if (!(o->adapt_frac >= 0.f && o->adapt_frac <= 1.f))
    return set_error(GL_E_INVALID, "adapt_frac must be in [0, 1]");
  if (o->adapt_mass != 0 && o->adapt_mass != 1)
    return set_error(GL_E_INVALID, "adapt_mass must be 0 or 1");
  const ModelCfg& c = m->sys.cfg;
  const int C = o->chains, d = c.d;
  gl_fit_opts fo;
  std::memset(&fo, 0, sizeof(fo));
  fo.P = C;
  fo.K = 1;
  fo.priors = o->priors;
  std::vector<Prior> pri;
  int rc = validate_fit_opts(&fo, d, pri);
  if (rc) return rc;
  // M^-1 = S = chol chol^T (identity, diagonal, dense or given as its factor), factored in
  // double on the host.
  const int form = o->inv_mass ? o->inv_mass_form : GL_MASS_DIAG;
  if (form != GL_MASS_DIAG && form != GL_MASS_DENSE && form != GL_MASS_CHOL)
    return set_error(GL_E_INVALID, "unknown inv_mass_form %d", form);
  std::vector<double> S(size_t(d) * d, 0.0);
  if (form == GL_MASS_DIAG) {
    for (int j = 0; j < d; ++j) S[size_t(j) * d + j] = o->inv_mass ? o->inv_mass[j] : 1.0;
  } else {
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const double v = o->inv_mass[i * d + j], vt = o->inv_mass[j * d + i];
        if (form == GL_MASS_CHOL) {
          if (j <= i && !std::isfinite(v)) return set_error(GL_E_INVALID, "inv_mass must be finite");
          S[size_t(i) * d + j] = j <= i ? v : 0.0;
        } else {
          if (!std::isfinite(v) || std::fabs(v - vt) > 1e-6 * (std::fabs(v) + std::fabs(vt)))
            return set_error(GL_E_INVALID, "inv_mass must be finite and symmetric");
          S[size_t(i) * d + j] = v;
        }
      }
  }
  if (form == GL_MASS_CHOL) {
    for (int i = 0; i < d; ++i)
      if (!(S[size_t(i) * d + i] > 0.0))
        return set_error(GL_E_INVALID, "the Cholesky factor needs a positive diagonal");
  } else if (!cholesky(S, d)) {
    return set_error(GL_E_INVALID, "inv_mass must be positive definite");
  }
  const std::vector<double> SIT = inverse_transpose_lower(S, d);
  std::vector<float> chol(S.begin(), S.end()), chol_it(SIT.begin(), SIT.end());
  if (z0 && (rc = check_device_ptr(z0, "z0"))) return rc;
  gl_hmc* h = new (std::nothrow) gl_hmc();
  if (!h) return set_error(GL_E_NOMEM, "host allocation failed");
  h->model = m;
  h->C = C;
  h->d = d;
  h->L = o->n_leapfrog;
  h->n_burn = o->n_burn;
  h->n_samples = o->n_samples;
  h->n_adapt = int(std::floor(double(o->adapt_frac) * o->n_burn));
  h->target = o->target_accept;
  if (o->adapt_mass) h->win = mass_windows(h->n_adapt);
  hipStream_t st = (hipStream_t)stream;
  rc = workspace_reserve(m->ws, C, choose_tiles(C, c.H * c.W), c.H * c.W, d, true,
                         beta_per_particle(c));
  if (!rc) rc = fit_buffers_alloc(h->fb, C, d, pri.data());
  const size_t cd = size_t(C) * d;
  const size_t bytes = sizeof(float) * (4 * cd + 2 * d * d + 2 * C + 12) +
                       sizeof(double) * (2 * cd + 4 * C + 12 + 2 * d + 1 + 2 * d + d * d) +
                       sizeof(float) * size_t(o->n_samples) * cd + 256 * 26;
  if (!rc && hipMalloc(&h->base, bytes) != hipSuccess) rc = set_error(GL_E_NOMEM, "hipMalloc failed");
  if (!rc && hipHostMalloc(&h->te_host, 4 * sizeof(float), hipHostMallocDefault) != hipSuccess)
    rc = set_error(GL_E_NOMEM, "hipHostMalloc failed");
  for (int i = 0; i < 2 && !rc; ++i)
    if (hipEventCreateWithFlags(&h->te_ev[i], hipEventDisableTiming) != hipSuccess)
      rc = set_error(GL_E_DEVICE, "hipEventCreate failed");
  if (rc) {
    hmc_free(h);
    return rc;
  }
  char* q = h->base;
  auto take = [&](size_t b) {
    char* r = q;
    q += (b + 255) & ~size_t(255);
    return r;
  };
  HmcArgs& a = h->a;
  a.C = C;
  a.d = d;
  a.n_burn = o->n_burn;
  a.n_adapt = h->n_adapt;
  a.target = o->target_accept;
  a.prior = h->fb.prior;
  a.z = reinterpret_cast<double*>(take(sizeof(double) * cd));
  a.z32 = reinterpret_cast<float*>(take(sizeof(float) * cd));
  a.p = reinterpret_cast<float*>(take(sizeof(float) * cd));
  a.g = reinterpret_cast<float*>(take(sizeof(float) * cd));
  a.zs = reinterpret_cast<double*>(take(sizeof(double) * cd));
  a.gs = reinterpret_cast<float*>(take(sizeof(float) * cd));
  float* chol_d = reinterpret_cast<float*>(take(sizeof(float) * d * d));
  float* chol_it_d = reinterpret_cast<float*>(take(sizeof(float) * d * d));
  a.chol = chol_d;
  a.chol_it = chol_it_d;
  a.traj = reinterpret_cast<int*>(take(sizeof(int) * 4));
  a.accept = reinterpret_cast<float*>(take(sizeof(float) * C));
  a.eps = reinterpret_cast<float*>(take(sizeof(float) * 4));
  a.bad = reinterpret_cast<int*>(take(sizeof(int) * C));
  a.lp = reinterpret_cast<double*>(take(sizeof(double) * C));
  a.lps = reinterpret_cast<double*>(take(sizeof(double) * C));
  a.k0 = reinterpret_cast<double*>(take(sizeof(double) * C));
  a.da = reinterpret_cast<double*>(take(sizeof(double) * 4));
  a.stats = reinterpret_cast<double*>(take(sizeof(double) * 4));
  a.samples = o->n_samples ? reinterpret_cast<float*>(take(sizeof(float) * size_t(o->n_samples) * cd))
                           : nullptr;
  a.T = reinterpret_cast<float*>(take(sizeof(float) * 4));
  a.la = reinterpret_cast<double*>(take(sizeof(double) * 4));
  a.zbar = reinterpret_cast<double*>(take(sizeof(double) * 2 * d));
  a.cg = reinterpret_cast<double*>(take(sizeof(double) * C));
  a.mom = reinterpret_cast<double*>(take(sizeof(double) * (1 + d + d * d)));
  a.zref = reinterpret_cast<double*>(take(sizeof(double) * d));
  h->chol_d = chol_d;
  h->chol_it_d = chol_it_d;
  a.adapt_len = o->adapt_length ? 1 : 0;
  h->max_leapfrog = o->max_leapfrog > 0 ? o->max_leapfrog : 1000;
  a.logl = m->ws.logl;
  a.grad = m->ws.grad;
  a.theta = m->ws.theta;
  a.seed_lo = uint32_t(o->seed);
  a.seed_hi = uint32_t(o->seed >> 32);
  const double da0[4] = {std::log(10.0 * o->step_size), 0.0, 0.0, 0.0};
  const double st0[4] = {0.0, 0.0, 0.0, 0.0};
  const float eps0 = o->step_size;
  const int zero = 0;
  bool ok = hipMemcpy(chol_d, chol.data(), sizeof(float) * d * d, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(chol_it_d, chol_it.data(), sizeof(float) * d * d, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.traj, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.da, da0, sizeof(da0), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.stats, st0, sizeof(st0), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(a.eps, &eps0, sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
  const float T0 = float(o->n_leapfrog) * o->step_size;
  h->T0 = T0;
  h->eps0 = eps0;
  const double la0[4] = {std::log(double(T0)), 0.0, 0.0, std::log(double(T0))};
  ok = ok && hipMemcpy(a.T, &T0, sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(a.la, la0, sizeof(la0), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && z0) ok = hipMemcpyAsync(a.z, z0, sizeof(double) * cd, hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (!ok) rc = set_error(GL_E_DEVICE, "upload failed");
  if (!rc) rc = hmc_launch1(z0 ? hmc_round_kernel : hmc_start_kernel, a, int(cd), 256, st);
  if (!rc) rc = hmc_gradient(h, 0.f, 0, st);
  if (rc) {
    hmc_free(h);
    return rc;
  }
  *out = h;
  return GL_OK;
}

int gl_hmc_destroy(gl_hmc* h) {
  clear_error();
  if (!h) return GL_OK;
  (void)hipDeviceSynchronize();
  hmc_free(h);
  return GL_OK;
}

int gl_hmc_run(gl_hmc* h, int n, void* stream) {
  clear_error();
  if (!h) return set_error(GL_E_INVALID, "state is NULL");
  if (n < 0) return set_error(GL_E_INVALID, "n must be >= 0");
  const int total = h->n_burn + h->n_samples;
  if (h->done + n > total)
    return set_error(GL_E_INVALID, "%d trajectories requested, %d left", n, total - h->done);
  h->a.eps_fixed = 0.f;
  h->pc_ready = false;  // another call on the model may have used its particle constants
  for (int i = 0; i < n; ++i) {
    int rc = hmc_trajectory(h, (hipStream_t)stream);
    if (rc) return rc;
  }
  return GL_OK;
}

int gl_hmc_samples(gl_hmc* h, float* theta, void* stream) {
  clear_error();
  if (!h) return set_error(GL_E_INVALID, "state is NULL");
  if (!h->n_samples) return GL_OK;
  int rc = check_device_ptr(theta, "theta");
  if (rc) return rc;
  GL_HIP(hipMemcpyAsync(theta, h->a.samples, sizeof(float) * size_t(h->n_samples) * h->C * h->d,
                        hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return GL_OK;
}

int gl_hmc_get_info(gl_hmc* h, gl_hmc_info* out, void* stream) {
  clear_error();
  if (!h || !out) return set_error(GL_E_INVALID, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  float eps = 0.f, T = 0.f;
  double stats[2] = {0.0, 0.0};
  GL_HIP(hipMemcpyAsync(&eps, h->a.eps, sizeof(float), hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(&T, h->a.T, sizeof(float), hipMemcpyDeviceToHost, st));
  GL_HIP(hipMemcpyAsync(stats, h->a.stats, sizeof(stats), hipMemcpyDeviceToHost, st));
  GL_HIP(hipStreamSynchronize(st));
  out->step_size = eps;
  out->accept_mean = stats[1] > 0 ? stats[0] / stats[1] : 0.0;
  out->trajectories = h->done;
  out->trajectory_length = h->a.adapt_len ? T : float(h->L) * eps;
  out->mean_leapfrog = h->done ? double(h->leapfrogs) / h->done : 0.0;
  out->mass_updates = h->mass_updates;
  return GL_OK;
}

int gl_hmc_get_mass(gl_hmc* h, float* chol, void* stream) {
  clear_error();
  if (!h) return set_error(GL_E_INVALID, "state is NULL");
  int rc = check_device_ptr(chol, "chol");
  if (rc) return rc;
  GL_HIP(hipMemcpyAsync(chol, h->chol_d, sizeof(float) * h->d * h->d, hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return GL_OK;
}

int gl_hmc_leapfrog(gl_hmc* h, const double* z, const float* p, int L, float eps,
                    double* z_out, float* p_out, double* logpost_out, void* stream) {
  clear_error();
  if (!h) return set_error(GL_E_INVALID, "state is NULL");
  if (L < 1 || !(eps > 0.f)) return set_error(GL_E_INVALID, "need L >= 1 and eps > 0");
  int rc;
  if ((rc = check_device_ptr(z, "z")) || (rc = check_device_ptr(p, "p")) ||
      (rc = check_device_ptr(z_out, "z_out")) || (rc = check_device_ptr(p_out, "p_out")) ||
      (rc = check_device_ptr(logpost_out, "logpost_out")))
    return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t b = sizeof(float) * size_t(h->C) * h->d;
  HmcArgs& a = h->a;
  GL_HIP(hipMemcpyAsync(a.z, z, 2 * b, hipMemcpyDeviceToDevice, st));
  GL_HIP(hipMemcpyAsync(a.p, p, b, hipMemcpyDeviceToDevice, st));
  a.eps_fixed = eps;
  h->pc_ready = false;  // new positions
  rc = hmc_launch1(hmc_round_kernel, a, h->C * h->d, 256, st);
  if (!rc) rc = hmc_gradient(h, 0.5f, 1, st);
  for (int l = 0; !rc && l < L; ++l) rc = hmc_gradient(h, l + 1 < L ? 1.0f : 0.5f, l + 1 < L, st);
  a.eps_fixed = 0.f;
  if (rc) return rc;
  GL_HIP(hipMemcpyAsync(z_out, a.z, 2 * b, hipMemcpyDeviceToDevice, st));
  GL_HIP(hipMemcpyAsync(p_out, a.p, b, hipMemcpyDeviceToDevice, st));
  GL_HIP(hipMemcpyAsync(logpost_out, a.lp, sizeof(double) * h->C, hipMemcpyDeviceToDevice, st));
  return GL_OK;
}

}  // extern "C"
