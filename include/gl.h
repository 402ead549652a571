/*
 * gl.h - C ABI of the MI355X lens-likelihood library (libglens.so).
 *
 * Batched GIGA-Lens forward model, Gaussian log-likelihood and its gradient, evaluated for
 * many parameter vectors at once on one GPU (Gu et al. 2022, arXiv:2202.07663), plus a
 * fixed-budget multi-start fit, variational inference, preconditioned HMC, and a
 * continuous-batching server for streams of systems.
 *
 * Conventions shared by every entry point
 *   - Return value: GL_OK (0) on success, GL_PENDING (1) from gl_poll only, a negative
 *     GL_E_* code on failure. No C++ exception crosses the ABI. gl_last_error() returns a
 *     thread-local, human-readable message for the last failure on the calling thread.
 *   - Device buffers (theta, img, logl, grad) are caller-owned device pointers on the
 *     current HIP device; they are never freed or retained by the library. Host buffers
 *     named in descriptors (psf, obs, priors) are copied before the call returns.
 *   - Compute calls are stream-ordered: `stream` is a hipStream_t (NULL = default stream).
 *     They enqueue work and return; outputs are valid once the stream is synchronised. The
 *     one exception: a call on a batch larger than the model's work space grows it first,
 *     which synchronises the device (gl_model_reserve sizes it up front).
 *     Calls on one gl_model must be ordered on one stream (the model owns the work space).
 *   - Parameter vectors theta are FP32, row-major [P][d], physical (constrained) values in
 *     this order (Sec. 2.1.2, eq. sim-dist; arcsec for lengths, counts/s for intensities):
 *        mass:       theta_E, [gamma_epl if EPL], eps1, eps2, x, y, [gamma_ext1, gamma_ext2]
 *        lens light: R, n, eps1, eps2, x, y, I                    (if lens_light)
 *        source:     R, n, eps1, eps2, x, y, I                    (always)
 *        shapelets:  beta, c_0 .. c_{M-1}, M = (n+1)(n+2)/2       (if shapelet_nmax >= 0)
 *     The shapelet centre is the source Sersic centre. d is reported by gl_model_nparams.
 *   - Non-finite per-particle results (e.g. NaN parameters) are not call failures: that
 *     particle's log-likelihood is -inf and its gradient row is zero.
 */
#ifndef GLENS_GL_H
#define GLENS_GL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GL_OK = 0,
  GL_PENDING = 1,
  GL_E_INVALID = -1,       /* bad argument (null pointer, size, flag, host pointer ...) */
  GL_E_NOMEM = -2,         /* device allocation failed */
  GL_E_DEVICE = -3,        /* HIP runtime error */
  GL_E_BUDGET = -4,        /* request larger than the server's HBM budget */
  GL_E_NOTFOUND = -5,      /* unknown ticket */
  GL_E_NUMERIC = -6,       /* fit produced no finite particle */
  GL_E_UNIMPLEMENTED = -7, /* configuration outside what the kernels support */
  GL_E_CLOSED = -8         /* server is shutting down */
};

enum { GL_MASS_SIE = 0, GL_MASS_EPL = 1 };

#define GL_MAX_PARAMS 68   /* EPL + shear + lens light + source + shapelets n_max = 8 */
#define GL_MAX_NMAX 8
#define GL_MAX_PSF 31
#define GL_MAX_IMAGE 128   /* H, W <= 128 */
#define GL_MAX_KSUPER 4

/*
 * Lens system description (Sec. 2.1: image grid, mass and light components, noise model,
 * PSF). Pixel (i, j) (row i, column j) has centre ((j - (W-1)/2) s, (i - (H-1)/2) s) with
 * s = pixel_scale; each pixel is evaluated on a k_super x k_super sub-grid and averaged
 * (Sec. 2.1.1, last paragraph), then convolved with the PSF (zero-padded, same size).
 */
typedef struct gl_model_desc {
  int H, W;            /* image rows and columns, 1..GL_MAX_IMAGE */
  float pixel_scale;   /* arcsec per pixel; pixel_scale / k_super >= 1e-4 */
  int k_super;         /* supersampling factor, 1..GL_MAX_KSUPER */
  int mass;            /* GL_MASS_SIE or GL_MASS_EPL */
  int shear;           /* 1: external shear (2 parameters), 0: none */
  int lens_light;      /* 1: elliptical Sersic lens light (7 parameters), 0: none */
  int shapelet_nmax;   /* -1: no shapelets; 0..GL_MAX_NMAX: Cartesian shapelets to n_max */
  int psf_size;        /* K, odd, 1..GL_MAX_PSF */
  const float* psf;    /* host, K*K row-major, used as given (not renormalised); copied */
  const float* obs;    /* host, H*W row-major observed image (counts/s); copied; may be
                          NULL for a model used only by gl_simulate */
  float sigma_bkg;     /* background noise sigma (counts/s), >= 0 */
  float t_exp;         /* exposure time (s), > 0 */
  float gain;          /* G (e-/count), > 0 */
} gl_model_desc;

typedef struct gl_model gl_model;

/* Validate `desc`, copy the PSF and observed image to the current device and return an
 * opaque handle in *out. GL_E_INVALID for a bad field, GL_E_UNIMPLEMENTED for sizes
 * beyond the GL_MAX_* limits, GL_E_NOMEM / GL_E_DEVICE on runtime failure. */
int gl_model_create(const gl_model_desc* desc, gl_model** out);

/* Free the model and its device work space (synchronises the device first). NULL is a
 * no-op. */
int gl_model_destroy(gl_model* model);

/* Number d of parameters per vector for this model (layout above). */
int gl_model_nparams(const gl_model* model, int* d);

/* Grow the model's device work space for calls of up to P parameter vectors (any batch size
 * up to P). The compute calls grow it on demand, and a call that grows it synchronises the
 * device and reallocates before it enqueues its work; reserving first keeps later calls
 * enqueue-only. with_fit = 1 also reserves the buffers of gl_fit_state_*, gl_vi_* and
 * gl_hmc_* (they are kept once present). GL_E_NOMEM if the device memory is not there. */
int gl_model_reserve(gl_model* model, int P, int with_fit);

/* Diagnostic: how a call with P parameter vectors is split on this model (no device work).
 *   psf_path:  GL_PSF_MFMA (matrix cores, one workgroup per vector: K <= 21, the image in
 *              at most 64 tiles of 16 rows, and one band: P >= 512 or at most 8 rows),
 *              GL_PSF_VALU (vector ALUs, one workgroup per vector) or GL_PSF_BANDED (vector
 *              ALUs, row bands of the image per vector, for P < 512);
 *   tiles, fwd_tiles: sub-pixel work tiles per vector of the adjoint and the forward pass;
 *   bands:     row bands of the PSF pass (1 unless banded);
 *   workspace_bytes: device work space of a likelihood call at this P (gl_model_reserve);
 *   workspace_reserved: what the model holds now;
 *   noalloc_max_P: the largest P gl_loglik_grad_noalloc accepts on this model;
 *   band_split: lanes that share one strip's PSF columns in the banded pass (1, 2 or 4:
 *              more than 1 only when the pass would have fewer work items than the GPU
 *              has lanes, P below about 100 at 60 x 60 pixels). */
enum { GL_PSF_MFMA = 0, GL_PSF_VALU = 1, GL_PSF_BANDED = 2 };
typedef struct gl_plan {
  int psf_path, tiles, fwd_tiles, bands;
  size_t workspace_bytes, workspace_reserved;
  int noalloc_max_P;
  int band_split;
} gl_plan;
int gl_model_plan(const gl_model* model, int P, gl_plan* out);

/* Noiseless model image I_model(x, y; Theta) (Sec. 2.1.1: deflect, ray trace, source plus
 * lens light, k x k mean, PSF) for P parameter vectors.
 *   theta: device, [P][d] FP32.  img: device, [P][H][W] FP32 (written).
 * P = 0 is a no-op. */
int gl_simulate(gl_model* model, const float* theta, int P, float* img, void* stream);

/* Log-likelihood of eq. model-def (Sec. 2.1.2) for P parameter vectors:
 *   log L = -1/2 sum_pixels [ (I_obs - I_model)^2 / s2 + log(2 pi s2) ],
 *   s2 = sigma_bkg^2 + max(I_model, 0) / (G t_exp).
 * Per-pixel terms in FP32, summed in FP64.
 *   theta: device [P][d] FP32.  logl: device [P] FP64 (written).
 * GL_E_INVALID if the model has no observed image. */
int gl_loglik(gl_model* model, const float* theta, int P, double* logl, void* stream);

/* log L (as gl_loglik) and its gradient d log L / d Theta in physical parameters
 * (Sec. 2.2: the paper obtains it by automatic differentiation; here a hand-written
 * adjoint of every step). grad: device [P][d] FP32 (written). */
int gl_loglik_grad(gl_model* model, const float* theta, int P, double* logl, float* grad,
                   void* stream);

/* gl_loglik_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results (bitwise, for the same P), with the work space taken from a fixed array of
 * 128 MiB that the library holds on every device it runs on until the process ends, instead
 * of the model's own allocation. The call allocates nothing and never grows anything; it
 * enqueues work on `stream` and returns.
 *   Limit: P up to gl_plan.noalloc_max_P of the model (about 800 vectors at 60 x 60 pixels
 *   and k_super = 2); a larger P returns GL_E_BUDGET with the sizes in gl_last_error().
 *   The array is shared by every call on one device and keeps the last call's contents:
 *   calls that overlap on one device (other streams, other threads) race, so the caller
 *   orders them. The current device must be the model's (GL_E_INVALID otherwise). */
int gl_loglik_grad_noalloc(gl_model* model, const float* theta, int P, double* logl,
                           float* grad, void* stream);

/* Diagnostic: run the gl_loglik_grad pipeline (with_grad = 1) or the gl_loglik pipeline
 * (with_grad = 0) once on `stream` with HIP events between its kernels, wait for it, and
 * write the duration of each stage in milliseconds to ms[GL_NSTAGES] (stages not run read
 * 0): prologue, sub-pixel forward, PSF + likelihood (+ adjoint seed), sub-pixel adjoint,
 * gradient finalize. logl and grad as in gl_loglik_grad (grad unused when with_grad = 0). */
#define GL_NSTAGES 5
int gl_model_stage_times(gl_model* model, const float* theta, int P, int with_grad,
                         double* logl, float* grad, float* ms, void* stream);

/* Diagnostic: as gl_model_stage_times, but n_calls (1 .. 10000) calls back to back on
 * `stream`, each with its own HIP events (created and destroyed here), one wait after the
 * last; ms[i] is the mean duration of stage i over the calls. The calls run as a loop of
 * gl_loglik_grad (or gl_loglik) calls would, so the durations are those of steady-state
 * launches. GL_E_INVALID for n_calls out of range; the other errors as gl_loglik_grad. */
int gl_model_stage_times_n(gl_model* model, const float* theta, int P, int with_grad,
                           int n_calls, double* logl, float* grad, float* ms, void* stream);

/* ---------------------------------------------------------------------------------------
 * Priors, bijectors and the fixed-budget multi-start fit (Sec. 2.2 bijectors and
 * Jacobian-corrected posterior; Sec. 2.3 multi-start gradient descent with Adam).
 * The bijector follows the prior family: NORMAL -> identity, LOGNORMAL -> exp,
 * TRUNCNORMAL and UNIFORM on (lo, hi) -> lo + (hi - lo) / (1 + exp(-z)).
 * ------------------------------------------------------------------------------------- */
enum { GL_PRIOR_NORMAL = 0, GL_PRIOR_LOGNORMAL = 1, GL_PRIOR_TRUNCNORMAL = 2,
       GL_PRIOR_UNIFORM = 3 };

typedef struct gl_prior {
  int family;      /* GL_PRIOR_* */
  float mu, sigma; /* NORMAL / TRUNCNORMAL: mean, sd; LOGNORMAL: mean, sd of log(theta) */
  float lo, hi;    /* TRUNCNORMAL / UNIFORM support, lo < hi */
} gl_prior;

typedef struct gl_fit_opts {
  int P;                  /* particles (multi-start samples), >= 1 */
  int K;                  /* Adam steps, >= 1 */
  float lr0, lr1;         /* learning rate, linear from lr0 to lr1 over the K steps */
  float beta1, beta2, eps;/* Adam constants (0.9, 0.999, 1e-8 if all three are 0) */
  uint64_t seed;          /* starts are drawn from the prior with a counter-based RNG */
  const gl_prior* priors; /* host, d entries, copied */
} gl_fit_opts;

typedef struct gl_fit_result {
  int status;             /* GL_OK, or GL_E_NUMERIC / GL_E_DEVICE ... for this request */
  int d;                  /* number of parameters */
  int best;               /* index of the best particle */
  float theta_best[GL_MAX_PARAMS];
  float z_best[GL_MAX_PARAMS];  /* the same particle in unconstrained space (g^-1) */
  double logl_best;       /* log L at theta_best */
  double logpost_best;    /* log L + log p + log|J| at the best particle's z */
  double chi2nu;          /* chi^2 / (H W - d) at theta_best */
  uint64_t t_submit, t_admit, t_done;  /* ns, CLOCK_MONOTONIC (server results only) */
} gl_fit_result;

/* One multi-start fit of one system, run to completion on `stream` (blocking): P starts
 * from the prior, K Adam steps on f = -(log L + log p + log|J|) in unconstrained space,
 * then the best particle by log posterior at its final position. */
int gl_fit(gl_model* model, const gl_fit_opts* opts, gl_fit_result* out, void* stream);

/* Lower-level fit state, for stepping and inspection. The state owns device arrays
 * z, m, v ([P][d] FP32: unconstrained parameters and Adam moments) and a step counter.
 * gl_fit_state_create draws the P starts from the prior (m = v = 0, step 0). */
typedef struct gl_fit_state gl_fit_state;
int gl_fit_state_create(gl_model* model, const gl_fit_opts* opts, gl_fit_state** out,
                        void* stream);
int gl_fit_state_destroy(gl_fit_state* st);
/* Run `n` Adam steps (continuing the schedule from the current step). */
int gl_fit_state_step(gl_fit_state* st, int n, void* stream);
/* Copy caller device arrays ([P][d] FP32) into the state and set the step counter. */
int gl_fit_state_load(gl_fit_state* st, const float* z, const float* m, const float* v,
                      int step, void* stream);
/* Copy the state out to caller device arrays (any of them may be NULL). */
int gl_fit_state_store(gl_fit_state* st, float* z, float* m, float* v, int* step, void* stream);
/* Evaluate log L at the current z, pick the best particle by log L + log p~, fill *out
 * (blocking). */
int gl_fit_state_result(gl_fit_state* st, gl_fit_result* out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Variational inference (Sec. 2.4): a multivariate normal surrogate q = N(mu, Sigma) of the
 * posterior in unconstrained space (the fit's target), fitted by minimising the ELBO loss
 * E_q[log q - log p~(I, z)] with Adam. Sigma = L L^T through the Cholesky bijector: d(d+1)/2
 * values v fill the lower triangle of L row by row (v[i(i+1)/2 + j] is L_ij) and the diagonal
 * is exponentiated. The state x = (mu [d], v [d(d+1)/2]) starts at (mu0, log(init_sd) on the
 * diagonal, 0 elsewhere), i.e. Sigma = init_sd^2 I (the paper: the MAP point and 1e-6 I).
 * Iteration k draws n_samples eps ~ N(0, I) (Philox4x32-10 keyed by seed, counter
 * (sample, parameter, k, 0x76690000); uniforms u = (k52 + 1/2) / 2^52 from 26 + 26 bits of
 * two words; Box-Muller cosine branch), evaluates the likelihood gradient at z = mu + L eps
 * for all samples in one batched launch, and takes the pathwise gradient estimate: the mean
 * over samples with a finite objective f = -log p~(z | I) of grad f for mu, of
 * (grad f)_i eps_j for L_ij (i > j), and of L_ii (grad f)_i eps_i - 1 for v_ii. (The paper
 * prints the score-function form of the same gradient; both estimate it without bias.)
 * Adam (beta1, beta2, eps; 0.9, 0.999, 1e-8 if all are 0) then steps x with learning rate
 * lr_max (1 - (1 - min(k, lr_warmup) / lr_warmup)^2) (the paper: 1e-3, warm-up 500), then
 * lr_max, or, with lr_final > 0 (not in the paper), a geometric decay after the warm-up:
 * lr_max (lr_final / lr_max)^((k - lr_warmup) / (K - 1 - lr_warmup)), which ends at lr_final
 * on the last iteration (k = K - 1). The decay lets the mean settle in posteriors whose
 * widths are far below lr_max: Adam moves every coordinate by about the learning rate per
 * iteration, so a constant rate keeps the mean that far from its optimum.
 * ------------------------------------------------------------------------------------- */
typedef struct gl_vi_opts {
  int n_samples;          /* n_VI, >= 1 */
  int K;                  /* iterations, >= 1 */
  float lr_max;           /* >= 0 */
  int lr_warmup;          /* >= 0 (0: constant lr_max) */
  float beta1, beta2, eps;
  float init_sd;          /* > 0 */
  uint64_t seed;
  const gl_prior* priors; /* host [d], copied */
  float lr_final;         /* 0: constant after the warm-up; > 0 (with lr_max > 0): the rate
                             on the last iteration, reached geometrically */
  int estimator;          /* GL_VI_PATHWISE (0, default): the mean of the pathwise terms
                             (grad f, grad f eps^T); GL_VI_SCORE: the score-function form
                             of Sec. 2.4's eq. elbo-grad, the mean of
                             (log q(z) - log p~(I, z)) grad log q(z) at fixed z. Both are
                             unbiased for the ELBO gradient; the score form uses only the
                             objective's value and has a far larger variance */
} gl_vi_opts;
enum { GL_VI_PATHWISE = 0, GL_VI_SCORE = 1 };

typedef struct gl_vi gl_vi;
/* Create the state on `model` (with an observed image); mu0: device [d] FP64 (copied). The
 * state holds (4 (d + d(d+1)/2) + n_samples (d + 1) + K) doubles and 2 n_samples d floats;
 * it uses the model's workspace (the model must outlive it; order calls on one stream). */
int gl_vi_create(gl_model* model, const gl_vi_opts* opts, const double* mu0, gl_vi** out,
                 void* stream);
int gl_vi_destroy(gl_vi* v);
/* Run the next n iterations on `stream`; GL_E_INVALID if fewer than n of K are left. An
 * iteration with no finite sample leaves the state as it was and records a NaN loss. */
int gl_vi_step(gl_vi* v, int n, void* stream);
/* Current mean (device [d]), dense Cholesky factor L and covariance L L^T (device [d][d]
 * row-major), all FP64; any may be NULL. */
int gl_vi_get(gl_vi* v, double* mu, double* chol, double* cov, void* stream);
/* n draws from the current surrogate, z = mu + L eps (device [n][d] FP64), eps from counter
 * (draw, parameter, 0, 0x76697371) under `seed` (e.g. HMC chain starts, as in the paper). */
int gl_vi_sample(gl_vi* v, int n, uint64_t seed, double* z, void* stream);
/* The optimiser state: x = (mu, v), Adam moments m and s (device [d + d(d+1)/2] FP64), the
 * iteration count k, and the loss history (device [K] FP64, NaN where not run); any pointer
 * may be NULL. set_state loads x, m, s and k (k <= K). */
int gl_vi_get_state(gl_vi* v, double* x, double* m, double* s, int* k, double* loss,
                    void* stream);
int gl_vi_set_state(gl_vi* v, const double* x, const double* m, const double* s, int k,
                    void* stream);

/* ---------------------------------------------------------------------------------------
 * Preconditioned Hamiltonian Monte Carlo (Sec. 2.5): `chains` independent chains on the
 * posterior in unconstrained space, log p~(z | I) = log L(g(z)) + log p~(z) (the fit's
 * target), momenta p ~ N(0, M) for a mass matrix M given by its inverse (the paper sets M
 * to the inverse of the variational posterior covariance, so M^-1 is that covariance),
 * H = -log p~(z | I) + p^T M^-1 p / 2, L leapfrog steps of size eps per trajectory and a
 * Metropolis accept with probability min(1, exp(H0 - H1)). Any non-finite log posterior
 * along a trajectory rejects it. During the first floor(adapt_frac n_burn) trajectories eps
 * follows dual averaging (Hoffman & Gelman 2014, gamma 0.05, t0 10, kappa 0.75,
 * mu = log(10 step_size)) of the chain-mean acceptance probability towards target_accept
 * (the paper: 0.75 over the first 80% of burn-in); it then stays at the averaged value.
 * With adapt_length the trajectory length T (initially n_leapfrog step_size) adapts too, as
 * in Hoffman, Radul & Sountsov (2021, ChEES): trajectory k runs L = ceil(u_k T / eps)
 * leapfrog steps (at most max_leapfrog) with u_k the k-th van der Corput number (base 2),
 * shared by all chains, and during the same adaptation window log T takes Adam steps
 * (beta1 0, beta2 0.95, rate 0.025) up the acceptance-weighted estimate of d ChEES / d log T,
 * ChEES = E[(|z' - E z'|^2 - |z - E z|^2)^2] / 4, whose per-chain term is
 * (|z' - zbar'|^2 - |z - zbar|^2) ((z' - zbar') . M^-1 p') u T (means over chains); T is then
 * fixed at its average with weights m^-0.75. The paper adapts both as in these references.
 * With adapt_mass (not in the paper, whose M^-1 is the variational covariance throughout),
 * M^-1 is re-estimated during the same adaptation window, as in Stan's windowed adaptation:
 * after an initial buffer of floor(0.15 n_adapt) trajectories, three windows of lengths in
 * the ratio 1 : 2 : 4 fill the trajectories up to a terminal buffer of floor(0.10 n_adapt)
 * (n_adapt = floor(adapt_frac n_burn); no windows if they would cover fewer than 7
 * trajectories). At the end of each window M^-1 becomes the sample covariance of the chains'
 * positions after that window's trajectories (n = chains x window length samples), its
 * off-diagonal entries scaled by n / (n + 5) (shrinkage towards the diagonal), unless that is
 * not positive definite; the step-size averaging then restarts with mu = log(10 eps). Each
 * window end waits for the stream (the estimate is factored on the host).
 * Every chain is one particle of the likelihood pipeline: a leapfrog step is one batched
 * gradient launch over all chains. Random numbers: Philox4x32-10 keyed by `seed`, counter
 * (chain, parameter, trajectory, purpose).
 * ------------------------------------------------------------------------------------- */
enum { GL_MASS_DIAG = 0, GL_MASS_DENSE = 1, GL_MASS_CHOL = 2 };

typedef struct gl_hmc_opts {
  int chains;                  /* >= 1 */
  int n_leapfrog;              /* L, >= 1 */
  int n_burn, n_samples;       /* trajectories discarded / recorded, >= 0 */
  float step_size;             /* initial eps, > 0 */
  float target_accept;         /* in (0, 1) */
  float adapt_frac;            /* share of burn-in with step-size adaptation, in [0, 1] */
  uint64_t seed;
  const float* inv_mass;       /* host, copied: M^-1, NULL for the identity; see form */
  int adapt_length;            /* 1: also adapt the trajectory length (see above) */
  int max_leapfrog;            /* cap on leapfrog steps per trajectory (0: 1000) */
  int inv_mass_form;           /* GL_MASS_DIAG: inv_mass is the diagonal [d] (> 0);
                                  GL_MASS_DENSE: the full symmetric positive definite [d][d]
                                  row-major (e.g. a posterior covariance of z);
                                  GL_MASS_CHOL: its lower Cholesky factor [d][d] row-major
                                  (positive diagonal; entries above it are ignored) */
  const gl_prior* priors;      /* host [d], copied */
  int adapt_mass;              /* 1: re-estimate M^-1 during adaptation (see above) */
} gl_hmc_opts;

typedef struct gl_hmc_info {
  float step_size;       /* current eps (the averaged one once adaptation ended) */
  double accept_mean;    /* mean acceptance probability over the recorded trajectories */
  int trajectories;      /* trajectories run so far */
  float trajectory_length; /* T (adapted), or n_leapfrog eps without length adaptation */
  double mean_leapfrog;  /* mean leapfrog steps per trajectory so far */
  int mass_updates;      /* times M^-1 was replaced by an estimate (adapt_mass) */
} gl_hmc_info;

typedef struct gl_hmc gl_hmc;
/* Create the sampler on `model` (which must hold an observed image) and evaluate the
 * gradient at the starts. Positions are kept in FP64 (the likelihood sees them rounded to
 * FP32); momenta in FP32. z0: device [chains][d] FP64 unconstrained starts (copied), or
 * NULL to draw them from the prior. GL_E_INVALID for bad options or an inv_mass that is
 * not symmetric positive definite. The state holds device arrays of
 * ((5 + n_samples) chains d + 2 d^2) floats; it uses the model's workspace, so the model
 * must outlive it and not be used concurrently from another stream. */
int gl_hmc_create(gl_model* model, const gl_hmc_opts* opts, const double* z0, gl_hmc** out,
                  void* stream);
int gl_hmc_destroy(gl_hmc* h);
/* Run the next `n` trajectories (burn-in first, then recorded ones) on `stream` (not
 * blocking). GL_E_INVALID if fewer than n are left of n_burn + n_samples. */
int gl_hmc_run(gl_hmc* h, int n, void* stream);
/* Copy the recorded samples, physical parameters g(z), to theta: device
 * [n_samples][chains][d] FP32 (rows not yet recorded hold unspecified values). */
int gl_hmc_samples(gl_hmc* h, float* theta, void* stream);
/* Step size, mean acceptance and progress (blocking). */
int gl_hmc_get_info(gl_hmc* h, gl_hmc_info* out, void* stream);
/* Copy the current lower Cholesky factor C of M^-1 = C C^T (the given one, or the last
 * estimate of the mass adaptation) to chol: device [d][d] FP32 row-major, zero above the
 * diagonal. */
int gl_hmc_get_mass(gl_hmc* h, float* chol, void* stream);
/* L leapfrog steps of size eps (no momentum draw, no accept, no adaptation) from caller
 * positions z (device [chains][d] FP64) and momenta p (device [chains][d] FP32), writing
 * the end point to z_out (FP64), p_out (FP32) and log p~(z_L | I) to logpost_out (device
 * [chains] FP64). The sampler's own chain state is overwritten; use a separate gl_hmc for
 * this. */
int gl_hmc_leapfrog(gl_hmc* h, const double* z, const float* p, int L, float eps,
                    double* z_out, float* p_out, double* logpost_out, void* stream);

/* ---------------------------------------------------------------------------------------
 * Continuous-batching server: systems of mixed sizes and component sets are admitted as
 * slots and HBM budget free up; each tick advances every active system by
 * steps_per_tick Adam steps, with the systems of one kernel configuration sharing one
 * launch per kernel.
 * ------------------------------------------------------------------------------------- */
typedef struct gl_server_opts {
  size_t hbm_budget_bytes; /* device memory the active systems may hold (state + scratch) */
  int max_systems;         /* active-system slots */
  int steps_per_tick;      /* Adam steps per system per tick, >= 1 */
  double fill_subpixels;   /* admit while the active systems' sub-pixel evaluations per
                              step (sum of P H W k^2) stay below this; one system is always
                              admitted when none is active. 0 selects 6e7, about what fills
                              one GPU; a huge value admits by slots and budget only */
} gl_server_opts;

typedef struct gl_server gl_server;

/* Start the scheduler thread on the current device. */
int gl_server_create(const gl_server_opts* opts, gl_server** out);
/* Stop accepting work, finish active systems, join the thread, free everything. */
int gl_server_destroy(gl_server* s);
/* Queue one fit request (desc and opts are copied; non-blocking). GL_E_BUDGET if the
 * request alone exceeds the HBM budget, GL_E_INVALID for a bad request. */
int gl_submit(gl_server* s, const gl_model_desc* desc, const gl_fit_opts* opts,
              uint64_t* ticket);
/* GL_PENDING while the request is queued or running; GL_OK with *out filled once done
 * (the ticket is then released); GL_E_NOTFOUND for an unknown ticket. */
int gl_poll(gl_server* s, uint64_t ticket, gl_fit_result* out);

/* Counters of the server. completed counts every retired request, failed those retired with
 * an error status (admission that could not allocate, a launch that failed, a device error:
 * gl_poll then returns the result with that status), last_error the code of the latest. */
typedef struct gl_server_stats {
  uint64_t submitted, admitted, completed, ticks;
  size_t hbm_in_use, hbm_peak;
  int active, queued;
  uint64_t failed;
  int last_error;
} gl_server_stats;
int gl_server_get_stats(gl_server* s, gl_server_stats* out);

/* Thread-local message for the last failure on this thread ("" if none). */
const char* gl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GLENS_GL_H */
