// Device helpers of the fit and the sampler: counter-based random numbers, prior draws,
// and the Jacobian-corrected log prior of one parameter in unconstrained space.
#pragma once

#include <hip/hip_runtime.h>

#include "glens_host.h"
#include "glens_types.h"

namespace glens {

// ------------------------------------------------------------------------------------------
// Counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random
// numbers: as easy as 1, 2, 3"), keyed by the request seed, counter (particle, parameter).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(M0) * c[0], p1 = uint64_t(M1) * c[2];
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = uint32_t(p1);
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = uint32_t(p0);
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += W0;
    k1 += W1;
  }
}

// Uniform double in (0, 1) from two 32-bit words: 52 random bits k (26 from each word),
// u = (k + 1/2) / 2^52, where k + 1/2 is exact so that u never rounds to 0 or 1.
__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
  return (double(a >> 6) * 67108864.0 + double(b >> 6) + 0.5) * (1.0 / 4503599627370496.0);
}

__device__ __forceinline__ double std_normal_cdf(double x) { return 0.5 * erfc(-x * 0.7071067811865476); }
__device__ __forceinline__ double std_normal_icdf(double p) { return 1.4142135623730951 * erfinv(2.0 * p - 1.0); }

// Draw the start z of one (particle, parameter) from the prior, in unconstrained space.
__device__ __forceinline__ float draw_start(const Prior& pr, uint32_t seed_lo, uint32_t seed_hi, int part, int j) {
  uint32_t c[4] = {uint32_t(part), uint32_t(j), 0x6c656e73u, 0u};
  philox4x32_10(c, seed_lo, seed_hi);
  const double u1 = u01(c[0], c[1]), u2 = u01(c[2], c[3]);
  switch (pr.family) {
    case GL_PRIOR_NORMAL:
    case GL_PRIOR_LOGNORMAL: {  // log-normal: z = log(theta) is normal
      const double n = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      return float(pr.mu + pr.sigma * n);
    }
    case GL_PRIOR_TRUNCNORMAL: {
      const double a = std_normal_cdf((pr.lo - pr.mu) / pr.sigma);
      const double b = std_normal_cdf((pr.hi - pr.mu) / pr.sigma);
      double x = pr.mu + pr.sigma * std_normal_icdf(a + u1 * (b - a));
      const double w = double(pr.hi) - pr.lo;
      double u = (x - pr.lo) / w;
      u = fmin(fmax(u, 1e-7), 1.0 - 1e-7);
      return float(log(u) - log1p(-u));
    }
    default: {  // uniform on (lo, hi): z = logit(u)
      const double u = fmin(fmax(u1, 1e-7), 1.0 - 1e-7);
      return float(log(u) - log1p(-u));
    }
  }
}

// theta = g(z): the bijector of the prior family (identity, exp, or a sigmoid onto (lo, hi)).
__device__ __forceinline__ float bijector_fwd(const Prior& pr, float z) {
  if (pr.family == GL_PRIOR_LOGNORMAL) return expf(z);
  if (pr.family == GL_PRIOR_TRUNCNORMAL || pr.family == GL_PRIOR_UNIFORM)
    return pr.lo + (pr.hi - pr.lo) / (1.0f + expf(-z));
  return z;
}

__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }

// log p~(z) = log p(g(z)) + log |g'(z)| of one parameter, and its derivative.
__device__ __forceinline__ float log_prior_z(const Prior& pr, float z, float th, float& dlp,
                                             float& dth) {
  const float isg = 1.0f / pr.sigma;
  switch (pr.family) {
    case GL_PRIOR_NORMAL:
    case GL_PRIOR_LOGNORMAL: {
      const float r = (z - pr.mu) * isg;
      dlp = -r * isg;
      dth = pr.family == GL_PRIOR_NORMAL ? 1.0f : th;
      return -0.5f * r * r + pr.logc;
    }
    case GL_PRIOR_TRUNCNORMAL: {
      const float sg = 1.0f / (1.0f + expf(-z)), w = pr.hi - pr.lo;
      const float r = (th - pr.mu) * isg;
      dth = w * sg * (1.0f - sg);
      dlp = -r * isg * dth + 1.0f - 2.0f * sg;
      return -0.5f * r * r + pr.logc - softplus(-z) - softplus(z);
    }
    default: {
      const float sg = 1.0f / (1.0f + expf(-z));
      dth = (pr.hi - pr.lo) * sg * (1.0f - sg);
      dlp = 1.0f - 2.0f * sg;
      return -softplus(-z) - softplus(z);
    }
  }
}

}  // namespace glens
