// Per-particle stages of the likelihood pipeline that run as one 64-lane block (a single
// wave) per particle: the decode (prologue) and the gradient finalize. The pipeline's
// prologue_kernel and finalize_kernel wrap them, and so do kernels that fuse them with a
// sampler's per-chain step (the HMC kick and drift), which saves a launch and its fixed cost
// per step at small batches.
#pragma once

#include <hip/hip_runtime.h>

#include "glens_device.h"
#include "glens_fit_device.h"

namespace glens {

// ------------------------------------------------------------------------------------------
// prologue: one 64-lane block per particle. Lane 0 decodes the mass, lanes 1 and 2 the
// light profiles and lanes 3 .. one shapelet coefficient each, while lane n (1 <= n <
// kMaxTerms) computes the series ratio c_n / c_(n-1) and the increment of d log c_n / dt;
// inclusive scans across the wave (product and sum) then give every lane its c_n and
// d log c_n / dt; lane 63 looks for the floored sub-pixel while the others fill the power
// tables; last, the lanes store the series coefficients.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void prologue_particle(const SysDesc& s, int p) {
  static_assert(kMaxTerms <= 63, "one lane per series term, lane 63 free");
  static_assert(3 + kMaxShp <= 64, "one lane per shapelet coefficient");
  __shared__ float th[kMaxParams];
  const int d = s.d, lane = threadIdx.x;
  for (int j = lane; j < d; j += blockDim.x) {
    const size_t i = (size_t)p * d + j;
    if (s.z) {
      th[j] = bijector_fwd(s.prior[j], s.z[i]);
      s.theta_out[i] = th[j];
    } else {
      th[j] = s.theta[i];
    }
  }
  __syncthreads();
  PConst& c = s.pc[p];
  // the decode, spread over lanes: the mass on lane 0, the lights and shapelet coefficients
  // on lanes 1 ..; the series ratios on lanes 1 .. kMaxTerms - 1
  if (lane == 0) decode_mass(th, s.mass, s.shear, c);
  decode_lights_lane(th, s.mass, s.shear, s.lens_light, s.nmax, c, lane);
  const double t = (s.mass == 1) ? double(th[1]) - 1.0 : 1.0;
  double cn = 1.0, dsum = 0.0;  // lane n: c_n / c_(n-1) and its d log / dt increment (n >= 1)
  if (lane > 0 && lane < kMaxTerms) series_step(lane, t, cn, dsum);
  for (int o = 1; o < 64; o <<= 1) {  // inclusive scans: c_n and d log c_n / dt on lane n
    const double pc = __shfl_up(cn, o, 64), pd = __shfl_up(dsum, o, 64);
    if (lane >= o) {
      cn *= pc;
      dsum += pd;
    }
  }
  __syncthreads();
  // lane 63 looks for the floored sub-pixel; the others fill the power tables (both from
  // decode_mass's constants, written before the barrier)
  if (lane == 63)
    decode_floor(s, c);
  else
    pow_tables_lane(c.t, log2(c.bmass), lane, 63, c.pw);
  if (lane < kMaxTerms) series_store(c, lane, cn, dsum);
}

// ------------------------------------------------------------------------------------------
// finalize: one 64-lane block (a single wave) per particle; lanes sum the tiles' partial
// accumulators (in tile order), lane 0 maps them to the parameter gradient (the shapelet
// coefficients' components one per lane); a vector whose log L or gradient is not finite
// gets log L = -inf and a zero gradient
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void finalize_particle(const SysDesc& s, int p) {
  __shared__ double a[kNAcc];
  const int ns = s.nmax < 0 ? A_SHP_BETA : A_SHP_C + (s.nmax + 1) * (s.nmax + 2) / 2;
  const double* acc = s.acc + (size_t)p * s.tiles * kNAcc;
  for (int q = threadIdx.x; q < ns; q += blockDim.x) {
    double v = 0.0;
#pragma unroll 8
    for (int t = 0; t < s.tiles; ++t) v += acc[t * kNAcc + q];
    a[q] = v;
  }
  __syncthreads();
  const PConst& c = s.pc[p];
  if (threadIdx.x == 0 && c.fl_i >= 0) {
    // the floored sub-pixel: g = sbar d(source light)/d(beta) there (FP64), contracted with
    // the prologue's exact deflection derivatives; shear terms as the main loop forms them
    const int k = s.k, HW = s.H * s.W;
    const int pi = c.fl_i / k, pj = c.fl_j / k, sub = (c.fl_i - pi * k) * k + (c.fl_j - pj * k);
    const int pix = pi * s.W + pj;
    const double sb = s.sbar[(size_t)p * HW + pix];
    const float2 bs = s.beta[((size_t)p * k * k + sub) * HW + pix];
    double gx, gy;
    source_light_grad(c, s.nmax, bs.x, bs.y, gx, gy);
    gx *= sb;
    gy *= sb;
    a[A_M_ALPHA] += gx * c.fl_a[0] + gy * c.fl_a[1];
    a[A_M_T] += gx * c.fl_d[0][0] + gy * c.fl_d[0][1];
    a[A_M_E1] += gx * c.fl_d[1][0] + gy * c.fl_d[1][1];
    a[A_M_E2] += gx * c.fl_d[2][0] + gy * c.fl_d[2][1];
    a[A_M_X] -= gx * c.fl_d[3][0] + gy * c.fl_d[3][1];  // d/dx = -d/dx_c
    a[A_M_Y] -= gx * c.fl_d[4][0] + gy * c.fl_d[4][1];
    const double x = float(subpix_coord(s.x0, c.fl_j, s.dxs));
    const double y = float(subpix_coord(s.y0, c.fl_i, s.dxs));
    a[A_M_G1] += gx * x - gy * y;
    a[A_M_G2] += gx * y + gy * x;
  }
  __syncthreads();
  // lane 0 maps the sums (to LDS, not to a lane-private array the compiler would spill);
  // the lanes then check and store the components
  __shared__ float gr[kMaxParams];
  // the shapelet coefficients' components (if any) follow the others, one per lane
  __shared__ int s_j0;
  if (threadIdx.x == 0) s_j0 = map_gradient(c, a, s.mass, s.shear, s.lens_light, s.nmax, gr);
  __syncthreads();
  const int M = s.nmax < 0 ? 0 : (s.nmax + 1) * (s.nmax + 2) / 2;
  for (int q = threadIdx.x; q < M; q += blockDim.x) gr[s_j0 + q] = shapelet_coef_grad(c, a, q);
  __syncthreads();
  const int j = s_j0 + M;
  int bad = 0;
  for (int q = threadIdx.x; q < j; q += blockDim.x) bad |= !isfinite(gr[q]);
  const bool ok = isfinite(s.logl[p]) && !__any(bad);
  float* out = s.grad + (size_t)p * s.d;
  for (int q = threadIdx.x; q < j; q += blockDim.x) out[q] = ok ? gr[q] : 0.f;
  if (threadIdx.x == 0 && !ok) s.logl[p] = -INFINITY;
}

}  // namespace glens
