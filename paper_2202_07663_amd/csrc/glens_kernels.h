// HIP kernels of the batched lens likelihood and its adjoint.
//
// One call runs, per lens system and parameter vector ("particle"):
//   prologue       per-particle constants (decode, series coefficients, bijector)
//   subpix_fwd     sub-pixel forward model, k x k mean -> m0[P][H][W]
//   conv           PSF convolution in LDS, per-pixel log-likelihood terms summed in FP64,
//                  and (adjoint) the pixel seed d logL / d m and its correlation with the
//                  PSF -> sbar[P][H][W] = d logL / d (sub-pixel brightness)
//   subpix_adj     sub-pixel adjoint: recompute, local derivatives, per-lane FP32
//                  accumulators, FP64 cross-lane and cross-wave sums -> acc[P][tiles][slot]
//   finalize       sum over tiles and map the accumulators onto d logL / d theta
// Every launch takes a Group of systems that share the kernel configuration, so a
// continuous-batching server can advance many systems in one launch.
#pragma once

#include <hip/hip_runtime.h>

#include "glens_device.h"
#include "glens_fit_device.h"

namespace glens {

constexpr int kSubThreads = 256;
constexpr int kConvThreads = 256;
constexpr int kConvRows = 8;  // output rows per lane in the PSF pass
constexpr int kConvMaxStrips = 8;  // strips per lane: (H/8 rounded up) * W <= 8 * 256

// ------------------------------------------------------------------------------------------
// prologue: one lane per particle
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64) prologue_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int p = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (p >= s.P) return;
  float th[kMaxParams];
  const int d = s.d;
  if (s.z) {
    for (int j = 0; j < d; ++j) {
      th[j] = bijector_fwd(s.prior[j], s.z[(size_t)p * d + j]);
      s.theta_out[(size_t)p * d + j] = th[j];
    }
  } else {
    for (int j = 0; j < d; ++j) th[j] = s.theta[(size_t)p * d + j];
  }
  PConst c;
  decode_particle(th, s.mass, s.shear, s.lens_light, s.nmax, c);
  s.pc[p] = c;
}

// ------------------------------------------------------------------------------------------
// sub-pixel forward: lanes own pixels, loop over the k x k sub-pixels
// ------------------------------------------------------------------------------------------
// Copies the particle's series coefficients to LDS (read uniformly by every lane).
__device__ __forceinline__ void stage_series(const PConst& c, double* s_c, float* s_nc,
                                             float* s_dc) {
  for (int n = threadIdx.x; n < kMaxTerms; n += blockDim.x) {
    s_c[n] = c.c[n];
    s_nc[n] = c.nc[n];
    s_dc[n] = c.dc[n];
  }
  __syncthreads();
}

template <int MASS, int NMAX>
__device__ __forceinline__ float surface_brightness(const PConst& c, const double* s_c,
                                                    int lens_light, double x, double y) {
  MassState m;
  mass_eval<MASS, false>(c, s_c, nullptr, nullptr, x, y, m);
  float v = sersic_fwd(c.src, m.sdx, m.sdy);
  if (NMAX >= 0) v += shapelet_fwd<(NMAX < 0 ? 0 : NMAX)>(c, m.sdx, m.sdy);
  if (lens_light) v += sersic_fwd(c.lens, float(x - c.lxs), float(y - c.lys));
  return v;
}

template <int MASS, int NMAX>
__global__ void __launch_bounds__(kSubThreads) subpix_fwd_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int lb = blockIdx.x - g.block0[si];
  const int part = lb / s.tiles, tile = lb - part * s.tiles;
  const PConst& c = s.pc[part];
  __shared__ double s_c[kMaxTerms];
  __shared__ float s_nc[kMaxTerms], s_dc[kMaxTerms];
  stage_series(c, s_c, s_nc, s_dc);
  const int HW = s.H * s.W, W = s.W, k = s.k;
  const int p0 = tile * s.pix_per_tile;
  const int p1 = min(HW, p0 + s.pix_per_tile);
  float* out = s.m0 + (size_t)part * HW;
  for (int pix = p0 + threadIdx.x; pix < p1; pix += blockDim.x) {
    const int i = pix / W, j = pix - i * W;
    float sum = 0.f;
    for (int a = 0; a < k; ++a) {
      const double y = s.y0 + double(i * k + a) * s.dxs;
      for (int b = 0; b < k; ++b) {
        const double x = s.x0 + double(j * k + b) * s.dxs;
        sum += surface_brightness<MASS, NMAX>(c, s_c, s.lens_light, x, y);
      }
    }
    out[pix] = sum * s.inv_k2;
  }
}

// ------------------------------------------------------------------------------------------
// PSF convolution + likelihood (+ adjoint seed). One workgroup per particle; the image and
// its zero halo live in LDS. Each lane computes kConvRows consecutive rows of one column:
// per tap column it loads kConvRows + K - 1 values and does K * kConvRows FMAs with the taps
// as wave-uniform (scalar) operands.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) tot += red[w];
  return tot;  // valid on lane 0 of wave 0
}

// The padded image sits in LDS column-major (column pitch Hs, odd so that the lanes of a wave,
// which own consecutive columns, hit distinct banks). A lane's strip of kConvRows output rows
// in column j reads, per tap column b, kConvRows + K - 1 consecutive words at immediate
// offsets from one base address.
template <int K>
__device__ __forceinline__ void correlate_strip(const float* __restrict__ buf, int Hs, int i0,
                                                int j, const float* __restrict__ taps,
                                                float* acc) {
  constexpr int R = kConvRows;
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.f;
#pragma unroll 1
  for (int b = 0; b < K; ++b) {
    const float* colp = buf + (j + b) * Hs + i0;
    float col[R + K - 1];
#pragma unroll
    for (int rr = 0; rr < R + K - 1; ++rr) col[rr] = colp[rr];
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const float kv = taps[a * K + b];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fmaf(kv, col[r + a], acc[r]);
    }
  }
}

template <int K>
__global__ void __launch_bounds__(kConvThreads) conv_kernel(Group g) {
  extern __shared__ float lds[];
  __shared__ double red[kConvThreads / 64];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int part = blockIdx.x - g.block0[si];
  constexpr int R = kConvRows, C = (K - 1) / 2;
  const int H = s.H, W = s.W, HW = H * W;
  const int nstrip = (H + R - 1) / R;
  const int Hs = (nstrip * R + K - 1) | 1, Wp = W + K - 1, NP = Hs * Wp;
  const int mode = s.mode;
  float* A = lds;  // padded image; in the adjoint pass it holds the padded pixel seed
  const float* m0 = s.m0 + (size_t)part * HW;
  for (int idx = threadIdx.x; idx < NP; idx += blockDim.x) A[idx] = 0.f;
  __syncthreads();
  for (int idx = threadIdx.x; idx < HW; idx += blockDim.x) {  // coalesced global read
    const int i = idx / W, j = idx - i * W;
    A[(j + C) * Hs + i + C] = m0[idx];
  }
  __syncthreads();
  double ll = 0.0, c2 = 0.0;
  const float* obs = s.obs;
  // A lane owns at most kConvMaxStrips strips (checked on the host); their pixel seeds stay
  // in registers until every lane has finished reading the image.
  float seed[kConvMaxStrips][R];
#pragma unroll
  for (int t = 0; t < kConvMaxStrips; ++t) {
    const int sidx = threadIdx.x + t * blockDim.x;
    if (sidx >= nstrip * W) break;
    const int st = sidx / W, j = sidx - st * W, i0 = st * R;
    float acc[R];
    correlate_strip<K>(A, Hs, i0, j, s.psf_flip, acc);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      seed[t][r] = 0.f;
      if (i >= H) continue;
      const float m = acc[r];
      if (mode == 0) {
        s.img[(size_t)part * HW + i * W + j] = m;
      } else {
        const float pos = m > 0.f ? m : 0.f;
        const float s2 = s.s2b + pos * s.inv_gt;
        const float res = obs[i * W + j] - m;
        const float is2 = rcp_f32(s2);
        const float chi = res * res * is2;
        c2 += double(chi);
        ll += double(chi + kLn2f * log2_f32(6.283185307179586f * s2));
        const float sp = m > 0.f ? s.inv_gt : 0.f;
        seed[t][r] = res * is2 + 0.5f * sp * (res * res * is2 * is2 - is2);
      }
    }
  }
  if (mode == 0) return;
  const double tot = block_sum(ll, red);
  if (threadIdx.x == 0) {
    const double v = -0.5 * tot;
    s.logl[part] = isfinite(v) ? v : -INFINITY;
  }
  if (s.chi2) {
    const double ctot = block_sum(c2, red);
    if (threadIdx.x == 0) s.chi2[part] = ctot;
  }
  if (mode != 2) return;
  __syncthreads();  // every lane is done with the image: overwrite its interior with the seed
#pragma unroll
  for (int t = 0; t < kConvMaxStrips; ++t) {
    const int sidx = threadIdx.x + t * blockDim.x;
    if (sidx >= nstrip * W) break;
    const int st = sidx / W, j = sidx - st * W, i0 = st * R;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (i0 + r < H) A[(j + C) * Hs + i0 + r + C] = seed[t][r];
  }
  __syncthreads();
  // d logL / d m0 = correlation of the pixel seed with the (unflipped) PSF
#pragma unroll
  for (int t = 0; t < kConvMaxStrips; ++t) {
    const int sidx = threadIdx.x + t * blockDim.x;
    if (sidx >= nstrip * W) break;
    const int st = sidx / W, j = sidx - st * W, i0 = st * R;
    float acc[R];
    correlate_strip<K>(A, Hs, i0, j, s.psf, acc);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      if (i >= H) break;
      s.sbar[(size_t)part * HW + i * W + j] = acc[r] * s.inv_k2;
    }
  }
}

// ------------------------------------------------------------------------------------------
// sub-pixel adjoint
// ------------------------------------------------------------------------------------------
template <int NMAX>
constexpr int n_slots() {
  return NMAX < 0 ? A_SHP_BETA : A_SHP_C + (NMAX + 1) * (NMAX + 2) / 2;
}

template <int MASS, int NMAX>
__global__ void __launch_bounds__(kSubThreads) __attribute__((amdgpu_waves_per_eu(3)))
subpix_adj_kernel(Group g) {
  constexpr int NS = n_slots<NMAX>();
  __shared__ double red[kSubThreads / 64][NS];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int lb = blockIdx.x - g.block0[si];
  const int part = lb / s.tiles, tile = lb - part * s.tiles;
  const PConst& c = s.pc[part];
  __shared__ double s_c[kMaxTerms];
  __shared__ float s_nc[kMaxTerms], s_dc[kMaxTerms];
  stage_series(c, s_c, s_nc, s_dc);
  const int HW = s.H * s.W, W = s.W, k = s.k;
  const int p0 = tile * s.pix_per_tile;
  const int p1 = min(HW, p0 + s.pix_per_tile);
  const float* sbar = s.sbar + (size_t)part * HW;
  float acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.f;
  for (int pix = p0 + threadIdx.x; pix < p1; pix += blockDim.x) {
    const int i = pix / W, j = pix - i * W;
    const float sb = sbar[pix];
    for (int a = 0; a < k; ++a) {
      const double y = s.y0 + double(i * k + a) * s.dxs;
      for (int b = 0; b < k; ++b) {
        const double x = s.x0 + double(j * k + b) * s.dxs;
        MassState m;
        mass_eval<MASS, true>(c, s_c, s_nc, s_dc, x, y, m);
        float gx, gy;
        sersic_adj(c.src, m.sdx, m.sdy, sb, acc + A_SRC, gx, gy);
        if (NMAX >= 0) {
          float hx, hy;
          shapelet_adj<(NMAX < 0 ? 0 : NMAX)>(c, m.sdx, m.sdy, sb, acc, hx, hy);
          gx += hx;
          gy += hy;
        }
        acc[A_SRC + L_DX] += sb * gx;
        acc[A_SRC + L_DY] += sb * gy;
        if (s.lens_light) {
          float lx, ly;
          sersic_adj(c.lens, float(x - c.lxs), float(y - c.lys), sb, acc + A_LENS, lx, ly);
          acc[A_LENS + L_DX] += sb * lx;
          acc[A_LENS + L_DY] += sb * ly;
        }
        mass_adjoint<MASS>(c, m, float(x), float(y), Cx{sb * gx, sb * gy}, acc);
      }
    }
  }
  // FP64 sums: across the wave, then across the waves of the block
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  double* out = s.acc + ((size_t)part * s.tiles + tile) * kNAcc;
  for (int q = threadIdx.x; q < NS; q += blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += red[w][q];
    out[q] = v;
  }
}

// ------------------------------------------------------------------------------------------
// finalize: one lane per particle
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64) finalize_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int p = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (p >= s.P) return;
  const PConst& c = s.pc[p];
  const int ns = s.nmax < 0 ? A_SHP_BETA : A_SHP_C + (s.nmax + 1) * (s.nmax + 2) / 2;
  double a[kNAcc];
  for (int q = 0; q < ns; ++q) {
    double v = 0.0;
    for (int t = 0; t < s.tiles; ++t) v += s.acc[((size_t)p * s.tiles + t) * kNAcc + q];
    a[q] = v;
  }
  float gr[kMaxParams];
  const int j = map_gradient(c, a, s.mass, s.shear, s.lens_light, s.nmax, gr);
  bool ok = isfinite(s.logl[p]);
  for (int q = 0; q < j; ++q) ok = ok && isfinite(gr[q]);
  if (!ok) s.logl[p] = -INFINITY;
  float* out = s.grad + (size_t)p * s.d;
  for (int q = 0; q < j; ++q) out[q] = ok ? gr[q] : 0.f;
}

}  // namespace glens
