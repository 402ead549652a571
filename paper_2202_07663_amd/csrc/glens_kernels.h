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
#include "glens_particle.h"

namespace glens {

constexpr int kSubThreads = 256;
constexpr int kConvThreads = 256;
constexpr int kConvRows = 8;  // output rows per lane in the PSF pass
constexpr int kConvMaxStrips = 8;  // strips per lane: (H/8 rounded up) * W <= 8 * 256

// prologue: one 64-lane block per particle (prologue_particle)
__global__ void __launch_bounds__(64) prologue_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  prologue_particle(g.sys[si], blockIdx.x - g.block0[si]);
}

// ------------------------------------------------------------------------------------------
// sub-pixel forward: lanes own pixels, loop over the k x k sub-pixels
// ------------------------------------------------------------------------------------------
// Copies the particle's derivative-series coefficients to LDS (read uniformly by every lane).
__device__ __forceinline__ void stage_series(const PConst& c, float* s_nc, float* s_dc) {
  for (int n = threadIdx.x; n < kMaxTerms; n += blockDim.x) {
    s_nc[n] = c.nc[n];
    s_dc[n] = c.dc[n];
  }
  __syncthreads();
}

template <int MASS, int LL, int NMAX>
__device__ __forceinline__ float surface_brightness(const PConst& c, const double* cs,
                                                    const double* s_pw, double x, double y,
                                                    bool at_floor, const float* shp,
                                                    float2& sd) {
  ray_trace<MASS>(c, cs, s_pw, x, y, at_floor, sd.x, sd.y);
  float v = sersic_fwd(c.src, sd.x, sd.y);
  if (NMAX >= 0) v += shapelet_fwd<(NMAX < 0 ? 0 : NMAX)>(c, sd.x, sd.y, shp);
  if (LL) v += sersic_fwd(c.lens, float(x - c.lxs), float(y - c.lys));
  return v;
}

// MASS: 0 SIE, 1 EPL; LL: lens light on (1) or off (0); NMAX: shapelet order (-1: none).
// Every system of one launch has the same (MASS, LL, NMAX).
// The pixels [p0, p1) of one particle's model image. The restrict qualifiers tell the compiler
// that the image stores do not write the particle's constants, which then stay scalar loads.
template <int MASS, int LL, int NMAX>
// beta (or null): where beta - x_s of each sub-pixel is kept for the adjoint, [k^2][H][W].
__device__ __forceinline__ void forward_pixels(const SysDesc& s, const PConst* __restrict__ c,
                                               const double* cs, const double* s_pw,
                                               float* __restrict__ out,
                                               float2* __restrict__ beta, int p0, int p1) {
  const int W = s.W, k = s.k;
  // shapelet coefficients held in vector registers for the whole loop (an empty asm with a
  // vector-register operand): the scalar registers, which the compiler had filled, keep the
  // other constants instead of reloading them every sub-pixel
  constexpr int M = NMAX < 0 ? 1 : (NMAX + 1) * (NMAX + 2) / 2;
  float shp[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    shp[q] = NMAX < 0 ? 0.f : c->shp[q];
    asm("" : "+v"(shp[q]));
  }
  for (int pix = p0 + threadIdx.x; pix < p1; pix += blockDim.x) {
    const int i = pix / W, j = pix - i * W;
    float sum = 0.f;
    for (int a = 0; a < k; ++a) {
      const double y = subpix_coord(s.y0, i * k + a, s.dxs);
      for (int b = 0; b < k; ++b) {
        const double x = subpix_coord(s.x0, j * k + b, s.dxs);
        // the SIE's floored sub-pixel takes the prologue's frozen-radius deflection
        const bool at_floor = MASS == 0 && i * k + a == c->fl_i && j * k + b == c->fl_j;
        float2 sd;
        sum += surface_brightness<MASS, LL, NMAX>(*c, cs, s_pw, x, y, at_floor, shp, sd);
        if (beta) {  // streamed past the caches: read once, by the adjoint, much later
          float* bp = reinterpret_cast<float*>(beta + (a * k + b) * (s.H * W) + pix);
          __builtin_nontemporal_store(sd.x, bp);
          __builtin_nontemporal_store(sd.y, bp + 1);
        }
      }
    }
    out[pix] = sum * s.inv_k2;
  }
}

template <int MASS, int LL, int NMAX>
__global__ void __launch_bounds__(kSubThreads) subpix_fwd_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int lb = blockIdx.x - g.block0[si];
  const int part = lb / s.ftiles, tile = lb - part * s.ftiles;
  const PConst& c = s.pc[part];
  // the power tables in LDS (lanes read entries of their own); the value series' coefficients
  // stay in the particle's constants, read through the scalar cache: uniform over the
  // workgroup, they enter the series' FMAs as scalar operands
  __shared__ double s_pw[kPowExp + kPowSeg * 8];
  for (int i = threadIdx.x; i < kPowExp + kPowSeg * 8; i += blockDim.x) s_pw[i] = c.pw[i];
  __syncthreads();
  const int HW = s.H * s.W;
  const int p0 = tile * s.fpix_per_tile;
  const int p1 = min(HW, p0 + s.fpix_per_tile);
  float2* beta = s.mode == 2 && s.beta ? s.beta + (size_t)part * s.k * s.k * HW : nullptr;
  forward_pixels<MASS, LL, NMAX>(s, &c, c.c, s_pw, s.m0 + (size_t)part * HW, beta, p0, p1);
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
                                                float* acc, int b0 = 0, int bstep = 1) {
  constexpr int R = kConvRows;
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.f;
#pragma unroll 1
  for (int b = b0; b < K; b += bstep) {
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
// PSF pass on matrix cores. One workgroup (4 waves) per particle. Each operand is scaled by a
// power of two (exact) so that its largest magnitude lies in [2^14, 2^15), then split into two
// fp16 parts, x = h + l with h = f16(x) and l = f16(x - h) (the difference is exact in FP32),
// which represents it to about 2^-22 of itself: the scaled padded image sits in LDS as two
// fp16 arrays, and the Toeplitz operands of the PSF are built (scaled and split) once per
// model. Each output tile of 16 rows x N columns takes, for every PSF row a, three
// v_mfma_f32_16x16x32_f16 accumulating in FP32 (hl + lh first, then hh; the dropped l.l term
// is below 2^-22 of the product), and the result is scaled back. Against an FP64 sum this
// keeps pixel errors near 6e-8, as an FP32 sum does. Operand layouts of the instruction (one
// wave; lane l, element e): A[m][k] in lane m + 16 (k / 8), element k % 8; B[k][n] in lane
// n + 16 (k / 8), element k % 8; D[m][n] in lane n + 16 (m / 4), element m % 4. Going from
// PSF row a to a + 1 moves a tile's image rows down by one: lane (m, k / 8) takes the
// fragment of lane (m + 1, k / 8) by a DPP row shift, and only the lanes with m = 15 read LDS.
// Per pixel the likelihood and seed arithmetic is that of conv_kernel.
// ------------------------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x -> two fp16 parts, stored at p[0], p[stride]
__device__ __forceinline__ void split2_f16(float x, uint16_t* p, int stride) {
  const _Float16 h = static_cast<_Float16>(x);
  p[0] = __builtin_bit_cast(uint16_t, h);
  p[stride] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(x - static_cast<float>(h)));
}

// Exponent s with max_abs 2^s in [2^14, 2^15) (0 for zero or non-finite values).
__device__ __forceinline__ int f16_scale_exp(float max_abs) {
  if (!(max_abs > 0.f) || !(max_abs < INFINITY)) return 0;
  int e;
  frexpf(max_abs, &e);  // max_abs = f 2^e, f in [0.5, 1)
  return 15 - e;
}

// Largest value over the block, returned to every thread.
__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  float m = red[0];
  for (int w = 1; w < nw; ++w) m = fmaxf(m, red[w]);
  return m;
}

// Eight consecutive fp16 from LDS at an 8-byte aligned address.
__device__ __forceinline__ f16x8 lds_frag(const uint16_t* p) {
  const uint2 a = reinterpret_cast<const uint2*>(p)[0], b = reinterpret_cast<const uint2*>(p)[1];
  return __builtin_bit_cast(f16x8, make_uint4(a.x, a.y, b.x, b.y));
}

// Lane i of each 16-lane row takes the fragment of lane i + 1 (DPP row_shl:1); lane 15 keeps
// its own.
__device__ __forceinline__ int dpp_row_next(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x101, 0xF, 0xF, false);
}
__device__ __forceinline__ f16x8 shift_rows(f16x8 f) {
  int4 v = __builtin_bit_cast(int4, f);
  v.x = dpp_row_next(v.x);
  v.y = dpp_row_next(v.y);
  v.z = dpp_row_next(v.z);
  v.w = dpp_row_next(v.w);
  return __builtin_bit_cast(f16x8, v);
}

__device__ __forceinline__ f32x4 mfma_f16(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// acc[v] = correlation of the scaled LDS image (parts x, x + nel) with the scaled PSF over
// the wave's tiles wave + 4 (U0 + v), v < G. tab: this direction's fragments [K][64][h, l];
// those of row a + 2 are loaded while row a is computed. Each product is issued over the G
// tiles before the next, so consecutive matrix instructions are independent.
template <int U0, int G>
__device__ __forceinline__ void mfma_tiles(const uint16_t* x, int nel, const MfmaGeom& q,
                                           const uint4* __restrict__ tab, int K, int wave,
                                           f32x4* acc) {
  const int lane = threadIdx.x & 63, mr = lane & 15, g = lane >> 4;
  int off[G];  // this lane's fragment offset in tile v at row a = 0
  f16x8 ah[G], al[G];
#pragma unroll
  for (int v = 0; v < G; ++v) {
    const int t = wave + 4 * (U0 + v);
    const int tr = t / q.TC, tc = t - tr * q.TC;
    off[v] = (tr * 16 + mr) * q.pitch + tc * q.N + 8 * g;
    ah[v] = lds_frag(x + off[v]);
    al[v] = lds_frag(x + off[v] + nel);
    acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // PSF fragments two rows ahead (an L2 round trip is longer than one row's products)
  const uint4* tb = tab + lane * 2;
  uint4 nh = tb[0], nl = tb[1], nnh = nh, nnl = nl;
  if (K > 1) {
    nnh = tb[128];
    nnl = tb[129];
  }
  for (int a = 0; a < K; ++a) {
    const f16x8 bh = __builtin_bit_cast(f16x8, nh);
    const f16x8 bl = __builtin_bit_cast(f16x8, nl);
    nh = nnh;
    nl = nnl;
    if (a + 2 < K) {
      nnh = tb[(a + 2) * 128];
      nnl = tb[(a + 2) * 128 + 1];
    }
#pragma unroll
    for (int v = 0; v < G; ++v) acc[v] = mfma_f16(ah[v], bl, acc[v]);
#pragma unroll
    for (int v = 0; v < G; ++v) acc[v] = mfma_f16(al[v], bh, acc[v]);
#pragma unroll
    for (int v = 0; v < G; ++v) acc[v] = mfma_f16(ah[v], bh, acc[v]);
    if (a + 1 < K) {
#pragma unroll
      for (int v = 0; v < G; ++v) {
        ah[v] = shift_rows(ah[v]);
        al[v] = shift_rows(al[v]);
      }
      if (mr == 15) {  // the new bottom row of each tile
        const int ro = (a + 1) * q.pitch;
#pragma unroll
        for (int v = 0; v < G; ++v) {
          ah[v] = lds_frag(x + off[v] + ro);
          al[v] = lds_frag(x + off[v] + ro + nel);
        }
      }
    }
  }
}

// Per-pixel state of the matrix-core PSF kernel. The launch descriptor's fields are copied
// here once: read through the descriptor (a dynamically indexed kernel argument) they were
// loaded again for every pixel.
struct MfmaPass {
  const MfmaGeom& q;
  int wave;
  int unscale;        // exponent that takes the scaled sums back: -(image scale + PSF scale)
  int H, W, mode;
  float s2b, inv_gt, inv_k2;
  const float* obs;   // [H][W]
  float* out;         // this particle's model image (mode 0) or sbar (adjoint pass)
  float* seed;        // LDS [H][W]
  double ll, c2;
};

// Pixels of tiles wave + 4 (U0 + v), v < G: element r of acc[v] is pixel (i0 + r, j).
// Forward (ADJ false): the model image, or the likelihood terms and the seed; adjoint: sbar.
template <int U0, int G, bool ADJ>
__device__ __forceinline__ void mfma_pixels(MfmaPass& P, const f32x4* acc) {
  const int lane = threadIdx.x & 63, n = lane & 15, r0 = 4 * (lane >> 4);
  const int H = P.H, W = P.W;
#pragma unroll
  for (int v = 0; v < G; ++v) {
    const int t = P.wave + 4 * (U0 + v), tr = t / P.q.TC, tc = t - tr * P.q.TC;
    const int j = tc * P.q.N + n, i0 = tr * 16 + r0;
    if (n >= P.q.N || j >= W) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + r;
      if (i >= H) break;
      const float m = ldexpf(acc[v][r], P.unscale);
      const int px = i * W + j;
      if (ADJ) {
        P.out[px] = m * P.inv_k2;
      } else if (P.mode == 0) {
        P.out[px] = m;
      } else {
        const float pos = m > 0.f ? m : 0.f;
        const float s2 = P.s2b + pos * P.inv_gt;
        const float res = P.obs[px] - m;
        const float is2 = rcp_f32(s2);
        const float chi = res * res * is2;
        P.c2 += double(chi);
        P.ll += double(chi + kLn2f * log2_f32(6.283185307179586f * s2));
        const float sp = m > 0.f ? P.inv_gt : 0.f;
        P.seed[px] = res * is2 + 0.5f * sp * (res * res * is2 * is2 - is2);
      }
    }
  }
}

// Tiles U0 .. U0 + G - 1 of the wave: correlate, then the per-pixel step.
template <int U0, int G, bool ADJ>
__device__ __forceinline__ void mfma_group(MfmaPass& P, const uint16_t* x, int nel,
                                           const uint4* tab, int K) {
  f32x4 acc[G];
  mfma_tiles<U0, G>(x, nel, P.q, tab, K, P.wave, acc);
  mfma_pixels<U0, G, ADJ>(P, acc);
}

// The wave's ntw tiles (wave-uniform) in groups of at most five, as even as possible: a
// group's products hide the latency of the PSF fragment loads only when it has several tiles.
template <bool ADJ>
__device__ __forceinline__ void mfma_pass(MfmaPass& P, const uint16_t* x, int nel,
                                          const uint4* tab, int K, int ntw) {
  static_assert(kMfmaWaveTiles == 16, "group table for up to 16 tiles");
#define GL_G(U0, G) mfma_group<U0, G, ADJ>(P, x, nel, tab, K)
  switch (ntw) {
    case 1: GL_G(0, 1); break;
    case 2: GL_G(0, 2); break;
    case 3: GL_G(0, 3); break;
    case 4: GL_G(0, 4); break;
    case 5: GL_G(0, 5); break;
    case 6: GL_G(0, 3); GL_G(3, 3); break;
    case 7: GL_G(0, 4); GL_G(4, 3); break;
    case 8: GL_G(0, 4); GL_G(4, 4); break;
    case 9: GL_G(0, 5); GL_G(5, 4); break;
    case 10: GL_G(0, 5); GL_G(5, 5); break;
    case 11: GL_G(0, 4); GL_G(4, 4); GL_G(8, 3); break;
    case 12: GL_G(0, 4); GL_G(4, 4); GL_G(8, 4); break;
    case 13: GL_G(0, 5); GL_G(5, 4); GL_G(9, 4); break;
    case 14: GL_G(0, 5); GL_G(5, 5); GL_G(10, 4); break;
    case 15: GL_G(0, 5); GL_G(5, 5); GL_G(10, 5); break;
    case 16: GL_G(0, 4); GL_G(4, 4); GL_G(8, 4); GL_G(12, 4); break;
    default: break;
  }
#undef GL_G
}

// Four waves per SIMD (at most 128 VGPRs) and at most 40 KB of LDS at the 60 x 60, K = 21
// size let four workgroups share a CU: 4096 particles then fill the chip in four rounds
// instead of five and a third.
__global__ void __launch_bounds__(kConvThreads) __attribute__((amdgpu_waves_per_eu(4)))
conv_mfma_kernel(Group g) {
  extern __shared__ __align__(16) uint16_t xlds[];
  __shared__ double red[kConvThreads / 64];
  __shared__ float redf[kConvThreads / 64];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int part = blockIdx.x - g.block0[si];
  const int H = s.H, W = s.W, HW = H * W, K = s.K, C = (K - 1) / 2, mode = s.mode;
  const MfmaGeom q = mfma_geom(H, W, K);
  const int nel = q.Hq * q.pitch;  // fp16 per part (a multiple of 4)
  float* seed = reinterpret_cast<float*>(xlds + 2 * nel);
  for (int i = threadIdx.x; i < nel / 4; i += blockDim.x)
    reinterpret_cast<uint4*>(xlds)[i] = make_uint4(0u, 0u, 0u, 0u);
  // the image goes through the (still unused) seed area: one coalesced pass over global
  // memory with many loads in flight, its largest magnitude found on the way
  const float* m0 = s.m0 + (size_t)part * HW;
  float mx = 0.f;
#pragma unroll 8
  for (int idx = threadIdx.x; idx < HW; idx += blockDim.x) {
    const float v = m0[idx];
    seed[idx] = v;
    mx = fmaxf(mx, fabsf(v));
  }
  const int sx = f16_scale_exp(block_max(mx, redf));  // its barriers also end the zero fill
  for (int idx = threadIdx.x; idx < HW; idx += blockDim.x) {
    const int i = idx / W, j = idx - i * W;
    split2_f16(ldexpf(seed[idx], sx), xlds + (i + C) * q.pitch + j + C, nel);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  // tiles of this wave (wave-uniform: kept in a scalar register)
  const int ntw = __builtin_amdgcn_readfirstlane(wave < q.T ? (q.T - wave + 3) / 4 : 0);
  MfmaPass P{q, wave, -(sx + s.psf_mfma_exp), H, W, mode, s.s2b, s.inv_gt, s.inv_k2, s.obs,
             (mode == 0 ? s.img : s.sbar) + (size_t)part * HW, seed, 0.0, 0.0};
  mfma_pass<false>(P, xlds, nel, s.psf_mfma, K, ntw);
  if (mode == 0) return;
  const double tot = block_sum(P.ll, red);
  if (threadIdx.x == 0) {
    const double v = -0.5 * tot;
    s.logl[part] = isfinite(v) ? v : -INFINITY;
  }
  if (s.chi2) {
    const double ctot = block_sum(P.c2, red);
    if (threadIdx.x == 0) s.chi2[part] = ctot;
  }
  if (mode != 2) return;
  // every wave is done with the image (block_max below starts with a barrier): its interior
  // takes the scaled seed
  mx = 0.f;
  for (int idx = threadIdx.x; idx < HW; idx += blockDim.x) mx = fmaxf(mx, fabsf(seed[idx]));
  const int ss = f16_scale_exp(block_max(mx, redf));
  for (int idx = threadIdx.x; idx < HW; idx += blockDim.x) {
    const int i = idx / W, j = idx - i * W;
    split2_f16(ldexpf(seed[idx], ss), xlds + (i + C) * q.pitch + j + C, nel);
  }
  __syncthreads();
  // d logL / d m0 = correlation of the pixel seed with the (unflipped) PSF
  P.unscale = -(ss + s.psf_mfma_exp);
  P.out = s.sbar + (size_t)part * HW;
  mfma_pass<true>(P, xlds, nel, s.psf_mfma + 2 * 64 * K, K, ntw);
}

// ------------------------------------------------------------------------------------------
// Banded PSF pass for small batches: one workgroup per (particle, band of rows), so that a
// few particles still spread over many CUs. Band b owns output rows [b R_b, (b+1) R_b) and
// loads the rows of its input it needs (C = (K-1)/2 more on either side). Three kernels:
//   conv_band_kernel       the PSF, the likelihood terms (partial sums per band) and the
//                          adjoint seed of each pixel (to a [P][H][W] buffer);
//   conv_band_adj_kernel   the correlation of the seed with the PSF; the first band of a
//                          particle also adds the likelihood partials (band order);
//   conv_band_sum_kernel   the same addition when there is no adjoint pass.
// With band_split = 1 the arithmetic per pixel is that of conv_kernel (only the order of the
// log L sum differs). Very small batches split each strip's K PSF columns over G = 2 or 4
// adjacent lanes (columns g, g + G, ...), whose partial sums are then added by an xor
// butterfly: more lanes in flight and K^2 kConvRows / G FMAs in each lane's chain.
// ------------------------------------------------------------------------------------------
static_assert(kConvThreads % 4 == 0, "whole lane groups of the split PSF columns");
struct Band {
  int part, band, r0, r1, nsr, Hs;
};

// Sums a strip's partial accumulators over the G lanes that share it (adjacent lanes, G a
// power of two <= 4, every lane of the group active); each lane ends with the full sums.
__device__ __forceinline__ void split_sum(float* acc, int G) {
  for (int o = 1; o < G; o <<= 1) {
#pragma unroll
    for (int r = 0; r < kConvRows; ++r) acc[r] += __shfl_xor(acc[r], o, 64);
  }
}

__device__ __forceinline__ Band band_of(const SysDesc& s, int local, int K) {
  Band b;
  b.part = local / s.bands;
  b.band = local - b.part * s.bands;
  b.r0 = b.band * s.band_rows;
  b.r1 = min(s.H, b.r0 + s.band_rows);
  b.nsr = (b.r1 - b.r0 + kConvRows - 1) / kConvRows;
  b.Hs = (b.nsr * kConvRows + K - 1) | 1;
  return b;
}

// Rows [r0 - C, r1 + C) of src (zero outside the image) into the column-major LDS tile.
template <int K>
__device__ __forceinline__ void load_band(const float* __restrict__ src, const SysDesc& s,
                                          const Band& b, float* A) {
  constexpr int C = (K - 1) / 2;
  const int W = s.W, Wp = W + K - 1;
  for (int idx = threadIdx.x; idx < b.Hs * Wp; idx += blockDim.x) A[idx] = 0.f;
  __syncthreads();
  const int lo = max(0, b.r0 - C), hi = min(s.H, b.r1 + C);
  for (int idx = threadIdx.x; idx < (hi - lo) * W; idx += blockDim.x) {
    const int i = lo + idx / W, j = idx - (idx / W) * W;
    A[(j + C) * b.Hs + (i - b.r0) + C] = src[(size_t)i * W + j];
  }
  __syncthreads();
}

template <int K>
__global__ void __launch_bounds__(kConvThreads) conv_band_kernel(Group g) {
  extern __shared__ float lds[];
  __shared__ double red[kConvThreads / 64];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const Band b = band_of(s, blockIdx.x - g.block0[si], K);
  constexpr int R = kConvRows;
  const int W = s.W, HW = s.H * W, mode = s.mode;
  load_band<K>(s.m0 + (size_t)b.part * HW, s, b, lds);
  double ll = 0.0, c2 = 0.0;
  // work items (strip, column, PSF-column share); the G lanes of one strip are adjacent, and
  // blockDim and the item count are multiples of G, so they run the loop together
  const int G = s.band_split, gs = G >> 1;  // G = 1, 2, 4: log2 G = G / 2
  for (int sidx = threadIdx.x; sidx < b.nsr * W * G; sidx += blockDim.x) {
    const int item = sidx >> gs, g0 = sidx & (G - 1);
    const int st = item / W, j = item - st * W, i0 = st * R;
    float acc[R];
    if (G == 1) {
      correlate_strip<K>(lds, b.Hs, i0, j, s.psf_flip, acc);
    } else {
      correlate_strip<K>(lds, b.Hs, i0, j, s.psf_flip, acc, g0, G);
      split_sum(acc, G);
      if (g0 != 0) continue;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = b.r0 + i0 + r;
      if (i >= b.r1) break;
      const float m = acc[r];
      const size_t o = (size_t)b.part * HW + i * W + j;
      if (mode == 0) {
        s.img[o] = m;
        continue;
      }
      const float pos = m > 0.f ? m : 0.f;
      const float s2 = s.s2b + pos * s.inv_gt;
      const float res = s.obs[i * W + j] - m;
      const float is2 = rcp_f32(s2);
      const float chi = res * res * is2;
      c2 += double(chi);
      ll += double(chi + kLn2f * log2_f32(6.283185307179586f * s2));
      if (mode == 2) {
        const float sp = m > 0.f ? s.inv_gt : 0.f;
        s.seed[o] = res * is2 + 0.5f * sp * (res * res * is2 * is2 - is2);
      }
    }
  }
  if (mode == 0) return;
  const double tot = block_sum(ll, red);
  const double ctot = block_sum(c2, red);
  if (threadIdx.x == 0) {
    double* lp = s.lpart + ((size_t)b.part * kConvMaxBands + b.band) * 2;
    lp[0] = tot;
    lp[1] = ctot;
  }
}

// log L and chi^2 of one particle from its bands' partial sums.
__device__ __forceinline__ void band_totals(const SysDesc& s, int part) {
  const double* lp = s.lpart + (size_t)part * kConvMaxBands * 2;
  double tot = 0.0, ctot = 0.0;
  for (int q = 0; q < s.bands; ++q) {
    tot += lp[2 * q];
    ctot += lp[2 * q + 1];
  }
  const double v = -0.5 * tot;
  s.logl[part] = isfinite(v) ? v : -INFINITY;
  if (s.chi2) s.chi2[part] = ctot;
}

template <int K>
__global__ void __launch_bounds__(kConvThreads) conv_band_adj_kernel(Group g) {
  extern __shared__ float lds[];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const Band b = band_of(s, blockIdx.x - g.block0[si], K);
  constexpr int R = kConvRows;
  const int W = s.W, HW = s.H * W;
  if (b.band == 0 && threadIdx.x == 0) band_totals(s, b.part);
  load_band<K>(s.seed + (size_t)b.part * HW, s, b, lds);
  const int G = s.band_split, gs = G >> 1;  // G = 1, 2, 4: log2 G = G / 2
  for (int sidx = threadIdx.x; sidx < b.nsr * W * G; sidx += blockDim.x) {
    const int item = sidx >> gs, g0 = sidx & (G - 1);
    const int st = item / W, j = item - st * W, i0 = st * R;
    float acc[R];
    if (G == 1) {
      correlate_strip<K>(lds, b.Hs, i0, j, s.psf, acc);
    } else {
      correlate_strip<K>(lds, b.Hs, i0, j, s.psf, acc, g0, G);
      split_sum(acc, G);
      if (g0 != 0) continue;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = b.r0 + i0 + r;
      if (i >= b.r1) break;
      s.sbar[(size_t)b.part * HW + i * W + j] = acc[r] * s.inv_k2;
    }
  }
}

__global__ void __launch_bounds__(64) conv_band_sum_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int p = (blockIdx.x - g.block0[si]) * blockDim.x + threadIdx.x;
  if (p < s.P) band_totals(s, p);
}

// ------------------------------------------------------------------------------------------
// sub-pixel adjoint
// ------------------------------------------------------------------------------------------
template <int NMAX>
constexpr int n_slots() {
  return NMAX < 0 ? A_SHP_BETA : A_SHP_C + (NMAX + 1) * (NMAX + 2) / 2;
}

constexpr int halved(int n) { return n > 1 ? n / 2 : 1; }

// One step of the transposed butterfly below for a lane holding NV values (all indices
// compile-time, so the values stay in registers).
template <int NV>
__device__ __forceinline__ void wave_sum_step(double* v, int off, int lane) {
  if constexpr (NV > 1) {
    const bool up = lane & off;
#pragma unroll
    for (int i = 0; i < NV / 2; ++i) {
      const double send = up ? v[i] : v[i + NV / 2];
      const double keep = up ? v[i + NV / 2] : v[i];
      v[i] = keep + __shfl_xor(send, off, 64);
    }
  } else {
    v[0] += __shfl_xor(v[0], off, 64);
  }
}

// Wave sums of NS per-lane FP32 values, in FP64, written to out[0 .. NS). A transposed
// butterfly: with the values padded to N (a power of two), at the step with lane offset o a
// lane keeps one half of its values, sends the other half to lane ^ o and adds what it
// receives, so each step halves the values a lane holds. Every sum pairs lanes in the same
// order as a separate xor butterfly per value would, with about N shuffles instead of
// 6 NS. The first step shuffles the FP32 values and adds them in FP64.
template <int NS>
__device__ __forceinline__ void wave_sums(const float* acc, double* out) {
  constexpr int N = NS <= 32 ? 32 : (NS <= 64 ? 64 : 128);
  static_assert(NS <= 128, "too many accumulators");
  const int lane = threadIdx.x & 63;
  double v[N / 2];
  {
    const bool up = lane & 32;
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const float lo = i < NS ? acc[i] : 0.f, hi = i + N / 2 < NS ? acc[i + N / 2] : 0.f;
      const float send = up ? lo : hi;
      v[i] = double(up ? hi : lo) + double(__shfl_xor(send, 32, 64));
    }
  }
  constexpr int n1 = N / 2, n2 = halved(n1), n3 = halved(n2), n4 = halved(n3), n5 = halved(n4);
  wave_sum_step<n1>(v, 16, lane);
  wave_sum_step<n2>(v, 8, lane);
  wave_sum_step<n3>(v, 4, lane);
  wave_sum_step<n4>(v, 2, lane);
  wave_sum_step<n5>(v, 1, lane);
  // lane l now holds value (l * N / 64) + i for i < N / 64 (N = 32: lanes 2q and 2q + 1
  // both hold value q)
  if (N >= 64) {
#pragma unroll
    for (int i = 0; i < N / 64; ++i) {
      const int q = lane * (N / 64) + i;
      if (q < NS) out[q] = v[i];
    }
  } else if ((lane & 1) == 0 && (lane >> 1) < NS) {
    out[lane >> 1] = v[0];
  }
}

// The sub-pixels of pixels [p0, p1) of one particle into the per-lane accumulators.
// GENERAL = false: the particle has no floored sub-pixel and |eps| >= kSxClosedMin.
template <int MASS, int LL, int NMAX, bool GENERAL>
__device__ __forceinline__ void adj_pixels(const SysDesc& s, const PConst& c,
                                           const float* s_nc, const float* s_dc,
                                           const float* shp, const float2* beta,
                                           const float* sbar, int p0, int p1, float* acc) {
  const int HW = s.H * s.W, W = s.W, k = s.k;
  const int fl_i = c.fl_i, fl_j = c.fl_j;
  for (int pix = p0 + threadIdx.x; pix < p1; pix += blockDim.x) {
    const int i = pix / W, j = pix - i * W;
    const float sb = sbar[pix];
    for (int a = 0; a < k; ++a) {
      const double y = subpix_coord(s.y0, i * k + a, s.dxs);
      for (int b = 0; b < k; ++b) {
        const double x = subpix_coord(s.x0, j * k + b, s.dxs);
        MassState m;
        const float* bp = reinterpret_cast<const float*>(beta + (a * k + b) * HW + pix);
        mass_jacobian_f32<MASS, GENERAL>(c, s_nc, s_dc, x, y, __builtin_nontemporal_load(bp),
                                         __builtin_nontemporal_load(bp + 1), m);
        // gx, gy: sb d(source light)/d(beta)
        float gx, gy;
        sersic_adj(c.src, m.sdx, m.sdy, sb, acc + A_SRC, gx, gy);
        if (NMAX >= 0) {
          float hx, hy;
          shapelet_adj<(NMAX < 0 ? 0 : NMAX)>(c, m.sdx, m.sdy, shp, sb, acc, hx, hy);
          gx += hx;
          gy += hy;
        }
        acc[A_SRC + L_DX] += gx;
        acc[A_SRC + L_DY] += gy;
        if (LL) {
          float lx, ly;
          sersic_adj(c.lens, float(x - c.lxs), float(y - c.lys), sb, acc + A_LENS, lx, ly);
          acc[A_LENS + L_DX] += lx;
          acc[A_LENS + L_DY] += ly;
        }
        // the floored sub-pixel's mass terms are added by finalize from the prologue's
        // exact derivatives
        const bool at_floor = GENERAL && i * k + a == fl_i && j * k + b == fl_j;
        mass_adjoint<MASS>(c, m, float(x), float(y),
                           at_floor ? Cx{0.f, 0.f} : Cx{gx, gy}, acc);
      }
    }
  }
}

template <int MASS, int LL, int NMAX>
__global__ void __launch_bounds__(kSubThreads) __attribute__((amdgpu_waves_per_eu(3)))
subpix_adj_kernel(Group g) {
  constexpr int NS = n_slots<NMAX>();
  __shared__ double red[kSubThreads / 64][NS];
  const int si = find_sys(g, blockIdx.x);
  const SysDesc& s = g.sys[si];
  const int lb = blockIdx.x - g.block0[si];
  const int part = lb / s.tiles, tile = lb - part * s.tiles;
  const PConst& c = s.pc[part];
  __shared__ float s_nc[kMaxTerms], s_dc[kMaxTerms];
  stage_series(c, s_nc, s_dc);
  // beta - x_s from the forward pass (kept there for gradient calls)
  const float2* beta = s.beta + (size_t)part * s.k * s.k * s.H * s.W;
  const int HW = s.H * s.W;
  const int p0 = tile * s.pix_per_tile;
  const int p1 = min(HW, p0 + s.pix_per_tile);
  const float* sbar = s.sbar + (size_t)part * HW;
  float acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.f;
  // shapelet coefficients in vector registers (as in the forward pass): their sums then start
  // from a register operand instead of a copy of a scalar one
  constexpr int M = NMAX < 0 ? 1 : (NMAX + 1) * (NMAX + 2) / 2;
  float shp[M];
#pragma unroll
  for (int q = 0; q < M; ++q) {
    shp[q] = NMAX < 0 ? 0.f : c.shp[q];
    asm("" : "+v"(shp[q]));
  }
  // the common case (no floored sub-pixel, |eps| >= kSxClosedMin) runs a loop without those
  // tests
  if (c.fl_i < 0 && !(c.epsabs < kSxClosedMin))
    adj_pixels<MASS, LL, NMAX, false>(s, c, s_nc, s_dc, shp, beta, sbar, p0, p1, acc);
  else
    adj_pixels<MASS, LL, NMAX, true>(s, c, s_nc, s_dc, shp, beta, sbar, p0, p1, acc);
  // FP64 sums: across the wave, then across the waves of the block
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  wave_sums<NS>(acc, red[wave]);
  __syncthreads();
  double* out = s.acc + ((size_t)part * s.tiles + tile) * kNAcc;
  for (int q = threadIdx.x; q < NS; q += blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += red[w][q];
    out[q] = v;
  }
}

// finalize: one 64-lane block per particle (finalize_particle)
__global__ void __launch_bounds__(64) finalize_kernel(Group g) {
  const int si = find_sys(g, blockIdx.x);
  finalize_particle(g.sys[si], blockIdx.x - g.block0[si]);
}

}  // namespace glens
