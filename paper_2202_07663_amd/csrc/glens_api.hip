// C ABI: models, gl_simulate, gl_loglik, gl_loglik_grad, errors; kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "glens_host.h"
#include "glens_kernels.h"

namespace glens {

// ------------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------------
static thread_local std::string t_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}
void clear_error() { t_err.clear(); }


int check_device_ptr(const void* p, const char* name) {
  if (!p) return set_error(GL_E_INVALID, "%s is NULL", name);
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(GL_E_INVALID, "%s is not a device pointer", name);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return set_error(GL_E_INVALID, "%s is not a device pointer", name);
  return GL_OK;
}

// ------------------------------------------------------------------------------------------
// descriptors
// ------------------------------------------------------------------------------------------
int nparams(int mass, int shear, int lens_light, int nmax) {
  return (mass == GL_MASS_EPL ? 6 : 5) + (shear ? 2 : 0) + (lens_light ? 7 : 0) + 7 +
         (nmax >= 0 ? 1 + (nmax + 1) * (nmax + 2) / 2 : 0);
}

int validate_desc(const gl_model_desc* d, ModelCfg* c) {
  if (!d) return set_error(GL_E_INVALID, "desc is NULL");
  if (d->H < 1 || d->W < 1) return set_error(GL_E_INVALID, "image size %dx%d", d->H, d->W);
  if (d->H > GL_MAX_IMAGE || d->W > GL_MAX_IMAGE)
    return set_error(GL_E_UNIMPLEMENTED, "image size %dx%d above %d", d->H, d->W, GL_MAX_IMAGE);
  if (!(d->pixel_scale > 0.f) || !std::isfinite(d->pixel_scale))
    return set_error(GL_E_INVALID, "pixel_scale must be > 0");
  if (d->k_super < 1) return set_error(GL_E_INVALID, "k_super must be >= 1");
  if (d->k_super > GL_MAX_KSUPER)
    return set_error(GL_E_UNIMPLEMENTED, "k_super above %d", GL_MAX_KSUPER);
  if (double(d->pixel_scale) / d->k_super < kMinPitch)
    return set_error(GL_E_UNIMPLEMENTED, "sub-pixel pitch pixel_scale / k_super below %g arcsec",
                     kMinPitch);
  if (d->mass != GL_MASS_SIE && d->mass != GL_MASS_EPL)
    return set_error(GL_E_INVALID, "mass must be GL_MASS_SIE or GL_MASS_EPL");
  if (d->shear != 0 && d->shear != 1) return set_error(GL_E_INVALID, "shear must be 0 or 1");
  if (d->lens_light != 0 && d->lens_light != 1)
    return set_error(GL_E_INVALID, "lens_light must be 0 or 1");
  if (d->shapelet_nmax < -1) return set_error(GL_E_INVALID, "shapelet_nmax must be >= -1");
  if (d->shapelet_nmax > GL_MAX_NMAX)
    return set_error(GL_E_UNIMPLEMENTED, "shapelet_nmax above %d", GL_MAX_NMAX);
  if (d->psf_size < 1 || d->psf_size % 2 == 0)
    return set_error(GL_E_INVALID, "psf_size must be odd and >= 1");
  if (d->psf_size > GL_MAX_PSF)
    return set_error(GL_E_UNIMPLEMENTED, "psf_size above %d", GL_MAX_PSF);
  if (!d->psf) return set_error(GL_E_INVALID, "psf is NULL");
  for (int i = 0; i < d->psf_size * d->psf_size; ++i)
    if (!std::isfinite(d->psf[i])) return set_error(GL_E_INVALID, "psf has non-finite values");
  if (!(d->sigma_bkg >= 0.f) || !std::isfinite(d->sigma_bkg))
    return set_error(GL_E_INVALID, "sigma_bkg must be >= 0");
  if (!(d->t_exp > 0.f) || !std::isfinite(d->t_exp)) return set_error(GL_E_INVALID, "t_exp must be > 0");
  if (!(d->gain > 0.f) || !std::isfinite(d->gain)) return set_error(GL_E_INVALID, "gain must be > 0");
  if (d->obs)
    for (int i = 0; i < d->H * d->W; ++i)
      if (!std::isfinite(d->obs[i])) return set_error(GL_E_INVALID, "obs has non-finite values");
  if (d->sigma_bkg == 0.f && d->obs == nullptr) {
    // fine: simulate-only
  }
  c->H = d->H;
  c->W = d->W;
  c->k = d->k_super;
  c->K = d->psf_size;
  c->pix = d->pixel_scale;
  c->mass = d->mass;
  c->shear = d->shear;
  c->lens_light = d->lens_light;
  c->nmax = d->shapelet_nmax;
  c->d = nparams(d->mass, d->shear, d->lens_light, d->shapelet_nmax);
  c->sigma_bkg = d->sigma_bkg;
  c->t_exp = d->t_exp;
  c->gain = d->gain;
  return GL_OK;
}

static uint16_t f16_bits(_Float16 h) {
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The device image of a system's fixed inputs, in the layout system_bind expects: the PSF,
// the flipped PSF, for K <= kMfmaMaxK the Toeplitz operands of the matrix-core PSF pass, and
// the observed image (zeros when there is none), each 256-byte aligned.
void system_image(const gl_model_desc* d, const ModelCfg& cfg, std::vector<uint8_t>& img,
                  int* psf_mfma_exp) {
  const int K = cfg.K, KK = K * K, HW = cfg.H * cfg.W;
  const size_t o_flip = align256(sizeof(float) * KK);
  const size_t o_tab = o_flip + align256(sizeof(float) * KK);
  const size_t tab_bytes = cfg.K <= kMfmaMaxK ? sizeof(uint16_t) * size_t(2) * K * 64 * 16 : 0;
  const size_t o_obs = o_tab + align256(tab_bytes);
  img.assign(o_obs + align256(sizeof(float) * HW), 0);
  float* psf = reinterpret_cast<float*>(img.data());
  float* flip = reinterpret_cast<float*>(img.data() + o_flip);
  std::memcpy(psf, d->psf, sizeof(float) * KK);
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) flip[a * K + b] = d->psf[(K - 1 - a) * K + (K - 1 - b)];
  *psf_mfma_exp = 0;
  if (tab_bytes) {
    // Toeplitz operands of the matrix-core PSF pass, per direction (0: flipped PSF, forward;
    // 1: PSF, adjoint), PSF row a and lane l = n + 16 g: elements e = 0..7 of column n,
    // rows 8g + e, of T_a[kk][n] = psf[a][kk - n] 2^t (zero outside 0 <= kk - n < K, n < N),
    // as two fp16 parts (v = h + l, l from the exact FP32 remainder); 2^t brings the largest
    // tap into [2^14, 2^15).
    const int N = mfma_geom(cfg.H, cfg.W, K).N;
    float pmax = 0.f;
    for (int i = 0; i < KK; ++i) pmax = std::max(pmax, std::fabs(d->psf[i]));
    int e = 0;
    if (pmax > 0.f) std::frexp(pmax, &e);
    const int sx = pmax > 0.f ? 15 - e : 0;
    *psf_mfma_exp = sx;
    uint16_t* tab = reinterpret_cast<uint16_t*>(img.data() + o_tab);
    for (int dir = 0; dir < 2; ++dir) {
      const float* kf = dir == 0 ? flip : d->psf;
      for (int a = 0; a < K; ++a)
        for (int l = 0; l < 64; ++l)
          for (int e8 = 0; e8 < 8; ++e8) {
            const int n = l % 16, b = 8 * (l / 16) + e8 - n;
            const float v = (n < N && b >= 0 && b < K) ? std::ldexp(kf[a * K + b], sx) : 0.f;
            const size_t o = ((size_t(dir) * K + a) * 64 + l) * 16;
            const _Float16 h = static_cast<_Float16>(v);
            tab[o + e8] = f16_bits(h);
            tab[o + 8 + e8] = f16_bits(static_cast<_Float16>(v - static_cast<float>(h)));
          }
    }
  }
  if (d->obs) std::memcpy(img.data() + o_obs, d->obs, sizeof(float) * HW);
}

// Points sd at a device copy of system_image (base, img_bytes long).
void system_bind(SystemData& sd, const ModelCfg& cfg, char* base, size_t img_bytes, int has_obs,
                 int psf_mfma_exp) {
  const int KK = cfg.K * cfg.K;
  const size_t o_flip = align256(sizeof(float) * KK);
  const size_t o_tab = o_flip + align256(sizeof(float) * KK);
  const size_t tab_bytes = cfg.K <= kMfmaMaxK ? sizeof(uint16_t) * size_t(2) * cfg.K * 64 * 16 : 0;
  sd.cfg = cfg;
  sd.base = base;
  sd.psf = reinterpret_cast<float*>(base);
  sd.psf_flip = reinterpret_cast<float*>(base + o_flip);
  sd.psf_mfma = tab_bytes ? reinterpret_cast<uint4*>(base + o_tab) : nullptr;
  sd.obs = reinterpret_cast<float*>(base + o_tab + align256(tab_bytes));
  sd.psf_mfma_exp = psf_mfma_exp;
  sd.has_obs = has_obs;
  sd.bytes = img_bytes;
}

int system_upload(const gl_model_desc* d, const ModelCfg& cfg, SystemData& sd) {
  std::vector<uint8_t> img;
  int sx = 0;
  system_image(d, cfg, img, &sx);
  char* base = nullptr;
  GL_HIP(hipMalloc(&base, img.size()));
  system_bind(sd, cfg, base, img.size(), d->obs != nullptr, sx);
  sd.owned = true;
  GL_HIP(hipMemcpy(base, img.data(), img.size(), hipMemcpyHostToDevice));
  return GL_OK;
}

void system_free(SystemData& sd) {
  if (sd.owned && sd.base) (void)hipFree(sd.base);
  sd = SystemData();
}

int choose_tiles(int P, int HW) {
  // aim at >= 2048 workgroups per launch (8 per CU); never fewer than 256 pixels a tile
  const int want = (2048 + P - 1) / std::max(P, 1);
  const int maxt = std::max(1, (HW + kSubThreads - 1) / kSubThreads);
  return std::max(1, std::min(want, maxt));
}

// The forward pass (6 workgroups per CU) gains from finer tiles where the adjoint (3 per CU,
// with a partial sum per tile) does not: aim at >= 12288 workgroups (8 rounds of the chip).
static int choose_fwd_tiles(int P, int HW) {
  const int want = (12288 + P - 1) / std::max(P, 1);
  const int maxt = std::max(1, (HW + kSubThreads - 1) / kSubThreads);
  return std::max(1, std::min(want, maxt));
}

int beta_per_particle(const ModelCfg& c) { return c.k * c.k * c.H * c.W; }

// Accumulator rows (particle x tile) that calls of up to P vectors need: the tile count
// grows as P shrinks (choose_tiles), so the largest P tiles is taken over every batch size
// up to P (above 2048 particles there is one tile each).
size_t acc_rows_upto(int P, int HW) {
  size_t rows = 0;
  for (int p = std::max(1, std::min(P, 2049)); p >= 1; --p)
    rows = std::max(rows, size_t(p) * choose_tiles(p, HW));
  return std::max(rows, size_t(std::max(P, 0)) * choose_tiles(std::max(P, 1), HW));
}

size_t workspace_bytes(int P, size_t rows, int HW, int d, bool fit, int beta_pp) {
  size_t b = align256(sizeof(PConst) * P) + 3 * align256(sizeof(float) * (size_t)P * HW) +
             align256(sizeof(double) * rows * kNAcc) +
             align256(sizeof(double) * (size_t)P * kConvMaxBands * 2) +
             align256(sizeof(float2) * (size_t)P * beta_pp);
  if (fit) b += align256(sizeof(double) * P) + 2 * align256(sizeof(float) * (size_t)P * d);
  return b;
}

void workspace_layout(Workspace& ws, char* base, int cP, size_t rows, int HW, int d, bool fit,
                      int beta_pp) {
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align256(b);
    return p;
  };
  ws.pc = reinterpret_cast<PConst*>(take(sizeof(PConst) * cP));
  ws.m0 = reinterpret_cast<float*>(take(sizeof(float) * (size_t)cP * HW));
  ws.sbar = reinterpret_cast<float*>(take(sizeof(float) * (size_t)cP * HW));
  ws.acc = reinterpret_cast<double*>(take(sizeof(double) * rows * kNAcc));
  ws.seed = reinterpret_cast<float*>(take(sizeof(float) * (size_t)cP * HW));
  ws.lpart = reinterpret_cast<double*>(take(sizeof(double) * (size_t)cP * kConvMaxBands * 2));
  ws.beta = beta_pp ? reinterpret_cast<float2*>(take(sizeof(float2) * (size_t)cP * beta_pp))
                    : nullptr;
  ws.beta_pp = beta_pp;
  ws.logl = nullptr;
  ws.grad = ws.theta = nullptr;
  if (fit) {
    ws.logl = reinterpret_cast<double*>(take(sizeof(double) * cP));
    ws.grad = reinterpret_cast<float*>(take(sizeof(float) * (size_t)cP * d));
    ws.theta = reinterpret_cast<float*>(take(sizeof(float) * (size_t)cP * d));
  }
  ws.cap_P = cP;
  ws.cap_rows = rows;
  ws.HW = HW;
  ws.bytes = off;
}

void workspace_free(Workspace& ws) {
  if (ws.pc) (void)hipFree(ws.pc);
  ws = Workspace();
}

int workspace_reserve(Workspace& ws, int P, int tiles, int HW, int d, bool fit, int beta_pp) {
  // a regrow keeps the fit buffers an earlier fit, VI or HMC call asked for: their users
  // rebuild their launch descriptors from ws after reserving, but a later plain likelihood
  // call on a larger batch must not drop them
  fit = fit || ws.logl != nullptr;
  const size_t rows = size_t(P) * tiles;
  if (ws.pc && P <= ws.cap_P && rows <= ws.cap_rows && HW == ws.HW && beta_pp == ws.beta_pp &&
      (!fit || ws.logl))
    return GL_OK;
  // grow to at least every batch size up to P, so that a smaller batch (more tiles per
  // particle) does not regrow it again
  const int cP = std::max(P, ws.cap_P);
  const size_t cR = std::max({rows, ws.cap_rows, acc_rows_upto(cP, HW)});
  if (ws.pc) {
    GL_HIP(hipDeviceSynchronize());
    workspace_free(ws);
  }
  const size_t bytes = workspace_bytes(cP, cR, HW, d, fit, beta_pp);
  char* base = nullptr;
  GL_HIP(hipMalloc(&base, bytes));
  workspace_layout(ws, base, cP, cR, HW, d, fit, beta_pp);
  return GL_OK;
}

SysDesc make_sys(const SystemData& sd, const Workspace& ws, int P, int tiles) {
  const ModelCfg& c = sd.cfg;
  SysDesc s;
  std::memset(&s, 0, sizeof(s));
  s.H = c.H;
  s.W = c.W;
  s.k = c.k;
  s.K = c.K;
  const double pix = c.pix;
  s.dxs = pix / c.k;
  s.x0 = -0.5 * (c.W - 1) * pix + (0.5 / c.k - 0.5) * pix;
  s.y0 = -0.5 * (c.H - 1) * pix + (0.5 / c.k - 0.5) * pix;
  s.inv_k2 = 1.0f / float(c.k * c.k);
  s.s2b = c.sigma_bkg * c.sigma_bkg;
  s.inv_gt = 1.0f / (c.gain * c.t_exp);
  s.mass = c.mass;
  s.shear = c.shear;
  s.lens_light = c.lens_light;
  s.nmax = c.nmax;
  s.d = c.d;
  s.P = P;
  s.tiles = tiles;
  const int HW = c.H * c.W;
  s.pix_per_tile = (HW + tiles - 1) / tiles;
  s.ftiles = choose_fwd_tiles(P, HW);
  s.fpix_per_tile = (HW + s.ftiles - 1) / s.ftiles;
  s.obs = sd.obs;
  s.psf = sd.psf;
  s.psf_flip = sd.psf_flip;
  s.psf_mfma = sd.psf_mfma;
  s.psf_mfma_exp = sd.psf_mfma_exp;
  s.pc = ws.pc;
  s.m0 = ws.m0;
  s.sbar = ws.sbar;
  s.acc = ws.acc;
  s.seed = ws.seed;
  s.beta = ws.beta;
  s.lpart = ws.lpart;
  conv_bands(P, c.H, c.W, &s.bands, &s.band_rows, &s.band_split);
  // matrix-core PSF pass for whole-image launches when the image's tiles and LDS fit; the
  // choice depends on this system alone, so its results do not depend on its launch partners
  const MfmaGeom q = mfma_geom(c.H, c.W, c.K);
  s.conv_mfma = sd.psf_mfma && s.bands == 1 && q.T <= 4 * kMfmaWaveTiles &&
                size_t(mfma_lds_bytes(q, c.H, c.W)) <= kConvLdsMax;
  return s;
}

void conv_bands(int P, int H, int W, int* bands, int* band_rows, int* split) {
  // aim at >= 512 workgroups in the PSF pass; bands of whole strips, at most kConvMaxBands
  const int nstrip = (H + kConvRows - 1) / kConvRows;
  const int want = P >= 512 ? 1 : (512 + std::max(P, 1) - 1) / std::max(P, 1);
  const int b = std::max(1, std::min({want, nstrip, kConvMaxBands}));
  const int spb = (nstrip + b - 1) / b;  // strip rows per band
  *band_rows = spb * kConvRows;
  *bands = (H + *band_rows - 1) / *band_rows;
  // small batches: split each strip's PSF columns over 2 or 4 lanes until the pass has about
  // one work item per lane of the GPU (256 CUs x 256 lanes), so that the per-lane chains of
  // K^2 kConvRows FMAs shorten; a one-band system keeps 1 (its bits then equal the whole-image
  // kernel's)
  const size_t items = size_t(P) * nstrip * W;
  int g = 1;
  while (*bands > 1 && g < 4 && items * g < size_t(256) * 256) g *= 2;
  *split = g;
}

int subpix_key(const ModelCfg& c) { return (c.mass * 2 + c.lens_light) * 16 + (c.nmax + 1); }

// ------------------------------------------------------------------------------------------
// kernel dispatch
// ------------------------------------------------------------------------------------------
using GroupKernel = void (*)(Group);

template <int MASS, int LL, int NMAX>
struct SubKernels {
  static constexpr GroupKernel fwd = subpix_fwd_kernel<MASS, LL, NMAX>;
  static constexpr GroupKernel adj = subpix_adj_kernel<MASS, LL, NMAX>;
};

template <int MASS, int LL, int... N>
static void fill_sub(GroupKernel* f, GroupKernel* a, std::integer_sequence<int, N...>) {
  ((f[(MASS * 2 + LL) * 16 + N] = SubKernels<MASS, LL, N - 1>::fwd), ...);
  ((a[(MASS * 2 + LL) * 16 + N] = SubKernels<MASS, LL, N - 1>::adj), ...);
}

// indexed by subpix_key
struct SubTable {
  GroupKernel fwd[64] = {};
  GroupKernel adj[64] = {};
  SubTable() {
    fill_sub<0, 0>(fwd, adj, std::make_integer_sequence<int, kMaxNmax + 2>{});
    fill_sub<0, 1>(fwd, adj, std::make_integer_sequence<int, kMaxNmax + 2>{});
    fill_sub<1, 0>(fwd, adj, std::make_integer_sequence<int, kMaxNmax + 2>{});
    fill_sub<1, 1>(fwd, adj, std::make_integer_sequence<int, kMaxNmax + 2>{});
  }
};
static const SubTable& sub_table() {
  static SubTable t;
  return t;
}

template <int... I>
static void fill_conv(GroupKernel* f, std::integer_sequence<int, I...>) {
  ((f[I] = conv_kernel<2 * I + 1>), ...);
}
template <int... I>
static void fill_conv_band(GroupKernel* f, GroupKernel* fa, std::integer_sequence<int, I...>) {
  ((f[I] = conv_band_kernel<2 * I + 1>), ...);
  ((fa[I] = conv_band_adj_kernel<2 * I + 1>), ...);
}
struct ConvTable {
  GroupKernel k[(GL_MAX_PSF + 1) / 2] = {};
  GroupKernel band[(GL_MAX_PSF + 1) / 2] = {};
  GroupKernel band_adj[(GL_MAX_PSF + 1) / 2] = {};
  ConvTable() {
    fill_conv(k, std::make_integer_sequence<int, (GL_MAX_PSF + 1) / 2>{});
    fill_conv_band(band, band_adj, std::make_integer_sequence<int, (GL_MAX_PSF + 1) / 2>{});
  }
};
static const ConvTable& conv_table() {
  static ConvTable t;
  return t;
}

static int launch(GroupKernel k, int blocks, int threads, size_t lds, const Group& g,
                  hipStream_t st) {
  if (blocks <= 0) return GL_OK;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, st, g);
  GL_HIP(hipGetLastError());
  return GL_OK;
}

int launch_prologue(const Group& g, hipStream_t st) {
  return launch(prologue_kernel, g.block0[g.nsys], 64, 0, g, st);
}
int launch_subpix_fwd(int key, const Group& g, hipStream_t st) {
  return launch(sub_table().fwd[key], g.block0[g.nsys], kSubThreads, 0, g, st);
}
int launch_subpix_adj(int key, const Group& g, hipStream_t st) {
  return launch(sub_table().adj[key], g.block0[g.nsys], kSubThreads, 0, g, st);
}
int launch_finalize(const Group& g, hipStream_t st) {
  return launch(finalize_kernel, g.block0[g.nsys], 64, 0, g, st);
}

size_t conv_lds_bytes(int H, int W, int K, int mode) {
  const int nstrip = (H + kConvRows - 1) / kConvRows;
  const size_t np = size_t((nstrip * kConvRows + K - 1) | 1) * (W + K - 1);
  (void)mode;
  return sizeof(float) * np;
}

// Raise the dynamic LDS limit of the PSF kernels once; fails only if `lds` needs it.
static int conv_lds_limit(size_t lds) {
  static std::once_flag once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(once, [] {
    const ConvTable& t = conv_table();
    for (const GroupKernel* tab : {t.k, t.band, t.band_adj})
      for (int i = 0; i < (GL_MAX_PSF + 1) / 2; ++i) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tab[i]),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(kConvLdsMax));
        if (e != hipSuccess) attr_err = e;
      }
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(conv_mfma_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(kConvLdsMax));
    if (e != hipSuccess) attr_err = e;
  });
  if (attr_err != hipSuccess && lds > 64 * 1024)
    return set_error(GL_E_DEVICE, "cannot raise the LDS limit: %s", hipGetErrorString(attr_err));
  return GL_OK;
}

static int launch_conv_mfma(const Group& g, size_t lds, hipStream_t st) {
  int rc = conv_lds_limit(lds);
  if (rc) return rc;
  return launch(conv_mfma_kernel, g.block0[g.nsys], kConvThreads, lds, g, st);
}

int launch_conv(int K, const Group& g, size_t lds, hipStream_t st) {
  for (int i = 0; i < g.nsys; ++i) {
    if (g.sys[i].conv_mfma) continue;
    const int nstrip = (g.sys[i].H + kConvRows - 1) / kConvRows;
    if (nstrip * g.sys[i].W > kConvMaxStrips * kConvThreads)
      return set_error(GL_E_UNIMPLEMENTED, "image too large for the PSF kernel");
  }
  int rc = conv_lds_limit(lds);
  if (rc) return rc;
  return launch(conv_table().k[(K - 1) / 2], g.block0[g.nsys], kConvThreads, lds, g, st);
}



// Block offsets of each system for one stage.
template <class F>
static void set_blocks(Group& g, F per_sys) {
  int b = 0;
  for (int i = 0; i < g.nsys; ++i) {
    g.block0[i] = b;
    b += per_sys(g.sys[i]);
  }
  g.block0[g.nsys] = b;
}

// The banded PSF pass (small batches): block offsets are set here for each kernel.
static int launch_conv_band(int K, Group& g, int mode, hipStream_t st) {
  size_t lds = 0;
  for (int i = 0; i < g.nsys; ++i) {
    const SysDesc& s = g.sys[i];
    if (s.conv_mfma) continue;
    const int nsr = s.band_rows / kConvRows;
    lds = std::max(lds, sizeof(float) * size_t((nsr * kConvRows + K - 1) | 1) * (s.W + K - 1));
  }
  int rc = conv_lds_limit(lds);
  if (rc) return rc;
  set_blocks(g, [](const SysDesc& s) { return s.conv_mfma ? 0 : blocks_conv_band(s); });
  if ((rc = launch(conv_table().band[(K - 1) / 2], g.block0[g.nsys], kConvThreads, lds, g, st)))
    return rc;
  if (mode == 2)
    return launch(conv_table().band_adj[(K - 1) / 2], g.block0[g.nsys], kConvThreads, lds, g, st);
  if (mode == 1) {
    set_blocks(g, [](const SysDesc& s) { return s.conv_mfma ? 0 : (s.P + 63) / 64; });
    return launch(conv_band_sum_kernel, g.block0[g.nsys], 64, 0, g, st);
  }
  return GL_OK;
}

int run_group(Group& g, int key, int K, int mode, hipStream_t st, hipEvent_t* ev,
              bool prologue, bool finalize) {
  int rc;
  auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
  GL_HIP(mark(0));
  if (prologue) {
    set_blocks(g, blocks_prologue);
    if ((rc = launch_prologue(g, st))) return rc;
  }
  GL_HIP(mark(1));
  for (int i = 0; i < g.nsys; ++i) g.sys[i].mode = mode;  // the forward pass keeps beta in mode 2
  set_blocks(g, blocks_subpix_fwd);
  if ((rc = launch_subpix_fwd(key, g, st))) return rc;
  GL_HIP(mark(2));
  // PSF pass: systems flagged for matrix cores in one launch, the others in the banded or the
  // whole-image VALU kernels (a system with one band gets the same bits from either)
  size_t lds = 0, lds_mfma = 0;
  bool banded = false, any_mfma = false, any_valu = false;
  for (int i = 0; i < g.nsys; ++i) {
    SysDesc& s = g.sys[i];
    s.mode = mode;
    if (s.conv_mfma) {
      any_mfma = true;
      lds_mfma = std::max(lds_mfma, size_t(mfma_lds_bytes(mfma_geom(s.H, s.W, s.K), s.H, s.W)));
    } else {
      any_valu = true;
      lds = std::max(lds, conv_lds_bytes(s.H, s.W, K, mode));
      banded = banded || s.bands > 1;
    }
  }
  if (any_mfma) {
    set_blocks(g, [](const SysDesc& s) { return s.conv_mfma ? blocks_conv(s) : 0; });
    if ((rc = launch_conv_mfma(g, lds_mfma, st))) return rc;
  }
  if (any_valu && banded) {
    if ((rc = launch_conv_band(K, g, mode, st))) return rc;
  } else if (any_valu) {
    set_blocks(g, [](const SysDesc& s) { return s.conv_mfma ? 0 : blocks_conv(s); });
    if ((rc = launch_conv(K, g, lds, st))) return rc;
  }
  GL_HIP(mark(3));
  if (mode != 2) return GL_OK;
  set_blocks(g, blocks_subpix);
  if ((rc = launch_subpix_adj(key, g, st))) return rc;
  GL_HIP(mark(4));
  if (!finalize) return GL_OK;
  set_blocks(g, blocks_prologue);
  if ((rc = launch_finalize(g, st))) return rc;
  GL_HIP(mark(5));
  return GL_OK;
}

}  // namespace glens

using namespace glens;

// ==========================================================================================
// C ABI
// ==========================================================================================
extern "C" {

const char* gl_last_error(void) { return t_err.c_str(); }

int gl_model_create(const gl_model_desc* desc, gl_model** out) {
  clear_error();
  if (!out) return set_error(GL_E_INVALID, "out is NULL");
  *out = nullptr;
  ModelCfg cfg;
  int rc = validate_desc(desc, &cfg);
  if (rc) return rc;
  gl_model* m = new (std::nothrow) gl_model();
  if (!m) return set_error(GL_E_NOMEM, "host allocation failed");
  GL_HIP(hipGetDevice(&m->device));
  rc = system_upload(desc, cfg, m->sys);
  if (rc) {
    system_free(m->sys);
    delete m;
    return rc;
  }
  *out = m;
  return GL_OK;
}

int gl_model_destroy(gl_model* m) {
  clear_error();
  if (!m) return GL_OK;
  (void)hipDeviceSynchronize();
  workspace_free(m->ws);
  system_free(m->sys);
  delete m;
  return GL_OK;
}

int gl_model_nparams(const gl_model* m, int* d) {
  clear_error();
  if (!m || !d) return set_error(GL_E_INVALID, "NULL argument");
  *d = m->sys.cfg.d;
  return GL_OK;
}

int gl_model_reserve(gl_model* m, int P, int with_fit) {
  clear_error();
  if (!m) return set_error(GL_E_INVALID, "model is NULL");
  if (P < 0) return set_error(GL_E_INVALID, "P must be >= 0");
  if (P == 0) return GL_OK;
  const ModelCfg& c = m->sys.cfg;
  const int HW = c.H * c.W;
  // every batch size up to P: workspace_reserve grows to acc_rows_upto(P) rows
  return workspace_reserve(m->ws, P, choose_tiles(P, HW), HW, c.d, with_fit != 0,
                           beta_per_particle(c));
}

int gl_model_plan(const gl_model* m, int P, gl_plan* out) {
  clear_error();
  if (!m || !out) return set_error(GL_E_INVALID, "NULL argument");
  if (P < 1) return set_error(GL_E_INVALID, "P must be >= 1");
  const ModelCfg& c = m->sys.cfg;
  const int HW = c.H * c.W;
  const int tiles = choose_tiles(P, HW);
  const SysDesc s = make_sys(m->sys, m->ws, P, tiles);
  out->psf_path = s.conv_mfma ? GL_PSF_MFMA : (s.bands > 1 ? GL_PSF_BANDED : GL_PSF_VALU);
  out->tiles = s.tiles;
  out->fwd_tiles = s.ftiles;
  out->bands = s.bands;
  out->workspace_bytes = workspace_bytes(P, acc_rows_upto(P, HW), HW, c.d, false,
                                         beta_per_particle(c));
  out->workspace_reserved = m->ws.bytes;
  out->noalloc_max_P = noalloc_max_particles(c);
  out->band_split = s.band_split;
  return GL_OK;
}

static int run_model(gl_model* m, const float* theta, int P, int mode, float* img, double* logl,
                     float* grad, hipStream_t st, hipEvent_t* ev = nullptr) {
  const ModelCfg& c = m->sys.cfg;
  const int HW = c.H * c.W;
  const int tiles = choose_tiles(P, HW);
  int rc = workspace_reserve(m->ws, P, tiles, HW, c.d, false, beta_per_particle(c));
  if (rc) return rc;
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = make_sys(m->sys, m->ws, P, tiles);
  g.sys[0].theta = theta;
  g.sys[0].img = img;
  g.sys[0].logl = logl;
  g.sys[0].grad = grad;
  return run_group(g, subpix_key(c), c.K, mode, st, ev);
}

static int common_checks(gl_model* m, const float* theta, int P) {
  if (!m) return set_error(GL_E_INVALID, "model is NULL");
  if (P < 0) return set_error(GL_E_INVALID, "P must be >= 0");
  if (P == 0) return GL_OK;
  return check_device_ptr(theta, "theta");
}

int gl_simulate(gl_model* m, const float* theta, int P, float* img, void* stream) {
  clear_error();
  int rc = common_checks(m, theta, P);
  if (rc || P == 0) return rc;
  if ((rc = check_device_ptr(img, "img"))) return rc;
  return run_model(m, theta, P, 0, img, nullptr, nullptr, (hipStream_t)stream);
}

int gl_loglik(gl_model* m, const float* theta, int P, double* logl, void* stream) {
  clear_error();
  int rc = common_checks(m, theta, P);
  if (rc || P == 0) return rc;
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  if ((rc = check_device_ptr(logl, "logl"))) return rc;
  return run_model(m, theta, P, 1, nullptr, logl, nullptr, (hipStream_t)stream);
}

int gl_loglik_grad(gl_model* m, const float* theta, int P, double* logl, float* grad,
                   void* stream) {
  clear_error();
  int rc = common_checks(m, theta, P);
  if (rc || P == 0) return rc;
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  if ((rc = check_device_ptr(logl, "logl"))) return rc;
  if ((rc = check_device_ptr(grad, "grad"))) return rc;
  return run_model(m, theta, P, 2, nullptr, logl, grad, (hipStream_t)stream);
}

int gl_model_stage_times_n(gl_model* m, const float* theta, int P, int with_grad, int n_calls,
                           double* logl, float* grad, float* ms, void* stream) {
  clear_error();
  int rc = common_checks(m, theta, P);
  if (rc) return rc;
  if (!ms) return set_error(GL_E_INVALID, "ms is NULL");
  for (int i = 0; i < GL_NSTAGES; ++i) ms[i] = 0.f;
  if (n_calls < 1 || n_calls > kStageTimesMaxCalls)
    return set_error(GL_E_INVALID, "n_calls must be in [1, %d]", kStageTimesMaxCalls);
  if (P == 0) return GL_OK;
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  if ((rc = check_device_ptr(logl, "logl"))) return rc;
  if (with_grad && (rc = check_device_ptr(grad, "grad"))) return rc;
  // one set of events per call, so that the calls run back to back with one wait at the end
  constexpr int NE = GL_NSTAGES + 1;
  std::vector<hipEvent_t> ev(size_t(n_calls) * NE, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      rc = set_error(GL_E_DEVICE, "hipEventCreate failed");
      break;
    }
  hipStream_t st = (hipStream_t)stream;
  for (int c = 0; rc == GL_OK && c < n_calls; ++c)
    rc = run_model(m, theta, P, with_grad ? 2 : 1, nullptr, logl, grad, st, &ev[size_t(c) * NE]);
  const int last = with_grad ? GL_NSTAGES : 3;
  if (rc == GL_OK && hipEventSynchronize(ev[size_t(n_calls - 1) * NE + last]) != hipSuccess)
    rc = set_error(GL_E_DEVICE, "event sync failed");
  if (rc == GL_OK) {
    double sum[GL_NSTAGES] = {};
    for (int c = 0; rc == GL_OK && c < n_calls; ++c)
      for (int i = 0; i < last; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[size_t(c) * NE + i], ev[size_t(c) * NE + i + 1]) !=
            hipSuccess) {
          rc = set_error(GL_E_DEVICE, "event timing failed");
          break;
        }
        sum[i] += t;
      }
    for (int i = 0; rc == GL_OK && i < last; ++i) ms[i] = float(sum[i] / n_calls);
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

int gl_model_stage_times(gl_model* m, const float* theta, int P, int with_grad, double* logl,
                         float* grad, float* ms, void* stream) {
  return gl_model_stage_times_n(m, theta, P, with_grad, 1, logl, grad, ms, stream);
}

}  // extern "C"
