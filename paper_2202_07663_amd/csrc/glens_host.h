// Host-side internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/gl.h"
#include "glens_types.h"

namespace glens {

int set_error(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Return GL_E_NOMEM / GL_E_DEVICE with a message when a HIP call fails. The runtime's
// last-error state is cleared on the way, so that a later launch check (hipGetLastError)
// does not report this failure again.
#define GL_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      (void)hipGetLastError();                                                           \
      return set_error(e_ == hipErrorOutOfMemory ? GL_E_NOMEM : GL_E_DEVICE, "%s: %s",   \
                       #call, hipGetErrorString(e_));                                    \
    }                                                                                    \
  } while (0)

// Validated copy of a model descriptor (host pointers dropped).
struct ModelCfg {
  int H, W, k, K;
  float pix;
  int mass, shear, lens_light, nmax, d;
  float sigma_bkg, t_exp, gain;
};

int validate_desc(const gl_model_desc* desc, ModelCfg* cfg);
int nparams(int mass, int shear, int lens_light, int nmax);

// Device work space of one system for P particles.
struct Workspace {
  int cap_P = 0, HW = 0;
  size_t cap_rows = 0;     // accumulator rows (particle x tile) of acc
  PConst* pc = nullptr;
  float* m0 = nullptr;
  float* sbar = nullptr;
  double* acc = nullptr;
  double* logl = nullptr;  // internal log L (fits)
  float* grad = nullptr;   // internal gradient (fits)
  float* theta = nullptr;  // internal theta (fits)
  float* seed = nullptr;   // adjoint seed of the banded PSF pass
  double* lpart = nullptr; // per-band likelihood partial sums
  float2* beta = nullptr;  // beta - x_s per sub-pixel, from the forward pass
  int beta_pp = 0;         // its float2 entries per particle
  size_t bytes = 0;
};
// beta_pp: float2 entries of the beta buffer per particle (beta_per_particle(cfg)); rows:
// accumulator rows, P x tiles for one batch size (acc_rows_upto for every size up to P).
size_t workspace_bytes(int P, size_t rows, int HW, int d, bool fit_buffers, int beta_pp);
size_t acc_rows_upto(int P, int HW);
// Carve the work space out of `base` (workspace_bytes long, 256-byte aligned).
void workspace_layout(Workspace& ws, char* base, int P, size_t rows, int HW, int d,
                      bool fit_buffers, int beta_pp);
// Grow ws (owned allocation) to hold a batch of P particles split into `tiles` tiles; a
// growth synchronises the device and reallocates, keeping the fit buffers once present.
int workspace_reserve(Workspace& ws, int P, int tiles, int HW, int d, bool fit_buffers,
                      int beta_pp);
void workspace_free(Workspace& ws);

// Number of sub-pixel work tiles per particle for P particles of an H x W image.
int choose_tiles(int P, int HW);

// Device copy of the fixed inputs of one system (one allocation, laid out by system_image).
struct SystemData {
  ModelCfg cfg;
  char* base = nullptr;       // the allocation (owned: freed by system_free)
  bool owned = false;
  float* psf = nullptr;
  float* psf_flip = nullptr;
  uint4* psf_mfma = nullptr;  // Toeplitz fragments of the PSF (K <= kMfmaMaxK), else null
  int psf_mfma_exp = 0;       // they hold psf 2^psf_mfma_exp
  float* obs = nullptr;
  int has_obs = 0;
  size_t bytes = 0;
};
int system_upload(const gl_model_desc* desc, const ModelCfg& cfg, SystemData& sd);
void system_free(SystemData& sd);
// The device image of a system's inputs (PSF, flipped PSF, matrix-core operands, observed
// image) in host memory, and the binding of SystemData to a device copy of it.
void system_image(const gl_model_desc* desc, const ModelCfg& cfg, std::vector<uint8_t>& img,
                  int* psf_mfma_exp);
void system_bind(SystemData& sd, const ModelCfg& cfg, char* base, size_t img_bytes, int has_obs,
                 int psf_mfma_exp);

// Fill the launch descriptor of one system.
SysDesc make_sys(const SystemData& sd, const Workspace& ws, int P, int tiles);

// Kernel configuration key of a system (systems with equal keys share launches).
// Sub-pixel source offsets kept from the forward pass for the adjoint (which takes the lens
// Jacobian in FP32 around them): k^2 H W per particle.
int beta_per_particle(const ModelCfg& c);

int subpix_key(const ModelCfg& c);  // (mass * 2 + lens_light) * 16 + (nmax + 1)

// Launch stages over a group of systems (all with the same key / PSF size).
int launch_prologue(const Group& g, hipStream_t st);
int launch_subpix_fwd(int key, const Group& g, hipStream_t st);
int launch_conv(int K, const Group& g, size_t lds_bytes, hipStream_t st);
int launch_subpix_adj(int key, const Group& g, hipStream_t st);
int launch_finalize(const Group& g, hipStream_t st);
size_t conv_lds_bytes(int H, int W, int K, int mode);
constexpr size_t kConvLdsMax = 160 * 1024 - 256;  // dynamic LDS allowed to the PSF kernels

// Block counts of one system per stage.
inline int blocks_prologue(const SysDesc& s) { return s.P; }  // prologue, finalize
inline int blocks_subpix(const SysDesc& s) { return s.P * s.tiles; }
inline int blocks_subpix_fwd(const SysDesc& s) { return s.P * s.ftiles; }
inline int blocks_conv(const SysDesc& s) { return s.P; }
inline int blocks_conv_band(const SysDesc& s) { return s.P * s.bands; }
// Row bands of the PSF pass for P particles of an H-row image (1: the whole-image kernel).
void conv_bands(int P, int H, int W, int* bands, int* band_rows, int* split);

// Run the forward (+adjoint) pipeline for a group of systems sharing key and PSF size.
// mode: 0 image, 1 log L, 2 log L + gradient.
// ev (optional): GL_NSTAGES + 1 events, recorded before the first and after every stage.
// prologue = false skips the decode (the particles' constants are already those of their
// current parameters); finalize = false stops after the sub-pixel adjoint (the caller runs
// finalize_particle itself, fused with its own per-particle step).
int run_group(Group& g, int key, int K, int mode, hipStream_t st, hipEvent_t* ev = nullptr,
              bool prologue = true, bool finalize = true);

int check_device_ptr(const void* p, const char* name);

// Most calls one gl_model_stage_times_n may time (events per call: GL_NSTAGES + 1).
constexpr int kStageTimesMaxCalls = 10000;

// Work space of gl_loglik_grad_noalloc: a fixed device array of kNoAllocBytes per device.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
size_t noalloc_bytes(const ModelCfg& c, int P);    // its work space at P particles
int noalloc_max_particles(const ModelCfg& c);      // the largest P that fits

}  // namespace glens

struct gl_model {
  int device = 0;
  glens::SystemData sys;
  glens::Workspace ws;
};
