// gl_loglik_grad_noalloc: the gl_loglik_grad pipeline with its work space in a fixed device
// array instead of the model's (growable) allocation, for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc. The call allocates nothing: no hipMalloc / hipFree, no library allocator.
//
// The work space (per-particle constants, pre-PSF image, pixel adjoint, accumulators, kept
// source positions) is carved from `scratch`, kNoAllocBytes long, which every device the
// library runs on holds until the process ends. Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept; host code never passes
// the array's own name to a kernel (on the host it is only a stand-in for the symbol).
//
// Every call on one device shares that device's array, and its contents are those of the
// last call: calls that overlap on one device (two streams, two threads) race and must be
// ordered by the caller. Nothing in it needs to start at zero: each kernel writes what the
// next one reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "glens_host.h"

namespace glens {

static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on first use there).
static int scratch_ptr(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GL_E_UNIMPLEMENTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(GL_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GL_OK;
}

size_t noalloc_bytes(const ModelCfg& c, int P) {
  const int HW = c.H * c.W;
  return workspace_bytes(P, size_t(P) * choose_tiles(P, HW), HW, c.d, false,
                         beta_per_particle(c));
}

int noalloc_max_particles(const ModelCfg& c) {
  // the per-particle arrays alone bound P from above; scan down from there to the largest P
  // whose work space (with its accumulator rows, which shrink as P grows) fits
  const size_t per = workspace_bytes(1, 0, c.H * c.W, c.d, false, beta_per_particle(c));
  int P = int(std::min<size_t>(kNoAllocBytes / per, size_t(1) << 24));
  while (P > 0 && noalloc_bytes(c, P) > kNoAllocBytes) --P;
  return P;
}

}  // namespace glens

using namespace glens;

extern "C" {

int gl_loglik_grad_noalloc(gl_model* m, const float* theta, int P, double* logl, float* grad,
                           void* stream) {
  clear_error();
  if (!m) return set_error(GL_E_INVALID, "model is NULL");
  if (P < 0) return set_error(GL_E_INVALID, "P must be >= 0");
  if (P == 0) return GL_OK;
  if (!m->sys.has_obs) return set_error(GL_E_INVALID, "model has no observed image");
  int rc;
  if ((rc = check_device_ptr(theta, "theta")) || (rc = check_device_ptr(logl, "logl")) ||
      (rc = check_device_ptr(grad, "grad")))
    return rc;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(GL_E_DEVICE, "hipGetDevice failed");
  if (dev != m->device)
    return set_error(GL_E_INVALID, "current device %d is not the model's device %d", dev,
                     m->device);
  const ModelCfg& c = m->sys.cfg;
  const size_t need = noalloc_bytes(c, P);
  if (need > kNoAllocBytes)
    return set_error(GL_E_BUDGET,
                     "P = %d needs %zu bytes of work space, above the fixed %zu of the "
                     "allocation-free call",
                     P, need, kNoAllocBytes);
  char* base = nullptr;
  if ((rc = scratch_ptr(dev, &base))) return rc;
  const int HW = c.H * c.W, tiles = choose_tiles(P, HW);
  Workspace ws;
  workspace_layout(ws, base, P, size_t(P) * tiles, HW, c.d, false, beta_per_particle(c));
  Group g;
  std::memset(&g, 0, sizeof(g));
  g.nsys = 1;
  g.sys[0] = make_sys(m->sys, ws, P, tiles);
  g.sys[0].theta = theta;
  g.sys[0].logl = logl;
  g.sys[0].grad = grad;
  return run_group(g, subpix_key(c), c.K, 2, (hipStream_t)stream);
}

}  // extern "C"
