// Host-side pieces of the multi-start fit shared by gl_fit* and the server.
#pragma once

#include <vector>

#include "glens_host.h"

namespace glens {

struct FitParams {
  int P = 0, K = 1, step = 0;
  float lr0 = 1e-2f, lr1 = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  uint64_t seed = 0;
};

// Device arrays of one fit: z, m, v [P][d], priors [d], log posterior and chi^2 [P].
struct FitBuffers {
  int P = 0, d = 0;
  char* base = nullptr;
  float* z = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  Prior* prior = nullptr;
  double* logpost = nullptr;
  double* chi2 = nullptr;
  size_t bytes = 0;
  bool owned = false;  // base from fit_buffers_alloc (freed by fit_buffers_free)
};

FitParams fit_params(const gl_fit_opts* o);
int validate_fit_opts(const gl_fit_opts* o, int d, std::vector<Prior>& pri);
size_t fit_buffers_bytes(int P, int d);
int fit_buffers_alloc(FitBuffers& fb, int P, int d, const Prior* host_priors);
// Carve the buffers out of `base` (fit_buffers_bytes long); the priors are not uploaded.
void fit_buffers_layout(FitBuffers& fb, char* base, int P, int d);
void fit_buffers_free(FitBuffers& fb);
void attach_fit(SysDesc& s, const FitBuffers& fb, const FitParams& fp, const Workspace& ws);
int launch_fit_init(Group& g, hipStream_t st);
int launch_adam(Group& g, hipStream_t st);
int launch_logpost(Group& g, hipStream_t st);
// The best particle of each system into its s.fit_out (after launch_logpost).
int launch_fit_best(Group& g, hipStream_t st);
// gl_fit_result from a FitOut copied to the host (timestamps left to the caller).
void fit_result_from_out(const FitOut& o, const ModelCfg& c, gl_fit_result* out);
// Copies log p~, chi^2 and the best particle to the host (synchronises `st`).
int fit_result_from_device(const FitBuffers& fb, const Workspace& ws, int P, const ModelCfg& c,
                           hipStream_t st, gl_fit_result* out);

}  // namespace glens
