// Fixed-budget multi-start fit and the continuous-batching server (not yet built).
#include <hip/hip_runtime.h>

#include "glens_host.h"

using namespace glens;

extern "C" {
int gl_fit(gl_model*, const gl_fit_opts*, gl_fit_result*, void*) {
  return set_error(GL_E_UNIMPLEMENTED, "gl_fit");
}
int gl_fit_state_create(gl_model*, const gl_fit_opts*, gl_fit_state** out, void*) {
  if (out) *out = nullptr;
  return set_error(GL_E_UNIMPLEMENTED, "gl_fit_state_create");
}
int gl_fit_state_destroy(gl_fit_state*) { return GL_OK; }
int gl_fit_state_step(gl_fit_state*, int, void*) { return set_error(GL_E_UNIMPLEMENTED, "step"); }
int gl_fit_state_arrays(gl_fit_state*, float**, float**, float**, int*) {
  return set_error(GL_E_UNIMPLEMENTED, "arrays");
}
int gl_fit_state_result(gl_fit_state*, gl_fit_result*, void*) {
  return set_error(GL_E_UNIMPLEMENTED, "result");
}
int gl_server_create(const gl_server_opts*, gl_server** out) {
  if (out) *out = nullptr;
  return set_error(GL_E_UNIMPLEMENTED, "gl_server_create");
}
int gl_server_destroy(gl_server*) { return GL_OK; }
int gl_submit(gl_server*, const gl_model_desc*, const gl_fit_opts*, uint64_t*) {
  return set_error(GL_E_UNIMPLEMENTED, "gl_submit");
}
int gl_poll(gl_server*, uint64_t, gl_fit_result*) { return set_error(GL_E_UNIMPLEMENTED, "gl_poll"); }
int gl_server_get_stats(gl_server*, gl_server_stats*) {
  return set_error(GL_E_UNIMPLEMENTED, "stats");
}
}
