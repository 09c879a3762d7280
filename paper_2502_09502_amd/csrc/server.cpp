// Request server (continuous batching over resident problems).
#include <hip/hip_runtime.h>

#include "common.h"
#include "engine.h"

extern "C" {

int cgl_server_create(cgl_ctx*, size_t, int32_t, cgl_server** out) {
  if (out) *out = nullptr;
  cgl::set_error("server not available in this build");
  return CGL_E_INTERNAL;
}
int cgl_server_submit(cgl_server*, cgl_problem*, const cgl_node*, uint64_t*) {
  return CGL_E_INTERNAL;
}
int cgl_server_poll(cgl_server*, int32_t, uint64_t*, cgl_result*, double*, int64_t, double*,
                    int32_t* got) {
  if (got) *got = 0;
  return CGL_E_INTERNAL;
}
int cgl_server_cancel(cgl_server*, uint64_t) { return CGL_E_INTERNAL; }
int cgl_server_stats(cgl_server*, int32_t*, int32_t*, int32_t*) { return CGL_E_INTERNAL; }
int cgl_server_destroy(cgl_server*) { return CGL_OK; }

}  // extern "C"
