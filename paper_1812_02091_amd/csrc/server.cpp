// Serving entry points (continuous batching); see include/lcemd.h.
#include "internal.h"

extern "C" {

int lcemd_server_start(lcemd_ctx*, const lcemd_server_cfg*, lcemd_server** out) {
  if (out) *out = nullptr;
  return LCEMD_E_UNSUPPORTED;
}
int lcemd_server_submit(lcemd_server*, const int32_t*, const float*, int32_t, uint64_t*) {
  return LCEMD_E_UNSUPPORTED;
}
int lcemd_server_wait(lcemd_server*, uint64_t, int64_t*, float*, double*) {
  return LCEMD_E_UNSUPPORTED;
}
void lcemd_server_stop(lcemd_server*) {}

}  // extern "C"
