// Entry points whose implementation lands in later steps.
#include "cm_context.h"

extern "C" {
cm_status cm_server_create(cm_context* ctx, uint64_t, int32_t, cm_server**) {
  return cm_fail(ctx, CM_ERR_INVALID_ARG, "server not available in this build");
}
cm_status cm_server_submit(cm_server*, const cm_request*, uint64_t*) { return CM_ERR_INVALID_ARG; }
cm_status cm_server_poll(cm_server*, uint64_t, cm_result*) { return CM_ERR_INVALID_ARG; }
cm_status cm_server_release(cm_server*, uint64_t) { return CM_ERR_INVALID_ARG; }
cm_status cm_server_stats(cm_server*, uint64_t*, int32_t*, int32_t*) { return CM_ERR_INVALID_ARG; }
cm_status cm_server_destroy(cm_server*) { return CM_ERR_INVALID_ARG; }
}
