// Batched engine (declarations in include/lbm.h).  Placeholder until the
// persistent batched kernels land: every entry point reports LBM_E_UNSUPPORTED.
#include "../../include/lbm.h"

extern "C" {
int lbm_batch_workspace_bytes(const lbm_params*, int32_t, size_t*) { return LBM_E_UNSUPPORTED; }
int lbm_batch_create(lbm_batch**, const lbm_params*, const int32_t*, int32_t, void*, size_t, const float* const*,
                     void*) {
  return LBM_E_UNSUPPORTED;
}
int lbm_batch_step(lbm_batch*, int32_t, void*) { return LBM_E_UNSUPPORTED; }
int lbm_batch_moments(lbm_batch*, int32_t, float*, float*, float*, float*, float*, void*) { return LBM_E_UNSUPPORTED; }
int lbm_batch_status(lbm_batch*, int32_t*, void*) { return LBM_E_UNSUPPORTED; }
int lbm_batch_destroy(lbm_batch*) { return LBM_OK; }
}
