// Switch-network kernels (placeholder until the kernels land).
#include <hip/hip_runtime.h>

#include "blest.h"

extern "C" {
blest_status blest_mlp_forward(const float*, const float*, int32_t, float*, void*) { return BLEST_ERR_UNSUPPORTED; }
blest_status blest_mlp_loss_grad(const float*, const float*, const int32_t*, const float*, int32_t, float*, float*,
                                 void*) {
  return BLEST_ERR_UNSUPPORTED;
}
blest_status blest_mlp_adam(float*, const float*, float*, float*, int32_t, int32_t, float, float, float, float, void*) {
  return BLEST_ERR_UNSUPPORTED;
}
blest_status blest_mlp_train(float*, float*, float*, const float*, const int32_t*, const float*, int32_t, int32_t,
                             int32_t, float, uint64_t, float*, void*) {
  return BLEST_ERR_UNSUPPORTED;
}
}
