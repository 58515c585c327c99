// Lyot coronagraph train over wavelengths (placeholder until the train orchestration lands).
#include "../../include/fresnel.h"

extern "C" {
size_t propagate_train_workspace_bytes(const fr_train_desc *, int32_t, const int32_t *, int32_t) {
  return 0;
}
int propagate_train(fr_ctx *, const fr_train_desc *, int32_t, const double *, const int32_t *,
                    const float *, int32_t, float *, const float *, float *, void *, size_t,
                    void *) {
  return FR_EUNSUPPORTED;
}
}
