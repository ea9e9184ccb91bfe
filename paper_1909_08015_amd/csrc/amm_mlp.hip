// amm_mlp.hip -- learned sector sampler entry points.
#include <hip/hip_runtime.h>

#include "../../include/amm.h"
#include "amm_mlp.h"

namespace amm {
void mlp_free(MlpState &m) {
    if (m.d_params) hipFree(m.d_params);
    m.d_params = nullptr;
}
}  // namespace amm

extern "C" {
int amm_pilot(amm_ctx *, uint64_t, uint64_t, int, int, void *) { return AMM_E_ARG; }
int amm_mlp_train(amm_ctx *, int, float, uint64_t, void *) { return AMM_E_ARG; }
int amm_mlp_params(const amm_ctx *, float *, size_t, size_t *) { return AMM_E_ARG; }
int amm_mlp_set_params(amm_ctx *, const float *, size_t) { return AMM_E_ARG; }
int amm_mlp_features(const amm_ctx *, int, float *, int32_t *, int32_t *, size_t, size_t *) { return AMM_E_ARG; }
int amm_mlp_loss_grad(amm_ctx *, const float *, const float *, const int32_t *, const float *, int, int, float *,
                      float *, void *) {
    return AMM_E_ARG;
}
}
