// amm_mlp.h -- learned sector sampler state (internal).
#pragma once
#include <stdint.h>

namespace amm {

struct MlpState {
    float *d_params = nullptr;   // device parameters
    int nparams = 0;
    bool trained = false;
};

void mlp_free(MlpState &m);

}  // namespace amm
