// amm_mlp.h -- learned sector sampler state (internal).
//
// A 16 -> 64 -> 64 -> 1 tanh MLP (FP32) maps features of (graph, s, j) to a
// logit correction of the plain sector probabilities; the trained network is
// tabulated into P_theta(j | s) per graph.  Parameter layout (flat):
// W1[64x16], b1[64], W2[64x64], b2[64], w3[64], b3[1].
#pragma once
#include <stdint.h>

#include <vector>

namespace amm {

constexpr int MLP_NF = 16;
constexpr int MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_NF + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;

struct MlpRows {                 // rows of one graph (host copy + device copy)
    std::vector<float> feat;     // [R x 16]
    std::vector<int32_t> s, j;   // set and line of each row
    std::vector<int32_t> goff;   // group offsets (G+1)
    float *d_feat = nullptr;
    int32_t *d_s = nullptr, *d_j = nullptr, *d_grp = nullptr, *d_goff = nullptr;
    bool built = false;
};

struct MlpState {
    float *d_params = nullptr;   // [NPARAM]
    float *d_m = nullptr, *d_v = nullptr;
    int step = 0;
    bool trained = false;
    std::vector<MlpRows> rows;   // per graph
};

void mlp_free(MlpState &m);
void mlp_free_rows(MlpState &m);   // drop the per-graph feature rows (graph set changed)

}  // namespace amm
