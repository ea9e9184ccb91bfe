// amm_host.h -- host plan builder interface (internal to the library).
#pragma once
#ifndef __HIPCC__
#define __host__
#define __device__
#endif
#include <array>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/amm.h"
#include "amm_plan.h"

#define AMM_LN2_HI 6.93147180369123816490e-01
#define AMM_LN2_LO 1.90821492927058770002e-10
#define AMM_INV_LN2 1.44269504088896338700e+00
#define AMM_SQRT_HALF 0.70710678118654752440

// Coefficients of the exp Taylor polynomial (c_0 = 1, c_i = c_{i-1}/i) and of
// the log atanh series (1/(2i+1)), each formed by IEEE double divisions.
__host__ __device__ inline double amm_exp_c(int i) {
    double c = 1.0;
    for (int k = 1; k <= i; ++k) c = c / (double)k;
    return c;
}
__host__ __device__ inline double amm_log_d(int i) { return 1.0 / (double)(2 * i + 1); }

namespace amm {

struct SEGraph {
    int n;
    std::vector<std::pair<int, int>> chords;
};

struct DensityTables {
    int M = 0;
    std::vector<double> deg1, deg3, W1, logdeg1, F1;
    double F1full = 0, logK[4] = {0, 0, 0, 0}, logc[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
};

struct PlanHost {
    int n = 0, M = 0, ninsert = 0;
    std::vector<LevelDesc> levels;
    std::vector<TermDesc> terms;
    std::vector<int32_t> ops;
    std::vector<Mono> monos;
    std::vector<std::pair<int, int>> ranges;            // per level (variant,out,c)
    std::vector<std::pair<int, int>> poly_ranges_store;  // cache of built polys
    int n_terms_expanded = 0;
    int64_t n_monos_per_sample = 0;
    double flops_per_sample = 0;
};

double host_log(double x);
std::vector<SEGraph> enumerate_se(int n);
std::array<int, 3> vertex_class(const SEGraph &g, int e);
void build_density(const SEGraph &g, const amm_density_params &p, DensityTables &d);
// nthreads: host threads that build the graph's distinct level polynomials
// (the result does not depend on it).
void build_plan(const SEGraph &g, PlanHost &P, int nthreads = 1);
double omega_set(const SEGraph &g, uint32_t mask);
void set_stats(const SEGraph &g, uint32_t mask, int *loops, int *comps, int *ng, int *ne);

}  // namespace amm
