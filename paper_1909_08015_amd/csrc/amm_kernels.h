// amm_kernels.h -- Monte Carlo kernels templated on the integrand evaluator
// (the table interpreter of amm_core.h, or a generated per-graph function).
//   k_eval       integrands at given points (FP64 + round-off bound, or DD)
//   k_integrate  sample + evaluate + round-off check (eq. interval_accept) +
//                per-chunk deterministic partial sums; flagged samples are
//                compacted per chunk in sample order
//   k_dd         double-double recompute of the flagged samples of a chunk
#pragma once
#include <type_traits>

#include "amm_ctx.h"

namespace amm {

// Evaluator using the plan tables (variables in LDS columns).
struct InterpEval {
    static constexpr bool kLds = true;
    PlanDev P;
    template <typename T, int N, typename Vars>
    __device__ __forceinline__ void eval(const double *z, T *I, T *absI, Vars &vars) const {
        eval_graph<T, N>(P, z, I, absI, vars);
    }
};

// Evaluator calling a generated straight-line function G::eval<T>.
template <class G>
struct GenEval {
    static constexpr bool kLds = false;
    template <typename T, int N, typename Vars>
    __device__ __forceinline__ void eval(const double *z, T *I, T *absI, Vars &) const {
        G::template eval<T>(z, I, absI);
    }
};

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

struct RunArgs {
    uint64_t seed, begin, end;      // sample index range [begin, end)
    uint32_t uid;
    int chunk0;                     // first chunk (relative to begin) of this launch
    int nchunks;
    double tau;                     // acceptance threshold (<0: flag all; inf: none)
    int ncls;
    int cls_of[MAXNE];
    int learned;
};

// T = ea: FP64 value with its round-off bound KAPPA u I.a; T = dd: double-double.
template <typename T, int N, class Ev>
__global__ void __launch_bounds__(BLOCK) k_eval(Ev EV, const double *z, uint64_t n, double *I, double *absI,
                                                double *bound) {
    constexpr int M = 3 * N - 1, NE = 2 * N - 1;
    uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double zz[M];
    for (int j = 0; j < M; ++j) zz[j] = z[i * M + j];
    T v[NE], a[NE];
    if constexpr (std::is_same<T, ea>::value && Ev::kLds) {
        __shared__ double vlds[Dims<N>::NV * BLOCK];
        __shared__ float rlds[Dims<N>::NV * BLOCK];
        VarsLdsEa vars{vlds + threadIdx.x, rlds + threadIdx.x, BLOCK};
        EV.template eval<T, N>(zz, v, a, vars);
    } else {
        VarsPriv<T, Ev::kLds ? Dims<N>::NV : 1> vars;
        EV.template eval<T, N>(zz, v, a, vars);
    }
    for (int e = 0; e < NE; ++e) {
        if (I) I[i * NE + e] = to_double(v[e]);
        if (absI) absI[i * NE + e] = to_double(a[e]);
        if (bound) bound[i * NE + e] = KAPPA * 0x1p-53 * mag(v[e]);
    }
}



// Statistic layout per graph:
//   [0, ne)        sum y_e       [ne, 2ne)  sum y_e^2     [2ne, 3ne) sum |y_e|
//   [3ne, 3ne+c)   sum y_class   [.., +c)   sum y_class^2
//   then n, n_flag, n_dd_fail, n_ood.
template <int N>
__device__ __forceinline__ void add_stats(double (&st)[3 * (2 * N - 1) + 2 * (2 * N - 1) + 4], const double *y,
                                          const RunArgs &A) {
    constexpr int NE = 2 * N - 1;
    double yc[NE];
    for (int c = 0; c < NE; ++c) yc[c] = 0.0;
    for (int e = 0; e < NE; ++e) {
        st[e] += y[e];
        st[NE + e] += y[e] * y[e];
        st[2 * NE + e] += fabs(y[e]);
        for (int c = 0; c < NE; ++c)
            if (A.cls_of[e] == c) yc[c] += y[e];
    }
    for (int c = 0; c < NE; ++c) {
        if (c >= A.ncls) break;
        st[3 * NE + c] += yc[c];
        st[3 * NE + A.ncls + c] += yc[c] * yc[c];
    }
}

template <int N, class Ev>
__device__ __forceinline__ void eval_sample(const Ev &EV, const DensityDev &D, const RunArgs &A, uint64_t idx,
                                            double *y, int &ood, int &flag, double *vlds, float *rlds) {
    constexpr int M = 3 * N - 1, NE = 2 * N - 1;
    double u[2 * M], z[M];
    int path[M];
    uniforms(A.seed, A.uid, idx, D.ptheta ? 2 * M : 2 * M - 1, u);
    SampleOut o = sample_point<M>(D, u, z, path);
    ood = o.ood;
    flag = 0;
    if (o.ood) {
        for (int e = 0; e < NE; ++e) y[e] = 0.0;
        return;
    }
    bool plain = false;
    if constexpr (Ev::kLds) plain = A.tau == INFINITY;    // interpreter: skip bounds if unchecked
    if (plain) {
        if constexpr (Ev::kLds) {
            double I[NE], aI[NE];
            VarsLdsD vars{vlds + threadIdx.x, BLOCK};
            EV.template eval<double, N>(z, I, aI, vars);
            for (int e = 0; e < NE; ++e) {
                y[e] = ldexp(I[e] / o.gx, -o.gj);
                if (!isfinite(y[e])) flag = 1;
            }
        }
    } else {
        ea I[NE], aI[NE];
        if constexpr (Ev::kLds) {
            VarsLdsEa vars{vlds + threadIdx.x, rlds + threadIdx.x, BLOCK};
            EV.template eval<ea, N>(z, I, aI, vars);
        } else {
            VarsPriv<ea, 1> vars;
            EV.template eval<ea, N>(z, I, aI, vars);
        }
        for (int e = 0; e < NE; ++e) {
            double ye = ldexp(I[e].v / o.gx, -o.gj);
            double r = KAPPA * 0x1p-53 * ldexp(I[e].a / o.gx, -o.gj);
            if (!(r <= A.tau) || !isfinite(ye)) flag = 1;
            y[e] = ye;
        }
    }
    if (flag)
        for (int e = 0; e < NE; ++e) y[e] = 0.0;
}

template <int N, class Ev>
__global__ void __launch_bounds__(BLOCK) k_integrate(Ev EV, DensityDev D, RunArgs A, double *part, uint32_t *flags,
                                                     int32_t *nflag) {
    constexpr int NE = 2 * N - 1;
    constexpr int NST = 3 * NE + 2 * NE + 4;
    __shared__ double sh[BLOCK];
    __shared__ int shc[BLOCK];
    __shared__ double vlds[(Ev::kLds ? Dims<N>::NV : 1) * BLOCK];
    __shared__ float rlds[(Ev::kLds ? Dims<N>::NV : 1) * BLOCK];
    const int nst = 3 * NE + 2 * A.ncls + 4;
    for (int ch = blockIdx.x; ch < A.nchunks; ch += gridDim.x) {
        double st[NST];
        for (int s = 0; s < NST; ++s) st[s] = 0.0;
        uint64_t base = A.begin + (uint64_t)(A.chunk0 + ch) * CHUNK;
        int fcount = 0;
        for (int r = 0; r < RPC; ++r) {
            uint64_t idx = base + (uint64_t)r * BLOCK + threadIdx.x;
            int flag = 0, ood = 0;
            double y[NE];
            bool live = idx < A.end;
            if (live) {
                eval_sample<N>(EV, D, A, idx, y, ood, flag, vlds, rlds);
                add_stats<N>(st, y, A);
                st[nst - 4] += 1.0;
                st[nst - 3] += flag;
                st[nst - 1] += ood;
            }
            // compact flagged offsets of this round in thread order
            shc[threadIdx.x] = (live && flag) ? 1 : 0;
            __syncthreads();
            int pos = 0;
            for (int t = 0; t < (int)threadIdx.x; ++t) pos += shc[t];
            int tot = 0;
            if (threadIdx.x == 0)
                for (int t = 0; t < BLOCK; ++t) tot += shc[t];
            if (live && flag) flags[(size_t)ch * CHUNK + fcount + pos] = (uint32_t)(r * BLOCK + threadIdx.x);
            __syncthreads();
            if (threadIdx.x == 0) shc[0] = tot;
            __syncthreads();
            fcount += shc[0];
            __syncthreads();
        }
        for (int s = 0; s < nst; ++s) {
            double v = block_sum(st[s], sh);
            if (threadIdx.x == 0) part[(size_t)ch * NSTAT_MAX + s] = v;
        }
        if (threadIdx.x == 0) nflag[ch] = fcount;
        __syncthreads();
    }
}

template <int N, class Ev>
__global__ void __launch_bounds__(BLOCK) k_dd(Ev EV, DensityDev D, RunArgs A, double *part, const uint32_t *flags,
                                              const int32_t *nflag) {
    constexpr int M = 3 * N - 1, NE = 2 * N - 1;
    constexpr int NST = 3 * NE + 2 * NE + 4;
    __shared__ double sh[BLOCK];
    const int nst = 3 * NE + 2 * A.ncls + 4;
    for (int ch = blockIdx.x; ch < A.nchunks; ch += gridDim.x) {
        int nf = nflag[ch];
        if (nf == 0) continue;
        double st[NST];
        for (int s = 0; s < NST; ++s) st[s] = 0.0;
        uint64_t base = A.begin + (uint64_t)(A.chunk0 + ch) * CHUNK;
        for (int f = threadIdx.x; f < nf; f += BLOCK) {
            uint64_t idx = base + flags[(size_t)ch * CHUNK + f];
            double u[2 * M], z[M];
            int path[M];
            uniforms(A.seed, A.uid, idx, D.ptheta ? 2 * M : 2 * M - 1, u);
            SampleOut o = sample_point<M>(D, u, z, path);
            ea Im[NE], aIm[NE];
            VarsPriv<ea, Ev::kLds ? Dims<N>::NV : 1> vm;
            EV.template eval<ea, N>(z, Im, aIm, vm);
            dd I[NE], aI[NE];
            VarsPriv<dd, Ev::kLds ? Dims<N>::NV : 1> vd;
            EV.template eval<dd, N>(z, I, aI, vd);
            double y[NE];
            int fail = 0;
            for (int e = 0; e < NE; ++e) {
                double ye = ldexp(to_double(I[e]) / o.gx, -o.gj);
                double r = KAPPA * 0x1p-104 * ldexp(Im[e].a / o.gx, -o.gj);
                if (!(r <= fabs(A.tau) || A.tau < 0) || !isfinite(ye)) fail = 1;
                y[e] = ye;
            }
            if (fail) {
                for (int e = 0; e < NE; ++e) y[e] = 0.0;
                st[nst - 2] += 1.0;
            }
            add_stats<N>(st, y, A);
        }
        for (int s = 0; s < nst; ++s) {
            double v = block_sum(st[s], sh);
            if (threadIdx.x == 0) part[(size_t)ch * NSTAT_MAX + s] += v;
        }
    }
}


// Launch the FP64 pass of one chunk batch.
template <int N, class Ev>
void launch_fp64_ev(const Ev &EV, const DensityDev &D, const RunArgs &A, int grid, double *part, uint32_t *flag,
                    int32_t *nflag, hipStream_t s) {
    hipLaunchKernelGGL((k_integrate<N, Ev>), dim3(grid), dim3(BLOCK), 0, s, EV, D, A, part, flag, nflag);
}

// Launch the double-double recompute of the flagged samples of a chunk batch.
template <int N, class Ev>
void launch_dd_ev(const Ev &EV, const DensityDev &D, const RunArgs &A, int grid, double *part, uint32_t *flag,
                  int32_t *nflag, hipStream_t s) {
    hipLaunchKernelGGL((k_dd<N, Ev>), dim3(grid), dim3(BLOCK), 0, s, EV, D, A, part, flag, nflag);
}

template <int N, class Ev, typename T>
void launch_eval_ev(const Ev &EV, const double *z, uint64_t n, double *I, double *a, double *b, hipStream_t s) {
    dim3 gr((unsigned)((n + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL((k_eval<T, N, Ev>), gr, dim3(BLOCK), 0, s, EV, z, n, I, a, b);
}

}  // namespace amm
