// amm_mlp.hip -- learned sector sampler: pilot statistics, MLP training and
// tabulation (an extension beyond the paper; the paper's density is the fallback).
//
// Pilot: samples from the plain density g; each sample's weight
// w = sqrt(sum_e y_e^2) (y = I/g per insertion), quantised to an integer
// relative to the mean weight, is added to W(s, j) for every (set s, chosen
// line j) on its sector path (integer sums: the table is reproducible).  Training minimises
// -sum w_row log P_theta(j|s) with P_theta = softmax_j(log P0(j|s) + d(s,j)),
// d the MLP output; the gradient is reduced per fixed tile in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "amm_ctx.h"

using namespace amm;

namespace {

constexpr int MB = 64;          // rows per backward tile
constexpr int BW_BLOCKS = 512;  // backward grid (fixed: deterministic sums)

// ---------------------------------------------------------------------------
// Pilot kernels
// ---------------------------------------------------------------------------
// Weight of sample i: w_i = sqrt(sum_e y_e^2), y_e = I_e / g.  The FP64 value
// is used when its round-off bound is below 1% of w; otherwise the point is
// recomputed in double-double (non-finite -> 0).
template <int N>
__global__ void __launch_bounds__(BLOCK) k_pilot_w(PlanDev P, DensityDev D, uint32_t uid, uint64_t seed, uint64_t c0,
                                                   uint64_t n, double *wbuf) {
    constexpr int M = 3 * N - 1, NE = 2 * N - 1;
    __shared__ double vlds[Dims<N>::NVL * BLOCK];
    set_one_slot<N>(vlds + threadIdx.x, BLOCK);
    uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double u[2 * M], z[M];
    int path[M];
    uniforms(seed, uid, c0 + i, 2 * M - 1, u);
    SampleOut o = sample_point<M>(D, u, z, path);
    if (o.ood) {
        wbuf[i] = 0.0;
        return;
    }
    ea I[NE], A[NE];
    VarsLdsEa vars{vlds + threadIdx.x, BLOCK, 0.0};
    eval_graph<ea, N>(P, z, I, A, vars);
    double w2 = 0.0, r = 0.0;
    for (int e = 0; e < NE; ++e) {
        double y = ldexp(I[e].v / o.gx, -o.gj);
        w2 += y * y;
        r += KAPPA * 0x1p-53 * ldexp(I[e].a / o.gx, -o.gj);
    }
    double w = sqrt(w2);
    if (!(r <= 0.01 * w) || !isfinite(w)) {
        dd Id[NE], Ad[NE];
        VarsPriv<dd, Dims<N>::NV> vd;
        eval_graph<dd, N>(P, z, Id, Ad, vd);
        w2 = 0.0;
        for (int e = 0; e < NE; ++e) {
            double y = ldexp(to_double(Id[e]) / o.gx, -o.gj);
            w2 += y * y;
        }
        w = sqrt(w2);
        if (!isfinite(w)) w = 0.0;
    }
    wbuf[i] = w;
}

// wref = mean of wbuf[0, n) in a fixed order (one block of 1024 threads).
__global__ void __launch_bounds__(1024) k_pilot_ref(const double *wbuf, uint64_t n, double *wref) {
    __shared__ double sh[1024];
    const int t = threadIdx.x;
    double s = 0.0;
    for (uint64_t i = t; i < n; i += 1024) s += wbuf[i];
    sh[t] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *wref = n ? sh[0] / (double)n : 0.0;
}

// Adds the quantised weight q_i = min(w_i / wref, 2^8) * 2^24 (an integer) to
// Wq(s, j) for every step (s, j) of the sample's sector path.  Integer atomics
// make the table independent of the order of the additions.
template <int N>
__global__ void __launch_bounds__(BLOCK) k_pilot_scatter(DensityDev D, uint32_t uid, uint64_t seed, uint64_t c0,
                                                         uint64_t n, const double *wbuf, const double *wref,
                                                         unsigned long long *Wq) {
    constexpr int M = 3 * N - 1;
    uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const double ref = *wref;
    const double w = wbuf[i];
    if (!(ref > 0.0) || !(w > 0.0)) return;
    const unsigned long long q = (unsigned long long)(fmin(w / ref, 256.0) * 16777216.0);
    if (q == 0ull) return;
    double u[2 * M], z[M];
    int path[M];
    uniforms(seed, uid, c0 + i, 2 * M - 1, u);
    sample_point<M>(D, u, z, path);
    uint32_t s = (1u << M) - 1u;
    for (int l = 0; l < M - 1; ++l) {
        atomicAdd(&Wq[(size_t)s * M + path[l]], q);
        s &= ~(1u << path[l]);
    }
}

__global__ void k_pilot_table(const unsigned long long *Wq, size_t cells, double *W) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cells) W[i] = (double)Wq[i];
}

// ---------------------------------------------------------------------------
// MLP kernels (FP32)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_params(const float *p, float *sh) {
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) sh[i] = p[i];
    __syncthreads();
}

// forward: d per row; optionally store activations h1, h2 [R x 64]
__global__ void __launch_bounds__(256) k_fwd(const float *params, const float *X, int R, float *d, float *h1o,
                                             float *h2o) {
    __shared__ float sp[MLP_NPARAM];
    load_params(params, sp);
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const float *W1 = sp, *b1 = W1 + MLP_H * MLP_NF, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H, *w3 = b2 + MLP_H,
                *b3 = w3 + MLP_H;
    float x[MLP_NF], h1[MLP_H];
    for (int k = 0; k < MLP_NF; ++k) x[k] = X[(size_t)r * MLP_NF + k];
    for (int a = 0; a < MLP_H; ++a) {
        float s = b1[a];
        for (int k = 0; k < MLP_NF; ++k) s = fmaf(W1[a * MLP_NF + k], x[k], s);
        h1[a] = tanhf(s);
        if (h1o) h1o[(size_t)r * MLP_H + a] = h1[a];
    }
    float out = b3[0];
    for (int a = 0; a < MLP_H; ++a) {
        float s = b2[a];
        for (int k = 0; k < MLP_H; ++k) s = fmaf(W2[a * MLP_H + k], h1[k], s);
        float h2 = tanhf(s);
        if (h2o) h2o[(size_t)r * MLP_H + a] = h2;
        out = fmaf(w3[a], h2, out);
    }
    d[r] = out;
}

// per group: softmax of (feature0 + d), gradient w.r.t. d, group loss; or
// (tab != null) write P_theta into the [2^M x M] table of the graph.
__global__ void k_group(const float *X, const float *d, const float *w, const int32_t *goff, int G, float *gd,
                        double *gloss, const int32_t *rs, const int32_t *rj, float *tab, int M) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    int a = goff[g], b = goff[g + 1];
    float mx = -INFINITY;
    for (int r = a; r < b; ++r) mx = fmaxf(mx, X[(size_t)r * MLP_NF] + d[r]);
    float den = 0.f;
    for (int r = a; r < b; ++r) den += expf(X[(size_t)r * MLP_NF] + d[r] - mx);
    if (tab) {
        for (int r = a; r < b; ++r) tab[(size_t)rs[r] * M + rj[r]] = expf(X[(size_t)r * MLP_NF] + d[r] - mx) / den;
        return;
    }
    float wsum = 0.f;
    for (int r = a; r < b; ++r) wsum += w[r];
    double loss = 0.0;
    for (int r = a; r < b; ++r) {
        float lp = X[(size_t)r * MLP_NF] + d[r] - mx - logf(den);
        float P = expf(lp);
        gd[r] = -w[r] + P * wsum;
        loss -= (double)w[r] * (double)lp;
    }
    gloss[g] = loss;
}

// backward: per tile of MB rows, thread t owns parameters t, t+256, ...
__global__ void __launch_bounds__(256) k_bwd(const float *params, const float *X, const float *h1, const float *h2,
                                             const float *gd, int R, float *partial) {
    __shared__ float sW2[MLP_H * MLP_H];
    __shared__ float sw3[MLP_H];
    __shared__ float g2s[MB][MLP_H];
    __shared__ float g1s[MB][MLP_H];
    __shared__ float h1s[MB][MLP_H];
    __shared__ float h2s[MB][MLP_H];
    __shared__ float xs[MB][MLP_NF];
    __shared__ float gds[MB];
    const float *W2g = params + MLP_H * MLP_NF + MLP_H;
    const float *w3g = W2g + MLP_H * MLP_H + MLP_H;
    for (int i = threadIdx.x; i < MLP_H * MLP_H; i += blockDim.x) sW2[i] = W2g[i];
    for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) sw3[i] = w3g[i];
    constexpr int PER = (MLP_NPARAM + 255) / 256;
    float acc[PER];
    for (int q = 0; q < PER; ++q) acc[q] = 0.f;
    __syncthreads();
    int ntiles = (R + MB - 1) / MB;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int r0 = tile * MB;
        // stage rows
        for (int i = threadIdx.x; i < MB * MLP_H; i += blockDim.x) {
            int rr = i / MLP_H, a = i % MLP_H;
            int r = r0 + rr;
            h1s[rr][a] = r < R ? h1[(size_t)r * MLP_H + a] : 0.f;
            h2s[rr][a] = r < R ? h2[(size_t)r * MLP_H + a] : 0.f;
        }
        for (int i = threadIdx.x; i < MB * MLP_NF; i += blockDim.x) {
            int rr = i / MLP_NF, k = i % MLP_NF;
            int r = r0 + rr;
            xs[rr][k] = r < R ? X[(size_t)r * MLP_NF + k] : 0.f;
        }
        for (int i = threadIdx.x; i < MB; i += blockDim.x) gds[i] = (r0 + i) < R ? gd[r0 + i] : 0.f;
        __syncthreads();
        // g2 = gd * w3 * (1 - h2^2)
        for (int i = threadIdx.x; i < MB * MLP_H; i += blockDim.x) {
            int rr = i / MLP_H, a = i % MLP_H;
            float h = h2s[rr][a];
            g2s[rr][a] = gds[rr] * sw3[a] * (1.f - h * h);
        }
        __syncthreads();
        // g1 = (W2^T g2) * (1 - h1^2)
        for (int i = threadIdx.x; i < MB * MLP_H; i += blockDim.x) {
            int rr = i / MLP_H, k = i % MLP_H;
            float s = 0.f;
            for (int a = 0; a < MLP_H; ++a) s = fmaf(sW2[a * MLP_H + k], g2s[rr][a], s);
            float h = h1s[rr][k];
            g1s[rr][k] = s * (1.f - h * h);
        }
        __syncthreads();
        for (int q = 0; q < PER; ++q) {
            int p = threadIdx.x + q * 256;
            if (p >= MLP_NPARAM) break;
            float s = 0.f;
            if (p < MLP_H * MLP_NF) {                       // W1[a][k]
                int a = p / MLP_NF, k = p % MLP_NF;
                for (int rr = 0; rr < MB; ++rr) s = fmaf(g1s[rr][a], xs[rr][k], s);
            } else if (p < MLP_H * MLP_NF + MLP_H) {        // b1
                int a = p - MLP_H * MLP_NF;
                for (int rr = 0; rr < MB; ++rr) s += g1s[rr][a];
            } else if (p < MLP_H * MLP_NF + MLP_H + MLP_H * MLP_H) {   // W2[a][k]
                int o = p - MLP_H * MLP_NF - MLP_H;
                int a = o / MLP_H, k = o % MLP_H;
                for (int rr = 0; rr < MB; ++rr) s = fmaf(g2s[rr][a], h1s[rr][k], s);
            } else if (p < MLP_H * MLP_NF + 2 * MLP_H + MLP_H * MLP_H) {   // b2
                int a = p - MLP_H * MLP_NF - MLP_H - MLP_H * MLP_H;
                for (int rr = 0; rr < MB; ++rr) s += g2s[rr][a];
            } else if (p < MLP_NPARAM - 1) {                // w3
                int a = p - (MLP_H * MLP_NF + 2 * MLP_H + MLP_H * MLP_H);
                for (int rr = 0; rr < MB; ++rr) s = fmaf(gds[rr], h2s[rr][a], s);
            } else {                                        // b3
                for (int rr = 0; rr < MB; ++rr) s += gds[rr];
            }
            acc[q] += s;
        }
        __syncthreads();
    }
    for (int q = 0; q < PER; ++q) {
        int p = threadIdx.x + q * 256;
        if (p < MLP_NPARAM) partial[(size_t)blockIdx.x * MLP_NPARAM + p] = acc[q];
    }
}

__global__ void k_reduce_grad(const float *partial, int nb, float *grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * MLP_NPARAM + p];
    grad[p] = s;
}

// loss = sum of the per-set losses: 256 threads sum strided slices, then a
// fixed tree, so the value does not depend on timing
__global__ void __launch_bounds__(256) k_reduce_loss(const double *gl, int G, float *loss) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int g = t; g < G; g += 256) s += gl[g];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *loss = (float)sh[0];
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int t, float lr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / (1.f - powf(b1, (float)t));
    float vh = vi / (1.f - powf(b2, (float)t));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_row_weights(const double *W, const int32_t *rs, const int32_t *rj, int R, int M, double inv_tot,
                              float *w) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    w[r] = (float)(W[(size_t)rs[r] * M + rj[r]] * inv_tot);
}

__global__ void k_singletons(float *tab, int M) {
    int j = threadIdx.x;
    if (j < M) tab[(size_t)(1u << j) * M + j] = 1.f;
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
int build_rows(amm_ctx *c, int g) {
    MlpRows &R = c->mlp.rows[g];
    if (R.built) return AMM_OK;
    const GraphSlot &s = c->slots[g];
    const SEGraph &G = c->graphs[g];
    int n = G.n, M = 3 * n - 1;
    uint32_t full = (1u << M) - 1u;
    R.feat.clear(); R.s.clear(); R.j.clear(); R.goff.clear();
    for (uint32_t m = 1; m <= full; ++m) {
        int cnt = __builtin_popcount(m);
        if (cnt < 2) continue;
        double tot = 0.0;
        for (int j = 0; j < M; ++j) if ((m >> j) & 1u) tot = tot + s.dens.W1[m & ~(1u << j)];
        int Ls, cs, ngs, nes;
        set_stats(G, m, &Ls, &cs, &ngs, &nes);
        double logF = std::log(s.dens.F1[m]);
        R.goff.push_back((int)R.s.size());
        for (int j = 0; j < M; ++j) {
            if (!((m >> j) & 1u)) continue;
            uint32_t r = m & ~(1u << j);
            int Lr, cr, ngr, ner;
            set_stats(G, r, &Lr, &cr, &ngr, &ner);
            double f[MLP_NF] = {std::log(s.dens.W1[r] / tot), s.dens.deg1[r], m != full ? s.dens.deg1[m] : 0.0,
                                (double)cnt / M, j < 2 * n - 1 ? 1.0 : 0.0, (double)j / M, omega_set(G, r),
                                (double)Lr / n, (double)Ls / n, (double)ngs / n, (double)nes / (2 * n - 1),
                                n / 5.0, (double)ngr / n, (double)cr / M, logF / M, 1.0};
            for (int k = 0; k < MLP_NF; ++k) R.feat.push_back((float)f[k]);
            R.s.push_back((int32_t)m);
            R.j.push_back(j);
        }
    }
    R.goff.push_back((int)R.s.size());
    size_t nr = R.s.size(), ng = R.goff.size() - 1;
    std::vector<int32_t> grp(nr);
    for (size_t q = 0; q < ng; ++q)
        for (int r = R.goff[q]; r < R.goff[q + 1]; ++r) grp[r] = (int32_t)q;
    HIPCHK(hipMalloc((void **)&R.d_feat, R.feat.size() * sizeof(float)));
    HIPCHK(hipMalloc((void **)&R.d_s, nr * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&R.d_j, nr * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&R.d_grp, nr * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&R.d_goff, R.goff.size() * sizeof(int32_t)));
    HIPCHK(hipMemcpy(R.d_feat, R.feat.data(), R.feat.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.d_s, R.s.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.d_j, R.j.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.d_grp, grp.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.d_goff, R.goff.data(), R.goff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    R.built = true;
    return AMM_OK;
}

// Initial parameters: W1, W2 uniform in +-sqrt(3/fan_in) from Philox draws
// u_k = uniform52(words 0,1 of philox(counter (k, 0, 0x4D4C50, 0), key (seed_lo, seed_hi))).
void init_params(uint64_t seed, std::vector<float> &p) {
    p.assign(MLP_NPARAM, 0.f);
    auto draw = [&](uint32_t k) {
        uint32_t cnt[4] = {k, 0u, 0x4D4C50u, 0u};
        philox4x32_10(cnt, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
        return uniform52(cnt[0], cnt[1]);
    };
    double a1 = std::sqrt(3.0 / MLP_NF), a2 = std::sqrt(3.0 / MLP_H);
    for (int k = 0; k < MLP_H * MLP_NF; ++k) p[k] = (float)((2.0 * draw(k) - 1.0) * a1);
    int o = MLP_H * MLP_NF + MLP_H;
    for (int k = 0; k < MLP_H * MLP_H; ++k) p[o + k] = (float)((2.0 * draw(o + k) - 1.0) * a2);
}

int ensure_params(amm_ctx *c, uint64_t seed, bool reinit) {
    MlpState &S = c->mlp;
    if (!S.d_params) {
        HIPCHK(hipMalloc((void **)&S.d_params, MLP_NPARAM * sizeof(float)));
        HIPCHK(hipMalloc((void **)&S.d_m, MLP_NPARAM * sizeof(float)));
        HIPCHK(hipMalloc((void **)&S.d_v, MLP_NPARAM * sizeof(float)));
        reinit = true;
    }
    if (reinit) {
        std::vector<float> p;
        init_params(seed, p);
        HIPCHK(hipMemcpy(S.d_params, p.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(hipMemset(S.d_m, 0, MLP_NPARAM * sizeof(float)));
        HIPCHK(hipMemset(S.d_v, 0, MLP_NPARAM * sizeof(float)));
        S.step = 0;
    }
    return AMM_OK;
}

// Loss and gradient on device rows; scratch buffers allocated per call.
int loss_grad(amm_ctx *c, const float *X, const float *w, const int32_t *goff, int R, int G, float *loss,
              float *grad, hipStream_t st) {
    float *d = nullptr, *h1 = nullptr, *h2 = nullptr, *gd = nullptr, *part = nullptr;
    double *gl = nullptr;
    HIPCHK(hipMalloc((void **)&d, (size_t)R * sizeof(float)));
    HIPCHK(hipMalloc((void **)&h1, (size_t)R * MLP_H * sizeof(float)));
    HIPCHK(hipMalloc((void **)&h2, (size_t)R * MLP_H * sizeof(float)));
    HIPCHK(hipMalloc((void **)&gd, (size_t)R * sizeof(float)));
    HIPCHK(hipMalloc((void **)&gl, (size_t)G * sizeof(double)));
    HIPCHK(hipMalloc((void **)&part, (size_t)BW_BLOCKS * MLP_NPARAM * sizeof(float)));
    hipLaunchKernelGGL(k_fwd, dim3((R + 255) / 256), dim3(256), 0, st, c->mlp.d_params, X, R, d, h1, h2);
    hipLaunchKernelGGL(k_group, dim3((G + 255) / 256), dim3(256), 0, st, X, d, w, goff, G, gd, gl, nullptr, nullptr,
                       nullptr, 0);
    hipLaunchKernelGGL(k_bwd, dim3(BW_BLOCKS), dim3(256), 0, st, c->mlp.d_params, X, h1, h2, gd, R, part);
    hipLaunchKernelGGL(k_reduce_grad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, part, BW_BLOCKS, grad);
    hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(256), 0, st, gl, G, loss);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    hipFree(d); hipFree(h1); hipFree(h2); hipFree(gd); hipFree(gl); hipFree(part);
    return AMM_OK;
}

}  // namespace

namespace amm {
void mlp_free_rows(MlpState &m) {
    for (auto &r : m.rows) {
        hipFree(r.d_feat); hipFree(r.d_s); hipFree(r.d_j); hipFree(r.d_grp); hipFree(r.d_goff);
    }
    m.rows.clear();
}

void mlp_free(MlpState &m) {
    hipFree(m.d_params); hipFree(m.d_m); hipFree(m.d_v);
    m.d_params = m.d_m = m.d_v = nullptr;
    mlp_free_rows(m);
}
}  // namespace amm

extern "C" {

int amm_pilot(amm_ctx *c, uint64_t seed, uint64_t n, int gb, int ge, void *stream) {
    if (!c || gb < 0 || ge > (int)c->slots.size() || gb >= ge || n == 0)
        return fail(AMM_E_ARG, "amm_pilot: bad graph range or sample count");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    const uint64_t step = (uint64_t)1 << 23;
    const uint64_t nbuf = std::min(step, n);
    double *wbuf = nullptr, *wref = nullptr;
    unsigned long long *Wq = nullptr;
    size_t maxcells = 0;
    for (int g = gb; g < ge; ++g) {
        if (!c->slots[g].has_plan) return fail(AMM_E_NOTBUILT, "amm_pilot: integrand tables not built");
        maxcells = std::max(maxcells, ((size_t)1 << c->slots[g].M) * c->slots[g].M);
    }
    HIPCHK(hipMalloc((void **)&wbuf, nbuf * sizeof(double)));
    HIPCHK(hipMalloc((void **)&wref, sizeof(double)));
    HIPCHK(hipMalloc((void **)&Wq, maxcells * sizeof(unsigned long long)));
    int rc = AMM_OK;
    for (int g = gb; g < ge && rc == AMM_OK; ++g) {
        GraphSlot &s = c->slots[g];
        size_t cells = ((size_t)1 << s.M) * s.M;
        if (!s.d_pilotW && hipMalloc((void **)&s.d_pilotW, cells * sizeof(double)) != hipSuccess) {
            rc = fail(AMM_E_HIP, "amm_pilot: out of device memory");
            break;
        }
        hipMemsetAsync(Wq, 0, cells * sizeof(unsigned long long), st);
        PlanDev P = s.plan_dev();
        DensityDev D = s.dens_dev(false);
        for (uint64_t c0 = 0; c0 < n; c0 += step) {
            uint64_t m = std::min(step, n - c0);
            dim3 gr((unsigned)((m + BLOCK - 1) / BLOCK)), bl(BLOCK);
            switch (s.n) {
                case 1: hipLaunchKernelGGL(k_pilot_w<1>, gr, bl, 0, st, P, D, s.uid, seed, c0, m, wbuf); break;
                case 2: hipLaunchKernelGGL(k_pilot_w<2>, gr, bl, 0, st, P, D, s.uid, seed, c0, m, wbuf); break;
                case 3: hipLaunchKernelGGL(k_pilot_w<3>, gr, bl, 0, st, P, D, s.uid, seed, c0, m, wbuf); break;
                case 4: hipLaunchKernelGGL(k_pilot_w<4>, gr, bl, 0, st, P, D, s.uid, seed, c0, m, wbuf); break;
                default: rc = fail(AMM_E_ARG, "amm_pilot: unsupported loop order");
            }
            if (rc) break;
            if (c0 == 0) hipLaunchKernelGGL(k_pilot_ref, dim3(1), dim3(1024), 0, st, wbuf, m, wref);
            switch (s.n) {
                case 1: hipLaunchKernelGGL(k_pilot_scatter<1>, gr, bl, 0, st, D, s.uid, seed, c0, m, wbuf, wref, Wq); break;
                case 2: hipLaunchKernelGGL(k_pilot_scatter<2>, gr, bl, 0, st, D, s.uid, seed, c0, m, wbuf, wref, Wq); break;
                case 3: hipLaunchKernelGGL(k_pilot_scatter<3>, gr, bl, 0, st, D, s.uid, seed, c0, m, wbuf, wref, Wq); break;
                case 4: hipLaunchKernelGGL(k_pilot_scatter<4>, gr, bl, 0, st, D, s.uid, seed, c0, m, wbuf, wref, Wq); break;
            }
        }
        if (rc) break;
        hipLaunchKernelGGL(k_pilot_table, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, Wq, cells,
                           s.d_pilotW);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            rc = fail(AMM_E_HIP, "amm_pilot: kernel failure");
    }
    hipStreamSynchronize(st);
    hipFree(wbuf); hipFree(wref); hipFree(Wq);
    c->last_stream = st;
    return rc;
}

int amm_pilot_table(const amm_ctx *c, int g, double *host, size_t cap) {
    if (!c || g < 0 || g >= (int)c->slots.size() || !host) return fail(AMM_E_ARG, "amm_pilot_table: bad argument");
    const GraphSlot &s = c->slots[g];
    size_t cells = ((size_t)1 << s.M) * s.M;
    if (!s.d_pilotW) return fail(AMM_E_NOTBUILT, "amm_pilot_table: run amm_pilot first");
    if (cap < cells) return fail(AMM_E_ARG, "amm_pilot_table: buffer too small");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpy(host, s.d_pilotW, cells * sizeof(double), hipMemcpyDeviceToHost));
    return AMM_OK;
}

int amm_mlp_train(amm_ctx *c, int epochs, float lr, uint64_t init_seed, void *stream) {
    if (!c || epochs < 0) return fail(AMM_E_ARG, "amm_mlp_train: bad argument");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    if (c->mlp.rows.size() != c->slots.size()) c->mlp.rows.resize(c->slots.size());
    // concatenated training rows of all graphs with a pilot table
    std::vector<int> gs;
    size_t Rtot = 0, Gtot = 0;
    for (int g = 0; g < (int)c->slots.size(); ++g) {
        if (!c->slots[g].built || !c->slots[g].d_pilotW) continue;
        int rc = build_rows(c, g);
        if (rc) return rc;
        gs.push_back(g);
        Rtot += c->mlp.rows[g].s.size();
        Gtot += c->mlp.rows[g].goff.size() - 1;
    }
    if (gs.empty()) return fail(AMM_E_ARG, "amm_mlp_train: run amm_pilot first");
    int rc = ensure_params(c, init_seed, true);
    if (rc) return rc;
    float *X = nullptr, *w = nullptr, *grad = nullptr, *loss = nullptr;
    int32_t *goff = nullptr;
    HIPCHK(hipMalloc((void **)&X, Rtot * MLP_NF * sizeof(float)));
    HIPCHK(hipMalloc((void **)&w, Rtot * sizeof(float)));
    HIPCHK(hipMalloc((void **)&goff, (Gtot + 1) * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&grad, MLP_NPARAM * sizeof(float)));
    HIPCHK(hipMalloc((void **)&loss, sizeof(float)));
    std::vector<int32_t> hgoff;
    size_t r0 = 0;
    for (int g : gs) {
        MlpRows &R = c->mlp.rows[g];
        size_t nr = R.s.size();
        HIPCHK(hipMemcpyAsync(X + r0 * MLP_NF, R.d_feat, nr * MLP_NF * sizeof(float), hipMemcpyDeviceToDevice, st));
        // per-graph normalisation: total pilot weight over the graph's rows
        std::vector<double> Wh(((size_t)1 << c->slots[g].M) * c->slots[g].M);
        HIPCHK(hipMemcpy(Wh.data(), c->slots[g].d_pilotW, Wh.size() * sizeof(double), hipMemcpyDeviceToHost));
        double tot = 0.0;
        for (size_t q = 0; q < nr; ++q) tot += Wh[(size_t)R.s[q] * c->slots[g].M + R.j[q]];
        double inv = tot > 0 ? 1.0 / (tot * gs.size()) : 0.0;
        hipLaunchKernelGGL(k_row_weights, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, c->slots[g].d_pilotW,
                           R.d_s, R.d_j, (int)nr, c->slots[g].M, inv, w + r0);
        for (size_t q = 0; q + 1 < R.goff.size(); ++q) hgoff.push_back((int32_t)(R.goff[q] + r0));
        r0 += nr;
    }
    hgoff.push_back((int32_t)Rtot);
    HIPCHK(hipMemcpy(goff, hgoff.data(), hgoff.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    for (int t = 1; t <= epochs; ++t) {
        rc = loss_grad(c, X, w, goff, (int)Rtot, (int)Gtot, loss, grad, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, c->mlp.d_params, grad,
                           c->mlp.d_m, c->mlp.d_v, t, lr);
    }
    HIPCHK(hipGetLastError());
    // tabulate P_theta for every built graph
    for (int g = 0; g < (int)c->slots.size(); ++g) {
        GraphSlot &s = c->slots[g];
        if (!s.built) continue;
        rc = build_rows(c, g);
        if (rc) return rc;
        MlpRows &R = c->mlp.rows[g];
        size_t nr = R.s.size();
        size_t cells = ((size_t)1 << s.M) * s.M;
        if (!s.d_ptheta) HIPCHK(hipMalloc((void **)&s.d_ptheta, cells * sizeof(float)));
        HIPCHK(hipMemsetAsync(s.d_ptheta, 0, cells * sizeof(float), st));
        float *d = nullptr;
        HIPCHK(hipMalloc((void **)&d, nr * sizeof(float)));
        hipLaunchKernelGGL(k_fwd, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, c->mlp.d_params, R.d_feat,
                           (int)nr, d, nullptr, nullptr);
        int G = (int)R.goff.size() - 1;
        hipLaunchKernelGGL(k_group, dim3((G + 255) / 256), dim3(256), 0, st, R.d_feat, d, nullptr, R.d_goff, G,
                           nullptr, nullptr, R.d_s, R.d_j, s.d_ptheta, s.M);
        hipLaunchKernelGGL(k_singletons, dim3(1), dim3(64), 0, st, s.d_ptheta, s.M);
        HIPCHK(hipStreamSynchronize(st));
        hipFree(d);
    }
    c->mlp.trained = true;
    hipFree(X); hipFree(w); hipFree(goff); hipFree(grad); hipFree(loss);
    c->last_stream = st;
    return AMM_OK;
}

int amm_mlp_params(const amm_ctx *c, float *host, size_t cap, size_t *count) {
    if (!c) return fail(AMM_E_ARG, "amm_mlp_params: ctx is NULL");
    if (count) *count = MLP_NPARAM;
    if (!host) return AMM_OK;
    if (cap < (size_t)MLP_NPARAM) return fail(AMM_E_ARG, "amm_mlp_params: buffer too small");
    if (!c->mlp.d_params) return fail(AMM_E_NOTBUILT, "amm_mlp_params: no parameters yet");
    HIPCHK(hipMemcpy(host, c->mlp.d_params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
    return AMM_OK;
}

int amm_mlp_get_params(const amm_ctx *c, float *host_buf, size_t n) {
    return amm_mlp_params(c, host_buf, n, nullptr);
}

int amm_mlp_adam(amm_ctx *c, const float *grad, int t, float lr, int reset_moments, void *stream) {
    if (!c || !grad || t < 1) return fail(AMM_E_ARG, "amm_mlp_adam: bad argument");
    if (!c->mlp.d_params) return fail(AMM_E_NOTBUILT, "amm_mlp_adam: set parameters first");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    if (reset_moments) {
        HIPCHK(hipMemsetAsync(c->mlp.d_m, 0, MLP_NPARAM * sizeof(float), st));
        HIPCHK(hipMemsetAsync(c->mlp.d_v, 0, MLP_NPARAM * sizeof(float), st));
    }
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, c->mlp.d_params, grad, c->mlp.d_m,
                       c->mlp.d_v, t, lr);
    HIPCHK(hipGetLastError());
    c->last_stream = st;
    return AMM_OK;
}

int amm_mlp_set_params(amm_ctx *c, const float *host, size_t count) {
    if (!c || !host || count != (size_t)MLP_NPARAM) return fail(AMM_E_ARG, "amm_mlp_set_params: bad argument");
    HIPCHK(hipSetDevice(c->device));
    int rc = ensure_params(c, 0, false);
    if (rc) return rc;
    HIPCHK(hipMemcpy(c->mlp.d_params, host, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    return AMM_OK;
}

int amm_mlp_features(const amm_ctx *cc, int g, float *rows, int32_t *mask_of_row, int32_t *line_of_row, size_t cap,
                     size_t *n_rows) {
    amm_ctx *c = const_cast<amm_ctx *>(cc);
    if (!c || g < 0 || g >= (int)c->slots.size() || !c->slots[g].built)
        return fail(AMM_E_ARG, "amm_mlp_features: bad graph");
    HIPCHK(hipSetDevice(c->device));
    if (c->mlp.rows.size() != c->slots.size()) c->mlp.rows.resize(c->slots.size());
    int rc = build_rows(c, g);
    if (rc) return rc;
    const MlpRows &R = c->mlp.rows[g];
    if (n_rows) *n_rows = R.s.size();
    if (!rows && !mask_of_row && !line_of_row) return AMM_OK;
    if (cap < R.s.size()) return fail(AMM_E_ARG, "amm_mlp_features: buffer too small");
    if (rows) std::memcpy(rows, R.feat.data(), R.feat.size() * sizeof(float));
    if (mask_of_row) std::memcpy(mask_of_row, R.s.data(), R.s.size() * sizeof(int32_t));
    if (line_of_row) std::memcpy(line_of_row, R.j.data(), R.j.size() * sizeof(int32_t));
    return AMM_OK;
}

int amm_mlp_loss_grad(amm_ctx *c, const float *rows, const float *w, const int32_t *goff, int n_rows, int n_groups,
                      float *loss, float *grad, void *stream) {
    if (!c || !rows || !w || !goff || !loss || !grad || n_rows <= 0 || n_groups <= 0)
        return fail(AMM_E_ARG, "amm_mlp_loss_grad: bad argument");
    if (!c->mlp.d_params) return fail(AMM_E_NOTBUILT, "amm_mlp_loss_grad: set parameters first");
    HIPCHK(hipSetDevice(c->device));
    return loss_grad(c, rows, w, goff, n_rows, n_groups, loss, grad, (hipStream_t)stream);
}

int amm_set_sector_table(amm_ctx *c, int g, const float *host_table) {
    if (!c || g < 0 || g >= (int)c->slots.size() || !c->slots[g].built)
        return fail(AMM_E_ARG, "amm_set_sector_table: bad graph");
    GraphSlot &s = c->slots[g];
    HIPCHK(hipSetDevice(c->device));
    size_t cells = ((size_t)1 << s.M) * s.M;
    if (!s.d_ptheta) HIPCHK(hipMalloc((void **)&s.d_ptheta, cells * sizeof(float)));
    if (host_table) HIPCHK(hipMemcpy(s.d_ptheta, host_table, cells * sizeof(float), hipMemcpyHostToDevice));
    else { hipFree(s.d_ptheta); s.d_ptheta = nullptr; }
    return AMM_OK;
}

}  // extern "C"
