// amm_kernels.h -- Monte Carlo kernels templated on the integrand evaluator
// (the table interpreter of amm_core.h, or a generated per-graph function).
//   k_eval       integrands at given points (FP64 + round-off bound, DD, or FP64 intervals)
//   k_integrate  sample + evaluate + round-off check (eq. interval_accept) +
//                per-chunk deterministic partial sums; flagged samples are
//                compacted per chunk in sample order
//   k_flag_scan  offsets of the flagged samples of a launch
//   k_dd_points  double-double recompute, 1, 4 or 16 lanes per flagged sample
//   k_dd_reduce  per-chunk sums of the recomputed samples, in flag order
#pragma once
#include <type_traits>

#include "amm_ctx.h"

namespace amm {

// Evaluator using the plan tables (variables in LDS columns).
struct InterpEval {
    static constexpr bool kLds = true;
    // Monte Carlo block size: 64-thread blocks keep the LDS variable columns
    // of a block at 64 x NV doubles, so more blocks fit on a compute unit
    static constexpr int kBlock = 64;
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
    static constexpr int kBlock = BLOCK;
    template <typename T, int N, typename Vars>
    __device__ __forceinline__ void eval(const double *z, T *I, T *absI, Vars &) const {
        G::template eval<T>(z, I, absI);
    }
};

struct RunArgs {
    uint64_t seed, begin, end;      // sample index range [begin, end)
    uint32_t uid;
    int chunk0;                     // first chunk (relative to begin) of this launch
    int nchunks;
    double tau;                     // acceptance threshold (<0: flag all; inf: none)
    int ncls;
    int cls_of[MAXNE];
    int learned;
    const uint64_t *base_dev;       // optional device word added to every sample index (graph replays)
    MrgStream mrg;                  // MRG32k3a stream of the graph (mrg.on), else Philox4x32-10
};

__device__ __forceinline__ uint64_t base_offset(const RunArgs &A) { return A.base_dev ? *A.base_dev : 0ull; }

// One segment of a group: graph g's chunks [A.chunk0, A.chunk0 + A.nchunks)
// of its sample range, stored at chunks [gchunk, gchunk + A.nchunks) of the
// group's buffers.
struct SegDev {
    RunArgs A;
    PlanDev P;
    DensityDev D;
    int g, nst, gchunk, pad;
};

// Segment holding group chunk ch (segments sorted by gchunk).
__device__ __forceinline__ int seg_of_chunk(const SegDev *segs, int nseg, int ch) {
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (segs[mid].gchunk <= ch) lo = mid;
        else hi = mid;
    }
    return lo;
}

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
        __shared__ double vlds[Dims<N>::NVL * BLOCK];
        set_one_slot<N>(vlds + threadIdx.x, BLOCK);
        VarsLdsEa vars{vlds + threadIdx.x, BLOCK, 0.0};
        EV.template eval<T, N>(zz, v, a, vars);
    } else {
        VarsPriv<T, Ev::kLds ? Dims<N>::NV : 1> vars;
        EV.template eval<T, N>(zz, v, a, vars);
    }
    for (int e = 0; e < NE; ++e) {
        if (I) I[i * NE + e] = to_double(v[e]);
        if (absI) absI[i * NE + e] = to_double(a[e]);
        if (bound) {
            if constexpr (std::is_same<T, iv>::value) bound[i * NE + e] = radius(v[e]);
            else bound[i * NE + e] = KAPPA * 0x1p-53 * mag(v[e]);
        }
    }
}



// Statistic layout per graph:
//   [0, ne)        sum y_e       [ne, 2ne)  sum y_e^2     [2ne, 3ne) sum |y_e|
//   [3ne, 3ne+c)   sum y_class   [.., +c)   sum y_class^2
//   [3ne+2c]       sum y_tot     [3ne+2c+1] sum y_tot^2   (y_tot = sum_e y_e)
//   then n, n_flag, n_dd_fail, n_ood.
// The insertions of a point share it, so the variance of a class or of the
// graph's total is that of the per-point sum (eq. sigma_down applied to it).
template <int N>
__device__ __forceinline__ void add_stats(double (&st)[nstat_of(2 * N - 1, 2 * N - 1)], const double *y,
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
    double yt = 0.0;
    for (int c = 0; c < NE; ++c) {
        if (c >= A.ncls) break;
        st[3 * NE + c] += yc[c];
        st[3 * NE + A.ncls + c] += yc[c] * yc[c];
    }
    for (int e = 0; e < NE; ++e) yt += y[e];
    st[3 * NE + 2 * A.ncls] += yt;
    st[3 * NE + 2 * A.ncls + 1] += yt * yt;
}

// One sample: point, density, FP64 integrands with their round-off bound and
// the acceptance test of eq. (interval_accept).  flag: the FP64 value is not
// accepted (its y is replaced by the recompute); ddbad: the double-double
// bound (KAPPA 2^-104 a / g) cannot pass either, so the recompute is skipped.
template <int N, class Ev>
__device__ __forceinline__ void eval_sample(const Ev &EV, const DensityDev &D, const RunArgs &A, uint64_t idx,
                                            double *y, int &ood, int &flag, int &ddbad, double *vlds) {
    constexpr int NB = Ev::kBlock;
    constexpr int M = 3 * N - 1, NE = 2 * N - 1;
    double u[2 * M], z[M];
    int path[M];
    draw_uniforms(A.seed, A.uid, A.mrg, idx, D.ptheta ? 2 * M : 2 * M - 1, u);
    SampleOut o = sample_point<M>(D, u, z, path);
    ood = o.ood;
    flag = 0;
    ddbad = 0;
    if (o.ood) {
        for (int e = 0; e < NE; ++e) y[e] = 0.0;
        return;
    }
    bool plain = false;
    if constexpr (Ev::kLds) {
        plain = A.tau == INFINITY;                       // interpreter: skip bounds if unchecked
        set_one_slot<N>(vlds + threadIdx.x, NB);
    }
    if (plain) {
        if constexpr (Ev::kLds) {
            double I[NE], aI[NE];
            VarsLdsD vars{vlds + threadIdx.x, NB};
            EV.template eval<double, N>(z, I, aI, vars);
            for (int e = 0; e < NE; ++e) {
                y[e] = ldexp(I[e] / o.gx, -o.gj);
                if (!isfinite(y[e])) flag = 1;
            }
            if constexpr (N == 1) ddbad = flag;
        }
    } else {
        ea I[NE], aI[NE];
        if constexpr (Ev::kLds) {
            VarsLdsEa vars{vlds + threadIdx.x, NB, 0.0};
            EV.template eval<ea, N>(z, I, aI, vars);
        } else {
            VarsPriv<ea, 1> vars;
            EV.template eval<ea, N>(z, I, aI, vars);
        }
        // the graph's threshold bounds the round-off of the point's total over
        // its insertions: the bounds of the insertions add
        double r = 0.0;
        for (int e = 0; e < NE; ++e) {
            double ye = ldexp(I[e].v / o.gx, -o.gj);
            r += ldexp(I[e].a / o.gx, -o.gj);
            if (!isfinite(ye)) flag = 1;
            // the running bound is first order: where it is not small against
            // the value's scale, second-order terms may exceed it, so the
            // point is recomputed whatever the threshold
            if (!(KAPPA * 0x1p-53 * I[e].a <= 1e-2 * fmax(fabs(I[e].v), aI[e].v))) flag = 1;
            y[e] = ye;
        }
        if (!(KAPPA * 0x1p-53 * r <= A.tau)) flag = 1;
        // hopeless for double-double only when the bound is finite and too
        // large even at the double-double unit (a non-finite bound says nothing)
        if (A.tau >= 0.0 && isfinite(r) && !(KAPPA * 0x1p-104 * r <= A.tau)) ddbad = 1;
        if constexpr (N == 1) ddbad = 1;            // no double-double recompute at one loop (disabled)
    }
    if (flag)
        for (int e = 0; e < NE; ++e) y[e] = 0.0;
}

// Sum over one wavefront (fixed butterfly order; lane 0's value is used).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sums of the statistics: one butterfly per wave, then the waves in
// order.  Every thread must call it; thread s < nst writes statistic s.
template <int NST, int NB>
__device__ __forceinline__ void block_stats(const double (&st)[NST], int nst, double (*shs)[NST], double *out,
                                            bool add) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int s = 0; s < NST; ++s) {
        if (s >= nst) break;
        double v = wave_sum(st[s]);
        if (lane == 0) shs[wv][s] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nst) {
        double v = shs[0][threadIdx.x];
        for (int w = 1; w < NB / 64; ++w) v += shs[w][threadIdx.x];
        if (add) out[threadIdx.x] += v;
        else out[threadIdx.x] = v;
    }
    __syncthreads();
}

// One chunk (CHUNK consecutive samples, local chunk ch of the run A): FP64
// pass, acceptance, flag compaction in sample order, per-chunk sums.  Called
// by every thread of an Ev::kBlock-thread block.
template <int N, class Ev>
__device__ __forceinline__ void process_chunk(const Ev &EV, const DensityDev &D, const RunArgs &A, int ch,
                                              double *part_ch, uint32_t *flags_ch, int32_t *nflag_ch,
                                              double (*shs)[nstat_of(2 * N - 1, 2 * N - 1)], int *shw,
                                              double *vlds) {
    constexpr int NE = 2 * N - 1;
    constexpr int NST = nstat_of(NE, NE);
    constexpr int NB = Ev::kBlock, NW = NB / 64, RND = CHUNK / NB;
    const int nst = nstat_of(NE, A.ncls);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double st[NST];
    for (int s = 0; s < NST; ++s) st[s] = 0.0;
    const uint64_t n_run = A.end - A.begin;
    const uint64_t local0 = (uint64_t)(A.chunk0 + ch) * CHUNK;
    const uint64_t base = base_offset(A) + A.begin + local0;
    int fcount = 0;
    for (int r = 0; r < RND; ++r) {
        const uint64_t off = (uint64_t)r * NB + threadIdx.x;
        int flag = 0, ood = 0, ddbad = 0;
        double y[NE];
        const bool live = local0 + off < n_run;
        if (live) {
            eval_sample<N>(EV, D, A, base + off, y, ood, flag, ddbad, vlds);
            add_stats<N>(st, y, A);
            st[nst - 4] += 1.0;
            st[nst - 3] += flag;
            st[nst - 1] += ood;
        }
        // compact the flagged offsets of this round in thread order
        const bool f = live && flag;
        const uint64_t m = __ballot(f);
        if (lane == 0) shw[wv] = __popcll(m);
        __syncthreads();
        int pos = fcount + __popcll(m & ((1ull << lane) - 1ull));
        for (int w = 0; w < wv; ++w) pos += shw[w];
        if (f) flags_ch[pos] = (uint32_t)off | (ddbad ? FLAG_DDFAIL : 0u);
        for (int w = 0; w < NW; ++w) fcount += shw[w];
        __syncthreads();
    }
    block_stats<NST, NB>(st, nst, shs, part_ch, false);
    if (threadIdx.x == 0) *nflag_ch = fcount;
}

// FP64 pass of one segment: blocks stride over its chunks.
template <int N, class Ev>
__global__ void __launch_bounds__(Ev::kBlock) k_integrate(Ev EV, DensityDev D, RunArgs A, double *part,
                                                          uint32_t *flags, int32_t *nflag) {
    constexpr int NE = 2 * N - 1;
    constexpr int NST = nstat_of(NE, NE);
    constexpr int NB = Ev::kBlock;
    __shared__ double shs[NB / 64][NST];
    __shared__ int shw[NB / 64];
    __shared__ double vlds[(Ev::kLds ? Dims<N>::NVL : 1) * NB];
    for (int ch = blockIdx.x; ch < A.nchunks; ch += gridDim.x)
        process_chunk<N>(EV, D, A, ch, part + (size_t)ch * NSTAT_MAX, flags + (size_t)ch * CHUNK, nflag + ch, shs,
                         shw, vlds);
}

// FP64 pass of a whole group with the table interpreter: a persistent grid
// whose blocks take the group's chunks in order from a work counter (segments
// are ordered heaviest graph first when grouping by cost).  Every block exits
// once the counter passes the group's chunk count.
template <int N>
__global__ void __launch_bounds__(InterpEval::kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_integrate_fused(const SegDev *segs, int nseg, int nch,
                                                                       int *work, double *part, uint32_t *flags,
                                                                       int32_t *nflag) {
    constexpr int NE = 2 * N - 1;
    constexpr int NST = nstat_of(NE, NE);
    constexpr int NB = InterpEval::kBlock;
    __shared__ double shs[NB / 64][NST];
    __shared__ int shw[NB / 64];
    __shared__ double vlds[Dims<N>::NVL * NB];
    __shared__ int item;
    for (;;) {
        if (threadIdx.x == 0) item = atomicAdd(work, 1);
        __syncthreads();
        const int gc = item;
        __syncthreads();
        if (gc >= nch) break;                 // uniform over the block
        const SegDev &S = segs[seg_of_chunk(segs, nseg, gc)];
        const InterpEval EV{S.P};
        process_chunk<N>(EV, S.D, S.A, gc - S.gchunk, part + (size_t)gc * NSTAT_MAX, flags + (size_t)gc * CHUNK,
                         nflag + gc, shs, shw, vlds);
    }
}

static __global__ void k_set_int(int *p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

static __global__ void k_set_u64(uint64_t *p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Advances the device-resident sample base after a replay of a captured batch.
static __global__ void k_advance(uint64_t *base, uint64_t step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += step;
}

// Exclusive scan of the per-chunk flag counts (one block of 1024 threads;
// nchunks <= MAX_GROUP_CHUNKS): off[0..nchunks], off[nchunks] = total.
static __global__ void __launch_bounds__(1024) k_flag_scan(const int32_t *nflag, int nchunks, int32_t *off) {
    constexpr int T = 1024, PER = (MAX_GROUP_CHUNKS + T - 1) / T;
    __shared__ int32_t sh[T];
    const int t = threadIdx.x;
    int32_t loc[PER], s = 0;
    for (int q = 0; q < PER; ++q) {
        int c = t * PER + q;
        loc[q] = c < nchunks ? nflag[c] : 0;
        s += loc[q];
    }
    sh[t] = s;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {          // inclusive Hillis-Steele scan
        int32_t v = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int32_t run = t ? sh[t - 1] : 0;
    for (int q = 0; q < PER; ++q) {
        int c = t * PER + q;
        if (c < nchunks) off[c] = run;
        run += loc[q];
    }
    if (t == T - 1) off[nchunks] = sh[T - 1];
}

// Double-double variables in LDS columns (hi and lo parts).
struct VarsLdsDd {
    double *hi, *lo;
    int stride;
    AMM_HDI void begin() {}
    AMM_HDI void drain() {}
    AMM_HDI void set(int i, const dd &x) { hi[i * stride] = x.hi; lo[i * stride] = x.lo; }
    AMM_HDI dd get(int i) const { return dd(hi[i * stride], lo[i * stride]); }
};

// Double-double recompute of the flagged samples of a group with L lanes per
// sample: lane l evaluates the forest terms l, l + L, ... and the lanes' sums
// are added in a fixed tree, so the result does not depend on the launch.
// y_e of flagged point f goes to ydd[e * cap + f]; a point that fails (bound,
// or a non-finite value) gets NaN in ydd[f].
template <int N, int L>
__device__ __forceinline__ void dd_points_pass(const SegDev *segs, int nseg, int nch, const uint32_t *flags,
                                               const int32_t *off, double *ydd, size_t cap, int32_t total,
                                               double *vh, double *vl) {
    constexpr int M = 3 * N - 1, NE = 2 * N - 1, PPB = DD_BLOCK / L;
    static_assert(DD_BLOCK % L == 0 && (L & (L - 1)) == 0 && L <= 64, "lanes per point");
    const int lane = threadIdx.x % L, slot = threadIdx.x / L;
    // the trip count depends on the block only: every lane reaches the shuffles
    for (int32_t f0 = blockIdx.x * PPB; f0 < total; f0 += gridDim.x * PPB) {
        const int32_t f = f0 + slot;
        bool fail = true;
        double gx = 1.0;
        int gj = 0;
        dd I[NE];
        for (int e = 0; e < NE; ++e) I[e] = dd(0.0);
        if (f < total) {
            int lo = 0, hi = nch;             // largest chunk with off[chunk] <= f
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (off[mid] <= f) lo = mid;
                else hi = mid;
            }
            const SegDev &S = segs[seg_of_chunk(segs, nseg, lo)];
            const uint32_t w = flags[(size_t)lo * CHUNK + (f - off[lo])];
            fail = (w & FLAG_DDFAIL) != 0u;
            if (!fail) {
                uint64_t idx = base_offset(S.A) + S.A.begin + (uint64_t)(S.A.chunk0 + (lo - S.gchunk)) * CHUNK +
                               (w & ~FLAG_DDFAIL);
                double u[2 * M], z[M];
                int path[M];
                draw_uniforms(S.A.seed, S.A.uid, S.A.mrg, idx, S.D.ptheta ? 2 * M : 2 * M - 1, u);
                SampleOut o = sample_point<M>(S.D, u, z, path);
                gx = o.gx;
                gj = o.gj;
                dd aI[NE];
                VarsLdsDd vars{vh + threadIdx.x, vl + threadIdx.x, DD_BLOCK};
                eval_graph<dd, N>(S.P, z, I, aI, vars, lane, L);
            }
        }
        for (int e = 0; e < NE; ++e)
            for (int d = L / 2; d > 0; d >>= 1) {
                const dd o(__shfl_down(I[e].hi, d, L), __shfl_down(I[e].lo, d, L));
                I[e] = I[e] + o;
            }
        if (f < total && lane == 0) {
            double y[NE];
            for (int e = 0; e < NE && !fail; ++e) {
                y[e] = ldexp(to_double(I[e]) / gx, -gj);
                if (!isfinite(y[e])) fail = true;
            }
            if (fail) {
                ydd[f] = NAN;
            } else {
                for (int e = 0; e < NE; ++e) ydd[(size_t)e * cap + f] = y[e];
            }
        }
    }
}

// The flagged samples of a group in double-double.  One lane per sample keeps
// the lanes of a wave on the same table entries (points are in chunk order,
// so a wave's points nearly always share a graph); when the samples alone
// would leave most of the DD_RESIDENT_LANES resident lanes idle, 4 or 16
// lanes share a sample (lower latency per pass).
template <int N>
__global__ void __launch_bounds__(DD_BLOCK) k_dd_points(const SegDev *segs, int nseg, int nch, const uint32_t *flags,
                                                        const int32_t *off, double *ydd, size_t cap) {
    __shared__ double vh[Dims<N>::NV * DD_BLOCK], vl[Dims<N>::NV * DD_BLOCK];
    const int32_t total = off[nch];
    if (total <= DD_RESIDENT_LANES / 16)
        dd_points_pass<N, 16>(segs, nseg, nch, flags, off, ydd, cap, total, vh, vl);
    else if (total <= DD_RESIDENT_LANES / 4)
        dd_points_pass<N, 4>(segs, nseg, nch, flags, off, ydd, cap, total, vh, vl);
    else
        dd_points_pass<N, 1>(segs, nseg, nch, flags, off, ydd, cap, total, vh, vl);
}

// Adds the recomputed samples of each chunk to its partial sums, in flag order.
template <int N>
__global__ void __launch_bounds__(BLOCK) k_dd_reduce(const SegDev *segs, int nseg, int nch, const int32_t *off,
                                                     const double *ydd, size_t cap, double *part) {
    constexpr int NE = 2 * N - 1;
    constexpr int NST = nstat_of(NE, NE);
    __shared__ double shs[BLOCK / 64][NST];
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int32_t a = off[ch], b = off[ch + 1];
        if (a == b) continue;                 // uniform over the block
        const RunArgs &A = segs[seg_of_chunk(segs, nseg, ch)].A;
        const int nst = nstat_of(NE, A.ncls);
        double st[NST];
        for (int s = 0; s < NST; ++s) st[s] = 0.0;
        for (int32_t f = a + threadIdx.x; f < b; f += BLOCK) {
            double y[NE];
            if (isnan(ydd[f])) {
                for (int e = 0; e < NE; ++e) y[e] = 0.0;
                st[nst - 2] += 1.0;
            } else {
                for (int e = 0; e < NE; ++e) y[e] = ydd[(size_t)e * cap + f];
            }
            add_stats<N>(st, y, A);
        }
        block_stats<NST, BLOCK>(st, nst, shs, part + (size_t)ch * NSTAT_MAX, true);
    }
}

// acc[g][s] += sum over the segment's chunks of part[chunk][s]: block
// (s, segment); thread t sums chunks t, t+256, ... in order, then a fixed tree.
static __global__ void __launch_bounds__(256) k_reduce_seg(const SegDev *segs, const double *part, double *acc) {
    __shared__ double sh[256];
    const SegDev &S = segs[blockIdx.y];
    const int s = blockIdx.x, t = threadIdx.x;
    if (s >= S.nst) return;                   // uniform over the block
    double v = 0.0;
    for (int c = t; c < S.A.nchunks; c += 256) v += part[(size_t)(S.gchunk + c) * NSTAT_MAX + s];
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) acc[(size_t)S.g * NSTAT_MAX + s] += sh[0];
}

// Launch the FP64 pass of one chunk batch.
template <int N, class Ev>
void launch_fp64_ev(const Ev &EV, const DensityDev &D, const RunArgs &A, int grid, double *part, uint32_t *flag,
                    int32_t *nflag, hipStream_t s) {
    hipLaunchKernelGGL((k_integrate<N, Ev>), dim3(grid), dim3(Ev::kBlock), 0, s, EV, D, A, part, flag, nflag);
}

// Double-double recompute of the flagged samples of a group (scan, per-point
// recompute, per-chunk sums), then the per-segment reduction into the graph
// accumulators.
template <int N>
void launch_dd_group(const SegDev *d_segs, int nseg, int nch, int grid_pts, int grid_red, double *part,
                     const uint32_t *flag, const int32_t *nflag, int32_t *off, double *ydd, size_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_flag_scan, dim3(1), dim3(1024), 0, s, nflag, nch, off);
    hipLaunchKernelGGL((k_dd_points<N>), dim3(grid_pts), dim3(DD_BLOCK), 0, s, d_segs, nseg, nch, flag, off, ydd, cap);
    hipLaunchKernelGGL((k_dd_reduce<N>), dim3(grid_red), dim3(BLOCK), 0, s, d_segs, nseg, nch, off, ydd, cap, part);
}

template <int N, class Ev, typename T>
void launch_eval_ev(const Ev &EV, const double *z, uint64_t n, double *I, double *a, double *b, hipStream_t s) {
    dim3 gr((unsigned)((n + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL((k_eval<T, N, Ev>), gr, dim3(BLOCK), 0, s, EV, z, n, I, a, b);
}

}  // namespace amm
