// amm_device.hip -- HIP kernels for gfx950 and the C ABI of libamm.
//
// Kernels (one thread = one sample, 128-thread blocks = 2 wave64; the Monte
// Carlo kernels are in amm_kernels.h):
//   k_sample     Philox4x32-10 or MRG32k3a -> density sample (Sec. III.A) -> z, g = x 2^j
//   k_eval       forest-subtracted integrands of all insertions at given z
//   k_integrate / k_integrate_fused
//                sample + evaluate + round-off check (eq. interval_accept) +
//                per-chunk deterministic partial sums; flagged samples are
//                compacted per chunk in sample order
//   k_flag_scan, k_dd_points, k_dd_reduce
//                double-double recompute of the flagged samples of a group
//   k_reduce_seg fixed-order sum of chunk partials into graph accumulators
// Sums are reduced in a fixed tree keyed by chunk, so results do not depend on
// the grid size.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <algorithm>
#include <thread>
#include <type_traits>
#include <string>
#include <vector>

#include "amm_ctx.h"
#include "amm_kernels.h"
#include "amm_gen.h"

using namespace amm;

namespace amm {
thread_local std::string g_err;
int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}
}  // namespace amm

amm_ctx::~amm_ctx() {
    hipSetDevice(device);
    if (run_ev) hipEventSynchronize(run_ev), hipEventDestroy(run_ev);
    for (int i = 0; i < NSIDE; ++i) {
        if (side[i]) hipStreamSynchronize(side[i]), hipStreamDestroy(side[i]);
        if (join_ev[i]) hipEventDestroy(join_ev[i]);
    }
    if (fork_ev) hipEventDestroy(fork_ev);
    for (auto &s : slots) {
        hipFree(s.d_levels); hipFree(s.d_terms); hipFree(s.d_ops); hipFree(s.d_monos); hipFree(s.d_ranges);
            hipFree(s.d_gwords); hipFree(s.d_granges);
        hipFree(s.d_deg1); hipFree(s.d_deg3); hipFree(s.d_W1); hipFree(s.d_logdeg1);
        hipFree(s.d_ptheta); hipFree(s.d_pilotW);
    }
    hipFree(d_acc);
    hipFree(own.part); hipFree(own.flag); hipFree(own.nflag); hipFree(own.foff); hipFree(own.ydd); hipFree(own.work);
    hipFree(d_segs); hipFree(d_base); hipFree(d_mrg_tab);
    if (seg_ev) hipEventSynchronize(seg_ev), hipEventDestroy(seg_ev);
    if (static_seg_ev) hipEventSynchronize(static_seg_ev), hipEventDestroy(static_seg_ev);
    delete[] (SegDev *)static_stage;
    if (cap_stream) hipStreamSynchronize(cap_stream), hipStreamDestroy(cap_stream);
    hipHostFree(h_segs);
    mlp_free(mlp);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(BLOCK) k_sample(DensityDev D, uint32_t uid, uint64_t seed, MrgStream R, uint64_t c0,
                                                  uint64_t n, double *z, double *gx, int32_t *gj, int32_t *path,
                                                  int32_t *comp) {
    uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double u[2 * M], zz[M];
    int pp[M];
    draw_uniforms(seed, uid, R, c0 + i, D.ptheta ? 2 * M : 2 * M - 1, u);
    SampleOut o = sample_point<M>(D, u, zz, pp);
    if (z) for (int j = 0; j < M; ++j) z[i * M + j] = zz[j];
    if (path) for (int j = 0; j < M; ++j) path[i * M + j] = pp[j];
    if (gx) gx[i] = o.gx;
    if (gj) gj[i] = o.gj;
    if (comp) comp[i] = o.comp;
}

// acc[s] += sum over chunks of part[chunk][s]: block s, thread t sums chunks
// t, t+256, ... in order, then a fixed tree over the threads.
__global__ void __launch_bounds__(256) k_reduce(const double *part, int nchunks, double *acc) {
    __shared__ double sh[256];
    const int s = blockIdx.x, t = threadIdx.x;
    double v = 0.0;
    for (int c = t; c < nchunks; c += 256) v += part[(size_t)c * NSTAT_MAX + s];
    sh[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) acc[s] += sh[0];
}

__global__ void k_zero(double *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// MRG32k3a, host side: companion matrices, their powers, stream start states
// (layout in amm_core.h).
// ---------------------------------------------------------------------------
namespace {
struct Mat3 {
    uint64_t a[9];
};
const uint64_t MRG_MOD[2] = {MRG_M1, MRG_M2};
Mat3 mat_mul(const Mat3 &x, const Mat3 &y, uint64_t m) {
    Mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            uint64_t v = 0;
            for (int k = 0; k < 3; ++k) v = (v + x.a[3 * i + k] * y.a[3 * k + j] % m) % m;
            r.a[3 * i + j] = v;
        }
    return r;
}
Mat3 mat_id() { return Mat3{{1, 0, 0, 0, 1, 0, 0, 0, 1}}; }
Mat3 mrg_companion(int comp) {
    if (comp == 0) return Mat3{{0, 1, 0, 0, 0, 1, MRG_A13N, MRG_A12, 0}};
    return Mat3{{0, 1, 0, 0, 0, 1, MRG_A23N, 0, MRG_A21}};
}
Mat3 mat_pow2(Mat3 a, int e, uint64_t m) {         // a^(2^e)
    for (int i = 0; i < e; ++i) a = mat_mul(a, a, m);
    return a;
}
}  // namespace

// Jump table (device) and the graph spacing power A^(2^100), once per context.
static int mrg_init(amm_ctx *c) {
    std::vector<uint32_t> tab(MRG_TABLE_WORDS, 0u);
    for (int comp = 0; comp < 2; ++comp) {
        const uint64_t m = MRG_MOD[comp];
        Mat3 w = mat_pow2(mrg_companion(comp), MRG_SAMPLE_SHIFT, m);       // A^(2^7)
        for (int k = 0; k < MRG_WINDOWS; ++k) {
            Mat3 p = mat_id();
            for (int d = 0; d < 16; ++d) {
                for (int q = 0; q < 9; ++q) tab[((comp * MRG_WINDOWS + k) * 16 + d) * 9 + q] = (uint32_t)p.a[q];
                p = mat_mul(p, w, m);                                      // A^((d + 1) 2^(7 + 4k))
            }
            w = mat_pow2(w, 4, m);
        }
        Mat3 j = mat_pow2(mrg_companion(comp), 100, m);
        for (int q = 0; q < 9; ++q) c->mrg_j100[comp][q] = j.a[q];
    }
    HIPCHK(hipMalloc((void **)&c->d_mrg_tab, tab.size() * sizeof(uint32_t)));
    HIPCHK(hipMemcpy(c->d_mrg_tab, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    return AMM_OK;
}

// Stream of graph uid: start state (A^(2^100))^uid s0(seed), s0 from the
// seed's 32-bit halves.
static MrgStream mrg_stream(const amm_ctx *c, uint64_t seed, uint32_t uid) {
    MrgStream R;
    R.tab = c->d_mrg_tab;
    R.on = c->generator == 1;
    const uint64_t half[2] = {seed & 0xffffffffull, (seed >> 32) & 0xffffffffull};
    for (int comp = 0; comp < 2; ++comp) {
        const uint64_t m = MRG_MOD[comp];
        Mat3 base, p = mat_id();
        for (int q = 0; q < 9; ++q) base.a[q] = c->mrg_j100[comp][q];
        for (uint32_t e = uid; e; e >>= 1) {
            if (e & 1u) p = mat_mul(p, base, m);
            base = mat_mul(base, base, m);
        }
        const uint64_t s0[3] = {1 + half[comp] % (m - 1), 12345, 12345};
        for (int i = 0; i < 3; ++i) {
            uint64_t v = 0;
            for (int k = 0; k < 3; ++k) v = (v + p.a[3 * i + k] * s0[k] % m) % m;
            R.s[3 * comp + i] = (uint32_t)v;
        }
    }
    return R;
}

// Sample indices of an MRG32k3a stream must stay below 2^44.
static bool mrg_range_ok(const amm_ctx *c, uint64_t end) {
    return c->generator != 1 || end <= (1ull << (4 * MRG_WINDOWS));
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
namespace {

template <typename X>
int upload(X **dst, const X *src, size_t count) {
    if (count == 0) count = 1;
    HIPCHK(hipMalloc((void **)dst, count * sizeof(X)));
    if (src) HIPCHK(hipMemcpy(*dst, src, count * sizeof(X), hipMemcpyHostToDevice));
    return AMM_OK;
}

// The FP64 interpreter's group stream of a plan (layout in amm_core.h): every
// range of the monomial table cut into records of four consecutive monomials,
// padded with the constant-1 slot (short monomials) and zero coefficients
// (the range's last record).  Identical ranges share their records.
static void group_stream(const PlanHost &P, std::vector<uint32_t> &words, std::vector<int2> &granges) {
    const uint32_t one = (uint32_t)amm_nvars(P.n);
    std::map<std::pair<int, int>, int2> done;
    words.clear();
    granges.resize(P.ranges.size());
    for (size_t ri = 0; ri < P.ranges.size(); ++ri) {
        const auto r = P.ranges[ri];
        auto it = done.find(r);
        if (it != done.end()) { granges[ri] = it->second; continue; }
        const int2 g = make_int2((int)words.size(), (r.second - r.first + 3) / 4);
        for (int m = r.first; m < r.second; m += 4) {
            int K = 0;
            for (int q = 0; q < 4 && m + q < r.second; ++q) K = std::max(K, (int)P.monos[m + q].nv);
            words.push_back((uint32_t)K);
            words.push_back(0u);
            for (int q = 0; q < 4; ++q) {
                const double c = m + q < r.second ? P.monos[m + q].coef : 0.0;
                uint64_t b;
                std::memcpy(&b, &c, 8);
                words.push_back((uint32_t)b);
                words.push_back((uint32_t)(b >> 32));
            }
            for (int i = 0; i < K; ++i)
                for (int q = 0; q < 4; ++q) {
                    const bool has = m + q < r.second && i < (int)P.monos[m + q].nv;
                    words.push_back(has ? (uint32_t)P.monos[m + q].v[i] : one);
                }
        }
        granges[ri] = g;
        done.emplace(r, g);
    }
    if (words.empty()) words.push_back(0u);
}

int grid_for(uint64_t n) { return (int)((n + BLOCK - 1) / BLOCK); }

template <int N>
void launch_eval(const GraphSlot &gs, int g, const double *z, uint64_t n, double *I, double *a, double *b, int prec,
                 hipStream_t s, bool use_gen) {
    InterpEval EV{gs.plan_dev()};
    if (prec == 1) {
        launch_eval_ev<N, InterpEval, dd>(EV, z, n, I, a, b, s);
        return;
    }
    if (prec == 2) {
        if constexpr (N <= 4) launch_eval_ev<N, InterpEval, iv>(EV, z, n, I, a, b, s);
        return;
    }
    if (use_gen && gen_launch(N, g)) {
        gen_launch(N, g)(GEN_EVAL, nullptr, nullptr, 0, z, n, I, a, b, s, nullptr, nullptr, nullptr);
        return;
    }
    launch_eval_ev<N, InterpEval, ea>(EV, z, n, I, a, b, s);
}

constexpr int DD_GRID = 4096;                 // blocks of the per-point DD recompute (grid-stride)

// FP64 pass of one segment into the group buffers at its chunk offset.
template <int N>
void launch_seg_fp64(const GraphSlot &gs, const SegDev &S, int grid, const Workspace &ws, hipStream_t s,
                     bool use_gen) {
    double *part = ws.part + (size_t)S.gchunk * NSTAT_MAX;
    uint32_t *flag = ws.flag + (size_t)S.gchunk * CHUNK;
    int32_t *nflag = ws.nflag + S.gchunk;
    if (use_gen && gen_launch(N, S.g))
        gen_launch(N, S.g)(GEN_RUN, &S.D, &S.A, grid, nullptr, 0, nullptr, nullptr, nullptr, s, part, flag, nflag);
    else
        launch_fp64_ev<N>(InterpEval{gs.plan_dev()}, S.D, S.A, grid, part, flag, nflag, s);
}

// DD pass and reduction of one group (segments [k0, k1) of the staged table).
template <int N>
void launch_group_tail(amm_ctx *c, const Workspace &ws, const SegDev *d_segs, int nseg, int nch, int grid_red,
                       hipStream_t s, amm_ctx::Ev *ev) {
    launch_dd_group<N>(d_segs, nseg, nch, DD_GRID, grid_red, ws.part, ws.flag, ws.nflag, ws.foff, ws.ydd,
                       ws.ydd_cap(), s);
    if (ev) hipEventRecord(ev->c, s);
    hipLaunchKernelGGL(k_reduce_seg, dim3(NSTAT_MAX, nseg), dim3(256), 0, s, d_segs, ws.part, c->d_acc);
}

// The context's own workspace (groups of MAX_GROUP_CHUNKS chunks), allocated
// on first use; the double-double region grows to ne insertions.
int ensure_own_ws(amm_ctx *c, int ne) {
    Workspace &w = c->own;
    if (!w.part) {
        w.max_chunks = MAX_GROUP_CHUNKS;
        HIPCHK(hipMalloc((void **)&w.part, (size_t)MAX_GROUP_CHUNKS * NSTAT_MAX * sizeof(double)));
        HIPCHK(hipMalloc((void **)&w.flag, (size_t)MAX_GROUP_CHUNKS * CHUNK * sizeof(uint32_t)));
        HIPCHK(hipMalloc((void **)&w.nflag, (size_t)MAX_GROUP_CHUNKS * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&w.foff, (size_t)(MAX_GROUP_CHUNKS + 1) * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&w.work, sizeof(int)));
    }
    if (w.ydd_ne < ne) {
        HIPCHK(hipFree(w.ydd));
        w.ydd = nullptr;
        w.ydd_ne = 0;
        HIPCHK(hipMalloc((void **)&w.ydd, (size_t)ne * MAX_GROUP_CHUNKS * CHUNK * sizeof(double)));
        w.ydd_ne = ne;
    }
    return AMM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of amm_integrate_static: the workspace for groups of
// STATIC_GROUP_CHUNKS chunks (any loop order), then a segment table of
// STATIC_MAX_SEGS entries.  One copy per device, held while the process
// lives; host code reaches it only through the address hipGetSymbolAddress
// returns for the device (static_setup).
// ---------------------------------------------------------------------------
constexpr int STATIC_GROUP_CHUNKS = 256;      // 262144 samples per group
constexpr int STATIC_MAX_SEGS = 1024;
constexpr size_t STATIC_WS_BYTES = ws_bytes(STATIC_GROUP_CHUNKS, MAXNE);
constexpr size_t STATIC_BYTES = STATIC_WS_BYTES + ws_align(STATIC_MAX_SEGS * sizeof(SegDev));
static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES] = {};

// Once per device (with the device current): the device address of `scratch`.
// Also the context's staging table and event of the static path.
int static_setup(amm_ctx *c) {
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (c->device >= STATIC_MAX_DEVICES) return fail(AMM_E_ARG, "amm_create: device index beyond 63");
        if (!g_static_ptr[c->device]) {
            void *ptr = nullptr;
            HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(AMM_E_HIP, "amm_create: no device address for the static scratch");
            g_static_ptr[c->device] = ptr;
        }
        c->static_base = g_static_ptr[c->device];
    }
    HIPCHK(hipEventCreateWithFlags(&c->static_seg_ev, hipEventDisableTiming));
    c->static_stage = new SegDev[STATIC_MAX_SEGS];
    return AMM_OK;
}

void prof_collect(amm_ctx *c) {
    for (auto &e : c->evs) {
        hipEventSynchronize(e.d);
        float t1 = 0, t2 = 0, t3 = 0;
        hipEventElapsedTime(&t1, e.a, e.b);
        hipEventElapsedTime(&t2, e.b, e.c);
        hipEventElapsedTime(&t3, e.c, e.d);
        c->prof_ms[0] += t1; c->prof_ms[1] += t2; c->prof_ms[2] += t3;
        c->prof_launch += e.nseg;
        c->prof_samples += e.samples;
        hipEventDestroy(e.a); hipEventDestroy(e.b); hipEventDestroy(e.c); hipEventDestroy(e.d);
    }
    c->evs.clear();
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *amm_last_error(void) { return amm::g_err.c_str(); }

int amm_create(amm_ctx **out, int device) {
    if (!out) return fail(AMM_E_ARG, "amm_create: out is NULL");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(AMM_E_ARG, "amm_create: no such device");
    HIPCHK(hipSetDevice(device));
    std::unique_ptr<amm_ctx> c(new amm_ctx);
    c->device = device;
    HIPCHK(hipEventCreateWithFlags(&c->seg_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->run_ev, hipEventDisableTiming));
    HIPCHK(hipMalloc((void **)&c->d_base, sizeof(uint64_t)));
    if (int rc = static_setup(c.get())) return rc;
    for (int i = 0; i < amm_ctx::NSIDE; ++i) {
        HIPCHK(hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    if (int rc = mrg_init(c.get())) return rc;
    *out = c.release();
    return AMM_OK;
}

void amm_destroy(amm_ctx *ctx) { delete ctx; }

int amm_enumerate(amm_ctx *c, int loops, int *n_se, int *n_vertex, int *M) {
    if (!c) return fail(AMM_E_ARG, "amm_enumerate: ctx is NULL");
    if (loops < 1 || loops > MAXN) return fail(AMM_E_ARG, "amm_enumerate: loops must be 1..5");
    if (c->loops != loops) {
        hipSetDevice(c->device);
        for (auto &s : c->slots) {
            hipFree(s.d_levels); hipFree(s.d_terms); hipFree(s.d_ops); hipFree(s.d_monos); hipFree(s.d_ranges);
            hipFree(s.d_gwords); hipFree(s.d_granges);
            hipFree(s.d_deg1); hipFree(s.d_deg3); hipFree(s.d_W1); hipFree(s.d_logdeg1);
            hipFree(s.d_ptheta); hipFree(s.d_pilotW);
        }
        c->slots.clear();
        mlp_free_rows(c->mlp);               // feature rows belong to the old graph set
        c->graphs = enumerate_se(loops);
        c->loops = loops;
        c->slots.resize(c->graphs.size());
        hipFree(c->d_acc);
        c->d_acc = nullptr;
        HIPCHK(hipMalloc((void **)&c->d_acc, c->graphs.size() * NSTAT_MAX * sizeof(double)));
        HIPCHK(hipMemset(c->d_acc, 0, c->graphs.size() * NSTAT_MAX * sizeof(double)));
    }
    if (n_se) *n_se = (int)c->graphs.size();
    if (n_vertex) *n_vertex = (int)c->graphs.size() * (2 * loops - 1);
    if (M) *M = 3 * loops - 1;
    return AMM_OK;
}

int amm_graph_desc(const amm_ctx *c, int g, int *chords, int *classes) {
    if (!c || g < 0 || g >= (int)c->graphs.size()) return fail(AMM_E_ARG, "amm_graph_desc: bad graph");
    const SEGraph &G = c->graphs[g];
    if (chords)
        for (size_t i = 0; i < G.chords.size(); ++i) { chords[2 * i] = G.chords[i].first; chords[2 * i + 1] = G.chords[i].second; }
    if (classes)
        for (int e = 0; e < 2 * G.n - 1; ++e) {
            auto k = vertex_class(G, e);
            for (int q = 0; q < 3; ++q) classes[3 * e + q] = k[q];
        }
    return AMM_OK;
}

int amm_build_tables(amm_ctx *c, const amm_density_params *params, int gb, int ge) {
    if (!c || c->loops == 0) return fail(AMM_E_ARG, "amm_build_tables: call amm_enumerate first");
    if (gb < 0 || ge > (int)c->graphs.size() || gb >= ge) return fail(AMM_E_ARG, "amm_build_tables: bad graph range");
    const bool plans = c->build_plans != 0;
    amm_density_params p;
    if (params) p = *params;
    else p = amm_density_params{0.256, 0.839, 0.786, 0.2, 0.0, 0.2, {((1.0 - 0.03) - 0.01) - 0.06, 0.03, 0.01, 0.06}, 0.75, 1.0};
    HIPCHK(hipSetDevice(c->device));
    // host plans and densities: independent per graph, built on a thread pool
    {
        std::atomic<int> next(gb);
        std::vector<std::string> errs(ge - gb);
        const unsigned hw = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
        unsigned nt = std::min<unsigned>(hw, (unsigned)(ge - gb));
        // few graphs: each one's distinct level polynomials on several threads
        const int inner = (int)std::max(1u, hw / nt);
        auto work = [&]() {
            for (int g = next++; g < ge; g = next++) {
                try {
                    build_density(c->graphs[g], p, c->slots[g].dens);
                    if (plans) build_plan(c->graphs[g], c->slots[g].plan, inner);
                    else c->slots[g].plan = PlanHost();
                } catch (const std::exception &ex) {
                    errs[g - gb] = ex.what();
                }
            }
        };
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work);
        work();
        for (auto &th : pool) th.join();
        for (auto &e : errs)
            if (!e.empty()) return fail(AMM_E_NUMERIC, std::string("amm_build_tables: ") + e);
    }
    for (int g = gb; g < ge; ++g) {
        GraphSlot &s = c->slots[g];
        const SEGraph &G = c->graphs[g];
        s.n = G.n; s.M = 3 * G.n - 1; s.ne = 2 * G.n - 1;
        s.uid = (uint32_t)((G.n << 20) | g);
        if (g < (int)c->mlp.rows.size() && c->mlp.rows[g].built) {   // features depend on the density tables
            MlpRows &R = c->mlp.rows[g];
            hipFree(R.d_feat); hipFree(R.d_s); hipFree(R.d_j); hipFree(R.d_grp); hipFree(R.d_goff);
            R = MlpRows();
        }
        // classes
        std::vector<std::array<int, 3>> ucls;
        for (int e = 0; e < s.ne; ++e) {
            auto k = vertex_class(G, e);
            int id = -1;
            for (size_t q = 0; q < ucls.size(); ++q) if (ucls[q] == k) id = (int)q;
            if (id < 0) { id = (int)ucls.size(); ucls.push_back(k); }
            s.cls_of[e] = id;
        }
        s.ncls = (int)ucls.size();
        for (int q = 0; q < s.ncls; ++q) for (int w = 0; w < 3; ++w) s.cls_kmm[q][w] = ucls[q][w];
        hipFree(s.d_levels); hipFree(s.d_terms); hipFree(s.d_ops); hipFree(s.d_monos); hipFree(s.d_ranges);
            hipFree(s.d_gwords); hipFree(s.d_granges);
        hipFree(s.d_deg1); hipFree(s.d_deg3); hipFree(s.d_W1); hipFree(s.d_logdeg1);
        std::vector<int2> rg(s.plan.ranges.size());
        for (size_t i = 0; i < rg.size(); ++i) rg[i] = make_int2(s.plan.ranges[i].first, s.plan.ranges[i].second);
        int rc;
        s.d_levels = nullptr; s.d_terms = nullptr; s.d_ops = nullptr; s.d_monos = nullptr; s.d_ranges = nullptr;
        s.d_gwords = nullptr; s.d_granges = nullptr; s.ngwords = 0;
        if (plans) {
            std::vector<uint32_t> gw;
            std::vector<int2> gr;
            group_stream(s.plan, gw, gr);
            s.ngwords = (int)gw.size();
            if ((rc = upload(&s.d_gwords, gw.data(), gw.size()))) return rc;
            if ((rc = upload(&s.d_granges, gr.data(), gr.size()))) return rc;
            if ((rc = upload(&s.d_levels, s.plan.levels.data(), s.plan.levels.size()))) return rc;
            if ((rc = upload(&s.d_terms, s.plan.terms.data(), s.plan.terms.size()))) return rc;
            if ((rc = upload(&s.d_ops, s.plan.ops.data(), s.plan.ops.size()))) return rc;
            if ((rc = upload(&s.d_monos, s.plan.monos.data(), s.plan.monos.size()))) return rc;
            if ((rc = upload(&s.d_ranges, rg.data(), rg.size()))) return rc;
        }
        if ((rc = upload(&s.d_deg1, s.dens.deg1.data(), s.dens.deg1.size()))) return rc;
        if ((rc = upload(&s.d_deg3, s.dens.deg3.data(), s.dens.deg3.size()))) return rc;
        if ((rc = upload(&s.d_W1, s.dens.W1.data(), s.dens.W1.size()))) return rc;
        if ((rc = upload(&s.d_logdeg1, s.dens.logdeg1.data(), s.dens.logdeg1.size()))) return rc;
        s.acc.assign(NSTAT_MAX, 0.0);
        s.built = true;
        s.has_plan = plans;
    }
    return AMM_OK;
}

int amm_plan_stats(const amm_ctx *c, int g, amm_plan_info *out) {
    if (!c || !out || g < 0 || g >= (int)c->slots.size()) return fail(AMM_E_ARG, "amm_plan_stats: bad argument");
    const GraphSlot &s = c->slots[g];
    if (!s.has_plan) return fail(AMM_E_NOTBUILT, "amm_plan_stats: integrand tables not built");
    out->n_insertions = s.ne;
    out->n_terms = (int)s.plan.terms.size();
    out->n_terms_expanded = s.plan.n_terms_expanded;
    out->n_level_evals = (int)s.plan.ops.size();
    out->n_monomials = s.plan.n_monos_per_sample;
    out->flops_per_sample = s.plan.flops_per_sample;
    return AMM_OK;
}

int amm_sample(amm_ctx *c, int g, uint64_t seed, uint64_t c0, uint64_t n, int learned, double *z, double *gx,
               int32_t *gj, int32_t *path, int32_t *comp, void *stream) {
    if (!c || g < 0 || g >= (int)c->slots.size()) return fail(AMM_E_ARG, "amm_sample: bad graph");
    GraphSlot &s = c->slots[g];
    if (!s.built) return fail(AMM_E_NOTBUILT, "amm_sample: tables not built");
    if (n == 0) return AMM_OK;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    if (learned && !s.d_ptheta) return fail(AMM_E_ARG, "amm_sample: no sector table for the learned mixture");
    DensityDev D = s.dens_dev(learned != 0);
    if (c0 + n < c0 || !mrg_range_ok(c, c0 + n)) return fail(AMM_E_ARG, "amm_sample: MRG32k3a sample indices >= 2^44");
    const MrgStream R = mrg_stream(c, seed, s.uid);
    dim3 gr(grid_for(n)), bl(BLOCK);
    switch (s.M) {
        case 2: hipLaunchKernelGGL(k_sample<2>, gr, bl, 0, st, D, s.uid, seed, R, c0, n, z, gx, gj, path, comp); break;
        case 5: hipLaunchKernelGGL(k_sample<5>, gr, bl, 0, st, D, s.uid, seed, R, c0, n, z, gx, gj, path, comp); break;
        case 8: hipLaunchKernelGGL(k_sample<8>, gr, bl, 0, st, D, s.uid, seed, R, c0, n, z, gx, gj, path, comp); break;
        case 11: hipLaunchKernelGGL(k_sample<11>, gr, bl, 0, st, D, s.uid, seed, R, c0, n, z, gx, gj, path, comp); break;
        case 14: hipLaunchKernelGGL(k_sample<14>, gr, bl, 0, st, D, s.uid, seed, R, c0, n, z, gx, gj, path, comp); break;
        default: return fail(AMM_E_ARG, "amm_sample: unsupported M");
    }
    HIPCHK(hipGetLastError());
    c->last_stream = st;
    return AMM_OK;
}

int amm_eval(amm_ctx *c, int g, const double *z, uint64_t n, double *I, double *absI, double *bound, int precision,
             void *stream) {
    if (!c || g < 0 || g >= (int)c->slots.size()) return fail(AMM_E_ARG, "amm_eval: bad argument");
    GraphSlot &s = c->slots[g];
    if (!s.has_plan) return fail(AMM_E_NOTBUILT, "amm_eval: integrand tables not built");
    if (n == 0) return AMM_OK;
    if (!z) return fail(AMM_E_ARG, "amm_eval: z is NULL");
    if (precision < 0 || precision > 2) return fail(AMM_E_ARG, "amm_eval: precision 0, 1 or 2");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    PlanDev P = s.plan_dev();
    switch (s.n) {
        case 1: launch_eval<1>(s, g, z, n, I, absI, bound, precision, st, c->use_gen); break;
        case 2: launch_eval<2>(s, g, z, n, I, absI, bound, precision, st, c->use_gen); break;
        case 3: launch_eval<3>(s, g, z, n, I, absI, bound, precision, st, c->use_gen); break;
        case 4: launch_eval<4>(s, g, z, n, I, absI, bound, precision, st, c->use_gen); break;
        case 5:
            if (precision == 2) return fail(AMM_E_ARG, "amm_eval: interval evaluation is built for 1-4 loops");
            launch_eval<5>(s, g, z, n, I, absI, bound, precision, st, c->use_gen);
            break;
        default: return fail(AMM_E_ARG, "amm_eval: unsupported loop order");
    }
    HIPCHK(hipGetLastError());
    c->last_stream = st;
    return AMM_OK;
}

// Checks a run's parameters against the context.
static int check_run(amm_ctx *c, const amm_run_params *r) {
    if (!c || !r) return fail(AMM_E_ARG, "amm_integrate: bad argument");
    if (r->graph_begin < 0 || r->graph_end > (int)c->slots.size() || r->graph_begin >= r->graph_end)
        return fail(AMM_E_ARG, "amm_integrate: bad graph range");
    for (int g = r->graph_begin; g < r->graph_end; ++g)
        if (!c->slots[g].has_plan) return fail(AMM_E_NOTBUILT, "amm_integrate: integrand tables not built");
    if (c->loops < 1 || c->loops > 5) return fail(AMM_E_ARG, "amm_integrate: unsupported loop order");
    if (c->loops == 1 && r->force_flag)
        return fail(AMM_E_ARG, "amm_integrate: double-double recompute is disabled at 1 loop (force_flag)");
    if (r->blocks_per_cu < 0 || r->blocks_per_cu > 64) return fail(AMM_E_ARG, "amm_integrate: blocks_per_cu 0..64");
    return AMM_OK;
}

// Number of segments a run is cut into with groups of max_chunks chunks.
static size_t count_segments(const amm_run_params *r, int max_chunks, const uint64_t *n_per_graph_arr) {
    size_t n = 0;
    for (int g = r->graph_begin; g < r->graph_end; ++g) {
        const uint64_t ng = n_per_graph_arr ? n_per_graph_arr[g - r->graph_begin] : r->n_per_graph;
        const uint64_t nch = (ng + CHUNK - 1) / CHUNK;
        n += (size_t)((nch + max_chunks - 1) / max_chunks);
    }
    return n;
}

// Segments: each graph's chunk range cut into pieces of at most max_chunks
// chunks; groups: consecutive segments of distinct graphs, at most
// max_chunks chunks in all.  Writes the segments to out (room for cap) and the
// first segment of every group, then the segment count, to gbeg (room for
// cap + 1).  Allocates nothing.
static int plan_segments(amm_ctx *c, const amm_run_params *r, const uint64_t *base_dev, int max_chunks,
                         const uint64_t *c0_per_graph, const uint64_t *n_per_graph_arr, SegDev *out, size_t cap,
                         int *gbeg, int *nseg_out, int *ngroups_out) {
    // graph order inside groups: heaviest plan first (cost grouping) or natural
    int order[1024];
    const int G = r->graph_end - r->graph_begin;
    if (G > 1024) return fail(AMM_E_TOOBIG, "amm_integrate: more than 1024 graphs in one run");
    for (int k = 0; k < G; ++k) order[k] = r->graph_begin + k;
    if (c->order_by_cost)
        std::sort(order, order + G, [&](int a, int b) {
            const double fa = c->slots[a].plan.flops_per_sample, fb = c->slots[b].plan.flops_per_sample;
            return fa > fb || (fa == fb && a < b);
        });
    size_t nseg = 0;
    int ngroups = 0;
    int gch = max_chunks, last_g = -1;
    for (int k = 0; k < G; ++k) {
        const int g = order[k];
        GraphSlot &s = c->slots[g];
        bool learned = r->sampler == 1 && s.d_ptheta != nullptr;
        const int kk = g - r->graph_begin;
        const uint64_t c0 = c0_per_graph ? c0_per_graph[kk] : r->counter0;
        const uint64_t ng = n_per_graph_arr ? n_per_graph_arr[kk] : r->n_per_graph;
        const uint64_t nchunks_total = (ng + CHUNK - 1) / CHUNK;
        if (c0 + ng < c0 || !mrg_range_ok(c, c0 + ng))
            return fail(AMM_E_ARG, "amm_integrate: MRG32k3a sample indices >= 2^44");
        for (uint64_t ch0 = 0; ch0 < nchunks_total; ch0 += max_chunks) {
            int nch = (int)std::min<uint64_t>(max_chunks, nchunks_total - ch0);
            if (nseg >= cap) return fail(AMM_E_TOOBIG, "amm_integrate: run needs more segments than the table holds");
            if (gch + nch > max_chunks || last_g == g) {
                gbeg[ngroups++] = (int)nseg;
                gch = 0;
            }
            SegDev &S = out[nseg];
            std::memset(&S, 0, sizeof(S));
            S.A.seed = r->seed;
            S.A.begin = c0;
            S.A.end = c0 + ng;
            S.A.uid = s.uid;
            S.A.chunk0 = (int)ch0;
            S.A.nchunks = nch;
            S.A.ncls = s.ncls;
            for (int e = 0; e < MAXNE; ++e) S.A.cls_of[e] = e < s.ne ? s.cls_of[e] : 0;
            S.A.learned = learned ? 1 : 0;
            S.A.base_dev = base_dev;
            S.A.mrg = mrg_stream(c, r->seed, s.uid);
            if (r->force_flag) S.A.tau = -1.0;
            else if (r->accept_tau) S.A.tau = r->accept_tau[g - r->graph_begin];
            else S.A.tau = INFINITY;
            S.P = s.plan_dev();
            S.D = s.dens_dev(learned);
            S.g = g;
            S.nst = s.nstat();
            S.gchunk = gch;
            ++nseg;
            gch += nch;
            last_g = g;
        }
    }
    gbeg[ngroups] = (int)nseg;
    *nseg_out = (int)nseg;
    *ngroups_out = ngroups;
    return AMM_OK;
}

// Validates a run, prepares the group buffers and stages the segment table of
// the run on `st` (base_dev: optional device word added to every sample index).
static int prepare_run(amm_ctx *c, const amm_run_params *r, hipStream_t st, const uint64_t *base_dev,
                       std::vector<SegDev> &segs, std::vector<int> &group_begin,
                       const uint64_t *c0_per_graph = nullptr, const uint64_t *n_per_graph_arr = nullptr) {
    if (int rc = check_run(c, r)) return rc;
    HIPCHK(hipSetDevice(c->device));
    const int ne_ctx = 2 * c->loops - 1;
    if (!c->use_user_ws)
        if (int rc = ensure_own_ws(c, ne_ctx)) return rc;
    const Workspace &ws = c->ws();
    const size_t nmax = count_segments(r, ws.max_chunks, n_per_graph_arr);
    segs.resize(nmax);
    group_begin.resize(nmax + 1);
    int nseg = 0, ngroups = 0;
    if (int rc = plan_segments(c, r, base_dev, ws.max_chunks, c0_per_graph, n_per_graph_arr, segs.data(), nmax,
                               group_begin.data(), &nseg, &ngroups))
        return rc;
    segs.resize(nseg);
    group_begin.resize(ngroups + 1);
    // The segment table and the workspace are shared by the context's runs: a
    // run enqueued on another stream than the previous one waits for that
    // run's last kernel before it restages or overwrites them.
    HIPCHK(hipStreamWaitEvent(st, c->run_ev, 0));
    // stage the table: wait until the previous call's copy has been consumed
    HIPCHK(hipEventSynchronize(c->seg_ev));
    if (segs.size() > c->seg_cap) {
        HIPCHK(hipFree(c->d_segs));
        HIPCHK(hipHostFree(c->h_segs));
        c->d_segs = c->h_segs = nullptr;
        c->seg_cap = 0;
        size_t cap = std::max<size_t>(segs.size(), 256);
        HIPCHK(hipMalloc(&c->d_segs, cap * sizeof(SegDev)));
        HIPCHK(hipHostMalloc(&c->h_segs, cap * sizeof(SegDev)));
        c->seg_cap = cap;
    }
    std::memcpy(c->h_segs, segs.data(), segs.size() * sizeof(SegDev));
    HIPCHK(hipMemcpyAsync(c->d_segs, c->h_segs, segs.size() * sizeof(SegDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(c->seg_ev, st));
    return AMM_OK;
}

// Whether a group's FP64 pass runs as one persistent interpreter launch.
static bool group_fused(const amm_ctx *c, const SegDev *segs, int k0, int k1) {
    if (!c->use_fused) return false;
    for (int k = k0; k < k1; ++k)
        if (c->use_gen && gen_launch(c->loops, segs[k].g)) return false;
    return true;
}

// Enqueues the kernels of every group of a prepared run on `st` (also used
// under stream capture; then `prof` must be false).  segs: the host copy of the
// staged table d_segs; group_begin: ngroups + 1 segment indices.
static void enqueue_run(amm_ctx *c, const amm_run_params *r, hipStream_t st, const SegDev *segs,
                        const int *group_begin, int ngroups, const SegDev *d_segs, const Workspace &ws, bool prof) {
    int dev_cus = 256;
    hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    const int bpc = r->blocks_per_cu > 0 ? r->blocks_per_cu : (c->blocks_per_cu > 0 ? c->blocks_per_cu : 8);
    const int grid_target = bpc * dev_cus;
    for (int q = 0; q < ngroups; ++q) {
        const int k0 = group_begin[q], k1 = group_begin[q + 1];
        const int nch = segs[k1 - 1].gchunk + segs[k1 - 1].A.nchunks;
        amm_ctx::Ev ev, *evp = nullptr;
        if (prof) {
            hipEventCreate(&ev.a); hipEventCreate(&ev.b); hipEventCreate(&ev.c); hipEventCreate(&ev.d);
            ev.samples = 0;
            ev.nseg = k1 - k0;
            for (int k = k0; k < k1; ++k) {
                uint64_t lo = (uint64_t)segs[k].A.chunk0 * CHUNK;
                uint64_t hi = std::min<uint64_t>(lo + (uint64_t)segs[k].A.nchunks * CHUNK,
                                                 segs[k].A.end - segs[k].A.begin);
                ev.samples += (int64_t)(hi - lo);
            }
            evp = &ev;
            hipEventRecord(ev.a, st);
        }
        if (group_fused(c, segs, k0, k1)) {
            const int grid = std::min(nch, grid_target);
            hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, ws.work, 0);
            switch (c->loops) {
                case 1: hipLaunchKernelGGL(k_integrate_fused<1>, dim3(grid), dim3(InterpEval::kBlock), 0, st, d_segs + k0, k1 - k0, nch, ws.work, ws.part, ws.flag, ws.nflag); break;
                case 2: hipLaunchKernelGGL(k_integrate_fused<2>, dim3(grid), dim3(InterpEval::kBlock), 0, st, d_segs + k0, k1 - k0, nch, ws.work, ws.part, ws.flag, ws.nflag); break;
                case 3: hipLaunchKernelGGL(k_integrate_fused<3>, dim3(grid), dim3(InterpEval::kBlock), 0, st, d_segs + k0, k1 - k0, nch, ws.work, ws.part, ws.flag, ws.nflag); break;
                case 4: hipLaunchKernelGGL(k_integrate_fused<4>, dim3(grid), dim3(InterpEval::kBlock), 0, st, d_segs + k0, k1 - k0, nch, ws.work, ws.part, ws.flag, ws.nflag); break;
                case 5: hipLaunchKernelGGL(k_integrate_fused<5>, dim3(grid), dim3(InterpEval::kBlock), 0, st, d_segs + k0, k1 - k0, nch, ws.work, ws.part, ws.flag, ws.nflag); break;
            }
        } else {
            // one launch per segment; they write disjoint chunks, so they run
            // concurrently on the side streams (forked from and joined to st)
            const int ns = std::min(k1 - k0, (int)amm_ctx::NSIDE);
            if (ns > 1) {
                hipEventRecord(c->fork_ev, st);
                for (int i = 0; i < ns; ++i) hipStreamWaitEvent(c->side[i], c->fork_ev, 0);
            }
            double load[amm_ctx::NSIDE] = {};
            for (int k = k0; k < k1; ++k) {
                const int grid = std::min(segs[k].A.nchunks, grid_target);
                int li = 0;                   // least-loaded stream (plan cost of its launches so far)
                for (int i = 1; i < ns; ++i)
                    if (load[i] < load[li]) li = i;
                load[li] += c->slots[segs[k].g].plan.flops_per_sample * (double)segs[k].A.nchunks;
                hipStream_t ls = ns > 1 ? c->side[li] : st;
                switch (c->loops) {
                    case 1: launch_seg_fp64<1>(c->slots[segs[k].g], segs[k], grid, ws, ls, c->use_gen); break;
                    case 2: launch_seg_fp64<2>(c->slots[segs[k].g], segs[k], grid, ws, ls, c->use_gen); break;
                    case 3: launch_seg_fp64<3>(c->slots[segs[k].g], segs[k], grid, ws, ls, c->use_gen); break;
                    case 4: launch_seg_fp64<4>(c->slots[segs[k].g], segs[k], grid, ws, ls, c->use_gen); break;
                    case 5: launch_seg_fp64<5>(c->slots[segs[k].g], segs[k], grid, ws, ls, c->use_gen); break;
                }
            }
            if (ns > 1)
                for (int i = 0; i < ns; ++i) {
                    hipEventRecord(c->join_ev[i], c->side[i]);
                    hipStreamWaitEvent(st, c->join_ev[i], 0);
                }
        }
        if (evp) hipEventRecord(ev.b, st);
        const int grid_red = std::min(nch, grid_target);
        switch (c->loops) {
            case 1: launch_group_tail<1>(c, ws, d_segs + k0, k1 - k0, nch, grid_red, st, evp); break;
            case 2: launch_group_tail<2>(c, ws, d_segs + k0, k1 - k0, nch, grid_red, st, evp); break;
            case 3: launch_group_tail<3>(c, ws, d_segs + k0, k1 - k0, nch, grid_red, st, evp); break;
            case 4: launch_group_tail<4>(c, ws, d_segs + k0, k1 - k0, nch, grid_red, st, evp); break;
            case 5: launch_group_tail<5>(c, ws, d_segs + k0, k1 - k0, nch, grid_red, st, evp); break;
        }
        if (evp) {
            hipEventRecord(ev.d, st);
            c->evs.push_back(ev);
        }
    }
}

static void zero_acc(amm_ctx *c, const amm_run_params *r, hipStream_t st) {
    if (!r->accumulate)
        for (int g = r->graph_begin; g < r->graph_end; ++g)
            hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, c->d_acc + (size_t)g * NSTAT_MAX, NSTAT_MAX);
}

int amm_integrate_static(amm_ctx *c, const amm_run_params *r, void *stream) {
    if (int rc = check_run(c, r)) return rc;
    if (!c->static_base || !c->static_stage) return fail(AMM_E_ARG, "amm_integrate_static: no static scratch");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    if (count_segments(r, STATIC_GROUP_CHUNKS, nullptr) > (size_t)STATIC_MAX_SEGS)
        return fail(AMM_E_TOOBIG, "amm_integrate_static: the run needs more than 1024 segments of 262144 samples "
                                  "(sum over graphs of ceil(n_per_graph / 262144))");
    const Workspace ws = ws_carve(c->static_base, STATIC_GROUP_CHUNKS, MAXNE);
    SegDev *d_segs = (SegDev *)((char *)c->static_base + STATIC_WS_BYTES);
    SegDev *h = (SegDev *)c->static_stage;
    int gbeg[STATIC_MAX_SEGS + 1];
    // the previous static call's staging copy has left the host table
    HIPCHK(hipEventSynchronize(c->static_seg_ev));
    int nseg = 0, ngroups = 0;
    if (int rc = plan_segments(c, r, nullptr, STATIC_GROUP_CHUNKS, nullptr, nullptr, h, STATIC_MAX_SEGS, gbeg, &nseg,
                               &ngroups))
        return rc;
    // after this context's previous run (any stream), which may use the scratch
    HIPCHK(hipStreamWaitEvent(st, c->run_ev, 0));
    HIPCHK(hipMemcpyAsync(d_segs, h, (size_t)nseg * sizeof(SegDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(c->static_seg_ev, st));
    zero_acc(c, r, st);
    enqueue_run(c, r, st, h, gbeg, ngroups, d_segs, ws, false);
    HIPCHK(hipEventRecord(c->run_ev, st));
    HIPCHK(hipGetLastError());
    c->last_stream = st;
    return AMM_OK;
}

size_t amm_workspace_bytes(int chunks_per_group) {
    if (chunks_per_group < 1 || chunks_per_group > MAX_GROUP_CHUNKS) return 0;
    return ws_bytes(chunks_per_group, MAXNE);
}

int amm_set_workspace(amm_ctx *c, void *dev_ptr, size_t bytes) {
    if (!c) return fail(AMM_E_ARG, "amm_set_workspace: ctx is NULL");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipEventSynchronize(c->run_ev));   // no enqueued run still uses the current workspace
    if (!dev_ptr) {
        c->use_user_ws = false;
        c->user = Workspace();
        return AMM_OK;
    }
    if ((uintptr_t)dev_ptr % 256 != 0) return fail(AMM_E_ARG, "amm_set_workspace: pointer not 256-byte aligned");
    int lo = 0, hi = MAX_GROUP_CHUNKS;        // largest chunk count whose workspace fits
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (ws_bytes(mid, MAXNE) <= bytes) lo = mid;
        else hi = mid - 1;
    }
    if (lo < 1) return fail(AMM_E_ARG, "amm_set_workspace: smaller than amm_workspace_bytes(1)");
    c->user = ws_carve(dev_ptr, lo, MAXNE);
    c->use_user_ws = true;
    // the context's own group buffers are not used while a workspace is set
    Workspace &w = c->own;
    HIPCHK(hipFree(w.part)); HIPCHK(hipFree(w.flag)); HIPCHK(hipFree(w.nflag)); HIPCHK(hipFree(w.foff));
    HIPCHK(hipFree(w.ydd)); HIPCHK(hipFree(w.work));
    w = Workspace();
    return AMM_OK;
}

int amm_integrate(amm_ctx *c, const amm_run_params *r, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    std::vector<SegDev> segs;
    std::vector<int> group_begin;
    int rc = prepare_run(c, r, st, nullptr, segs, group_begin);
    if (rc) return rc;
    zero_acc(c, r, st);
    enqueue_run(c, r, st, segs.data(), group_begin.data(), (int)group_begin.size() - 1, (const SegDev *)c->d_segs, c->ws(),
                c->prof);
    HIPCHK(hipEventRecord(c->run_ev, st));
    HIPCHK(hipGetLastError());
    c->last_stream = st;
    return AMM_OK;
}

int amm_integrate_batches(amm_ctx *c, const amm_run_params *r, uint64_t n_batches, void *stream) {
    if (!c || !r || n_batches == 0) return fail(AMM_E_ARG, "amm_integrate_batches: bad argument");
    if (r->n_per_graph > (~0ull - r->counter0) / n_batches ||
        !mrg_range_ok(c, r->counter0 + n_batches * r->n_per_graph))
        return fail(AMM_E_ARG, "amm_integrate_batches: sample indices out of range");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = c->cap_stream;
    std::vector<SegDev> segs;
    std::vector<int> group_begin;
    int rc = prepare_run(c, r, st, c->d_base, segs, group_begin);
    if (rc) return rc;
    zero_acc(c, r, st);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, st, c->d_base, (uint64_t)0);   // first batch at counter0
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
    HIPCHK(hipEventRecord(e0, st));
    HIPCHK(hipStreamWaitEvent(cs, e0, 0));
    // one batch: the groups' kernels, then the sample base advances by n_per_graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    enqueue_run(c, r, cs, segs.data(), group_begin.data(), (int)group_begin.size() - 1, (const SegDev *)c->d_segs, c->ws(),
                false);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, cs, c->d_base, r->n_per_graph);
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (ce != hipSuccess) {
        hipEventDestroy(e0); hipEventDestroy(e1);
        return fail(AMM_E_HIP, std::string("amm_integrate_batches: capture: ") + hipGetErrorString(ce));
    }
    ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (uint64_t b = 0; b < n_batches && ce == hipSuccess; ++b) ce = hipGraphLaunch(exec, cs);
    if (ce == hipSuccess) ce = hipEventRecord(e1, cs);
    if (ce == hipSuccess) ce = hipStreamWaitEvent(st, e1, 0);
    if (ce == hipSuccess) ce = hipEventRecord(c->run_ev, st);
    hipStreamSynchronize(cs);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (ce != hipSuccess) return fail(AMM_E_HIP, std::string("amm_integrate_batches: ") + hipGetErrorString(ce));
    c->last_stream = st;
    return AMM_OK;
}

int amm_autotune(amm_ctx *c, const amm_run_params *r, int *blocks_per_cu, int *order_by_cost, double *ms_best,
                 void *stream) {
    if (!c || !r || r->n_per_graph == 0) return fail(AMM_E_ARG, "amm_autotune: bad argument");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(c->device));
    // the probe runs overwrite the accumulators of the graphs: keep a copy
    const size_t nacc = c->slots.size() * NSTAT_MAX;
    double *saved = nullptr;
    HIPCHK(hipMalloc((void **)&saved, nacc * sizeof(double)));
    HIPCHK(hipMemcpyAsync(saved, c->d_acc, nacc * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int bpcs[] = {1, 2, 4, 8, 16};
    const int keep_order = c->order_by_cost, keep_prof = c->prof;
    c->prof = false;
    int best_b = 8, best_o = keep_order, rc = AMM_OK;
    float best = 3.4e38f;
    amm_run_params q = *r;
    q.accumulate = 0;
    for (int o = 0; o < 2 && rc == AMM_OK; ++o) {
        c->order_by_cost = o;
        for (int b : bpcs) {
            q.blocks_per_cu = b;
            if ((rc = amm_integrate(c, &q, st))) break;          // warm-up
            hipEventRecord(e0, st);
            if ((rc = amm_integrate(c, &q, st))) break;
            hipEventRecord(e1, st);
            hipEventSynchronize(e1);
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; best_b = b; best_o = o; }
        }
    }
    c->prof = keep_prof;
    hipMemcpyAsync(c->d_acc, saved, nacc * sizeof(double), hipMemcpyDeviceToDevice, st);
    hipStreamSynchronize(st);
    hipFree(saved);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) { c->order_by_cost = keep_order; return rc; }
    c->blocks_per_cu = best_b;
    c->order_by_cost = best_o;
    if (blocks_per_cu) *blocks_per_cu = best_b;
    if (order_by_cost) *order_by_cost = best_o;
    if (ms_best) *ms_best = best;
    c->last_stream = st;
    return AMM_OK;
}

// Sec. IV.C: the share of graph j is proportional to C_j / sqrt(t_j), which
// minimises sum_j C_j^2 / n_j (the variance of the summed estimate, eq.
// sigma_sum) at a fixed cost sum_j n_j t_j; a share floor_frac of the budget
// is split equally (the stabilisation that keeps graphs with an
// underestimated C_j sampled).  The operation order is fixed (no contraction).
int amm_adaptive_split(int n, const double *C, const double *t, double budget, double floor_frac, uint64_t *n_out) {
    if (n < 1 || !C || !t || !n_out || !std::isfinite(budget) || !(budget >= 0.0) || !(floor_frac >= 0.0) ||
        !(floor_frac <= 1.0))
        return fail(AMM_E_ARG, "amm_adaptive_split: bad argument");
    double st = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!std::isfinite(t[j]) || !(t[j] > 0.0) || !std::isfinite(C[j]) || !(C[j] >= 0.0))
            return fail(AMM_E_ARG, "amm_adaptive_split: C must be >= 0 and t > 0, finite");
        st = st + t[j];
    }
    std::vector<double> w(n);
    double swt = 0.0;
    for (int j = 0; j < n; ++j) {
        const double r = std::sqrt(t[j]);
        w[j] = C[j] / r;
        const double wt = w[j] * t[j];
        swt = swt + wt;
    }
    const double f = swt > 0.0 ? floor_frac : 1.0;   // all C_j = 0: equal split
    const double eq = budget / st;
    for (int j = 0; j < n; ++j) {
        double x = f * eq;
        if (swt > 0.0) {
            double ney = budget * w[j];
            ney = ney / swt;
            ney = ney * (1.0 - f);
            x = x + ney;
        }
        if (!(x < 9.2e18)) return fail(AMM_E_ARG, "amm_adaptive_split: sample count out of range");
        n_out[j] = (uint64_t)std::floor(x);
    }
    return AMM_OK;
}

int amm_combine(int n, const double *mean1, const double *sigma1, const double *mean2, const double *sigma2,
                double *mean, double *sigma, double *total_mean, double *total_sigma) {
    if (n < 0 || (n > 0 && (!mean1 || !sigma1 || !mean2 || !sigma2)))
        return fail(AMM_E_ARG, "amm_combine: bad argument");
    double tm = 0.0, tv = 0.0;
    for (int j = 0; j < n; ++j) {
        const double s1 = sigma1[j], s2 = sigma2[j];
        if (!(s1 >= 0.0) || !(s2 >= 0.0)) return fail(AMM_E_ARG, "amm_combine: sigma must be >= 0");
        double m, s;
        if (s1 == 0.0 && s2 == 0.0) {
            m = 0.5 * (mean1[j] + mean2[j]);
            s = 0.0;
        } else if (s1 == 0.0) {
            m = mean1[j];
            s = 0.0;
        } else if (s2 == 0.0) {
            m = mean2[j];
            s = 0.0;
        } else {
            const double w1 = 1.0 / (s1 * s1), w2 = 1.0 / (s2 * s2);
            const double w = w1 + w2;
            const double a = mean1[j] * w1, b = mean2[j] * w2;
            m = (a + b) / w;
            s = std::sqrt(1.0 / w);
        }
        if (mean) mean[j] = m;
        if (sigma) sigma[j] = s;
        tm = tm + m;
        tv = tv + s * s;
    }
    if (total_mean) *total_mean = tm;
    if (total_sigma) *total_sigma = std::sqrt(tv);
    return AMM_OK;
}

int amm_integrate_adaptive(amm_ctx *c, const amm_run_params *r, uint64_t budget_per_graph, int n_rounds,
                           double floor_frac, const double *cost, uint64_t *n_done, void *stream) {
    if (!c || !r || n_rounds < 1 || budget_per_graph < r->n_per_graph || !(floor_frac >= 0.0) ||
        !(floor_frac <= 1.0))
        return fail(AMM_E_ARG, "amm_integrate_adaptive: bad argument");
    if (r->graph_begin < 0 || r->graph_end > (int)c->slots.size() || r->graph_begin >= r->graph_end)
        return fail(AMM_E_ARG, "amm_integrate_adaptive: bad graph range");
    const int gb = r->graph_begin, G = r->graph_end - r->graph_begin;
    for (int g = gb; g < r->graph_end; ++g)
        if (!c->slots[g].has_plan) return fail(AMM_E_NOTBUILT, "amm_integrate_adaptive: integrand tables not built");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> t(G), Cj(G);
    double tsum = 0.0;
    for (int j = 0; j < G; ++j) {
        t[j] = cost ? cost[j] : c->slots[gb + j].plan.flops_per_sample;
        if (!std::isfinite(t[j]) || !(t[j] > 0.0)) return fail(AMM_E_ARG, "amm_integrate_adaptive: cost must be > 0");
        tsum = tsum + t[j];
    }
    const double total = (double)budget_per_graph * tsum;
    std::vector<uint64_t> done(G, 0), nr(G, r->n_per_graph), c0(G);
    double spent = 0.0;
    amm_run_params q = *r;
    std::vector<SegDev> segs;
    std::vector<int> group_begin;
    for (int round = 0; round < n_rounds; ++round) {
        if (round > 0) {
            // C_j = sigma_j sqrt(N_j) from the accumulators (this run's earlier rounds)
            for (int j = 0; j < G; ++j) {
                amm_estimate e;
                int rc = amm_read(c, gb + j, -1, -1, -1, -1, &e);
                if (rc) return rc;
                Cj[j] = e.n > 0 ? e.sigma * std::sqrt((double)e.n) : 0.0;
            }
            const double left = total - spent;
            if (!(left > 0.0)) break;
            int rc = amm_adaptive_split(G, Cj.data(), t.data(), left / (double)(n_rounds - round), floor_frac,
                                        nr.data());
            if (rc) return rc;
        }
        for (int j = 0; j < G; ++j) c0[j] = r->counter0 + done[j];
        q.accumulate = round == 0 ? r->accumulate : 1;
        int rc = prepare_run(c, &q, st, nullptr, segs, group_begin, c0.data(), nr.data());
        if (rc) return rc;
        zero_acc(c, &q, st);
        enqueue_run(c, &q, st, segs.data(), group_begin.data(), (int)group_begin.size() - 1, (const SegDev *)c->d_segs,
                    c->ws(), c->prof);
        HIPCHK(hipEventRecord(c->run_ev, st));
        HIPCHK(hipGetLastError());
        c->last_stream = st;
        for (int j = 0; j < G; ++j) {
            done[j] += nr[j];
            spent = spent + (double)nr[j] * t[j];
        }
    }
    if (n_done)
        for (int j = 0; j < G; ++j) n_done[j] = done[j];
    return AMM_OK;
}

int amm_profile(amm_ctx *c, int enable, double *ms_fp64, double *ms_dd, double *ms_reduce, int64_t *n_launches,
                int64_t *n_samples) {
    if (!c) return fail(AMM_E_ARG, "amm_profile: ctx is NULL");
    HIPCHK(hipSetDevice(c->device));
    prof_collect(c);
    if (ms_fp64) *ms_fp64 = c->prof_ms[0];
    if (ms_dd) *ms_dd = c->prof_ms[1];
    if (ms_reduce) *ms_reduce = c->prof_ms[2];
    if (n_launches) *n_launches = c->prof_launch;
    if (n_samples) *n_samples = c->prof_samples;
    if (enable && !c->prof) {
        c->prof_ms[0] = c->prof_ms[1] = c->prof_ms[2] = 0;
        c->prof_launch = c->prof_samples = 0;
    }
    c->prof = enable != 0;
    return AMM_OK;
}

int amm_set_option(amm_ctx *c, int option, int value) {
    if (!c) return fail(AMM_E_ARG, "amm_set_option: ctx is NULL");
    if (option == AMM_OPT_GENERATED) c->use_gen = value != 0;
    else if (option == AMM_OPT_FUSED) c->use_fused = value != 0;
    else if (option == AMM_OPT_ORDER_BY_COST) c->order_by_cost = value != 0;
    else if (option == AMM_OPT_BLOCKS_PER_CU) {
        if (value < 0 || value > 64) return fail(AMM_E_ARG, "amm_set_option: blocks per CU 0..64");
        c->blocks_per_cu = value;
    } else if (option == AMM_OPT_GENERATOR) {
        if (value != 0 && value != 1) return fail(AMM_E_ARG, "amm_set_option: generator 0 (Philox) or 1 (MRG32k3a)");
        c->generator = value;
    } else if (option == AMM_OPT_PLANS) c->build_plans = value != 0;
    else return fail(AMM_E_ARG, "amm_set_option: unknown option");
    return AMM_OK;
}

int amm_accept_thresholds(amm_ctx *c, int gb, int ge, uint64_t n_run, double *tau) {
    if (!c || !tau || gb < 0 || ge > (int)c->slots.size() || gb >= ge || n_run == 0)
        return fail(AMM_E_ARG, "amm_accept_thresholds: bad argument");
    std::vector<double> sig(ge - gb);
    double s1 = 0.0, s2 = 0.0;
    for (int g = gb; g < ge; ++g) {
        amm_estimate est;
        int rc = amm_read(c, g, -1, -1, -1, -1, &est);
        if (rc) return rc;
        if (est.n == 0) return fail(AMM_E_ARG, "amm_accept_thresholds: no pilot samples");
        double sj = est.sigma * std::sqrt((double)est.n / (double)n_run);
        sig[g - gb] = sj;
        s1 += sj;
        s2 += sj * sj;
    }
    for (int g = gb; g < ge; ++g) tau[g - gb] = s1 > 0 ? 0.25 * sig[g - gb] * std::sqrt(s2) / s1 : INFINITY;
    return AMM_OK;
}

int amm_read(amm_ctx *c, int g, int e, int ck, int cm, int cmp, amm_estimate *out) {
    if (!c || !out) return fail(AMM_E_ARG, "amm_read: bad argument");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->last_stream));
    std::vector<double> all(c->slots.size() * NSTAT_MAX);
    if (!all.empty())
        HIPCHK(hipMemcpy(all.data(), c->d_acc, all.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    auto fin = [&](double s, double s2, double n) {
        out->mean = n > 0 ? s / n : 0.0;
        double var = n > 0 ? s2 / (n * n) - s * s / (n * n * n) : 0.0;
        out->sigma = std::sqrt(var > 0 ? var : 0.0);
    };
    if (g >= 0) {
        if (g >= (int)c->slots.size() || !c->slots[g].built) return fail(AMM_E_ARG, "amm_read: graph not built");
        const GraphSlot &s = c->slots[g];
        const double *a = &all[(size_t)g * NSTAT_MAX];
        int ne = s.ne, nst = s.nstat();
        out->n = (uint64_t)a[nst - 4];
        out->n_flag = (uint64_t)a[nst - 3];
        out->n_dd_fail = (uint64_t)a[nst - 2];
        out->n_ood = (uint64_t)a[nst - 1];
        if (e >= 0) {
            if (e >= ne) return fail(AMM_E_ARG, "amm_read: bad insertion");
            out->sum_y = a[e]; out->sum_y2 = a[ne + e]; out->sum_abs = a[2 * ne + e];
            fin(out->sum_y, out->sum_y2, (double)out->n);
        } else {
            // sum over insertions: the per-point total keeps their covariance
            double sa = 0;
            for (int q = 0; q < ne; ++q) sa += a[2 * ne + q];
            out->sum_y = a[3 * ne + 2 * s.ncls];
            out->sum_y2 = a[3 * ne + 2 * s.ncls + 1];
            out->sum_abs = sa;
            fin(out->sum_y, out->sum_y2, (double)out->n);
        }
        return AMM_OK;
    }
    // class over all built graphs: means add, sigma^2 add (eq. sigma_sum)
    double mean = 0, var = 0;
    uint64_t ntot = 0, nfl = 0, ndd = 0, nood = 0;
    for (size_t gi = 0; gi < c->slots.size(); ++gi) {
        const GraphSlot &s = c->slots[gi];
        if (!s.built) continue;
        const double *a = &all[gi * NSTAT_MAX];
        int ne = s.ne, nst = s.nstat();
        double n = a[nst - 4];
        // one class: its per-point sums; all classes: the per-point totals
        for (int q = 0; q < (ck >= 0 ? s.ncls : 1); ++q) {
            if (ck >= 0 && (s.cls_kmm[q][0] != ck || s.cls_kmm[q][1] != cm || s.cls_kmm[q][2] != cmp)) continue;
            const double cs = ck >= 0 ? a[3 * ne + q] : a[3 * ne + 2 * s.ncls];
            const double cs2 = ck >= 0 ? a[3 * ne + s.ncls + q] : a[3 * ne + 2 * s.ncls + 1];
            if (n > 0) {
                mean += cs / n;
                double v = cs2 / (n * n) - cs * cs / (n * n * n);
                var += v > 0 ? v : 0;
            }
        }
        ntot += (uint64_t)n; nfl += (uint64_t)a[nst - 3]; ndd += (uint64_t)a[nst - 2]; nood += (uint64_t)a[nst - 1];
    }
    out->mean = mean; out->sigma = std::sqrt(var);
    out->n = ntot; out->n_flag = nfl; out->n_dd_fail = ndd; out->n_ood = nood;
    return AMM_OK;
}

}  // extern "C"
