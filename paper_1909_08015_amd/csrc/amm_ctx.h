// amm_ctx.h -- library context (internal; shared by the HIP translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "amm_core.h"
#include "amm_mlp.h"

namespace amm {

int fail(int code, const std::string &msg);

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess)                                                          \
            return ::amm::fail(AMM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int BLOCK = 128;
constexpr int RPC = 8;                        // rounds per chunk
constexpr int CHUNK = BLOCK * RPC;            // samples per chunk (the unit of the fixed-order sums)
constexpr int MAX_GROUP_CHUNKS = 32768;       // chunks per group (33.5M samples): one DD pass each
constexpr int DD_BLOCK = 64;                  // one wave per block in the double-double recompute
constexpr int DD_RESIDENT_LANES = 65536;      // lanes of the double-double recompute resident at once (about)
constexpr uint32_t FLAG_DDFAIL = 0x80000000u; // flag word: the DD bound cannot pass either
constexpr double KAPPA = 2.0;                 // safety factor on the first-order running error bound
constexpr int MAXNE = 2 * MAXN - 1;
// Statistics per graph: 3 per insertion, 2 per class, 2 for the per-point
// total over the insertions, 4 counters (layout at add_stats).
__host__ __device__ constexpr int nstat_of(int ne, int ncls) { return 3 * ne + 2 * ncls + 6; }
constexpr int NSTAT_MAX = nstat_of(MAXNE, MAXNE);

// Scratch of a Monte Carlo run, used one group of chunks at a time: chunk
// partial sums, flag words, flag counts and their scan, the double-double
// results of the group's flagged points (room for every point) and the work
// counter of the fused launch.
struct Workspace {
    double *part = nullptr;     // [max_chunks * NSTAT_MAX]
    uint32_t *flag = nullptr;   // [max_chunks * CHUNK]
    int32_t *nflag = nullptr;   // [max_chunks]
    int32_t *foff = nullptr;    // [max_chunks + 1]
    double *ydd = nullptr;      // [ydd_ne][max_chunks * CHUNK]
    int *work = nullptr;        // [1]
    int max_chunks = 0;         // chunks per group (<= MAX_GROUP_CHUNKS)
    int ydd_ne = 0;             // insertions the ydd region holds
    size_t ydd_cap() const { return (size_t)max_chunks * CHUNK; }
};

// Byte layout of a workspace carved from one region (256-byte aligned parts).
constexpr size_t ws_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t ws_bytes(int max_chunks, int ne) {
    return ws_align((size_t)max_chunks * NSTAT_MAX * sizeof(double)) +
           ws_align((size_t)max_chunks * CHUNK * sizeof(uint32_t)) + ws_align((size_t)max_chunks * sizeof(int32_t)) +
           ws_align((size_t)(max_chunks + 1) * sizeof(int32_t)) +
           ws_align((size_t)ne * max_chunks * CHUNK * sizeof(double)) + ws_align(sizeof(int));
}
inline Workspace ws_carve(void *base, int max_chunks, int ne) {
    Workspace w;
    char *p = (char *)base;
    w.part = (double *)p;    p += ws_align((size_t)max_chunks * NSTAT_MAX * sizeof(double));
    w.flag = (uint32_t *)p;  p += ws_align((size_t)max_chunks * CHUNK * sizeof(uint32_t));
    w.nflag = (int32_t *)p;  p += ws_align((size_t)max_chunks * sizeof(int32_t));
    w.foff = (int32_t *)p;   p += ws_align((size_t)(max_chunks + 1) * sizeof(int32_t));
    w.ydd = (double *)p;     p += ws_align((size_t)ne * max_chunks * CHUNK * sizeof(double));
    w.work = (int *)p;
    w.max_chunks = max_chunks;
    w.ydd_ne = ne;
    return w;
}

struct GraphSlot {
    bool built = false;                       // density tables (sampling)
    bool has_plan = false;                    // integrand tables (evaluation)
    int n = 0, M = 0, ne = 0, ncls = 0;
    int cls_of[MAXNE] = {0};
    int cls_kmm[MAXNE][3];
    uint32_t uid = 0;
    PlanHost plan;
    DensityTables dens;
    // device copies
    LevelDesc *d_levels = nullptr;
    TermDesc *d_terms = nullptr;
    int32_t *d_ops = nullptr;
    Mono *d_monos = nullptr;
    int2 *d_ranges = nullptr;
    uint32_t *d_gwords = nullptr;             // FP64 group stream and its ranges
    int2 *d_granges = nullptr;
    int ngwords = 0;
    double *d_deg1 = nullptr, *d_deg3 = nullptr, *d_W1 = nullptr, *d_logdeg1 = nullptr;
    float *d_ptheta = nullptr;                // learned P_theta(j|s) [2^M * M]
    double *d_pilotW = nullptr;               // pilot W(s, j) [2^M * M]
    // accumulators (host mirror after read)
    std::vector<double> acc;                  // NSTAT
    int nstat() const { return nstat_of(ne, ncls); }
    PlanDev plan_dev() const {
        PlanDev p;
        p.levels = d_levels; p.terms = d_terms; p.ops = d_ops; p.monos = d_monos; p.ranges = d_ranges;
        p.nterms = (int)plan.terms.size(); p.n = n; p.ninsert = ne;
        p.gwords = d_gwords; p.granges = d_granges; p.ngwords = ngwords;
        return p;
    }
    DensityDev dens_dev(bool learned) const {
        DensityDev D;
        D.deg1 = d_deg1; D.deg3 = d_deg3; D.W1 = d_W1; D.logdeg1 = d_logdeg1;
        for (int c = 0; c < 4; ++c) { D.logK[c] = dens.logK[c]; D.logc[c] = dens.logc[c]; D.c[c] = dens.c[c]; }
        D.ptheta = learned ? d_ptheta : nullptr;
        D.logc_mix = 0;
        return D;
    }
};

}  // namespace amm

struct amm_ctx {
    int device = 0;
    int loops = 0;
    std::vector<amm::SEGraph> graphs;
    std::vector<amm::GraphSlot> slots;
    hipStream_t last_stream = nullptr;
    double *d_acc = nullptr;            // [graphs * NSTAT_MAX]
    amm::Workspace own;                 // allocated by the context (groups of MAX_GROUP_CHUNKS), on first use
    amm::Workspace user;                // carved from amm_set_workspace memory (caller-owned)
    bool use_user_ws = false;
    const amm::Workspace &ws() const { return use_user_ws ? user : own; }
    void *static_base = nullptr;        // this device's static scratch (amm_integrate_static)
    hipEvent_t static_seg_ev = nullptr; // recorded after the last staging copy of the static path
    void *static_stage = nullptr;       // host staging of the static path's segment table (SegDev[])
    void *d_segs = nullptr;             // segment tables of one call (SegDev), device
    void *h_segs = nullptr;             // pinned staging copy
    size_t seg_cap = 0;                 // capacity in segments
    hipEvent_t seg_ev = nullptr;        // recorded after the last staging copy
    hipEvent_t run_ev = nullptr;        // recorded after the last kernel of a run (on its stream)
    uint64_t *d_base = nullptr;         // sample base added by replays of a captured batch
    hipStream_t cap_stream = nullptr;   // internal stream for graph capture and replay
    int generator = 0;                  // 0 Philox4x32-10, 1 MRG32k3a (AMM_OPT_GENERATOR)
    uint32_t *d_mrg_tab = nullptr;      // MRG32k3a jump powers (MRG_TABLE_WORDS words)
    uint64_t mrg_j100[2][9] = {};       // A^(2^100) of both components (graph stream spacing)
    static constexpr int NSIDE = 4;
    hipStream_t side[NSIDE] = {};       // the per-graph launches of a group run concurrently on these
    hipEvent_t fork_ev = nullptr, join_ev[NSIDE] = {};
    // launch configuration (set by amm_autotune or amm_set_option)
    int use_fused = 1;                  // interpreter graphs: one persistent launch per group
    int build_plans = 1;                // amm_build_tables builds integrand tables (AMM_OPT_PLANS)
    int order_by_cost = 1;              // segments of a group heaviest graph first
    int blocks_per_cu = 0;              // 0: default
    amm::MlpState mlp;
    bool use_gen = true;                // generated integrand code when built
    // profiling
    bool prof = false;
    struct Ev { hipEvent_t a, b, c, d; int64_t samples; int nseg; };
    std::vector<Ev> evs;
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_launch = 0, prof_samples = 0;
    ~amm_ctx();
};

