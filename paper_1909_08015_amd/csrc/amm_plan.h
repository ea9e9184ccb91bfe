// amm_plan.h -- flattened per-graph evaluation plan (host builder -> device).
//
// A plan describes, for one SE graph, everything the device needs per sample:
// density tables (Sec. III.A) and, for every insertion of the external photon,
// the terms of the forest formula R^new (Sec. II) as post-order programs over
// "levels" (a forest element with its maximal sub-elements contracted).
#pragma once
#include <stdint.h>

namespace amm {

constexpr int MAXN = 5;            // loops
constexpr int MAXM = 3 * MAXN - 1; // Feynman parameters
constexpr int MAXK = 12;           // electron segments of one level
constexpr int MAXL = MAXN;         // photons (loops) of one level
constexpr int MAXMONO_VARS = 14;   // variables of one numerator monomial

enum LevelOp : int32_t { OP_A = 0, OP_U = 1, OP_L = 2, OP_LU = 3, OP_SE = 4 };

// One numerator monomial: coef * prod vars[v[i]], i < nv.
struct Mono {
    double coef;
    uint8_t nv;
    uint8_t v[MAXMONO_VARS + 1];
};

// Variable layout of a level with K segments:
//   x_{kk'} (1 <= k <= k' <= K) at xidx(K, k, k'), then A_k at XN(K) + k - 1,
//   then C_k at XN(K) + K + k - 1.
__host__ __device__ inline int amm_xn(int K) { return K * (K + 1) / 2; }
// Number of variable slots of a level at n loops (K <= 2n segments); the slot
// with this index holds the constant 1 in the FP64 interpreter (padding of
// monomial groups, see the group stream in amm_core.h).
__host__ __device__ constexpr int amm_nvars(int n) { return (2 * n) * (2 * n + 1) / 2 + 2 * (2 * n); }
__host__ __device__ inline int amm_xidx(int K, int k, int k2) {
    return (k - 1) * (2 * K - k + 2) / 2 + (k2 - k);
}

struct LevelDesc {
    int32_t K, L, op, ext_node, has_X;
    int32_t nvar;           // variables used (x, A, C)
    int32_t nout;           // 1 (vertex) or 2 (SE: u, v)
    int32_t nvariants;      // 2^(number of SE children)
    int32_t nkids;          // children in node order
    uint32_t kid_is_se;     // bit i: child i is an SE child
    int32_t mono_range;     // index into the range table: (variant*nout+out)*(n+1)+c
    int32_t seg_param[MAXK];
    int32_t seg_half[MAXK]; // 1 if the segment is half of the merged line
    int32_t ph_param[MAXL];
    uint32_t span[MAXL];    // bit k-1 set if photon a spans segment k
    double pref;            // 4^-L (-1)^N
};

struct TermDesc {
    int32_t e;              // insertion
    int32_t sign;
    int32_t op_begin, op_end;  // level ids (post-order) in the term op list
};

// Host-side plan of one graph (device copies hold the same arrays).
struct PlanCounts {
    int32_t n, M, ninsert, nlevels, nterms, nops, nranges;
    int64_t nmonos;
};

}  // namespace amm
