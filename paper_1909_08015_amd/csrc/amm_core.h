// amm_core.h -- per-sample device code: Philox, density sampling, level
// quantities and the forest-term interpreter.  Written once for the HIP
// kernels; every function is __host__ __device__.
//
// Paper references: sampling and density Sec. III.A (eq. pdf, pdf_final),
// g stored as x 2^j Sec. IV.A, forest formula Sec. II, estimator Sec. III.B.
#pragma once
#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "amm_host.h"
#include "amm_plan.h"

#define AMM_HD __host__ __device__
#define AMM_HDI __host__ __device__ __forceinline__

namespace amm {

// ---------------------------------------------------------------------------
// Double-double arithmetic (Dekker; Knuth two-sum; two-product via fma), as in
// Hida, Li & Bailey's quad-double library.  Used for recomputing flagged points.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
    AMM_HDI dd() : hi(0), lo(0) {}
    AMM_HDI dd(double x) : hi(x), lo(0) {}
    AMM_HDI dd(double h, double l) : hi(h), lo(l) {}
};
AMM_HDI dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd(s, e);
}
AMM_HDI dd quick_two_sum(double a, double b) {
    double s = a + b;
    return dd(s, b - (s - a));
}
AMM_HDI dd two_prod(double a, double b) {
    double p = a * b;
    return dd(p, fma(a, b, -p));
}
AMM_HDI dd operator+(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
AMM_HDI dd operator-(dd a) { return dd(-a.hi, -a.lo); }
AMM_HDI dd operator-(dd a, dd b) { return a + (-b); }
AMM_HDI dd operator*(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
AMM_HDI dd operator/(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = a - b * dd(q1);
    double q2 = r.hi / b.hi;
    r = r - b * dd(q2);
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return q + dd(q3);
}
AMM_HDI dd &operator+=(dd &a, dd b) { a = a + b; return a; }
AMM_HDI dd &operator-=(dd &a, dd b) { a = a - b; return a; }
AMM_HDI dd &operator*=(dd &a, dd b) { a = a * b; return a; }
AMM_HDI double to_double(double x) { return x; }
AMM_HDI double to_double(dd x) { return x.hi + x.lo; }
AMM_HDI double absd(double x) { return fabs(x); }
AMM_HDI dd absd(dd x) { return x.hi < 0 ? -x : x; }
AMM_HDI double mul_add(double a, double b, double c) { return fma(a, b, c); }
AMM_HDI dd mul_add(dd a, dd b, dd c) { return a * b + c; }

// ---------------------------------------------------------------------------
// FP64 value with a running round-off magnitude (reading R11, in the spirit
// of the paper's "eliminated interval arithmetic": operations on centres and
// a cheap radius formula).  a >= |v| is the value of the same computation
// done on magnitudes, extended through divisions by first-order error
// propagation; the rounding error of v is bounded by ~k u a for an
// operation-chain depth k.
// ---------------------------------------------------------------------------
// FP64 value with a first-order running error bound (Wilkinson's running
// error analysis): |v - exact| <= u a, u = 2^-53.  Every operation adds the
// rounding of its own result, |result|, to the propagated errors of its
// operands; constants are counted as rounded once.
struct ea {
    double v, a;
    AMM_HDI ea() : v(0), a(0) {}
    AMM_HDI ea(double x) : v(x), a(fabs(x)) {}
    AMM_HDI ea(double x, double m) : v(x), a(m) {}
};
AMM_HDI ea operator+(ea x, ea y) {
    double z = x.v + y.v;
    return ea(z, (x.a + y.a) + fabs(z));
}
AMM_HDI ea operator-(ea x) { return ea(-x.v, x.a); }
AMM_HDI ea operator-(ea x, ea y) {
    double z = x.v - y.v;
    return ea(z, (x.a + y.a) + fabs(z));
}
AMM_HDI ea operator*(ea x, ea y) {
    double z = x.v * y.v;
    return ea(z, fma(x.a, fabs(y.v), fma(y.a, fabs(x.v), fabs(z))));
}
AMM_HDI ea operator/(ea x, ea y) {
    double q = x.v / y.v, ay = fabs(y.v);
    return ea(q, fma(fabs(q), y.a, x.a) / ay + fabs(q));
}
AMM_HDI ea &operator+=(ea &x, ea y) { x = x + y; return x; }
AMM_HDI ea &operator-=(ea &x, ea y) { x = x - y; return x; }
AMM_HDI ea &operator*=(ea &x, ea y) { x = x * y; return x; }
AMM_HDI double to_double(ea x) { return x.v; }
AMM_HDI ea absd(ea x) { return ea(fabs(x.v), x.a); }
AMM_HDI ea mul_add(ea x, ea y, ea z) {
    double w = fma(x.v, y.v, z.v);
    return ea(w, fma(x.a, fabs(y.v), fma(y.a, fabs(x.v), z.a + fabs(w))));
}
AMM_HDI double mag(ea x) { return x.a; }
// Kept as an identity: every operation's error is propagated.
AMM_HDI ea strip(ea x) { return x; }
// Relative error bound a / |v| (units of u); infinite for a zero value with a
// nonzero error.  On the device the reciprocal is the hardware approximation,
// enlarged by 2^-16 so that the result stays an upper bound.
AMM_HDI double relerr(ea x) {
    if (!(x.a > 0.0)) return 0.0;
#if defined(__HIP_DEVICE_COMPILE__)
    return x.a * __builtin_amdgcn_rcp(fabs(x.v)) * (1.0 + 0x1p-16);
#else
    return x.a / fabs(x.v);
#endif
}
// FP64 interval [lo, hi] with outward rounding (the first interval rung of
// Sec. IV.A's ladder).  Directed rounding is emulated from round-to-nearest:
// the exact error of a sum (two-sum), a product (fma) or a quotient (fma
// residual) shows on which side of the exact value the rounded result lies,
// and a bound moves one ulp outward when it lies inside.  Every operation on
// enclosing operands encloses the exact result, as long as nothing
// overflows, underflows or turns NaN.
struct iv {
    double lo, hi;
    AMM_HDI iv() : lo(0), hi(0) {}
    AMM_HDI iv(double x) : lo(x), hi(x) {}
    AMM_HDI iv(double l, double h) : lo(l), hi(h) {}
};
AMM_HDI double round_dn(double s, double err) { return err < 0.0 ? nextafter(s, -INFINITY) : s; }
AMM_HDI double round_up(double s, double err) { return err > 0.0 ? nextafter(s, INFINITY) : s; }
AMM_HDI double sum_err(double a, double b, double s) {
    const double bb = s - a;
    return (a - (s - bb)) + (b - bb);
}
AMM_HDI double add_dn(double a, double b) { const double s = a + b; return round_dn(s, sum_err(a, b, s)); }
AMM_HDI double add_up(double a, double b) { const double s = a + b; return round_up(s, sum_err(a, b, s)); }
AMM_HDI double mul_dn(double a, double b) { const double p = a * b; return round_dn(p, fma(a, b, -p)); }
AMM_HDI double mul_up(double a, double b) { const double p = a * b; return round_up(p, fma(a, b, -p)); }
// a / b = q + r / b exactly, r = a - q b (exact by fma)
AMM_HDI double div_dn(double a, double b) {
    const double q = a / b, r = fma(-q, b, a);
    return (r != 0.0 && ((r < 0.0) != (b < 0.0))) ? nextafter(q, -INFINITY) : q;
}
AMM_HDI double div_up(double a, double b) {
    const double q = a / b, r = fma(-q, b, a);
    return (r != 0.0 && ((r < 0.0) == (b < 0.0))) ? nextafter(q, INFINITY) : q;
}
AMM_HDI iv operator+(iv x, iv y) { return iv(add_dn(x.lo, y.lo), add_up(x.hi, y.hi)); }
AMM_HDI iv operator-(iv x) { return iv(-x.hi, -x.lo); }
AMM_HDI iv operator-(iv x, iv y) { return x + (-y); }
AMM_HDI iv operator*(iv x, iv y) {
    const double l = fmin(fmin(mul_dn(x.lo, y.lo), mul_dn(x.lo, y.hi)), fmin(mul_dn(x.hi, y.lo), mul_dn(x.hi, y.hi)));
    const double h = fmax(fmax(mul_up(x.lo, y.lo), mul_up(x.lo, y.hi)), fmax(mul_up(x.hi, y.lo), mul_up(x.hi, y.hi)));
    return iv(l, h);
}
AMM_HDI iv operator/(iv x, iv y) {
    if (y.lo <= 0.0 && y.hi >= 0.0) return iv(-INFINITY, INFINITY);
    const double l = fmin(fmin(div_dn(x.lo, y.lo), div_dn(x.lo, y.hi)), fmin(div_dn(x.hi, y.lo), div_dn(x.hi, y.hi)));
    const double h = fmax(fmax(div_up(x.lo, y.lo), div_up(x.lo, y.hi)), fmax(div_up(x.hi, y.lo), div_up(x.hi, y.hi)));
    return iv(l, h);
}
AMM_HDI iv &operator+=(iv &x, iv y) { x = x + y; return x; }
AMM_HDI iv &operator-=(iv &x, iv y) { x = x - y; return x; }
AMM_HDI iv &operator*=(iv &x, iv y) { x = x * y; return x; }
AMM_HDI double to_double(iv x) { return 0.5 * x.lo + 0.5 * x.hi; }
AMM_HDI iv absd(iv x) {
    if (x.lo >= 0.0) return x;
    if (x.hi <= 0.0) return -x;
    return iv(0.0, fmax(-x.lo, x.hi));
}
AMM_HDI iv mul_add(iv x, iv y, iv z) { return x * y + z; }
AMM_HDI iv strip(iv x) { return x; }
AMM_HDI double mag(iv x) { return fmax(fabs(x.lo), fabs(x.hi)); }
// Half-width about the midpoint, rounded up: |exact - to_double(x)| <= radius(x).
AMM_HDI double radius(iv x) {
    const double m = to_double(x);
    return fmax(add_up(x.hi, -m), add_up(m, -x.lo));
}
// A monomial coefficient: the double nearest a rational, so as an interval it
// spans its two neighbours.
template <typename T> AMM_HDI T coef_of(double c) { return T(c); }
template <> AMM_HDI iv coef_of<iv>(double c) { return iv(nextafter(c, -INFINITY), nextafter(c, INFINITY)); }

AMM_HDI double strip(double x) { return x; }
AMM_HDI dd strip(dd x) { return x; }
AMM_HDI double mag(double x) { return fabs(x); }
AMM_HDI double mag(dd x) { return fabs(x.hi); }

// ---------------------------------------------------------------------------
// exp / log with the fixed operation order (no contraction): Cody-Waite
// reduction + degree-13 Taylor polynomial; atanh series for log.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
AMM_HDI double amm_exp(double x) {
    if (x < -745.2) return 0.0;
    if (x > 709.78) return INFINITY;
    double k = rint(x * AMM_INV_LN2);
    double r = (x - k * AMM_LN2_HI) - k * AMM_LN2_LO;
    double p = amm_exp_c(13);
#pragma unroll
    for (int i = 12; i >= 0; --i) p = p * r + amm_exp_c(i);
    return ldexp(p, (int)k);
}
AMM_HDI double amm_log(double x) {
    int k;
    double m = frexp(x, &k);
    if (m < AMM_SQRT_HALF) { m = m * 2.0; k = k - 1; }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
    double q = amm_log_d(11);
#pragma unroll
    for (int i = 10; i >= 0; --i) q = q * s + amm_log_d(i);
    double lm = (2.0 * f) * q;
    double kd = (double)k;
    return (kd * AMM_LN2_LO + lm) + kd * AMM_LN2_HI;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the uniform conversion.
// ---------------------------------------------------------------------------
AMM_HDI void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}
AMM_HDI double uniform52(uint32_t a, uint32_t b) {
    return ((double)(a >> 6) * 67108864.0 + (double)(b >> 6) + 0.5) * 0x1p-52;
}
AMM_HDI void uniforms(uint64_t seed, uint32_t uid, uint64_t idx, int count, double *u) {
    uint32_t k0 = (uint32_t)(seed & 0xffffffffu) ^ uid, k1 = (uint32_t)(seed >> 32);
    for (int b = 0; 2 * b < count; ++b) {
        uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), (uint32_t)b, 0u};
        philox4x32_10(c, k0, k1);
        u[2 * b] = uniform52(c[0], c[1]);
        if (2 * b + 1 < count) u[2 * b + 1] = uniform52(c[2], c[3]);
    }
}

// ---------------------------------------------------------------------------
// MRG32k3a (L'Ecuyer, Oper. Res. 47 (1999) 159) as counter-addressed streams,
// the generator of the paper's first calculation (Sec. V).  Two order-3
// recurrences modulo m1 = 2^32 - 209 and m2 = 2^32 - 22853, output
// (x1 - x2) mod m1.  Sample i of a graph starts i 2^7 steps after the graph's
// start state s (computed on the host); the jump multiplies s by table
// powers A^(d 2^(7 + 4k)), d the k-th 4-bit digit of i (i < 2^44).
// Uniform: ((za >> 1) 2^21 + (zb >> 11) + 1/2) 2^-52 from two outputs.
// ---------------------------------------------------------------------------
constexpr uint32_t MRG_M1 = 4294967087u, MRG_M2 = 4294944443u;
constexpr uint32_t MRG_C1 = 209u, MRG_C2 = 22853u;                 // m = 2^32 - c
constexpr uint32_t MRG_A12 = 1403580u, MRG_A13N = MRG_M1 - 810728u;
constexpr uint32_t MRG_A21 = 527612u, MRG_A23N = MRG_M2 - 1370589u;
constexpr int MRG_SAMPLE_SHIFT = 7, MRG_WINDOWS = 11;              // sample indices < 2^44
constexpr int MRG_TABLE_WORDS = 2 * MRG_WINDOWS * 16 * 9;          // [component][window][digit][3][3]

// t mod (2^32 - c) by folding the high word (t < 2^64, c < 2^15)
AMM_HDI uint32_t mrg_mod(uint64_t t, uint32_t c, uint32_t m) {
    t = (t >> 32) * c + (t & 0xffffffffull);
    t = (t >> 32) * c + (t & 0xffffffffull);
    return (uint32_t)(t >= m ? t - m : t);
}
AMM_HDI uint32_t mrg_mul(uint32_t a, uint32_t b, uint32_t c, uint32_t m) { return mrg_mod((uint64_t)a * b, c, m); }
AMM_HDI void mrg_matvec(const uint32_t *A, uint32_t *x, uint32_t c, uint32_t m) {
    uint32_t y[3];
    for (int i = 0; i < 3; ++i)
        y[i] = mrg_mod((uint64_t)mrg_mul(A[3 * i], x[0], c, m) + mrg_mul(A[3 * i + 1], x[1], c, m) +
                           mrg_mul(A[3 * i + 2], x[2], c, m), c, m);
    x[0] = y[0]; x[1] = y[1]; x[2] = y[2];
}
// one step of both components (state x[n-3], x[n-2], x[n-1]); returns z[n]
AMM_HDI uint32_t mrg_step(uint32_t *p, uint32_t *q) {
    const uint32_t x1 = mrg_mod((uint64_t)mrg_mul(MRG_A12, p[1], MRG_C1, MRG_M1) + mrg_mul(MRG_A13N, p[0], MRG_C1, MRG_M1),
                                MRG_C1, MRG_M1);
    const uint32_t x2 = mrg_mod((uint64_t)mrg_mul(MRG_A21, q[2], MRG_C2, MRG_M2) + mrg_mul(MRG_A23N, q[0], MRG_C2, MRG_M2),
                                MRG_C2, MRG_M2);
    p[0] = p[1]; p[1] = p[2]; p[2] = x1;
    q[0] = q[1]; q[1] = q[2]; q[2] = x2;
    return x1 >= x2 ? x1 - x2 : x1 + (MRG_M1 - x2);
}
struct MrgStream {
    const uint32_t *tab;      // jump powers (device), MRG_TABLE_WORDS words
    uint32_t s[6];            // graph start state: x1[n-3..n-1], x2[n-3..n-1]
    int on;                   // 0: Philox4x32-10 instead
};
AMM_HDI void mrg_uniforms(const MrgStream &R, uint64_t idx, int count, double *u) {
    uint32_t p[3] = {R.s[0], R.s[1], R.s[2]}, q[3] = {R.s[3], R.s[4], R.s[5]};
    for (int k = 0; k < MRG_WINDOWS; ++k) {
        const int d = (int)((idx >> (4 * k)) & 15u);
        if (d) {
            mrg_matvec(R.tab + (k * 16 + d) * 9, p, MRG_C1, MRG_M1);
            mrg_matvec(R.tab + ((MRG_WINDOWS + k) * 16 + d) * 9, q, MRG_C2, MRG_M2);
        }
    }
    for (int i = 0; i < count; ++i) {
        const uint32_t za = mrg_step(p, q), zb = mrg_step(p, q);
        const uint64_t k = ((uint64_t)(za >> 1) << 21) + (zb >> 11);
        u[i] = ((double)k + 0.5) * 0x1p-52;
    }
}
// The sample's uniforms from the run's generator.
AMM_HDI void draw_uniforms(uint64_t seed, uint32_t uid, const MrgStream &R, uint64_t idx, int count, double *u) {
    if (R.on) mrg_uniforms(R, idx, count, u);
    else uniforms(seed, uid, idx, count, u);
}

AMM_HDI int popc(uint32_t x) {
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

struct DensityDev {
    const double *deg1, *deg3, *W1, *logdeg1;
    double logK[4], logc[4], c[4];
    const float *ptheta;      // learned P_theta(j | s) table [2^M * M] or null
    double logc_mix;          // unused placeholder for alignment
};

struct SampleOut {
    int comp;
    int ood;
    int gj;
    double gx;
};

// Sample one point of an M-parameter graph from u[0 .. 2M-2] (Sec. III.A
// sampling reading: mixture component, sector path, t = u^{1/Deg}).
// z[M] receives the point, path[M] the line order.
template <int M>
AMM_HDI SampleOut sample_point(const DensityDev &D, const double *u, double *z, int *path) {
    SampleOut o;
    const uint32_t full = (1u << M) - 1u;
    const float *P = D.ptheta;    // learned mixture when non-null: u has 2M entries
    // mixture component
    double thr = u[0], cum = 0.0;
    int comp = 3;
    bool chosen = false;
    for (int ci = 0; ci < 4; ++ci) {
        cum = cum + D.c[ci];
        if (!chosen && thr < cum) { comp = ci; chosen = true; }
    }
    if (P && u[2 * M - 1] < 0.5) comp = 4;
    o.comp = comp;
    bool uni = (comp == 1) || (comp == 3);
    uint32_t s = full;
    for (int l = 0; l < M - 1; ++l) {
        double ul = u[1 + l];
        int pick;
        if (comp == 4) {
            double total = 0.0;
            for (int j = 0; j < M; ++j)
                if ((s >> j) & 1u) total = total + (double)P[s * M + j];
            double t = ul * total;
            double cw = 0.0;
            pick = -1;
            int last = -1;
            for (int j = 0; j < M; ++j) {
                if (!((s >> j) & 1u)) continue;
                cw = cw + (double)P[s * M + j];
                if (pick < 0 && t < cw) pick = j;
                last = j;
            }
            if (pick < 0) pick = last;
        } else if (!uni) {
            double total = 0.0;
            for (int j = 0; j < M; ++j)
                if ((s >> j) & 1u) total = total + D.W1[s & ~(1u << j)];
            double t = ul * total;
            double cw = 0.0;
            pick = -1;
            int last = -1;
            for (int j = 0; j < M; ++j) {
                if (!((s >> j) & 1u)) continue;
                cw = cw + D.W1[s & ~(1u << j)];
                if (pick < 0 && t < cw) pick = j;
                last = j;
            }
            if (pick < 0) pick = last;
        } else {
            int size = popc(s);
            int k = (int)floor(ul * (double)size);
            int cnt = 0;
            pick = -1;
            for (int j = 0; j < M; ++j) {
                if (!((s >> j) & 1u)) continue;
                if (pick < 0 && cnt == k) pick = j;
                ++cnt;
            }
        }
        path[l] = pick;
        s &= ~(1u << pick);
    }
    for (int j = 0; j < M; ++j)
        if ((s >> j) & 1u) path[M - 1] = j;
    // continuous part
    uint32_t masks[M];
    uint32_t acc = 0;
    for (int l = M - 1; l >= 0; --l) { acc |= 1u << path[l]; masks[l] = acc; }
    double logt[M];
    logt[0] = 0.0;
    for (int l = 1; l < M; ++l) {
        uint32_t sl = masks[l];
        double dsel;
        if (comp == 1) dsel = (double)popc(sl);
        else if (comp == 2) dsel = D.deg3[sl];
        else dsel = D.deg1[sl];
        logt[l] = amm_log(u[M + l - 1]) / dsel;
    }
    double p[M], lp[M];
    p[0] = 1.0; lp[0] = 0.0;
    for (int l = 1; l < M; ++l) {
        double tt = amm_exp(logt[l]);
        p[l] = p[l - 1] * tt;
        lp[l] = lp[l - 1] + logt[l];
    }
    double norm = 0.0;
    for (int l = 0; l < M; ++l) norm = norm + p[l];
    double zmin = INFINITY;
    for (int l = 0; l < M; ++l) {
        double zl = p[l] / norm;
        z[path[l]] = zl;
        zmin = zl < zmin ? zl : zmin;
    }
    o.ood = !(zmin >= 2.2250738585072014e-308);
    double lognorm = amm_log(norm);
    double sumlogz = 0.0;
    for (int l = 0; l < M; ++l) sumlogz = sumlogz + lp[l];
    sumlogz = sumlogz - (double)M * lognorm;
    double E0 = 0.0, E1 = 0.0, E2 = 0.0, lds = 0.0;
    for (int l = 1; l < M; ++l) {
        uint32_t sl = masks[l];
        E0 = E0 + D.deg1[sl] * logt[l];
        E1 = E1 + (double)popc(sl) * logt[l];
        E2 = E2 + D.deg3[sl] * logt[l];
        lds = lds + D.logdeg1[sl];
    }
    double Lc[4];
    Lc[0] = (D.logc[0] + D.logK[0]) + E0;
    Lc[1] = (D.logc[1] + D.logK[1]) + E1;
    Lc[2] = (D.logc[2] + D.logK[2]) + E2;
    Lc[3] = ((D.logc[3] + D.logK[3]) + E0) + lds;
    double L4 = -INFINITY;
    int ncomp = 4;
    if (P) {
        const double loghalf = amm_log(0.5);
        double sumlogp = 0.0;
        for (int l = 0; l < M - 1; ++l) {
            uint32_t sl = masks[l];
            double tot = 0.0;
            for (int j = 0; j < M; ++j)
                if ((sl >> j) & 1u) tot = tot + (double)P[sl * M + j];
            sumlogp = sumlogp + amm_log((double)P[sl * M + path[l]] / tot);
        }
        L4 = ((loghalf + sumlogp) + lds) + E0;
        for (int ci = 0; ci < 4; ++ci) Lc[ci] = Lc[ci] + loghalf;
        ncomp = 5;
    }
    double a = Lc[0] > Lc[1] ? Lc[0] : Lc[1];
    double b = Lc[2] > Lc[3] ? Lc[2] : Lc[3];
    double Lmax = a > b ? a : b;
    if (ncomp == 5) Lmax = Lmax > L4 ? Lmax : L4;
    double S = 0.0;
    for (int ci = 0; ci < 4; ++ci) S = S + amm_exp(Lc[ci] - Lmax);
    if (ncomp == 5) S = S + amm_exp(L4 - Lmax);
    double Ltot = Lmax - sumlogz;
    double k = rint(Ltot * AMM_INV_LN2);
    double r = (Ltot - k * AMM_LN2_HI) - k * AMM_LN2_LO;
    double x0 = amm_exp(r) * S;
    int e;
    double xm = frexp(x0, &e);
    o.gx = xm;
    o.gj = (int)k + e;
    return o;
}
#pragma clang fp contract(on)

// ---------------------------------------------------------------------------
// Integrand: level quantities (LDL^T of the loop matrix), numerator
// polynomials, children combination, term sum.
// ---------------------------------------------------------------------------
struct PlanDev {
    const LevelDesc *levels;
    const TermDesc *terms;
    const int32_t *ops;
    const Mono *monos;
    const int2 *ranges;
    int nterms;
    int n;
    int ninsert;
    // FP64 interpreter tables: the group stream (four monomials per record,
    // see poly_groups) and, per range, its first word and number of records
    const uint32_t *gwords;
    const int2 *granges;
    int ngwords;
};

template <int N> struct Dims {
    static constexpr int KM = 2 * N;
    static constexpr int NV = KM * (KM + 1) / 2 + 2 * KM;
    static constexpr int NVL = NV + 1;      // LDS columns: the variables and the constant-1 slot
    static constexpr int DEPTH = 2 * N + 1;
    static_assert(NV == amm_nvars(N), "variable slots");
};

// Sum of the monomials coef * prod vars of one range.  Generic arithmetic,
// or, for T = ea, the value in FP64 with a first-order error bound: with
// rmax the largest relative error (units of u) of the level's variables, the
// product p = coef x_1 ... x_nv has relative error at most
// nv (rmax + 1) + 1 (its variables, its nv roundings, the rounded
// coefficient), and each accumulation adds |partial sum|.
// A monomial read with one 24-byte load into registers: coefficient, number
// of variables and their 15 index bytes (layout of Mono).
struct MonoRegs {
    double coef;
    uint64_t w1, w2;       // byte 0 of w1: nv; then v[0..6] in w1, v[7..14] in w2
    AMM_HDI int nv() const { return (int)(w1 & 0xffu); }
    AMM_HDI int var(int i) const { return (int)(i < 7 ? (w1 >> (8 * (i + 1))) : (w2 >> (8 * (i - 7)))) & 0xff; }
};
AMM_HDI MonoRegs load_mono(const Mono *p) {
    static_assert(sizeof(Mono) == 24, "Mono layout");
    MonoRegs r;
#if defined(__HIP_DEVICE_COMPILE__)
    // plan tables live in global memory: global loads, which (unlike flat
    // loads) do not hold up the waits for the LDS variable reads
    typedef const uint64_t __attribute__((address_space(1))) *gptr;
    const gptr q = (gptr)(const void *)p;
    r.coef = __builtin_bit_cast(double, q[0]);
    r.w1 = q[1];
    r.w2 = q[2];
#else
    __builtin_memcpy(&r, p, sizeof(Mono));
#endif
    return r;
}

// Index shared by the lanes of a wave.  The FP64 interpreter paths run every
// lane of a wave on the same graph, term and level (one graph per launch or
// per chunk), so the monomial ranges are wave-uniform and the table reads can
// be scalar.
AMM_HDI int wave_uniform(int x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(x);
#else
    return x;
#endif
}

// The FP64 interpreter's monomial table: the group stream.  Each range (the
// monomials of one (level, variant, output, c), sorted by degree) is cut into
// records of four consecutive monomials:
//   word 0      K, the largest degree of the four;  word 1: 0
//   words 2-9   the four coefficients (double, low word first; 0 past the
//               range's end)
//   words 10..  4K variable indices, factor-major: index i of monomial q at
//               10 + 4i + q; a monomial of degree below K, and a padding
//               monomial, use the constant-1 slot amm_nvars(n)
// so a record is 10 + 4K words.  Multiplying by the exact 1 leaves a product
// unchanged, so every monomial is still coef * x_1 ... x_nv in index order.
// The indices go to scalar registers with scalar loads: one vector address
// operation, one LDS read and one multiply per factor.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const uint32_t __attribute__((address_space(4))) *GroupWords;
AMM_HDI GroupWords uniform_words(const uint32_t *p) {
    const uint64_t a = (uint64_t)(const void *)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (GroupWords)(((uint64_t)hi << 32) | lo);
}
#else
typedef const uint32_t *GroupWords;
AMM_HDI GroupWords uniform_words(const uint32_t *p) { return p; }
#endif
constexpr int GROUP_HEAD = 10;

// Software prefetch of the group stream into L2.  Without it the scalar loads
// of the records wait on HBM every few records: the streams of a 4-loop graph
// set do not fit in L2, and each wave walks its graph's stream once per 64
// samples.  Every few records, lanes 0-15 load one word from each of the 16
// 64-byte lines that start 1 KB past the current record (clamped to the
// stream), through the vector memory path, whose counter the LDS waits do not
// share.  A loaded word is consumed (XORed into a carried word) at the next
// prefetch, before the new load is issued, so the load can land in the same
// register and its latency is never waited for in the loop; drain() consumes
// the last one at the end of a sample.
struct TablePf {
    uint32_t acc = 0, pend = 0;
};
AMM_HDI void table_prefetch(const PlanDev &P, int word, TablePf &pf) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t last = (uint32_t)P.ngwords - 1u;
    uint32_t w = (uint32_t)word + 256u + (threadIdx.x & 15u) * 16u;
    w = w < last ? w : last;
    typedef const uint32_t __attribute__((address_space(1))) *gptr;
    pf.acc ^= pf.pend;
    asm volatile("" : "+v"(pf.acc) : : "memory");
    pf.pend = *((gptr)(const void *)P.gwords + w);
#endif
}
AMM_HDI void table_drain(TablePf &pf) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t w = pf.acc ^ pf.pend;
    asm volatile("" ::"v"(w));
    pf.acc = pf.pend = 0;
#endif
}

// p[q] *= x_{I0} ... x_{I0+K-1} of monomial q of the record at w: the 4K LDS
// reads are issued together, then the products in index order.
template <int K, int I0, typename Vars>
AMM_HDI void group_factors(GroupWords w, const Vars &vars, double (&p)[4]) {
    double x[K][4];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) x[i][q] = vars.val((int)w[GROUP_HEAD + 4 * (I0 + i) + q]);
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) p[q] = p[q] * x[i][q];
}

// Sum of a range over its records in FP64 (Bound = false) or FP64 with the
// first-order bound, the four monomials of a record on four accumulators.
// The bound term of a monomial, |p| (nv (rmax + 1) + 1), is taken with the
// record's K for nv (at least the monomial's degree), one fma per monomial;
// each accumulation adds |partial sum|, and so does each addition of the four
// partial sums at the end.
template <bool Bound, typename Vars>
AMM_HDI void poly_groups(const PlanDev &P, int2 gr, Vars &vars, double r1, double &sum, double &err) {
    const int w0 = wave_uniform(gr.x), ng = wave_uniform(gr.y);
    const GroupWords W = uniform_words(P.gwords);
    double av[4] = {0.0, 0.0, 0.0, 0.0}, an[4] = {0.0, 0.0, 0.0, 0.0}, aa[4] = {0.0, 0.0, 0.0, 0.0};
    int off = w0;
    uint32_t touch = 0;
    const int lastw = P.ngwords - 1;
    for (int g = 0; g < ng; ++g) {
        if ((g & 7) == 0) table_prefetch(P, off, vars.pf);
        const GroupWords w = W + off;
        const int K = (int)w[0];
        {
            // bring the next record's two lines into the scalar cache while
            // this record's variable reads are in flight
            const int nx = off + GROUP_HEAD + 4 * K;
            const int n2 = nx + 16;
            touch ^= W[nx < lastw ? nx : lastw] ^ W[n2 < lastw ? n2 : lastw];
        }
        double p[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) p[q] = __builtin_bit_cast(double, (uint64_t)w[2 + 2 * q] | ((uint64_t)w[3 + 2 * q] << 32));
        switch (K) {
        case 0: break;
        case 1: group_factors<1, 0>(w, vars, p); break;
        case 2: group_factors<2, 0>(w, vars, p); break;
        case 3: group_factors<3, 0>(w, vars, p); break;
        case 4: group_factors<4, 0>(w, vars, p); break;
        case 5: group_factors<5, 0>(w, vars, p); break;
        case 6: group_factors<3, 0>(w, vars, p); group_factors<3, 3>(w, vars, p); break;
        case 7: group_factors<4, 0>(w, vars, p); group_factors<3, 4>(w, vars, p); break;
        case 8: group_factors<4, 0>(w, vars, p); group_factors<4, 4>(w, vars, p); break;
        default:
            group_factors<4, 0>(w, vars, p);
            group_factors<4, 4>(w, vars, p);
            for (int i = 8; i < K; ++i) {
#pragma unroll
                for (int q = 0; q < 4; ++q) p[q] = p[q] * vars.val((int)w[GROUP_HEAD + 4 * i + q]);
            }
        }
        const double cK = fma((double)K, r1, 1.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            av[q] = av[q] + p[q];
            if (Bound) {
                an[q] = fma(fabs(p[q]), cK, an[q]);
                aa[q] = aa[q] + fabs(av[q]);
            }
        }
        off += GROUP_HEAD + 4 * K;
    }
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::"s"(touch));
#endif
    const double s01 = av[0] + av[1], s23 = av[2] + av[3];
    sum = s01 + s23;
    if (Bound)
        err = ((an[0] + an[1]) + (an[2] + an[3])) + ((aa[0] + aa[1]) + (aa[2] + aa[3])) +
              ((fabs(s01) + fabs(s23)) + fabs(sum));
}

// Range table entry at a wave-uniform index (scalar load).
AMM_HDI int2 load_range_uniform(const int2 *t, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint64_t a = (uint64_t)(const void *)(t + wave_uniform(i));
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    typedef const int2 __attribute__((address_space(4))) *cptr;
    return *(cptr)(((uint64_t)hi << 32) | lo);
#else
    return t[i];
#endif
}

template <typename T, typename Vars>
AMM_HDI T poly_range(const PlanDev &P, int ri, Vars &vars, double rmax) {
    if constexpr (std::is_same<T, ea>::value) {
        double av = 0.0, ae = 0.0;
        poly_groups<true>(P, load_range_uniform(P.granges, ri), vars, rmax + 1.0, av, ae);
        return ea(av, ae);
    } else if constexpr (std::is_same<T, double>::value) {
        double av = 0.0, ae = 0.0;
        poly_groups<false>(P, load_range_uniform(P.granges, ri), vars, 0.0, av, ae);
        return av;
    } else if constexpr (std::is_same<T, dd>::value) {
        // two monomials per step on separate accumulators (independent
        // dependency chains), the next two already loading
        const int2 r = P.ranges[ri];
        dd acc0(0.0), acc1(0.0);
        const int m0 = r.x < r.y ? r.x : 0;
        MonoRegs na = load_mono(P.monos + m0);
        MonoRegs nb = load_mono(P.monos + (r.x + 1 < r.y ? r.x + 1 : m0));
        for (int m = r.x; m < r.y; m += 2) {
            const MonoRegs a = na, b = nb;
            const bool two = m + 1 < r.y;
            na = load_mono(P.monos + (m + 2 < r.y ? m + 2 : m));
            nb = load_mono(P.monos + (m + 3 < r.y ? m + 3 : m));
            const int ka = a.nv(), kb = two ? b.nv() : 0;
            dd ta = ka ? vars.get(a.var(0)) : dd(1.0);
            dd tb = kb ? vars.get(b.var(0)) : dd(1.0);
            const int kmax = ka > kb ? ka : kb;
            for (int i = 1; i < kmax; ++i) {
                // branch-free: past its degree a monomial reads variable 0 and
                // multiplies by exactly 1, so both reads issue together
                const bool ua = i < ka, ub = i < kb;
                dd xa = vars.get(ua ? a.var(i) : 0), xb = vars.get(ub ? b.var(i) : 0);
                xa.hi = ua ? xa.hi : 1.0;
                xa.lo = ua ? xa.lo : 0.0;
                xb.hi = ub ? xb.hi : 1.0;
                xb.lo = ub ? xb.lo : 0.0;
                ta = ta * xa;
                tb = tb * xb;
            }
            acc0 = mul_add(dd(a.coef), ta, acc0);
            if (two) acc1 = mul_add(dd(b.coef), tb, acc1);
        }
        return acc0 + acc1;
    } else {
        const int2 r = P.ranges[ri];
        T acc = T(0.0);
        for (int m = r.x; m < r.y; ++m) {
            const MonoRegs mo = load_mono(P.monos + m);
            const int nv = mo.nv();
            T t = nv ? vars.get(mo.var(0)) : T(1.0);
            for (int i = 1; i < nv; ++i) t = t * vars.get(mo.var(i));
            acc = mul_add(coef_of<T>(mo.coef), t, acc);
        }
        return acc;
    }
}

// Largest relative error bound of a level's variables 0..n-1 (ea only).
template <typename T, typename Vars>
AMM_HDI double level_rmax(const Vars &vars, int n) {
    if constexpr (std::is_same<T, ea>::value) return vars.max_rel(n);
    else return 0.0;
}

// Truncated convolution of two c-vectors of length N.
template <typename T, int N>
AMM_HDI void conv_into(const T *a, const T *b, T *out) {
    for (int c = 0; c < N; ++c) {
        T s = T(0.0);
        for (int i = 0; i <= c; ++i) s = mul_add(a[i], b[c - i], s);
        out[c] = s;
    }
}

// Storage of a level's polynomial variables.  VarsPriv keeps them in a
// private array (double-double path); VarsLds keeps one LDS column per thread
// (address base + i * stride, conflict-free for wave-uniform i).  For the
// magnitude type only the values are stored; the magnitude of a variable is
// |v| times the level's largest magnitude/value ratio.  Slot amm_nvars(n)
// holds the constant 1 that pads the FP64 group stream: VarsPriv sets it, the
// kernels set it in their LDS columns (set_one_slot) before evaluating.
template <typename T, int NV> struct VarsPriv {
    T v[NV + 1];            // the variables and the constant-1 slot
    TablePf pf;
    AMM_HDI VarsPriv() { v[NV] = T(1.0); }
    AMM_HDI void begin() {}
    AMM_HDI void drain() { table_drain(pf); }
    AMM_HDI void set(int i, const T &x) { v[i] = x; }
    AMM_HDI T get(int i) const { return v[i]; }
    AMM_HDI double val(int i) const { return to_double(v[i]); }
    AMM_HDI double max_rel(int n) const {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, relerr(v[i]));
        return m;
    }
};
struct VarsLdsD {
    double *base;
    int stride;
    TablePf pf;
    AMM_HDI void begin() {}
    AMM_HDI void drain() { table_drain(pf); }
    AMM_HDI void set(int i, double x) { base[i * stride] = x; }
    AMM_HDI double get(int i) const { return base[i * stride]; }
    AMM_HDI double val(int i) const { return base[i * stride]; }
};
template <int N>
AMM_HDI void set_one_slot(double *column, int stride) { column[Dims<N>::NV * stride] = 1.0; }
struct VarsLdsEa {
    double *base;      // values, one LDS column per thread
    int stride;
    double rmax;       // largest relative error bound of the variables set since begin()
    TablePf pf;
    AMM_HDI void begin() { rmax = 0.0; }
    AMM_HDI void drain() { table_drain(pf); }
    AMM_HDI void set(int i, const ea &x) {
        base[i * stride] = x.v;
        rmax = fmax(rmax, relerr(x));
    }
    AMM_HDI ea get(int i) const {
        double v = base[i * stride];
        return ea(v, fabs(v) * rmax);
    }
    AMM_HDI double val(int i) const { return base[i * stride]; }
    AMM_HDI double max_rel(int) const { return rmax; }
};

// Evaluate one level: c-vectors per output (pushed on the value stack) given
// the children's values on the stack.  Adds the level's V to vtot.
template <typename T, int N, typename Vars>
AMM_HDI void eval_level(const PlanDev &P, const LevelDesc &d, const double *z, T (*stk)[2][N], int &sp, T &vtot,
                        Vars &vars) {
    constexpr int KM = Dims<N>::KM;
    const int K = d.K, L = d.L;
    T zseg[KM + 1], zph[N];
#pragma unroll
    for (int k = 1; k <= KM; ++k) {
        if (k <= K) {
            double zz = z[d.seg_param[k - 1]];
            zseg[k] = d.seg_half[k - 1] ? T(zz * 0.5) : T(zz);
        } else {
            zseg[k] = T(0.0);
        }
    }
#pragma unroll
    for (int a = 0; a < N; ++a) zph[a] = a < L ? T(z[d.ph_param[a]]) : T(1.0);
    uint32_t span[N];
#pragma unroll
    for (int a = 0; a < N; ++a) span[a] = a < L ? d.span[a] : 0u;
    // loop matrix Lambda_ab = delta_ab z_gamma_a + sum_{k in span a & span b} z_k
    T Lam[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            T v = (a == b) ? zph[a] : T(0.0);
            uint32_t both = span[a] & span[b];
#pragma unroll
            for (int k = 1; k <= KM; ++k)
                if ((both >> (k - 1)) & 1u) v += zseg[k];
            Lam[a][b] = v;
        }
    // LDL^T (rows a >= L are decoupled identity-like rows with pivot z_ph = 1)
    T Lw[N][N], D[N], Dinv[N];
    T U = T(1.0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T di = Lam[i][i];
#pragma unroll
        for (int j = 0; j < i; ++j) di -= Lw[i][j] * Lw[i][j] * D[j];
        D[i] = di;
        if (i < L) U *= di;
        Dinv[i] = T(1.0) / di;
#pragma unroll
        for (int r = i + 1; r < N; ++r) {
            T v = Lam[r][i];
#pragma unroll
            for (int j = 0; j < i; ++j) v -= Lw[r][j] * Lw[i][j] * D[j];
            Lw[r][i] = v * Dinv[i];
        }
    }
    // y_k = L^{-1} s_k
    T y[KM + 1][N];
#pragma unroll
    for (int k = 1; k <= KM; ++k)
#pragma unroll
        for (int a = 0; a < N; ++a) {
            T v = ((span[a] >> (k - 1)) & 1u) ? T(1.0) : T(0.0);
#pragma unroll
            for (int b = 0; b < a; ++b) v -= Lw[a][b] * y[k][b];
            y[k][a] = v;
        }
    // sigma, w = L^{-1} sigma, V = sum w^2 / D
    T w[N];
    T V = T(0.0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
        T sg = T(0.0);
#pragma unroll
        for (int k = 1; k <= KM; ++k)
            if ((span[a] >> (k - 1)) & 1u) sg += zseg[k];
#pragma unroll
        for (int b = 0; b < a; ++b) sg -= Lw[a][b] * w[b];
        w[a] = sg;
        V += w[a] * w[a] * Dinv[a];
    }
    vtot += strip(V);
    U = strip(U);
#pragma unroll
    for (int a = 0; a < N; ++a) {
        w[a] = strip(w[a]);
        Dinv[a] = strip(Dinv[a]);
#pragma unroll
        for (int k = 1; k <= KM; ++k) y[k][a] = strip(y[k][a]);
    }
    vars.begin();
    const int XN = amm_xn(K);
#pragma unroll
    for (int k = 1; k <= KM; ++k) {
        if (k > K) break;
#pragma unroll
        for (int k2 = k; k2 <= KM; ++k2) {
            if (k2 > K) break;
            T s = T(0.0);
#pragma unroll
            for (int a = 0; a < N; ++a) s += y[k][a] * y[k2][a] * Dinv[a];
            vars.set(amm_xidx(K, k, k2), s);
        }
        T s = T(0.0);
#pragma unroll
        for (int a = 0; a < N; ++a) s += y[k][a] * w[a] * Dinv[a];
        vars.set(XN + k - 1, T(1.0) - s);
    }
    if (d.op == OP_A) {
        T wc[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            T jc = T(0.0);
#pragma unroll
            for (int k = 1; k <= KM; ++k)
                if ((span[a] >> (k - 1)) & 1u) jc += zseg[k] * T(k <= d.ext_node ? -0.5 : 0.5);
#pragma unroll
            for (int b = 0; b < a; ++b) jc -= Lw[a][b] * wc[b];
            wc[a] = jc;
        }
#pragma unroll
        for (int a = 0; a < N; ++a) wc[a] = strip(wc[a]);
#pragma unroll
        for (int k = 1; k <= KM; ++k) {
            if (k > K) break;
            T s = T(0.0);
#pragma unroll
            for (int a = 0; a < N; ++a) s += y[k][a] * wc[a] * Dinv[a];
            vars.set(XN + K + k - 1, T(k <= d.ext_node ? -0.5 : 0.5) - s);
        }
    }
    const double rmax = level_rmax<T>(vars, d.op == OP_A ? XN + 2 * K : XN + K);
    // prefactor per c: pref (-1/2)^c / U^2 (* z_e for the merged line)
    T base = T(d.pref) / (U * U);
    if (d.has_X) {
#pragma unroll
        for (int k = 1; k <= KM; ++k)
            if (k <= K && d.seg_half[k - 1]) { base = base * (zseg[k] + zseg[k]); break; }
    }
    // children: on stack at sp - nkids .. sp - 1 (node order)
    const int nk = d.nkids;
    const int kid0 = sp - nk;
    T prodV[N];
    prodV[0] = T(1.0);
#pragma unroll
    for (int c = 1; c < N; ++c) prodV[c] = T(0.0);
    for (int q = 0; q < nk; ++q) {
        if ((d.kid_is_se >> q) & 1u) continue;
        T tmp[N];
        conv_into<T, N>(prodV, stk[kid0 + q][0], tmp);
#pragma unroll
        for (int c = 0; c < N; ++c) prodV[c] = tmp[c];
    }
    T res[2][N];
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int c = 0; c < N; ++c) res[o][c] = T(0.0);
    for (int var = 0; var < d.nvariants; ++var) {
        // product of SE children's chosen outputs
        T sev[N];
#pragma unroll
        for (int c = 0; c < N; ++c) sev[c] = prodV[c];
        int bit = 0;
        for (int q = 0; q < nk; ++q) {
            if (!((d.kid_is_se >> q) & 1u)) continue;
            int ch = (var >> bit) & 1;
            ++bit;
            T tmp[N];
            if (ch) conv_into<T, N>(sev, stk[kid0 + q][1], tmp);
            else conv_into<T, N>(sev, stk[kid0 + q][0], tmp);
#pragma unroll
            for (int c = 0; c < N; ++c) sev[c] = tmp[c];
        }
        for (int o = 0; o < 2; ++o) {
            if (o >= d.nout) break;
            T own[N];
            T fac = base;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                T acc = poly_range<T>(P, d.mono_range + (var * d.nout + o) * (P.n + 1) + c, vars, rmax);
                own[c] = acc * fac;
                fac = fac * T(-0.5);
            }
#ifdef AMM_DEBUG_LEVELS
            printf("  level op%d var%d out%d own:", d.op, var, o);
            for (int c = 0; c < N; ++c) printf(" %.10g", to_double(own[c]));
            printf(" U %.10g V-so-far %.10g\n", to_double(U), to_double(vtot));
#endif
            T tmp[N];
            conv_into<T, N>(own, sev, tmp);
#pragma unroll
            for (int c = 0; c < N; ++c) res[o][c] += tmp[c];
        }
    }
    sp = kid0;
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int c = 0; c < N; ++c) stk[sp][o][c] = res[o][c];
    ++sp;
}

// Insertion integrands of one SE graph at z summed over the forest terms
// t0, t0 + tstep, ... (eq. for R^new): I[e], and sum |term| absI[e].
template <typename T, int N, typename Vars>
AMM_HDI void eval_graph(const PlanDev &P, const double *z, T *I, T *absI, Vars &vars, int t0 = 0, int tstep = 1) {
    for (int e = 0; e < P.ninsert; ++e) { I[e] = T(0.0); absI[e] = T(0.0); }
    T stk[Dims<N>::DEPTH][2][N];
    for (int t = t0; t < P.nterms; t += tstep) {
        const TermDesc td = P.terms[t];
        int sp = 0;
        T vtot = T(0.0);
        for (int o = td.op_begin; o < td.op_end; ++o) {
            const LevelDesc &d = P.levels[P.ops[o]];
            eval_level<T, N>(P, d, z, stk, sp, vtot, vars);
        }
        // sum_c vec[c] Gamma(n-c) / V^{n-c}
        T val = T(0.0);
        T vinv = T(1.0) / vtot;
        T vp = vinv;                     // V^-(n-c) built from c = n-1 down
        double gam = 1.0;                // Gamma(n-c) = (n-c-1)!
#pragma unroll
        for (int c = N - 1; c >= 0; --c) {
            val = mul_add(stk[0][0][c] * T(gam), vp, val);
            vp = vp * vinv;
            gam = gam * (double)(N - c);
        }
        T sv = td.sign > 0 ? val : -val;
        I[td.e] += sv;
        absI[td.e] += absd(val);
    }
    vars.drain();
}

// Private-storage convenience overload (host tests, double-double path).
template <typename T, int N>
AMM_HDI void eval_graph(const PlanDev &P, const double *z, T *I, T *absI) {
    VarsPriv<T, Dims<N>::NV> vars;
    eval_graph<T, N>(P, z, I, absI, vars);
}

}  // namespace amm
