"""Oracle: exp and log with a fixed, published evaluation order.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Sample points must be bit-identical between independent implementations, so
neither side may call a vendor math library.  Both follow the same textbook
methods, operation by operation, with every operation an IEEE-754 double
operation rounded to nearest (no fused multiply-add):

exp(x): Cody & Waite argument reduction (Software Manual for the Elementary
  Functions, 1980): k = rint(x / ln2), r = (x - k*LN2_HI) - k*LN2_LO, then the
  Taylor polynomial sum_{i<=13} r^i / i! by Horner with c_0 = 1,
  c_i = c_{i-1} / i, and the result scaled by 2^k.
log(x): x = m 2^k with m in [sqrt(1/2), sqrt(2)), f = (m-1)/(m+1),
  log m = 2 f sum_{i<=11} f^{2i}/(2i+1) (the atanh series) by Horner in s = f^2
  with d_i = 1/(2i+1); log x = (k*LN2_LO + log m) + k*LN2_HI.

LN2_HI has its low 32 bits zero so that k*LN2_HI is exact for |k| < 2^20
(the split used by Cody & Waite and by fdlibm).
"""
from __future__ import annotations

import numpy as np

LN2_HI = 6.93147180369123816490e-01
LN2_LO = 1.90821492927058770002e-10
INV_LN2 = 1.44269504088896338700e+00
SQRT_HALF = 0.70710678118654752440

EXP_C = [1.0]
for _i in range(1, 14):
    EXP_C.append(EXP_C[-1] / float(_i))
LOG_D = [1.0 / float(2 * i + 1) for i in range(12)]


def amm_exp(x):
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(all='ignore'):
        k = np.rint(x * INV_LN2)
        r = (x - k * LN2_HI) - k * LN2_LO
        p = np.full_like(r, EXP_C[13])
        for i in range(12, -1, -1):
            p = p * r + EXP_C[i]
        kk = np.nan_to_num(np.clip(k, -2000, 2000)).astype(np.int64)
        out = np.ldexp(p, kk)
    out = np.where(x < -745.2, 0.0, out)
    out = np.where(x > 709.78, np.inf, out)
    return out


def amm_log(x):
    x = np.asarray(x, dtype=np.float64)
    m, k = np.frexp(x)
    small = m < SQRT_HALF
    m = np.where(small, m * 2.0, m)
    k = np.where(small, k - 1, k).astype(np.float64)
    f = (m - 1.0) / (m + 1.0)
    s = f * f
    q = np.full_like(s, LOG_D[11])
    for i in range(10, -1, -1):
        q = q * s + LOG_D[i]
    lm = (2.0 * f) * q
    return (k * LN2_LO + lm) + k * LN2_HI
