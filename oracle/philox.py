"""Oracle: Philox4x32-10 counter-based generator and the sample stream layout.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random
numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 bit
multiplies with the Weyl key schedule.  The paper's second calculation used a
Philox_4x32_10 stream (Sec. V); the stream layout below is this project's own
(reading R10): it does not reproduce any vendor library's sequence.

Layout:
  key     = (seed_lo ^ graph_uid, seed_hi)
  counter = (sample_lo, sample_hi, block, 0)
  block b yields two uniforms: u_{2b} from words (0, 1), u_{2b+1} from (2, 3),
  u = ((w_a >> 6) * 2^26 + (w_b >> 6) + 1/2) * 2^-52   in (0, 1), exact.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised over numpy uint64 arrays holding 32-bit words.

    ctr: 4 arrays, key: 2 arrays (or ints).  Returns 4 arrays."""
    c0, c1, c2, c3 = [np.asarray(c, dtype=np.uint64) & MASK for c in ctr]
    k0, k1 = [np.asarray(k, dtype=np.uint64) & MASK for k in key]
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def graph_uid(loops, gi):
    return (loops << 20) | gi


def uniform_pair(w_a, w_b):
    a = (np.asarray(w_a, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    b = (np.asarray(w_b, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b + 0.5) * (2.0 ** -52)


def uniforms(seed, uid, sample_idx, count):
    """count uniforms per sample for the given sample indices (uint64 array).

    Returns an array of shape (len(sample_idx), count)."""
    s = np.asarray(sample_idx, dtype=np.uint64)
    key0 = (seed & MASK) ^ uid
    key1 = (seed >> 32) & MASK
    out = np.empty((s.shape[0], count), dtype=np.float64)
    nblk = (count + 1) // 2
    lo = s & np.uint64(MASK)
    hi = s >> np.uint64(32)
    zero = np.zeros_like(s)
    for b in range(nblk):
        w = philox4x32_10((lo, hi, zero + np.uint64(b), zero), (key0, key1))
        out[:, 2 * b] = uniform_pair(w[0], w[1])
        if 2 * b + 1 < count:
            out[:, 2 * b + 1] = uniform_pair(w[2], w[3])
    return out
