"""Oracle: the MRG32k3a generator as counter-addressed streams (Calc 1).

TEST INFRASTRUCTURE (see oracle/graphs.py).

Sec. V: the first of the paper's two calculations draws its samples with
MRG32k3a (L'Ecuyer, Operations Research 47 (1999) 159), the second with
Philox4x32-10.  MRG32k3a combines two order-3 recurrences

    x1[n] = (a12 x1[n-2] - a13 x1[n-3]) mod m1,  m1 = 2^32 - 209,
    x2[n] = (a21 x2[n-1] - a23 x2[n-3]) mod m2,  m2 = 2^32 - 22853,

with output z[n] = (x1[n] - x2[n]) mod m1.  A state is the pair of vectors
(x[n-3], x[n-2], x[n-1]); one step multiplies each by its companion matrix,
so n steps are a matrix power (jump ahead).

Stream layout (a reading: the paper uses the library's own layout, which is
not reproduced; any layout of disjoint substreams serves):
  * the seed gives the start state s0 = ((1 + lo mod (m1 - 1), 12345, 12345),
    (1 + hi mod (m2 - 1), 12345, 12345)), lo/hi the seed's 32-bit halves;
  * graph uid starts uid * 2^100 steps after s0;
  * sample i of a graph starts i * 2^7 steps after the graph's start and
    uses the next 2 * count outputs (count <= 64);
  * uniform k of a sample is ((za >> 1) 2^21 + (zb >> 11) + 1/2) 2^-52 from its
    outputs za = z[2k + 1], zb = z[2k + 2]: 52 random bits, exact in FP64 and
    strictly inside (0, 1) (za < m1 < 2^32).
"""
from __future__ import annotations

import numpy as np

M1 = 4294967087
M2 = 4294944443
A12, A13 = 1403580, 810728
A21, A23 = 527612, 1370589

# companion matrices acting on (x[n-3], x[n-2], x[n-1])
MAT1 = ((0, 1, 0), (0, 0, 1), ((-A13) % M1, A12, 0))
MAT2 = ((0, 1, 0), (0, 0, 1), ((-A23) % M2, 0, A21))

SAMPLE_SHIFT = 7
GRAPH_SHIFT = 100


def mat_mul(a, b, m):
    return tuple(tuple(sum(a[i][k] * b[k][j] for k in range(3)) % m for j in range(3)) for i in range(3))


def mat_vec(a, v, m):
    return tuple(sum(a[i][k] * v[k] for k in range(3)) % m for i in range(3))


def mat_pow(a, e, m):
    """a^e mod m by binary exponentiation."""
    r = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    while e:
        if e & 1:
            r = mat_mul(r, a, m)
        a = mat_mul(a, a, m)
        e >>= 1
    return r


def step(state):
    """One step of both recurrences; returns (new state, output z)."""
    (p0, p1, p2), (q0, q1, q2) = state
    x1 = (A12 * p1 - A13 * p0) % M1
    x2 = (A21 * q2 - A23 * q0) % M2
    return ((p1, p2, x1), (q1, q2, x2)), (x1 - x2) % M1


def jump(state, e):
    """The state e steps later."""
    return (mat_vec(mat_pow(MAT1, e, M1), state[0], M1), mat_vec(mat_pow(MAT2, e, M2), state[1], M2))


def seed_state(seed):
    lo, hi = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    return ((1 + lo % (M1 - 1), 12345, 12345), (1 + hi % (M2 - 1), 12345, 12345))


def graph_state(seed, uid):
    return jump(seed_state(seed), uid << GRAPH_SHIFT)


def uniform_of(za, zb):
    k = ((za >> 1) << 21) + (zb >> 11)
    return (k + 0.5) * 2.0 ** -52


def sample_uniforms(gstate, idx, count):
    """count uniforms of sample idx of the graph whose start state is gstate."""
    s = jump(gstate, int(idx) << SAMPLE_SHIFT)
    out = []
    for _ in range(count):
        s, za = step(s)
        s, zb = step(s)
        out.append(uniform_of(za, zb))
    return out


def uniforms(seed, uid, sample_idx, count):
    """Same interface as oracle.philox.uniforms: (len(sample_idx), count)."""
    g = graph_state(seed, uid)
    return np.array([sample_uniforms(g, i, count) for i in np.asarray(sample_idx, dtype=np.uint64)],
                    dtype=np.float64).reshape(len(sample_idx), count)
