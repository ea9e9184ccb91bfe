"""Oracle: graph-by-graph combination of two independent calculations.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Sec. V: the two calculations (different generators and density constants)
are first combined graph by graph, then summed over graphs with eq.
sigma_sum.  Reading: the per-graph combination is the inverse-variance
weighted mean, m = (m1/s1^2 + m2/s2^2) / (1/s1^2 + 1/s2^2), with
s^2 = 1 / (1/s1^2 + 1/s2^2); a calculation with sigma 0 (no spread seen)
gets all the weight, and two such give the plain average with sigma 0.
"""
from __future__ import annotations

import math


def combine_graph(m1, s1, m2, s2):
    if s1 == 0.0 and s2 == 0.0:
        return 0.5 * (m1 + m2), 0.0
    if s1 == 0.0:
        return m1, 0.0
    if s2 == 0.0:
        return m2, 0.0
    w1 = 1.0 / (s1 * s1)
    w2 = 1.0 / (s2 * s2)
    w = w1 + w2
    return (m1 * w1 + m2 * w2) / w, math.sqrt(1.0 / w)


def combine(means1, sigmas1, means2, sigmas2):
    """Per-graph combination, then the sum over graphs (eq. sigma_sum):
    returns (per-graph means, per-graph sigmas, total mean, total sigma)."""
    ms, ss = [], []
    for a, b, c, d in zip(means1, sigmas1, means2, sigmas2):
        m, s = combine_graph(a, b, c, d)
        ms.append(m)
        ss.append(s)
    return ms, ss, sum(ms), math.sqrt(sum(s * s for s in ss))
