"""Oracle: adaptive distribution of Monte Carlo samples over the graphs.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Sec. IV.C: graph j has the per-sample standard deviation C_j = sigma_j
sqrt(N_j) (sigma_j after N_j samples, eq. sigma_down) and an average cost
t_j per sample.  The next sample goes to graph j with probability
p_j = (C_j / sqrt(t_j)) / sum_l (C_l / sqrt(t_l)).  A cost T spent that way
gives graph j about n_j = T p_j / sum_l p_l t_l samples; this minimises the
variance sum_j C_j^2 / n_j of the summed estimate (eq. sigma_sum) at fixed
cost sum_j n_j t_j = T.

The paper stabilises the choice by giving a little more weight to graphs
whose sigma may be underestimated, judged by a sigma estimate defined in
another paper.  Here (a reading) a share f of each round's cost is split
equally over the graphs instead.

Rounds (the deterministic form of the paper's random choice of graphs): a
first round of equal sample counts, then rounds that each spend an equal part
of the remaining cost, split by the current C_j.
"""
from __future__ import annotations

import math


def shares(C, t):
    """p_j of Sec. IV.C (all C_j = 0: equal shares)."""
    w = [c / math.sqrt(x) for c, x in zip(C, t)]
    s = sum(w)
    if s == 0.0:
        return [1.0 / len(C)] * len(C)
    return [v / s for v in w]


def split_real(C, t, budget, floor_frac):
    """Real-valued sample counts of one round of cost `budget`: a share
    floor_frac split equally, the rest in proportion to p_j.

    Evaluated step by step in FP64 in a fixed order, so that the integer
    split below is reproducible exactly."""
    st = 0.0
    for x in t:
        st = st + x
    w = []
    swt = 0.0
    for c, x in zip(C, t):
        r = math.sqrt(x)
        w.append(c / r)
        wt = w[-1] * x
        swt = swt + wt
    f = floor_frac if swt > 0.0 else 1.0
    eq = budget / st
    out = []
    for wj in w:
        v = f * eq
        if swt > 0.0:
            ney = budget * wj
            ney = ney / swt
            ney = ney * (1.0 - f)
            v = v + ney
        out.append(v)
    return out


def split(C, t, budget, floor_frac):
    """Integer sample counts of one round: floor of split_real."""
    return [int(math.floor(v)) for v in split_real(C, t, budget, floor_frac)]


def round_budgets(total, spent, rounds_left):
    """Cost of the next round: an equal part of what is left."""
    return (total - spent) / rounds_left
