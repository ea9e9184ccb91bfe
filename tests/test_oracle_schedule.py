"""Pins of the oracle's adaptive sample split (Sec. IV.C) and parity of the
library's host split with it.

The split is pinned by what fixes it mathematically: the minimum of
sum_j C_j^2 / n_j at fixed cost found by a general-purpose constrained
optimiser, first-order optimality under cost-preserving moves, the equal split
at floor 1 or with no variance information, and the paper's probabilities."""
import math
import os

import numpy as np
import pytest

from oracle import schedule as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, 'paper_1909_08015_amd', 'libamm.so')


def _instance(seed, n=7):
    rng = np.random.default_rng(seed)
    C = list(np.exp(rng.normal(0.0, 1.5, n)))
    t = list(np.exp(rng.normal(0.0, 1.0, n)) * 1e4)
    return C, t


@pytest.mark.parametrize('seed', [0, 1, 2])
def test_neyman_split_is_the_constrained_minimum(seed):
    from scipy.optimize import minimize
    C, t = _instance(seed)
    C, t = np.array(C), np.array(t)
    budget = 1e9
    x = np.array(S.split_real(list(C), list(t), budget, 0.0))
    # numerical minimum of sum C^2/n subject to sum n t = budget (scaled variables)
    n0 = budget / t.sum()

    def var(u):
        return float(np.sum(C ** 2 / (u * n0)))

    res = minimize(var, np.ones(len(C)), method='SLSQP', bounds=[(1e-6, None)] * len(C),
                   constraints=[dict(type='eq', fun=lambda u: float(np.dot(u * n0, t) / budget - 1.0))],
                   options=dict(ftol=1e-14, maxiter=500))
    assert res.success
    assert np.allclose(x, res.x * n0, rtol=2e-3)
    assert var(x / n0) <= res.fun * (1 + 1e-9)
    assert abs(np.dot(x, t) - budget) <= 1e-12 * budget


def test_cost_preserving_moves_raise_the_variance():
    C, t = _instance(5)
    budget = 1e8
    x = np.array(S.split_real(C, t, budget, 0.0))
    C, t = np.array(C), np.array(t)
    v0 = np.sum(C ** 2 / x)
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, k = rng.choice(len(C), 2, replace=False)
        d = rng.uniform(-0.2, 0.2) * x[i]
        y = x.copy()
        y[i] += d
        y[k] -= d * t[i] / t[k]
        if y[k] <= 0:
            continue
        assert np.sum(C ** 2 / y) >= v0 * (1 - 1e-12)


def test_paper_probabilities_and_mixture():
    C, t = _instance(3)
    budget = 5e7
    x = S.split_real(C, t, budget, 0.0)
    p = S.shares(C, t)
    for j in range(len(C)):
        assert math.isclose(x[j] / sum(x), p[j], rel_tol=1e-12)
    eq = budget / sum(t)
    for f in (0.1, 0.5):
        y = S.split_real(C, t, budget, f)
        for j in range(len(C)):
            assert math.isclose(y[j], f * eq + (1 - f) * x[j], rel_tol=1e-12)


def test_equal_split_cases():
    C, t = _instance(4)
    budget = 3.3e7
    eq = math.floor(budget / sum(t))
    assert S.split(C, t, budget, 1.0) == [eq] * len(C)
    assert S.split([0.0] * len(C), t, budget, 0.0) == [eq] * len(C)
    n = S.split(C, t, budget, 0.3)
    assert sum(a * b for a, b in zip(n, t)) <= budget
    assert S.split(C, t, 0.0, 0.3) == [0] * len(C)


@pytest.mark.skipif(not os.path.exists(LIB), reason='libamm.so not built')
def test_library_split_matches_oracle_exactly():
    """amm_adaptive_split is host code: callable without a GPU."""
    from paper_1909_08015_amd.amm import adaptive_split, AmmError
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(1, 80))
        C = list(np.exp(rng.normal(0, 2, n)) * (rng.random(n) > 0.1))
        t = list(np.exp(rng.normal(8, 1.5, n)))
        budget = float(np.exp(rng.uniform(0, 40)))
        f = float(rng.choice([0.0, 0.25, rng.random(), 1.0]))
        assert adaptive_split(C, t, budget, f) == S.split(C, t, budget, f), trial
    with pytest.raises(AmmError):
        adaptive_split([1.0], [0.0], 1.0, 0.0)
    with pytest.raises(AmmError):
        adaptive_split([1.0], [1.0], 1.0, 1.5)
    with pytest.raises(AmmError):
        adaptive_split([-1.0], [1.0], 1.0, 0.0)
