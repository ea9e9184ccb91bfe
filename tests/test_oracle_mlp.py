"""Oracle pins for the learned sector sampler (FP64)."""
import math

import numpy as np
import pytest

from oracle import graphs as G
from oracle import mlp as OM
from oracle import sampler as S
from oracle.philox import uniforms, graph_uid


def _setup(seed=3):
    rows, X, goff = OM.rows_and_features(2, 0)
    rng = np.random.default_rng(seed)
    p = OM.init_params(rng.random(OM.NPARAM)).astype(np.float64)
    p[OM.NPARAM - 65:] = rng.random(65) - 0.5
    w = rng.random(len(rows)) ** 2
    w /= w.sum()
    return rows, X.astype(np.float64), goff, p, w


def test_backprop_matches_finite_differences():
    rows, X, goff, p, w = _setup()
    _, g = OM.loss_and_grad(p, X, w, goff)
    rng = np.random.default_rng(1)
    for idx in rng.choice(OM.NPARAM, 40, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (OM.loss_and_grad(pp, X, w, goff)[0] - OM.loss_and_grad(pm, X, w, goff)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-5, abs=1e-9)


def test_zero_last_layer_reproduces_plain_sector_probabilities():
    rows, X, goff = OM.rows_and_features(2, 1)
    p = OM.init_params(np.random.default_rng(0).random(OM.NPARAM))
    d, _ = OM.forward(p, X)
    P = OM.group_softmax(X[:, 0].astype(np.float64) + d, goff)
    dens = S.Density(2, G.se_graphs(2)[1])
    for (s, j), pr in zip(rows, P):
        tot = sum(dens.W1[s & ~(1 << k)] for k in range(dens.M) if (s >> k) & 1)
        assert pr == pytest.approx(dens.W1[s & ~(1 << j)] / tot, rel=1e-6)


def test_learned_mixture_is_a_normalised_density():
    n, gi = 2, 1
    d = S.Density(n, G.se_graphs(n)[gi])
    M = d.M
    tab = (0.05 + 0.95 * np.random.default_rng(4).random((1 << M, M))).astype(np.float32)
    u = uniforms(0, graph_uid(n, gi), np.arange(200000, dtype=np.uint64), 2 * M)
    out = d.sample(u, tab)
    assert set(np.unique(out['comp'])) <= {0, 1, 2, 3, 4}
    assert abs((out['comp'] == 4).mean() - 0.5) < 0.01
    q = np.ldexp(out['gx'], out['gj'])
    w = math.factorial(M - 1) / q
    assert abs(w.mean() - 1) < 5 * w.std() / math.sqrt(len(w))
