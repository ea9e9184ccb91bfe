"""Pins of the estimator pieces of the oracle (Sec. III.B, Sec. IV.A)."""
import math

import numpy as np
import pytest

from oracle import estimate as E


def test_accept_thresholds_closed_forms():
    """eq. (interval_accept): tau_j = (1/4) s_j sqrt(sum s^2) / sum s.
    Equal sigmas over G graphs give s / (4 sqrt(G)); the thresholds add up to
    a quarter of the total sigma sqrt(sum s^2) (eq. sigma_sum), which is what
    the criterion allots to round-off; sigmas scale with sqrt(N_pilot/N_run)."""
    for G in (1, 3, 10):
        tau = E.accept_thresholds([2.0] * G, 400, 100)
        assert np.allclose(tau, 2.0 * 2.0 / (4 * math.sqrt(G)), rtol=1e-15)
    rng = np.random.default_rng(5)
    s = rng.random(17) * 3
    tau = E.accept_thresholds(s, 1000, 1000)
    assert tau.sum() == pytest.approx(0.25 * math.sqrt((s * s).sum()), rel=1e-14)
    assert np.all(np.diff(tau[np.argsort(s)]) >= 0)          # monotone in sigma_j
    assert np.all(np.isinf(E.accept_thresholds([0.0, 0.0], 10, 10)))


def test_flagged_estimate_takes_the_reference_where_the_bound_fails():
    rng = np.random.default_rng(2)
    y = rng.normal(size=(1000, 3))
    ref = y + 1e-9 * rng.normal(size=y.shape)
    b = np.abs(rng.normal(size=y.shape)) * 1e-3
    b[5, 1] = np.inf
    y[7, 2] = np.nan
    out, flag = E.flagged_estimate(y, b, ref, tau=2e-3)
    expect = (b.sum(1) > 2e-3) | np.isnan(y).any(1)
    assert np.array_equal(flag, expect) and flag[5] and flag[7]
    assert np.array_equal(out[flag], ref[flag]) and np.array_equal(out[~flag], y[~flag])


def test_graph_total_carries_the_insertion_covariance():
    """All insertions of an SE graph are evaluated at the same point, so the
    graph's variance is that of the per-point total, not the sum of the
    per-insertion (or per-class) variances.  At 2 loops the insertions are
    strongly correlated: the two differ, and the per-point total equals the
    sum of the class sums."""
    for gi in range(2):
        a = E.run(2, gi, 0, 0, 40000)
        m, s = E.mean_sigma(a['tsum'], a['tsum2'], a['n'])
        assert a['tsum'] == pytest.approx(sum(a['csum'].values()), rel=1e-12, abs=1e-12)
        var_cls = sum(E.mean_sigma(a['csum'][c], a['csum2'][c], a['n'])[1] ** 2 for c in a['csum'])
        var_ins = float((E.mean_sigma(a['sum'], a['sum2'], a['n'])[1] ** 2).sum())
        assert abs(s ** 2 - var_cls) > 0.05 * var_cls
        assert abs(s ** 2 - var_ins) > 0.05 * var_ins
