"""Pins of the second calculation's pieces (Sec. V): the MRG32k3a
generator as counter-addressed streams, and the graph-by-graph combination of
two calculations."""
import math

import numpy as np
import pytest

from oracle import mrg32k3a as R
from oracle import combine as K

I3 = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def test_component_recurrences_have_full_period_order():
    """Each component's characteristic polynomial is primitive modulo its
    prime, so the companion matrix has order m^3 - 1: its power m^3 - 1 is the
    identity (a wrong multiplier or modulus fails this), and the power
    (m^3 - 1) / (m - 1) is not (it is a scalar matrix, the norm)."""
    for mat, m in ((R.MAT1, R.M1), (R.MAT2, R.M2)):
        assert R.mat_pow(mat, m ** 3 - 1, m) == I3
        p = R.mat_pow(mat, (m ** 3 - 1) // (m - 1), m)
        assert p != I3
        assert p[0][1] == p[0][2] == p[1][0] == p[1][2] == p[2][0] == p[2][1] == 0 and p[0][0] == p[1][1] == p[2][2]


def test_jump_equals_stepping():
    rng = np.random.default_rng(3)
    for e in (0, 1, 2, 3, 17, 1000, 4321):
        s = ((int(rng.integers(1, R.M1)), int(rng.integers(0, R.M1)), int(rng.integers(0, R.M1))),
             (int(rng.integers(1, R.M2)), int(rng.integers(0, R.M2)), int(rng.integers(0, R.M2))))
        t = s
        for _ in range(e):
            t, _ = R.step(t)
        assert R.jump(s, e) == t, e


def test_samples_are_consecutive_disjoint_windows():
    g = R.graph_state(0x1234_5678_9ABC_DEF0, (3 << 20) | 5)
    s = R.jump(g, 41 << R.SAMPLE_SHIFT)
    outs = []
    for _ in range(1 << R.SAMPLE_SHIFT):
        s, z = R.step(s)
        outs.append(z)
    assert s == R.jump(g, 42 << R.SAMPLE_SHIFT)           # next sample starts where this window ends
    u = R.sample_uniforms(g, 41, 5)
    assert u == [R.uniform_of(outs[2 * k], outs[2 * k + 1]) for k in range(5)]


def test_uniforms_are_in_the_open_interval_and_uniform():
    u = R.uniforms(7, (2 << 20) | 1, np.arange(4000, dtype=np.uint64), 5).ravel()
    assert np.all(u > 0.0) and np.all(u < 1.0)
    n = u.size
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 5 * math.sqrt(1 / 180 / n)
    # extremes of the mapping
    assert R.uniform_of(0, 0) == 2.0 ** -53
    assert R.uniform_of(R.M1 - 1, R.M1 - 1) < 1.0
    # different graphs and seeds give different streams
    a = R.uniforms(7, 1, np.arange(3, dtype=np.uint64), 4)
    assert not np.array_equal(a, R.uniforms(7, 2, np.arange(3, dtype=np.uint64), 4))
    assert not np.array_equal(a, R.uniforms(8, 1, np.arange(3, dtype=np.uint64), 4))


def test_combination_special_cases():
    m, s = K.combine_graph(1.0, 2.0, 3.0, 2.0)
    assert m == 2.0 and math.isclose(s, math.sqrt(2.0))
    m, s = K.combine_graph(1.0, 1.0, 5.0, 1e9)
    assert math.isclose(m, 1.0, rel_tol=1e-12) and math.isclose(s, 1.0, rel_tol=1e-12)
    assert K.combine_graph(1.0, 0.0, 5.0, 1.0) == (1.0, 0.0)
    assert K.combine_graph(1.0, 0.0, 5.0, 0.0) == (3.0, 0.0)
    # symmetric in the two calculations; the weighted mean is the
    # minimum-variance unbiased combination: any other weight does worse
    m1, s1, m2, s2 = 0.3, 0.2, 0.5, 0.1
    assert K.combine_graph(m1, s1, m2, s2) == pytest.approx(K.combine_graph(m2, s2, m1, s1), rel=1e-15)
    _, s = K.combine_graph(m1, s1, m2, s2)
    for lam in np.linspace(0, 1, 21):
        assert (lam * s1) ** 2 + ((1 - lam) * s2) ** 2 >= s * s * (1 - 1e-12)


def test_combination_sums_graphs_after_combining():
    ms, ss, tm, ts = K.combine([1.0, 2.0], [1.0, 1.0], [3.0, 2.0], [1.0, 1.0])
    assert ms == [2.0, 2.0] and tm == 4.0 and math.isclose(ts, 1.0)


LIB = __import__('os').path.join(__import__('os').path.dirname(__import__('os').path.dirname(
    __import__('os').path.abspath(__file__))), 'paper_1909_08015_amd', 'libamm.so')


@pytest.mark.skipif(not __import__('os').path.exists(LIB), reason='libamm.so not built')
def test_library_combination_matches_oracle_exactly():
    """amm_combine is host code: callable without a GPU."""
    from paper_1909_08015_amd.amm import combine, AmmError
    rng = np.random.default_rng(5)
    for trial in range(100):
        n = int(rng.integers(1, 80))
        m1, m2 = list(rng.normal(0, 3, n)), list(rng.normal(0, 3, n))
        s1 = list(np.exp(rng.normal(-2, 2, n)) * (rng.random(n) > 0.05))
        s2 = list(np.exp(rng.normal(-2, 2, n)) * (rng.random(n) > 0.05))
        assert combine(m1, s1, m2, s2) == K.combine(m1, s1, m2, s2), trial
    with pytest.raises(AmmError):
        combine([1.0], [-1.0], [1.0], [1.0])


def test_calculation_constants_are_the_papers():
    """Sec. V: Calc 1 uses C2, C3, C4 = 0.03, 0.035, 0.035 and Calc 2 0.03, 0.01,
    0.06, both with D = 0.75 and C1 = 1 - C2 - C3 - C4."""
    from oracle.sampler import CALC1, CALC2
    for params, (c2, c3, c4) in ((CALC1, (0.03, 0.035, 0.035)), (CALC2, (0.03, 0.01, 0.06))):
        assert params['c'][1:] == (c2, c3, c4) and params['d'] == 0.75
        assert params['c'][0] == ((1.0 - c2) - c3) - c4
        assert abs(sum(params['c']) - 1.0) < 1e-15
