"""Pins of the second calculation's pieces (Sec. V): the MRG32k3a
generator as counter-addressed streams, and the graph-by-graph combination of
two calculations."""
import math

import numpy as np
import pytest

from oracle import mrg32k3a as R
from oracle import combine as K

I3 = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def _is_prime(n):
    """Deterministic Miller-Rabin: the first twelve primes as bases decide
    every n below 3.3e24."""
    if n < 2:
        return False
    bases = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in bases:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


# m^3 - 1 = (m - 1)(m^2 + m + 1); both m - 1 = 2 p and m^2 + m + 1 are checked
# below to be these products of primes.
PERIOD_FACTORS = {R.M1: (2, 2147483543, 18446742282708232657),
                  R.M2: (2, 2147472221, 18446547772751524693)}


def test_component_recurrences_have_full_period_order():
    """Each component's characteristic polynomial is primitive modulo its
    prime: the companion matrix has order exactly m^3 - 1, i.e. its power
    m^3 - 1 is the identity and its power (m^3 - 1)/r is not, for every prime
    r dividing m^3 - 1 (a wrong multiplier or modulus fails one of these)."""
    for mat, m in ((R.MAT1, R.M1), (R.MAT2, R.M2)):
        assert _is_prime(m)
        fac = PERIOD_FACTORS[m]
        assert math.prod(fac) == m ** 3 - 1 and all(_is_prime(r) for r in fac)
        assert fac[0] * fac[1] == m - 1 and fac[2] == m * m + m + 1
        assert R.mat_pow(mat, m ** 3 - 1, m) == I3
        for r in fac:
            assert R.mat_pow(mat, (m ** 3 - 1) // r, m) != I3, r


def test_a_wrong_multiplier_fails_the_order_pin():
    """Negative control: changing one multiplier of component 1 breaks the
    order pin above."""
    bad = [list(r) for r in R.MAT1]
    for i in range(3):
        for j in range(3):
            if bad[i][j] not in (0, 1):
                bad[i][j] = (bad[i][j] + 1) % R.M1
                break
        else:
            continue
        break
    bad = tuple(tuple(r) for r in bad)
    m = R.M1
    ok = R.mat_pow(bad, m ** 3 - 1, m) == I3 and all(
        R.mat_pow(bad, (m ** 3 - 1) // r, m) != I3 for r in PERIOD_FACTORS[m])
    assert not ok


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
