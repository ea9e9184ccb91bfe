"""Oracle pins: Philox, exp/log, the density and the sampler."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import gammaln

from oracle import graphs as G
from oracle import sampler as S
from oracle.mathfn import amm_exp, amm_log
from oracle.philox import philox4x32_10, uniforms


def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Random123 distribution,
    Salmon et al. SC'11)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
        ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
        ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
         (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
    ]
    for ctr, key, want in cases:
        assert tuple(int(x) for x in philox4x32_10(ctr, key)) == want


def test_uniforms_open_interval():
    u = uniforms(0, 7, np.arange(100000, dtype=np.uint64), 5)
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)


def test_exp_log_accuracy():
    x = np.random.default_rng(0).uniform(-700, 700, 20000)
    assert np.max(np.abs(amm_exp(x) / np.exp(x) - 1)) < 4.5e-16
    y = np.random.default_rng(1).uniform(0, 1, 20000) ** 25 + 1e-300
    assert np.max(np.abs(amm_log(y) - np.log(y)) / np.abs(np.log(y))) < 4.5e-16
    assert amm_exp(np.array([0.0]))[0] == 1.0 and amm_log(np.array([1.0]))[0] == 0.0


def brute_F(deg, M):
    tot = 0.0
    for perm in itertools.permutations(range(M)):
        p = 1.0
        for l in range(1, M):
            s = sum(1 << j for j in perm[l:])
            p /= deg[s]
        tot += p
    return tot


@pytest.mark.parametrize('n,gi', [(1, 0), (2, 0), (2, 1)])
def test_normalisation_dp_matches_permutations(n, gi):
    d = S.Density(n, G.se_graphs(n)[gi])
    assert d.F1[d.full] == pytest.approx(brute_F(d.deg1, d.M), rel=1e-12)


def test_sector_frequencies_chi2():
    """g1 sector probabilities prod W(s_{l+1})/F(s_l) vs observed frequencies."""
    n, gi = 2, 1
    d = S.Density(n, G.se_graphs(n)[gi], params=dict(S.CALC2, c=(1.0, 0.0, 0.0, 0.0)))
    N = 60000
    out, _ = S.sample_graph(n, gi, 5, 0, N, d)
    M = d.M
    counts = {}
    for row in out['path']:
        counts[tuple(row)] = counts.get(tuple(row), 0) + 1
    chi2 = 0.0
    dof = 0
    for perm in itertools.permutations(range(M)):
        p = 1.0
        s = d.full
        for l in range(M - 1):
            j = perm[l]
            p *= d.W1[s & ~(1 << j)] / d.F1[s]
            s &= ~(1 << j)
        exp_ = N * p
        if exp_ > 5:
            chi2 += (counts.get(perm, 0) - exp_) ** 2 / exp_
            dof += 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


@pytest.mark.parametrize('n,gi', [(2, 0), (3, 4)])
def test_density_normalised_and_dirichlet(n, gi):
    """E_g[(M-1)!/g] = 1 (the simplex volume is 1/(M-1)!) and
    E_g[prod z^(a-1)/g] = prod Gamma(a)/Gamma(sum a)."""
    out, d = S.sample_graph(n, gi, 11, 0, 100000)
    g = S.g_value(out['gx'], out['gj'])
    M = d.M
    w = math.factorial(M - 1) / g
    assert abs(w.mean() - 1) < 5 * w.std() / math.sqrt(len(w))
    a = np.linspace(0.4, 1.6, M)
    val = np.exp(((a - 1) * np.log(out['z'])).sum(1)) / g
    ref = math.exp(gammaln(a).sum() - gammaln(a.sum()))
    assert abs(val.mean() / ref - 1) < 5 * val.std() / ref / math.sqrt(len(val))


def test_g_mantissa_exponent_form():
    out, d = S.sample_graph(3, 0, 3, 0, 2000)
    assert np.all((out['gx'] >= 0.5) & (out['gx'] < 1.0))


def test_one_loop_variance_closed_form():
    """Pure g1 with Deg({gamma}) = 1, Deg({e}) = 1/2 at 1 loop: E[y] = 1/2 and
    Var(y) equals the closed-form integral of z_gamma^2/g - 1/4."""
    n = 1
    deg = np.zeros(4)
    deg[1] = 0.5      # {e}   (line 0 = segment)
    deg[2] = 1.0      # {gamma}
    params = dict(S.CALC2, c=(1.0, 0.0, 0.0, 0.0))
    d = S.Density(n, G.se_graphs(1)[0], params, deg=deg)
    C = 1.0 / d.F1[3]

    def g(ze):
        zg = 1 - ze
        if ze >= zg:   # sector e >= gamma: s_2 = {gamma}
            return C * (zg / ze) ** 1.0 / (ze * zg)
        return C * (ze / zg) ** 0.5 / (ze * zg)
    second = integrate.quad(lambda ze: (1 - ze) ** 2 / g(ze), 0, 1, points=[0.5], limit=200)[0]
    var_exact = second - 0.25
    assert var_exact == pytest.approx(0.0351043861823939, rel=1e-9)
    out, _ = S.sample_graph(1, 0, 0, 0, 400000, d)
    y = out['z'][:, 1] / S.g_value(out['gx'], out['gj'])
    assert abs(y.mean() - 0.5) < 5 * math.sqrt(var_exact / len(y))
    assert abs(y.var() / var_exact - 1) < 0.05
