"""Oracle pins: Dirac traces, projectors, the forest-subtracted integrand and
the 1- and 2-loop values."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import dirac as D
from oracle import estimate as E
from oracle import graphs as G
from oracle import integrand as I


def test_clifford_relation_and_traces():
    g = np.diag([1, -1, -1, -1])
    for m in range(4):
        for n in range(4):
            ac = D.GAMMA_UP[m] @ D.GAMMA_UP[n] + D.GAMMA_UP[n] @ D.GAMMA_UP[m]
            assert np.allclose(ac, 2 * g[m, n] * np.eye(4))
    # gamma^mu gamma_mu = 4, Tr[a b c d] = 4[(ab)(cd) - (ac)(bd) + (ad)(bc)]
    assert D.trace_chain([('idx', 0), ('idx', 0)]) == pytest.approx(16)
    rng = np.random.default_rng(0)
    v = rng.normal(size=(4, 4))
    dot = lambda x, y: x @ g @ y
    t = np.trace(D.slash(v[0]) @ D.slash(v[1]) @ D.slash(v[2]) @ D.slash(v[3]))
    ref = 4 * (dot(v[0], v[1]) * dot(v[2], v[3]) - dot(v[0], v[2]) * dot(v[1], v[3])
               + dot(v[0], v[3]) * dot(v[1], v[2]))
    assert t == pytest.approx(ref)
    # gamma^a x gamma_a = -2 x for a vector
    x = D.slash(v[0])
    assert np.allclose(sum(D.GAMMA_UP[a] @ x @ D.GAMMA_LO[a] for a in range(4)), -2 * x)


@pytest.mark.parametrize('ze', [Fr(1, 3), Fr(5, 7), Fr(1, 1000)])
def test_one_loop_integrand_exact(ze):
    """The 1-loop AMM integrand on the simplex is z_gamma/(z_e+z_gamma)^3,
    whose simplex integral is 1/2 = A1^(2) (Sec. I)."""
    vg = G.make_vertex_graph(G.se_graphs(1)[0], 0)
    z = [ze, 1 - ze]
    v, _ = I.vertex_integrand(vg, z, exact=True)
    assert v == z[1] / (z[0] + z[1]) ** 3


def test_one_loop_integrand_projector_is_gauge_of_q_direction():
    """The O(q^2) projector trace is isotropic: every spacelike direction
    gives the same F2 (Lorentz covariance after the loop integration)."""
    vg = G.make_vertex_graph(G.se_graphs(2)[1], 1)
    t = G.terms(vg)[0]
    levels, _ = G.build_levels(vg, t)
    items = I.level_chain(vg, levels[0], t.forest, {})
    saved = list(D.Q_DIRS)
    try:
        res = []
        for q in saved:
            D.Q_DIRS[:] = [q, q, q]
            res.append(I._level_poly(items, 'A', 'V'))
        assert res[0] == res[1] == res[2]
    finally:
        D.Q_DIRS[:] = saved


def _rand_point(M, seed):
    rng = np.random.default_rng(seed)
    w = [Fr(int(x)) for x in rng.integers(1, 1000, M)]
    s = sum(w)
    return [x / s for x in w]


@pytest.mark.parametrize('gi,e', [(0, 0), (0, 1), (1, 0), (1, 1), (1, 2)])
def test_top_contraction_order_vanishes(gi, e):
    """Terms with c = n contractions would carry Gamma(0); their coefficient
    is structurally zero after the AMM / (L-U) projection (exact)."""
    vg = G.make_vertex_graph(G.se_graphs(2)[gi], e)
    z = _rand_point(5, gi * 10 + e)
    for t in G.terms(vg):
        _, vec = I.term_value(vg, t, z, exact=True)
        assert all(c == 0 for c in vec[2:])


def test_float_path_matches_exact():
    n = 2
    for gi in range(2):
        z = _rand_point(5, 77 + gi)
        zf = np.array([[float(x) for x in z]])
        vals, _ = E.evaluate_points(n, gi, zf)
        ex = [float(v) for v, _ in I.se_integrands(n, gi, z, exact=True)]
        assert np.allclose(vals[0], ex, rtol=1e-11, atol=0)


def _scaled(z, idx, rho):
    z2 = list(z)
    for i in idx:
        z2[i] = z2[i] * rho
    s = sum(z2)
    return [x / s for x in z2]


def test_subtraction_makes_uv_subgraphs_integrable():
    """Finiteness at the simplex boundary: for every UV subgraph s of every
    2-loop vertex graph, rho^{|s|} |I(rho z_s)| -> 0 (integrable), while the
    unsubtracted A_G f_G alone does not decrease (negative control)."""
    n = 2
    base = _rand_point(5, 3)
    checked = 0
    for gi, ch in enumerate(G.se_graphs(n)):
        for e in range(3):
            vg = G.make_vertex_graph(ch, e)
            for a, b, kind in G.uv_subgraphs(vg):
                if (a, b) == (0, 4):
                    continue
                idx = set()
                for v in range(a, b):
                    idx.add(G.line_index(vg, seg=v))
                for ci, (c, d) in enumerate(vg.chords):
                    if a <= c and d <= b:
                        idx.add(G.line_index(vg, chord=ci))
                vals, raw = [], []
                for rho in (Fr(1, 10 ** 4), Fr(1, 10 ** 6)):
                    z = _scaled(base, idx, rho)
                    v, _ = I.vertex_integrand(vg, z, exact=True)
                    vals.append(abs(v) * rho ** len(idx))
                    t0 = [t for t in G.terms(vg) if len(t.forest) == 1][0]
                    r, _ = I.term_value(vg, t0, z, exact=True)
                    raw.append(abs(r) * rho ** len(idx))
                assert vals[1] < vals[0] / 10
                assert raw[1] > raw[0] / 2
                checked += 1
    assert checked >= 2


def a4_no_lepton_loops():
    """A1^(4) (Petermann/Sommerfield closed form) minus its electron
    vacuum-polarisation part 119/36 - pi^2/3 (literature values, not in the
    paper).  The closed form is first pinned to the digits the paper prints."""
    z3 = 1.2020569031595942
    a4 = 197 / 144 + math.pi ** 2 / 12 - math.pi ** 2 / 2 * math.log(2) + 0.75 * z3
    assert abs(a4 - (-0.328478965579)) < 1e-12        # Sec. I printed value
    return a4 - (119 / 36 - math.pi ** 2 / 3)


def test_one_and_two_loop_values():
    """A1^(2) = 0.5 (Sec. I) and the 2-loop no-lepton-loop value within 4
    sigma, through the full sampler + integrand + estimator."""
    a = E.run(1, 0, 0, 0, 200000)
    m, s = E.mean_sigma(a['sum'], a['sum2'], a['n'])
    assert abs(m[0] - 0.5) < 4 * s[0]
    tot, var = 0.0, 0.0
    for gi in range(2):
        a = E.run(2, gi, 0, 0, 150000)
        for c in a['csum']:
            cm, cs = E.mean_sigma(a['csum'][c], a['csum2'][c], a['n'])
            tot += cm
            var += cs ** 2
    target = a4_no_lepton_loops()
    assert abs(target - (-0.344166387438296)) < 1e-12
    assert abs(tot - target) < 4 * math.sqrt(var)
    assert math.sqrt(var) < 0.05
