"""GPU parity: the HIP path through the C ABI against the oracle.

Bars (reading R14): sample points, densities and sector paths
bit-exact on identical Philox streams; per-point integrands within 1e-10 of
the oracle's exact value relative to max(|I|, sum|terms|) (FP64) and 1e-13
(double-double); estimates within 1e-3 of the oracle's sigma."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from oracle import estimate as E            # noqa: E402
from oracle import graphs as G              # noqa: E402
from oracle import integrand as I           # noqa: E402
from oracle import sampler as S             # noqa: E402
from oracle.philox import uniforms, graph_uid   # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), 'golden')


@pytest.fixture(scope='module')
def amm():
    from paper_1909_08015_amd import Context
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return Context(0)


def _ctx_for(amm, n, build=True):
    amm.enumerate(n)
    if build:
        amm.build_tables()
    return amm


def oracle_sample(n, gi, counters):
    d = S.Density(n, G.se_graphs(n)[gi])
    u = uniforms(0, graph_uid(n, gi), np.asarray(counters, dtype=np.uint64), 2 * d.M - 1)
    return d.sample(u)


@pytest.mark.parametrize('n', [1, 2, 3])
def test_graph_set_and_classes(amm, n):
    _ctx_for(amm, n, build=False)
    assert amm.n_se == len(G.se_graphs(n))
    for gi, ch in enumerate(G.se_graphs(n)):
        chords, classes = amm.graph_desc(gi)
        assert chords == ch
        assert classes == [G.vertex_class(ch, e) for e in range(2 * n - 1)]


@pytest.mark.parametrize('n,graphs', [(1, [0]), (2, [0, 1]), (3, [0, 4, 9])])
def test_sample_bit_exact(amm, n, graphs):
    _ctx_for(amm, n)
    for gi in graphs:
        for start, count in ((0, 5003), (999_999_000, 1000)):
            out = amm.sample(gi, 0, start, count)
            torch.cuda.synchronize()
            ref = oracle_sample(n, gi, range(start, start + count))
            assert np.array_equal(out['z'].cpu().numpy(), ref['z'])
            assert np.array_equal(out['gx'].cpu().numpy(), ref['gx'])
            assert np.array_equal(out['gj'].cpu().numpy(), ref['gj'])
            assert np.array_equal(out['comp'].cpu().numpy(), ref['comp'])
            assert np.array_equal(out['path'].cpu().numpy(), ref['path'])


def _check_points(I64, Idd, ref, absref):
    scale = np.maximum(np.abs(ref), absref)
    err64 = np.abs(I64 - ref) / scale
    errdd = np.abs(Idd - ref) / scale
    assert errdd.max() < 1e-13, errdd.max()
    assert err64.max() < 1e-10, (err64.max(), np.argmax(err64))
    return err64


@pytest.mark.parametrize('n', [1, 2])
def test_eval_vs_exact_1_2_loops(amm, n):
    _ctx_for(amm, n)
    for gi in range(len(G.se_graphs(n))):
        ref = oracle_sample(n, gi, range(0, 40))
        z = torch.tensor(ref['z'], device='cuda')
        I64, A64 = amm.eval(gi, z, precision=0)
        Idd, _ = amm.eval(gi, z, precision=1)
        torch.cuda.synchronize()
        ex = np.array([[float(v) for v, _ in I.se_integrands(n, gi, [Fraction(x) for x in row], exact=True)]
                       for row in ref['z']])
        ab = np.array([[float(a) for _, a in I.se_integrands(n, gi, [Fraction(x) for x in row], exact=True)]
                       for row in ref['z']])
        _check_points(I64.cpu().numpy(), Idd.cpu().numpy(), ex, ab)
        assert np.allclose(A64.cpu().numpy(), ab, rtol=1e-8)


def test_eval_3_loops_against_golden(amm):
    """Counters at both ends of the 1e9-sample range of every 3-loop graph:
    points bit-exact, integrands against the oracle's exact values."""
    data = np.load(os.path.join(GOLD, 'oracle_points_3loop.npz'))
    counters = data['counters']
    _ctx_for(amm, 3)
    for gi in range(len(G.se_graphs(3))):
        # the stored points are reproduced by the GPU sampler at those counters
        for lo, hi in ((0, 48), (48, 96)):
            out = amm.sample(gi, 0, int(counters[lo]), hi - lo)
            torch.cuda.synchronize()
            assert np.array_equal(out['z'].cpu().numpy(), data[f'g{gi}_z'][lo:hi])
            assert np.array_equal(out['gj'].cpu().numpy(), data[f'g{gi}_gj'][lo:hi])
        z = torch.tensor(data[f'g{gi}_z'], device='cuda')
        I64, _ = amm.eval(gi, z, precision=0)
        Idd, _ = amm.eval(gi, z, precision=1)
        torch.cuda.synchronize()
        _check_points(I64.cpu().numpy(), Idd.cpu().numpy(), data[f'g{gi}_I'], data[f'g{gi}_absI'])


def test_eval_empty_and_ragged(amm):
    _ctx_for(amm, 2)
    z = torch.empty((0, 5), dtype=torch.float64, device='cuda')
    I64, _ = amm.eval(0, z)
    assert I64.shape == (0, 3)
    ref = oracle_sample(2, 1, range(7, 7 + 257))
    Idd, _ = amm.eval(1, torch.tensor(ref['z'], device='cuda'), precision=1)
    torch.cuda.synchronize()
    ex = [[v for v, _ in I.se_integrands(2, 1, [Fraction(x) for x in row], exact=True)] for row in ref['z']]
    err = [abs(Fraction(float(g)) - e) / abs(e) for grow, erow in zip(Idd.cpu().numpy(), ex)
           for g, e in zip(grow, erow) if e != 0]
    assert max(err) < 1e-13


@pytest.mark.parametrize('n,N', [(1, 300_000), (2, 200_000)])
def test_estimate_parity(amm, n, N):
    """GPU estimate vs the oracle's on identical counters (no flagging)."""
    _ctx_for(amm, n)
    amm.integrate(seed=0, n_per_graph=N)
    for gi in range(len(G.se_graphs(n))):
        acc = E.run(n, gi, 0, 0, N)
        m, s = E.mean_sigma(acc['sum'], acc['sum2'], acc['n'])
        for e in range(2 * n - 1):
            r = amm.read(gi, e)
            assert r['n'] == N and r['n_ood'] == acc['n_ood']
            assert abs(r['mean'] - m[e]) <= 1e-3 * s[e], (gi, e, r['mean'], m[e], s[e])
            assert r['sigma'] == pytest.approx(s[e], rel=1e-6)


def test_one_and_two_loop_values_full_size(amm):
    """Configuration C1: 1e7 samples per graph; A1^(2) = 0.5 (Sec. I) and the
    2-loop no-lepton-loop value within 4 sigma."""
    _ctx_for(amm, 1)
    amm.integrate(seed=0, n_per_graph=10_000_000)
    r = amm.read(0, 0)
    assert abs(r['mean'] - 0.5) < 4 * r['sigma'] and r['sigma'] < 1e-4
    _ctx_for(amm, 2)
    amm.integrate(seed=0, n_per_graph=10_000_000)
    tot = amm.read(-1, -1, None)
    target = -0.344166387438296
    assert abs(tot['mean'] - target) < 4 * tot['sigma'], tot
    assert tot['sigma'] < 0.005


def test_determinism_across_grid_sizes(amm):
    _ctx_for(amm, 2)
    amm.integrate(seed=3, n_per_graph=700_001, samples_per_thread=1)
    a = [amm.read(g, e) for g in range(2) for e in range(3)]
    amm.integrate(seed=3, n_per_graph=700_001, samples_per_thread=7)
    b = [amm.read(g, e) for g in range(2) for e in range(3)]
    assert a == b


def test_split_counter_range_resumes(amm):
    """Two runs over adjacent counter ranges accumulate to one run over both
    (counter-based streams make checkpoint/resume exact)."""
    _ctx_for(amm, 1)
    amm.integrate(seed=5, n_per_graph=2 * 16384 * 64)
    one = amm.read(0, 0)
    amm.integrate(seed=5, n_per_graph=16384 * 64)
    amm.integrate(seed=5, n_per_graph=16384 * 64, counter0=16384 * 64, accumulate=1)
    two = amm.read(0, 0)
    assert one['n'] == two['n']
    assert two['mean'] == pytest.approx(one['mean'], rel=1e-14)


def test_force_flag_double_double(amm):
    """Every point recomputed in double-double gives the FP64 estimate."""
    _ctx_for(amm, 2)
    amm.integrate(seed=1, n_per_graph=100_000)
    a = [amm.read(g, e) for g in range(2) for e in range(3)]
    amm.integrate(seed=1, n_per_graph=100_000, force_flag=1)
    b = [amm.read(g, e) for g in range(2) for e in range(3)]
    for x, y in zip(a, b):
        assert y['n_flag'] == 100_000 and y['n_dd_fail'] == 0
        assert abs(x['mean'] - y['mean']) <= 1e-9 * abs(x['sum_abs'] / x['n'])
