"""GPU: the paper's first calculation (Sec. V): MRG32k3a samples and the Calc 1
density constants, and its graph-by-graph combination with the Philox4x32-10
calculation."""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from oracle import graphs as G              # noqa: E402
from oracle import sampler as S             # noqa: E402
from oracle import mrg32k3a as R            # noqa: E402
from oracle.philox import graph_uid         # noqa: E402

# A1^(4) without lepton loops: the closed form of the full coefficient minus
# its vacuum-polarisation part
A4_NO_LOOPS = -0.344166387438296


@pytest.fixture(scope='module')
def amm():
    from paper_1909_08015_amd import Context
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return Context(0)


@pytest.fixture
def mrg(amm):
    from paper_1909_08015_amd.amm import OPT_GENERATOR
    amm.set_option(OPT_GENERATOR, 1)
    yield amm
    amm.set_option(OPT_GENERATOR, 0)


@pytest.mark.parametrize('n,graphs', [(2, (0, 1)), (3, (0, 4, 9))])
def test_mrg32k3a_sampling_bit_exact(mrg, n, graphs):
    from paper_1909_08015_amd import CALC1
    amm = mrg
    amm.enumerate(n)
    amm.build_tables(params=CALC1)
    seed = 0x0123_4567_89AB_CDEF
    for gi in graphs:
        d = S.Density(n, G.se_graphs(n)[gi], params=S.CALC1)
        c0 = (1 << 40) - 100                     # high digits of the jump exercised
        cnt = np.arange(c0, c0 + 200, dtype=np.uint64)
        ref = d.sample(R.uniforms(seed, graph_uid(n, gi), cnt, 2 * d.M - 1))
        out = amm.sample(gi, seed, c0, 200)
        torch.cuda.synchronize()
        for k in ('z', 'gx', 'gj', 'path', 'comp'):
            assert np.array_equal(out[k].cpu().numpy(), ref[k]), (n, gi, k)
        out = amm.sample(gi, seed, 3, 50)
        torch.cuda.synchronize()
        ref = d.sample(R.uniforms(seed, graph_uid(n, gi), np.arange(3, 53, dtype=np.uint64), 2 * d.M - 1))
        assert np.array_equal(out['z'].cpu().numpy(), ref['z'])


def test_mrg32k3a_learned_mixture_sampling_bit_exact(mrg):
    """The learned mixture (2M uniforms per sample) on MRG32k3a streams, with a
    seeded synthetic sector table: points, densities, paths bit-exact."""
    amm = mrg
    n, gi = 3, 6
    amm.enumerate(n)
    amm.build_tables()
    M = 3 * n - 1
    tab = (0.05 + 0.95 * np.random.default_rng(7).random(((1 << M), M))).astype(np.float32)
    amm.set_sector_table(gi, tab)
    try:
        out = amm.sample(gi, 11, 5000, 1500, learned=1)
        torch.cuda.synchronize()
        d = S.Density(n, G.se_graphs(n)[gi])
        ref = d.sample(R.uniforms(11, graph_uid(n, gi), np.arange(5000, 6500, dtype=np.uint64), 2 * M), tab)
        for k in ('z', 'gx', 'gj', 'path', 'comp'):
            assert np.array_equal(out[k].cpu().numpy(), ref[k]), k
    finally:
        amm.set_sector_table(gi, None)


def test_mrg32k3a_index_range_is_checked(mrg):
    from paper_1909_08015_amd import AmmError
    amm = mrg
    amm.enumerate(2)
    amm.build_tables()
    with pytest.raises(AmmError):
        amm.integrate(seed=0, n_per_graph=10, counter0=(1 << 44) - 5)
    with pytest.raises(AmmError):
        amm.sample(0, 0, (1 << 44) - 5, 10)


def test_two_calculations_and_their_combination_2_loops(amm):
    """Calc 1 (MRG32k3a, C = .03/.035/.035) and Calc 2 (Philox, .03/.01/.06)
    each reproduce A1^(4) without lepton loops; so does their graph-by-graph
    combination, whose sigma is below both."""
    from paper_1909_08015_amd import CALC1, CALC2
    from paper_1909_08015_amd.amm import OPT_GENERATOR, combine
    amm.enumerate(2)
    N = 1 << 23
    res = {}
    try:
        for name, gen, params in (('calc1', 1, CALC1), ('calc2', 0, CALC2)):
            amm.set_option(OPT_GENERATOR, gen)
            amm.build_tables(params=params)
            amm.integrate(seed=1, n_per_graph=30_000, force_flag=1)
            tau = amm.accept_thresholds(N)
            amm.integrate(seed=5, n_per_graph=N, accept_tau=tau)
            per = [amm.read(g) for g in range(amm.n_se)]
            res[name] = ([p['mean'] for p in per], [p['sigma'] for p in per])
            tot = amm.read(-1, -1)
            print(f'\n2 loops, {name}: {tot["mean"]:.9f} +- {tot["sigma"]:.2g}')
            assert abs(tot['mean'] - A4_NO_LOOPS) < 5 * tot['sigma'], name
    finally:
        amm.set_option(OPT_GENERATOR, 0)
        amm.build_tables(params=CALC2)
    assert res['calc1'][0] != res['calc2'][0]
    ms, ss, tm, ts = combine(res['calc1'][0], res['calc1'][1], res['calc2'][0], res['calc2'][1])
    print(f'combined: {tm:.9f} +- {ts:.2g}')
    assert abs(tm - A4_NO_LOOPS) < 5 * ts
    for j in range(len(ms)):
        assert ss[j] <= min(res['calc1'][1][j], res['calc2'][1][j])


def test_mrg32k3a_run_is_deterministic_across_launches(mrg):
    from paper_1909_08015_amd import CALC1
    amm = mrg
    amm.enumerate(3)
    amm.build_tables(params=CALC1)
    amm.integrate(seed=2, n_per_graph=200_000, blocks_per_cu=1)
    a = [amm.read(g, e) for g in range(amm.n_se) for e in range(5)]
    amm.integrate(seed=2, n_per_graph=200_000, blocks_per_cu=6)
    b = [amm.read(g, e) for g in range(amm.n_se) for e in range(5)]
    for x, y in zip(a, b):
        assert x['n'] == y['n'] and x['mean'] == y['mean'] and x['sigma'] == y['sigma']
    amm.build_tables()
