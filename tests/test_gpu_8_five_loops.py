"""GPU: the 5-loop graph set (Sec. V, Table I: 706 SE graphs, 6354 oriented
vertex graphs in nine classes) and its density tables (Sec. III.A, M = 14).

Sampling on identical Philox streams is bit-exact against the oracle: points,
densities g = gx 2^gj, sector paths and mixture components, at both ends of a
1e9-sample counter range and for graphs spread over the set."""
import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from oracle import graphs as G              # noqa: E402
from oracle import sampler as S             # noqa: E402
from oracle.philox import uniforms, graph_uid   # noqa: E402


@pytest.fixture(scope='module')
def amm():
    from paper_1909_08015_amd import Context
    from paper_1909_08015_amd.amm import OPT_PLANS
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    c = Context(0)
    c.enumerate(5)
    c.set_option(OPT_PLANS, 0)
    c.build_tables()
    yield c
    c.set_option(OPT_PLANS, 1)


def test_five_loop_graph_set_and_classes(amm):
    assert (amm.n_se, amm.n_vertex, amm.M) == (706, 706 * 9, 14)
    counts = {}
    for gi, ch in enumerate(G.se_graphs(5)):
        chords, classes = amm.graph_desc(gi)
        assert chords == ch
        assert classes == [G.vertex_class(ch, e) for e in range(9)]
        for k in classes:
            counts[k] = counts.get(k, 0) + 1
    # oriented vertex graphs per class; Table I counts unoriented ones
    assert sum(counts.values()) == 6354 and len(counts) == 9


@pytest.mark.parametrize('gi', [0, 117, 353, 588, 705])
def test_five_loop_sampling_bit_exact(amm, gi):
    d = S.Density(5, G.se_graphs(5)[gi])
    for start, count in ((0, 3001), (999_999_000, 1000)):
        print(f'5-loop sampling: graph {gi} counters {start}+{count}', flush=True)
        out = amm.sample(gi, 0, start, count)
        torch.cuda.synchronize()
        u = uniforms(0, graph_uid(5, gi), np.arange(start, start + count, dtype=np.uint64), 2 * d.M - 1)
        ref = d.sample(u)
        assert np.array_equal(out['comp'].cpu().numpy(), ref['comp'])
        assert np.array_equal(out['path'].cpu().numpy(), ref['path'])
        assert np.array_equal(out['z'].cpu().numpy(), ref['z'])
        assert np.array_equal(out['gx'].cpu().numpy(), ref['gx'])
        assert np.array_equal(out['gj'].cpu().numpy(), ref['gj'])


def test_five_loop_evaluation_refused_without_integrand_tables(amm):
    from paper_1909_08015_amd.amm import AmmError
    z = torch.full((4, 14), 1.0 / 14, dtype=torch.float64, device='cuda')
    with pytest.raises(AmmError, match='not built'):
        amm.eval(1, z)


def test_five_loop_integrands_graph0(amm):
    """5-loop SE graph 0 with its integrand tables (2.8 million monomials, 9
    insertions, built on the host's threads): FP64 integrands within their
    round-off bound of the double-double ones at sampled points, and a short
    run with the round-off check and double-double recompute whose per-class
    and total accumulators are consistent.  Parity with the oracle is not
    pinned at 5 loops: the oracle's explicit-matrix numerators take hours per
    graph there."""
    from paper_1909_08015_amd.amm import OPT_PLANS
    amm.set_option(OPT_PLANS, 1)
    try:
        amm.build_tables(0, 1)
    finally:
        amm.set_option(OPT_PLANS, 0)
    st = amm.plan_stats(0)
    assert st['n_insertions'] == 9 and st['n_monomials'] > 2_000_000
    s = amm.sample(0, 0, 0, 512)
    I64, _, B64 = amm.eval(0, s['z'], precision=0, with_bound=True)
    Idd, Add = amm.eval(0, s['z'], precision=1)
    torch.cuda.synchronize()
    I64, B64, Idd, Add = (t.cpu().numpy() for t in (I64, B64, Idd, Add))
    scale = np.maximum(np.abs(Idd), Add)
    assert np.all(np.abs(I64 - Idd) <= B64 + 1e-13 * scale)
    assert (B64 <= 1e-10 * scale).mean() > 0.2
    amm.integrate(seed=1, n_per_graph=2048, graph_begin=0, graph_end=1, force_flag=1)
    tau = amm.accept_thresholds(10 ** 8, 0, 1)
    amm.integrate(seed=0, n_per_graph=32768, graph_begin=0, graph_end=1, accept_tau=tau)
    tot = amm.read(0, -1)
    assert tot['n'] == 32768 and np.isfinite(tot['mean']) and tot['sigma'] > 0
    _, classes = amm.graph_desc(0)
    ins = [amm.read(0, e) for e in range(9)]
    assert sum(r['sum_y'] for r in ins) == pytest.approx(tot['sum_y'], rel=1e-9, abs=1e-9 * tot['sum_abs'])
    print('5-loop graph 0:', tot, 'classes', sorted(set(classes)))
