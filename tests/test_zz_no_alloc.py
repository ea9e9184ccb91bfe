"""amm_integrate_static (no allocation: the library's static device scratch)
against amm_integrate on the same runs, through the C ABI: two calls in a
row, the second smaller, at 2 loops (round-off check with double-double
recompute), 3 loops (generated kernels) and 4 loops (fused interpreter
launch).  Counters must agree exactly; sums to rounding (the two entry points
add segment sums in a different order: 262144-sample groups against
33.5M-sample groups), here 1e-12 relative to the sums of |y|."""
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu


@pytest.fixture(scope='module')
def amm():
    from paper_1909_08015_amd import Context
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return Context(0)


def _reads(amm, graphs):
    ne = 2 * amm.loops - 1
    return [amm.read(g, e) for g in graphs for e in list(range(ne)) + [-1]]


def _agree(a, b):
    for x, y in zip(a, b):
        for k in ('n', 'n_flag', 'n_dd_fail', 'n_ood'):
            assert x[k] == y[k], (k, x, y)
        assert abs(x['sum_y'] - y['sum_y']) <= 1e-12 * y['sum_abs'] + 1e-300, (x, y)
        assert abs(x['sum_y2'] - y['sum_y2']) <= 1e-12 * y['sum_y2'] + 1e-300, (x, y)
        assert x['sum_abs'] == pytest.approx(y['sum_abs'], rel=1e-12)


@pytest.mark.parametrize('loops,sizes,graphs', [(2, (700_001, 100_003), None), (3, (600_000, 50_000), None),
                                                (4, (20_000, 5_000), (0, 12))])
def test_static_entry_point_matches_integrate(amm, loops, sizes, graphs):
    print(f'static vs integrate: loops={loops} sizes={sizes} graphs={graphs}', flush=True)
    amm.enumerate(loops)
    gb, ge = graphs if graphs else (0, amm.n_se)
    amm.build_tables(gb, ge)
    tau = None
    if loops == 2:
        amm.integrate(seed=1, n_per_graph=50_000, force_flag=1, graph_begin=gb, graph_end=ge)
        tau = amm.accept_thresholds(sizes[0], gb, ge)
    for n in sizes:
        amm.integrate(seed=4, n_per_graph=n, graph_begin=gb, graph_end=ge, accept_tau=tau)
        ref = _reads(amm, range(gb, ge))
        amm.integrate_static(seed=4, n_per_graph=n, graph_begin=gb, graph_end=ge, accept_tau=tau)
        got = _reads(amm, range(gb, ge))
        _agree(got, ref)
        if loops == 2:
            assert sum(r['n_flag'] for r in got) > 0      # the recompute ran


def test_static_entry_point_rejects_oversized_runs(amm):
    from paper_1909_08015_amd.amm import AmmError
    amm.enumerate(2)
    amm.build_tables()
    with pytest.raises(AmmError, match='1024 segments'):
        amm.integrate_static(seed=0, n_per_graph=600 * 262144)
