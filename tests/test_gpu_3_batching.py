"""GPU: batching of a loop order's graphs (persistent fused launch, captured
batches, autotuned launch configuration) and the 4-loop graph set.

Results are keyed by 1024-sample chunk, so launch shape, graph order, fusion
and graph replay must leave every accumulator bit-identical."""
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
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    return Context(0)


def _acc(amm):
    return [amm.read(g, e) for g in range(amm.n_se) for e in range(2 * amm.loops - 1)]


def _same(a, b):
    for x, y in zip(a, b):
        assert x['n'] == y['n'] and x['n_flag'] == y['n_flag'] and x['n_dd_fail'] == y['n_dd_fail']
        assert x['mean'] == y['mean'] and x['sigma'] == y['sigma'], (x, y)


def _tau(amm, n_run, n_pilot=30_000):
    amm.integrate(seed=1, n_per_graph=n_pilot, force_flag=1)
    return amm.accept_thresholds(n_run)


def test_caller_workspace(amm):
    """amm_set_workspace: a torch-owned workspace of 300 chunks per group gives
    the own-buffer run's counters exactly and its sums to rounding (segment sums
    added in another order); back on the own buffers the run is bit-identical."""
    amm.enumerate(2)
    amm.build_tables()
    N = 700_001
    tau = _tau(amm, N)
    amm.integrate(seed=6, n_per_graph=N, accept_tau=tau)
    a = _acc(amm)
    nbytes = amm.workspace_bytes(300)
    assert nbytes > 0 and amm.workspace_bytes(0) == 0 and amm.workspace_bytes(32769) == 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device='cuda')
    try:
        amm.set_workspace(ws)
        amm.integrate(seed=6, n_per_graph=N, accept_tau=tau)
        b = _acc(amm)
    finally:
        amm.set_workspace(None)
    for x, y in zip(a, b):
        assert x['n'] == y['n'] and x['n_flag'] == y['n_flag'] and x['n_dd_fail'] == y['n_dd_fail']
        assert abs(x['sum_y'] - y['sum_y']) <= 1e-12 * y['sum_abs']
    assert sum(x['n_flag'] for x in a) > 0
    amm.integrate(seed=6, n_per_graph=N, accept_tau=tau)
    _same(a, _acc(amm))
    from paper_1909_08015_amd.amm import AmmError
    with pytest.raises(AmmError):
        amm.set_workspace(ws[: amm.workspace_bytes(1) - 256])


def test_fused_launch_matches_per_graph_launches(amm):
    from paper_1909_08015_amd.amm import OPT_GENERATED, OPT_FUSED, OPT_ORDER_BY_COST
    amm.enumerate(3)
    amm.build_tables()
    N = 300_001
    tau = _tau(amm, N)
    try:
        amm.set_option(OPT_GENERATED, 0)
        amm.set_option(OPT_FUSED, 0)
        amm.integrate(seed=4, n_per_graph=N, accept_tau=tau)
        a = _acc(amm)
        amm.set_option(OPT_FUSED, 1)
        for order in (0, 1):
            amm.set_option(OPT_ORDER_BY_COST, order)
            for bpc in (1, 3):
                amm.integrate(seed=4, n_per_graph=N, accept_tau=tau, blocks_per_cu=bpc)
                _same(a, _acc(amm))
        # generated code: same samples and flags up to the bound, estimates agree far inside sigma
        amm.set_option(OPT_GENERATED, 1)
        amm.integrate(seed=4, n_per_graph=N, accept_tau=tau)
        for x, y in zip(a, _acc(amm)):
            assert x['n'] == y['n']
            assert abs(x['mean'] - y['mean']) <= 1e-6 * max(x['sigma'], 1e-300) + 1e-12 * abs(x['mean'])
    finally:
        amm.set_option(OPT_GENERATED, 1)
        amm.set_option(OPT_FUSED, 1)
        amm.set_option(OPT_ORDER_BY_COST, 1)


@pytest.mark.parametrize('n', [2, 3])
def test_captured_batches_equal_separate_calls(amm, n):
    amm.enumerate(n)
    amm.build_tables()
    B, K = 200_000, 3
    tau = _tau(amm, B * K)
    for b in range(K):
        amm.integrate(seed=6, n_per_graph=B, counter0=b * B, accumulate=int(b > 0), accept_tau=tau)
    a = _acc(amm)
    amm.integrate_batches(seed=6, n_per_graph=B, n_batches=K, accept_tau=tau)
    _same(a, _acc(amm))
    # a second capture continues from a counter offset and accumulates
    amm.integrate(seed=6, n_per_graph=B, counter0=5 * B, accept_tau=tau)
    amm.integrate(seed=6, n_per_graph=B, counter0=6 * B, accumulate=1, accept_tau=tau)
    c = _acc(amm)
    amm.integrate_batches(seed=6, n_per_graph=B, n_batches=2, counter0=5 * B, accept_tau=tau)
    _same(c, _acc(amm))


def test_autotune_keeps_results(amm):
    amm.enumerate(3)
    amm.build_tables()
    N = 100_000
    tau = _tau(amm, N)
    amm.integrate(seed=8, n_per_graph=N, accept_tau=tau)
    a = _acc(amm)
    cfg = amm.autotune(seed=0, n_per_graph=65_536, accept_tau=tau)
    assert cfg['blocks_per_cu'] in (1, 2, 4, 8, 16) and cfg['order_by_cost'] in (0, 1) and cfg['ms'] > 0
    _same(a, _acc(amm))                        # accumulators restored
    amm.integrate(seed=8, n_per_graph=N, accept_tau=tau)
    _same(a, _acc(amm))                        # tuned configuration, same results


@pytest.fixture(scope='module')
def four_loops(amm):
    amm.enumerate(4)
    amm.build_tables()
    assert amm.n_se == 74
    return amm


def test_four_loop_sampling_bit_exact(four_loops):
    amm = four_loops
    for gi in (0, 17, 44, 73):
        d = S.Density(4, G.se_graphs(4)[gi])
        cnt = np.arange(1000, 1000 + 513, dtype=np.uint64)
        ref = d.sample(uniforms(0, graph_uid(4, gi), cnt, 2 * d.M - 1))
        out = amm.sample(gi, 0, 1000, 513)
        torch.cuda.synchronize()
        for k in ('z', 'gx', 'gj', 'path', 'comp'):
            assert np.array_equal(out[k].cpu().numpy(), ref[k]), (gi, k)


def test_four_loop_fp64_within_bound_of_double_double(four_loops):
    """Parity unpinned against the oracle at 4 loops (its numerator derivation
    is too slow there): the FP64 integrand lies within its propagated bound of
    the double-double value, the bound certifies a share of the points, and
    the sum of |terms| agrees for typical points.  Points out of the double
    range are skipped."""
    amm = four_loops
    cert = []
    for gi in (0, 9, 37, 56, 73):
        out = amm.sample(gi, 0, 0, 256)
        keep = out['z'].min(dim=1).values >= 2.2250738585072014e-308
        z = out['z'][keep].contiguous()
        I64, A64, B64 = amm.eval(gi, z, precision=0, with_bound=True)
        Idd, Add = amm.eval(gi, z, precision=1)
        torch.cuda.synchronize()
        I64, A64, B64 = I64.cpu().numpy(), A64.cpu().numpy(), B64.cpu().numpy()
        Idd, Add = Idd.cpu().numpy(), Add.cpu().numpy()
        assert np.all(np.isfinite(Idd)) and np.all(np.isfinite(I64))
        # the running bound is first order: it must hold wherever it is small
        # against the value (relative error << 1); where FP64 has lost every
        # digit the bound exceeds the value and the point is always flagged
        scale = np.maximum(np.abs(Idd), Add)
        ratio = np.abs(I64 - Idd) / np.maximum(B64, 1e-300)
        first_order = B64 <= 1e-2 * scale
        k = np.unravel_index(np.argmax(ratio), ratio.shape)
        print(f'\n4-loop graph {gi}: max error/bound {ratio.max():.3g} (bound/scale there {B64[k] / scale[k]:.3g}); '
              f'first-order points {first_order.mean():.3f}, their max error/bound '
              f'{ratio[first_order].max() if first_order.any() else 0:.3g}')
        assert np.all(ratio[first_order] <= 1.0), gi
        # a single term can cancel internally at 4 loops, so |term| in FP64 is
        # only accurate for most points
        assert np.median(np.abs(A64 - Add) / Add) < 1e-10
        cert.append(B64 <= 1e-10 * np.maximum(np.abs(Idd), Add))
        # the Monte Carlo pass flags every point outside the first-order regime
        # whatever the threshold (here one no bound reaches): its flag count
        # equals the number of points with a bound above 1e-2 of the FP64
        # value's scale in some insertion (the same FP64 numbers)
        outside = ~np.all(B64 <= 1e-2 * np.maximum(np.abs(I64), A64), axis=1)
        nonfinite = ~np.all(np.isfinite(I64), axis=1)
        if bool(keep.all()):
            amm.integrate(seed=0, n_per_graph=256, graph_begin=gi, graph_end=gi + 1, accept_tau=[1e300])
            r = amm.read(gi, -1)
            assert r['n_flag'] == int((outside | nonfinite).sum()), (gi, r['n_flag'], int(outside.sum()))
    assert np.concatenate([c.ravel() for c in cert]).mean() > 0.05


def test_four_loop_fused_run_is_deterministic(four_loops):
    amm = four_loops
    N = 40_000
    tau = _tau(amm, 10 ** 10 // 74, n_pilot=10_000)
    amm.integrate(seed=0, n_per_graph=N, accept_tau=tau, blocks_per_cu=2)
    a = _acc(amm)
    for x in a:
        assert x['n'] == N and np.isfinite(x['mean']) and np.isfinite(x['sigma'])
    amm.integrate(seed=0, n_per_graph=N, accept_tau=tau, blocks_per_cu=5)
    _same(a, _acc(amm))
    tot = amm.read(-1, -1, None)
    print('\n4-loop estimate after', N, 'samples per graph:', tot)
    assert tot['n_dd_fail'] <= 1e-3 * tot['n']
