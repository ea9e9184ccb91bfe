"""GPU: FP64 interval arithmetic with outward rounding, the first interval rung
of the reliability ladder of Sec. IV.A (amm_eval precision 2).

Every interval must enclose the oracle's exact integrand: checked exactly with
Fractions at 1 and 2 loops, and against the stored exact 3-loop values (which
are themselves rounded once to double).  The widths are compared with the
first-order running bound of the FP64 pass."""
import os
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

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


def _points(n, gi, counters):
    d = S.Density(n, G.se_graphs(n)[gi])
    return d.sample(uniforms(0, graph_uid(n, gi), np.asarray(counters, dtype=np.uint64), 2 * d.M - 1))['z']


@pytest.mark.parametrize('n', [1, 2])
def test_intervals_enclose_exact_values_1_2_loops(amm, n):
    amm.enumerate(n)
    amm.build_tables()
    for gi in range(len(G.se_graphs(n))):
        z = _points(n, gi, range(100, 140))
        Im, Am, R = amm.eval(gi, torch.tensor(z, device='cuda'), precision=2, with_bound=True)
        torch.cuda.synchronize()
        Im, R = Im.cpu().numpy(), R.cpu().numpy()
        assert np.all(np.isfinite(R)) and np.all(R >= 0)
        for p, row in enumerate(z):
            ex = [v for v, _ in I.se_integrands(n, gi, [Fraction(x) for x in row], exact=True)]
            for e, v in enumerate(ex):
                assert abs(Fraction(float(Im[p, e])) - v) <= Fraction(float(R[p, e])), (n, gi, p, e)


def test_intervals_enclose_exact_values_3_loops(amm):
    data = np.load(os.path.join(GOLD, 'oracle_points_3loop.npz'))
    amm.enumerate(3)
    amm.build_tables()
    widths = []
    for gi in range(len(G.se_graphs(3))):
        z = torch.tensor(data[f'g{gi}_z'], device='cuda')
        Im, Am, R = amm.eval(gi, z, precision=2, with_bound=True)
        I64, A64, B64 = amm.eval(gi, z, precision=0, with_bound=True)
        torch.cuda.synchronize()
        Im, R, B64 = Im.cpu().numpy(), R.cpu().numpy(), B64.cpu().numpy()
        ex = data[f'g{gi}_I']                       # exact values rounded once to double
        slack = np.spacing(np.abs(ex))
        ok = np.abs(Im - ex) <= R + slack
        assert np.all(ok | ~np.isfinite(R)), gi
        assert np.mean(np.isfinite(R)) > 0.99, gi
        fin = np.isfinite(R) & (B64 > 0)
        widths.append(R[fin] / B64[fin])
    w = np.concatenate(widths)
    print(f'\n3 loops: interval radius / running bound: median {np.median(w):.3g}, '
          f'90th percentile {np.percentile(w, 90):.3g}')


def test_interval_precision_is_validated(amm):
    from paper_1909_08015_amd import AmmError
    amm.enumerate(2)
    amm.build_tables()
    z = torch.tensor(_points(2, 0, range(4)), device='cuda')
    with pytest.raises(AmmError):
        amm.eval(0, z, precision=3)
