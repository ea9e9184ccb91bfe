"""GPU: 4-loop integrands against the oracle (Sec. II, forest formula R^new;
reading R14 bars).

tests/golden/oracle_points_4loop.npz (written by make_golden_4loop.py, oracle
only) holds, for 12 of the 74 four-loop SE graphs, seed-0 counters 0..255: the
oracle's points, densities and paths, every insertion integrand and its sum
of |term| in x87 extended precision (hi + lo doubles), and exact rational
values at the first four counters.  Checked here through the C ABI:
  * sampling bit-exact (points, g = gx 2^gj, components, sector paths);
  * FP64 integrands within their own round-off bound B wherever they are
    finite, and within 1e-10 of max(|I|, sum|terms|) wherever B certifies
    1e-10; non-finite FP64 values carry an infinite bound (always flagged);
  * double-double integrands within 1e-13 of the exact values, and against
    the extended-precision ones within 1e-13 of the scale plus 2^-11 B: the
    x87 sum rounds with 11 more bits than FP64 but, at 4 loops, single terms
    cancel internally (B up to the scale itself), so its own error is of the
    order of 2^-11 of the FP64 bound, not of the scale (measured: at most
    4e-7 B); where FP64 is not finite, within 1e-10 of the scale;
  * the FP64 sum of |terms| within B of the oracle's (each |term| moves by
    at most its share of the round-off);
  * the Monte Carlo sums over those 256 counters (every point recomputed in
    double-double) against the sums of the oracle's values."""
import os

import numpy as np
import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), 'golden', 'oracle_points_4loop.npz')


@pytest.fixture(scope='module')
def data():
    return np.load(GOLD)


@pytest.fixture(scope='module')
def amm():
    from paper_1909_08015_amd import Context
    assert torch.cuda.is_available(), 'GPU tests need a GPU'
    c = Context(0)
    c.enumerate(4)
    c.build_tables()
    return c


def _ref(data, gi, what):
    return data[f'g{gi}_{what}_hi'] + data[f'g{gi}_{what}_lo']


def test_four_loop_points_bit_exact(amm, data):
    counters = data['counters']
    for gi in data['graphs']:
        print(f'4-loop sampling: graph {gi}', flush=True)
        out = amm.sample(int(gi), 0, int(counters[0]), len(counters))
        torch.cuda.synchronize()
        for k in ('z', 'gx', 'gj', 'comp', 'path'):
            assert np.array_equal(out[k].cpu().numpy(), data[f'g{gi}_{k}']), (gi, k)


def test_four_loop_integrands_against_oracle(amm, data):
    cert = []
    for gi in data['graphs']:
        print(f'4-loop integrands: graph {gi}', flush=True)
        z = torch.tensor(data[f'g{gi}_z'], device='cuda')
        I64, A64, B64 = amm.eval(int(gi), z, precision=0, with_bound=True)
        Idd, _ = amm.eval(int(gi), z, precision=1)
        torch.cuda.synchronize()
        I64, A64, B64, Idd = (t.cpu().numpy() for t in (I64, A64, B64, Idd))
        ref, aref = _ref(data, gi, 'I'), _ref(data, gi, 'absI')
        scale = np.maximum(np.abs(ref), aref)
        fin = np.isfinite(I64) & np.isfinite(A64)
        assert np.all(np.isinf(B64[~fin])), gi
        fin &= np.isfinite(B64)
        print(f'   non-finite FP64 values: {int((~fin).sum())}', flush=True)
        err = np.abs(I64 - ref)
        assert np.all(err[fin] <= B64[fin] + 1e-15 * scale[fin]), (gi, (err[fin] / np.maximum(B64[fin], 1e-300)).max())
        ok = fin & (B64 <= 1e-10 * scale)
        assert np.all(err[ok] <= 1e-10 * scale[ok]), gi
        cert.append(ok)
        assert np.all(np.abs(A64 - aref)[fin] <= B64[fin] + 1e-13 * aref[fin]), gi
        assert np.all(np.isfinite(Idd)), gi
        ddev = np.abs(Idd - ref)
        assert np.all(ddev[fin] <= 1e-13 * scale[fin] + 2.0 ** -11 * B64[fin]), (gi, (ddev / scale).max())
        assert np.all(ddev[~fin] <= 1e-10 * scale[~fin]), (gi, (ddev[~fin] / scale[~fin]).max())
        ex, aex = data[f'g{gi}_I_exact'], data[f'g{gi}_absI_exact']
        k = ex.shape[0]
        sx = np.maximum(np.abs(ex), aex)
        assert np.all(np.abs(Idd[:k] - ex) <= 1e-13 * sx), gi
    frac = np.concatenate(cert).mean()
    print(f'FP64 points certified to 1e-10: {frac:.2f}')
    assert frac > 0.3


def test_four_loop_sums_against_oracle(amm, data):
    """Sums of y = I/g over the 256 stored counters (every point recomputed in
    double-double) against the sums of the oracle's values: per insertion
    within 1e-12 of the sum of |I|/g, and the per-point totals likewise."""
    counters = data['counters']
    for gi in data['graphs']:
        g = np.ldexp(data[f'g{gi}_gx'], data[f'g{gi}_gj'])
        y = _ref(data, gi, 'I') / g[:, None]
        ya = _ref(data, gi, 'absI') / g[:, None]
        amm.integrate(seed=0, n_per_graph=len(counters), counter0=int(counters[0]), graph_begin=int(gi),
                      graph_end=int(gi) + 1, force_flag=1)
        for e in range(7):
            r = amm.read(int(gi), e)
            assert r['n'] == len(counters) and r['n_flag'] == len(counters) and r['n_dd_fail'] == 0
            assert abs(r['sum_y'] - y[:, e].sum()) <= 1e-12 * ya[:, e].sum(), (gi, e)
        t = amm.read(int(gi), -1)
        assert abs(t['sum_y'] - y.sum()) <= 1e-12 * ya.sum(), gi
        assert abs(t['sum_y2'] - (y.sum(1) ** 2).sum()) <= 1e-11 * (ya.sum(1) ** 2).sum(), gi
