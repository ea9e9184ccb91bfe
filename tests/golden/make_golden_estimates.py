"""Write oracle Monte Carlo sums for the 3-loop estimate parity test.

Calls only oracle/.  Output (this directory): oracle_estimates_3loop.json with,
for every 3-loop SE graph and Philox seed 0, sample counters [0, N_PER_GRAPH):
the sums of eq. (integral_approx) and eq. (sigma_down) per insertion, per class
(insertions of the class summed at each point) and for the per-point total,
plus the out-of-double count.  Every integrand is evaluated in x87 extended
precision (64-bit significand) and in FP64, each rounded to double before
y = I / g.  The forest sum cancels pointwise (Sec. II), near the boundaries by
factors of 1e20 and more, where the x87 value loses every digit (3-loop graph
7, counter 928702: x87 y = 2.8e6, exact -6.1e-12); even the x87 sum of |terms|
is then unreliable.  A point whose x87 and FP64 values of y differ by more
than EXACT_DELTA in some insertion is evaluated exactly (rational arithmetic)
instead: two independent roundings agree that closely only where both are
close to the exact value.  The sums are then those of (nearly) exact
integrands, whichever points an FP64 pass would have flagged.

Run: python tests/golden/make_golden_estimates.py   (about 30 minutes on 8 cores)
"""
import json
from fractions import Fraction
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import graphs as G            # noqa: E402
from oracle import integrand as I         # noqa: E402
from oracle import sampler as S           # noqa: E402
from oracle.estimate import DBL_MIN, classes_of   # noqa: E402

N_LOOPS = 3
N_PER_GRAPH = 1 << 20
CHUNK = 1 << 15
EXACT_DELTA = 1e-4


def job(args):
    gi, c0 = args
    ch = G.se_graphs(N_LOOPS)[gi]
    out, _ = S.sample_graph(N_LOOPS, gi, 0, c0, CHUNK)
    z = out['z']
    zl = [np.asarray(z[:, i], dtype=np.longdouble) for i in range(z.shape[1])]
    ne = 2 * N_LOOPS - 1
    vals = np.zeros((CHUNK, ne))
    v64 = np.zeros((CHUNK, ne))
    zd = [z[:, i] for i in range(z.shape[1])]
    with np.errstate(all='ignore'):
        for e in range(ne):
            vg = G.make_vertex_graph(ch, e)
            v, _ = I.vertex_integrand(vg, zl, exact='ld')
            vals[:, e] = np.broadcast_to(np.asarray(v, dtype=np.longdouble), (CHUNK,)).astype(np.float64)
            v, _ = I.vertex_integrand(vg, zd)
            v64[:, e] = np.broadcast_to(np.asarray(v, dtype=np.float64), (CHUNK,))
        y = np.ldexp(vals / out['gx'][:, None], -out['gj'][:, None])
        y64 = np.ldexp(v64 / out['gx'][:, None], -out['gj'][:, None])
        agree = np.all(np.abs(y - y64) <= EXACT_DELTA, 1)
    bad = z.min(1) < DBL_MIN                     # out of the double range: contributes 0, counted
    redo = np.where(~bad & ~(agree & np.all(np.isfinite(y), 1)))[0]
    for i in redo:
        ex = I.se_integrands(N_LOOPS, gi, [Fraction(x) for x in z[i]], exact=True)
        y[i] = [np.ldexp(float(v) / out['gx'][i], -int(out['gj'][i])) for v, _ in ex]
    y[bad] = 0.0
    return gi, c0, y, int(bad.sum()), len(redo)


def main():
    I.load_poly_cache(os.path.join(HERE, 'oracle_level_polys.json.gz'))
    ngr = len(G.se_graphs(N_LOOPS))
    jobs = [(gi, c0) for gi in range(ngr) for c0 in range(0, N_PER_GRAPH, CHUNK)]
    res = {}
    with Pool(int(os.environ.get('AMM_GOLDEN_JOBS', '8'))) as pool:
        for gi, c0, y, nbad, nexact in pool.imap_unordered(job, jobs, chunksize=1):
            res[(gi, c0)] = (y, nbad, nexact)
    out = {'loops': N_LOOPS, 'seed': 0, 'n_per_graph': N_PER_GRAPH, 'graphs': []}
    for gi in range(ngr):
        cls = classes_of(N_LOOPS, gi)
        ucls = sorted(set(cls))
        # fixed order: chunks in counter order, numpy sums within a chunk
        s = np.zeros(2 * N_LOOPS - 1); s2 = np.zeros_like(s)
        cs = {c: 0.0 for c in ucls}; cs2 = {c: 0.0 for c in ucls}
        ts = ts2 = 0.0
        nood = nexact = 0
        for c0 in range(0, N_PER_GRAPH, CHUNK):
            y, nbad, nex = res[(gi, c0)]
            nood += nbad
            nexact += nex
            s += y.sum(0); s2 += (y * y).sum(0)
            for c in ucls:
                yc = sum(y[:, e] for e in range(y.shape[1]) if cls[e] == c)
                cs[c] += float(yc.sum()); cs2[c] += float((yc * yc).sum())
            yt = y.sum(1)
            ts += float(yt.sum()); ts2 += float((yt * yt).sum())
        out['graphs'].append(dict(graph=gi, n=N_PER_GRAPH, n_ood=nood, n_exact=nexact, sum=s.tolist(), sum2=s2.tolist(),
                                  classes=[list(c) for c in ucls], csum=[cs[c] for c in ucls],
                                  csum2=[cs2[c] for c in ucls], tsum=ts, tsum2=ts2))
    with open(os.path.join(HERE, 'oracle_estimates_3loop.json'), 'w') as f:
        json.dump(out, f, indent=1)
    print('estimates done', flush=True)


if __name__ == '__main__':
    main()
