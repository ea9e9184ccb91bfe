"""Write 4-loop oracle reference points for the GPU parity tests.

Calls only oracle/.  Output (this directory): oracle_points_4loop.npz with, for
each graph in GRAPHS (spread over the 74 four-loop SE graphs), seed-0 sample
counters COUNTERS: the oracle's z, g = gx 2^gj, component and path; every
insertion integrand and its sum of |term| in x87 extended precision (64-bit
significand), stored as a double hi part and the double remainder lo; and for
the first N_EXACT counters the exact rational integrands rounded to double.
The script checks that the extended values agree with the exact ones to
1e-12 of max(|I|, sum|terms|): at 4 loops single terms cancel internally, and
x87 values were seen 1.4e-14 of that scale off (graph 28, counter 0).

Run: python tests/golden/make_golden_4loop.py   (a few hours on 8 cores;
the oracle derives every level polynomial with explicit 4x4 matrices).
"""
import os
import sys
import time
from fractions import Fraction
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import graphs as G            # noqa: E402
from oracle import integrand as I         # noqa: E402
from oracle import sampler as S           # noqa: E402
from oracle.philox import uniforms, graph_uid   # noqa: E402

N_LOOPS = 4
GRAPHS = [0, 7, 14, 21, 28, 35, 42, 49, 56, 63, 70, 73]
COUNTERS = list(range(0, 256))
N_EXACT = 4
POLY_CACHE = os.environ.get('AMM_GOLDEN4_POLYS', '')


def polys_for(job):
    gi, e = job
    t0 = time.time()
    ch = G.se_graphs(N_LOOPS)[gi]
    z = [Fraction(1, 3 * N_LOOPS - 1)] * (3 * N_LOOPS - 1)
    I.vertex_integrand(G.make_vertex_graph(ch, e), z, exact=True)
    print(f'polys graph {gi} insertion {e}: {time.time() - t0:.0f} s', flush=True)
    return dict(I._POLY_STORE)


def points_for(gi):
    t0 = time.time()
    ch = G.se_graphs(N_LOOPS)[gi]
    d = S.Density(N_LOOPS, ch)
    idx = np.array(COUNTERS, dtype=np.uint64)
    u = uniforms(0, graph_uid(N_LOOPS, gi), idx, 2 * d.M - 1)
    s = d.sample(u)
    zl = [np.asarray(s['z'][:, i], dtype=np.longdouble) for i in range(d.M)]
    ne = 2 * N_LOOPS - 1
    hi = np.zeros((len(COUNTERS), ne)); lo = np.zeros_like(hi)
    ahi = np.zeros_like(hi); alo = np.zeros_like(hi)
    ex = np.zeros((N_EXACT, ne)); aex = np.zeros_like(ex)
    with np.errstate(all='ignore'):
        for e in range(ne):
            vg = G.make_vertex_graph(ch, e)
            v, a = I.vertex_integrand(vg, zl, exact='ld')
            v = np.broadcast_to(np.asarray(v, dtype=np.longdouble), (len(COUNTERS),))
            a = np.broadcast_to(np.asarray(a, dtype=np.longdouble), (len(COUNTERS),))
            hi[:, e] = v.astype(np.float64); lo[:, e] = (v - hi[:, e].astype(np.longdouble)).astype(np.float64)
            ahi[:, e] = a.astype(np.float64); alo[:, e] = (a - ahi[:, e].astype(np.longdouble)).astype(np.float64)
            for i in range(N_EXACT):
                val, ab = I.vertex_integrand(vg, [Fraction(x) for x in s['z'][i]], exact=True)
                ex[i, e] = float(val); aex[i, e] = float(ab)
                scale = max(abs(float(val)), float(ab))
                dev = abs(float(Fraction(float(v[i])) + Fraction(float(lo[i, e])) - val))
                assert dev <= 1e-12 * scale, (gi, e, i, dev, scale)
    print(f'points graph {gi}: {time.time() - t0:.0f} s', flush=True)
    return gi, dict(z=s['z'], gx=s['gx'], gj=s['gj'], comp=s['comp'], path=s['path'],
                    I_hi=hi, I_lo=lo, absI_hi=ahi, absI_lo=alo, I_exact=ex, absI_exact=aex)


def main():
    if POLY_CACHE and os.path.exists(POLY_CACHE):
        I.load_poly_cache(POLY_CACHE)
    else:
        jobs = [(gi, e) for gi in GRAPHS for e in range(2 * N_LOOPS - 1)]
        with Pool(8) as pool:
            for store in pool.imap_unordered(polys_for, jobs):
                I._POLY_STORE.update(store)
        if POLY_CACHE:
            I.dump_poly_cache(POLY_CACHE)
    print('polys', len(I._POLY_STORE), flush=True)
    with Pool(8) as pool:
        res = dict(pool.imap_unordered(points_for, GRAPHS))
    arrays = {'counters': np.array(COUNTERS, dtype=np.uint64), 'graphs': np.array(GRAPHS)}
    for gi, d in res.items():
        for k, v in d.items():
            arrays[f'g{gi}_{k}'] = v
    np.savez_compressed(os.path.join(HERE, 'oracle_points_4loop.npz'), **arrays)
    print('points done', flush=True)


if __name__ == '__main__':
    main()
