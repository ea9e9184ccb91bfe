"""Write oracle reference data for the GPU parity tests.

Calls only oracle/.  Outputs (this directory):
  oracle_level_polys.json.gz   the oracle's numerator polynomials (1-3 loops)
  oracle_points_3loop.npz      for every 3-loop SE graph, sample counters
                               0..47 and 999999952..999999999 of seed 0
                               (the ends of the 1e9-sample range): the
                               oracle's z, g = gx 2^gj, component, path and the
                               exact (rational) integrands rounded to double.
Run: python tests/golden/make_golden.py [--polys]   (about 5 minutes on 8
cores; --polys derives the polynomials again instead of loading the cache)
"""
import os
import sys
from fractions import Fraction
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import graphs as G            # noqa: E402
from oracle import integrand as I         # noqa: E402
from oracle import sampler as S           # noqa: E402

COUNTERS = list(range(0, 48)) + list(range(999_999_952, 1_000_000_000))


def polys_for(args):
    n, gi = args
    ch = G.se_graphs(n)[gi]
    z = [Fraction(1, 3 * n - 1)] * (3 * n - 1)
    for e in range(2 * n - 1):
        I.vertex_integrand(G.make_vertex_graph(ch, e), z, exact=True)
    return dict(I._POLY_STORE)


def points_for(gi):
    n = 3
    out = {}
    d = S.Density(n, G.se_graphs(n)[gi])
    idx = np.array(COUNTERS, dtype=np.uint64)
    from oracle.philox import uniforms, graph_uid
    u = uniforms(0, graph_uid(n, gi), idx, 2 * d.M - 1)
    s = d.sample(u)
    ex, ab = [], []
    for i in range(len(COUNTERS)):
        vals = I.se_integrands(n, gi, [Fraction(x) for x in s['z'][i]], exact=True)
        ex.append([float(v) for v, _ in vals])
        ab.append([float(a) for _, a in vals])
    out.update(z=s['z'], gx=s['gx'], gj=s['gj'], comp=s['comp'], path=s['path'],
               I=np.array(ex), absI=np.array(ab))
    return gi, out


def main():
    cache = os.path.join(HERE, 'oracle_level_polys.json.gz')
    if os.path.exists(cache) and '--polys' not in sys.argv:
        I.load_poly_cache(cache)        # the oracle's own earlier output
    else:
        jobs = [(n, gi) for n in (1, 2, 3) for gi in range(len(G.se_graphs(n)))]
        with Pool(8) as pool:
            for store in pool.imap_unordered(polys_for, jobs):
                I._POLY_STORE.update(store)
        I.dump_poly_cache(cache)
    print('polys', len(I._POLY_STORE), flush=True)
    with Pool(8) as pool:
        res = dict(pool.map(points_for, range(len(G.se_graphs(3)))))
    arrays = {'counters': np.array(COUNTERS, dtype=np.uint64)}
    for gi, d in res.items():
        for k, v in d.items():
            arrays[f'g{gi}_{k}'] = v
    np.savez_compressed(os.path.join(HERE, 'oracle_points_3loop.npz'), **arrays)
    print('points done', flush=True)


if __name__ == '__main__':
    main()
