"""Write the oracle's numerator-polynomial cache for one 4-loop SE graph.

Calls only oracle/.  Output (this directory):
oracle_level_polys_4loop_g<G>.json.gz, the level polynomials the oracle needs
to evaluate every insertion of 4-loop SE graph G (default 0).  With --from
PATH, polynomials already derived by the oracle (a cache written by
dump_poly_cache, e.g. by make_golden_4loop.py) are reused and only the
missing ones are derived; the output holds exactly the ones graph G uses.
Used by bench.py's CPU baseline (the oracle timed on the host) and by the CPU
finiteness pins at 4 loops.

Run: python tests/golden/make_poly_cache_4loop.py [--graph G] [--from PATH]
(minutes with a cache covering G, else about an hour).
"""
import argparse
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import graphs as G            # noqa: E402
from oracle import integrand as I         # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--graph', type=int, default=0)
    ap.add_argument('--from', dest='src', default='')
    args = ap.parse_args()
    if args.src:
        I.load_poly_cache(args.src)
    used = set()
    orig = I._level_poly_cached

    def tracked(key):
        used.add(key)
        return orig(key)
    I._level_poly_cached = tracked
    ch = G.se_graphs(4)[args.graph]
    z = [Fraction(1, 11)] * 11
    for e in range(7):
        I.vertex_integrand(G.make_vertex_graph(ch, e), z, exact=True)
    full = I._POLY_STORE
    I._POLY_STORE = {k: full[k] for k in used}
    out = os.path.join(HERE, f'oracle_level_polys_4loop_g{args.graph}.json.gz')
    I.dump_poly_cache(out)
    print(out, len(used), 'polynomials', os.path.getsize(out), 'bytes')


if __name__ == '__main__':
    main()
