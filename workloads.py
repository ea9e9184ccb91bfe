"""Seeded synthetic workloads (no method arithmetic here).

The inputs of this path are the exactly enumerated graph sets of one loop
order plus Philox seeds and sample-counter ranges; the paper's runs used
seeds of their own and ~1e9-sample blocks per graph (Sec. IV.A).  Both the
oracle and the library read their configurations from here."""

# name -> (loops, samples per graph, seed)
CONFIGS = {
    'C1-1loop': dict(loops=1, n_per_graph=10_000_000, seed=0),
    'C1-2loop': dict(loops=2, n_per_graph=10_000_000, seed=0),
    'C2-3loop': dict(loops=3, n_per_graph=1_000_000_000, seed=0),
    'C3-4loop': dict(loops=4, n_per_graph=135_135_135, seed=0),
}


def counters(start, count):
    """Sample indices [start, start+count) as a list-like range."""
    return range(start, start + count)


def random_simplex_points(M, count, seed):
    """Uniform points on the simplex (sorted-uniform spacings), seeded."""
    import numpy as np
    rng = np.random.default_rng(seed)
    u = np.sort(rng.random((count, M - 1)), axis=1)
    z = np.diff(np.concatenate([np.zeros((count, 1)), u, np.ones((count, 1))], axis=1), axis=1)
    return z
