"""Oracle: nonadaptive Monte Carlo estimate of one SE graph's insertions.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Estimator (Sec. III.B): mean = (1/N) sum y_j, y_j = I(z_j)/g(z_j)
(eq. integral_approx), sigma^2 = sum y^2 / N^2 - (sum y)^2 / N^3
(eq. sigma_down).  Per class, the y of the class's insertions at the same
point are summed before squaring, and so are all insertions for the graph's
total (they share the point, so their covariances belong in its variance);
class and total sigma^2 add over graphs, which are sampled independently
(eq. sigma_sum).

Round-off acceptance (Sec. IV.A, eq. interval_accept): a point of graph j is
accepted when its round-off bound does not exceed
tau_j = (1/4) s_j sqrt(sum_l s_l^2) / sum_l s_l, s_j being graph j's sigma
of a pilot run scaled to the planned run, sigma_j sqrt(N_pilot / N_run).  A
rejected point is recomputed in higher precision.

A sample whose point leaves the double range (a z below the smallest normal
double) or whose integrand is not finite contributes 0 and is counted
(Sec. IV.A reports such 'out of double' samples; reading R13).
"""
from __future__ import annotations

import numpy as np

from . import graphs as G
from . import integrand as I
from .sampler import sample_graph, CALC2

DBL_MIN = 2.2250738585072014e-308


def evaluate_points(n, gi, z):
    """I_{S,e}(z) and sum|terms| for all insertions e; z: (N, M) float64.

    Returns (vals (N, 2n-1), abs (N, 2n-1))."""
    ch = G.se_graphs(n)[gi]
    cols = [z[:, i] for i in range(z.shape[1])]
    vals, absv = [], []
    with np.errstate(all='ignore'):
        for e in range(2 * n - 1):
            vg = G.make_vertex_graph(ch, e)
            v, a = I.vertex_integrand(vg, cols)
            vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), (z.shape[0],)))
            absv.append(np.broadcast_to(np.asarray(a, dtype=np.float64), (z.shape[0],)))
    return np.stack(vals, 1), np.stack(absv, 1)


def classes_of(n, gi):
    ch = G.se_graphs(n)[gi]
    return [G.vertex_class(ch, e) for e in range(2 * n - 1)]


def run(n, gi, seed, start, count, params=CALC2, chunk=50000):
    """Plain FP64 estimate over sample indices [start, start+count)."""
    ne = 2 * n - 1
    cls = classes_of(n, gi)
    ucls = sorted(set(cls))
    acc = dict(n=0, sum=np.zeros(ne), sum2=np.zeros(ne), sumabs=np.zeros(ne), n_ood=0,
               csum={c: 0.0 for c in ucls}, csum2={c: 0.0 for c in ucls}, tsum=0.0, tsum2=0.0)
    dens = None
    for c0 in range(start, start + count, chunk):
        cnt = min(chunk, start + count - c0)
        out, dens = sample_graph(n, gi, seed, c0, cnt, dens, params)
        z = out['z']
        vals, _ = evaluate_points(n, gi, z)
        with np.errstate(all='ignore'):
            y = np.ldexp(vals / out['gx'][:, None], -out['gj'][:, None])
        bad = (z.min(1) < DBL_MIN) | ~np.all(np.isfinite(y), 1)
        y[bad] = 0.0
        acc['n'] += cnt
        acc['n_ood'] += int(bad.sum())
        acc['sum'] += y.sum(0)
        acc['sum2'] += (y * y).sum(0)
        acc['sumabs'] += np.abs(y).sum(0)
        for c in ucls:
            yc = sum(y[:, e] for e in range(ne) if cls[e] == c)
            acc['csum'][c] += float(yc.sum())
            acc['csum2'][c] += float((yc * yc).sum())
        yt = y.sum(1)
        acc['tsum'] += float(yt.sum())
        acc['tsum2'] += float((yt * yt).sum())
    return acc


def accept_thresholds(sigmas, n_pilot, n_run):
    """tau_j of eq. (interval_accept) from pilot sigmas (one per graph).

    n_pilot: samples of each graph's pilot (scalar or per graph); n_run the
    planned samples per graph.  All sigmas zero gives no check (inf)."""
    sig = np.asarray(sigmas, dtype=np.float64) * np.sqrt(np.asarray(n_pilot, dtype=np.float64) / float(n_run))
    tot = float(sig.sum())
    if tot <= 0.0:
        return np.full(sig.shape, np.inf)
    return 0.25 * sig * np.sqrt(float((sig * sig).sum())) / tot


def flagged_estimate(y_fp64, bound, y_ref, tau):
    """Sums of the accepted-or-recomputed y of one graph.

    y_fp64, bound, y_ref: (N, ne) FP64 values, their round-off bounds (both
    already divided by g) and higher-precision values at the same points;
    tau: the graph's threshold.  A point whose bound summed over the
    insertions exceeds tau, or whose FP64 value is not finite, takes y_ref.
    Returns (y used (N, ne), flag mask (N,))."""
    rsum = np.asarray(bound).sum(1)
    with np.errstate(invalid='ignore'):
        flag = ~(rsum <= tau) | ~np.all(np.isfinite(y_fp64), 1)
    y = np.where(flag[:, None], y_ref, y_fp64)
    return y, flag


def mean_sigma(s, s2, N):
    mean = s / N
    var = s2 / N ** 2 - s ** 2 / N ** 3
    return mean, np.sqrt(np.maximum(var, 0.0))
