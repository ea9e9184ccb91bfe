"""Oracle: the learned sector sampler (FP64 reference).

TEST INFRASTRUCTURE (see oracle/graphs.py).

This part is not in the paper; it follows this project's specification of
the learned sampler:

* rows: every (s, j) with j in s, |s| >= 2, of an SE graph's M lines, ordered
  by s ascending then j ascending; a group = the rows of one s;
* 16 features per row (FP64, then rounded to FP32):
   0 log P0(j|s) with P0(j|s) = W1(s\\j) / sum_{j' in s} W1(s\\j')
   1 Deg1(s\\j)            2 Deg1(s) (0 for the full set)
   3 |s| / M               4 1 if j is an electron segment else 0
   5 j / M                 6 w(s\\j) (minus UV degree)
   7 L(s\\j) / n           8 L(s) / n
   9 photons in s / n      10 segments in s / (2n-1)
  11 n / 5                 12 photons in s\\j / n
  13 components of s\\j / M    14 log F1(s) / M        15 1
* MLP: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), d = w3 . h2 + b3,
  widths 16 -> 64 -> 64 -> 1; parameters flat as W1[64x16], b1[64],
  W2[64x64], b2[64], w3[64], b3[1] (5313 floats);
* P_theta(j|s) = softmax over the group of (feature0 + d);
* loss = - sum_rows w_row log P_theta(j|s), w_row = pilot weight of (s, j)
  divided by the graph's total pilot weight;
* Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) with bias correction;
* init: W1, W2 uniform in +-sqrt(3/fan_in) from the seeded input generator,
  all biases and w3 zero (so P_theta = P0 at start).
"""
from __future__ import annotations

import math

import numpy as np

from . import graphs as G
from . import sampler as S

NF = 16
H = 64
NPARAM = H * NF + H + H * H + H + H + 1


def _set_stats(n, chords, mask):
    """(loops, components, photons, segments) of a line set."""
    lines = S.se_lines(n, chords)
    sel = [lines[i] for i in range(len(lines)) if (mask >> i) & 1]
    parent = {}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for _, u, v in sel:
        parent.setdefault(u, u)
        parent.setdefault(v, v)
    comps = len(parent)
    for _, u, v in sel:
        a, b = find(u), find(v)
        if a != b:
            parent[a] = b
            comps -= 1
    loops = len(sel) - len(parent) + comps
    ng = sum(1 for l in sel if l[0] == 'g')
    return loops, comps, ng, len(sel) - ng


def rows_and_features(n, gi, dens=None):
    chords = G.se_graphs(n)[gi]
    if dens is None:
        dens = S.Density(n, chords)
    M = dens.M
    full = (1 << M) - 1
    rows, feats, groups = [], [], []
    for s in range(1, full + 1):
        if bin(s).count('1') < 2:
            continue
        members = [j for j in range(M) if (s >> j) & 1]
        tot = 0.0
        for j in members:
            tot = tot + dens.W1[s & ~(1 << j)]
        Ls, _, _, _ = _set_stats(n, chords, s)
        ng_s = sum(1 for j in members if j >= 2 * n - 1)
        ne_s = len(members) - ng_s
        logF = math.log(dens.F1[s])
        groups.append(len(rows))
        for j in members:
            r = s & ~(1 << j)
            p0 = dens.W1[r] / tot
            Lr, cr, ngr, _ = _set_stats(n, chords, r)
            f = [math.log(p0), dens.deg1[r], dens.deg1[s] if s != full else 0.0,
                 len(members) / M, 1.0 if j < 2 * n - 1 else 0.0, j / M,
                 S.omega(n, chords, r), Lr / n, Ls / n, ng_s / n, ne_s / (2 * n - 1), n / 5.0,
                 ngr / n, cr / M, logF / M, 1.0]
            rows.append((s, j))
            feats.append(f)
    return rows, np.array(feats, dtype=np.float64).astype(np.float32), np.array(groups + [len(rows)])


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def init_draws(seed):
    """The NPARAM uniforms of the seeded initialisation (this library's stream
    layout): uniform k is built from words 0 and 1 of the Philox4x32-10 block
    with counter (k, 0, 0x4D4C50, 0) and key (seed_lo, seed_hi), converted as
    the sampler's uniforms are."""
    from .philox import philox4x32_10, uniform_pair, MASK
    k = np.arange(NPARAM, dtype=np.uint64)
    zero = np.zeros_like(k)
    w = philox4x32_10((k, zero, zero + np.uint64(0x4D4C50), zero), (seed & MASK, (seed >> 32) & MASK))
    return uniform_pair(w[0], w[1])


def init_params(uniform_draws):
    """uniform_draws: NPARAM uniforms in (0,1) from the seeded generator."""
    u = np.asarray(uniform_draws, dtype=np.float64)
    p = np.zeros(NPARAM)
    a1 = math.sqrt(3.0 / NF)
    a2 = math.sqrt(3.0 / H)
    p[:H * NF] = (2 * u[:H * NF] - 1) * a1
    o = H * NF + H
    p[o:o + H * H] = (2 * u[o:o + H * H] - 1) * a2
    return p.astype(np.float32)


def forward(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    d = h2 @ w3 + b3
    return d, (X, h1, h2)


def group_softmax(logits, groups):
    P = np.empty_like(logits)
    for a, b in zip(groups[:-1], groups[1:]):
        v = logits[a:b]
        m = v.max()
        e = np.exp(v - m)
        P[a:b] = e / e.sum()
    return P


def loss_and_grad(p, X, w, groups):
    """Loss and its gradient w.r.t. the flat parameters (FP64)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    d, (X, h1, h2) = forward(p, X)
    logits = np.asarray(X[:, 0], dtype=np.float64) + d
    P = group_softmax(logits, groups)
    loss = -float(np.sum(w * np.log(P)))
    gd = np.empty_like(d)
    for a, b in zip(groups[:-1], groups[1:]):
        gd[a:b] = -w[a:b] + P[a:b] * w[a:b].sum()
    gw3 = h2.T @ gd
    gb3 = gd.sum()
    g2 = np.outer(gd, w3) * (1 - h2 ** 2)
    gW2 = g2.T @ h1
    gb2 = g2.sum(0)
    g1 = (g2 @ W2) * (1 - h1 ** 2)
    gW1 = g1.T @ X
    gb1 = g1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, grad


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def pilot_weights(n, gi, seed, count, chunk=20000):
    """Per-sample pilot weights w_i = sqrt(sum_e y_e^2), y_e = I_e / g, for the
    samples [0, count) of `seed` drawn from the plain density; out-of-double or
    non-finite samples get 0.  Returns (w, paths)."""
    from .estimate import evaluate_points, DBL_MIN
    ws, paths = [], []
    dens = None
    for c0 in range(0, count, chunk):
        cnt = min(chunk, count - c0)
        out, dens = S.sample_graph(n, gi, seed, c0, cnt, dens)
        vals, _ = evaluate_points(n, gi, out['z'])
        with np.errstate(all='ignore'):
            y = np.ldexp(vals / out['gx'][:, None], -out['gj'][:, None])
            w = np.sqrt((y * y).sum(1))
        w[(out['z'].min(1) < DBL_MIN) | ~np.isfinite(w)] = 0.0
        ws.append(w)
        paths.append(out['path'])
    return np.concatenate(ws), np.concatenate(paths)


def pilot_table(n, gi, seed, count, w=None, paths=None):
    """Pilot table of the learned sampler: W(s, j) = sum of q_i over the samples
    whose sector path takes line j from set s, with the integer weights
    q_i = floor(min(w_i / wref, 256) * 2^24) and wref the mean of w over the
    first min(count, 2^23) samples (integers: the table does not depend on the
    order of the additions).  Returns W as float64 [2^M, M]."""
    if w is None:
        w, paths = pilot_weights(n, gi, seed, count)
    M = 3 * n - 1
    m0 = min(count, 1 << 23)
    wref = float(np.mean(w[:m0])) if m0 else 0.0
    W = np.zeros((1 << M, M), dtype=np.int64)
    if not wref > 0.0:
        return W.astype(np.float64)
    q = np.floor(np.minimum(w / wref, 256.0) * 16777216.0).astype(np.int64)
    full = (1 << M) - 1
    for i in range(len(w)):
        if q[i] == 0:
            continue
        s = full
        for l in range(M - 1):
            j = int(paths[i][l])
            W[s, j] += q[i]
            s &= ~(1 << j)
    return W.astype(np.float64)
