"""Oracle: graph-specific combinatorial density and its sampler.

TEST INFRASTRUCTURE (see oracle/graphs.py).

Paper (Sec. III.A): Hepp sectors z_{j1} >= ... >= z_{jM}; the density
  g = C1 g1 + C2 g2 + C3 g3 + C4 g4                        (eq. pdf_final)
  g1 = C prod_{l=2}^M (z_{jl}/z_{jl-1})^{Deg(s_l)} / prod z,  s_l = {j_l..j_M}
                                                              (eq. pdf)
with Deg(s) > 0 for every nonempty proper line set; Calc 2 constants
C2 = 0.03, C3 = 0.01, C4 = 0.06, D = 0.75, C1 = 1 - C2 - C3 - C4 (Sec. V);
g stored as x 2^j with 0.5 <= x < 1 and a 32-bit j (Sec. IV.A).

The sampling algorithm, g2..g4 and the Deg(s) algorithm are in references the
paper cites but does not reproduce.  Readings used here (R6-R8):

  * sector coordinates t_l = z_{jl}/z_{jl-1} in (0,1) give
    delta(1-sum z) dz / prod z = prod_{l>=2} dt_l / t_l, so the g1 mass of a
    sector is prod 1/Deg(s_l) and C^{-1} = F(full) with
    F({x}) = 1,  F(s) = sum_{j in s} F(s\\j)/Deg(s\\j)  (j ascending);
  * sampling: choose j_1, j_2, ... one at a time with probability
    W(s\\j)/F(s), W = F/Deg, then t_l = u_l^{1/Deg(s_l)};
  * g2: Deg(s) = |s| (uniform sector choice, F(full) = M);
    g3: Deg3 = D*Deg1 (same sector choice as g1);
    g4: uniform sector choice with g1's continuous part;
  * Deg1(s) = max(C_bigZ, min(C_bigF * w(s), Deg_max)) with w(s) = n_gamma(s)
    + n_e(s)/2 - 2 L(s) the minus-UV-degree of the line set in Feynman-parameter
    scale (Speer's exponent), L(s) its cyclomatic number, and Deg_max = 1.
    Unbiasedness does not depend on this choice; the variance does: near the
    face z_s -> 0 the mixture scales like rho^(min_c Deg_c(s) - |s|) and the
    subtracted integrand like rho^(w_f(s) - |s|), so the variance is finite
    only if min_c Deg_c(s) < 2 w_f(s).  The smallest boundary exponent w_f
    of the subtracted integrands is 1 (every subset of every 1-3 loop graph,
    min over insertions), while C_bigF w(s) reaches 2.9 at 3 loops; the cap
    keeps f/g bounded at every face.

Every arithmetic step is a plain IEEE double operation in a fixed order so
that an independent implementation of the same steps yields identical bits.
"""
from __future__ import annotations

import math
import numpy as np

from . import graphs as G
from .mathfn import amm_exp, amm_log, LN2_HI, LN2_LO, INV_LN2
from .philox import uniforms, graph_uid

CALC2 = dict(cbigz=0.256, cbigf=0.839, cadd=0.786, csubi=0.2, csubse=0.0, csubo=0.2,
             c=(0.9, 0.03, 0.01, 0.06), d=0.75, degmax=1.0)
# C1 = 1 - C2 - C3 - C4 evaluated once in double: 1 - 0.03 - 0.01 - 0.06
CALC2['c'] = (((1.0 - 0.03) - 0.01) - 0.06, 0.03, 0.01, 0.06)
# Calc 1 (Sec. V, the MRG32k3a calculation): C2, C3, C4 = 0.03, 0.035, 0.035, D = 0.75
CALC1 = dict(CALC2, c=(((1.0 - 0.03) - 0.035) - 0.035, 0.03, 0.035, 0.035), d=0.75)


def se_lines(n, chords):
    """Lines of an SE graph as (kind, u, v): segments i|i+1 then photons."""
    lines = [('e', i, i + 1) for i in range(2 * n - 1)]
    lines += [('g', a, b) for a, b in chords]
    return lines


def omega(n, chords, mask):
    """n_gamma + n_e/2 - 2 L for the line set mask (SE-graph numbering)."""
    lines = se_lines(n, chords)
    sel = [lines[i] for i in range(len(lines)) if (mask >> i) & 1]
    ne = sum(1 for l in sel if l[0] == 'e')
    ng = len(sel) - ne
    verts = set()
    parent = {}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for _, u, v in sel:
        for w in (u, v):
            if w not in parent:
                parent[w] = w
            verts.add(w)
    comps = len(verts)
    for _, u, v in sel:
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[ru] = rv
            comps -= 1
    loops = len(sel) - len(verts) + comps
    return ng + ne / 2.0 - 2.0 * loops


def deg_table(n, chords, params=CALC2):
    M = 3 * n - 1
    full = (1 << M) - 1
    deg = np.zeros(1 << M)
    cap = params.get('degmax', 0.0)
    for mask in range(1, full):
        w = params['cbigf'] * omega(n, chords, mask)
        if cap > 0.0:
            w = min(w, cap)
        deg[mask] = max(params['cbigz'], w)
    return deg


def f_table(deg, M):
    """F(s) and W(s) = F(s)/Deg(s) over all masks (W only for proper s)."""
    full = (1 << M) - 1
    F = np.zeros(1 << M)
    W = np.zeros(1 << M)
    for mask in range(1, full + 1):
        if mask & (mask - 1) == 0:
            F[mask] = 1.0
        else:
            acc = 0.0
            for j in range(M):
                if (mask >> j) & 1:
                    acc = acc + W[mask & ~(1 << j)]
            F[mask] = acc
        if mask != full:
            W[mask] = F[mask] / deg[mask]
    return F, W


class Density:
    """Tables of the four-component density of one SE graph."""

    def __init__(self, n, chords, params=CALC2, deg=None):
        self.n = n
        self.M = M = 3 * n - 1
        self.full = (1 << M) - 1
        self.params = params
        self.deg1 = deg if deg is not None else deg_table(n, chords, params)
        self.F1, self.W1 = f_table(self.deg1, M)
        D = params['d']
        self.deg3 = np.array([D * d for d in self.deg1])
        self.logdeg1 = np.zeros(1 << M)
        ok = self.deg1 > 0
        self.logdeg1[ok] = amm_log(self.deg1[ok])
        c = params['c']
        self.logc = [float(amm_log(ci)) if ci > 0 else -np.inf for ci in c]
        logF1 = float(amm_log(self.F1[self.full]))
        logM = float(amm_log(float(M)))
        logMfact = float(amm_log(float(math.factorial(M))))
        logD = float(amm_log(D))
        # log K_c (path-independent part)
        self.logK = [-logF1, -logM, float(M - 1) * logD - logF1, -logMfact]

    def sample(self, u, ptheta=None):
        """u: (N, 2M-1) uniforms (2M with a learned table).  Returns dict with
        z (N, M), path (N, M), and the density as (x, j) with g = x 2^j.

        With ptheta (P_theta(j|s) as a [2^M, M] float32 table) the density is
        the learned mixture q = (q_theta + g)/2: uniform 2M-1 picks q_theta
        (component 4) when below 1/2; q_theta chooses sectors by the table and
        shares g1's continuous part."""
        M = self.M
        N = u.shape[0]
        comp = np.zeros(N, dtype=np.int64)
        c = self.params['c']
        thr = u[:, 0]
        cum = 0.0
        comp[:] = 3
        chosen = np.zeros(N, dtype=bool)
        for ci in range(4):
            cum = cum + c[ci]
            take = (~chosen) & (thr < cum)
            comp[take] = ci
            chosen |= take
        if ptheta is not None:
            P = np.asarray(ptheta, dtype=np.float32).astype(np.float64)
            comp[u[:, 2 * M - 1] < 0.5] = 4
        path = np.zeros((N, M), dtype=np.int64)
        s = np.full(N, self.full, dtype=np.int64)
        uniform_sel = (comp == 1) | (comp == 3)
        for l in range(M - 1):
            ul = u[:, 1 + l]
            # g1 / g3 weights
            total = np.zeros(N)
            for j in range(M):
                inset = ((s >> j) & 1).astype(bool)
                w = np.where(inset, self.W1[s & ~(1 << j)], 0.0)
                total = total + w
            t = ul * total
            cumw = np.zeros(N)
            pick = np.full(N, -1, dtype=np.int64)
            last = np.full(N, -1, dtype=np.int64)
            for j in range(M):
                inset = ((s >> j) & 1).astype(bool)
                w = np.where(inset, self.W1[s & ~(1 << j)], 0.0)
                cumw = cumw + w
                hit = inset & (pick < 0) & (t < cumw)
                pick[hit] = j
                last[inset] = j
            pick = np.where(pick < 0, last, pick)
            # uniform choice for g2 / g4: k-th element ascending
            size = np.zeros(N, dtype=np.int64)
            for j in range(M):
                size += (s >> j) & 1
            k = np.floor(ul * size.astype(np.float64)).astype(np.int64)
            upick = np.full(N, -1, dtype=np.int64)
            cnt = np.zeros(N, dtype=np.int64)
            for j in range(M):
                inset = ((s >> j) & 1).astype(bool)
                hit = inset & (cnt == k) & (upick < 0)
                upick[hit] = j
                cnt += inset
            pick = np.where(uniform_sel, upick, pick)
            if ptheta is not None:
                # table choice for component 4
                ttot = np.zeros(N)
                for j in range(M):
                    inset = ((s >> j) & 1).astype(bool)
                    ttot = ttot + np.where(inset, P[s, j], 0.0)
                tt = ul * ttot
                cumw = np.zeros(N)
                tpick = np.full(N, -1, dtype=np.int64)
                tlast = np.full(N, -1, dtype=np.int64)
                for j in range(M):
                    inset = ((s >> j) & 1).astype(bool)
                    cumw = cumw + np.where(inset, P[s, j], 0.0)
                    hit = inset & (tpick < 0) & (tt < cumw)
                    tpick[hit] = j
                    tlast[inset] = j
                tpick = np.where(tpick < 0, tlast, tpick)
                pick = np.where(comp == 4, tpick, pick)
            path[:, l] = pick
            s = s & ~(np.int64(1) << pick)
        # last line
        lastj = np.zeros(N, dtype=np.int64)
        for j in range(M):
            lastj[((s >> j) & 1).astype(bool)] = j
        path[:, M - 1] = lastj
        # continuous part: t_l, l = 2..M, with s_l = set of path[l-1..]
        masks = np.zeros((N, M), dtype=np.int64)
        acc = np.zeros(N, dtype=np.int64)
        for l in range(M - 1, -1, -1):
            acc = acc | (np.int64(1) << path[:, l])
            masks[:, l] = acc
        logt = np.zeros((N, M))
        for l in range(1, M):
            sl = masks[:, l]
            d1 = self.deg1[sl]
            size = np.zeros(N)
            for j in range(M):
                size = size + ((sl >> j) & 1)
            dsel = np.where(comp == 1, size, np.where(comp == 2, self.deg3[sl], d1))
            logt[:, l] = amm_log(u[:, M + l - 1]) / dsel
        tt = amm_exp(logt)
        p = np.ones((N, M))
        lp = np.zeros((N, M))
        for l in range(1, M):
            p[:, l] = p[:, l - 1] * tt[:, l]
            lp[:, l] = lp[:, l - 1] + logt[:, l]
        norm = np.zeros(N)
        for l in range(M):
            norm = norm + p[:, l]
        z = np.zeros((N, M))
        for l in range(M):
            z[np.arange(N), path[:, l]] = p[:, l] / norm
        lognorm = amm_log(norm)
        sumlogz = np.zeros(N)
        for l in range(M):
            sumlogz = sumlogz + lp[:, l]
        sumlogz = sumlogz - float(M) * lognorm
        # component exponents E_c = sum_l Deg_c(s_l) log t_l
        E = np.zeros((4, N))
        logdegsum = np.zeros(N)
        for l in range(1, M):
            sl = masks[:, l]
            size = np.zeros(N)
            for j in range(M):
                size = size + ((sl >> j) & 1)
            E[0] = E[0] + self.deg1[sl] * logt[:, l]
            E[1] = E[1] + size * logt[:, l]
            E[2] = E[2] + self.deg3[sl] * logt[:, l]
            logdegsum = logdegsum + self.logdeg1[sl]
        E[3] = E[0]
        Lc = np.zeros((4, N))
        for ci in range(4):
            Lc[ci] = (self.logc[ci] + self.logK[ci]) + E[ci]
        Lc[3] = Lc[3] + logdegsum
        ncomp = 4
        if ptheta is not None:
            loghalf = float(amm_log(0.5))
            sumlogp = np.zeros(N)
            for l in range(M - 1):
                sl = masks[:, l]
                tot = np.zeros(N)
                for j in range(M):
                    tot = tot + np.where(((sl >> j) & 1).astype(bool), P[sl, j], 0.0)
                sumlogp = sumlogp + amm_log(P[sl, path[:, l]] / tot)
            Lt = ((loghalf + sumlogp) + logdegsum) + E[0]
            Lc = np.vstack([Lc + loghalf, Lt[None, :]])
            ncomp = 5
        Lmax = np.maximum(np.maximum(Lc[0], Lc[1]), np.maximum(Lc[2], Lc[3]))
        if ncomp == 5:
            Lmax = np.maximum(Lmax, Lc[4])
        S = np.zeros(N)
        for ci in range(ncomp):
            S = S + amm_exp(Lc[ci] - Lmax)
        Ltot = Lmax - sumlogz
        k = np.rint(Ltot * INV_LN2)
        r = (Ltot - k * LN2_HI) - k * LN2_LO
        x0 = amm_exp(r) * S
        xm, e = np.frexp(x0)
        j = k.astype(np.int64) + e
        return dict(z=z, path=path, comp=comp, gx=xm, gj=j, logt=logt)


def sample_graph(n, gi, seed, start, count, dens=None, params=CALC2, ptheta=None):
    chords = G.se_graphs(n)[gi]
    if dens is None:
        dens = Density(n, chords, params)
    idx = np.arange(start, start + count, dtype=np.uint64)
    u = uniforms(seed, graph_uid(n, gi), idx, 2 * dens.M - (1 if ptheta is None else 0))
    out = dens.sample(u, ptheta)
    out['u'] = u
    return out, dens


def g_value(gx, gj):
    return np.ldexp(gx, gj)
