"""Oracle: the forest-subtracted AMM integrand I_{S,e}(z) of a vertex graph.

TEST INFRASTRUCTURE (see oracle/graphs.py).

The paper (Sec. II) defines the operators A, U, L and the forest sum R^new and
says the operators act on subgraph amplitudes in Feynman-parametric space via
Schwinger parameters; it does not print the parametric integrand.  This module
writes that integrand out from first principles (readings R3/R4):

Level.  Each forest element G_i with its maximal sub-elements contracted is a
level with L_i loops and N_i lines.  Its Schwinger-parametric amplitude, after
the Gaussian loop integration, has the numerator expanded in Wick contractions;
with c_i contractions the level contributes

    4^{-L_i} (-1)^{N_i} (-1/2)^{c_i} U_i^{-2} * proj(N_{c_i})

where U_i = det Lambda_i (Lambda_i = loop-momentum quadratic form),
a contraction of the momenta of lines l, l' gives x_{ll'} g^{mu nu} with
x_{ll'} = s_l^T Lambda_i^{-1} s_l' and an uncontracted electron momentum is
A_l P (+ C_l q), A and C being Kirchhoff currents with resistances z.

Term.  All levels share one overall scale (alpha = lambda z on the common
simplex, Sec. II last paragraphs), so a term is

    sign * sum_c [conv_c prod_i f_i(c_i)] * Gamma(n-c) / V^{n-c},
    V = sum_i V_i,  V_i = sigma^T Lambda_i^{-1} sigma  (on shell, m = 1).

Projections (m = 1, P^2 = 1):
  SE + U:     u = Tr[N]/4,  v = Tr[Pslash N]/4     (U Sigma = u + v pslash)
  vertex at q=0, Gamma_mu(p,0) = a gamma + b p + c pslash p + d[..]
              (eq. gamma_general_q0):  X = Tr[N_mu gamma^mu], Y = Tr[P N_mu P^mu],
              Z = Tr[N_mu P^mu];  a = (X-Y)/12,  b + c = Z/4 + (4Y-X)/12,
              a + b + c = (Y+Z)/4
              U -> a,  L -> a+b+c,  (L-U) -> b+c
  A (AMM):    F2 = (T_sigma/q^2 - 3 T_gamma)/16 with
              T_gamma = Tr[(P+1) Gamma_mu (P+1) gamma^mu] at q = 0 and
              T_sigma = Tr[(p'+1) Gamma_mu (p+1) [gamma^mu, qslash]] to O(q^2),
              p = P - q/2, p' = P + q/2; the q^alpha q^beta average over the
              three unit spacelike directions orthogonal to P.

Trick (Sec. III.A footnote): the two lines next to the external vertex carry
the same loop momentum; their Schwinger parameters are written as
alpha_e * (x, 1-x); the integrand is affine in x, so integrating x equals
evaluating at x = 1/2, and the Jacobian gives a factor z_e.

Everything here is a rational function of z, so the same code runs on
Fractions (exact reference) and on numpy float64 arrays (vectorised points).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
import math

import numpy as np

from . import graphs as G
from .dirac import I4, PSLASH, Q_DIRS, slash, trace_chain, exact_int

HALF = Fraction(1, 2)


# ----------------------------------------------------------------------------
# Chains and polynomial coefficients of one level
# ----------------------------------------------------------------------------

def _node_photon(vg, lev, forest, node):
    """Chord index attached to a node, or 'X' for the external vertex."""
    if node[0] == 'v':
        return G.chord_at(vg)[node[1]]
    if node[0] == 'X':
        return 'X'
    a, b, kind = forest[node[1]]
    if a <= vg.X <= b:
        return 'X'
    for ci, (c, d) in enumerate(vg.chords):
        if (a <= c <= b) != (a <= d <= b):
            return ci
    return None        # SE child


def level_chain(vg, lev, forest, choice):
    """Chain items in matrix order (last node first).

    Items: ('g', label) gamma with label ('ph', ci) or 'mu';
           ('seg', k) propagator of level segment k (between nodes k-1, k);
           ('kv', k)  v-insertion kslash with the momentum of segment k."""
    level_chords = {p[2] for p in lev.photons}
    items = []
    K = len(lev.nodes) - 1
    for k in range(K, -1, -1):
        node = lev.nodes[k]
        ph = _node_photon(vg, lev, forest, node)
        if ph is None:                      # contracted SE child
            if choice[k] == 'v':
                items.append(('kv', k))
        elif ph != 'X' and ph in level_chords:
            items.append(('g', ('ph', ph)))
        else:
            items.append(('g', 'mu'))
        if k > 0:
            items.append(('seg', k))
    return items


def _partial_matchings(slots):
    if not slots:
        yield [], []
        return
    first, rest = slots[0], slots[1:]
    for pairs, un in _partial_matchings(rest):
        yield pairs, [first] + un
    for i, s in enumerate(rest):
        rest2 = rest[:i] + rest[i + 1:]
        for pairs, un in _partial_matchings(rest2):
            yield [(first, s)] + pairs, un


def _sub_mu(factors, repl):
    return [repl if (isinstance(f, tuple) and f[1] == 'mu') else f for f in factors]


def _comm_mu_q(q):
    """[gamma^mu, qslash] as two factor lists with coefficients."""
    return [(1, [('idx', 'mu'), q]), (-1, [q, ('idx', 'mu')])]


_POLY_STORE = {}


def _level_poly_cached(key):
    if key not in _POLY_STORE:
        items, op, kind = key
        _POLY_STORE[key] = _level_poly(list(items), op, kind)
    return _POLY_STORE[key]


def _level_poly(items, op, kind):
    """Numerator polynomial(s) of a level: {output: {monomial: Fraction}}.

    monomial = (pairs, Alist, Cseg): pairs are sorted (k, k') segment pairs,
    Alist sorted segment ids carrying A_k P-slash, Cseg a segment carrying
    C_k q-slash (A-level only) or -1."""
    kpos = [i for i, it in enumerate(items) if it[0] in ('seg', 'kv')]
    out = {}

    def add(name, mono, val):
        d = out.setdefault(name, {})
        d[mono] = d.get(mono, 0) + val

    P1 = PSLASH + I4
    for pairs, un in _partial_matchings(kpos):
        pair_lab = {}
        for t, (i, j) in enumerate(pairs):
            pair_lab[i] = ('idx', ('k', t))
            pair_lab[j] = ('idx', ('k', t))
        mono_pairs = tuple(sorted(tuple(sorted((items[i][1], items[j][1]))) for i, j in pairs))
        nun = len(un)
        c_opts = [None] + (list(range(nun)) if op == 'A' else [])
        # a v-insertion slot is kslash alone: it has no mass term
        kv_mask = sum(1 << t for t in range(nun) if items[un[t]][0] == 'kv')
        for amask in range(1 << nun):
            for cpos in c_opts:
                if cpos is not None and (amask >> cpos) & 1:
                    continue
                chosen = amask | (0 if cpos is None else 1 << cpos)
                if kv_mask & ~chosen:
                    continue
                Alist = tuple(sorted(items[un[t]][1] for t in range(nun) if (amask >> t) & 1))
                Cseg = items[un[cpos]][1] if cpos is not None else -1
                mono = (mono_pairs, Alist, Cseg)

                def chain(qs):
                    f = []
                    for i, it in enumerate(items):
                        if it[0] == 'g':
                            f.append(('idx', it[1]))
                        elif i in pair_lab:
                            f.append(pair_lab[i])
                        else:
                            t = un.index(i)
                            if cpos == t:
                                f.append(qs)
                            elif (amask >> t) & 1:
                                f.append(PSLASH)
                            else:
                                f.append(I4)
                    return f

                if kind == 'SE':
                    ch = chain(None)
                    add('u', mono, Fraction(exact_int(trace_chain(ch)), 4))
                    add('v', mono, Fraction(exact_int(trace_chain([PSLASH] + ch)), 4))
                    continue
                if op in ('U', 'L', 'LU'):
                    ch = chain(None)
                    X = exact_int(trace_chain(ch + [('idx', 'mu')]))
                    Y = exact_int(trace_chain([PSLASH] + _sub_mu(ch, PSLASH)))
                    Z = exact_int(trace_chain(_sub_mu(ch, PSLASH)))
                    if op == 'U':
                        v = Fraction(X - Y, 12)
                    elif op == 'L':
                        v = Fraction(Y + Z, 4)
                    else:
                        v = Fraction(Z, 4) + Fraction(4 * Y - X, 12)
                    add('s', mono, v)
                    continue
                # AMM projector
                tsig = Fraction(0)
                tgam = 0
                if cpos is None:
                    ch = chain(None)
                    tgam = exact_int(trace_chain([P1] + ch + [P1, ('idx', 'mu')]))
                    for q in Q_DIRS:
                        qs = slash(q)
                        for sgn, cm in _comm_mu_q(qs):
                            t1 = exact_int(trace_chain([qs] + ch + [P1] + cm))
                            t2 = exact_int(trace_chain([P1] + ch + [qs] + cm))
                            tsig += Fraction(sgn * (t1 - t2), 2)
                else:
                    for q in Q_DIRS:
                        qs = slash(q)
                        ch = chain(qs)
                        for sgn, cm in _comm_mu_q(qs):
                            tsig += sgn * exact_int(trace_chain([P1] + ch + [P1] + cm))
                # T_sigma / q^2 = -(1/3) sum_dirs T2(dir)   (q^2 = -1)
                f2 = (-tsig / 3 - 3 * tgam) / 16
                add('s', mono, f2)
    # drop zeros
    return {k: {m: v for m, v in d.items() if v != 0} for k, d in out.items()}


# ----------------------------------------------------------------------------
# Per-point quantities of a level graph (generic arithmetic)
# ----------------------------------------------------------------------------

def _solve(Lam, rhs_list):
    """Gaussian elimination (no pivoting; Lambda is symmetric positive
    definite).  Works entrywise on Fractions, floats or numpy arrays."""
    n = len(Lam)
    A = [row[:] for row in Lam]
    B = [list(r) for r in rhs_list]       # each rhs a list of length n
    det = 1
    for i in range(n):
        piv = A[i][i]
        det = det * piv
        for r in range(i + 1, n):
            f = A[r][i] / piv
            for c in range(i, n):
                A[r][c] = A[r][c] - f * A[i][c]
            for b in B:
                b[r] = b[r] - f * b[i]
    sols = []
    for b in B:
        x = [0] * n
        for i in range(n - 1, -1, -1):
            s = b[i]
            for c in range(i + 1, n):
                s = s - A[i][c] * x[c]
            x[i] = s / A[i][i]
        sols.append(x)
    return det, sols


def level_quantities(vg, lev, z, zero, one):
    """U, V, x_{kk'}, A_k, C_k for a level at point z (list by parameter)."""
    half = HALF if isinstance(one, Fraction) else 0.5
    K = len(lev.nodes) - 1
    zseg = {}
    for k in range(1, K + 1):
        v = lev.segs[k - 1]
        zi = z[G.line_index(vg, seg=v)]
        if v in (vg.X - 1, vg.X):        # halves of the merged line
            zi = zi * half
        zseg[k] = zi
    ph = lev.photons
    L = len(ph)
    span = [[k for k in range(1, K + 1) if p[0] <= k - 1 and k <= p[1]] for p in ph]
    Lam = [[zero] * L for _ in range(L)]
    for a in range(L):
        Lam[a][a] = Lam[a][a] + z[G.line_index(vg, chord=ph[a][2])]
        for b in range(L):
            for k in span[a]:
                if k in span[b]:
                    Lam[a][b] = Lam[a][b] + zseg[k]
    sigma = [sum((zseg[k] for k in span[a]), zero) for a in range(L)]
    # unit vectors for x_{kk'}: s_k = indicator of photons spanning k
    svec = {k: [one if k in span[a] else zero for a in range(L)] for k in range(1, K + 1)}
    rhs = [sigma] + [svec[k] for k in range(1, K + 1)]
    C0 = None
    if lev.op == 'A':
        x = lev.ext_node
        C0 = {k: (-half if k <= x else half) for k in range(1, K + 1)}
        jc = [sum((zseg[k] * C0[k] for k in span[a]), zero) for a in range(L)]
        rhs.append(jc)
    U, sols = _solve(Lam, rhs)
    ell = sols[0]
    inv_s = {k: sols[k] for k in range(1, K + 1)}
    V = sum((sigma[a] * ell[a] for a in range(L)), zero)
    A = {k: one - sum((ell[a] for a in range(L) if k in span[a]), zero) for k in range(1, K + 1)}
    X = {}
    for k in range(1, K + 1):
        for k2 in range(k, K + 1):
            X[(k, k2)] = sum((svec[k][a] * inv_s[k2][a] for a in range(L)), zero)
    C = None
    if lev.op == 'A':
        ellc = sols[-1]
        C = {k: C0[k] - sum((ellc[a] for a in range(L) if k in span[a]), zero)
             for k in range(1, K + 1)}
    nlines = K + L
    return dict(U=U, V=V, X=X, A=A, C=C, L=L, N=nlines)


def eval_poly(poly, q, zero, maxc):
    """Evaluate {mono: coef} into a c-vector of length maxc+1."""
    vec = [zero] * (maxc + 1)
    X, A, C = q['X'], q['A'], q['C']
    for (pairs, Al, Cs), coef in poly.items():
        t = coef
        for p in pairs:
            t = t * X[p]
        for k in Al:
            t = t * A[k]
        if Cs != -1:
            t = t * C[Cs]
        vec[len(pairs)] = vec[len(pairs)] + t
    return vec


def _conv(a, b, zero):
    out = [zero] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = out[i + j] + x * y
    return out


# ----------------------------------------------------------------------------
# Term and vertex-graph integrand
# ----------------------------------------------------------------------------

def _conv_num(x):
    return x


def term_value(vg, term, z, exact):
    """Value of one forest term at z; returns (value, V_total)."""
    levels, parent = G.build_levels(vg, term)
    forest = term.forest
    if exact == 'ld':
        # x87 extended precision (64-bit significand), elementwise in numpy:
        # a reference about 2^11 times finer than FP64 for vectorised points
        zero, one = np.longdouble(0), np.longdouble(1)
        conv_coef = lambda c: np.longdouble(c.numerator) / np.longdouble(c.denominator)
    elif exact:
        zero, one = Fraction(0), Fraction(1)
        conv_coef = lambda c: c
    else:
        zero, one = 0.0, 1.0
        conv_coef = float
    quants = [level_quantities(vg, lv, z, zero, one) for lv in levels]
    Vtot = sum((q['V'] for q in quants), zero)
    n = vg.n

    def value(i):
        lv = levels[i]
        q = quants[i]
        se_kids = [k for k, nd in enumerate(lv.nodes)
                   if nd[0] == 'c' and forest[nd[1]][2] == 'SE']
        v_kids = [nd[1] for nd in lv.nodes if nd[0] == 'c' and forest[nd[1]][2] == 'V']
        pref_base = Fraction(1, 4 ** q['L']) * (-1) ** q['N']
        U2 = q['U'] * q['U']
        if lv.has_X:
            zfac = z[vg.e]
        else:
            zfac = one
        results = {}
        for mask in range(1 << len(se_kids)):
            choice = {}
            for t, k in enumerate(se_kids):
                choice[k] = 'v' if (mask >> t) & 1 else 'u'
            items = tuple(level_chain(vg, lv, forest, choice))
            kind = 'SE' if lv.kind == 'SE' else 'V'
            poly = _level_poly_cached((items, lv.op, kind))
            maxc = len([it for it in items if it[0] in ('seg', 'kv')]) // 2
            for name, pd in poly.items():
                pdc = {m: conv_coef(c) for m, c in pd.items()}
                vec = eval_poly(pdc, q, zero, maxc)
                vec = [conv_coef(pref_base * Fraction(-1, 2) ** c) * vec[c] / U2 * zfac
                       for c in range(len(vec))]
                # children
                for t, k in enumerate(se_kids):
                    child = lv.nodes[k][1]
                    cv = value(child)[choice[k]]
                    vec = _conv(vec, cv, zero)
                for child in v_kids:
                    vec = _conv(vec, value(child)['s'], zero)
                if name in results:
                    r = results[name]
                    m = max(len(r), len(vec))
                    r = r + [zero] * (m - len(r))
                    vec = vec + [zero] * (m - len(vec))
                    results[name] = [a + b for a, b in zip(r, vec)]
                else:
                    results[name] = vec
        return results

    root = [i for i in range(len(levels)) if parent[i] is None][0]
    vec = value(root)['s']
    tot = zero
    for c, coef in enumerate(vec):
        if c >= n:
            # Gamma(n - c) diverges for c >= n, so a finite integrand needs
            # this coefficient to vanish identically; it is checked at every
            # evaluation instead of being dropped.
            if np.any(np.asarray(coef) != 0):
                raise ArithmeticError(f'non-zero Gamma({n - c}) coefficient {coef!r}')
            continue
        g = math.factorial(n - c - 1)
        tot = tot + coef * g / Vtot ** (n - c)
    return term.sign * tot, vec


def vertex_integrand(vg, z, exact=False, with_terms=False):
    """I_{S,e}(z) summed over forest terms; z indexed by SE-graph parameter
    (segments 0..2n-2, photons 2n-1..3n-2).  Also returns sum |term|."""
    if exact == 'ld':
        tot, absum = np.longdouble(0), np.longdouble(0)
    else:
        tot = 0 if not exact else Fraction(0)
        absum = 0 if not exact else Fraction(0)
    vals = []
    for t in G.terms(vg):
        v, _ = term_value(vg, t, z, exact)
        tot = tot + v
        absum = absum + abs(v)
        vals.append(v)
    if with_terms:
        return tot, absum, vals
    return tot, absum


def se_integrands(n, gi, z, exact=False):
    """All 2n-1 insertion integrands of SE graph gi at point z."""
    ch = G.se_graphs(n)[gi]
    out = []
    for e in range(2 * n - 1):
        vg = G.make_vertex_graph(ch, e)
        out.append(vertex_integrand(vg, z, exact))
    return out


# ----------------------------------------------------------------------------
# Persisting the oracle's own level polynomials (they are slow to derive with
# explicit matrices).  Only files written by dump_poly_cache are read back.
# ----------------------------------------------------------------------------

def _key_to_str(key):
    return repr(key)


def dump_poly_cache(path):
    import gzip
    import json
    out = {}
    for key in list(_POLY_STORE.keys()):
        polys = _POLY_STORE[key]
        out[_key_to_str(key)] = {name: [[list(map(list, m[0])), list(m[1]), m[2], f'{c.numerator}/{c.denominator}']
                                        for m, c in d.items()] for name, d in polys.items()}
    with gzip.open(path, 'wt') as f:
        json.dump(out, f)


def load_poly_cache(path):
    import ast
    import gzip
    import json
    with gzip.open(path, 'rt') as f:
        data = json.load(f)
    for ks, polys in data.items():
        key = ast.literal_eval(ks)
        _POLY_STORE[key] = {name: {(tuple(tuple(p) for p in m[0]), tuple(m[1]), m[2]): Fraction(m[3])
                                   for m in lst} for name, lst in polys.items()}
