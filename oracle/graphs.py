"""Oracle: graph enumeration, UV subgraphs, forests and forest-formula terms.

TEST INFRASTRUCTURE.  Only tests/, the smoke entry point and the bench's CPU
baseline may import this package.  It shares no code with the HIP library.

What is followed (the paper, arXiv:1909.08015):
  * graph set: QED vertex graphs without lepton loops, counted modulo arrow
    reversal (Sec. I, footnote to the 3213-graph statement); gauge-invariant
    classes (k, m, m') (Sec. V, definition before Table I);
  * UV-divergent subgraphs: electron self-energy (N_e=2, N_gamma=0) and
    vertexlike (N_e=2, N_gamma=1), strongly connected and containing every line
    joining their vertexes (Sec. II, with its footnote);
  * overlap, forests, the set F[G] and the set I[G] (Sec. II);
  * the forest operator R^new with the four-case M^{G'}_{G''} (Sec. II,
    equation after the definition of the operator L);
  * the 3n -> 3n-1 variable trick: the two electron lines adjacent to the
    external photon vertex count as one line (Sec. III.A, footnotes).

Readings (the paper does not spell these out):
  * a self-energy (SE) graph with n photons is a perfect matching of the 2n
    vertexes 0..2n-1 of the electron line in which every segment i|i+1 is
    spanned by some photon (1PI); graphs are ordered lexicographically by their
    sorted chord lists;
  * a vertex graph is (S, e): the external photon vertex X sits inside
    electron segment e of S.  In vertex-graph numbering the vertexes are
    0..2n, X = e+1, and SE vertex i maps to i (i <= e) or i+1 (i > e);
  * without lepton loops a UV subgraph has one electron path, so it is an
    interval [a, b] of consecutive vertexes together with every photon whose
    two ends lie in [a, b].
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from functools import lru_cache


# ----------------------------------------------------------------------------
# Enumeration (O1)
# ----------------------------------------------------------------------------

def _matchings(points):
    if not points:
        yield ()
        return
    a = points[0]
    for i in range(1, len(points)):
        b = points[i]
        rest = points[1:i] + points[i + 1:]
        for m in _matchings(rest):
            yield ((a, b),) + m


def is_1pi(chords, nvert):
    """Every segment i|i+1 (0 <= i < nvert-1) is spanned by a chord."""
    for i in range(nvert - 1):
        if not any(a <= i < b for a, b in chords):
            return False
    return True


@lru_cache(maxsize=None)
def se_graphs(n):
    """All n-loop SE graphs without lepton loops, lexicographic order."""
    pts = tuple(range(2 * n))
    out = []
    for m in _matchings(pts):
        ch = tuple(sorted(m))
        if is_1pi(ch, 2 * n):
            out.append(ch)
    out.sort()
    return tuple(out)


def reverse_se(chords, n):
    r = 2 * n - 1
    return tuple(sorted(tuple(sorted((r - a, r - b))) for a, b in chords))


def vertex_class(chords, e):
    """Gauge-invariant class (k, m, m') of the vertex graph (S, e).

    k photons span the external vertex, m and m' photons lie entirely on
    either side; m >= m' (the paper's 'or vice versa')."""
    k = sum(1 for a, b in chords if a <= e < b)
    left = sum(1 for a, b in chords if b <= e)
    right = sum(1 for a, b in chords if a >= e + 1)
    return (k, max(left, right), min(left, right))


def vertex_graphs(n):
    """Oriented vertex graphs (S_index, e) in (S order, e ascending)."""
    return [(i, e) for i, _ in enumerate(se_graphs(n)) for e in range(2 * n - 1)]


def unoriented_vertex_count(n):
    seen = set()
    graphs = se_graphs(n)
    for ch in graphs:
        for e in range(2 * n - 1):
            key = (ch, e)
            mirror = (reverse_se(ch, n), 2 * n - 2 - e)
            seen.add(min(key, mirror))
    return len(seen)


# ----------------------------------------------------------------------------
# Vertex graph structure, UV subgraphs (O2, O3)
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class VertexGraph:
    n: int
    se_chords: tuple      # chords of S in SE numbering
    e: int                # insertion segment of S
    chords: tuple         # chords in vertex-graph numbering
    X: int                # external photon vertex

    @property
    def nvert(self):
        return 2 * self.n + 1


def make_vertex_graph(se_chords, e):
    n = len(se_chords)

    def mp(i):
        return i if i <= e else i + 1
    chords = tuple(sorted((mp(a), mp(b)) for a, b in se_chords))
    return VertexGraph(n, tuple(se_chords), e, chords, e + 1)


def chord_at(vg):
    """Map vertex -> chord index (None for X)."""
    d = {}
    for i, (a, b) in enumerate(vg.chords):
        d[a] = i
        d[b] = i
    return d


def uv_subgraphs(vg):
    """UV-divergent subgraphs as (a, b, kind) with kind 'SE' or 'V'.

    Includes G itself = (0, 2n, 'V')."""
    out = []
    nv = vg.nvert
    for a in range(nv):
        for b in range(a + 1, nv):
            inside = [(c, d) for c, d in vg.chords if a <= c and d <= b]
            # 1PI: every segment v|v+1 with a <= v < b spanned internally
            ok = all(any(c <= v < d for c, d in inside) for v in range(a, b))
            if not ok:
                continue
            crossing = sum(1 for c, d in vg.chords if (a <= c <= b) != (a <= d <= b))
            ngam = crossing + (1 if a <= vg.X <= b else 0)
            if ngam == 0:
                out.append((a, b, 'SE'))
            elif ngam == 1:
                out.append((a, b, 'V'))
    return out


def overlap(s1, s2):
    """Two interval subgraphs overlap: they share a line, neither contains
    the other (Sec. II)."""
    a, b = s1[0], s1[1]
    c, d = s2[0], s2[1]
    share = max(a, c) < min(b, d)
    contains = (a <= c and d <= b) or (c <= a and b <= d)
    return share and not contains


def contains(big, small):
    return big[0] <= small[0] and small[1] <= big[1] and big[:2] != small[:2]


def forests(vg):
    """All forests F in F[G]: sets of pairwise non-overlapping UV subgraphs
    that contain G."""
    subs = uv_subgraphs(vg)
    G = (0, 2 * vg.n, 'V')
    others = [s for s in subs if s[:2] != G[:2]]
    res = []
    # simple backtracking over subsets
    def rec(i, chosen):
        if i == len(others):
            res.append(tuple([G] + chosen))
            return
        rec(i + 1, chosen)
        s = others[i]
        if all(not overlap(s, t) for t in chosen):
            rec(i + 1, chosen + [s])
    rec(0, [])
    return res


def in_I(vg, s):
    """s is in I[G]: vertexlike and contains the external photon vertex."""
    return s[2] == 'V' and s[0] <= vg.X <= s[1]


@dataclass(frozen=True)
class Term:
    sign: int
    forest: tuple          # subgraphs (a, b, kind)
    ops: tuple             # operator per forest element: 'A','U','L','LU'


def terms(vg, expand_lu=False):
    """Terms of R^new_G (Sec. II): one per (F, G') with G' in I[G] cap F.

    Operators: A on G'; U on elements not in I[G] or strictly inside G';
    L on I[G] elements strictly containing G' other than G; (L - U) on G when
    G' != G.  With expand_lu the (L - U) factor gives two terms."""
    G = (0, 2 * vg.n, 'V')
    out = []
    for F in forests(vg):
        sign = -1 if (len(F) - 1) % 2 else 1
        for Gp in F:
            if not in_I(vg, Gp):
                continue
            ops = []
            for Gpp in F:
                if Gpp == Gp:
                    ops.append('A')
                elif (not in_I(vg, Gpp)) or contains(Gp, Gpp):
                    ops.append('U')
                elif Gpp != G:
                    ops.append('L')      # Gpp in I, Gp strictly inside Gpp
                else:
                    ops.append('LU')
            if expand_lu and 'LU' in ops:
                i = ops.index('LU')
                o1 = list(ops); o1[i] = 'L'
                o2 = list(ops); o2[i] = 'U'
                out.append(Term(sign, F, tuple(o1)))
                out.append(Term(-sign, F, tuple(o2)))
            else:
                out.append(Term(sign, F, tuple(ops)))
    return out


# ----------------------------------------------------------------------------
# Level decomposition of a forest term (O4)
# ----------------------------------------------------------------------------

@dataclass
class Level:
    """One forest element with its maximal sub-elements contracted.

    nodes: path items in order from the incoming electron end; each item is
      ('v', vertex) for an ordinary vertex, ('X',) for the external vertex,
      ('c', child_index) for a contracted child element.
    segs: electron lines between consecutive nodes; each is the original
      vertex-graph segment index v (the segment v|v+1).
    photons: (node_i, node_j, chord_index) with node_i < node_j.
    ext_node: node index carrying the level's external photon (vertex type),
      or None (SE type).
    """
    interval: tuple
    kind: str
    op: str
    nodes: list
    segs: list
    photons: list
    ext_node: object
    children: list = field(default_factory=list)   # indices into term levels
    has_X: bool = False


def build_levels(vg, term):
    F = list(term.forest)
    ops = list(term.ops)
    # parent: smallest element strictly containing
    idx = list(range(len(F)))
    parent = {}
    for i in idx:
        best = None
        for j in idx:
            if j != i and contains(F[j], F[i]):
                if best is None or contains(F[best], F[j]):
                    best = j
        parent[i] = best
    cat = chord_at(vg)
    levels = []
    for i in idx:
        a, b, kind = F[i]
        kids = sorted([j for j in idx if parent[j] == i], key=lambda j: F[j][0])
        nodes = []
        segs = []
        v = a
        kid_of_vertex = {}
        for j in kids:
            for w in range(F[j][0], F[j][1] + 1):
                kid_of_vertex[w] = j
        prev_end = None
        while v <= b:
            if v in kid_of_vertex:
                j = kid_of_vertex[v]
                item = ('c', j)
                last = F[j][1]
            elif v == vg.X:
                item = ('X',)
                last = v
            else:
                item = ('v', v)
                last = v
            if prev_end is not None:
                segs.append(prev_end)        # segment prev_end | prev_end+1
            nodes.append(item)
            prev_end = last
            v = last + 1
        # photons of this level: chords with both ends in [a,b] not inside one child
        node_of_vertex = {}
        for k, item in enumerate(nodes):
            if item[0] == 'c':
                j = item[1]
                for w in range(F[j][0], F[j][1] + 1):
                    node_of_vertex[w] = k
            elif item[0] == 'X':
                node_of_vertex[vg.X] = k
            else:
                node_of_vertex[item[1]] = k
        photons = []
        for ci, (c, d) in enumerate(vg.chords):
            if a <= c <= b and a <= d <= b:
                nc, nd = node_of_vertex[c], node_of_vertex[d]
                if nc != nd:
                    photons.append((min(nc, nd), max(nc, nd), ci))
        ext = None
        if kind == 'V':
            if a <= vg.X <= b:
                ext = node_of_vertex[vg.X]
            else:
                for c, d in vg.chords:
                    if (a <= c <= b) != (a <= d <= b):
                        inner = c if a <= c <= b else d
                        ext = node_of_vertex[inner]
        lev = Level((a, b), kind, ops[i], nodes, segs, photons, ext,
                    children=kids, has_X=any(it[0] == 'X' for it in nodes))
        levels.append(lev)
    return levels, parent


def line_index(vg, seg=None, chord=None):
    """Parameter index of a vertex-graph line in the SE-graph numbering:
    SE segments 0..2n-2 then photons 2n-1..3n-2 (order of S's sorted chords).

    The two segments adjacent to X (vertex-graph segments e and e+1) are the
    merged line e (the trick)."""
    n = vg.n
    if seg is not None:
        v = seg
        if v <= vg.e:
            return v
        if v == vg.e + 1:
            return vg.e      # second half of the merged line
        return v - 1
    return 2 * n - 1 + chord
