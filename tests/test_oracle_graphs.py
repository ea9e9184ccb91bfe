"""Oracle pins: enumeration, classes, subgraphs and forest terms.

Pinned against the paper's printed counts (Sec. I: 3213 graphs; Table I:
N_diag per class) and the structure of eq. (example_expression), and against
an independent brute force written here."""
import itertools
import json
import os

import pytest

from oracle import graphs as G

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'paper_counts.json')))


def brute_se(n):
    """Independent brute force: every pairing of 2n points, 1PI checked by
    deleting each electron segment and testing connectivity."""
    out = set()
    pts = list(range(2 * n))
    for perm in itertools.permutations(pts):
        pairs = tuple(sorted(tuple(sorted(perm[i:i + 2])) for i in range(0, 2 * n, 2)))
        if pairs in out:
            continue
        ok = True
        for cut in range(2 * n - 1):
            edges = [(i, i + 1) for i in range(2 * n - 1) if i != cut] + list(pairs)
            comp = {0}
            changed = True
            while changed:
                changed = False
                for a, b in edges:
                    if (a in comp) != (b in comp):
                        comp |= {a, b}
                        changed = True
            if len(comp) != 2 * n:
                ok = False
                break
        if ok:
            out.add(pairs)
    return sorted(out)


@pytest.mark.parametrize('n', [1, 2, 3, 4])
def test_se_graphs_match_brute_force(n):
    assert list(G.se_graphs(n)) == brute_se(n)


def test_counts_per_loop_order():
    assert [len(G.se_graphs(n)) for n in range(1, 6)] == [1, 2, 10, 74, 706]
    assert [len(G.vertex_graphs(n)) for n in range(1, 6)] == [1, 6, 50, 518, 6354]
    assert [G.unoriented_vertex_count(n) for n in range(1, 5)] == [1, 4, 28, 269]


def test_paper_3213_and_table1():
    n = 5
    assert G.unoriented_vertex_count(n) == GOLD['unoriented_vertex_graphs_5loop']
    seen = set()
    cnt = {}
    for ch in G.se_graphs(n):
        for e in range(2 * n - 1):
            key = min((ch, e), (G.reverse_se(ch, n), 2 * n - 2 - e))
            if key in seen:
                continue
            seen.add(key)
            c = ','.join(map(str, G.vertex_class(ch, e)))
            cnt[c] = cnt.get(c, 0) + 1
    assert cnt == GOLD['table1_ndiag']


def test_term_totals():
    tot = []
    for n in (1, 2, 3):
        t = 0
        for ch in G.se_graphs(n):
            for e in range(2 * n - 1):
                t += len(G.terms(G.make_vertex_graph(ch, e), expand_lu=True))
        tot.append(t)
    assert tot == [1, 13, 203]


def test_one_loop_term_is_A():
    vg = G.make_vertex_graph(G.se_graphs(1)[0], 0)
    T = G.terms(vg)
    assert len(T) == 1 and T[0].ops == ('A',) and T[0].sign == 1


def test_example_expression_structure():
    """eq. (example_expression): [A_G(1-U_x)-(L_G-U_G)A_x](1-U)(1-U)(1-U-U)
    with x = bcdefghij (vertexes b..j of a..k), cd, fghi, fgh, ghi: 48 terms.
    Search the 5-loop set for vertex graphs with exactly that UV-subgraph
    family and check the expansion."""
    want = {(1, 9), (2, 3), (5, 8), (5, 7), (6, 8)}
    found = 0
    for ch in G.se_graphs(5):
        for e in range(9):
            vg = G.make_vertex_graph(ch, e)
            subs = G.uv_subgraphs(vg)
            ivs = {(a, b) for a, b, k in subs if (a, b) != (0, 10)}
            if ivs != want:
                continue
            kinds = {(a, b): k for a, b, k in subs}
            assert kinds[(1, 9)] == 'V' and G.in_I(vg, (1, 9, 'V'))
            T = G.terms(vg, expand_lu=True)
            assert len(T) == 48
            # operator content: A on G or on x; x gets U, A or nothing
            for t in T:
                ops = dict(zip([s[:2] for s in t.forest], t.ops))
                assert ops[(0, 10)] in ('A', 'L', 'U')
                if ops[(0, 10)] != 'A':
                    assert ops[(1, 9)] == 'A'
                # fgh and ghi overlap: never together
                assert not ((5, 7) in ops and (6, 8) in ops)
            found += 1
    assert found >= 1


def test_overlap_definition():
    # share a line, neither contains the other
    assert G.overlap((1, 4, 'V'), (3, 6, 'V'))
    assert not G.overlap((1, 4, 'V'), (4, 6, 'V'))     # share only a vertex
    assert not G.overlap((1, 6, 'V'), (2, 3, 'SE'))    # nested
