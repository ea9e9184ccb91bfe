// amm_host.cpp -- host-side plan builder.
//
// Builds, for every SE graph of one loop order:
//   * the graph set (Sec. I: QED graphs without lepton loops; 1PI electron
//     self-energy graphs with the external photon inserted in a segment),
//   * the UV-divergent subgraphs, forests and forest-formula terms of each
//     insertion (Sec. II: self-energy and vertexlike subgraphs, overlap,
//     F[G], I[G], R^new with the four-case operator M),
//   * per level (forest element with its maximal sub-elements contracted) the
//     numerator polynomial after Wick contraction and projection (A: AMM;
//     U, L per eq. gamma_general_q0; U on self-energies),
//   * the density tables of Sec. III.A (Deg(s), the normalisation DP).
//
// Dirac traces are reduced symbolically with the 4-dimensional contraction
// identities  g^a S g_a = -2 S^R (|S| odd),  2 (S_n S_1..S_{n-1} +
// S_{n-1}..S_1 S_n) (|S| even >= 2), 4 (S empty), and P-slash^2 = m^2 = 1.
#include "amm_host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <thread>
#include <atomic>

namespace amm {

// ---------------------------------------------------------------------------
// exp / log with the fixed evaluation order of the sampler (Cody-Waite
// reduction + Taylor; atanh series).  Host copy used for table constants.
// ---------------------------------------------------------------------------
double host_log(double x) {
    int k;
    double m = std::frexp(x, &k);
    if (m < AMM_SQRT_HALF) { m = m * 2.0; k = k - 1; }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
    double q = amm_log_d(11);
    for (int i = 10; i >= 0; --i) q = q * s + amm_log_d(i);
    double lm = (2.0 * f) * q;
    double kd = (double)k;
    return (kd * AMM_LN2_LO + lm) + kd * AMM_LN2_HI;
}

// ---------------------------------------------------------------------------
// Graphs
// ---------------------------------------------------------------------------
static void matchings(std::vector<int> &pts, std::vector<std::pair<int, int>> &cur,
                      std::vector<std::vector<std::pair<int, int>>> &out) {
    if (pts.empty()) { out.push_back(cur); return; }
    int a = pts[0];
    for (size_t i = 1; i < pts.size(); ++i) {
        int b = pts[i];
        std::vector<int> rest;
        for (size_t k = 1; k < pts.size(); ++k) if (k != i) rest.push_back(pts[k]);
        cur.push_back({a, b});
        matchings(rest, cur, out);
        cur.pop_back();
    }
}

std::vector<SEGraph> enumerate_se(int n) {
    std::vector<int> pts(2 * n);
    for (int i = 0; i < 2 * n; ++i) pts[i] = i;
    std::vector<std::vector<std::pair<int, int>>> all;
    std::vector<std::pair<int, int>> cur;
    matchings(pts, cur, all);
    std::vector<SEGraph> out;
    for (auto &m : all) {
        std::sort(m.begin(), m.end());
        bool ok = true;
        for (int i = 0; i < 2 * n - 1 && ok; ++i) {
            bool sp = false;
            for (auto &c : m) if (c.first <= i && i < c.second) sp = true;
            ok = sp;
        }
        if (ok) out.push_back({n, m});
    }
    std::sort(out.begin(), out.end(), [](const SEGraph &x, const SEGraph &y) { return x.chords < y.chords; });
    return out;
}

std::array<int, 3> vertex_class(const SEGraph &g, int e) {
    int k = 0, l = 0, r = 0;
    for (auto &c : g.chords) {
        if (c.first <= e && e < c.second) ++k;
        else if (c.second <= e) ++l;
        else ++r;
    }
    return {k, std::max(l, r), std::min(l, r)};
}

namespace {

struct VG {
    int n, e, X, nv;
    std::vector<std::pair<int, int>> chords;  // vertex-graph numbering, S's order
    std::vector<int> chord_of;                 // vertex -> chord or -1
};

VG make_vg(const SEGraph &g, int e) {
    VG v;
    v.n = g.n; v.e = e; v.X = e + 1; v.nv = 2 * g.n + 1;
    auto mp = [&](int i) { return i <= e ? i : i + 1; };
    for (auto &c : g.chords) v.chords.push_back({mp(c.first), mp(c.second)});
    v.chord_of.assign(v.nv, -1);
    for (size_t i = 0; i < v.chords.size(); ++i) {
        v.chord_of[v.chords[i].first] = (int)i;
        v.chord_of[v.chords[i].second] = (int)i;
    }
    return v;
}

struct Sub { int a, b; bool se; };

inline bool in_iv(int x, int a, int b) { return a <= x && x <= b; }

std::vector<Sub> uv_subgraphs(const VG &g) {
    std::vector<Sub> out;
    for (int a = 0; a < g.nv; ++a)
        for (int b = a + 1; b < g.nv; ++b) {
            bool ok = true;
            for (int v = a; v < b && ok; ++v) {
                bool sp = false;
                for (auto &c : g.chords)
                    if (c.first >= a && c.second <= b && c.first <= v && v < c.second) sp = true;
                ok = sp;
            }
            if (!ok) continue;
            int cross = 0;
            for (auto &c : g.chords) if (in_iv(c.first, a, b) != in_iv(c.second, a, b)) ++cross;
            int ng = cross + (in_iv(g.X, a, b) ? 1 : 0);
            if (ng == 0) out.push_back({a, b, true});
            else if (ng == 1) out.push_back({a, b, false});
        }
    return out;
}

bool overlaps(const Sub &p, const Sub &q) {
    bool share = std::max(p.a, q.a) < std::min(p.b, q.b);
    bool cont = (p.a <= q.a && q.b <= p.b) || (q.a <= p.a && p.b <= q.b);
    return share && !cont;
}
bool strictly_contains(const Sub &big, const Sub &s) {
    return big.a <= s.a && s.b <= big.b && !(big.a == s.a && big.b == s.b);
}
bool in_I(const VG &g, const Sub &s) { return !s.se && in_iv(g.X, s.a, s.b); }

struct Term { int sign; std::vector<Sub> forest; std::vector<int> ops; };

std::vector<Term> build_terms(const VG &g, int *n_expanded) {
    auto subs = uv_subgraphs(g);
    Sub G{0, 2 * g.n, false};
    std::vector<Sub> others;
    for (auto &s : subs) if (!(s.a == G.a && s.b == G.b)) others.push_back(s);
    std::vector<std::vector<Sub>> forests;
    std::vector<Sub> chosen;
    std::function<void(size_t)> rec = [&](size_t i) {
        if (i == others.size()) {
            std::vector<Sub> f{G};
            f.insert(f.end(), chosen.begin(), chosen.end());
            forests.push_back(f);
            return;
        }
        rec(i + 1);
        bool ok = true;
        for (auto &t : chosen) if (overlaps(others[i], t)) { ok = false; break; }
        if (ok) { chosen.push_back(others[i]); rec(i + 1); chosen.pop_back(); }
    };
    rec(0);
    std::vector<Term> out;
    int nexp = 0;
    for (auto &F : forests) {
        int sign = ((F.size() - 1) % 2) ? -1 : 1;
        for (auto &Gp : F) {
            if (!in_I(g, Gp)) continue;
            Term t;
            t.sign = sign;
            t.forest = F;
            bool lu = false;
            for (auto &Gpp : F) {
                int op;
                if (Gpp.a == Gp.a && Gpp.b == Gp.b) op = OP_A;
                else if (!in_I(g, Gpp) || strictly_contains(Gp, Gpp)) op = OP_U;
                else if (!(Gpp.a == G.a && Gpp.b == G.b)) op = OP_L;
                else { op = OP_LU; lu = true; }
                if (Gpp.se) op = OP_SE;
                t.ops.push_back(op);
            }
            nexp += lu ? 2 : 1;
            out.push_back(t);
        }
    }
    if (n_expanded) *n_expanded = nexp;
    return out;
}

// A level: forest element with children contracted.
struct Node { int kind; int v; };   // kind 0 vertex, 1 X, 2 child (v = forest index)
struct LevelInfo {
    int fi;                 // forest index
    int op;
    bool se;
    std::vector<Node> nodes;
    std::vector<int> segs;  // vertex-graph segment (v|v+1) between node k-1 and k
    struct Ph { int i, j, chord; };
    std::vector<Ph> photons;
    int ext;                // node with the external photon (vertex levels)
    std::vector<int> kids;  // forest indices in node order
};

std::vector<LevelInfo> build_levels(const VG &g, const Term &t, std::vector<int> &parent) {
    const auto &F = t.forest;
    int nf = (int)F.size();
    parent.assign(nf, -1);
    for (int i = 0; i < nf; ++i) {
        int best = -1;
        for (int j = 0; j < nf; ++j)
            if (j != i && strictly_contains(F[j], F[i]))
                if (best < 0 || strictly_contains(F[best], F[j])) best = j;
        parent[i] = best;
    }
    std::vector<LevelInfo> lv(nf);
    for (int i = 0; i < nf; ++i) {
        LevelInfo &L = lv[i];
        L.fi = i; L.op = t.ops[i]; L.se = F[i].se;
        std::vector<int> owner(g.nv, -1);
        for (int j = 0; j < nf; ++j)
            if (parent[j] == i)
                for (int w = F[j].a; w <= F[j].b; ++w) owner[w] = j;
        int prev_end = -1;
        std::vector<int> node_of(g.nv, -1);
        for (int v = F[i].a; v <= F[i].b;) {
            Node nd;
            int last;
            if (owner[v] >= 0) { nd = {2, owner[v]}; last = F[owner[v]].b; L.kids.push_back(owner[v]); }
            else if (v == g.X) { nd = {1, v}; last = v; }
            else { nd = {0, v}; last = v; }
            if (prev_end >= 0) L.segs.push_back(prev_end);
            int k = (int)L.nodes.size();
            for (int w = v; w <= last; ++w) node_of[w] = k;
            L.nodes.push_back(nd);
            prev_end = last;
            v = last + 1;
        }
        for (size_t ci = 0; ci < g.chords.size(); ++ci) {
            auto c = g.chords[ci];
            if (in_iv(c.first, F[i].a, F[i].b) && in_iv(c.second, F[i].a, F[i].b)) {
                int a = node_of[c.first], b = node_of[c.second];
                if (a != b) L.photons.push_back({std::min(a, b), std::max(a, b), (int)ci});
            }
        }
        L.ext = -1;
        if (!F[i].se) {
            if (in_iv(g.X, F[i].a, F[i].b)) L.ext = node_of[g.X];
            else
                for (auto &c : g.chords)
                    if (in_iv(c.first, F[i].a, F[i].b) != in_iv(c.second, F[i].a, F[i].b))
                        L.ext = node_of[in_iv(c.first, F[i].a, F[i].b) ? c.first : c.second];
        }
    }
    return lv;
}

int line_param(const VG &g, int seg) {
    if (seg <= g.e) return seg;
    if (seg == g.e + 1) return g.e;
    return seg - 1;
}

// ---------------------------------------------------------------------------
// Symbolic Dirac traces.  Symbols: SYM_P = P-slash, SYM_Q = q-slash (before
// the q-pair average), labels >= SYM_LAB0 occur exactly twice (contracted).
// ---------------------------------------------------------------------------
constexpr int8_t SYM_P = 0, SYM_Q = 1, SYM_LAB0 = 2;
constexpr int8_t LAB_MU = SYM_LAB0 + 8;
constexpr int8_t LAB_KAP0 = SYM_LAB0 + 16;
constexpr int8_t LAB_QQ = SYM_LAB0 + 40;

using Str = std::basic_string<int8_t>;

struct TraceEngine {
    std::unordered_map<std::string, int64_t> memo;

    int64_t tr(const Str &s0) {
        // simplify adjacent P P and adjacent equal labels
        Str s;
        int64_t fac = 1;
        for (int8_t c : s0) {
            if (!s.empty() && s.back() == c && (c == SYM_P || c >= SYM_LAB0)) {
                s.pop_back();
                if (c != SYM_P) fac *= 4;
            } else {
                s.push_back(c);
            }
        }
        if (s.empty()) return 4 * fac;
        std::string key(reinterpret_cast<const char *>(s.data()), s.size());
        auto it = memo.find(key);
        if (it != memo.end()) return fac * it->second;
        int64_t val;
        // innermost contracted pair
        int bi = -1, bj = -1;
        for (size_t i = 0; i < s.size(); ++i) {
            if (s[i] < SYM_LAB0) continue;
            for (size_t j = i + 1; j < s.size(); ++j)
                if (s[j] == s[i]) {
                    if (bi < 0 || (int)(j - i) < bj - bi) { bi = (int)i; bj = (int)j; }
                    break;
                }
        }
        if (bi < 0) {
            int np = 0;
            for (int8_t c : s) {
                if (c != SYM_P) throw std::runtime_error("trace: unexpected symbol");
                ++np;
            }
            val = (np % 2) ? 0 : 4;
        } else {
            Str pre = s.substr(0, bi), S = s.substr(bi + 1, bj - bi - 1), suf = s.substr(bj + 1);
            size_t n = S.size();
            if (n == 0) {
                val = 4 * tr(pre + suf);
            } else if (n % 2 == 1) {
                Str r(S.rbegin(), S.rend());
                val = -2 * tr(pre + r + suf);
            } else {
                Str head = S.substr(0, n - 1);
                Str t1 = pre; t1.push_back(S[n - 1]); t1 += head; t1 += suf;
                Str rh(head.rbegin(), head.rend());
                Str t2 = pre + rh; t2.push_back(S[n - 1]); t2 += suf;
                val = 2 * tr(t1) + 2 * tr(t2);
            }
        }
        memo.emplace(key, val);
        return fac * val;
    }

    // Replace the two q symbols by (g - P P): returns label-pair trace minus P-P trace.
    int64_t tr_qq(const Str &s) {
        Str a = s, b = s;
        int cnt = 0;
        for (size_t i = 0; i < s.size(); ++i)
            if (s[i] == SYM_Q) { a[i] = LAB_QQ; b[i] = SYM_P; ++cnt; }
        if (cnt != 2) throw std::runtime_error("tr_qq: need exactly two q");
        return tr(a) - tr(b);
    }
};

TraceEngine &engine() {
    static thread_local TraceEngine e;
    return e;
}

// Chain items: type 0 gamma(label), 1 seg(k), 2 kv(k)
struct Item { int type; int val; };

std::vector<Item> level_chain(const VG &g, const LevelInfo &L, const std::vector<Sub> &F,
                              const std::vector<LevelInfo> &lv, unsigned variant) {
    std::vector<Item> items;
    std::vector<int> level_chords;
    for (auto &p : L.photons) level_chords.push_back(p.chord);
    int K = (int)L.nodes.size() - 1;
    // SE children in node order -> variant bit index
    int se_idx = 0;
    std::vector<int> se_bit(L.nodes.size(), -1);
    for (size_t k = 0; k < L.nodes.size(); ++k)
        if (L.nodes[k].kind == 2 && F[L.nodes[k].v].se) se_bit[k] = se_idx++;
    for (int k = K; k >= 0; --k) {
        const Node &nd = L.nodes[k];
        int chord = -2;   // -1 = external (X), >= 0 chord, -2 = SE child
        if (nd.kind == 0) chord = g.chord_of[nd.v];
        else if (nd.kind == 1) chord = -1;
        else {
            const Sub &c = F[nd.v];
            if (c.se) chord = -2;
            else if (in_iv(g.X, c.a, c.b)) chord = -1;
            else
                for (size_t ci = 0; ci < g.chords.size(); ++ci)
                    if (in_iv(g.chords[ci].first, c.a, c.b) != in_iv(g.chords[ci].second, c.a, c.b)) chord = (int)ci;
        }
        if (chord == -2) {
            if ((variant >> se_bit[k]) & 1u) items.push_back({2, k});
        } else if (chord >= 0 && std::find(level_chords.begin(), level_chords.end(), chord) != level_chords.end()) {
            items.push_back({0, SYM_LAB0 + chord});
        } else {
            items.push_back({0, LAB_MU});
        }
        if (k > 0) items.push_back({1, k});
    }
    (void)lv;
    return items;
}

// Monomial key: sorted pair list, sorted A list, C segment (-1 none)
struct MonoKey {
    std::vector<std::pair<int, int>> pairs;
    std::vector<int> A;
    int C;
    bool operator<(const MonoKey &o) const {
        if (pairs != o.pairs) return pairs < o.pairs;
        if (A != o.A) return A < o.A;
        return C < o.C;
    }
};

struct LevelPoly {
    int nout;
    double denom;
    std::vector<std::map<MonoKey, int64_t>> out;   // per output
};

void partial_matchings(const std::vector<int> &slots, size_t from, std::vector<std::pair<int, int>> &pairs,
                       std::vector<int> &un, std::vector<bool> &used,
                       const std::function<void()> &cb) {
    // find first unused slot >= from
    size_t i = from;
    while (i < slots.size() && used[i]) ++i;
    if (i == slots.size()) { cb(); return; }
    used[i] = true;
    un.push_back(slots[i]);
    partial_matchings(slots, i + 1, pairs, un, used, cb);
    un.pop_back();
    for (size_t j = i + 1; j < slots.size(); ++j) {
        if (used[j]) continue;
        used[j] = true;
        pairs.push_back({slots[i], slots[j]});
        partial_matchings(slots, i + 1, pairs, un, used, cb);
        pairs.pop_back();
        used[j] = false;
    }
    used[i] = false;
}

LevelPoly build_level_poly(const std::vector<Item> &items, int op) {
    TraceEngine &E = engine();
    LevelPoly P;
    P.nout = (op == OP_SE) ? 2 : 1;
    P.denom = (op == OP_SE) ? 4.0 : (op == OP_A ? 96.0 : 12.0);
    P.out.resize(P.nout);
    std::vector<int> kpos;
    for (size_t i = 0; i < items.size(); ++i) if (items[i].type != 0) kpos.push_back((int)i);
    std::vector<std::pair<int, int>> pairs;
    std::vector<int> un;
    std::vector<bool> used(kpos.size(), false);
    auto cb = [&]() {
        std::map<int, int8_t> lab;
        MonoKey base;
        for (size_t t = 0; t < pairs.size(); ++t) {
            lab[pairs[t].first] = (int8_t)(LAB_KAP0 + t);
            lab[pairs[t].second] = (int8_t)(LAB_KAP0 + t);
            int a = items[pairs[t].first].val, b = items[pairs[t].second].val;
            base.pairs.push_back({std::min(a, b), std::max(a, b)});
        }
        std::sort(base.pairs.begin(), base.pairs.end());
        int nun = (int)un.size();
        unsigned kvmask = 0;
        for (int t = 0; t < nun; ++t) if (items[un[t]].type == 2) kvmask |= 1u << t;
        std::vector<int> copts{-1};
        if (op == OP_A) for (int t = 0; t < nun; ++t) copts.push_back(t);
        for (unsigned am = 0; am < (1u << nun); ++am) {
            for (int cp : copts) {
                if (cp >= 0 && ((am >> cp) & 1u)) continue;
                unsigned chosen = am | (cp >= 0 ? 1u << cp : 0u);
                if (kvmask & ~chosen) continue;      // kslash has no mass term
                MonoKey key = base;
                for (int t = 0; t < nun; ++t) if ((am >> t) & 1u) key.A.push_back(items[un[t]].val);
                std::sort(key.A.begin(), key.A.end());
                key.C = cp >= 0 ? items[un[cp]].val : -1;
                // chain string (matrix order); 1 contributes nothing
                Str ch;
                for (size_t i = 0; i < items.size(); ++i) {
                    if (items[i].type == 0) { ch.push_back((int8_t)items[i].val); continue; }
                    auto l = lab.find((int)i);
                    if (l != lab.end()) { ch.push_back(l->second); continue; }
                    int t = (int)(std::find(un.begin(), un.end(), (int)i) - un.begin());
                    if (t == cp) ch.push_back(SYM_Q);
                    else if ((am >> t) & 1u) ch.push_back(SYM_P);
                }
                auto sub_mu = [&](const Str &s) { Str r = s; for (auto &c : r) if (c == LAB_MU) c = SYM_P; return r; };
                if (op == OP_SE) {
                    Str pn; pn.push_back(SYM_P); pn += ch;
                    P.out[0][key] += E.tr(ch);
                    P.out[1][key] += E.tr(pn);
                    continue;
                }
                if (op != OP_A) {
                    Str xs = ch; xs.push_back(LAB_MU);
                    int64_t X = E.tr(xs);
                    Str ys; ys.push_back(SYM_P); ys += sub_mu(ch);
                    int64_t Y = E.tr(ys);
                    int64_t Z = E.tr(sub_mu(ch));
                    int64_t v;
                    if (op == OP_U) v = X - Y;
                    else if (op == OP_L) v = 3 * Y + 3 * Z;
                    else v = 3 * Z + 4 * Y - X;
                    P.out[0][key] += v;
                    continue;
                }
                // AMM: 96 F2 = R1 - R2 + 2 R3 - 18 T_gamma
                // (P+1) factors expanded; [gamma^mu, q] = mu q - q mu
                int64_t acc = 0;
                auto with_p1 = [&](const Str &mid_left, const Str &mid_right,
                                   bool left_p1, bool right_p1, const std::function<int64_t(const Str &)> &f) {
                    int64_t s = 0;
                    for (int lp = 0; lp < (left_p1 ? 2 : 1); ++lp)
                        for (int rp = 0; rp < (right_p1 ? 2 : 1); ++rp) {
                            Str st;
                            if (left_p1 && lp) st.push_back(SYM_P);
                            st += mid_left;
                            if (right_p1 && rp) st.push_back(SYM_P);
                            st += mid_right;
                            s += f(st);
                        }
                    return s;
                };
                Str comm1, comm2;
                comm1.push_back(LAB_MU); comm1.push_back(SYM_Q);
                comm2.push_back(SYM_Q); comm2.push_back(LAB_MU);
                auto trq = [&](const Str &s) { return E.tr_qq(s); };
                auto trp = [&](const Str &s) { return E.tr(s); };
                if (cp < 0) {
                    // T_gamma = Tr[(P+1) N (P+1) gamma^mu]
                    Str mu; mu.push_back(LAB_MU);
                    int64_t tg = with_p1(ch, mu, true, true, trp);
                    // R1 = Tr[q N (P+1) [mu, q]]
                    Str qn; qn.push_back(SYM_Q); qn += ch;
                    int64_t r1 = 0, r2 = 0;
                    for (int p = 0; p < 2; ++p) {
                        Str s1 = qn; if (p) s1.push_back(SYM_P);
                        r1 += trq(s1 + comm1) - trq(s1 + comm2);
                    }
                    // R2 = Tr[(P+1) N q [mu, q]]
                    for (int p = 0; p < 2; ++p) {
                        Str s2; if (p) s2.push_back(SYM_P);
                        s2 += ch; s2.push_back(SYM_Q);
                        r2 += trq(s2 + comm1) - trq(s2 + comm2);
                    }
                    acc = r1 - r2 - 18 * tg;
                } else {
                    // R3 = Tr[(P+1) N1 (P+1) [mu, q]]
                    int64_t r3 = with_p1(ch, comm1, true, true, trq) - with_p1(ch, comm2, true, true, trq);
                    acc = 2 * r3;
                }
                P.out[0][key] += acc;
            }
        }
    };
    partial_matchings(kpos, 0, pairs, un, used, cb);
    return P;
}

std::string poly_key(const std::vector<Item> &items, int op) {
    std::string s = std::to_string(op) + ":";
    for (auto &it : items) s += std::to_string(it.type) + "," + std::to_string(it.val) + ";";
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Density tables (Sec. III.A readings: Deg1 = max(C_bigZ, min(C_bigF w(s), Deg_max)))
// ---------------------------------------------------------------------------
void set_stats(const SEGraph &g, uint32_t mask, int *loops_out, int *comps_out, int *ng_out, int *ne_out) {
    int n = g.n, M = 3 * n - 1;
    std::vector<int> par(2 * n);
    for (int i = 0; i < 2 * n; ++i) par[i] = i;
    std::function<int(int)> find = [&](int x) { while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; } return x; };
    std::vector<bool> touched(2 * n, false);
    int nl = 0, ng = 0;
    for (int i = 0; i < M; ++i) {
        if (!((mask >> i) & 1u)) continue;
        int u, v;
        if (i < 2 * n - 1) { u = i; v = i + 1; }
        else { u = g.chords[i - (2 * n - 1)].first; v = g.chords[i - (2 * n - 1)].second; ++ng; }
        touched[u] = touched[v] = true;
        ++nl;
    }
    int verts = 0;
    for (int i = 0; i < 2 * n; ++i) if (touched[i]) ++verts;
    int comps = verts;
    for (int i = 0; i < M; ++i) {
        if (!((mask >> i) & 1u)) continue;
        int u, v;
        if (i < 2 * n - 1) { u = i; v = i + 1; }
        else { u = g.chords[i - (2 * n - 1)].first; v = g.chords[i - (2 * n - 1)].second; }
        int ru = find(u), rv = find(v);
        if (ru != rv) { par[ru] = rv; --comps; }
    }
    if (loops_out) *loops_out = nl - verts + comps;
    if (comps_out) *comps_out = comps;
    if (ng_out) *ng_out = ng;
    if (ne_out) *ne_out = nl - ng;
}

double omega_set(const SEGraph &g, uint32_t mask) {
    int n = g.n, M = 3 * n - 1;
    int ne = 0, ng = 0;
    std::vector<int> par(2 * n);
    for (int i = 0; i < 2 * n; ++i) par[i] = i;
    std::function<int(int)> find = [&](int x) { while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; } return x; };
    std::vector<bool> touched(2 * n, false);
    int nl = 0;
    for (int i = 0; i < M; ++i) {
        if (!((mask >> i) & 1u)) continue;
        int u, v;
        if (i < 2 * n - 1) { u = i; v = i + 1; ++ne; }
        else { u = g.chords[i - (2 * n - 1)].first; v = g.chords[i - (2 * n - 1)].second; ++ng; }
        touched[u] = touched[v] = true;
        ++nl;
    }
    int verts = 0;
    for (int i = 0; i < 2 * n; ++i) if (touched[i]) ++verts;
    int comps = verts;
    for (int i = 0; i < M; ++i) {
        if (!((mask >> i) & 1u)) continue;
        int u, v;
        if (i < 2 * n - 1) { u = i; v = i + 1; }
        else { u = g.chords[i - (2 * n - 1)].first; v = g.chords[i - (2 * n - 1)].second; }
        int ru = find(u), rv = find(v);
        if (ru != rv) { par[ru] = rv; --comps; }
    }
    int loops = nl - verts + comps;
    return (double)ng + (double)ne / 2.0 - 2.0 * (double)loops;
}

void build_density(const SEGraph &g, const amm_density_params &p, DensityTables &d) {
    int M = 3 * g.n - 1;
    uint32_t full = (1u << M) - 1;
    d.M = M;
    d.deg1.assign(1u << M, 0.0);
    d.deg3.assign(1u << M, 0.0);
    d.W1.assign(1u << M, 0.0);
    d.logdeg1.assign(1u << M, 0.0);
    std::vector<double> F(1u << M, 0.0);
    for (uint32_t m = 1; m < full; ++m) {
        double w = p.cbigf * omega_set(g, m);
        if (p.degmax > 0.0) w = std::min(w, p.degmax);
        d.deg1[m] = std::max(p.cbigz, w);
        d.deg3[m] = p.d * d.deg1[m];
        d.logdeg1[m] = host_log(d.deg1[m]);
    }
    for (uint32_t m = 1; m <= full; ++m) {
        if ((m & (m - 1)) == 0) F[m] = 1.0;
        else {
            double acc = 0.0;
            for (int j = 0; j < M; ++j) if ((m >> j) & 1u) acc = acc + d.W1[m & ~(1u << j)];
            F[m] = acc;
        }
        if (m != full) d.W1[m] = F[m] / d.deg1[m];
    }
    d.F1full = F[full];
    d.F1 = F;
    double logF1 = host_log(F[full]);
    double logM = host_log((double)M);
    double fact = 1.0;
    for (int i = 2; i <= M; ++i) fact *= (double)i;
    double logMf = host_log(fact);
    double logD = host_log(p.d);
    d.logK[0] = -logF1;
    d.logK[1] = -logM;
    d.logK[2] = (double)(M - 1) * logD - logF1;
    d.logK[3] = -logMf;
    for (int c = 0; c < 4; ++c) {
        d.c[c] = p.c[c];
        d.logc[c] = p.c[c] > 0 ? host_log(p.c[c]) : -INFINITY;
    }
}

// ---------------------------------------------------------------------------
// Plan assembly
// ---------------------------------------------------------------------------
// The distinct level polynomials of a graph (chain and operator of every
// level variant of every term), built on `nthreads` threads: each distinct
// chain once, in parallel (each thread has its own trace memo).
static std::map<std::string, LevelPoly> build_graph_polys(const SEGraph &g, int nthreads) {
    const int n = g.n;
    std::vector<std::string> keys;
    std::vector<std::pair<std::vector<Item>, int>> jobs;
    std::map<std::string, int> seen;
    for (int e = 0; e < 2 * n - 1; ++e) {
        VG vg = make_vg(g, e);
        for (auto &t : build_terms(vg, nullptr)) {
            std::vector<int> parent;
            auto lv = build_levels(vg, t, parent);
            for (auto &L : lv) {
                int nse = 0;
                for (int kid : L.kids) if (t.forest[kid].se) ++nse;
                const int K = (int)L.nodes.size() - 1;
                for (int var = 0; var < (1 << nse); ++var) {
                    auto items = level_chain(vg, L, t.forest, lv, (unsigned)var);
                    std::string key = poly_key(items, L.op) + "K" + std::to_string(K);
                    if (seen.emplace(key, (int)keys.size()).second) {
                        keys.push_back(key);
                        jobs.push_back({items, L.op});
                    }
                }
            }
        }
    }
    std::vector<LevelPoly> polys(jobs.size());
    std::vector<std::string> errs(nthreads > 0 ? nthreads : 1);
    std::atomic<size_t> next(0);
    auto work = [&](int w) {
        try {
            for (size_t i = next++; i < jobs.size(); i = next++) polys[i] = build_level_poly(jobs[i].first, jobs[i].second);
        } catch (const std::exception &ex) {
            errs[w] = ex.what();
        }
    };
    const int nt = std::max(1, std::min<int>(nthreads, (int)jobs.size()));
    std::vector<std::thread> pool;
    for (int w = 1; w < nt; ++w) pool.emplace_back(work, w);
    work(0);
    for (auto &th : pool) th.join();
    for (auto &e : errs)
        if (!e.empty()) throw std::runtime_error(e);
    std::map<std::string, LevelPoly> out;
    for (size_t i = 0; i < keys.size(); ++i) out.emplace(keys[i], std::move(polys[i]));
    return out;
}

void build_plan(const SEGraph &g, PlanHost &P, int nthreads) {
    int n = g.n;
    P.n = n;
    P.M = 3 * n - 1;
    P.ninsert = 2 * n - 1;
    P.levels.clear(); P.terms.clear(); P.ops.clear(); P.monos.clear(); P.ranges.clear();
    P.n_terms_expanded = 0;
    P.n_monos_per_sample = 0;
    P.flops_per_sample = 0;
    const std::map<std::string, LevelPoly> built = build_graph_polys(g, nthreads);
    std::map<std::string, std::pair<int, int>> poly_cache_n;   // key -> (nvar-independent) (range base, count)
    for (int e = 0; e < 2 * n - 1; ++e) {
        VG vg = make_vg(g, e);
        int nexp = 0;
        auto terms = build_terms(vg, &nexp);
        P.n_terms_expanded += nexp;
        for (auto &t : terms) {
            std::vector<int> parent;
            auto lv = build_levels(vg, t, parent);
            if ((int)lv.size() > 2 * n + 1) throw std::runtime_error("forest deeper than the value stack");
            TermDesc td;
            td.e = e;
            td.sign = t.sign;
            td.op_begin = (int)P.ops.size();
            // post-order from the root
            int root = -1;
            for (size_t i = 0; i < lv.size(); ++i) if (parent[i] < 0) root = (int)i;
            std::function<void(int)> visit = [&](int i) {
                for (int kid : lv[i].kids) visit(kid);
                const LevelInfo &L = lv[i];
                LevelDesc d;
                std::memset(&d, 0, sizeof(d));
                int K = (int)L.nodes.size() - 1;
                // the kernels size their per-level arrays by the loop order n:
                // K <= 2n segments, L <= n photons
                if (K > MAXK || K > 2 * n || (int)L.photons.size() > n) throw std::runtime_error("level too large");
                d.K = K;
                d.L = (int)L.photons.size();
                d.op = L.op;
                d.ext_node = L.ext;
                d.has_X = 0;
                for (auto &nd : L.nodes) if (nd.kind == 1) d.has_X = 1;
                for (int k = 1; k <= K; ++k) {
                    int seg = L.segs[k - 1];
                    d.seg_param[k - 1] = line_param(vg, seg);
                    d.seg_half[k - 1] = (seg == vg.X - 1 || seg == vg.X) ? 1 : 0;
                }
                for (int a = 0; a < d.L; ++a) {
                    d.ph_param[a] = 2 * n - 1 + L.photons[a].chord;
                    uint32_t sp = 0;
                    for (int k = 1; k <= K; ++k)
                        if (L.photons[a].i <= k - 1 && k <= L.photons[a].j) sp |= 1u << (k - 1);
                    d.span[a] = sp;
                }
                int N = K + d.L;
                d.pref = std::ldexp(1.0, -2 * d.L) * ((N % 2) ? -1.0 : 1.0);
                d.nout = L.se ? 2 : 1;
                int nse = 0;
                d.nkids = (int)L.kids.size();
                d.kid_is_se = 0;
                for (size_t q = 0; q < L.kids.size(); ++q)
                    if (t.forest[L.kids[q]].se) { d.kid_is_se |= 1u << q; ++nse; }
                d.nvariants = 1 << nse;
                d.nvar = amm_xn(K) + 2 * K;
                d.mono_range = (int)P.ranges.size();
                // ranges: (variant*nout + out)*(n+1) + c  -> [begin, end)
                P.ranges.resize(P.ranges.size() + (size_t)d.nvariants * d.nout * (n + 1));
                for (int var = 0; var < d.nvariants; ++var) {
                    auto items = level_chain(vg, L, t.forest, lv, (unsigned)var);
                    std::string key = poly_key(items, L.op) + "K" + std::to_string(K);
                    auto it = poly_cache_n.find(key);
                    int base;
                    if (it == poly_cache_n.end()) {
                        const LevelPoly &lp = built.at(key);
                        base = (int)P.poly_ranges_store.size();
                        for (int o = 0; o < d.nout; ++o) {
                            for (int c = 0; c <= n; ++c) {
                                const int beg = (int)P.monos.size();
                                for (auto &kv : lp.out[o]) {
                                    if ((int)kv.first.pairs.size() != c || kv.second == 0) continue;
                                    Mono m;
                                    std::memset(&m, 0, sizeof(m));
                                    m.coef = (double)kv.second / lp.denom;
                                    int nv = 0;
                                    for (auto &pr : kv.first.pairs) m.v[nv++] = (uint8_t)amm_xidx(K, pr.first, pr.second);
                                    for (int a : kv.first.A) m.v[nv++] = (uint8_t)(amm_xn(K) + a - 1);
                                    if (kv.first.C >= 0) m.v[nv++] = (uint8_t)(amm_xn(K) + K + kv.first.C - 1);
                                    if (nv > MAXMONO_VARS) throw std::runtime_error("monomial too long");
                                    for (int q = 0; q < nv; ++q)
                                        if (m.v[q] >= amm_xn(K) + 2 * K) throw std::runtime_error("variable index out of range");
                                    m.nv = (uint8_t)nv;
                                    P.monos.push_back(m);
                                }
                                // degree-sorted ranges: the kernels read monomials of equal degree together
                                std::stable_sort(P.monos.begin() + beg, P.monos.end(),
                                                 [](const Mono &x, const Mono &y) { return x.nv > y.nv; });
                                P.poly_ranges_store.push_back({beg, (int)P.monos.size()});
                            }
                        }
                        poly_cache_n[key] = {base, d.nout * (n + 1)};
                    } else {
                        base = it->second.first;
                    }
                    for (int o = 0; o < d.nout; ++o)
                        for (int c = 0; c <= n; ++c)
                            P.ranges[d.mono_range + (var * d.nout + o) * (n + 1) + c] =
                                P.poly_ranges_store[base + o * (n + 1) + c];
                }
                // cost accounting
                for (int var = 0; var < d.nvariants; ++var)
                    for (int o = 0; o < d.nout; ++o)
                        for (int c = 0; c <= n; ++c) {
                            auto r = P.ranges[d.mono_range + (var * d.nout + o) * (n + 1) + c];
                            for (int m = r.first; m < r.second; ++m) {
                                P.n_monos_per_sample += 1;
                                P.flops_per_sample += P.monos[m].nv + 1.0;   // nv multiplies + 1 add
                            }
                        }
                int Lq = d.L;
                // LDL^T of L x L, solves for K+2 right-hand sides, Gram products
                P.flops_per_sample += (double)(Lq * Lq * Lq) / 3.0 * 2.0 + (K + 2) * Lq * Lq * 2.0 +
                                      amm_xn(K) * Lq * 2.0 + 6.0 * K;
                P.levels.push_back(d);
                P.ops.push_back((int)P.levels.size() - 1);
            };
            visit(root);
            td.op_end = (int)P.ops.size();
            P.terms.push_back(td);
            P.flops_per_sample += 4.0 * n;   // Gamma/V^k tail
        }
    }
}

}  // namespace amm
