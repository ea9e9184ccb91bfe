// amm_codegen.cpp -- emits straight-line HIP for the integrands of one loop
// order (build-time tool, part of the library build).
//
// For every SE graph the generated device function evaluates all insertion
// integrands at a point exactly as the table interpreter (amm_core.h
// eval_graph) does -- same levels, same operation order inside each level,
// same numerator polynomials -- but with every index, span and loop bound
// resolved at generation time, so all intermediate values live in
// registers.  Each forest term is its own non-inlined device function; a
// term's levels are evaluated inside it (identical subtrees of different
// terms are evaluated again, as in the interpreter).
//
// Usage: amm_codegen graph <loops> <g> <dir> | dispatch <out.hip> <loops>...
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "amm_host.h"

using namespace amm;

namespace {

std::string lit(double x) {
    char b[64];
    std::snprintf(b, sizeof b, "%a", x);
    return std::string("T(") + b + ")";
}

struct Emitter {
    std::ostringstream os;
    int tmp = 0;
    std::string fresh(const char *p) { return std::string(p) + std::to_string(tmp++); }
};

// Key of a level subtree within a plan: the op list of the subtree in post-order.
std::string subtree_key(const PlanHost &P, const std::vector<int> &ops, int end, int &begin_out) {
    // walk back from end-1 (the subtree root) consuming children recursively
    int pos = end - 1;
    std::function<void()> take = [&]() {
        const LevelDesc &d = P.levels[ops[pos]];
        --pos;
        for (int q = 0; q < d.nkids; ++q) take();
    };
    take();
    begin_out = pos + 1;
    std::ostringstream k;
    for (int i = begin_out; i < end; ++i) {
        const LevelDesc &d = P.levels[ops[i]];
        k << d.K << ',' << d.L << ',' << d.op << ',' << d.ext_node << ',' << d.has_X << ',' << d.nkids << ','
          << d.kid_is_se << ',' << d.nvariants << ',' << d.nout << ':';
        for (int q = 0; q < d.K; ++q) k << d.seg_param[q] << '/' << d.seg_half[q] << ' ';
        for (int a = 0; a < d.L; ++a) k << d.ph_param[a] << '/' << d.span[a] << ' ';
        // polynomial identity: mono ranges content
        for (int v = 0; v < d.nvariants; ++v)
            for (int o = 0; o < d.nout; ++o)
                for (int c = 0; c <= P.n; ++c) {
                    auto r = P.ranges[d.mono_range + (v * d.nout + o) * (P.n + 1) + c];
                    k << r.first << '-' << r.second << ' ';
                }
        k << '|';
    }
    return k.str();
}

struct SubVal {             // generated names of a subtree's value
    std::string vec[2];     // c-vector arrays (length N)
    std::string V;          // sum of V over the subtree's levels
};

class GraphGen {
  public:
    GraphGen(const PlanHost &P, int gi) : P(P), gi(gi), N(P.n) {}

    // One non-inlined device function per forest term (its level values, with
    // the few sub-levels it shares with other terms recomputed, live only
    // inside it), called in term order by Fun::eval.  Small functions keep the
    // register allocation per term and the compile time near linear in size.
    std::string run() {
        std::ostringstream funcs, body;
        int t = 0;
        for (const TermDesc &td : P.terms) {
            E.os.str("");
            E.os.clear();
            memo.clear();
            for (int j = 0; j < P.M; ++j) E.os << "  const double z" << j << " = z[" << j << "];\n";
            std::vector<int> ops(P.ops.begin() + td.op_begin, P.ops.begin() + td.op_end);
            SubVal root = subtree(ops, (int)ops.size());
            // sum_c vec[c] Gamma(n-c) / V^{n-c}
            std::string val = E.fresh("val");
            E.os << "  {\n    T vinv = T(1.0) / " << root.V << ";\n    T vp = vinv;\n    T " << val << " = T(0.0);\n";
            double gam = 1.0;
            for (int c = N - 1; c >= 0; --c) {
                char b[64];
                std::snprintf(b, sizeof b, "%a", gam);
                E.os << "    " << val << " = mul_add(" << root.vec[0] << "[" << c << "] * T(" << b << "), vp, " << val
                     << ");\n";
                if (c > 0) E.os << "    vp = vp * vinv;\n";
                gam = gam * (double)(N - c);
            }
            E.os << "    I[" << td.e << "] += " << (td.sign > 0 ? "" : "-") << val << ";\n";
            E.os << "    absI[" << td.e << "] += absd(" << val << ");\n  }\n";
            funcs << "template <typename T>\nstatic __device__ __attribute__((noinline)) void term" << t
                  << "(const double *z, T *I, T *absI) {\n" << E.os.str() << "}\n";
            body << "  term" << t << "<T>(z, I, absI);\n";
            ++t;
        }
        std::ostringstream out;
        out << funcs.str();
        out << "struct Fun {\ntemplate <typename T>\nstatic __device__ __forceinline__ void eval(const double *z, T *I, T *absI) {\n";
        for (int e = 0; e < P.ninsert; ++e) out << "  I[" << e << "] = T(0.0); absI[" << e << "] = T(0.0);\n";
        out << body.str() << "}\n};\n";
        return out.str();
    }

  private:
    const PlanHost &P;
    int gi, N;
    Emitter E;
    std::map<std::string, SubVal> memo;

    SubVal subtree(const std::vector<int> &ops, int end) {
        int begin;
        std::string key = subtree_key(P, ops, end, begin);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
        // children subtrees: walk forward over the kid slots of the root
        const LevelDesc &d = P.levels[ops[end - 1]];
        std::vector<SubVal> kids(d.nkids);
        int pos = end - 1;
        for (int q = d.nkids - 1; q >= 0; --q) {
            int b;
            subtree_key(P, ops, pos, b);
            kids[q] = subtree(ops, pos);
            pos = b;
        }
        SubVal out = level(d, kids);
        memo[key] = out;
        return out;
    }

    std::string zexpr(int param, int half) {
        std::string s = "z" + std::to_string(param);
        return half ? "T(" + s + " * 0.5)" : "T(" + s + ")";
    }

    SubVal level(const LevelDesc &d, const std::vector<SubVal> &kids) {
        const int K = d.K, L = d.L;
        std::string pf = E.fresh("l");
        auto nm = [&](const std::string &s) { return pf + "_" + s; };
        std::ostringstream &o = E.os;
        SubVal out;
        out.vec[0] = nm("r0");
        out.vec[1] = nm("r1");
        out.V = nm("V");
        o << "  T " << out.vec[0] << "[" << N << "], " << out.vec[1] << "[" << N << "], " << out.V << ";\n  {\n";
        for (int k = 1; k <= K; ++k) o << "    const T zs" << k << " = " << zexpr(d.seg_param[k - 1], d.seg_half[k - 1]) << ";\n";
        for (int a = 0; a < L; ++a) o << "    const T zp" << a << " = " << zexpr(d.ph_param[a], 0) << ";\n";
        // Lambda
        for (int a = 0; a < L; ++a)
            for (int b = 0; b < L; ++b) {
                o << "    T Lam" << a << "_" << b << " = ";
                std::string v = (a == b) ? "zp" + std::to_string(a) : "T(0.0)";
                uint32_t both = d.span[a] & d.span[b];
                for (int k = 1; k <= K; ++k)
                    if ((both >> (k - 1)) & 1u) v = "(" + v + " + zs" + std::to_string(k) + ")";
                o << v << ";\n";
            }
        // LDL^T
        o << "    T U = T(1.0);\n";
        for (int i = 0; i < L; ++i) {
            o << "    T D" << i << " = Lam" << i << "_" << i << ";\n";
            for (int j = 0; j < i; ++j) o << "    D" << i << " -= Lw" << i << "_" << j << " * Lw" << i << "_" << j << " * D" << j << ";\n";
            o << "    U *= D" << i << ";\n    T Di" << i << " = T(1.0) / D" << i << ";\n";
            for (int r = i + 1; r < L; ++r) {
                o << "    T Lw" << r << "_" << i << " = Lam" << r << "_" << i << ";\n";
                for (int j = 0; j < i; ++j)
                    o << "    Lw" << r << "_" << i << " -= Lw" << r << "_" << j << " * Lw" << i << "_" << j << " * D" << j << ";\n";
                o << "    Lw" << r << "_" << i << " = Lw" << r << "_" << i << " * Di" << i << ";\n";
            }
        }
        // y_k = L^{-1} s_k
        for (int k = 1; k <= K; ++k)
            for (int a = 0; a < L; ++a) {
                o << "    T y" << k << "_" << a << " = " << (((d.span[a] >> (k - 1)) & 1u) ? "T(1.0)" : "T(0.0)") << ";\n";
                for (int b = 0; b < a; ++b) o << "    y" << k << "_" << a << " -= Lw" << a << "_" << b << " * y" << k << "_" << b << ";\n";
            }
        // w, V
        o << "    T Vl = T(0.0);\n";
        for (int a = 0; a < L; ++a) {
            std::string sg = "T(0.0)";
            for (int k = 1; k <= K; ++k)
                if ((d.span[a] >> (k - 1)) & 1u) sg = "(" + sg + " + zs" + std::to_string(k) + ")";
            o << "    T w" << a << " = " << sg << ";\n";
            for (int b = 0; b < a; ++b) o << "    w" << a << " -= Lw" << a << "_" << b << " * w" << b << ";\n";
            o << "    Vl += w" << a << " * w" << a << " * Di" << a << ";\n";
        }
        // children V sums
        std::string Vsum = "strip(Vl)";
        for (auto &k : kids) Vsum += " + " + k.V;
        o << "    " << out.V << " = " << Vsum << ";\n    U = strip(U);\n";
        for (int a = 0; a < L; ++a) {
            o << "    w" << a << " = strip(w" << a << "); Di" << a << " = strip(Di" << a << ");\n";
            for (int k = 1; k <= K; ++k) o << "    y" << k << "_" << a << " = strip(y" << k << "_" << a << ");\n";
        }
        // which variables are used
        std::vector<bool> used(amm_xn(K) + 2 * K, false);
        for (int var = 0; var < d.nvariants; ++var)
            for (int oo = 0; oo < d.nout; ++oo)
                for (int c = 0; c < N; ++c) {
                    auto r = P.ranges[d.mono_range + (var * d.nout + oo) * (P.n + 1) + c];
                    for (int m = r.first; m < r.second; ++m)
                        for (int i = 0; i < P.monos[m].nv; ++i) used[P.monos[m].v[i]] = true;
                }
        const int XN = amm_xn(K);
        for (int k = 1; k <= K; ++k)
            for (int k2 = k; k2 <= K; ++k2) {
                int id = amm_xidx(K, k, k2);
                if (!used[id]) continue;
                o << "    const T v" << id << " = T(0.0)";
                for (int a = 0; a < L; ++a) o << " + y" << k << "_" << a << " * y" << k2 << "_" << a << " * Di" << a;
                o << ";\n";
            }
        for (int k = 1; k <= K; ++k) {
            int id = XN + k - 1;
            if (!used[id]) continue;
            o << "    const T v" << id << " = T(1.0) - (T(0.0)";
            for (int a = 0; a < L; ++a) o << " + y" << k << "_" << a << " * w" << a << " * Di" << a;
            o << ");\n";
        }
        if (d.op == OP_A) {
            for (int a = 0; a < L; ++a) {
                std::string jc = "T(0.0)";
                for (int k = 1; k <= K; ++k)
                    if ((d.span[a] >> (k - 1)) & 1u)
                        jc = "(" + jc + " + zs" + std::to_string(k) + " * T(" + (k <= d.ext_node ? "-0.5" : "0.5") + "))";
                o << "    T wc" << a << " = " << jc << ";\n";
                for (int b = 0; b < a; ++b) o << "    wc" << a << " -= Lw" << a << "_" << b << " * wc" << b << ";\n";
            }
            for (int a = 0; a < L; ++a) o << "    wc" << a << " = strip(wc" << a << ");\n";
            for (int k = 1; k <= K; ++k) {
                int id = XN + K + k - 1;
                if (!used[id]) continue;
                o << "    const T v" << id << " = T(" << (k <= d.ext_node ? "-0.5" : "0.5") << ") - (T(0.0)";
                for (int a = 0; a < L; ++a) o << " + y" << k << "_" << a << " * wc" << a << " * Di" << a;
                o << ");\n";
            }
        }
        // values of the used variables and their largest relative error (T = ea)
        o << "    double rmx = 0.0;\n";
        for (size_t id = 0; id < used.size(); ++id)
            if (used[id])
                o << "    const double x" << id << " = to_double(v" << id << "); rmx = fmax(rmx, relerr(v" << id
                  << "));\n";
        o << "    const double rm1 = rmx + 1.0;\n";
        // base prefactor
        char pb[64];
        std::snprintf(pb, sizeof pb, "%a", d.pref);
        o << "    T base = T(" << pb << ") / (U * U);\n";
        if (d.has_X)
            for (int k = 1; k <= K; ++k)
                if (d.seg_half[k - 1]) { o << "    base = base * (zs" << k << " + zs" << k << ");\n"; break; }
        // product of vertex children
        o << "    T pv[" << N << "] = {T(1.0)";
        for (int c = 1; c < N; ++c) o << ", T(0.0)";
        o << "};\n";
        for (int q = 0; q < d.nkids; ++q) {
            if ((d.kid_is_se >> q) & 1u) continue;
            o << "    { T t[" << N << "]; conv_into<T, " << N << ">(pv, " << kids[q].vec[0] << ", t); for (int c = 0; c < "
              << N << "; ++c) pv[c] = t[c]; }\n";
        }
        o << "    for (int c = 0; c < " << N << "; ++c) { " << out.vec[0] << "[c] = T(0.0); " << out.vec[1] << "[c] = T(0.0); }\n";
        for (int var = 0; var < d.nvariants; ++var) {
            o << "    {\n      T sev[" << N << "]; for (int c = 0; c < " << N << "; ++c) sev[c] = pv[c];\n";
            int bit = 0;
            for (int q = 0; q < d.nkids; ++q) {
                if (!((d.kid_is_se >> q) & 1u)) continue;
                int ch = (var >> bit) & 1;
                ++bit;
                o << "      { T t[" << N << "]; conv_into<T, " << N << ">(sev, " << kids[q].vec[ch] << ", t); for (int c = 0; c < "
                  << N << "; ++c) sev[c] = t[c]; }\n";
            }
            for (int oo = 0; oo < d.nout; ++oo) {
                o << "      {\n      T own[" << N << "];\n      T fac = base;\n";
                for (int c = 0; c < N; ++c) {
                    auto r = P.ranges[d.mono_range + (var * d.nout + oo) * (P.n + 1) + c];
                    // FP64 value and first-order error bound of the range (as the
                    // interpreter's ea path): p = coef x_1 ... x_nv has relative
                    // error at most nv (rmax + 1) + 1; each accumulation adds |av|
                    o << "      {\n        double av = 0.0, ae = 0.0;\n";
                    for (int m = r.first; m < r.second; ++m) {
                        const Mono &mo = P.monos[m];
                        char cb[64];
                        std::snprintf(cb, sizeof cb, "%a", mo.coef);
                        std::string pe = cb;
                        for (int i = 0; i < mo.nv; ++i) pe = pe + " * x" + std::to_string(mo.v[i]);
                        o << "        { const double p = " << pe << "; av = av + p; ae = fma(fabs(p), fma("
                          << (int)mo.nv << ".0, rm1, 1.0), ae) + fabs(av); }\n";
                    }
                    o << "        own[" << c << "] = ea(av, ae) * fac;\n";
                    if (c + 1 < N) o << "        fac = fac * T(-0.5);\n";
                    o << "      }\n";
                }
                o << "      { T t[" << N << "]; conv_into<T, " << N << ">(own, sev, t); for (int c = 0; c < " << N
                  << "; ++c) " << out.vec[oo] << "[c] += t[c]; }\n      }\n";
            }
            o << "    }\n";
        }
        o << "  }\n";
        return out;
    }
};

}  // namespace

// Usage:  amm_codegen graph <loops> <g> <out_dir>   -> gen_<loops>_<g>.h/.hip
//         amm_codegen dispatch <out.hip> <loops>...    -> gen_launch table
int main(int argc, char **argv) {
    if (argc >= 5 && std::strcmp(argv[1], "graph") == 0) {
        int n = std::atoi(argv[2]), g = std::atoi(argv[3]);
        std::string dir = argv[4];
        auto graphs = enumerate_se(n);
        if (g < 0 || g >= (int)graphs.size()) return 2;
        PlanHost P;
        build_plan(graphs[g], P);
        GraphGen G(P, g);
        std::string tag = std::to_string(n) + "_" + std::to_string(g);
        std::ostringstream h;
        h << "// Generated by amm_codegen: integrands of " << n << "-loop SE graph " << g << ".  Do not edit.\n"
          << "#pragma once\n#include \"amm_core.h\"\nnamespace amm {\nnamespace gen_" << tag << " {\n"
          << G.run() << "}  // namespace gen_" << tag << "\n}  // namespace amm\n";
        std::ostringstream u;
        u << "// Generated by amm_codegen.  Do not edit.\n#include \"amm_gen.h\"\n#include \"gen_" << tag << ".h\"\n"
          << "namespace amm {\nvoid gen_launch_" << tag << "(int kind, const DensityDev *D, const RunArgs *A, int grid, "
          << "const double *z, uint64_t n, double *I, double *absI, double *bound, hipStream_t s, "
          << "double *part, uint32_t *flag, int32_t *nflag) {\n"
          << "  GenEval<gen_" << tag << "::Fun> EV;\n"
          << "  if (kind == GEN_RUN) launch_fp64_ev<" << n << ">(EV, *D, *A, grid, part, flag, nflag, s);\n"
          << "  else launch_eval_ev<" << n << ", GenEval<gen_" << tag << "::Fun>, ea>(EV, z, n, I, absI, bound, s);\n"
          << "}\n}  // namespace amm\n";
        for (auto &pr : {std::make_pair(std::string(".h"), h.str()), std::make_pair(std::string(".hip"), u.str())}) {
            FILE *f = std::fopen((dir + "/gen_" + tag + pr.first).c_str(), "w");
            if (!f) return 1;
            std::fwrite(pr.second.data(), 1, pr.second.size(), f);
            std::fclose(f);
        }
        return 0;
    }
    if (argc >= 3 && std::strcmp(argv[1], "dispatch") == 0) {
        std::ostringstream d;
        d << "// Generated by amm_codegen.  Do not edit.\n#include \"amm_gen.h\"\nnamespace amm {\n";
        std::vector<std::pair<int, int>> all;
        for (int i = 3; i < argc; ++i) {
            int n = std::atoi(argv[i]);
            int ng = (int)enumerate_se(n).size();
            for (int g = 0; g < ng; ++g) {
                all.push_back({n, g});
                d << "void gen_launch_" << n << "_" << g << "(int, const DensityDev *, const RunArgs *, int, "
                  << "const double *, uint64_t, double *, double *, double *, hipStream_t, double *, uint32_t *, "
                  << "int32_t *);\n";
            }
        }
        d << "GenLaunchFn gen_launch(int loops, int g) {\n";
        for (auto &pr : all)
            d << "  if (loops == " << pr.first << " && g == " << pr.second << ") return gen_launch_" << pr.first << "_"
              << pr.second << ";\n";
        d << "  return nullptr;\n}\n}  // namespace amm\n";
        FILE *f = std::fopen(argv[2], "w");
        if (!f) return 1;
        std::string s2 = d.str();
        std::fwrite(s2.data(), 1, s2.size(), f);
        std::fclose(f);
        return 0;
    }
    std::fprintf(stderr, "usage: %s graph <loops> <g> <dir> | dispatch <out.hip> <loops>...\n", argv[0]);
    return 2;
}
