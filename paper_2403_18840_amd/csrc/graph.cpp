// Diagram front end and graph compiler.
//
// Front end (eq. sigma_integration, eq. ueg_action): the n-th order self-energy diagrams are
// permutations sigma of 2n vertices (interaction line i joins vertices 2i and 2i+1; the
// propagator leaving v enters sigma[v]; the external legs enter vertex 0 and leave the vertex
// o with sigma[o] == 0).  Canonical forms are produced directly by an orderly generation: the
// vertices are visited in label order and the propagator leaving the visited vertex either
// enters an already-labelled vertex or opens the next interaction line, whose ends take the
// next two labels.  Each connected diagram is produced exactly once, in the labelling in which
// a breadth-first walk from the in-vertex discovers the vertices in label order.  Diagrams with
// a bridge are dropped: an interaction-line bridge forces q = 0 (a Hartree tadpole, removed by
// q != 0), a propagator bridge makes the self-energy one-particle reducible.
//
// Routing: propagators in order of their source vertex become chords (loop momenta q_0, q_1,
// ...) whenever removing them keeps the internal graph connected; the spanning tree left over
// carries the loop momenta back along tree paths and the external k from vertex 0 to the
// out-vertex.
//
// IR and back end (Sec. V.A): leaves are deduplicated (a propagator depends on |p|^2 and the
// ordered pair of interaction lines at its ends; an interaction depends on |p|^2), and every
// root (one per out-vertex time line and lambda group) is the sum of products over its
// diagrams.  That sum is factored greedily (repeatedly pulling out the factor common to most
// terms, external-momentum-dependent factors first), with structural hashing of every product
// and sum, so that the part of the graph that does not depend on k is computed once per sample
// outside the loop over external momenta.
#include "graph.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <set>
#include <sstream>

namespace dmc {

namespace {

struct Edge {
    char kind;
    int a, b;
};

bool connected(int nv, const std::vector<Edge>& es, int skip) {
    std::vector<std::vector<int>> adj(nv);
    for (int i = 0; i < (int)es.size(); ++i) {
        if (i == skip) continue;
        adj[es[i].a].push_back(es[i].b);
        adj[es[i].b].push_back(es[i].a);
    }
    std::vector<char> seen(nv, 0);
    std::vector<int> st{0};
    seen[0] = 1;
    int cnt = 1;
    while (!st.empty()) {
        int v = st.back();
        st.pop_back();
        for (int w : adj[v])
            if (!seen[w]) {
                seen[w] = 1;
                ++cnt;
                st.push_back(w);
            }
    }
    return cnt == nv;
}

std::vector<Edge> internal_edges(const std::vector<int>& sigma, int& n_fermion) {
    const int nv = (int)sigma.size();
    std::vector<Edge> es;
    for (int v = 0; v < nv; ++v)
        if (sigma[v] != 0) es.push_back({'G', v, sigma[v]});
    n_fermion = (int)es.size();
    for (int i = 0; i < nv / 2; ++i) es.push_back({'V', 2 * i, 2 * i + 1});
    return es;
}

bool bridgeless(const std::vector<int>& sigma) {
    int nf;
    auto es = internal_edges(sigma, nf);
    for (int i = 0; i < (int)es.size(); ++i)
        if (!connected((int)sigma.size(), es, i)) return false;
    return true;
}

int count_cycles(const std::vector<int>& sigma) {
    std::vector<char> seen(sigma.size(), 0);
    int c = 0;
    for (size_t s = 0; s < sigma.size(); ++s) {
        if (seen[s]) continue;
        ++c;
        for (int v = (int)s; !seen[v]; v = sigma[v]) seen[v] = 1;
    }
    return c;
}

// The external momentum's path: a simple path from the in-vertex 0 to the out-vertex with the fewest
// propagators, then the fewest lines, then the smallest sequence of line indices.  Returned as line
// indices in path order with the traversal sign (+1 along the line's reference direction).
std::vector<std::pair<int, int>> k_path(int nv, const std::vector<Edge>& es, int out) {
    std::vector<std::vector<std::pair<int, int>>> adj(nv);  // (line, +-1)
    for (int i = 0; i < (int)es.size(); ++i) {
        adj[es[i].a].push_back({i, +1});
        adj[es[i].b].push_back({i, -1});
    }
    for (auto& a : adj) std::sort(a.begin(), a.end());
    std::vector<std::pair<int, int>> best, cur;
    int best_g = 1 << 30;
    std::vector<char> onv(nv, 0);
    std::function<void(int, int)> dfs = [&](int v, int g) {
        if (v == out) {
            bool take = best.empty() || g < best_g || (g == best_g && cur.size() < best.size());
            if (!take && g == best_g && cur.size() == best.size())
                for (size_t i = 0; i < cur.size(); ++i)
                    if (cur[i].first != best[i].first) {
                        take = cur[i].first < best[i].first;
                        break;
                    }
            if (take) {
                best = cur;
                best_g = g;
            }
            return;
        }
        // no extension of a path that already has more propagators, or as many and at least as many lines
        if (!best.empty() && (g > best_g || (g == best_g && cur.size() >= best.size()))) return;
        for (auto [e, sg] : adj[v]) {
            const int w = sg > 0 ? es[e].b : es[e].a;
            if (onv[w]) continue;
            onv[w] = 1;
            cur.push_back({e, sg});
            dfs(w, g + (es[e].kind == 'G'));
            cur.pop_back();
            onv[w] = 0;
        }
    };
    onv[0] = 1;
    dfs(0, 0);
    return best;
}

Diagram route(const std::vector<int>& sigma) {
    const int nv = (int)sigma.size(), n = nv / 2;
    Diagram d;
    d.sigma = sigma;
    d.order = n;
    for (int v = 0; v < nv; ++v)
        if (sigma[v] == 0) d.out_vertex = v;
    d.n_fermion_loops = count_cycles(sigma) - 1;
    d.weight = ((n + d.n_fermion_loops) % 2 ? -1.0 : 1.0) * std::ldexp(1.0, d.n_fermion_loops);

    int nf;
    std::vector<Edge> es = internal_edges(sigma, nf);
    std::vector<char> in_tree(es.size(), 1);
    std::vector<int> chord_of(es.size(), -1), chord_sgn(es.size(), 1);
    int n_ch = 0;
    // chords by reverse delete: the external momentum's path first (in path order), then the other lines
    // in order; a line becomes a chord when the lines left still connect every vertex
    const auto kp = k_path(nv, es, d.out_vertex);
    std::vector<int> order_, path_sgn(es.size(), 0);
    for (auto [e, sg] : kp) {
        order_.push_back(e);
        path_sgn[e] = sg;
    }
    for (int i = 0; i < (int)es.size(); ++i)
        if (!path_sgn[i]) order_.push_back(i);
    for (int i : order_) {
        if (n_ch == n) break;
        std::vector<Edge> rest;
        for (int j = 0; j < (int)es.size(); ++j)
            if (in_tree[j] && j != i) rest.push_back(es[j]);
        if (connected(nv, rest, -1)) {
            in_tree[i] = 0;
            chord_of[i] = n_ch++;
            if (path_sgn[i]) chord_sgn[i] = path_sgn[i];
        }
    }
    // tree adjacency
    std::vector<std::vector<std::pair<int, int>>> adj(nv);  // (neighbour, edge index)
    for (int j = 0; j < (int)es.size(); ++j)
        if (in_tree[j]) {
            adj[es[j].a].push_back({es[j].b, j});
            adj[es[j].b].push_back({es[j].a, j});
        }
    std::vector<std::array<int, kMaxOrder + 1>> mom(es.size());
    for (auto& m : mom) m.fill(0);
    // add one unit of momentum component `comp` along the tree path from a to b
    auto flow = [&](int a, int b, int comp) {
        std::vector<int> prev_v(nv, -2), prev_e(nv, -1);
        std::vector<int> st{a};
        prev_v[a] = -1;
        while (!st.empty()) {
            int v = st.back();
            st.pop_back();
            for (auto [w, j] : adj[v])
                if (prev_v[w] == -2) {
                    prev_v[w] = v;
                    prev_e[w] = j;
                    st.push_back(w);
                }
        }
        for (int v = b; v != a; v = prev_v[v]) {
            int j = prev_e[v], u = prev_v[v];
            mom[j][comp] += (es[j].a == u && es[j].b == v) ? 1 : -1;
        }
    };
    for (int i = 0; i < (int)es.size(); ++i)
        if (chord_of[i] >= 0) {
            // a chord carries its loop momentum along the external path's direction (chords on that
            // path) or its reference direction, and the tree carries it back
            const int sg = chord_sgn[i];
            mom[i][chord_of[i]] = sg;
            if (sg > 0)
                flow(es[i].b, es[i].a, chord_of[i]);
            else
                flow(es[i].a, es[i].b, chord_of[i]);
        }
    for (auto [e, sg] : kp) mom[e][n] += sg;  // the external momentum along its path
    for (int i = 0; i < (int)es.size(); ++i) {
        Line ln;
        ln.kind = es[i].kind;
        ln.src = es[i].a;
        ln.dst = es[i].b;
        ln.mom.fill(0);
        for (int c = 0; c <= n; ++c) ln.mom[c] = mom[i][c];
        d.lines.push_back(ln);
    }
    return d;
}

void generate(int n, int j, int labelled, std::vector<int>& sigma, std::vector<char>& used,
              std::vector<Diagram>& out) {
    const int nv = 2 * n;
    if (j == nv) {
        if (labelled == nv && bridgeless(sigma)) out.push_back(route(sigma));
        return;
    }
    if (j >= labelled) return;  // the walk closed before reaching every line: disconnected
    for (int w = 0; w < labelled; ++w) {
        if (used[w]) continue;
        used[w] = 1;
        sigma[j] = w;
        generate(n, j + 1, labelled, sigma, used, out);
        used[w] = 0;
    }
    if (labelled < nv) {
        const int w = labelled;  // opens a new interaction line (labels w, w + 1)
        used[w] = 1;
        sigma[j] = w;
        generate(n, j + 1, labelled + 2, sigma, used, out);
        used[w] = 0;
    }
}

}  // namespace

std::vector<Diagram> enumerate_sigma(int n) {
    std::vector<Diagram> out;
    std::vector<int> sigma(2 * n, -1);
    std::vector<char> used(2 * n, 0);
    generate(n, 0, 2, sigma, used, out);
    return out;
}

// ----------------------------------------------------------------------------------------
// Code emission
// ----------------------------------------------------------------------------------------
namespace {

using Mom = std::array<int, kMaxOrder + 1>;

Mom normalise(Mom m, int n) {
    // p and -p give the same |p|^2: make the first nonzero coefficient positive
    for (int c = 0; c <= n; ++c) {
        if (m[c] > 0) break;
        if (m[c] < 0) {
            for (int e = 0; e <= n; ++e) m[e] = -m[e];
            break;
        }
    }
    return m;
}

std::string fstr(double v) {
    std::ostringstream s;
    s.precision(9);
    s << std::scientific << v << "f";
    return s.str();
}

// The coefficients a value of the generated code carries: entry 0 is the value, entry j > 0 the
// coefficient of dmu^m dlambda^l dk^e with (m, l, e) = idx[j].  The set is downward closed, so the
// product of two series keeps, for each of its entries, every pair of factor entries whose
// multi-indices add up to it.  First-order mode holds the value and one tangent per masked
// direction; Taylor mode (eq. taylor_node) holds every coefficient with m + l <= T and, with the k
// direction, their k tangents.  Coefficients are normalised (Taylor coefficients, not derivatives).
struct CoefSet {
    std::vector<std::array<int, 3>> idx;
    std::vector<std::vector<std::pair<int, int>>> conv;  // (a, b) with idx[a] + idx[b] = idx[j], a ascending
    int max_m = 0, max_l = 0;

    int find(int m, int l, int e) const {
        for (size_t j = 0; j < idx.size(); ++j)
            if (idx[j][0] == m && idx[j][1] == l && idx[j][2] == e) return (int)j;
        return -1;
    }
    void finish() {
        conv.assign(idx.size(), {});
        for (size_t j = 0; j < idx.size(); ++j) {
            max_m = std::max(max_m, idx[j][0]);
            max_l = std::max(max_l, idx[j][1]);
            for (size_t a = 0; a < idx.size(); ++a) {
                const int m = idx[j][0] - idx[a][0], l = idx[j][1] - idx[a][1], e = idx[j][2] - idx[a][2];
                if (m < 0 || l < 0 || e < 0) continue;
                const int b = find(m, l, e);
                if (b >= 0) conv[j].push_back({(int)a, b});
            }
        }
    }
    static CoefSet first_order(uint32_t mask) {
        CoefSet s;
        s.idx.push_back({0, 0, 0});
        for (int i = 0; i < 3; ++i)
            if (mask & (1u << i)) s.idx.push_back({i == 0, i == 1, i == 2});
        s.finish();
        return s;
    }
    static CoefSet taylor(uint32_t mask, int T) {
        CoefSet s;
        for (int e = 0; e <= ((mask & 4u) ? 1 : 0); ++e)
            for (int d = 0; d <= T; ++d)
                for (int m = d; m >= 0; --m) {
                    const int l = d - m;
                    if ((m && !(mask & 1u)) || (l && !(mask & 2u))) continue;
                    s.idx.push_back({m, l, e});
                }
        s.finish();
        return s;
    }
};

// A value of the generated code and its coefficients 1.. of the set (d[j - 1]); an empty name means
// structurally zero.
struct Val {
    std::string name;
    bool kdep;
    std::vector<std::string> d{};
};

class Emitter {
   public:
    std::ostringstream pre, loop, loopd;
    int64_t cnt_pre[4] = {0, 0, 0, 0}, cnt_loop[4] = {0, 0, 0, 0}, cnt_loopd[4] = {0, 0, 0, 0};  // add mul fma trans
    // With split_deriv, k-dependent code that forms a coefficient entry j > 0 (a derivative root's
    // value) goes to loopd, which the kernel runs only at the momenta that carry derivative roots;
    // dlevel > 0 while such code is emitted.  Cached helpers that value code may share are created with
    // dlevel 0 (ValueScope).
    bool split_deriv = false;
    int dlevel = 0;
    struct DerivScope {
        Emitter& e;
        explicit DerivScope(Emitter& em) : e(em) { ++e.dlevel; }
        ~DerivScope() { --e.dlevel; }
    };
    struct ValueScope {
        Emitter& e;
        int saved;
        explicit ValueScope(Emitter& em) : e(em), saved(em.dlevel) { e.dlevel = 0; }
        ~ValueScope() { e.dlevel = saved; }
    };
    bool to_d(bool kdep) const { return kdep && split_deriv && dlevel > 0; }
    int64_t* cnt(bool kdep) { return to_d(kdep) ? cnt_loopd : kdep ? cnt_loop : cnt_pre; }
    bool act[3] = {false, false, false};  // directions with a first-order entry (mu, lambda, k)
    const CoefSet* cs = nullptr;

    std::string prefix = "v";  // name prefix (distinct per part of a partitioned kernel)
    std::string tag;           // prefix of the few names not made by def (empty for one part)

    void set_coefs(const CoefSet* s) {
        cs = s;
        act[0] = s->find(1, 0, 0) > 0;
        act[1] = s->find(0, 1, 0) > 0;
        act[2] = s->find(0, 0, 1) > 0;
    }
    int nco() const { return (int)cs->idx.size(); }
    static const std::string& cf(const Val& v, int j) { return j == 0 ? v.name : v.d[j - 1]; }
    // the entry of direction i's first-order coefficient (mu 0, lambda 1, k 2), or -1
    int dir(int i) const { return cs->find(i == 0, i == 1, i == 2); }

    Val def(bool kdep, const std::string& expr, int opclass, int nops = 1) {
        std::string nm = prefix + std::to_string(tmp_++);
        (to_d(kdep) ? loopd : kdep ? loop : pre) << "    const float " << nm << " = " << expr << ";\n";
        if (opclass >= 0) cnt(kdep)[opclass] += nops;
        return {nm, kdep, std::vector<std::string>(nco() - 1)};
    }
    Val hashed(const std::string& key, bool kdep, const std::string& expr, int opclass,
               const std::function<void(Val&)>& tangents) {
        auto it = cse_.find(key);
        if (it != cse_.end()) return it->second;
        Val v = def(kdep, expr, opclass);
        {
            DerivScope ds(*this);
            tangents(v);
        }
        cse_[key] = v;
        return v;
    }
    Val mul(const Val& a, const Val& b) {
        const Val& x = a.name < b.name ? a : b;
        const Val& y = a.name < b.name ? b : a;
        const bool kd = a.kdep || b.kdep;
        return hashed("*" + x.name + "," + y.name, kd, x.name + " * " + y.name, 1, [&](Val& v) {
            for (int j = 1; j < nco(); ++j) {
                std::string acc;
                int t = 0;
                for (auto [ia, ib] : cs->conv[j]) {
                    const std::string &xa = cf(x, ia), &yb = cf(y, ib);
                    if (xa.empty() || yb.empty()) continue;
                    acc = acc.empty() ? xa + " * " + yb : "__builtin_fmaf(" + xa + ", " + yb + ", " + acc + ")";
                    ++t;
                }
                if (t == 0) continue;
                if (t == 1) {
                    v.d[j - 1] = def(kd, acc, 1).name;
                } else {
                    v.d[j - 1] = def(kd, acc, 2, t - 1).name;
                    cnt(kd)[1] += 1;
                }
            }
        });
    }
    Val fma(const Val& a, const Val& b, const Val& c) {
        const Val& x = a.name < b.name ? a : b;
        const Val& y = a.name < b.name ? b : a;
        const bool kd = a.kdep || b.kdep || c.kdep;
        return hashed("f" + x.name + "," + y.name + "," + c.name, kd,
                      "__builtin_fmaf(" + x.name + ", " + y.name + ", " + c.name + ")", 2, [&](Val& v) {
                          for (int j = 1; j < nco(); ++j) {
                              std::string acc = cf(c, j);
                              int nf = 0;
                              for (auto [ia, ib] : cs->conv[j]) {
                                  const std::string &xa = cf(x, ia), &yb = cf(y, ib);
                                  if (xa.empty() || yb.empty()) continue;
                                  acc = acc.empty() ? xa + " * " + yb
                                                    : "__builtin_fmaf(" + xa + ", " + yb + ", " + acc + ")";
                                  ++nf;
                              }
                              if (acc.empty()) continue;
                              if (nf == 0) {
                                  v.d[j - 1] = acc;  // only the addend carries this coefficient
                              } else {
                                  v.d[j - 1] = def(kd, acc, 2, nf).name;
                              }
                          }
                      });
    }
    Val add(const Val& a, const Val& b) {
        const Val& x = a.name < b.name ? a : b;
        const Val& y = a.name < b.name ? b : a;
        const bool kd = a.kdep || b.kdep;
        return hashed("+" + x.name + "," + y.name, kd, x.name + " + " + y.name, 0, [&](Val& v) {
            for (int j = 1; j < nco(); ++j) {
                const std::string &xj = cf(x, j), &yj = cf(y, j);
                if (xj.empty())
                    v.d[j - 1] = yj;
                else if (yj.empty())
                    v.d[j - 1] = xj;
                else
                    v.d[j - 1] = def(kd, xj + " + " + yj, 0).name;
            }
        });
    }
    Val scale(const Val& a, double c) {
        if (c == 1.0) return a;
        std::ostringstream k;
        k << "c" << c << "*" << a.name;
        return hashed(k.str(), a.kdep, fstr(c) + " * " + a.name, c == -1.0 ? -1 : 1, [&](Val& v) {
            for (int j = 1; j < nco(); ++j)
                if (!cf(a, j).empty()) v.d[j - 1] = def(a.kdep, fstr(c) + " * " + cf(a, j), c == -1.0 ? -1 : 1).name;
        });
    }
    Val constant(double c) { return {fstr(c), false, std::vector<std::string>(nco() - 1)}; }

   private:
    int tmp_ = 0;
    std::map<std::string, Val> cse_;
};

struct Term {
    double coef;
    std::vector<int> f;  // factor ids into the `vals` table, sorted
};

struct Builder {
    const Compiled& c;
    int n, n_groups;
    Emitter em;
    std::vector<Val> vals;      // factor values
    std::vector<char> val_k;    // k-dependence of each factor
    std::vector<int> val_sgn;   // a k-dependent propagator's sign factor (+-1, hoisted), or -1
    std::vector<char> is_sgn;   // the factor is a propagator sign
    std::map<std::pair<int, int>, int> sgn_id_;  // time pair -> sign factor
    // momentum, time-pair, energy caches
    std::map<Mom, int> mom_id;
    std::vector<Mom> moms;
    std::map<int, std::array<std::string, 3>> mom_q;   // Qx Qy Qz
    std::map<int, Val> mom_q2, mom_p2;
    std::map<std::pair<int, int>, std::pair<std::string, std::string>> tpair;  // T2, pos
    std::map<std::pair<int, int>, std::string> tcomp;                            // beta - tau' (log2 units)
    // per momentum: |eps| = ||p|^2 - mu|, eps >= 0, em = 2^(-beta |eps| log2 e), r = 1 / (1 + em);
    // nF = em r (eps >= 0) or r (eps < 0), 1 - nF the other one
    struct Energy {
        std::string ae, pos, em, r;
        bool k;
    };
    std::map<int, Energy> energy;
    std::map<std::tuple<int, int, int>, int> gleaf;  // (mom, a, b) -> factor id
    std::map<std::pair<int, int>, int> vleaf;        // (mom, group) -> factor id
    int n_g = 0, n_v = 0;

    std::map<int, std::string> mom_t;     // Qz + ck k of k-dependent momenta
    std::map<int, Val> mom_qxy2;          // Qx^2 + Qy^2 of k-dependent momenta
    std::map<int, std::string> mom_dp2;   // d|p|^2/dk of k-dependent momenta
    std::map<int, std::string> mom_bnf;   // beta nF(eps) per momentum
    CoefSet coefs;

    Builder(const Compiled& cc, int ng) : c(cc), n(cc.order), n_groups(ng) {
        coefs = cc.taylor_order > 0 ? CoefSet::taylor(cc.deriv_mask, cc.taylor_order) : CoefSet::first_order(cc.deriv_mask);
        em.set_coefs(&coefs);
    }

    bool is_k(int m) const { return moms[m][n] != 0; }

    int momentum(const Mom& raw) {
        Mom m = normalise(raw, n);
        auto it = mom_id.find(m);
        if (it != mom_id.end()) return it->second;
        int id = (int)moms.size();
        moms.push_back(m);
        mom_id[m] = id;
        return id;
    }

    std::array<std::string, 3> Q(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_q.find(m);
        if (it != mom_q.end()) return it->second;
        std::array<std::string, 3> r;
        const char* ax = "xyz";
        for (int a = 0; a < 3; ++a) {
            std::string e;
            int nterms = 0;
            for (int j = 0; j < n; ++j) {
                int cf = moms[m][j];
                if (!cf) continue;
                std::string t = em.tag + "q" + std::to_string(j) + ax[a];
                if (nterms == 0)
                    e = (cf == 1 ? "" : cf == -1 ? "-" : std::to_string(cf) + ".0f * ") + t;
                else
                    e += (cf > 0 ? " + " : " - ") + (std::abs(cf) == 1 ? "" : std::to_string(std::abs(cf)) + ".0f * ") + t;
                ++nterms;
            }
            if (nterms == 0) e = "0.0f";
            if (nterms <= 1 && (e.empty() || e[0] != '-'))
                r[a] = e;
            else
                r[a] = em.def(false, e, 0, std::max(1, nterms - 1)).name;
        }
        mom_q[m] = r;
        return r;
    }

    Val q2(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_q2.find(m);
        if (it != mom_q2.end()) return it->second;
        auto q = Q(m);
        Val v = em.def(false, "__builtin_fmaf(" + q[0] + ", " + q[0] + ", __builtin_fmaf(" + q[1] + ", " + q[1] + ", " +
                                  q[2] + " * " + q[2] + "))",
                       2, 2);
        em.cnt_pre[1] += 1;
        mom_q2[m] = v;
        return v;
    }

    // Qx^2 + Qy^2 of a k-dependent momentum Q + ck k z (hoisted)
    Val qxy2(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_qxy2.find(m);
        if (it != mom_qxy2.end()) return it->second;
        auto q = Q(m);
        Val v = em.def(false, "__builtin_fmaf(" + q[0] + ", " + q[0] + ", " + q[1] + " * " + q[1] + ")", 2);
        em.cnt_pre[1] += 1;
        return mom_qxy2[m] = v;
    }

    // Qz + ck k of a k-dependent momentum (a line carries k at most once: ck = +-1), so that
    // |Q + ck k z|^2 = Qx^2 + Qy^2 + (Qz + ck k)^2 is formed without cancelling against |Q|^2; and
    // d|p|^2/dk = 2 ck (Qz + ck k)
    const std::string& kz(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_t.find(m);
        if (it != mom_t.end()) return it->second;
        auto q = Q(m);
        const int ck = moms[m][n];
        const std::string t = ck == 1    ? em.def(true, q[2] + " + kk", 0).name
                              : ck == -1 ? em.def(true, q[2] + " - kk", 0).name
                                         : em.def(true, "__builtin_fmaf(" + fstr(ck) + ", kk, " + q[2] + ")", 2).name;
        if (em.act[2]) mom_dp2[m] = em.def(true, fstr(2.0 * ck) + " * " + t, 1).name;
        return mom_t[m] = t;
    }

    Val p2(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_p2.find(m);
        if (it != mom_p2.end()) return it->second;
        Val v;
        if (is_k(m)) {
            const std::string& t = kz(m);
            v = em.def(true, "__builtin_fmaf(" + t + ", " + t + ", " + qxy2(m).name + ")", 2);
        } else {
            v = q2(m);
        }
        mom_p2[m] = v;
        return v;
    }

    // |p|^2 + lambda_g, the interaction's denominator: for a k-dependent momentum lambda joins the hoisted
    // Qx^2 + Qy^2, so that the loop spends one fused multiply-add on it
    Val p2_lam(int m, int grp) {
        Emitter::ValueScope vs_(em);
        const std::string lam = "LAM" + std::to_string(grp);
        if (!is_k(m)) return em.def(false, p2(m).name + " + " + lam, 0);
        Val base = em.def(false, qxy2(m).name + " + " + lam, 0);
        const std::string& t = kz(m);
        return em.def(true, "__builtin_fmaf(" + t + ", " + t + ", " + base.name + ")", 2);
    }

    // time pair: propagator from interaction line a to line b (a != b)
    std::pair<std::string, std::string> T(int a, int b) {
        Emitter::ValueScope vs_(em);
        auto key = std::make_pair(a, b);
        auto it = tpair.find(key);
        if (it != tpair.end()) return it->second;
        std::string ta = a == 0 ? "0.0f" : em.tag + "t" + std::to_string(a);
        std::string tb = b == 0 ? "0.0f" : em.tag + "t" + std::to_string(b);
        std::string la = a == 0 ? "" : em.tag + "tl" + std::to_string(a);
        std::string lb = b == 0 ? "" : em.tag + "tl" + std::to_string(b);
        std::string pos = em.tag + "ps" + std::to_string(a) + "_" + std::to_string(b);
        em.pre << "    const bool " << pos << " = " << tb << " > " << ta << ";\n";
        std::string dexpr = lb.empty() ? "-" + la : la.empty() ? lb : lb + " - " + la;
        Val d = em.def(false, dexpr, 0, (la.empty() || lb.empty()) ? 0 : 1);
        Val t2 = em.def(false, pos + " ? " + d.name + " : " + d.name + " + BL", 0, 2);  // add + select
        em.cnt_pre[0] += 1;  // the compare
        // beta - tau' (log2 units), formed from the time difference so that it is exact as tau' -> beta
        Val c2 = em.def(false, pos + " ? BL - " + d.name + " : -" + d.name, 0, 2);
        tcomp[key] = c2.name;
        tpair[key] = {t2.name, pos};
        return tpair[key];
    }

    // the exponent's time for a propagator from line a to line b: tau' when eps >= 0, beta - tau' when
    // eps < 0 (log2 units), so that G0 = s 2^(-|eps| S) / (1 + 2^(-beta |eps|)) has no factor above 1
    Val S(int m, int a, int b) {
        Emitter::ValueScope vs_(em);
        T(a, b);
        const auto& en = E(m);
        return em.def(is_k(m), en.pos + " ? " + tpair[{a, b}].first + " : " + tcomp[{a, b}], 0);
    }

    int add_factor(const Val& v, bool k, int sgn = -1) {
        vals.push_back(v);
        val_k.push_back(k);
        val_sgn.push_back(sgn);
        is_sgn.push_back(0);
        return (int)vals.size() - 1;
    }

    // the sign of the propagator from line a to line b (-1 when b precedes a) as a hoisted factor: a
    // k-dependent propagator is computed without it and the sign joins the hoisted multipliers
    int sign_factor(int a, int b) {
        Emitter::ValueScope vs_(em);
        auto key = std::make_pair(a, b);
        auto it = sgn_id_.find(key);
        if (it != sgn_id_.end()) return it->second;
        Val sv = em.def(false, T(a, b).second + " ? -1.0f : 1.0f", 0);
        const int id = add_factor(sv, false);
        is_sgn[id] = 1;
        return sgn_id_[key] = id;
    }

    const Energy& E(int m) {
        Emitter::ValueScope vs_(em);
        auto it = energy.find(m);
        if (it != energy.end()) return it->second;
        const bool k = is_k(m);
        Val p = p2(m);
        Energy en;
        en.k = k;
        Val e = em.def(k, p.name + " - MU", 0);
        en.ae = "__builtin_fabsf(" + e.name + ")";  // an operand modifier: free
        en.pos = em.tag + "pe" + std::to_string(m);
        (k ? em.loop : em.pre) << "    const bool " << en.pos << " = " << e.name << " >= 0.0f;\n";
        em.cnt(k)[0] += 1;
        en.em = em.def(k, "__builtin_amdgcn_exp2f(-BL * " + en.ae + ")", 3).name;
        em.cnt(k)[1] += 1;
        Val den = em.def(k, en.em + " + 1.0f", 0);
        en.r = em.def(k, "__builtin_amdgcn_rcpf(" + den.name + ")", 3).name;
        energy[m] = en;
        return energy[m];
    }

    // nF(eps) and 1 - nF(eps) of a momentum
    std::map<int, std::string> mom_nf, mom_omnf;
    const std::string& nF(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_nf.find(m);
        if (it != mom_nf.end()) return it->second;
        const Energy& en = E(m);
        Val p = em.def(en.k, en.em + " * " + en.r, 1);
        return mom_nf[m] = em.def(en.k, en.pos + " ? " + p.name + " : " + en.r, 0).name;
    }
    const std::string& omnF(int m) {
        Emitter::ValueScope vs_(em);
        auto it = mom_omnf.find(m);
        if (it != mom_omnf.end()) return it->second;
        const Energy& en = E(m);
        Val p = em.def(en.k, en.em + " * " + en.r, 1);
        return mom_omnf[m] = em.def(en.k, en.pos + " ? " + en.r + " : " + p.name, 0).name;
    }

    // |G0| = 2^(-|eps| S) / (1 + 2^(-beta |eps|)) of the propagator from line a to line b (a != b)
    Val gmag(int m, int a, int b) {
        Emitter::ValueScope vs_(em);
        const bool k = is_k(m);
        Val sv = S(m, a, b);
        const Energy& en = E(m);
        Val ex = em.def(k, "__builtin_amdgcn_exp2f(-" + en.ae + " * " + sv.name + ")", 3);
        em.cnt(k)[1] += 1;
        return em.def(k, ex.name + " * " + en.r, 1);
    }

    // ---- Taylor mode (eq. taylor_node; eq. green_ct and eq. interaction_ct are the leaves' series) ----
    std::map<int, std::string> bfac_;                         // beta^i / i!
    std::map<std::pair<int, int>, std::vector<std::string>> tser_;  // tau'^i / i! per time pair

    const std::string& bfac(int i) {
        Emitter::ValueScope vs_(em);
        auto it = bfac_.find(i);
        if (it != bfac_.end()) return it->second;
        std::string v = i == 1 ? std::string("BETA") : em.def(false, bfac(i - 1) + " * BETA * " + fstr(1.0 / i), 1, 2).name;
        return bfac_[i] = v;
    }

    // tau'^i / i!, i = 0..M, for the propagator from line a to line b (tau' in (0, beta])
    const std::vector<std::string>& tser(int a, int b, int M) {
        Emitter::ValueScope vs_(em);
        auto key = std::make_pair(a, b);
        auto& t = tser_[key];
        if (t.empty()) {
            t.push_back("1.0f");
            t.push_back(em.def(false, T(a, b).first + " * 0.693147181f", 1).name);
        }
        while ((int)t.size() <= M) {
            const int i = (int)t.size();
            t.push_back(em.def(false, t[i - 1] + " * " + t[1] + " * " + fstr(1.0 / i), 1, 2).name);
        }
        return t;
    }

    // G0 as a series in dmu: eps = |p|^2 - mu - dmu, so G0(eps) = +-exp(-eps tau') D(eps) with
    // D = 1 / (1 + exp(-beta eps)) = 1 - nF (or nF at equal time).  exp(dmu tau') has coefficients tau'^i / i!;
    // D's coefficients relative to D follow from (1 + e exp(beta dmu)) D = 1: delta_0 = 1,
    // delta_j = -nF sum_{i=1..j} beta^i/i! delta_{j-i}, and G0's coefficient j is
    // |G0| sum_{i=0..j} tau'^i/i! delta_{j-i} (with the sign).  The k tangent of coefficient m is
    // -(m + 1) g_{m+1} d|p|^2/dk.
    int g_leaf_taylor(const Line& ln) {
        int m = momentum(ln.mom);
        int a = ln.src / 2, b = ln.dst / 2;
        auto key = std::make_tuple(m, a, b);
        auto it = gleaf.find(key);
        if (it != gleaf.end()) return it->second;
        const bool k = is_k(m);
        E(m);
        const bool kt = em.act[2] && k;
        const int M = coefs.max_m + (kt ? 1 : 0);
        std::vector<std::string> dser(M + 1);
        dser[0] = "1.0f";
        const std::string nf = M >= 1 ? nF(m) : std::string();
        const std::string d0 = a == b ? omnF(m) : std::string();
        Val g0;
        if (a != b) g0 = gmag(m, a, b);
        if (a != b) tser(a, b, M);
        Emitter::DerivScope ds(em);
        for (int j = 1; j <= M; ++j) {
            std::string acc;
            int t = 0;
            for (int i = 1; i <= j; ++i) {
                if (i == j) {
                    acc = acc.empty() ? bfac(i) : acc + " + " + bfac(i);
                } else {
                    acc = acc.empty() ? bfac(i) + " * " + dser[j - i]
                                      : "__builtin_fmaf(" + bfac(i) + ", " + dser[j - i] + ", " + acc + ")";
                }
                ++t;
            }
            std::string sum = t == 1 ? acc : em.def(k, acc, 2, t - 1).name;
            dser[j] = em.def(k, "-" + nf + " * " + sum, 1).name;
        }
        std::vector<std::string> g(M + 1);
        Val v;
        if (a == b) {
            // equal time (0^-): nF(eps - dmu) = 1 - D(eps - dmu), D = 1 - nF
            v = Val{nF(m), k, std::vector<std::string>(em.nco() - 1)};
            for (int j = 1; j <= M; ++j) g[j] = em.def(k, "-" + d0 + " * " + dser[j], 1).name;
        } else {
            auto tp = T(a, b);
            {
                Emitter::ValueScope vs(em);
                v = k ? g0 : em.def(k, tp.second + " ? -" + g0.name + " : " + g0.name, 0);
            }
            const auto& ts = tser(a, b, M);
            for (int j = 1; j <= M; ++j) {
                std::string acc = dser[j];
                for (int i = 1; i <= j; ++i)
                    acc = i == j ? acc + " + " + ts[i] : "__builtin_fmaf(" + ts[i] + ", " + dser[j - i] + ", " + acc + ")";
                Val u = em.def(k, acc, 2, j);
                Val gj = em.def(k, g0.name + " * " + u.name, 1);
                g[j] = k ? gj.name : em.def(k, tp.second + " ? -" + gj.name + " : " + gj.name, 0).name;
            }
        }
        g[0] = v.name;
        for (int j = 1; j <= coefs.max_m; ++j) {
            const int e = coefs.find(j, 0, 0);
            if (e > 0) v.d[e - 1] = g[j];
        }
        if (kt) {
            for (int j = 0; j <= coefs.max_m; ++j) {
                const int e = coefs.find(j, 0, 1);
                if (e <= 0) continue;
                v.d[e - 1] = j == 0 ? em.def(true, "-" + g[1] + " * " + mom_dp2[m], 1).name
                                    : em.def(true, fstr(-(double)(j + 1)) + " * " + g[j + 1] + " * " + mom_dp2[m], 1, 2).name;
            }
        }
        const int id = add_factor(v, k, k && a != b ? sign_factor(a, b) : -1);
        gleaf[key] = id;
        ++n_g;
        return id;
    }

    // V as a series in dlambda: 1 / (|p|^2 + lambda + dlambda) has coefficients (-1)^l r^(l+1) (the
    // factor 8 pi gamma is applied at the end); the k tangent of coefficient l is (l + 1) c_{l+1} d|p|^2/dk.
    int v_leaf_taylor(const Line& ln, int grp) {
        int m = momentum(ln.mom);
        auto key = std::make_pair(m, grp);
        auto it = vleaf.find(key);
        if (it != vleaf.end()) return it->second;
        const bool k = is_k(m);
        Val s = p2_lam(m, grp);
        Val v = em.def(k, "__builtin_amdgcn_rcpf(" + s.name + ")", 3);
        const bool kt = em.act[2] && k;
        const int L = coefs.max_l + (kt ? 1 : 0);
        std::vector<std::string> c(L + 1);
        c[0] = v.name;
        Emitter::DerivScope ds(em);
        for (int l = 1; l <= L; ++l) c[l] = em.def(k, "-" + c[l - 1] + " * " + v.name, 1).name;
        for (int l = 1; l <= coefs.max_l; ++l) {
            const int e = coefs.find(0, l, 0);
            if (e > 0) v.d[e - 1] = c[l];
        }
        if (kt) {
            for (int l = 0; l <= coefs.max_l; ++l) {
                const int e = coefs.find(0, l, 1);
                if (e <= 0) continue;
                v.d[e - 1] = l == 0 ? em.def(true, c[1] + " * " + mom_dp2[m], 1).name
                                    : em.def(true, fstr((double)(l + 1)) + " * " + c[l + 1] + " * " + mom_dp2[m], 1, 2).name;
            }
        }
        const int id = add_factor(v, k);
        vleaf[key] = id;
        ++n_v;
        return id;
    }

    int g_leaf(const Line& ln) {
        if (c.taylor_order > 0) return g_leaf_taylor(ln);
        int m = momentum(ln.mom);
        int a = ln.src / 2, b = ln.dst / 2;
        auto key = std::make_tuple(m, a, b);
        auto it = gleaf.find(key);
        if (it != gleaf.end()) return it->second;
        bool k = is_k(m);
        E(m);
        Val v;
        std::string tprime;  // tau' (the propagator's time shifted into (0, beta])
        if (a == b) {
            // equal time (0^-): nF(eps)
            v = Val{nF(m), k, std::vector<std::string>(em.nco() - 1)};
            tprime = "BETA";
        } else {
            auto tp = T(a, b);
            Val g = gmag(m, a, b);
            v = k ? g : em.def(k, tp.second + " ? -" + g.name + " : " + g.name, 0);
            tprime = tp.first + " * 0.693147181f";
        }
        if (em.act[0] || (em.act[2] && k)) {
            Emitter::DerivScope ds(em);
            // d G0 / d mu = G0 (tau' - beta nF);  d G0 / dk = -(d G0 / d mu) d|p|^2/dk.  At equal
            // time tau' = beta and tau' - beta nF = beta (1 - nF), taken without cancellation.
            auto bi = mom_bnf.find(m);
            if (a != b && bi == mom_bnf.end()) bi = mom_bnf.emplace(m, em.def(k, "BETA * " + nF(m), 1).name).first;
            Val lg = a == b ? em.def(k, "BETA * " + omnF(m), 1)
                            : em.def(k, tprime + " - " + bi->second, 0, 2);
            Val gm = em.def(k, v.name + " * " + lg.name, 1);
            if (em.act[0]) v.d[em.dir(0) - 1] = gm.name;
            if (em.act[2] && k) v.d[em.dir(2) - 1] = em.def(true, "-" + gm.name + " * " + mom_dp2[m], 1).name;
        }
        const int id = add_factor(v, k, k && a != b ? sign_factor(a, b) : -1);
        gleaf[key] = id;
        ++n_g;
        return id;
    }

    int v_leaf(const Line& ln, int grp) {
        if (c.taylor_order > 0) return v_leaf_taylor(ln, grp);
        int m = momentum(ln.mom);
        auto key = std::make_pair(m, grp);
        auto it = vleaf.find(key);
        if (it != vleaf.end()) return it->second;
        bool k = is_k(m);
        Val s = p2_lam(m, grp);
        Val v = em.def(k, "__builtin_amdgcn_rcpf(" + s.name + ")", 3);
        if (em.act[1] || (em.act[2] && k)) {
            Emitter::DerivScope ds(em);
            // d V / d lambda = -V^2 (times 8 pi gamma, applied at the end); d V / dk = -V^2 d|p|^2/dk
            Val vl = em.def(k, "-" + v.name + " * " + v.name, 1);
            if (em.act[1]) v.d[em.dir(1) - 1] = vl.name;
            if (em.act[2] && k) v.d[em.dir(2) - 1] = em.def(true, vl.name + " * " + mom_dp2[m], 1).name;
        }
        const int id = add_factor(v, k);
        vleaf[key] = id;
        ++n_v;
        return id;
    }

    // A factored value with a pending multiplier: c * prod_{i in m} vals[i] * v, where m is a sorted multiset
    // of hoisted factors (k-independent values and the signs of k-dependent propagators) and c a constant.
    // Multipliers travel up the factored sum and are applied where the external-momentum loop pays least
    // for them: folded into a hoisted operand, as the constant of a fused multiply-add, or (value-only
    // graphs) on the root's per-sample phase factor.  A sign flip is free anywhere (an operand modifier).
    // Invariant: a hoisted v carries no m.
    struct SVal {
        Val v;
        std::vector<int> m{};
        double c = 1.0;
    };

    std::map<std::vector<int>, Val> hoist_;

    // the hoisted product c prod vals[ids]
    Val hoist(const std::vector<int>& ids, double c = 1.0) {
        if (ids.empty()) return em.constant(c);
        auto it = hoist_.find(ids);
        Val p;
        if (it != hoist_.end()) {
            p = it->second;
        } else {
            p = vals[ids[0]];
            for (size_t i = 1; i < ids.size(); ++i) p = em.mul(p, vals[ids[i]]);
            hoist_[ids] = p;
        }
        return em.scale(p, c);
    }

    // m with pairs of equal signs cancelled, sorted
    std::vector<int> msort(std::vector<int> m) const {
        std::sort(m.begin(), m.end());
        std::vector<int> out;
        for (size_t i = 0; i < m.size(); ++i) {
            if (is_sgn[m[i]] && i + 1 < m.size() && m[i + 1] == m[i]) {
                ++i;
                continue;
            }
            out.push_back(m[i]);
        }
        return out;
    }

    SVal norm(SVal s) {
        s.m = msort(s.m);
        if (!s.v.kdep && !s.m.empty()) {
            s.v = em.mul(s.v, hoist(s.m));
            s.m.clear();
        }
        return s;
    }

    // x times the hoisted r prod vals[q]: free when x is hoisted or the multiplier is +-1
    Val apply(const Val& x, const std::vector<int>& q, double r) {
        if (q.empty()) return em.scale(x, r);
        return em.mul(x, hoist(q, r));
    }

    static std::vector<int> common(const std::vector<int>& a, const std::vector<int>& b) {
        std::vector<int> o;
        std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
        return o;
    }
    static std::vector<int> minus(const std::vector<int>& a, const std::vector<int>& b) {
        std::vector<int> o;
        std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(o));
        return o;
    }
    // the loop cost of applying (q, r) to x
    static int cost(const Val& x, const std::vector<int>& q, double r) {
        return x.kdep && (!q.empty() || (r != 1.0 && r != -1.0)) ? 1 : 0;
    }

    // r prod vals[q] * x + y in one operation
    Val madd(const Val& x, const std::vector<int>& q, double r, const Val& y) {
        if (q.empty() && r == 1.0) return em.add(x, y);
        if (q.empty() && r == -1.0) return em.add(em.scale(x, -1.0), y);
        return em.fma(hoist(q, r), x, y);
    }

    // f a + b for a k-dependent factor f, or a + b when f is null.  The multipliers both sides share stay
    // pending; the rest are applied, each side's constant ratio riding on whichever operand is cheapest.
    SVal combine(const Val* f, SVal a, SVal b) {
        a = norm(a);
        b = norm(b);
        const std::vector<int> P = common(a.m, b.m);
        const std::vector<int> qa = minus(a.m, P), qb = minus(b.m, P);
        const double r = a.c / b.c;
        if (!f) {
            if (!a.v.kdep && !b.v.kdep) return norm({em.add(em.scale(a.v, r), b.v), P, b.c});
            if (cost(b.v, qb, 1.0) <= cost(a.v, qa, 1.0)) return norm({madd(a.v, qa, r, apply(b.v, qb, 1.0)), P, b.c});
            return norm({madd(b.v, qb, 1.0 / r, apply(a.v, qa, 1.0)), P, a.c});
        }
        if (cost(a.v, qa, r) + cost(b.v, qb, 1.0) <= cost(a.v, qa, 1.0) + cost(b.v, qb, 1.0 / r))
            return norm({em.fma(*f, apply(a.v, qa, r), apply(b.v, qb, 1.0)), P, b.c});
        return norm({em.fma(*f, apply(a.v, qa, 1.0), apply(b.v, qb, 1.0 / r)), P, a.c});
    }

    // greedy multivariate Horner factoring of sum_t coef_t prod f_t
    SVal horner(std::vector<Term> terms) {
        terms.erase(std::remove_if(terms.begin(), terms.end(), [](const Term& t) { return t.coef == 0.0; }),
                    terms.end());
        if (terms.empty()) return {em.constant(0.0)};
        if (terms.size() == 1) return product(terms[0]);
        std::map<int, int> count;
        for (auto& t : terms) {
            std::set<int> s(t.f.begin(), t.f.end());
            for (int f : s) count[f]++;
        }
        int best = -1, bc = 1;
        bool bk = false;
        for (auto [f, cnt] : count) {
            bool k = val_k[f];
            // external-momentum dependent factors first, then the most frequent
            if (cnt >= 2 && (best < 0 || (k && !bk) || (k == bk && cnt > bc))) {
                best = f;
                bc = cnt;
                bk = k;
            }
        }
        if (best < 0) {
            // no shared factor: plain sum
            SVal acc = product(terms[0]);
            for (size_t i = 1; i < terms.size(); ++i) acc = combine(nullptr, product(terms[i]), acc);
            return acc;
        }
        std::vector<Term> A, B;
        for (auto& t : terms) {
            auto it = std::find(t.f.begin(), t.f.end(), best);
            if (it != t.f.end()) {
                Term u = t;
                u.f.erase(u.f.begin() + (it - t.f.begin()));
                A.push_back(u);
            } else {
                B.push_back(t);
            }
        }
        SVal ha = horner(A);
        if (B.empty()) return times(ha, best);
        SVal hb = horner(B);
        if (!val_k[best]) return combine(nullptr, times(ha, best), hb);
        if (val_sgn[best] >= 0) ha.m.push_back(val_sgn[best]);
        return combine(&vals[best], ha, hb);
    }

    std::map<std::string, int> hoisted_id_;

    // a hoisted value (a factored sum) as a factor of its own, so that it can join a multiplier
    int hoisted_factor(const Val& v) {
        auto it = hoisted_id_.find(v.name);
        if (it != hoisted_id_.end()) return it->second;
        return hoisted_id_[v.name] = add_factor(v, false);
    }

    // s times factor f: a hoisted factor (and a propagator's sign) joins the multiplier; a hoisted s
    // times a k-dependent f becomes f with s as its multiplier
    SVal times(SVal s, int f) {
        if (!val_k[f]) {
            s.m.push_back(f);
        } else if (!s.v.kdep) {
            const bool one = s.v.name == em.constant(1.0).name;
            if (!one) s.m = {hoisted_factor(s.v)};
            s.v = vals[f];
            if (val_sgn[f] >= 0) s.m.push_back(val_sgn[f]);
        } else {
            s.v = em.mul(vals[f], s.v);
            if (val_sgn[f] >= 0) s.m.push_back(val_sgn[f]);
        }
        return norm(s);
    }

    SVal product(const Term& t) {
        SVal s{em.constant(1.0), {}, t.coef};
        bool have = false;
        std::vector<int> f = t.f;
        std::stable_sort(f.begin(), f.end(), [&](int a, int b) { return val_k[a] < val_k[b]; });
        for (int id : f) {
            if (!val_k[id]) {
                s.m.push_back(id);
                continue;
            }
            s.v = have ? em.mul(s.v, vals[id]) : vals[id];
            have = true;
            if (val_sgn[id] >= 0) s.m.push_back(val_sgn[id]);
        }
        if (!have) {
            s.v = hoist(msort(s.m));
            s.m.clear();
            return s;
        }
        return norm(s);
    }
};

}  // namespace

int default_part_size(int n_diagrams, int n_roots);

bool compile(int order, uint32_t deriv_mask, int taylor_order, int diagram_index, int part_size, int deriv_k,
             int routing, int spin_deg, int generation, Compiled& out, std::string& err) {
    if (order < 1 || order > kMaxOrder) {
        err = "order must be in 1..6";
        return false;
    }
    if (deriv_mask & ~7u) {
        err = "unknown derivative bits";
        return false;
    }
    if (taylor_order < 0 || taylor_order > kMaxTaylor) {
        err = "taylor_order must be in 0..6";
        return false;
    }
    if (deriv_k < 0 || deriv_k > 64) {
        err = "deriv_k must be in 0..64";
        return false;
    }
    if (routing != 0 && routing != 1) {
        err = "routing must be 0 (path) or 1 (building blocks)";
        return false;
    }
    if (spin_deg != 1 && spin_deg != 2) {
        err = "spin_deg must be 1 or 2";
        return false;
    }
    if (generation != 0 && generation != 1) {
        err = "generation must be 0 (enumeration) or 1 (construction)";
        return false;
    }
    out = Compiled{};
    out.deriv_k = deriv_k;
    out.routing = routing;
    out.spin_deg = spin_deg;
    out.generation = generation;
    out.order = order;
    out.dim = 4 * order - 1;
    out.deriv_mask = deriv_mask;
    out.taylor_order = taylor_order;
    const CoefSet cs = taylor_order > 0 ? CoefSet::taylor(deriv_mask, taylor_order) : CoefSet::first_order(deriv_mask);
    out.root_orders = cs.idx;
    out.n_roots = (int)cs.idx.size();
    if (generation == 1) {
        std::vector<std::vector<int>> sigmas;
        if (!construct_sigma(order, sigmas, err)) return false;
        out.diagrams.clear();
        for (auto& sg : sigmas) out.diagrams.push_back(route(sg));
    } else {
        out.diagrams = enumerate_sigma(order);
    }
    if (spin_deg == 1)  // spinless: each closed fermion loop gives its sign only
        for (auto& d : out.diagrams) d.weight = (order + d.n_fermion_loops) % 2 ? -1.0 : 1.0;
    if (routing == 1) {
        // loop momenta and interaction lines from the building blocks, k along the shortest path
        for (auto& d : out.diagrams) {
            Diagram r;
            if (!relabel_building_blocks(d, r, err)) return false;
            int nf;
            auto es = internal_edges(r.sigma, nf);
            for (auto& ln : r.lines) ln.mom[order] = 0;
            for (auto [e, sg] : k_path(2 * order, es, r.out_vertex)) r.lines[e].mom[order] += sg;
            d = std::move(r);
        }
    }
    if (diagram_index >= 0) {
        if (diagram_index >= (int)out.diagrams.size()) {
            err = "diagram_index out of range";
            return false;
        }
        out.diagrams = {out.diagrams[diagram_index]};
    }
    std::set<int> cls;
    for (auto& d : out.diagrams) cls.insert(d.ext_line());
    out.n_root_classes = (int)cls.size();
    if (part_size < 0) {
        err = "part_size must be >= 0";
        return false;
    }
    out.part_size = part_size > 0 ? part_size : default_part_size((int)out.diagrams.size(), out.n_roots);
    CodeStats st;
    emit_eval_source(out, 1, &st);
    for (int i = 0; i < 4; ++i) {
        st.sample_exec[i] = st.sample[i];
        st.k_exec[i] = st.k[i];
        st.k_deriv_exec[i] = st.k_deriv[i];
    }
    if (st.parts > 1) {
        // algorithmic counts: the same graph emitted as one part (no leaf evaluated twice)
        Compiled whole = out;
        whole.part_size = 0;
        CodeStats one;
        emit_eval_source(whole, 1, &one);
        for (int i = 0; i < 4; ++i) {
            st.sample[i] = one.sample[i];
            st.k[i] = one.k[i];
            st.k_deriv[i] = one.k_deriv[i];
        }
    }
    out.stats = st;
    return true;
}

std::string export_text(const Compiled& c) {
    std::ostringstream s;
    const int n = c.order;
    for (auto& d : c.diagrams) {
        for (int v : d.sigma) s << v << " ";
        s << "| w " << d.weight << " | ext " << d.ext_line();
        for (char kind : {'G', 'V'}) {
            s << " | " << kind;
            for (auto& l : d.lines) {
                if (l.kind != kind) continue;
                s << " " << l.src << " " << l.dst;
                for (int j = 0; j <= n; ++j) s << " " << l.mom[j];
                s << " ;";
            }
        }
        s << "\n";
    }
    return s.str();
}

}  // namespace dmc

// ----------------------------------------------------------------------------------------
// Evaluation kernel source.  One lane evaluates one sample; the k-independent part of the
// graph is computed once per sample, then the lane loops over the external momenta.  Every
// weight w = f J is staged (FP32) in the wave's slice of LDS; after each chunk of k values the
// wave transposes the stage so that four lanes own each (k, group, Re/Im) slot, widen to FP64,
// sum w and w^2 over the chunk's 64 samples in a fixed order and add into FP64 running totals in
// LDS.  At the end the block folds its four waves in order and writes one FP64 partial per slot.
// ----------------------------------------------------------------------------------------
namespace dmc {

std::string kernel_name(const Compiled& c, int n_groups) {
    const int nd = (int)c.diagrams.size();
    const int np = c.part_size > 0 && nd > c.part_size ? (nd + c.part_size - 1) / c.part_size : 1;
    return "dmc_eval_o" + std::to_string(c.order) + "_g" + std::to_string(n_groups) + "_r" + std::to_string(c.n_roots) +
           (c.taylor_order > 0 ? "_t" + std::to_string(c.taylor_order) : "") + (nd == 1 ? "_single" : "") +
           (np > 1 ? "_p" + std::to_string(np) : "") + (c.routing == 1 ? "_b" : "");
}

// Diagram parts of a partitioned kernel.  Every part re-evaluates the leaves its diagrams use (and the
// products they share), so parts are grown around shared leaves: diagrams are ranked by root class and by the
// leaves that carry the external momentum; each part then repeatedly takes the unplaced diagram whose leaves
// not yet in the part cost least (a leaf that carries k weighs kKLeafWeight, being evaluated once per external
// momentum; the others 1; ties by rank), starting from an empty part, until it holds part_size diagrams.  One
// part = the whole graph when it fits.
static std::vector<std::vector<int>> diagram_parts(const Compiled& c, int part_size) {
    constexpr int kKLeafWeight = 8;
    const int n = c.order;
    const int nd = (int)c.diagrams.size();
    std::vector<std::vector<int>> parts;
    if (part_size <= 0 || nd <= part_size) {
        parts.emplace_back();
        for (int i = 0; i < nd; ++i) parts[0].push_back(i);
        return parts;
    }
    std::vector<std::pair<std::vector<int>, int>> keyed;
    for (int i = 0; i < nd; ++i) {
        const Diagram& d = c.diagrams[i];
        std::vector<int> key{d.ext_line()};
        std::vector<std::vector<int>> kl;
        for (auto& ln : d.lines) {
            Mom m = normalise(ln.mom, n);
            if (m[n] == 0) continue;
            std::vector<int> e{ln.kind == 'G' ? 0 : 1, ln.src / 2, ln.dst / 2};
            if (ln.kind == 'V') e[1] = e[2] = 0;
            e.insert(e.end(), m.begin(), m.end());
            kl.push_back(e);
        }
        std::sort(kl.begin(), kl.end());
        for (auto& e : kl) key.insert(key.end(), e.begin(), e.end());
        keyed.push_back({key, i});
    }
    std::stable_sort(keyed.begin(), keyed.end());
    std::vector<int> rank(nd);
    for (int r = 0; r < nd; ++r) rank[keyed[r].second] = r;
    // leaves: a propagator by its time pair and momentum (up to sign), an interaction by its momentum
    std::map<std::vector<int>, int> leaf_id;
    std::vector<std::vector<std::pair<int, int>>> dl(nd);  // (leaf, weight)
    for (int i = 0; i < nd; ++i) {
        for (auto& ln : c.diagrams[i].lines) {
            Mom m = normalise(ln.mom, n);
            const bool g = ln.kind == 'G';
            std::vector<int> key{g ? 0 : 1, g ? ln.src / 2 : 0, g ? ln.dst / 2 : 0};
            key.insert(key.end(), m.begin(), m.begin() + n + 1);
            const int id = leaf_id.emplace(key, (int)leaf_id.size()).first->second;
            dl[i].push_back({id, m[n] != 0 ? kKLeafWeight : 1});
        }
        std::sort(dl[i].begin(), dl[i].end());
        dl[i].erase(std::unique(dl[i].begin(), dl[i].end()), dl[i].end());
    }
    std::vector<std::vector<int>> users(leaf_id.size());
    for (int i = 0; i < nd; ++i)
        for (auto [l, w] : dl[i]) users[l].push_back(i);
    std::vector<char> placed(nd, 0);
    std::vector<int> cost(nd, 0);
    int left = nd;
    while (left > 0) {
        std::set<std::pair<int, int>> q;  // (cost of the leaves it would add, rank) of every unplaced diagram
        for (int i = 0; i < nd; ++i)
            if (!placed[i]) {
                cost[i] = 0;
                for (auto [l, w] : dl[i]) cost[i] += w;
                q.insert({cost[i], rank[i]});
            }
        std::vector<char> in(leaf_id.size(), 0);
        parts.emplace_back();
        int next = keyed[q.begin()->second].second;
        while (true) {
            q.erase({cost[next], rank[next]});
            placed[next] = 1;
            --left;
            parts.back().push_back(next);
            for (auto [l, w] : dl[next]) {
                if (in[l]) continue;
                in[l] = 1;
                for (int j : users[l])
                    if (!placed[j]) {
                        q.erase({cost[j], rank[j]});
                        cost[j] -= w;
                        q.insert({cost[j], rank[j]});
                    }
            }
            if ((int)parts.back().size() >= part_size || q.empty()) break;
            next = keyed[q.begin()->second].second;
        }
    }
    return parts;
}

int default_part_size(int n_diagrams, int n_roots) {
    // Measured on MI355X with the external momentum on a path of chords (a part's k-independent code dominates
    // and runs once per chunk of momenta) and leaf-grown parts.  Per 2^22 samples x 32 k: order 5 in one part
    // 3.1 ms, in 3 parts 5.0 ms; order 6 in parts of 1600, 2400, 3200 diagrams 32.4, 31.7, 33.6 ms (sorted, not
    // grown: 37.1 ms at 1600).  The order-6 d/dk graph at k_F with 3 lambda groups and 33 k, per 2^26 samples:
    // 1697, 1603, 1684 ms (sorted, not grown: 1881 ms at 1600); with the momentum loop in scalar control, parts
    // of 2000, 2400, 2800 diagrams: 1433, 1414, 1418 ms.  Bigger parts evaluate fewer leaves twice; past
    // ~2400 diagrams their register pressure costs more.  More roots (derivative or Taylor coefficients) multiply
    // a part's live values: parts shrink as R^1.5.
    const double base = 2400.0;
    const int per = std::max(16, (int)(base / std::pow(std::max(1.0, n_roots / 2.0), 1.5)));
    return n_diagrams <= per ? 0 : per;
}

std::string emit_eval_source(const Compiled& c, int n_groups, CodeStats* stats) {
    const int n = c.order;
    std::vector<int> cls;
    for (auto& d : c.diagrams) cls.push_back(d.ext_line());
    std::sort(cls.begin(), cls.end());
    cls.erase(std::unique(cls.begin(), cls.end()), cls.end());
    const int NR = c.n_roots;
    const auto parts = diagram_parts(c, c.part_size);
    const bool split = parts.size() > 1;

    // derivative roots (coefficient entries j > 0) are emitted apart from the value (root 0): their
    // k-dependent code and epilogue run only at the first KD external momenta (all of them when KD is 0)
    const int KD = NR > 1 ? c.deriv_k : 0;
    struct Part {
        std::vector<int> cls;
        std::string pre, loop, epi, loopd, epid;
        std::vector<std::string> fplain;  // one straight-line part: f per (group, root, component) without J
        int64_t cnt_pre[4], cnt_loop[4], cnt_loopd[4];
    };
    std::vector<Part> pc;
    int64_t epi_ops[4] = {0, 0, 0, 0}, epi_ops_d[4] = {0, 0, 0, 0};
    for (size_t pi = 0; pi < parts.size(); ++pi) {
        // a kernel in parts builds each part for one lambda group, passed at run time
        const int pg = split ? 1 : n_groups;
        Builder b(c, pg);
        b.em.split_deriv = NR > 1;
        if (split) {
            b.em.tag = "p" + std::to_string(pi) + "_";
            b.em.prefix = b.em.tag + "v";
        }
        std::vector<int> pcls;
        for (int di : parts[pi]) pcls.push_back(c.diagrams[di].ext_line());
        std::sort(pcls.begin(), pcls.end());
        pcls.erase(std::unique(pcls.begin(), pcls.end()), pcls.end());
        // roots[g][class index within the part]
        std::vector<std::vector<Builder::SVal>> roots(pg);
        for (int g = 0; g < pg; ++g) {
            for (int r : pcls) {
                std::vector<Term> terms;
                for (int di : parts[pi]) {
                    const Diagram& d = c.diagrams[di];
                    if (d.ext_line() != r) continue;
                    Term t;
                    t.coef = d.weight;
                    for (auto& ln : d.lines) t.f.push_back(ln.kind == 'G' ? b.g_leaf(ln) : b.v_leaf(ln, g));
                    std::sort(t.f.begin(), t.f.end());
                    terms.push_back(t);
                }
                Builder::SVal rt = b.horner(terms);
                // with derivative entries the multiplier's own coefficients enter by the product rule
                if (b.em.nco() > 1 && !rt.m.empty()) {
                    rt.v = b.em.mul(rt.v, b.hoist(rt.m));
                    rt.m.clear();
                }
                roots[g].push_back(rt);
            }
        }
        // epilogue: f = sum_r root_r * (scale_g cos, scale_g sin)(pi tau_r / beta), and the same for
        // every derivative root (the phases and scale depend on none of mu, lambda, k)
        std::ostringstream epi, epid;
        std::vector<std::string> fplain;
        for (int g = 0; g < pg; ++g) {
            for (int ro = 0; ro < NR; ++ro) {
                std::ostringstream& eo = ro == 0 ? epi : epid;
                int64_t* eops = ro == 0 ? epi_ops : epi_ops_d;
                std::string fr, fi, frp, fip;  // with J folded in (one straight-line part), and without
                for (size_t ri = 0; ri < pcls.size(); ++ri) {
                    int r = pcls[ri];
                    const std::string rv = Emitter::cf(roots[g][ri].v, ro);
                    if (rv.empty()) continue;
                    // the root's pending coefficient and, for Taylor coefficients becoming derivatives, m! l!,
                    // go onto the per-sample phase factors
                    const auto& mo = c.root_orders[ro];
                    double fac = roots[g][ri].c;
                    for (int i = 2; i <= mo[0]; ++i) fac *= i;
                    for (int i = 2; i <= mo[1]; ++i) fac *= i;
                    std::string pcn = "PC" + std::to_string(g) + "_" + std::to_string(r);
                    std::string psn = "PS" + std::to_string(g) + "_" + std::to_string(r);
                    if (!roots[g][ri].m.empty()) {
                        const std::string mh = b.hoist(roots[g][ri].m).name;
                        pcn = b.em.def(false, mh + " * " + pcn, 1).name;
                        if (r != 0) psn = b.em.def(false, mh + " * " + psn, 1).name;
                    }
                    if (fac != 1.0) {
                        pcn = b.em.def(false, fstr(fac) + " * " + pcn, 1).name;
                        if (r != 0) psn = b.em.def(false, fstr(fac) + " * " + psn, 1).name;
                    }
                    // one straight-line part: the Jacobian joins the per-sample factors, so the weight f J
                    // comes out of the root sum itself (f alone is formed only for f_out)
                    const std::string pcj = split ? pcn : b.em.def(false, pcn + " * J", 1).name;
                    const std::string psj = split || r == 0 ? psn : b.em.def(false, psn + " * J", 1).name;
                    auto term = [](std::string& acc, const std::string& x, const std::string& y) {
                        acc = acc.empty() ? x + " * " + y : "__builtin_fmaf(" + x + ", " + y + ", " + acc + ")";
                    };
                    eops[fr.empty() ? 1 : 2]++;
                    term(fr, rv, pcj);
                    term(frp, rv, pcn);
                    if (r == 0) continue;
                    eops[fi.empty() ? 1 : 2]++;
                    term(fi, rv, psj);
                    term(fip, rv, psn);
                }
                if (!split) {
                    if (fr.empty()) fr = frp = "0.0f";
                    if (fi.empty()) fi = fip = "0.0f";
                    eo << "        const float FR" << g << "_" << ro << " = " << fr << ";\n";
                    eo << "        const float FI" << g << "_" << ro << " = " << fi << ";\n";
                    fplain.push_back(frp);
                    fplain.push_back(fip);
                } else {
                    const int slot = ro * 2;
                    if (!fr.empty()) eo << "        st[(row + " << slot << ") * 64] += " << fr << ";\n";
                    if (!fi.empty()) eo << "        st[(row + " << slot + 1 << ") * 64] += " << fi << ";\n";
                    eops[0] += (!fr.empty()) + (!fi.empty());
                }
            }
        }
        Part p;
        p.cls = pcls;
        p.pre = b.em.pre.str();
        p.loop = b.em.loop.str();
        p.epi = epi.str();
        p.loopd = b.em.loopd.str();
        p.epid = epid.str();
        p.fplain = fplain;
        for (int i = 0; i < 4; ++i) {
            p.cnt_pre[i] = b.em.cnt_pre[i];
            p.cnt_loop[i] = b.em.cnt_loop[i];
            p.cnt_loopd[i] = b.em.cnt_loopd[i];
        }
        pc.push_back(std::move(p));
    }

    // a graph whose roots all sit at external time 0 (order 1) has no phase: its imaginary parts are zero, so
    // only the real slots are staged and reduced (the imaginary sums stay 0; f_out still receives zeros)
    const bool real_only = !split && cls.size() == 1 && cls[0] == 0;
    const int SPK = (real_only ? 1 : 2) * n_groups * NR;
    const int KC = SPK <= 16 ? 16 / SPK : 1;
    const int SCH = KC * SPK;
    const int M = (SCH + 15) / 16;
    int zero_slots = 0;  // one straight-line part: (group, root, component) slots with no term

    auto indent = [](std::ostringstream& out, const std::string& text, const std::string& pad) {
        std::istringstream in(text);
        std::string line;
        while (std::getline(in, line)) out << pad << line << "\n";
    };

    std::ostringstream s;
    s << "// generated: order " << n << ", " << c.diagrams.size() << " diagrams, " << n_groups << " lambda group(s)";
    if (split) s << ", " << parts.size() << " parts";
    s << "\n";
    s << "#define KERNEL_NAME " << kernel_name(c, n_groups) << "\n";
    s << "#define DIM " << c.dim << "\n#define NGRP " << n_groups << "\n#define NROOT " << NR << "\n#define SPK " << SPK
      << "\n#define KC " << KC << "\n#define SCH " << SCH << "\n#define MST " << M << "\n#define SPK1 " << 2 * NR
      << "\n#define KD " << KD << "\n";
    s << R"K(
struct EvalArgs {
    const float* x; long long ld; const float* jac; long long n;
    double* partial; unsigned int* nonfinite; float* f_out; float* imp_out;
    int n_k; int s_total; int kc; int imp_roots;
    float mu, beta, bl, blmu, inv2beta, pad2;
    float lam[8]; float scale[8];
    float k[64];
};
)K";
    const char* ax = "xyz";
    // inputs of a part, one LDS row of 64 lanes each: q (3n), t (n - 1), t log2(e) (n - 1)
    std::vector<std::string> ins;
    for (int j = 0; j < n; ++j)
        for (int e = 0; e < 3; ++e) ins.push_back(std::string("q") + std::to_string(j) + ax[e]);
    for (int j = 1; j < n; ++j) ins.push_back("t" + std::to_string(j));
    for (int j = 1; j < n; ++j) ins.push_back("tl" + std::to_string(j));
    if (split) {
        // every part is a function of its own (never inlined): the compiler allocates registers and
        // schedules each part alone, so compile time and register use grow with the part, not
        // with the whole graph.  in: this lane's inputs (stride 64); st: this lane's stage column.
        s << "typedef __attribute__((address_space(3))) float LdsF;\n";
        for (size_t pi = 0; pi < pc.size(); ++pi) {
            const std::string tg = "p" + std::to_string(pi) + "_";
            s << "\n// part " << pi << " (" << parts[pi].size() << " diagrams)\n";
            // the inputs and the stage live in LDS: typed as such, the part reads and writes them with ds_
            // instructions instead of flat ones (a flat access waits on both the vector-memory and LDS counters)
            s << "__device__ __attribute__((noinline)) void dmc_part_" << pi
              << "(const EvalArgs* __restrict__ ap, const LdsF* __restrict__ in, LdsF* __restrict__ st, "
                 "const LdsF* __restrict__ kl, const int kb_, const int nkc_, const int grp_, const int ml_) {\n";
            // a device function receives its arguments in vector registers; the chunk and group indices are the same
            // in every lane, and saying so keeps the momentum loop and its branches scalar
            s << "    const int kb = __builtin_amdgcn_readfirstlane(kb_), nkc = __builtin_amdgcn_readfirstlane(nkc_);\n";
            s << "    const int grp = __builtin_amdgcn_readfirstlane(grp_), ml = __builtin_amdgcn_readfirstlane(ml_);\n";
            s << "    const float MU = ap->mu, BL = ap->bl, BLMU = ap->blmu, BETA = ap->beta;\n";
            s << "    (void)MU; (void)BL; (void)BLMU; (void)BETA;\n";
            s << "    const float LAM0 = ap->lam[grp];\n";
            for (size_t i = 0; i < ins.size(); ++i)
                s << "    const float " << tg << ins[i] << " = in[" << i * 64 << "];\n";
            for (int r : pc[pi].cls) {
                if (r == 0) {
                    s << "    const float PC0_0 = ap->scale[grp];\n";
                } else {
                    s << "    float sn0_" << r << ", cs0_" << r << ";\n";
                    s << "    sincospif(" << tg << "t" << r << " * (2.0f * ap->inv2beta), &sn0_" << r << ", &cs0_" << r << ");\n";
                    s << "    const float PC0_" << r << " = ap->scale[grp] * cs0_" << r << ";\n";
                    s << "    const float PS0_" << r << " = ap->scale[grp] * sn0_" << r << ";\n";
                }
            }
            s << pc[pi].pre;
            // the part's k-independent values are computed once and serve every momentum of the chunk
            s << "    for (int kq = 0; kq < nkc; ++kq) {\n";
            s << "        const int ki = kb + kq;\n";
            // the momentum comes from the block's LDS copy (one broadcast ds_ load), where ap, the kernel's
            // private copy of its arguments, would cost a flat load and a full wait on every pass
            s << "        const float kk = kl[ki];\n";
            s << "        const int row = kq < ml ? kq * SPK1 : ml * SPK1 + (kq - ml) * 2;  // this momentum's stage rows\n";
            s << "        (void)ki;\n";
            indent(s, pc[pi].loop, "    ");
            indent(s, pc[pi].epi, "");
            if (!pc[pi].loopd.empty() || !pc[pi].epid.empty()) {
                s << "        if (kq < ml) {\n";
                indent(s, pc[pi].loopd, "        ");
                indent(s, pc[pi].epid, "    ");
                s << "        }\n";
            }
            s << "    }\n}\n";
        }
    }
    // small single-part value graphs (orders 1-3) are held to 5 waves per SIMD: order 3 otherwise takes 98
    // registers, 4 waves, and the fifth hides more of the transcendentals' latency
    const bool five = !split && NR == 1 && n <= 3;
    // floats of stage per wave: a kernel in parts stages a run-time chunk of a.kc momenta for one group,
    // SPK1 floats per lane for each of the first min(KD, kc) momenta (all kc when KD is 0), 2 for the others;
    // the host sizes the block's LDS by the same count
    const std::string sfw = split ? "(SFL * 64)" : "(16 * MST * 64)";
    s << "\nextern \"C\" __global__ void __launch_bounds__(256" << (five ? ", 5" : "") << ") KERNEL_NAME(const EvalArgs a) {";
    s << R"K(

    extern __shared__ __attribute__((aligned(16))) float smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
)K";
    if (split) {
        s << "    const int ML0 = KD ? min(KD, a.kc) : a.kc, SFL = ML0 * SPK1 + (a.kc - ML0) * 2;\n";
        // the external momenta, copied once per block into LDS for the parts (every thread reaches the barrier)
        s << "    __shared__ float kl_s[64];\n";
        s << "    if ((int)threadIdx.x < a.n_k) kl_s[threadIdx.x] = a.k[threadIdx.x];\n";
        s << "    __syncthreads();\n";
    }
    s << R"K(    float* stage = smem + wv * )K" << sfw << R"K(;
    double* tot = (double*)(smem + 4 * )K" << sfw << R"K() + wv * (2 * a.s_total);
    for (int i = lane; i < 2 * a.s_total; i += 64) tot[i] = 0.0;
    unsigned int nonfin = 0;
    const float MU = a.mu, BL = a.bl, BLMU = a.blmu, BETA = a.beta;
    const float* __restrict__ X = a.x;
    const long long ld = a.ld;
)K";
    for (int g = 0; g < n_groups; ++g) s << "    const float LAM" << g << " = a.lam[" << g << "];\n";
    s << R"K(    const long long ntiles = (a.n + 255) >> 8;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long s = tile * 256 + threadIdx.x;
        const bool valid = s < a.n;
        const long long si = valid ? s : a.n - 1;
        const float J = valid ? a.jac[si] : 0.0f;
)K";
    for (int j = 0; j < n; ++j)
        for (int e = 0; e < 3; ++e)
            s << "        const float q" << j << ax[e] << " = X[" << (3 * j + e) << " * ld + si];\n";
    for (int j = 1; j < n; ++j) {
        s << "        const float t" << j << " = X[" << (3 * n + j - 1) << " * ld + si];\n";
        s << "        const float tl" << j << " = t" << j << " * 1.44269504089f;\n";
    }
    for (int g = 0; g < n_groups && !split; ++g)
        for (int r : cls) {
            if (r == 0) {
                s << "        const float PC" << g << "_0 = a.scale[" << g << "];\n";
            } else {
                s << "        float sn" << g << "_" << r << ", cs" << g << "_" << r << ";\n";
                s << "        sincospif(t" << r << " * (2.0f * a.inv2beta), &sn" << g << "_" << r << ", &cs" << g << "_" << r
                  << ");\n";
                s << "        const float PC" << g << "_" << r << " = a.scale[" << g << "] * cs" << g << "_" << r << ";\n";
                s << "        const float PS" << g << "_" << r << " = a.scale[" << g << "] * sn" << g << "_" << r << ";\n";
            }
        }
    if (!split) {
        s << pc[0].pre;
        // slots whose weight is structurally zero: 0 * J is not finite exactly when J is not, counted once per
        // such slot and external momentum after the tile
        for (const auto& f : pc[0].fplain) zero_slots += f == "0.0f";
        if (zero_slots) s << "        const unsigned int jbad = (valid && !__builtin_isfinite(J)) ? 1u : 0u;\n";
        s << R"K(        float imp = 0.0f;
        for (int kb = 0; kb < a.n_k; kb += KC) {
            float impc = 0.0f, chk = 0.0f;  // this chunk's importance, and the sum of the other weights
            for (int kq = 0; kq < KC; ++kq) {
                const int ki = kb + kq;
                if (ki >= a.n_k) {
                    // past the last external momentum: empty stage slots and no graph work (uniform)
                    for (int sl = 0; sl < SPK; ++sl) stage[(kq * SPK + sl) * 64 + lane] = 0.0f;
                    continue;
                }
                const bool kv = true;
                const float kk = a.k[ki];
)K";
        indent(s, pc[0].loop, "            ");
        indent(s, pc[0].epi, "            ");
        // the staging of one (group, root, component) slot: weight f J into the stage, f into f_out
        auto stage_slot = [&](std::ostringstream& o, int g, int ro, int comp, bool zero, const std::string& pad) {
            const std::string fo = "if (a.f_out && valid) a.f_out[(((long long)(" + std::to_string(g * NR + ro) +
                                   ") * a.n_k + ki) * 2 + " + std::to_string(comp) + ") * a.n + s] = ";
            if (real_only && comp == 1) {
                o << pad << fo << "0.0f;\n";
                return;
            }
            const int slot = real_only ? g * NR + ro : (g * NR + ro) * 2 + comp;
            if (zero) {
                o << pad << "stage[(kq * SPK + " << slot << ") * 64 + lane] = 0.0f;\n";
                o << pad << fo << "0.0f;\n";
                return;
            }
            o << pad << "{\n";
            o << pad << "    const float w = " << (comp ? "FI" : "FR") << g << "_" << ro << ";  // f J\n";
            if (ro == 0)
                o << pad << "    impc += __builtin_fabsf(w);\n";
            else
                o << pad << "    chk += w; if (a.imp_roots > " << ro << ") impc += __builtin_fabsf(w);\n";
            o << pad << "    stage[(kq * SPK + " << slot << ") * 64 + lane] = w;\n";
            o << pad << "    " << fo << pc[0].fplain[(g * NR + ro) * 2 + comp] << ";\n";
            o << pad << "}\n";
        };
        for (int g = 0; g < n_groups; ++g)
            for (int comp = 0; comp < 2; ++comp) stage_slot(s, g, 0, comp, false, "                ");
        if (NR > 1) {
            // derivative roots: at every momentum (KD = 0) or at the first KD only (zeros elsewhere)
            const std::string pad = KD ? "                    " : "                ";
            if (KD) s << "                if (ki < KD) {\n";
            indent(s, pc[0].loopd, KD ? "                " : "            ");
            indent(s, pc[0].epid, KD ? "                " : "            ");
            for (int g = 0; g < n_groups; ++g)
                for (int ro = 1; ro < NR; ++ro)
                    for (int comp = 0; comp < 2; ++comp) stage_slot(s, g, ro, comp, false, pad);
            if (KD) {
                s << "                } else {\n";
                for (int g = 0; g < n_groups; ++g)
                    for (int ro = 1; ro < NR; ++ro)
                        for (int comp = 0; comp < 2; ++comp) stage_slot(s, g, ro, comp, true, pad);
                s << "                }\n";
            }
        }
        s << "            }\n";
    } else {
        // partitioned: for each chunk of a.kc external momenta and each lambda group, every part adds its
        // roots into the stage (its k-independent code runs once per chunk and group), then the group's
        // weights are formed, checked and folded
        s << "        float* cin = (float*)((double*)(smem + 4 * " << sfw << ") + 4 * 2 * a.s_total) + wv * "
          << ins.size() * 64 << " + lane;\n";
        for (size_t i = 0; i < ins.size(); ++i) s << "        cin[" << i * 64 << "] = " << ins[i] << ";\n";
        s << R"K(        float imp = 0.0f;
        for (int kb = 0; kb < a.n_k; kb += a.kc) {
            const int nkc = min(a.kc, a.n_k - kb);
            // momenta with derivative roots in this chunk (the first ml), and the staged slots: SPK1 per such
            // momentum, 2 (the value) per other
            const int ml = KD ? max(0, min(nkc, KD - kb)) : nkc;
            const int nsl = ml * SPK1 + (nkc - ml) * 2;
            for (int grp = 0; grp < NGRP; ++grp) {
                float impc = 0.0f, chk = 0.0f;  // this chunk's importance, and the sum of the other weights
                for (int i = 0; i < nsl; ++i) stage[i * 64 + lane] = 0.0f;
)K";
        for (size_t pi = 0; pi < pc.size(); ++pi)
            s << "                dmc_part_" << pi << "(&a, (const LdsF*)cin, (LdsF*)(stage + lane), (const LdsF*)kl_s, kb, nkc, grp, ml);\n";
        s << "                for (int kq = 0; kq < nkc; ++kq) {\n";
        s << "                    const int ki = kb + kq;\n";
        s << "                    const int row = kq < ml ? kq * SPK1 : ml * SPK1 + (kq - ml) * 2;\n";
        for (int ro = 0; ro < NR; ++ro)
            for (int comp = 0; comp < 2; ++comp) {
                const int slot = ro * 2 + comp;
                const std::string fo = "if (a.f_out && valid) a.f_out[(((long long)(grp * NROOT + " + std::to_string(ro) +
                                       ") * a.n_k + ki) * 2 + " + std::to_string(comp) + ") * a.n + s] = ";
                s << "                    " << (ro ? "if (kq < ml) {" : "{") << "\n";
                s << "                        const float f = stage[(row + " << slot << ") * 64 + lane];\n";
                s << "                        const float w = f * J;\n";
                if (ro == 0)
                    s << "                        impc += __builtin_fabsf(w);\n";
                else
                    s << "                        chk += w; if (a.imp_roots > " << ro << ") impc += __builtin_fabsf(w);\n";
                s << "                        stage[(row + " << slot << ") * 64 + lane] = w;\n";
                s << "                        " << fo << "f;\n";
                s << "                    }" << (ro ? " else {\n                        " + fo + "0.0f;\n                    }" : "")
                  << "\n";
            }
        s << "                }\n";
        s << R"K(                if (!__builtin_isfinite(impc + chk)) {
                    impc = 0.0f;
                    for (int sl = 0; sl < nsl; ++sl) {
                        float v = stage[sl * 64 + lane];
                        if (!__builtin_isfinite(v)) {
                            if (valid) nonfin += 1u;
                            v = 0.0f;
                            stage[sl * 64 + lane] = 0.0f;
                        }
                        const int slot = sl < ml * SPK1 ? sl % SPK1 : (sl - ml * SPK1) % 2;
                        if (slot < 2 * a.imp_roots) impc += __builtin_fabsf(v);
                    }
                }
                imp += impc;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int m = 0; 16 * m < nsl; ++m) {
                    const int sl = (lane >> 2) + 16 * m;
                    double s1 = 0.0, s2 = 0.0;
                    if (sl < nsl) {
                        const float4* src = (const float4*)(stage + sl * 64 + (lane & 3) * 16);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float4 v = src[j];
                            double d = (double)v.x; s1 += d; s2 = __builtin_fma(d, d, s2);
                            d = (double)v.y; s1 += d; s2 = __builtin_fma(d, d, s2);
                            d = (double)v.z; s1 += d; s2 = __builtin_fma(d, d, s2);
                            d = (double)v.w; s1 += d; s2 = __builtin_fma(d, d, s2);
                        }
                    }
                    s1 += __shfl_xor(s1, 1); s2 += __shfl_xor(s2, 1);
                    s1 += __shfl_xor(s1, 2); s2 += __shfl_xor(s2, 2);
                    // device slot order [k][group][root][comp]
                    const int kq = sl < ml * SPK1 ? sl / SPK1 : ml + (sl - ml * SPK1) / 2;
                    const int slot = sl < ml * SPK1 ? sl % SPK1 : (sl - ml * SPK1) % 2;
                    const int gs = (kb + kq) * SPK + grp * SPK1 + slot;
                    if ((lane & 3) == 0 && sl < nsl) { tot[2 * gs] += s1; tot[2 * gs + 1] += s2; }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (a.imp_out && valid) a.imp_out[s] = imp;
)K";
    }
    if (!split) {
    // a weight that is not finite makes the chunk's sums non-finite: only then (rarely, per lane) are this
    // lane's staged weights scanned, each non-finite one zeroed and counted (valid samples only), and the
    // chunk's importance recomputed
    const std::string imp_slot = real_only ? "(j % NROOT) < a.imp_roots" : "((j >> 1) % NROOT) < a.imp_roots";
    s << R"K(            if (!__builtin_isfinite(impc + chk)) {
                impc = 0.0f;
                for (int sl = 0; sl < SCH; ++sl) {
                    const int j = sl % SPK;
                    float v = stage[sl * 64 + lane];
                    if (!__builtin_isfinite(v)) {
                        if (valid) nonfin += 1u;
                        v = 0.0f;
                        stage[sl * 64 + lane] = 0.0f;
                    }
                    if ()K" << imp_slot << R"K() impc += __builtin_fabsf(v);
                }
            }
            imp += impc;
)K";
    s << R"K(            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int m = 0; m < MST; ++m) {
                const int sl = (lane >> 2) + 16 * m;
                const float4* src = (const float4*)(stage + sl * 64 + (lane & 3) * 16);
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 v = src[j];
                    double d = (double)v.x; s1 += d; s2 = __builtin_fma(d, d, s2);
                    d = (double)v.y; s1 += d; s2 = __builtin_fma(d, d, s2);
                    d = (double)v.z; s1 += d; s2 = __builtin_fma(d, d, s2);
                    d = (double)v.w; s1 += d; s2 = __builtin_fma(d, d, s2);
                }
                s1 += __shfl_xor(s1, 1); s2 += __shfl_xor(s2, 1);
                s1 += __shfl_xor(s1, 2); s2 += __shfl_xor(s2, 2);
)K";
    if (real_only)  // staged slot sl = (k - kb) SPK + j holds the real part of slot 2 j of momentum k
        s << "                const int gs = (kb + sl / SPK) * (2 * SPK) + 2 * (sl % SPK);\n";
    else
        s << "                const int gs = (kb / KC) * SCH + sl;\n";
    s << R"K(                if ((lane & 3) == 0 && sl < SCH && gs < a.s_total) { tot[2 * gs] += s1; tot[2 * gs + 1] += s2; }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (a.imp_out && valid) a.imp_out[s] = imp;
)K";
    }
    if (zero_slots) s << "        nonfin += jbad * (unsigned int)(a.n_k * " << zero_slots << ");\n";
    s << R"K(    }
    // fold the four waves in a fixed order into one FP64 partial per slot
    for (int o = 32; o > 0; o >>= 1) nonfin += __shfl_xor(nonfin, o);
    __shared__ unsigned int nf_w[4];
    if (lane == 0) nf_w[wv] = nonfin;
    __syncthreads();
    const double* t0 = (const double*)(smem + 4 * )K" << sfw << R"K();
    const int st2 = 2 * a.s_total;
    for (int i = threadIdx.x; i < st2; i += 256)
        a.partial[(long long)blockIdx.x * st2 + i] = ((t0[i] + t0[st2 + i]) + t0[2 * st2 + i]) + t0[3 * st2 + i];
    if (threadIdx.x == 0) a.nonfinite[blockIdx.x] = nf_w[0] + nf_w[1] + nf_w[2] + nf_w[3];
}
)K";
    if (stats) {
        *stats = CodeStats{};
        for (auto& p : pc)
            for (int i = 0; i < 4; ++i) {
                stats->sample[i] += p.cnt_pre[i];
                stats->k[i] += p.cnt_loop[i] + p.cnt_loopd[i];
                stats->k_deriv[i] += p.cnt_loopd[i];
            }
        for (int i = 0; i < 4; ++i) {
            stats->k[i] += epi_ops[i] + epi_ops_d[i];
            stats->k_deriv[i] += epi_ops_d[i];
        }
        stats->parts = (int)parts.size();
        // naive: every diagram as a plain product of its lines, every leaf evaluated per diagram
        for (auto& d : c.diagrams) {
            int ng = 0, nv = 0, neq = 0;
            for (auto& l : d.lines) {
                if (l.kind == 'G') {
                    ++ng;
                    if (l.src / 2 == l.dst / 2) ++neq;
                } else
                    ++nv;
            }
            // G: p^2 (3 fma-class) + energy (fma, exp2, add, rcp, sub) + leaf (mul, exp2, mul, select)
            // V: p^2 + add + rcp; product chain: (lines - 1) mul + 1 fma into the sum
            stats->naive[2] += (int64_t)(ng + nv) * 3 + ng;
            stats->naive[3] += (int64_t)ng * 3 - neq + nv;
            stats->naive[0] += (int64_t)ng * 3 + nv;
            stats->naive[1] += (int64_t)ng * 2 + (ng + nv - 1);
        }
    }
    return s.str();
}

}  // namespace dmc
