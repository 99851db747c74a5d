// Bottom-up construction of the self-energy diagrams (Sec. II.C: eq. sigma_pq, eq. Dyson, eq. vertex3,
// eq. parquet_eqns, eq. phi_ph, eq. phi_phbar, eq. phi_pp).
//
// The order-N self-energies are built from lower-order pieces, each an explicit Feynman-diagram fragment with
// distinct legs:
//   Sigma^(N)  = V  G^(m)  Gamma3^(N-1-m)              the interaction line at the in-vertex, a dressed line
//   G^(m)      = G0 Sigma G0 Sigma ... G0                insertions in every order (eq. Dyson)
//   Gamma3^(i) = bare vertex (i = 0), or Gamma4^(j) [G^(m1) G^(m2)] with j + 1 + m1 + m2 = i
//   Gamma4^(j) = I^(j) + sum_c Gamma4 [G G] Gamma4_c     c in {ph, ph-bar, pp}, Gamma4_c irreducible in c
// with the channels of the building-block variables (ph: L.out2 -> R.in1, R.out1 -> L.in2; ph-bar: L.out1 ->
// R.in1, R.out2 -> L.in2; pp: L.out1 -> R.in1, L.out2 -> R.in2 with L's in1 fermion leaving by L.out1), so that
// every diagram comes out once and keeps its own sign (the zeta and 1/2 of the antisymmetrised equations do not
// appear).  The fully irreducible vertices I (j + 1 interaction lines, distinct legs) come from an orderly
// generation of connected four-point topologies kept when amputated, tadpole free and irreducible in the three
// channels.  Every finished self-energy is brought to the canonical labelling (breadth-first from the in-vertex).
#include "graph.hpp"

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <memory>
#include <set>

namespace dmc {

namespace {

// A fragment: vertices 0..nv-1, interaction lines (pairs), internal propagators (src, dst).
struct Frag {
    int nv = 0;
    std::vector<std::array<int, 2>> vl;
    std::vector<std::array<int, 2>> g;
};

// `add` appended to `host` with its ids shifted; returns the shift.
int append(Frag& host, const Frag& add) {
    const int off = host.nv;
    host.nv += add.nv;
    for (auto l : add.vl) host.vl.push_back({l[0] + off, l[1] + off});
    for (auto p : add.g) host.g.push_back({p[0] + off, p[1] + off});
    return off;
}

struct Sig {
    Frag f;
    int a, b;
};
struct G3 {
    Frag f;
    int in, out, bos;
};
struct G4 {
    Frag f;
    int in1, in2, out1, out2;
};

class Builder {
public:
    explicit Builder(int max_order) : maxn_(max_order) {}

    const std::vector<Sig>& sigma(int N) {
        auto it = sig_.find(N);
        if (it != sig_.end()) return it->second;
        std::vector<Sig> out;
        for (int m = 0; m < N; ++m) {
            const int i = N - 1 - m;
            for (const G3& g3 : gamma3(i)) {
                for_chains(m, [&](const std::vector<const Sig*>& pieces) {
                    Sig s;
                    s.f = g3.f;
                    const int a = s.f.nv++;
                    s.f.vl.push_back({a, g3.bos});
                    link_chain(s.f, a, g3.in, pieces);
                    s.a = a;
                    s.b = g3.out;
                    out.push_back(std::move(s));
                });
            }
        }
        return sig_[N] = std::move(out);
    }

    const std::vector<G3>& gamma3(int N) {
        auto it = g3_.find(N);
        if (it != g3_.end()) return it->second;
        std::vector<G3> out;
        if (N == 0) {
            G3 g;
            g.f.nv = 1;
            g.in = g.out = g.bos = 0;
            out.push_back(g);
        }
        for (int j = 0; j < N; ++j) {  // Gamma4 with j + 1 lines
            const int M = N - 1 - j;
            for (const G4& v : gamma4(j, 0)) {
                for (int m1 = 0; m1 <= M; ++m1)
                    for_chains(m1, [&](const std::vector<const Sig*>& p1) {
                        for_chains(M - m1, [&](const std::vector<const Sig*>& p2) {
                            G3 g;
                            g.f = v.f;
                            const int bos = g.f.nv++;
                            link_chain(g.f, bos, v.in2, p1);
                            link_chain(g.f, v.out2, bos, p2);
                            g.in = v.in1;
                            g.out = v.out1;
                            g.bos = bos;
                            out.push_back(std::move(g));
                        });
                    });
            }
        }
        return g3_[N] = std::move(out);
    }

    // kind 0: the full vertex; 1 ph, 2 ph-bar, 3 pp: irreducible in that channel
    const std::vector<G4>& gamma4(int j, int kind) {
        const auto key = std::make_pair(j, kind);
        auto it = g4_.find(key);
        if (it != g4_.end()) return it->second;
        std::vector<G4> out = irreducible(j + 1);
        for (int c = 1; c <= 3; ++c) {
            if (kind != 0 && c == kind) continue;
            const auto& r = reducible(j, c);
            out.insert(out.end(), r.begin(), r.end());
        }
        return g4_[key] = std::move(out);
    }

private:
    int maxn_;
    std::map<int, std::vector<Sig>> sig_;
    std::map<int, std::vector<G3>> g3_;
    std::map<std::pair<int, int>, std::vector<G4>> g4_, red_;
    std::map<int, std::vector<G4>> irr_;

    // calls fn with every ordered choice of self-energy insertions totalling m lines
    void for_chains(int m, const std::function<void(const std::vector<const Sig*>&)>& fn) {
        std::vector<const Sig*> cur;
        std::function<void(int)> rec = [&](int left) {
            if (left == 0) {
                fn(cur);
                return;
            }
            for (int k = 1; k <= left; ++k)
                for (const Sig& s : sigma(k)) {
                    cur.push_back(&s);
                    rec(left - k);
                    cur.pop_back();
                }
        };
        rec(m);
    }

    // propagators src -> insertion 1 -> ... -> dst
    static void link_chain(Frag& f, int src, int dst, const std::vector<const Sig*>& pieces) {
        int prev = src;
        for (const Sig* s : pieces) {
            const int off = append(f, s->f);
            f.g.push_back({prev, s->a + off});
            prev = s->b + off;
        }
        f.g.push_back({prev, dst});
    }

    const std::vector<G4>& reducible(int j, int c) {
        const auto key = std::make_pair(j, c);
        auto it = red_.find(key);
        if (it != red_.end()) return it->second;
        std::vector<G4> out;
        const int total = j + 1;
        for (int jl = 0; jl < total; ++jl)
            for (int jr = 0; jr < total; ++jr) {
                const int M = total - (jl + 1) - (jr + 1);
                if (M < 0) continue;
                for (const G4& L : gamma4(jl, 0)) {
                    if (c == 3 && !exits_at(L.f, L.in1, L.out1)) continue;
                    for (const G4& R : gamma4(jr, c)) {
                        for (int m1 = 0; m1 <= M; ++m1)
                            for_chains(m1, [&](const std::vector<const Sig*>& p1) {
                                for_chains(M - m1, [&](const std::vector<const Sig*>& p2) {
                                    G4 v;
                                    v.f = L.f;
                                    const int o = append(v.f, R.f);
                                    const int r1 = R.in1 + o, r2 = R.in2 + o, ro1 = R.out1 + o, ro2 = R.out2 + o;
                                    if (c == 1) {  // ph
                                        link_chain(v.f, L.out2, r1, p1);
                                        link_chain(v.f, ro1, L.in2, p2);
                                        v.in1 = L.in1, v.in2 = r2, v.out1 = L.out1, v.out2 = ro2;
                                    } else if (c == 2) {  // ph-bar
                                        link_chain(v.f, L.out1, r1, p1);
                                        link_chain(v.f, ro2, L.in2, p2);
                                        v.in1 = L.in1, v.in2 = r2, v.out1 = ro1, v.out2 = L.out2;
                                    } else {  // pp
                                        link_chain(v.f, L.out1, r1, p1);
                                        link_chain(v.f, L.out2, r2, p2);
                                        v.in1 = L.in1, v.in2 = L.in2, v.out1 = ro1, v.out2 = ro2;
                                    }
                                    out.push_back(std::move(v));
                                });
                            });
                    }
                }
            }
        return red_[key] = std::move(out);
    }

    static bool exits_at(const Frag& f, int start, int want) {
        std::vector<int> nxt(f.nv, -1);
        for (auto p : f.g) nxt[p[0]] = p[1];
        int v = start;
        for (int s = 0; s <= f.nv && nxt[v] >= 0; ++s) v = nxt[v];
        return v == want;
    }

    const std::vector<G4>& irreducible(int lines);
};

// ---- fully irreducible four-point vertices by orderly generation -------------------------------------------
// Nodes 0..nv-1 are vertices (line t = 2t, 2t+1); node nv closes out1 -> in1, nv + 1 closes out2 -> in2.

std::vector<int> four_point_key(const std::vector<int>& sg, int nv) {
    const int P1 = nv, P2 = nv + 1;
    std::vector<int> pred(nv + 2, -1);
    for (int v = 0; v < nv + 2; ++v) pred[sg[v]] = v;
    std::vector<int> lab(nv, -1), order{sg[P1]};
    std::vector<char> seen(nv, 0);
    seen[sg[P1]] = 1;
    int nxt = 0;
    for (size_t j = 0; j < order.size(); ++j) {
        const int v = order[j];
        if (lab[v] < 0 && lab[v ^ 1] < 0) {
            lab[v] = 2 * nxt;
            lab[v ^ 1] = 2 * nxt + 1;
            ++nxt;
        }
        for (int w : {sg[v] < nv ? sg[v] : -1, v ^ 1, pred[v] < nv ? pred[v] : -1})
            if (w >= 0 && !seen[w]) {
                seen[w] = 1;
                order.push_back(w);
            }
    }
    if ((int)order.size() != nv) return {};
    std::vector<int> key(nv + 1);
    for (int v = 0; v < nv; ++v) key[lab[v]] = sg[v] < nv ? lab[sg[v]] : (sg[v] == P1 ? -1 : -2);
    key[nv] = lab[sg[P2]];
    return key;
}

bool irreducible_ok(const std::vector<int>& sg, int nv) {
    const int P1 = nv, P2 = nv + 1;
    std::vector<int> pred(nv + 2, -1);
    for (int v = 0; v < nv + 2; ++v) pred[sg[v]] = v;
    const int legs[4] = {sg[P1], sg[P2], pred[P1], pred[P2]};  // in1, in2, out1, out2
    std::vector<int> props;
    for (int v = 0; v < nv; ++v)
        if (sg[v] < nv) props.push_back(v);
    auto comp = [&](int start, int g1, int g2, int voff) {
        std::vector<char> got(nv, 0);
        std::vector<int> st{start};
        got[start] = 1;
        while (!st.empty()) {
            const int v = st.back();
            st.pop_back();
            int nb[3] = {-1, -1, -1};
            if (sg[v] < nv && v != g1 && v != g2) nb[0] = sg[v];
            if (pred[v] < nv && pred[v] != g1 && pred[v] != g2) nb[1] = pred[v];
            if (v / 2 != voff) nb[2] = v ^ 1;
            for (int w : nb)
                if (w >= 0 && !got[w]) {
                    got[w] = 1;
                    st.push_back(w);
                }
        }
        return got;
    };
    auto count = [&](const std::vector<char>& c) { return (int)std::count(c.begin(), c.end(), 1); };
    for (int x : props)  // a propagator bridge is an insertion on a leg
        if (count(comp(0, x, -1, -1)) != nv) return false;
    for (int t = 0; t < nv / 2; ++t) {  // an interaction-line bridge with a leg-free side is a tadpole
        auto c = comp(2 * t, -1, -1, t);
        if (count(c) == nv) continue;
        bool in_c = false, out_c = false;
        for (int l : legs) (c[l] ? in_c : out_c) = true;
        if (!in_c || !out_c) return false;
    }
    for (size_t i = 0; i < props.size(); ++i)
        for (size_t k = i + 1; k < props.size(); ++k) {
            auto c = comp(legs[0], props[i], props[k], -1);
            if (count(c) == nv) continue;
            // legs on in1's side: {in1,out1} ph, {in1,out2} ph-bar, {in1,in2} pp
            const bool i2 = c[legs[1]], o1 = c[legs[2]], o2 = c[legs[3]];
            if (i2 + o1 + o2 != 1) continue;
            int other = -1;
            for (int v = 0; v < nv; ++v)
                if (!c[v]) other = v;
            auto d = comp(other, props[i], props[k], -1);
            if (count(c) + count(d) == nv) return false;
        }
    return true;
}

const std::vector<G4>& Builder::irreducible(int lines) {
    auto it = irr_.find(lines);
    if (it != irr_.end()) return it->second;
    const int nv = 2 * lines, P1 = nv, P2 = nv + 1;
    std::set<std::vector<int>> seen;
    std::vector<G4> out;
    std::vector<int> sg(nv + 2, -1);
    std::vector<char> entered(nv, 0);
    std::function<void(int, int, int)> rec = [&](int j, int labelled, int outs) {
        if (j == labelled) {
            if (labelled != nv || outs != 3) return;
            int free = -1, nfree = 0;
            for (int v = 1; v < nv; ++v)
                if (!entered[v]) free = v, ++nfree;
            if (nfree != 1) return;
            std::vector<int> full = sg;
            full[P1] = 0;
            full[P2] = free;
            auto key = four_point_key(full, nv);
            if (key.empty() || !seen.insert(key).second) return;
            if (!irreducible_ok(full, nv)) return;
            G4 v;
            v.f.nv = nv;
            for (int t = 0; t < lines; ++t) v.f.vl.push_back({2 * t, 2 * t + 1});
            for (int x = 0; x < nv; ++x)
                if (full[x] < nv) v.f.g.push_back({x, full[x]});
            for (int x = 0; x < nv; ++x) {
                if (full[x] == P1) v.out1 = x;
                if (full[x] == P2) v.out2 = x;
            }
            v.in1 = 0;
            v.in2 = free;
            out.push_back(std::move(v));
            return;
        }
        for (int w = 1; w < labelled; ++w)
            if (!entered[w]) {
                entered[w] = 1;
                sg[j] = w;
                rec(j + 1, labelled, outs);
                entered[w] = 0;
            }
        if (labelled < nv) {
            entered[labelled] = 1;
            sg[j] = labelled;
            rec(j + 1, labelled + 2, outs);
            entered[labelled] = 0;
        }
        for (int o = 0; o < 2; ++o)
            if (!(outs & (1 << o))) {
                sg[j] = o ? P2 : P1;
                rec(j + 1, labelled, outs | (1 << o));
            }
        sg[j] = -1;
    };
    if (lines <= maxn_) rec(0, 2, 0);
    return irr_[lines] = std::move(out);
}

// the permutation representation of a finished self-energy, canonical (breadth-first from the in-vertex a)
std::vector<int> canonical_sigma(const Sig& s) {
    const Frag& f = s.f;
    std::vector<int> partner(f.nv, -1), nxt(f.nv, -1);
    for (auto l : f.vl) partner[l[0]] = l[1], partner[l[1]] = l[0];
    for (auto p : f.g) nxt[p[0]] = p[1];
    nxt[s.b] = s.a;  // the external legs close the loop through the in-vertex
    std::vector<int> lab(f.nv, -1), order{s.a, partner[s.a]};
    lab[s.a] = 0;
    lab[partner[s.a]] = 1;
    int next_label = 2;
    for (size_t j = 0; j < order.size(); ++j) {
        const int w = nxt[order[j]];
        if (lab[w] < 0) {
            lab[w] = next_label;
            lab[partner[w]] = next_label + 1;
            next_label += 2;
            order.push_back(w);
            order.push_back(partner[w]);
        }
    }
    std::vector<int> sig(f.nv);
    for (int v = 0; v < f.nv; ++v) sig[lab[v]] = lab[nxt[v]];
    return sig;
}

}  // namespace

bool construct_sigma(int n, std::vector<std::vector<int>>& out, std::string& err) {
    if (n < 1 || n > kMaxOrder) {
        err = "order must be in 1..6";
        return false;
    }
    Builder b(n);
    std::map<std::vector<int>, int> count;
    for (const Sig& s : b.sigma(n)) {
        if ((int)s.f.vl.size() != n || s.f.nv != 2 * n) {
            err = "construction: a diagram of the wrong order";
            return false;
        }
        ++count[canonical_sigma(s)];
    }
    out.clear();
    for (auto& [sig, c] : count) {
        if (c != 1) {
            err = "construction: a diagram built more than once";
            return false;
        }
        out.push_back(sig);
    }
    return true;
}

}  // namespace dmc
