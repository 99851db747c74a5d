// Building-block variables for the self-energy diagrams (Sec. II.C: eq. Dyson, eq. sigma_pq,
// eq. vertex3, eq. parquet_eqns, eq. phi_ph, eq. phi_phbar, eq. phi_pp).
//
// Every diagram of the canonical set is decomposed top-down by the equations the paper uses to
// build the set bottom-up:
//   Sigma(K) = V_q G(K - q) Gamma3(K - q -> K; q)      the interaction line at the in-vertex
//   G        = G0 Sigma G0 Sigma ... G0                 a dressed line: a chain of insertions
//   Gamma3   = bare vertex, or Gamma4 [G_{p+q} G_p]     the pair closes at the boson end
//   Gamma4   = I, or Gamma4 [G G] Gamma4_c              c in {ph, ph-bar, pp}, Gamma4_c irreducible in c
// Each building block takes its interaction lines (its time variables) and loop momenta from
// running counters in a fixed traversal, and writes its momenta in its own leg momenta.  Two
// diagrams that hold the same block at the same place of the decomposition then hold the same
// leaves, and the factoring of the diagram sum evaluates that block once for all of them.
//
// Rules of the decomposition (readings of the equations for Feynman diagrams with distinct legs):
//  * Sigma: the interaction line at the in-vertex a carries q from a to its other end a'; the
//    fermion leaving a runs through a chain into Gamma3's in-vertex; Gamma3's boson end is a'.
//    Gamma3 is bare when the chain enters a' and the fermion leaves the block there.
//  * Chains: with the block's own interaction line (Sigma), its boson end (Gamma3) or the channel's
//    right block (Gamma4) taken out, the propagators of a chain are cut lines; the piece between
//    two of them that holds none of the block's other legs is a self-energy insertion.
//  * Gamma4 legs: in1, in2 enter, out1, out2 leave.  Channels: two propagators separate
//    {in1,out1}|{in2,out2} (ph), {in1,out2}|{in2,out1} (ph-bar) or {in1,in2}|{out1,out2} (pp).  The
//    right block (the side without in1) is the smallest such side: it is irreducible in the channel,
//    and the left block is a full vertex.  In pp, the left block's out1 is the line the fermion
//    entering at in1 leaves it by.
//  * Momenta: a vertex block's external momentum enters at in1 and leaves at out1.  The loop momentum r
//    of a reducible vertex rides on the pair line that does not carry the external momentum across:
//    ph: L.out2 -> R.in1; ph-bar: R.out2 -> L.in2; pp: L.out2 -> R.in2.
//  * A fully irreducible vertex (one interaction line, or an envelope-like block) is labelled by a
//    breadth-first walk from in1 and routed on a spanning tree, chords taken in walk order.
#include "graph.hpp"

#include <algorithm>
#include <functional>
#include <memory>

namespace dmc {

namespace {

using MomV = std::vector<int>;  // coefficients over (q_0..q_{n-1}, k)

MomV operator+(const MomV& a, const MomV& b) {
    MomV r(a);
    for (size_t i = 0; i < r.size(); ++i) r[i] += b[i];
    return r;
}
MomV operator-(const MomV& a, const MomV& b) {
    MomV r(a);
    for (size_t i = 0; i < r.size(); ++i) r[i] -= b[i];
    return r;
}

struct Chain {
    std::vector<int> g0;  // the chain's propagators (source vertices), in fermion order from its start
    std::vector<struct Block*> ins;
};

struct Block {
    enum Kind { Sigma, Gamma3, Gamma4Bare, Gamma4Irr, Gamma4Red } kind = Sigma;
    std::vector<int> verts;
    int a = -1, b = -1, boson = -1;        // Sigma: in a, out b; Gamma3: in a, out b, boson end
    int in1 = -1, in2 = -1, out1 = -1, out2 = -1;
    int channel = -1;                      // 0 ph, 1 ph-bar, 2 pp
    bool bare3 = false;
    Chain c1, c2;                          // Sigma: c1 from a; Gamma3: c1 out of, c2 into the boson end;
                                           // Gamma4: c1 the pair line with r, c2 the other
    Block *g3 = nullptr, *left = nullptr, *right = nullptr;
};

struct Parser {
    const std::vector<int>& sg;
    int nv, n;
    std::vector<int> inv;
    std::vector<std::unique_ptr<Block>> pool;
    std::string err;

    explicit Parser(const std::vector<int>& s) : sg(s), nv((int)s.size()), n((int)s.size() / 2), inv(s.size(), -1) {
        for (int v = 0; v < nv; ++v) inv[s[v]] = v;
    }
    Block* make() {
        pool.push_back(std::make_unique<Block>());
        return pool.back().get();
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = m;
        return false;
    }

    // the sub-graph: a vertex set, with some propagators (by source vertex) and interaction lines off
    struct Sub {
        std::vector<char> in, g_off, v_off;
    };
    Sub sub(const std::vector<int>& verts) const {
        Sub s{std::vector<char>(nv, 0), std::vector<char>(nv, 0), std::vector<char>(n, 0)};
        for (int v : verts) s.in[v] = 1;
        return s;
    }
    bool internal_g(const Sub& s, int x) const {  // propagator x -> sg[x] inside the sub-graph
        return sg[x] != 0 && s.in[x] && s.in[sg[x]] && !s.g_off[x];
    }
    std::vector<char> component(const Sub& s, int start) const {
        std::vector<char> seen(nv, 0);
        std::vector<int> st{start};
        seen[start] = 1;
        while (!st.empty()) {
            const int v = st.back();
            st.pop_back();
            auto visit = [&](int w) {
                if (s.in[w] && !seen[w]) {
                    seen[w] = 1;
                    st.push_back(w);
                }
            };
            if (internal_g(s, v)) visit(sg[v]);
            if (v != 0 && internal_g(s, inv[v])) visit(inv[v]);
            if (!s.v_off[v / 2] && s.in[v ^ 1]) visit(v ^ 1);
        }
        return seen;
    }

    // A chain from the propagator `e` (source vertex), walked forward (e enters the chain's next
    // vertex) or backward (e leaves it).  Insertions are parsed and taken out of `s`; returns the
    // terminal vertex (-1 on error).
    int chain(Sub& s, int e, bool forward, const std::vector<int>& prot, Chain& ch) {
        ch.g0.push_back(e);
        for (;;) {
            const int cur = forward ? sg[e] : e;
            if (std::find(prot.begin(), prot.end(), cur) != prot.end()) return cur;
            Sub t = s;
            t.g_off[e] = 1;
            int found = -1, x = cur;
            std::vector<char> comp;
            for (int steps = 0; steps < nv; ++steps) {
                int line, nxt;
                if (forward) {
                    line = x;
                    if (!internal_g(t, line)) break;
                    nxt = sg[x];
                } else {
                    if (x == 0) break;
                    line = inv[x];
                    if (!internal_g(t, line)) break;
                    nxt = line;
                }
                Sub u = t;
                u.g_off[line] = 1;
                auto cc = component(u, cur);
                bool ok = !cc[nxt];
                for (int p : prot)
                    if (p >= 0 && cc[p]) ok = false;
                if (ok) {
                    found = line;
                    comp = cc;
                    break;
                }
                x = nxt;
            }
            if (found < 0) return cur;
            std::vector<int> xs;
            for (int v = 0; v < nv; ++v)
                if (comp[v]) xs.push_back(v);
            const int sin = forward ? cur : sg[found];
            const int sout = forward ? found : cur;
            Block* ins = sigma(xs, sin, sout);
            if (!ins) return -1;
            ch.ins.push_back(ins);
            for (int v : xs) s.in[v] = 0;
            ch.g0.push_back(found);
            e = found;
        }
    }

    Block* sigma(const std::vector<int>& verts, int a, int b) {
        Block* B = make();
        B->kind = Block::Sigma;
        B->verts = verts;
        B->a = a;
        B->b = b;
        const int ap = a ^ 1;
        Sub s = sub(verts);
        if (!s.in[ap]) return fail("sigma: the in-vertex's partner is outside the block"), nullptr;
        s.v_off[a / 2] = 1;
        s.in[a] = 0;
        if (sg[a] == 0 || !s.in[sg[a]]) return fail("sigma: no propagator out of the in-vertex"), nullptr;
        const int c = chain(s, a, true, {b, ap}, B->c1);
        if (c < 0) return nullptr;
        std::vector<int> rest;
        for (int v : verts)
            if (s.in[v]) rest.push_back(v);
        if (c == ap) {
            if (b != ap || rest.size() != 1) return fail("sigma: a chain into the boson end that does not end there"), nullptr;
            B->g3 = make();
            B->g3->kind = Block::Gamma3;
            B->g3->bare3 = true;
            B->g3->verts = rest;
            B->g3->a = B->g3->b = B->g3->boson = ap;
            return B;
        }
        B->g3 = gamma3(rest, c, b, ap);
        return B->g3 ? B : nullptr;
    }

    Block* gamma3(const std::vector<int>& verts, int c, int b, int bos) {
        Block* B = make();
        B->kind = Block::Gamma3;
        B->verts = verts;
        B->a = c;
        B->b = b;
        B->boson = bos;
        Sub s = sub(verts);
        s.in[bos] = 0;
        if (!s.in[sg[bos]] || inv[bos] < 0 || !s.in[inv[bos]]) return fail("gamma3: open boson end"), nullptr;
        const int in2 = chain(s, bos, true, {c, b}, B->c1);
        if (in2 < 0) return nullptr;
        const int out2 = chain(s, inv[bos], false, {c, b}, B->c2);
        if (out2 < 0) return nullptr;
        std::vector<int> rest;
        for (int v : verts)
            if (s.in[v]) rest.push_back(v);
        B->left = gamma4(rest, c, in2, b, out2);
        return B->left ? B : nullptr;
    }

    Block* gamma4(const std::vector<int>& verts, int in1, int in2, int out1, int out2) {
        Block* B = make();
        B->verts = verts;
        B->in1 = in1;
        B->in2 = in2;
        B->out1 = out1;
        B->out2 = out2;
        if (verts.size() == 2 && (verts[0] ^ 1) == verts[1]) {
            B->kind = Block::Gamma4Bare;
            return B;
        }
        Sub s = sub(verts);
        std::vector<int> gl;
        for (int x : verts)
            if (internal_g(s, x)) gl.push_back(x);
        // the channel cut with the smallest right side
        int best = -1, bch = -1, bl1 = -1, bl2 = -1;
        std::vector<char> bright;
        for (size_t i = 0; i < gl.size(); ++i)
            for (size_t j = i + 1; j < gl.size(); ++j) {
                Sub t = s;
                t.g_off[gl[i]] = t.g_off[gl[j]] = 1;
                auto L = component(t, in1);
                int other = -1;
                for (int v : verts)
                    if (!L[v]) {
                        other = v;
                        break;
                    }
                if (other < 0) continue;
                auto R = component(t, other);
                bool two = true;
                int nr = 0;
                for (int v : verts) {
                    if (!L[v] && !R[v]) two = false;
                    nr += R[v];
                }
                if (!two) continue;
                // both cut lines must join the two sides
                bool cross = true;
                for (int x : {gl[i], gl[j]})
                    if (L[x] == L[sg[x]]) cross = false;
                if (!cross) continue;
                int ch = -1;
                if (L[out1] && R[in2] && R[out2]) ch = 0;
                else if (L[out2] && R[in2] && R[out1]) ch = 1;
                else if (L[in2] && R[out1] && R[out2]) ch = 2;
                if (ch < 0) continue;
                if (bch >= 0 && ch != bch) return fail("gamma4: reducible in two channels"), nullptr;
                if (best < 0 || nr < best) {
                    best = nr;
                    bch = ch;
                    bl1 = gl[i];
                    bl2 = gl[j];
                    bright = R;
                }
            }
        if (bch < 0) {
            B->kind = Block::Gamma4Irr;
            return B;
        }
        B->kind = Block::Gamma4Red;
        B->channel = bch;
        std::vector<int> rv;
        for (int v : verts)
            if (bright[v]) rv.push_back(v);
        Sub w = s;
        for (int v : rv) w.in[v] = 0;
        // the left block's external legs
        std::vector<int> lprot = bch == 0 ? std::vector<int>{in1, out1}
                                 : bch == 1 ? std::vector<int>{in1, out2}
                                            : std::vector<int>{in1, in2};
        // R-side vertices of the cut lines
        int r_in[2] = {-1, -1}, r_out = -1, r_out_line = -1, l_term[2] = {-1, -1};
        Chain tmp[2];
        int k = 0;
        for (int x : {bl1, bl2}) {
            if (bright[x]) {  // leaves R: a forward chain into the left block
                r_out = x;
                r_out_line = k;
                l_term[k] = chain(w, x, true, lprot, tmp[k]);
            } else {          // enters R: a backward chain out of the left block
                r_in[k] = sg[x];
                l_term[k] = chain(w, x, false, lprot, tmp[k]);
            }
            if (l_term[k] < 0) return nullptr;
            ++k;
        }
        std::vector<int> lv;
        for (int v : verts)
            if (w.in[v]) lv.push_back(v);
        if (bch == 0 || bch == 1) {
            if (r_out < 0) return fail("gamma4: ph cut without a line out of the right block"), nullptr;
            const int ol = r_out_line, il = 1 - r_out_line;
            const int R_in1 = r_in[il], L_o = l_term[il], L_i2 = l_term[ol];
            if (bch == 0) {
                // L(in1, in2 = L_i2, out1, out2 = L_o), R(in1 = R_in1, in2, out1 = r_out, out2)
                B->left = gamma4(lv, in1, L_i2, out1, L_o);
                if (!B->left) return nullptr;
                B->right = gamma4(rv, R_in1, in2, r_out, out2);
                B->c1 = std::move(tmp[il]);   // L.out2 -> R.in1 carries r
                B->c2 = std::move(tmp[ol]);   // R.out1 -> L.in2
            } else {
                // L(in1, in2 = L_i2, out1 = L_o, out2), R(in1 = R_in1, in2, out1, out2 = r_out)
                B->left = gamma4(lv, in1, L_i2, L_o, out2);
                if (!B->left) return nullptr;
                B->right = gamma4(rv, R_in1, in2, out1, r_out);
                B->c1 = std::move(tmp[ol]);   // R.out2 -> L.in2 carries r
                B->c2 = std::move(tmp[il]);   // L.out1 -> R.in1
            }
        } else {
            // pp: both lines enter R.  L.out1 is where the fermion entering at in1 leaves L.
            std::vector<char> inl(nv, 0);
            for (int v : lv) inl[v] = 1;
            int x = in1;
            for (int steps = 0; steps < nv && sg[x] != 0 && inl[sg[x]]; ++steps) x = sg[x];
            int i1 = -1;
            for (int q = 0; q < 2; ++q)
                if (l_term[q] == x) i1 = q;
            if (i1 < 0) return fail("gamma4: pp pair not found from in1"), nullptr;
            const int i2 = 1 - i1;
            B->left = gamma4(lv, in1, in2, l_term[i1], l_term[i2]);
            if (!B->left) return nullptr;
            B->right = gamma4(rv, r_in[i1], r_in[i2], out1, out2);
            B->c1 = std::move(tmp[i2]);       // L.out2 -> R.in2 carries r
            B->c2 = std::move(tmp[i1]);       // L.out1 -> R.in1
        }
        return B->right ? B : nullptr;
    }
};

// Label and route the parsed blocks.
struct Assign {
    const Parser& P;
    int n;
    std::vector<int> lab;              // old vertex -> new vertex
    std::vector<MomV> gm;              // propagator momenta by old source vertex
    std::vector<MomV> vm;              // interaction momenta by old line, from the new even end to the odd one
    std::vector<char> gset, vset;
    int next_line = 0, next_loop = 0;
    std::string err;

    explicit Assign(const Parser& p)
        : P(p), n(p.n), lab(p.nv, -1), gm(p.nv), vm(p.n), gset(p.nv, 0), vset(p.n, 0) {}
    MomV zero() const { return MomV(n + 1, 0); }
    MomV unit(int j) const {
        MomV m = zero();
        m[j] = 1;
        return m;
    }
    bool fail(const std::string& m) {
        if (err.empty()) err = m;
        return false;
    }
    bool new_line(int first) {  // the interaction line of old vertex `first`; `first` becomes its even end
        if (lab[first] >= 0 || lab[first ^ 1] >= 0) return fail("vertex labelled twice");
        const int t = next_line++;
        lab[first] = 2 * t;
        lab[first ^ 1] = 2 * t + 1;
        return true;
    }
    bool set_g(int x, const MomV& m) {
        if (gset[x]) return fail("propagator routed twice");
        gset[x] = 1;
        gm[x] = m;
        return true;
    }
    bool set_v(int line, const MomV& m) {
        if (vset[line]) return fail("interaction routed twice");
        vset[line] = 1;
        vm[line] = m;
        return true;
    }
    bool chain(const Chain& c, const MomV& m) {
        for (int x : c.g0)
            if (!set_g(x, m)) return false;
        for (const Block* b : c.ins)
            if (!sigma(b, m)) return false;
        return true;
    }
    bool sigma(const Block* B, const MomV& K) {
        if (!new_line(B->a)) return false;
        const MomV q = unit(next_loop++);
        if (!set_v(B->a / 2, q)) return false;   // from a (the even end) to a'
        const MomV kc = K - q;
        if (!chain(B->c1, kc)) return false;
        return gamma3(B->g3, kc, K, q);
    }
    bool gamma3(const Block* B, const MomV& pin, const MomV& pout, const MomV& qb) {
        if (B->bare3) return true;
        const MomV p = unit(next_loop++);
        if (!gamma4(B->left, pin, p + qb, pout, p)) return false;
        if (!chain(B->c1, p + qb)) return false;
        return chain(B->c2, p);
    }
    bool gamma4(const Block* B, const MomV& P1, const MomV& P2, const MomV& P3, const MomV& P4) {
        switch (B->kind) {
            case Block::Gamma4Bare: {
                const int x = B->in1;
                if (!new_line(x)) return false;
                // what enters x by its legs flows to the other end
                MomV m = P1;
                if (B->out1 == x) m = m - P3;
                else if (B->out2 == x) m = m - P4;
                else return fail("bare vertex: in1 without an outgoing leg");
                return set_v(x / 2, m);
            }
            case Block::Gamma4Red: {
                const MomV r = unit(next_loop++);
                if (B->channel == 0) {
                    const MomV y = r + P3 - P1;
                    if (!gamma4(B->left, P1, y, P3, r) || !gamma4(B->right, r, P2, y, P4)) return false;
                    return chain(B->c1, r) && chain(B->c2, y);
                }
                if (B->channel == 1) {
                    const MomV x = r + P1 - P4;
                    if (!gamma4(B->left, P1, r, x, P4) || !gamma4(B->right, x, P2, P3, r)) return false;
                    return chain(B->c1, r) && chain(B->c2, x);
                }
                const MomV x = P1 + P2 - r;
                if (!gamma4(B->left, P1, P2, x, r) || !gamma4(B->right, x, r, P3, P4)) return false;
                return chain(B->c1, r) && chain(B->c2, x);
            }
            case Block::Gamma4Irr:
                return irreducible(B, P1, P2, P3, P4);
            default:
                return fail("not a vertex block");
        }
    }
    // breadth-first labelling from in1, chords in walk order, spanning-tree flow of the leg momenta
    bool irreducible(const Block* B, const MomV& P1, const MomV& P2, const MomV& P3, const MomV& P4) {
        const auto& sg = P.sg;
        const auto& inv = P.inv;
        std::vector<char> in(P.nv, 0);
        for (int v : B->verts) in[v] = 1;
        auto ing = [&](int x) { return sg[x] != 0 && in[x] && in[sg[x]]; };
        std::vector<int> order{B->in1};
        std::vector<char> seen(P.nv, 0);
        seen[B->in1] = 1;
        for (size_t j = 0; j < order.size(); ++j) {
            const int v = order[j];
            if (lab[v] < 0 && lab[v ^ 1] < 0 && !new_line(v)) return false;
            for (int w : {ing(v) ? sg[v] : -1, in[v ^ 1] ? (v ^ 1) : -1, (v != 0 && ing(inv[v])) ? inv[v] : -1})
                if (w >= 0 && !seen[w]) {
                    seen[w] = 1;
                    order.push_back(w);
                }
        }
        if (order.size() != B->verts.size()) return fail("irreducible block not connected");
        // lines in walk order: propagators by new source label, then interaction lines by index
        struct L {
            bool g;
            int key, a, b;  // old id (source vertex or line), ends in the reference direction
        };
        std::vector<L> ls;
        for (int v : B->verts)
            if (ing(v)) ls.push_back({true, v, v, sg[v]});
        std::sort(ls.begin(), ls.end(), [&](const L& x, const L& y) { return lab[x.a] < lab[y.a]; });
        std::vector<L> vl;
        for (int v : B->verts)
            if (lab[v] % 2 == 0) vl.push_back({false, v / 2, v, v ^ 1});
        std::sort(vl.begin(), vl.end(), [&](const L& x, const L& y) { return lab[x.a] < lab[y.a]; });
        ls.insert(ls.end(), vl.begin(), vl.end());
        const int nvb = (int)B->verts.size(), nl = (int)ls.size(), nch = nl - nvb + 1;
        std::vector<char> tree(nl, 1);
        auto conn = [&]() {
            std::vector<char> s(P.nv, 0);
            std::vector<int> st{B->in1};
            s[B->in1] = 1;
            int cnt = 1;
            while (!st.empty()) {
                const int v = st.back();
                st.pop_back();
                for (int i = 0; i < nl; ++i) {
                    if (!tree[i]) continue;
                    int w = ls[i].a == v ? ls[i].b : ls[i].b == v ? ls[i].a : -1;
                    if (w >= 0 && !s[w]) {
                        s[w] = 1;
                        ++cnt;
                        st.push_back(w);
                    }
                }
            }
            return cnt == nvb;
        };
        std::vector<MomV> lm(nl, zero());
        int got = 0;
        std::vector<int> chords;
        for (int i = 0; i < nl && got < nch; ++i) {
            tree[i] = 0;
            if (conn()) {
                chords.push_back(i);
                ++got;
            } else {
                tree[i] = 1;
            }
        }
        if (got != nch) return fail("irreducible block: chords");
        // tree paths
        auto tree_path = [&](int from, int to, const MomV& m) {
            // add m along the tree path from -> to
            std::vector<int> pv(P.nv, -2), pe(P.nv, -1);
            std::vector<int> st{from};
            pv[from] = -1;
            while (!st.empty()) {
                const int v = st.back();
                st.pop_back();
                for (int i = 0; i < nl; ++i) {
                    if (!tree[i]) continue;
                    int w = ls[i].a == v ? ls[i].b : ls[i].b == v ? ls[i].a : -1;
                    if (w >= 0 && pv[w] == -2) {
                        pv[w] = v;
                        pe[w] = i;
                        st.push_back(w);
                    }
                }
            }
            for (int v = to; v != from; v = pv[v]) {
                const int i = pe[v], u = pv[v];
                lm[i] = (ls[i].a == u) ? lm[i] + m : lm[i] - m;
            }
        };
        for (int i : chords) {
            const MomV q = unit(next_loop++);
            lm[i] = lm[i] + q;
            tree_path(ls[i].b, ls[i].a, q);  // back along the tree from the chord's head to its tail
        }
        // the leg momenta: each enters at its vertex and leaves at out1's / out2's vertex; send
        // everything entering through the tree to in1's vertex, then out to the outgoing legs
        tree_path(B->in2, B->in1, P2);
        tree_path(B->in1, B->out1, P3);
        tree_path(B->in1, B->out2, P4);
        (void)P1;
        for (int i = 0; i < nl; ++i) {
            if (ls[i].g) {
                if (!set_g(ls[i].key, lm[i])) return false;
            } else if (!set_v(ls[i].key, lm[i])) {
                return false;
            }
        }
        return true;
    }
};

}  // namespace

bool relabel_building_blocks(const Diagram& d, Diagram& out, std::string& err) {
    const int n = d.order, nv = 2 * n;
    Parser P(d.sigma);
    std::vector<int> all(nv);
    for (int v = 0; v < nv; ++v) all[v] = v;
    Block* top = P.sigma(all, 0, d.out_vertex);
    if (!top) {
        err = P.err;
        return false;
    }
    Assign A(P);
    MomV K = A.zero();
    K[n] = 1;
    if (!A.sigma(top, K)) {
        err = A.err;
        return false;
    }
    for (int v = 0; v < nv; ++v)
        if (A.lab[v] < 0) {
            err = "vertex left unlabelled";
            return false;
        }
    for (int x = 0; x < nv; ++x)
        if (d.sigma[x] != 0 && !A.gset[x]) {
            err = "propagator left unrouted";
            return false;
        }
    for (int i = 0; i < n; ++i)
        if (!A.vset[i]) {
            err = "interaction left unrouted";
            return false;
        }
    if (A.next_loop != n || A.next_line != n) {
        err = "loop or line count";
        return false;
    }
    out = Diagram{};
    out.order = n;
    out.sigma.assign(nv, -1);
    for (int v = 0; v < nv; ++v) out.sigma[A.lab[v]] = A.lab[d.sigma[v]];
    out.out_vertex = A.lab[d.out_vertex];
    out.n_fermion_loops = d.n_fermion_loops;
    out.weight = d.weight;
    std::vector<int> old_of(nv);
    for (int v = 0; v < nv; ++v) old_of[A.lab[v]] = v;
    for (int nvx = 0; nvx < nv; ++nvx) {
        if (out.sigma[nvx] == 0) continue;
        Line ln;
        ln.kind = 'G';
        ln.src = nvx;
        ln.dst = out.sigma[nvx];
        ln.mom.fill(0);
        const MomV& m = A.gm[old_of[nvx]];
        for (int c = 0; c <= n; ++c) ln.mom[c] = m[c];
        out.lines.push_back(ln);
    }
    for (int t = 0; t < n; ++t) {
        Line ln;
        ln.kind = 'V';
        ln.src = 2 * t;
        ln.dst = 2 * t + 1;
        ln.mom.fill(0);
        const MomV& m = A.vm[old_of[2 * t] / 2];  // stored from the new even end to the odd end
        for (int c = 0; c <= n; ++c) ln.mom[c] = m[c];
        out.lines.push_back(ln);
    }
    // momentum conservation at every vertex, k in at 0 and out at the out-vertex
    std::vector<MomV> net(nv, MomV(n + 1, 0));
    for (auto& ln : out.lines)
        for (int c = 0; c <= n; ++c) {
            net[ln.src][c] -= ln.mom[c];
            net[ln.dst][c] += ln.mom[c];
        }
    net[0][n] += 1;
    net[out.out_vertex][n] -= 1;
    for (auto& r : net)
        for (int x : r)
            if (x != 0) {
                err = "momentum not conserved";
                return false;
            }
    return true;
}

}  // namespace dmc
