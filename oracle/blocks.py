"""Building-block integration variables of a self-energy diagram -- TEST INFRASTRUCTURE (oracle).

Only the tests, the smoke check and the bench's CPU-baseline leg use this module.

What it follows
---------------
Sec. II.C builds the self-energy from its building blocks: eq. sigma_pq writes Sigma = V G Gamma3,
eq. Dyson writes the dressed line G as G0 chained with self-energy insertions, eq. vertex3 writes
Gamma3 as the bare vertex or Gamma4 closed by a propagator pair, and eq. parquet_eqns with eqs.
phi_ph, phi_phbar, phi_pp writes Gamma4 as a fully irreducible vertex or a channel-reducible one,
Gamma4 [G G] Gamma4_c with the right factor irreducible in the channel c.  Every diagram of the
brute-force set is decomposed by these equations, top-down, and each block takes its interaction
lines (time variables) and loop momenta from running counters, its momenta written in its own leg
momenta.  The external momentum k is then put on the diagram's shortest path (the rule of
`diagrams.external_path`): the k column of a routing is any unit flow from the in-vertex to the
out-vertex, independent of the loop columns.

The decomposition is a convention shared with the library (written twice, like the routing rule of
`diagrams.route`): the blocks, their order and the variable each takes.
  * Sigma (in-vertex a, out-vertex b): the interaction line at a is the block's first line and
    carries the block's first loop momentum q from a to its partner a'.  The fermion leaving a
    carries K - q through a chain into Gamma3, whose boson end is a'.  Gamma3 is bare when that
    chain enters a' and the fermion leaves the block there.
  * A chain is walked along the fermion: with the block's own interaction line (Sigma), its boson
    end (Gamma3) or the right block (Gamma4) removed, a stretch closed off by two propagators that
    holds none of the block's other legs is a self-energy insertion.
  * Gamma3 (not bare): its loop momentum p; Gamma4 with legs in1 = Gamma3's in-vertex (K - q),
    in2 = the end of the chain leaving a' (p + q), out1 = b (K), out2 = the start of the chain into
    a' (p); then the chain out of a', then the chain into a'.
  * Gamma4: the channels ph {in1,out1}|{in2,out2}, ph-bar {in1,out2}|{in2,out1}, pp {in1,in2}|{out1,out2}
    are cuts by two propagators; the right block is the smallest side without in1.  Its loop momentum
    r; then the left block, the right block, and the two pair chains (ph: L.out2 -> R.in1 with r, then
    R.out1 -> L.in2; ph-bar: R.out2 -> L.in2 with r, then L.out1 -> R.in1; pp: L.out2 -> R.in2 with r,
    then L.out1 -> R.in1, where L.out1 is where the fermion entering L at in1 leaves it).
  * Fully irreducible Gamma4: one interaction line (its first end the in1 vertex, carrying what
    enters there), or a larger block labelled by a breadth-first walk from in1 (out-propagator,
    partner, in-propagator; a line is numbered when its first vertex is taken from the queue),
    chords by reverse delete over its propagators (by new source label) then its interaction lines,
    leg momenta sent in2 -> in1 -> out1 and in1 -> out2 along the spanning tree.
"""
from __future__ import annotations

from . import diagrams as dg


class _Graph:
    def __init__(self, sigma):
        self.sg = list(sigma)
        self.nv = len(sigma)
        self.n = self.nv // 2
        self.inv = [0] * self.nv
        for v, w in enumerate(self.sg):
            self.inv[w] = v

    def g_inside(self, verts, g_off, x):
        """The propagator x -> sigma[x] is internal to `verts` and not taken out."""
        return self.sg[x] != 0 and x in verts and self.sg[x] in verts and x not in g_off

    def reach(self, verts, g_off, v_off, start):
        seen = {start}
        todo = [start]
        while todo:
            v = todo.pop()
            nbrs = []
            if self.g_inside(verts, g_off, v):
                nbrs.append(self.sg[v])
            if v != 0 and self.g_inside(verts, g_off, self.inv[v]):
                nbrs.append(self.inv[v])
            if v // 2 not in v_off and (v ^ 1) in verts:
                nbrs.append(v ^ 1)
            for w in nbrs:
                if w not in seen:
                    seen.add(w)
                    todo.append(w)
        return seen


def _walk_chain(g, verts, v_off, e, forward, prot):
    """Chain from propagator e (its source vertex).  `verts` loses the insertions' vertices.
    Returns (terminal vertex, chain propagators, insertion blocks), in walk order."""
    lines, inserts = [e], []
    while True:
        cur = g.sg[e] if forward else e
        if cur in prot:
            return cur, lines, inserts
        off = {e}
        found, piece = None, None
        x = cur
        for _ in range(g.nv):
            if forward:
                line, nxt = x, g.sg[x]
            else:
                if x == 0:
                    break
                line = nxt = g.inv[x]
            if not g.g_inside(verts, off, line):
                break
            comp = g.reach(verts, off | {line}, v_off, cur)
            if nxt not in comp and not any(p in comp for p in prot):
                found, piece = line, comp
                break
            x = nxt
        if found is None:
            return cur, lines, inserts
        s_in, s_out = (cur, found) if forward else (g.sg[found], cur)
        inserts.append(_sigma(g, sorted(piece), s_in, s_out))
        verts -= piece
        lines.append(found)
        e = found


def _sigma(g, verts, a, b):
    ap = a ^ 1
    work = set(verts) - {a}
    c, lines, ins = _walk_chain(g, work, {a // 2}, a, True, {b, ap})
    blk = {"kind": "sigma", "a": a, "b": b, "chain": (lines, ins)}
    if c == ap:
        assert b == ap and work == {ap}, "chain into the boson end that does not end the block"
        blk["g3"] = None
        return blk
    blk["g3"] = _gamma3(g, sorted(work), c, b, ap)
    return blk


def _gamma3(g, verts, c, b, bos):
    work = set(verts) - {bos}
    in2, l1, i1 = _walk_chain(g, work, set(), bos, True, {c, b})
    out2, l2, i2 = _walk_chain(g, work, set(), g.inv[bos], False, {c, b})
    return {"kind": "gamma3", "out_chain": (l1, i1), "in_chain": (l2, i2),
            "g4": _gamma4(g, sorted(work), c, in2, b, out2)}


def _gamma4(g, verts, in1, in2, out1, out2):
    vs = set(verts)
    if len(verts) == 2 and verts[0] ^ 1 == verts[1]:
        return {"kind": "bare", "in1": in1, "out1": out1, "out2": out2}
    gl = [x for x in verts if g.g_inside(vs, set(), x)]
    best = None
    for i in range(len(gl)):
        for j in range(i + 1, len(gl)):
            off = {gl[i], gl[j]}
            left = g.reach(vs, off, set(), in1)
            rest = vs - left
            if not rest:
                continue
            right = g.reach(vs, off, set(), min(rest))
            if left | right != vs:
                continue
            if any((x in left) == (g.sg[x] in left) for x in off):
                continue
            if out1 in left and {in2, out2} <= right:
                ch = "ph"
            elif out2 in left and {in2, out1} <= right:
                ch = "phbar"
            elif in2 in left and {out1, out2} <= right:
                ch = "pp"
            else:
                continue
            assert best is None or best[0] == ch, "reducible in two channels"
            if best is None or len(right) < len(best[1]):
                best = (ch, right, (gl[i], gl[j]))
    if best is None:
        return {"kind": "irr", "verts": list(verts), "in1": in1, "in2": in2, "out1": out1, "out2": out2}
    ch, right, cut = best
    work = vs - right
    lprot = {"ph": {in1, out1}, "phbar": {in1, out2}, "pp": {in1, in2}}[ch]
    chains = []
    for x in cut:
        if x in right:      # leaves R: the chain runs forward into L
            term, lines, ins = _walk_chain(g, work, set(), x, True, lprot)
            chains.append(("out", x, term, (lines, ins)))
        else:               # enters R at sigma[x]: the chain runs backward into L
            term, lines, ins = _walk_chain(g, work, set(), x, False, lprot)
            chains.append(("in", g.sg[x], term, (lines, ins)))
    lv, rv = sorted(work), sorted(right)
    blk = {"kind": "red", "channel": ch}
    if ch in ("ph", "phbar"):
        (_, r_out, l_in2, c_out), = [c for c in chains if c[0] == "out"]
        (_, r_in1, l_out, c_in), = [c for c in chains if c[0] == "in"]
        if ch == "ph":
            blk["left"] = _gamma4(g, lv, in1, l_in2, out1, l_out)
            blk["right"] = _gamma4(g, rv, r_in1, in2, r_out, out2)
            blk["chains"] = (c_in, c_out)          # L.out2 -> R.in1 carries r
        else:
            blk["left"] = _gamma4(g, lv, in1, l_in2, l_out, out2)
            blk["right"] = _gamma4(g, rv, r_in1, in2, out1, r_out)
            blk["chains"] = (c_out, c_in)          # R.out2 -> L.in2 carries r
        return blk
    # pp: the fermion entering L at in1 leaves it at L.out1
    x = in1
    while g.sg[x] != 0 and g.sg[x] in work:
        x = g.sg[x]
    first = [c for c in chains if c[2] == x]
    second = [c for c in chains if c[2] != x]
    assert len(first) == 1 and len(second) == 1, "pp pair"
    (_, r1, l1, c1), (_, r2, l2, c2) = first[0], second[0]
    blk["left"] = _gamma4(g, lv, in1, in2, l1, l2)
    blk["right"] = _gamma4(g, rv, r1, r2, out1, out2)
    blk["chains"] = (c2, c1)                        # L.out2 -> R.in2 carries r
    return blk


class _Labels:
    """Numbers interaction lines and loop momenta block by block; momenta as coefficient lists over
    (q_0..q_{n-1}, k)."""

    def __init__(self, g):
        self.g = g
        self.n = g.n
        self.lab = {}
        self.gmom = {}
        self.vmom = {}       # by old line index, from the new even end to the odd end
        self.line = 0
        self.loop = 0

    def vec(self, j=None):
        v = [0] * (self.n + 1)
        if j is not None:
            v[j] = 1
        return v

    def new_loop(self):
        self.loop += 1
        return self.vec(self.loop - 1)

    def new_line(self, first):
        assert first not in self.lab and (first ^ 1) not in self.lab
        self.lab[first] = 2 * self.line
        self.lab[first ^ 1] = 2 * self.line + 1
        self.line += 1

    def set_g(self, x, m):
        assert x not in self.gmom
        self.gmom[x] = list(m)

    def set_v(self, line, m):
        assert line not in self.vmom
        self.vmom[line] = list(m)

    def chain(self, ch, m):
        lines, ins = ch
        for x in lines:
            self.set_g(x, m)
        for blk in ins:
            self.sigma(blk, m)

    def sigma(self, blk, K):
        self.new_line(blk["a"])
        q = self.new_loop()
        self.set_v(blk["a"] // 2, q)
        kc = _sub(K, q)
        self.chain(blk["chain"], kc)
        if blk["g3"] is not None:
            g3 = blk["g3"]
            p = self.new_loop()
            self.gamma4(g3["g4"], kc, _add(p, q), K, p)
            self.chain(g3["out_chain"], _add(p, q))
            self.chain(g3["in_chain"], p)

    def gamma4(self, blk, P1, P2, P3, P4):
        kind = blk["kind"]
        if kind == "bare":
            x = blk["in1"]
            self.new_line(x)
            if blk["out1"] == x:
                self.set_v(x // 2, _sub(P1, P3))
            else:
                assert blk["out2"] == x
                self.set_v(x // 2, _sub(P1, P4))
        elif kind == "red":
            r = self.new_loop()
            ch = blk["channel"]
            c_r, c_o = blk["chains"]
            if ch == "ph":
                o = _add(r, _sub(P3, P1))
                self.gamma4(blk["left"], P1, o, P3, r)
                self.gamma4(blk["right"], r, P2, o, P4)
            elif ch == "phbar":
                o = _add(r, _sub(P1, P4))
                self.gamma4(blk["left"], P1, r, o, P4)
                self.gamma4(blk["right"], o, P2, P3, r)
            else:
                o = _sub(_add(P1, P2), r)
                self.gamma4(blk["left"], P1, P2, o, r)
                self.gamma4(blk["right"], o, r, P3, P4)
            self.chain(c_r, r)
            self.chain(c_o, o)
        else:
            self.irreducible(blk, P2, P3, P4)

    def irreducible(self, blk, P2, P3, P4):
        g = self.g
        vs = set(blk["verts"])
        order, seen = [blk["in1"]], {blk["in1"]}
        j = 0
        while j < len(order):
            v = order[j]
            j += 1
            if v not in self.lab and (v ^ 1) not in self.lab:
                self.new_line(v)
            nb = [g.sg[v] if g.g_inside(vs, set(), v) else None,
                  (v ^ 1) if (v ^ 1) in vs else None,
                  g.inv[v] if v != 0 and g.g_inside(vs, set(), g.inv[v]) else None]
            for w in nb:
                if w is not None and w not in seen:
                    seen.add(w)
                    order.append(w)
        assert seen == vs
        glines = sorted((x for x in vs if g.g_inside(vs, set(), x)), key=lambda x: self.lab[x])
        vlines = sorted((x for x in vs if self.lab[x] % 2 == 0), key=lambda x: self.lab[x])
        ls = [("G", x, x, g.sg[x]) for x in glines] + [("V", x // 2, x, x ^ 1) for x in vlines]
        tree = [True] * len(ls)

        def connected():
            adj = {v: [] for v in vs}
            for i, (_, _, a, b) in enumerate(ls):
                if tree[i]:
                    adj[a].append(b)
                    adj[b].append(a)
            got, todo = {blk["in1"]}, [blk["in1"]]
            while todo:
                for w in adj[todo.pop()]:
                    if w not in got:
                        got.add(w)
                        todo.append(w)
            return got == vs

        n_chords = len(ls) - len(vs) + 1
        chords = []
        for i in range(len(ls)):
            if len(chords) == n_chords:
                break
            tree[i] = False
            if connected():
                chords.append(i)
            else:
                tree[i] = True
        assert len(chords) == n_chords
        mom = [self.vec() for _ in ls]

        def along_tree(src, dst, m):
            # the unique tree path src -> dst, adding m in the direction of travel
            prev = {src: None}
            todo = [src]
            while todo:
                v = todo.pop()
                for i, (_, _, a, b) in enumerate(ls):
                    if not tree[i] or v not in (a, b):
                        continue
                    w = b if a == v else a
                    if w not in prev:
                        prev[w] = (v, i)
                        todo.append(w)
            v = dst
            while prev[v] is not None:
                u, i = prev[v]
                s = 1 if ls[i][2] == u else -1
                mom[i] = [x + s * y for x, y in zip(mom[i], m)]
                v = u

        for i in chords:
            q = self.new_loop()
            mom[i] = _add(mom[i], q)
            along_tree(ls[i][3], ls[i][2], q)
        along_tree(blk["in2"], blk["in1"], P2)
        along_tree(blk["in1"], blk["out1"], P3)
        along_tree(blk["in1"], blk["out2"], P4)
        for (kind, key, _, _), m in zip(ls, mom):
            if kind == "G":
                self.set_g(key, m)
            else:
                self.set_v(key, m)


def _add(a, b):
    return [x + y for x, y in zip(a, b)]


def _sub(a, b):
    return [x - y for x, y in zip(a, b)]


def decompose(d: dg.Diagram):
    """The block tree of a canonical diagram (nested dicts; see the module notes)."""
    g = _Graph(d.sigma)
    return _sigma(g, list(range(g.nv)), 0, d.out_vertex)


def relabel(d: dg.Diagram) -> dg.Diagram:
    """The diagram d (canonical labelling) with building-block interaction lines and loop momenta, k on
    the shortest path."""
    return relabelling(d)[0]


def relabelling(d: dg.Diagram):
    """(relabelled diagram, {old vertex: new vertex})."""
    g = _Graph(d.sigma)
    n = g.n
    top = _sigma(g, list(range(g.nv)), 0, d.out_vertex)
    L = _Labels(g)
    L.sigma(top, L.vec(n))
    assert L.line == n and L.loop == n and len(L.lab) == g.nv
    lab = L.lab
    sigma = [0] * g.nv
    for v in range(g.nv):
        sigma[lab[v]] = lab[g.sg[v]]
    out = sigma.index(0)
    old = {lab[v]: v for v in range(g.nv)}
    lines = []
    for v in range(g.nv):
        if sigma[v] != 0:
            lines.append(dg.Line("G", v, sigma[v], tuple(L.gmom[old[v]])))
    for t in range(n):
        lines.append(dg.Line("V", 2 * t, 2 * t + 1, tuple(L.vmom[old[2 * t] // 2])))
    # k on the shortest path from the in-vertex to the out-vertex
    fe, ve = dg._edges(sigma)
    path = dg.external_path(g.nv, fe + ve, out)
    moms = [list(ln.mom[:n]) + [0] for ln in lines]
    for idx, sgn in path:
        moms[idx][n] += sgn
    lines = [dg.Line(ln.kind, ln.src, ln.dst, tuple(m)) for ln, m in zip(lines, moms)]
    return dg.Diagram(sigma=tuple(sigma), order=n, out_vertex=out, n_loops_f=d.n_loops_f, weight=d.weight,
                      lines=lines, chords=[], k_path=[i for i, _ in path]), dict(lab)


def block_diagrams(diagrams):
    """Relabel a routed canonical diagram list (same order)."""
    return [relabel(d) for d in diagrams]
