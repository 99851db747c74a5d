"""Bottom-up construction of the self-energy diagrams from their building blocks -- TEST INFRASTRUCTURE (oracle).

Only the tests use this module.

What it follows
---------------
Sec. II.C builds the diagrams of order N from lower-order pieces: eq. sigma_pq (Sigma = V G Gamma3), eq. Dyson
(a dressed line is G0 chained with self-energy insertions), eq. vertex3 (Gamma3 is the bare vertex, or Gamma4
closed by a pair of dressed lines) and eq. parquet_eqns with eqs. phi_ph, phi_phbar, phi_pp (Gamma4 is a fully
irreducible vertex or a channel-reducible one, Gamma4 [G G] Gamma4_c with the right factor irreducible in the
channel).  Here the pieces are explicit Feynman-diagram fragments with distinct legs, combined by those equations
with the rules of the library's building-block variables (the channel cuts, and in the pp channel the left
block's out1 being where the fermion entering at in1 leaves it), so every diagram comes out once and keeps its own
sign (the zeta and 1/2 of the antisymmetrised equations do not appear).

The fully irreducible vertices come from a brute force over four-point topologies (`irreducible_vertices`):
the bare interaction, none with two or three lines, the envelopes with four.  Through four lines they make the
construction complete through order 5; at order 6 the five-line ones would be needed as well.

A fragment is a set of interaction lines (pairs of vertex ids, both ends at the line's time) and internal
propagators (a successor map); its legs are vertex ids.  A finished self-energy is turned into the permutation
representation of `diagrams` (line t joins vertices 2t and 2t + 1, the in-vertex is 0, sigma[out] = 0).
"""
from __future__ import annotations

import functools
import itertools

from . import diagrams as dg

_ids = itertools.count()

# fully irreducible four-point vertices are taken through this many interaction lines: the construction is then
# complete through order MAX_IRREDUCIBLE_LINES + 1
MAX_IRREDUCIBLE_LINES = 5


def _new():
    return next(_ids)


class Frag:
    __slots__ = ("vl", "succ")

    def __init__(self, vl=(), succ=None):
        self.vl = list(vl)
        self.succ = dict(succ or {})

    def join(self, *others):
        f = Frag(self.vl, self.succ)
        for o in others:
            f.vl += o.vl
            f.succ.update(o.succ)
        return f

    def renamed(self):
        """A copy with fresh vertex ids, and the renaming."""
        ren = {}

        def r(v):
            if v not in ren:
                ren[v] = _new()
            return ren[v]
        f = Frag([(r(a), r(b)) for a, b in self.vl], {r(a): r(b) for a, b in self.succ.items()})
        return f, r


def _compositions(m):
    """Ordered tuples of positive integers summing to m (m = 0: the empty tuple)."""
    if m == 0:
        return [()]
    out = []
    for first in range(1, m + 1):
        for rest in _compositions(m - first):
            out.append((first,) + rest)
    return out


def chains(m, src, dst):
    """Dressed lines of m interaction lines from vertex src to vertex dst (eq. Dyson): G0, then self-energy
    insertions joined by G0, in every order and every choice of insertion."""
    out = []
    for comp in _compositions(m):
        for pieces in itertools.product(*[sigma(k) for k in comp]):
            f = Frag()
            prev = src
            for frag, a, b in pieces:
                g, r = frag.renamed()
                f = f.join(g)
                f.succ[prev] = r(a)
                prev = r(b)
            f.succ[prev] = dst
            out.append(f)
    return out


@functools.lru_cache(maxsize=None)
def sigma(N):
    """Self-energies of N interaction lines (eq. sigma_pq): [(fragment, in-vertex, out-vertex)]."""
    out = []
    for m in range(N):
        i = N - 1 - m
        for g3, c, b, bos in gamma3(i):
            g, r = g3.renamed()
            a = _new()
            ap = r(bos)
            for ch in chains(m, a, r(c)):
                f = g.join(ch)
                f.vl.append((a, ap))
                out.append((f, a, r(b)))
    return tuple(out)


@functools.lru_cache(maxsize=None)
def gamma3(N):
    """Three-point vertices with N interaction lines besides the boson's (eq. vertex3): [(fragment, fermion in,
    fermion out, boson end)].  N = 0: the bare vertex (one vertex, in = out = boson end)."""
    if N == 0:
        v = _new()
        return ((Frag(), v, v, v),)
    out = []
    for j in range(N):                       # Gamma4 with j + 1 interaction lines
        M = N - 1 - j
        for g4, in1, in2, out1, out2 in gamma4(j, "full"):
            g, r = g4.renamed()
            bos = _new()
            for m1 in range(M + 1):
                for c1 in chains(m1, bos, r(in2)):
                    for c2 in chains(M - m1, r(out2), bos):
                        out.append((g.join(c1, c2), r(in1), r(out1), bos))
    return tuple(out)


def _exits_at(f, start, want):
    """The fermion entering at `start` leaves the fragment at vertex `want`."""
    v = start
    while v in f.succ:
        v = f.succ[v]
    return v == want


@functools.lru_cache(maxsize=None)
def gamma4(j, kind):
    """Four-point vertices with j + 1 interaction lines: [(fragment, in1, in2, out1, out2)].  kind "full" is
    eq. parquet_eqns (I + the three channels); "ph", "phbar", "pp" are the vertices irreducible in that channel
    (I + the other two)."""
    out = []
    if j + 1 <= MAX_IRREDUCIBLE_LINES:
        # the fully irreducible vertices (the bare interaction in its direct and exchange forms, none with two or
        # three lines, the envelopes with four), found by brute force
        out += list(irreducible_vertices(j + 1))
    channels = [c for c in ("ph", "phbar", "pp") if kind == "full" or c != kind]
    for c in channels:
        out += _reducible(j, c)
    return tuple(out)


@functools.lru_cache(maxsize=None)
def _reducible(j, c):
    """Gamma4 [G G] Gamma4_c with j + 1 interaction lines in all (eqs. phi_ph, phi_phbar, phi_pp)."""
    out = []
    total = j + 1
    for jl in range(total):
        for jr in range(total):
            M = total - (jl + 1) - (jr + 1)
            if M < 0:
                continue
            for L in gamma4(jl, "full"):
                fl, l1, l2, lo1, lo2 = L
                if c == "pp" and not _exits_at(fl, l1, lo1):
                    continue
                for R in gamma4(jr, c):
                    gl, rl = fl.renamed()
                    gr, rr = R[0].renamed()
                    r1, r2, ro1, ro2 = (rr(v) for v in R[1:])
                    L1, L2, LO1, LO2 = (rl(v) for v in (l1, l2, lo1, lo2))
                    for m1 in range(M + 1):
                        if c == "ph":      # L.out2 -> R.in1, R.out1 -> L.in2
                            pairs, legs = ((LO2, r1), (ro1, L2)), (L1, r2, LO1, ro2)
                        elif c == "phbar":  # L.out1 -> R.in1, R.out2 -> L.in2
                            pairs, legs = ((LO1, r1), (ro2, L2)), (L1, r2, ro1, LO2)
                        else:              # L.out1 -> R.in1, L.out2 -> R.in2
                            pairs, legs = ((LO1, r1), (LO2, r2)), (L1, L2, ro1, ro2)
                        for ca in chains(m1, *pairs[0]):
                            for cb in chains(M - m1, *pairs[1]):
                                out.append((gl.join(gr, ca, cb),) + legs)
    return tuple(out)


def to_sigma(frag, a, b):
    """The permutation representation: the in-vertex a's line is line 0 with a = 0, other lines in order of
    discovery; propagator out of the out-vertex closes onto 0."""
    partner = {}
    for x, y in frag.vl:
        partner[x], partner[y] = y, x
    lab = {a: 0, partner[a]: 1}
    nxt = 1
    for x, y in frag.vl:
        if x not in lab:
            lab[x], lab[y] = 2 * nxt, 2 * nxt + 1
            nxt += 1
    n = len(frag.vl)
    sig = [None] * (2 * n)
    for s, t in frag.succ.items():
        sig[lab[s]] = lab[t]
    sig[lab[b]] = 0
    assert all(v is not None for v in sig) and sorted(sig) == list(range(2 * n))
    return tuple(sig)


def sigma_topologies(N):
    """The canonical forms of the constructed order-N self-energies, with multiplicity."""
    out = {}
    for frag, a, b in sigma(N):
        c = dg.canonical(to_sigma(frag, a, b))
        out[c] = out.get(c, 0) + 1
    return out


def _four_point_key(sg, nv):
    """Canonical key of a four-point topology: nodes 0..nv-1 are vertices (line t = 2t, 2t + 1), node nv closes
    out1 -> in1 and node nv + 1 closes out2 -> in2 (sg is the successor map on nv + 2 nodes).  Breadth-first
    relabelling from in1's vertex (out-propagator, partner, in-propagator), each line's first-found end even."""
    P1, P2 = nv, nv + 1
    pred = [0] * (nv + 2)
    for v, w in enumerate(sg):
        pred[w] = v
    lab, order = {}, [sg[P1]]
    seen = {sg[P1]}
    nxt = 0
    j = 0
    while j < len(order):
        v = order[j]
        j += 1
        if v not in lab and (v ^ 1) not in lab:
            lab[v], lab[v ^ 1] = 2 * nxt, 2 * nxt + 1
            nxt += 1
        for w in (sg[v] if sg[v] < nv else None, v ^ 1, pred[v] if pred[v] < nv else None):
            if w is not None and w not in seen:
                seen.add(w)
                order.append(w)
    if len(lab) != nv:
        return None                                   # not connected
    name = lambda w: lab[w] if w < nv else ("o1" if w == P1 else "o2")
    out = [None] * nv
    for v in range(nv):
        out[lab[v]] = name(sg[v])
    return tuple(out) + (lab[sg[P2]],)


def _irreducible_ok(sg, nv):
    """Amputated (no propagator bridge), no tadpole (no interaction-line bridge with a leg-free side) and
    irreducible in the three channels (no two propagators separate {in1,out1}|{in2,out2}, {in1,out2}|{in2,out1}
    or {in1,in2}|{out1,out2})."""
    P1, P2 = nv, nv + 1
    pred = [0] * (nv + 2)
    for v, w in enumerate(sg):
        pred[w] = v
    legs = {"in1": sg[P1], "in2": sg[P2], "out1": pred[P1], "out2": pred[P2]}
    props = [v for v in range(nv) if sg[v] < nv]

    def comp(start, off_g, off_v):
        got, todo = {start}, [start]
        while todo:
            v = todo.pop()
            nb = []
            if sg[v] < nv and v not in off_g:
                nb.append(sg[v])
            if pred[v] < nv and pred[v] not in off_g:
                nb.append(pred[v])
            if v // 2 not in off_v:
                nb.append(v ^ 1)
            for w in nb:
                if w not in got:
                    got.add(w)
                    todo.append(w)
        return got

    for x in props:                                     # propagator bridges: an insertion on a leg
        if len(comp(0, {x}, set())) != nv:
            return False
    for t in range(nv // 2):                            # interaction-line bridges with a leg-free side
        c = comp(2 * t, set(), {t})
        if len(c) != nv:
            side = c if not any(l in c for l in legs.values()) else set(range(nv)) - c
            if not any(l in side for l in legs.values()):
                return False
    for i in range(len(props)):
        for k in range(i + 1, len(props)):
            c = comp(legs["in1"], {props[i], props[k]}, set())
            if len(c) == nv:
                continue
            inside = {name for name, v in legs.items() if v in c}
            if inside in ({"in1", "out1"}, {"in1", "out2"}, {"in1", "in2"}):
                rest = set(range(nv)) - c
                if len(comp(next(iter(rest)), {props[i], props[k]}, set()) | c) == nv:
                    return False
    return True


def _four_point_maps(lines):
    """Successor maps of connected four-point topologies with `lines` interaction lines, in1 entering vertex 0:
    the vertices are visited in label order and the propagator leaving the visited vertex enters a labelled vertex
    not yet entered (never vertex 0, in1's), opens the next line (whose ends take the next two labels) or leaves
    by out1 or out2; in2 then enters the one vertex left without an incoming propagator.  Every connected topology
    comes out at least once (in the labelling in which a breadth-first walk along out-propagators and partners
    from in1's vertex meets the lines in order); duplicates are removed by the canonical key."""
    nv = 2 * lines
    P1, P2 = nv, nv + 1
    sg = [None] * (nv + 2)
    entered = [False] * nv

    def rec(j, labelled, outs):
        if j == labelled:
            if labelled == nv and outs == 3:
                free = [v for v in range(1, nv) if not entered[v]]
                if len(free) == 1:
                    full = list(sg)
                    full[P1], full[P2] = 0, free[0]
                    yield full
            return
        for w in range(1, labelled):
            if not entered[w]:
                entered[w] = True
                sg[j] = w
                yield from rec(j + 1, labelled, outs)
                entered[w] = False
        if labelled < nv:
            entered[labelled] = True
            sg[j] = labelled
            yield from rec(j + 1, labelled + 2, outs)
            entered[labelled] = False
        for o, bit in ((P1, 1), (P2, 2)):
            if not outs & bit:
                sg[j] = o
                yield from rec(j + 1, labelled, outs | bit)
        sg[j] = None

    yield from rec(0, 2, 0)


@functools.lru_cache(maxsize=None)
def irreducible_vertices(lines):
    """The fully irreducible four-point topologies with `lines` interaction lines and distinct legs (connected,
    amputated, tadpole free, irreducible in the three channels): [(fragment, in1, in2, out1, out2)]."""
    nv = 2 * lines
    P1, P2 = nv, nv + 1
    keys = {}
    for sg in _four_point_maps(lines):
        key = _four_point_key(sg, nv)
        if key is None or key in keys:
            continue
        keys[key] = sg if _irreducible_ok(sg, nv) else None
    out = []
    for sg in keys.values():
        if sg is None:
            continue
        ids = [_new() for _ in range(nv)]
        pred = {w: v for v, w in enumerate(sg)}
        f = Frag([(ids[2 * t], ids[2 * t + 1]) for t in range(lines)],
                 {ids[v]: ids[sg[v]] for v in range(nv) if sg[v] < nv})
        out.append((f, ids[sg[P1]], ids[sg[P2]], ids[pred[P1]], ids[pred[P2]]))
    return tuple(out)
