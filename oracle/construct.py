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

The fully irreducible vertex is taken as the bare interaction only: the first larger one (the envelope, four
interaction lines) enters a self-energy at order 5, so the construction is complete through order 4.

A fragment is a set of interaction lines (pairs of vertex ids, both ends at the line's time) and internal
propagators (a successor map); its legs are vertex ids.  A finished self-energy is turned into the permutation
representation of `diagrams` (line t joins vertices 2t and 2t + 1, the in-vertex is 0, sigma[out] = 0).
"""
from __future__ import annotations

import functools
import itertools

from . import diagrams as dg

_ids = itertools.count()


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
    if j == 0 and kind in ("full", "ph", "phbar", "pp"):
        # the bare interaction, direct (in1 and out1 at one end) and exchange (in1 and out2 at one end)
        x, y = _new(), _new()
        out.append((Frag([(x, y)]), x, y, x, y))
        x, y = _new(), _new()
        out.append((Frag([(x, y)]), x, y, y, x))
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
