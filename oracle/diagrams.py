"""Oracle diagram enumerator: brute force over Wick contractions (test infrastructure).

What it follows
---------------
* The n-th order self-energy is a sum over all diagram topologies with n instantaneous
  interaction lines and 2n vertices (paper, Sec. II.A, eq. sigma_integration).
* The UEG action drops the q = 0 interaction (paper, Sec. VI.A, eq. ueg_action), so every
  diagram in which an interaction line is forced to carry zero momentum (a Hartree tadpole)
  is excluded.
* A self-energy is one-particle irreducible: cutting one internal propagator must not split it
  (this is what makes the Dyson relation, eq. Dyson, a unique decomposition).

Representation (a reading; the paper draws diagrams but prints no data format)
------------------------------------------------------------------------------
Interaction line i joins vertices 2i and 2i+1; both sit at time tau_i and tau_0 = 0.
A labelled contraction is a permutation sigma of the 2n vertices: the propagator leaving
vertex v enters vertex sigma[v].  The incoming external leg enters vertex 0; the vertex o
with sigma[o] == 0 is the out-vertex and the "line" o -> 0 stands for the amputated external
legs.  F = (number of cycles of sigma) - 1 closed fermion loops.

This module enumerates ALL (2n)! permutations and tests each one with a plain graph search,
which is slow on purpose and shares nothing with the library's generator.  Each topology is
reduced to a canonical labelling by a breadth-first relabelling that starts at the in-vertex;
the routing puts the external momentum on a short path of chords and the other loop momenta on
a reverse-delete spanning tree over the canonical labels.  Both rules are stated in the
functions below; they are the agreed naming of variables (a data convention), not arithmetic of
the method.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field


def partner(v: int) -> int:
    return v ^ 1


def n_cycles(sigma) -> int:
    seen = [False] * len(sigma)
    c = 0
    for s in range(len(sigma)):
        if not seen[s]:
            c += 1
            v = s
            while not seen[v]:
                seen[v] = True
                v = sigma[v]
    return c


def _edges(sigma):
    """Internal edges: ('f', v, sigma[v]) for every propagator except the external o->0,
    then ('v', 2i, 2i+1) for every interaction line."""
    n2 = len(sigma)
    o = sigma.index(0)
    fe = [("f", v, sigma[v]) for v in range(n2) if v != o]
    ve = [("v", 2 * i, 2 * i + 1) for i in range(n2 // 2)]
    return fe, ve


def _connected(n_vertices, edges) -> bool:
    adj = [[] for _ in range(n_vertices)]
    for _, a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    stack = [0]
    while stack:
        v = stack.pop()
        for w in adj[v]:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return len(seen) == n_vertices


def is_connected(sigma) -> bool:
    fe, ve = _edges(sigma)
    return _connected(len(sigma), fe + ve)


def bridges(sigma):
    """Edges whose removal disconnects the internal graph (brute force, one search per edge)."""
    fe, ve = _edges(sigma)
    allE = fe + ve
    out = []
    for i, e in enumerate(allE):
        rest = allE[:i] + allE[i + 1:]
        if not _connected(len(sigma), rest):
            out.append(e)
    return out


def is_sigma_diagram(sigma) -> bool:
    """Connected, no interaction line forced to q = 0, one-particle irreducible.

    An interaction-line bridge separates a piece with no external leg, so momentum
    conservation forces q = 0 through it (tadpole, excluded by q != 0 in eq. ueg_action).
    A propagator bridge lies on the open path in -> out and cutting it splits the diagram
    into two pieces that each hold one external leg (one-particle reducible)."""
    if not is_connected(sigma):
        return False
    return len(bridges(sigma)) == 0


def is_green_diagram(sigma) -> bool:
    """Connected Green's-function diagram without tadpoles (propagator bridges allowed)."""
    if not is_connected(sigma):
        return False
    return all(e[0] != "v" for e in bridges(sigma))


def canonical(sigma):
    """Breadth-first relabelling from the in-vertex.

    Vertex 0 keeps label 0 and its partner label 1.  Labelled vertices are visited in label
    order; when the propagator leaving the visited vertex enters a vertex with no label yet,
    that vertex gets the next even label 2m and its partner 2m+1.  The result depends only on
    the topology (the in-vertex is fixed and the graph is connected)."""
    n2 = len(sigma)
    new = {0: 0, 1: 1}
    order = [0, 1]
    nxt = 1
    j = 0
    while j < len(order):
        v = order[j]
        w = sigma[v]
        if w not in new:
            new[w] = 2 * nxt
            new[partner(w)] = 2 * nxt + 1
            order += [w, partner(w)]
            nxt += 1
        j += 1
    assert len(new) == n2
    out = [0] * n2
    for v in range(n2):
        out[new[v]] = new[sigma[v]]
    return tuple(out)


def enumerate_labelled(n: int, pred=is_sigma_diagram):
    """All labelled permutations of 2n vertices accepted by `pred` (brute force)."""
    for sigma in itertools.permutations(range(2 * n)):
        if pred(sigma):
            yield sigma


def enumerate_topologies(n: int, pred=is_sigma_diagram):
    """Distinct canonical forms (sorted), and the count of labelled representatives."""
    tops = set()
    n_lab = 0
    for sigma in enumerate_labelled(n, pred):
        n_lab += 1
        tops.add(canonical(sigma))
    return sorted(tops), n_lab


@dataclass
class Line:
    kind: str            # 'G' propagator or 'V' interaction
    src: int             # vertex the reference direction leaves
    dst: int             # vertex it enters
    mom: tuple = field(default=())   # coefficients over (q_0..q_{n-1}, k)


@dataclass
class Diagram:
    sigma: tuple
    order: int
    out_vertex: int
    n_loops_f: int       # closed fermion loops F
    weight: float        # (-1)^(n+F) 2^F
    lines: list          # propagators then interaction lines
    chords: list         # the lines carrying q_0..q_{n-1}: (kind, src, dst) each
    k_path: list = field(default_factory=list)   # indices into `lines` of the lines that carry k

    @property
    def ext_line(self) -> int:
        """Interaction line that holds the out-vertex: the external time is tau_ext_line."""
        return self.out_vertex // 2


def external_path(n2, edges, o):
    """The lines that carry the external momentum: a simple path from the in-vertex 0 to the
    out-vertex o with the fewest propagators, then the fewest lines, then the first in the order
    of line indices (compared position by position).  Returned as [(line index, +1 or -1)], +1
    when the walk from 0 to o follows the line's reference direction.

    Search: for each (propagator count g, length L) in increasing order, a depth-first walk that
    tries the lines at each vertex in index order finds the first path of exactly that count and
    length; the first (g, L) that has one wins."""
    inc = [[] for _ in range(n2)]
    for idx, (_, a, b) in enumerate(edges):
        inc[a].append((idx, +1, b))
        inc[b].append((idx, -1, a))
    for row in inc:
        row.sort()

    def search(g, L):
        path, seen = [], {0}

        def walk(v, g_left):
            if len(path) == L:
                return v == o and g_left == 0
            for idx, sgn, w in inc[v]:
                if w in seen:
                    continue
                isg = edges[idx][0] == "f"
                if isg and g_left == 0:
                    continue
                path.append((idx, sgn))
                seen.add(w)
                if walk(w, g_left - isg):
                    return True
                path.pop()
                seen.discard(w)
            return False

        return list(path) if walk(0, g) else None

    for g in range(len(edges) + 1):
        for L in range(max(g, 1), n2):
            p = search(g, L)
            if p is not None:
                return p
    raise AssertionError("the out-vertex is not reachable")


def route(sigma) -> Diagram:
    """Momentum routing with the external momentum on a path of chords.

    Internal lines, in this order, are the propagators v -> sigma[v] by source vertex (the
    external o -> 0 skipped), then the interaction lines (reference direction 2i -> 2i+1).
    1. Chords by reverse delete: first the lines of `external_path` in path order, then the
       other lines in order; a line becomes the next chord when the lines still left connect
       every vertex, until there are n chords.  The j-th chord carries q_j, along the walk from
       the in-vertex to the out-vertex if it lies on that path, else along its reference
       direction.
    2. What is left is a spanning tree.  The loop momentum of a chord returns along the tree
       path from its head to its tail.
    3. k enters at the in-vertex and follows `external_path` to the out-vertex.
    Only the lines of the external path depend on k, and a chord on it carries q_j + k."""
    n2 = len(sigma)
    n = n2 // 2
    o = sigma.index(0)
    fe, ve = _edges(sigma)
    edges = fe + ve
    kp = external_path(n2, edges, o)
    on_path = dict(kp)
    chord = {}                      # line index -> (loop index, direction)
    for idx in [i for i, _ in kp] + [i for i in range(len(edges)) if i not in on_path]:
        if len(chord) == n:
            break
        rest = [e for i, e in enumerate(edges) if i not in chord and i != idx]
        if _connected(n2, rest):
            chord[idx] = (len(chord), on_path.get(idx, +1))
    assert len(chord) == n
    tree = [i for i in range(len(edges)) if i not in chord]
    assert len(tree) == n2 - 1

    def tree_path(a, b):
        """(line index, +1/-1) along the unique tree path a -> b."""
        adj = [[] for _ in range(n2)]
        for idx in tree:
            _, x, y = edges[idx]
            adj[x].append((y, idx, +1))
            adj[y].append((x, idx, -1))
        prev = {a: None}
        stack = [a]
        while stack:
            v = stack.pop()
            for w, idx, sgn in adj[v]:
                if w not in prev:
                    prev[w] = (v, idx, sgn)
                    stack.append(w)
        path = []
        v = b
        while prev[v] is not None:
            u, idx, sgn = prev[v]
            path.append((idx, sgn))
            v = u
        return path

    mom = [[0] * (n + 1) for _ in edges]
    for idx, (j, sgn) in chord.items():
        mom[idx][j] = sgn
        _, u, w = edges[idx]
        head, tail = (w, u) if sgn > 0 else (u, w)
        for t, s in tree_path(head, tail):
            mom[t][j] += s
    for idx, sgn in kp:
        mom[idx][n] += sgn

    lines = [Line("G" if e[0] == "f" else "V", e[1], e[2], tuple(mom[i])) for i, e in enumerate(edges)]
    F = n_cycles(sigma) - 1
    chords = [None] * n
    for idx, (j, _) in chord.items():
        chords[j] = (lines[idx].kind, lines[idx].src, lines[idx].dst)
    return Diagram(sigma=tuple(sigma), order=n, out_vertex=o, n_loops_f=F,
                   weight=float((-1) ** (n + F) * 2 ** F), lines=lines,
                   chords=chords, k_path=[i for i, _ in kp])


def check_conservation(d: Diagram) -> bool:
    """Momentum in = momentum out at every vertex (external k in at 0, out at o)."""
    n = d.order
    n2 = 2 * n
    net = [[0] * (n + 1) for _ in range(n2)]
    for ln in d.lines:
        for c in range(n + 1):
            net[ln.src][c] -= ln.mom[c]
            net[ln.dst][c] += ln.mom[c]
    net[0][n] += 1
    net[d.out_vertex][n] -= 1
    return all(all(x == 0 for x in row) for row in net)


_CACHE: dict = {}


def sigma_diagrams(n: int):
    """Routed canonical self-energy diagrams of order n (sorted by canonical permutation)."""
    if n not in _CACHE:
        tops, _ = enumerate_topologies(n)
        _CACHE[n] = [route(s) for s in tops]
    return _CACHE[n]
