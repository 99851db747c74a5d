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
the routing of loop momenta is a reverse-delete spanning tree over the canonical labels.  Both
rules are stated in the functions below; they are the agreed naming of variables (a data
convention), not arithmetic of the method.
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
    chords: list         # propagator source vertices carrying q_0..q_{n-1}

    @property
    def ext_line(self) -> int:
        """Interaction line that holds the out-vertex: the external time is tau_ext_line."""
        return self.out_vertex // 2


def route(sigma) -> Diagram:
    """Momentum routing by reverse delete.

    Propagators are visited in order of their source vertex (the external o->0 skipped); a
    propagator is removed if the remaining internal graph stays connected.  The removed
    propagators are the chords: the j-th removed carries loop momentum q_j along its own
    direction.  What is left (all interaction lines and n-1 propagators) is a spanning tree.
    The loop momentum of chord u->w returns from w to u along the tree path; the external k
    enters at vertex 0 and leaves at the out-vertex along the tree path.  Interaction line i
    has reference direction 2i -> 2i+1."""
    n2 = len(sigma)
    n = n2 // 2
    o = sigma.index(0)
    fe, ve = _edges(sigma)
    tree = fe + ve
    chords = []
    for e in fe:
        trial = [x for x in tree if x != e]
        if _connected(n2, trial):
            tree = trial
            chords.append(e)
    assert len(chords) == n and len(tree) == n2 - 1

    def tree_path(a, b):
        """Edges (with +1/-1 traversal sign) of the unique tree path a -> b."""
        adj = [[] for _ in range(n2)]
        for idx, (_, x, y) in enumerate(tree):
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

    mom = {e: [0] * (n + 1) for e in tree}
    chord_mom = {}
    for j, e in enumerate(chords):
        c = [0] * (n + 1)
        c[j] = 1
        chord_mom[e] = c
        _, u, w = e
        for idx, sgn in tree_path(w, u):
            mom[tree[idx]][j] += sgn
    for idx, sgn in tree_path(0, o):
        mom[tree[idx]][n] += sgn

    lines = []
    for e in fe:
        c = chord_mom[e] if e in chord_mom else mom[e]
        lines.append(Line("G", e[1], e[2], tuple(c)))
    for e in ve:
        lines.append(Line("V", e[1], e[2], tuple(mom[e])))
    F = n_cycles(sigma) - 1
    return Diagram(sigma=tuple(sigma), order=n, out_vertex=o, n_loops_f=F,
                   weight=float((-1) ** (n + F) * 2 ** F), lines=lines,
                   chords=[e[1] for e in chords])


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
