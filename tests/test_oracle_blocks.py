"""Pins of the oracle's building-block variables (oracle/blocks.py) and the library's match to them."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
from oracle import blocks
from oracle import diagrams as dg

from golden_diagrams import oracle_diagrams

COUNTS = {1: 1, 2: 3, 3: 20, 4: 189, 5: 2232}


def _dyson_g(m):
    """Number of tadpole-free diagrams of the dressed propagator with m interaction lines, from the self-energy
    counts by the Dyson series G = G0 + G0 Sigma G (eq. Dyson): g_m = sum_i s_i g_{m-i}."""
    g = [1]
    for j in range(1, m + 1):
        g.append(sum(COUNTS[i] * g[j - i] for i in range(1, j + 1)))
    return g[m]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_relabelling_is_the_same_diagram_with_unit_jacobian(n):
    """Each relabelled diagram is the same topology with the in-vertex kept, conserves momentum, and its variables
    are the canonical ones under an integer map of unit determinant (loop momenta, plus a multiple of k) and a
    permutation of the interaction lines that keeps line 0 at tau = 0: the same integrand up to that change of
    variables."""
    for d in oracle_diagrams(n):
        b, lab = blocks.relabelling(d)
        assert lab[0] == 0 and dg.canonical(b.sigma) == d.sigma and dg.check_conservation(b)
        assert b.weight == d.weight and b.out_vertex == lab[d.out_vertex]
        mb = {(ln.kind, ln.src, ln.dst): np.array(ln.mom) for ln in b.lines}

        def key(kind, s, t):
            # an interaction line's reference direction is from its even end; relabelling may swap the ends
            return ((kind, lab[t], lab[s]), -1) if kind == "V" and lab[s] > lab[t] else ((kind, lab[s], lab[t]), 1)

        mc = {}
        for ln in d.lines:
            kk, sg = key(ln.kind, ln.src, ln.dst)
            mc[kk] = sg * np.array(ln.mom)
        if n == 1:
            continue
        # canonical chord j carries +-q_j (and k on the path): its new momentum gives row j of q = A q' + a k
        A, a = [], []
        for j, (kind, s, t) in enumerate(d.chords):
            c, _ = key(kind, s, t)
            sj = mc[c][j]
            assert abs(sj) == 1 and np.count_nonzero(mc[c][:n]) == 1
            A.append(sj * mb[c][:n])
            a.append(sj * (mb[c][n] - mc[c][n]))
        A, a = np.array(A), np.array(a)
        assert abs(round(np.linalg.det(A))) == 1
        for key, m in mc.items():
            lhs = mb[key]
            rhs_q = m[:n] @ A
            rhs_k = m[:n] @ a + m[n]
            assert np.array_equal(lhs[:n], rhs_q) and lhs[n] == rhs_k, (key, lhs, m)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_bare_vertex_diagrams_follow_the_dyson_count(n):
    """Sigma = V G Gamma3 with a bare Gamma3 is V times a dressed line of n - 1 interactions: exactly g_{n-1} of
    the order-n diagrams (1, 1, 4, 27, 248) decompose that way."""
    bare = sum(blocks.decompose(d)["g3"] is None for d in oracle_diagrams(n))
    assert bare == _dyson_g(n - 1)


def _vertex_blocks(blk, out):
    if blk is None:
        return
    if blk["kind"] == "sigma":
        for ins in blk["chain"][1]:
            _vertex_blocks(ins, out)
        g3 = blk["g3"]
        if g3 is not None:
            for ch in (g3["out_chain"], g3["in_chain"]):
                for ins in ch[1]:
                    _vertex_blocks(ins, out)
            _vertex_blocks(g3["g4"], out)
    else:
        out.append(blk)
        if blk["kind"] == "red":
            _vertex_blocks(blk["left"], out)
            _vertex_blocks(blk["right"], out)
            for ch in blk["chains"]:
                for ins in ch[1]:
                    _vertex_blocks(ins, out)


def test_fully_irreducible_vertices_start_with_the_envelope():
    """Beyond the bare interaction, the first fully two-particle-irreducible four-point vertex has four interaction
    lines (the envelope); inside a self-energy it needs five lines in all.  So no larger irreducible block occurs
    below order 5, every channel-reducible vertex up to order 4 ends in bare interactions, and order 5 has some."""
    def irr_sizes(n):
        sizes = []
        for d in oracle_diagrams(n):
            vb = []
            _vertex_blocks(blocks.decompose(d), vb)
            sizes += [len(b["verts"]) // 2 for b in vb if b["kind"] == "irr"]
        return sizes
    for n in (2, 3, 4):
        assert irr_sizes(n) == []
    s5 = irr_sizes(5)
    assert s5 and set(s5) == {4}


def _parse(text):
    out = []
    for row in text.strip().splitlines():
        f = row.split("|")
        sig = tuple(int(v) for v in f[0].split())
        lines = []
        for seg in f[3:]:
            kind, *rest = seg.split(None, 1)
            for grp in rest[0].split(";") if rest else []:
                v = [int(t) for t in grp.split()]
                if v:
                    lines.append((kind, v[0], v[1], tuple(v[2:])))
        out.append((sig, sorted(lines)))
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_library_building_block_routing_equals_oracle(n):
    """dmc_graph_spec.routing = DMC_ROUTING_BLOCKS: the library's labelling and momenta, diagram by diagram,
    equal the oracle's (the convention is written twice)."""
    got = _parse(dmc.Graph(n, routing=dmc.ROUTING_BLOCKS).export())
    want = [(tuple(b.sigma), sorted((l.kind, l.src, l.dst, tuple(l.mom)) for l in b.lines))
            for b in blocks.block_diagrams(oracle_diagrams(n))]
    assert got == want


def test_building_block_routing_op_counts():
    """The blocks share more of the k-independent work (order 5: 14 % less) and carry k through
    more distinct leaves than the path routing."""
    a = dmc.Graph(5).info()
    b = dmc.Graph(5, routing=dmc.ROUTING_BLOCKS).info()
    assert b.routing == 1 and a.routing == 0
    # the kernel names tell the routings apart in a profiler's trace
    name = lambda g: g.source(1).splitlines()[1].split()[-1]
    assert name(dmc.Graph(5, routing=dmc.ROUTING_BLOCKS)) == name(dmc.Graph(5)) + "_b"
    assert sum(b.ops_sample) < 0.9 * sum(a.ops_sample)
    assert sum(b.ops_k) > sum(a.ops_k)
