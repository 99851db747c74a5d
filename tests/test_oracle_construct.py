"""The bottom-up construction of the self-energy diagrams from the Dyson-Schwinger and parquet equations
(oracle/construct.py) against the brute-force set, and its irreducible vertices against the top-down decomposition
(oracle/blocks.py)."""
import collections

import pytest

from oracle import blocks
from oracle import construct as cs

from golden_diagrams import oracle_diagrams
from test_oracle_blocks import _vertex_blocks


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_construction_gives_every_diagram_once(n):
    """The equations, with the channel cuts and the pp pairing of the building-block rules and the fully
    irreducible vertices of the orderly generation, produce each brute-force topology exactly once: 1, 3, 20, 189,
    2232."""
    got = cs.sigma_topologies(n)
    assert set(got) == {d.sigma for d in oracle_diagrams(n)}
    assert all(v == 1 for v in got.values())


def test_construction_at_order6():
    """All 31130 order-6 topologies, each exactly once (the five-line irreducible vertices enter here)."""
    got = cs.sigma_topologies(6)
    assert len(got) == 31130 and all(v == 1 for v in got.values())
    assert set(got) == {d.sigma for d in oracle_diagrams(6)}


def test_irreducible_vertices_against_the_decomposition():
    """Fully irreducible four-point vertices with distinct legs: 2 with one interaction line (the bare interaction,
    direct and exchange), none with two or three, 64 with four (the envelopes).  Each with L lines closes into
    exactly one self-energy of order L + 1 (a bare line into it, a bare pair at the boson end), so the count
    equals the irreducible blocks of L lines that the top-down decomposition finds at order L + 1."""
    counts = [len(cs.irreducible_vertices(L)) for L in (1, 2, 3, 4)]
    assert counts == [2, 0, 0, 64]
    sizes = collections.Counter()
    for d in oracle_diagrams(5):
        vb = []
        _vertex_blocks(blocks.decompose(d), vb)
        sizes.update(len(b["verts"]) // 2 for b in vb if b["kind"] == "irr")
    assert dict(sizes) == {4: 64}
