"""The bottom-up construction of the self-energy diagrams from the Dyson-Schwinger and parquet equations
(oracle/construct.py) against the brute-force set, and against the top-down decomposition (oracle/blocks.py)."""
import pytest

from oracle import blocks
from oracle import construct as cs

from golden_diagrams import oracle_diagrams
from test_oracle_blocks import _vertex_blocks


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_construction_gives_every_diagram_once(n):
    """Through order 4 the only fully irreducible vertex is the bare interaction, and the equations (with the
    channel cuts and the pp pairing of the building-block rules) produce each brute-force topology exactly once:
    1, 3, 20, 189."""
    got = cs.sigma_topologies(n)
    assert set(got) == {d.sigma for d in oracle_diagrams(n)}
    assert all(v == 1 for v in got.values())


def test_order5_misses_exactly_the_envelope_diagrams():
    """At order 5 the construction without the envelope (the first fully irreducible vertex beyond the bare
    interaction, four lines) produces no diagram twice and none outside the set, and misses exactly the diagrams
    whose top-down decomposition holds an irreducible four-point block."""
    got = cs.sigma_topologies(5)
    ods = oracle_diagrams(5)
    want = {d.sigma for d in ods}
    assert set(got) <= want and all(v == 1 for v in got.values())
    with_envelope = set()
    for d in ods:
        vb = []
        _vertex_blocks(blocks.decompose(d), vb)
        if any(b["kind"] == "irr" for b in vb):
            with_envelope.add(d.sigma)
    assert want - set(got) == with_envelope
    assert len(with_envelope) == 64 and len(got) == 2168
