"""The oracle's diagrams of an order: its brute force for orders up to 4; for orders 5 and 6 the
canonical topologies that tests/golden/make_sigma_topologies.py wrote from the oracle's brute
force (tests/golden/sigma_topologies_o5.txt, and sigma_topologies_o6.txt.xz from the C version of
the same brute force), routed by the oracle."""
import functools
import lzma
import os

from oracle import diagrams as dg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_text(n):
    plain = os.path.join(GOLDEN, f"sigma_topologies_o{n}.txt")
    if os.path.exists(plain):
        return open(plain).read()
    return lzma.decompress(open(plain + ".xz", "rb").read()).decode()


@functools.lru_cache(maxsize=None)
def golden_topologies(n):
    lines = _golden_text(n).splitlines()
    return [tuple(int(v) for v in ln.split()) for ln in lines[1:] if ln.strip()]


@functools.lru_cache(maxsize=None)
def oracle_diagrams(n):
    if n <= 4:
        return dg.sigma_diagrams(n)
    return [dg.route(s) for s in golden_topologies(n)]


def golden_counts(n):
    """(topologies, labelled permutations) from the golden file's header."""
    head = _golden_text(n).splitlines()[0].split()
    return int(head[3]), int(head[5])
