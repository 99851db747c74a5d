"""The oracle's diagrams of an order: its brute force for orders up to 4, and for order 5 the
canonical topologies that tests/golden/make_sigma_topologies.py wrote from the same brute force
(tests/golden/sigma_topologies_o5.txt; about four minutes to regenerate), routed by the oracle."""
import functools
import os

from oracle import diagrams as dg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@functools.lru_cache(maxsize=None)
def oracle_diagrams(n):
    if n <= 4:
        return dg.sigma_diagrams(n)
    path = os.path.join(GOLDEN, f"sigma_topologies_o{n}.txt")
    tops = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tops.append(tuple(int(v) for v in line.split()))
    return [dg.route(s) for s in tops]


def golden_counts(n):
    """(topologies, labelled permutations) from the golden file's header."""
    with open(os.path.join(GOLDEN, f"sigma_topologies_o{n}.txt")) as f:
        head = f.readline().split()
    return int(head[3]), int(head[5])
