"""Write the oracle's order-5 self-energy topologies (brute force over all 10! labelled
permutations, canonical forms) to sigma_topologies_o5.txt.  Calls only oracle/.  About three
minutes of CPU; the file holds one canonical permutation per line and a header with the counts."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import diagrams as dg  # noqa: E402


def main(n=5):
    tops, n_lab = dg.enumerate_topologies(n)
    path = os.path.join(HERE, f"sigma_topologies_o{n}.txt")
    with open(path, "w") as f:
        f.write(f"# order {n}: {len(tops)} topologies, {n_lab} labelled permutations "
                f"(oracle brute force, oracle/diagrams.py enumerate_topologies)\n")
        for s in tops:
            f.write(" ".join(str(v) for v in s) + "\n")
    print(path, len(tops), n_lab)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 5)
