"""Write the oracle's self-energy topologies of one order to tests/golden:
  order 5: sigma_topologies_o5.txt from oracle/diagrams.py (Python brute force over all 10!
           labelled permutations, about four minutes);
  order 6: sigma_topologies_o6.txt.xz from oracle/enumerate.c (the same brute force in C over
           all 12! permutations, about two minutes on 8 threads; xz-compressed text).
Calls only oracle/.  Each file holds a header with the counts and one canonical permutation per
line, in lexicographic order."""
import lzma
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import build as ob  # noqa: E402
from oracle import diagrams as dg  # noqa: E402


def main(n=5):
    if n <= 5:
        tops, n_lab = dg.enumerate_topologies(n)
        src = "oracle brute force, oracle/diagrams.py enumerate_topologies"
    else:
        tops, n_lab = ob.enumerate_topologies(n)
        src = "oracle brute force in C, oracle/enumerate.c"
    text = f"# order {n}: {len(tops)} topologies, {n_lab} labelled permutations ({src})\n"
    text += "".join(" ".join(str(v) for v in s) + "\n" for s in tops)
    if n <= 5:
        path = os.path.join(HERE, f"sigma_topologies_o{n}.txt")
        open(path, "w").write(text)
    else:
        path = os.path.join(HERE, f"sigma_topologies_o{n}.txt.xz")
        open(path, "wb").write(lzma.compress(text.encode(), preset=9))
    print(path, len(tops), n_lab)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 5)
