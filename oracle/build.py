"""Build step of the C part of the oracle (test infrastructure): the brute-force diagram
enumerator oracle/enumerate.c -> oracle/enumerate_topologies (gcc, OpenMP)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "enumerate.c")
EXE = os.path.join(HERE, "enumerate_topologies")


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-Wall", "-o", EXE + ".tmp", SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle enumerator build failed:\n" + r.stdout + r.stderr)
    os.replace(EXE + ".tmp", EXE)
    return EXE


def executable() -> str:
    """The enumerator, built if it is missing or older than its source."""
    if not os.path.exists(EXE) or os.path.getmtime(EXE) < os.path.getmtime(SRC):
        build()
    return EXE


def enumerate_topologies(n: int):
    """(sorted canonical permutations, labelled count) from the C brute force."""
    out = subprocess.run([executable(), str(n)], capture_output=True, text=True, check=True).stdout
    lines = out.splitlines()
    head = lines[0].split()
    tops = [tuple(int(v) for v in ln.split()) for ln in lines[1:] if ln.strip()]
    assert int(head[3]) == len(tops)
    return tops, int(head[5])
