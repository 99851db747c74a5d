"""Build step of the C part of the oracle (test infrastructure): the brute-force diagram
enumerator oracle/enumerate.c -> oracle/enumerate_topologies, and the diagram-by-diagram FP64
integrand oracle/evaluate.c -> oracle/liboracle_eval.so (gcc, OpenMP)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "enumerate.c")
EXE = os.path.join(HERE, "enumerate_topologies")
EVAL_SRC = os.path.join(HERE, "evaluate.c")
EVAL_LIB = os.path.join(HERE, "liboracle_eval.so")


def _gcc(args, what):
    r = subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-Wall", *args], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle {what} build failed:\n" + r.stdout + r.stderr)


def build() -> str:
    _gcc(["-o", EXE + ".tmp", SRC], "enumerator")
    os.replace(EXE + ".tmp", EXE)
    _gcc(["-shared", "-fPIC", "-o", EVAL_LIB + ".tmp", EVAL_SRC, "-lm"], "evaluator")
    os.replace(EVAL_LIB + ".tmp", EVAL_LIB)
    return EXE


def eval_library() -> str:
    """The C evaluator, built if it is missing or older than its source."""
    if not os.path.exists(EVAL_LIB) or os.path.getmtime(EVAL_LIB) < os.path.getmtime(EVAL_SRC):
        build()
    return EVAL_LIB


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
