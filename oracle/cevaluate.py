"""The oracle's integrand in plain C (oracle/evaluate.c; test infrastructure): the same
diagram-by-diagram FP64 products as integrand.py, for many samples at high orders.  Pinned to
integrand.py sample by sample (tests/test_oracle_cevaluate.py)."""
from __future__ import annotations

import ctypes
import functools
import os

import numpy as np

from . import build as ob
from . import diagrams as dg


@functools.lru_cache(maxsize=None)
def _lib():
    L = ctypes.CDLL(ob.eval_library())
    P = ctypes.c_void_p
    L.oracle_evaluate.restype = ctypes.c_int
    L.oracle_evaluate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_longlong, P,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, P]
    return L


def table(diagrams, n):
    """(line table int32 [Ndiag, lines, 3 + n + 1] of (kind, a, b, c_0..c_n), weights, ext lines): the routed
    diagrams as data."""
    rows = []
    for d in diagrams:
        rows.append([[0 if ln.kind == "G" else 1, ln.src // 2, ln.dst // 2, *ln.mom] for ln in d.lines])
    t = np.ascontiguousarray(np.array(rows, dtype=np.int32))
    w = np.ascontiguousarray(np.array([d.weight for d in diagrams], dtype=np.float64))
    e = np.ascontiguousarray(np.array([d.ext_line for d in diagrams], dtype=np.int32))
    return t, w, e


def evaluate(x, n, k, beta, mu, lam, gamma, diagrams=None, derivs=False, threads=None, tab=None):
    """Per sample [N, q, 4] with q = value (and d/dmu, d/dlambda, d/dk with derivs): Re, Im, sum of the
    terms' magnitudes, and that sum weighted by each diagram's exponent condition C_d."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    t, w, e = tab if tab is not None else table(diagrams, n)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    N = x.shape[0]
    nq = 4 if derivs else 1
    out = np.empty((N, nq, 4), dtype=np.float64)
    if threads:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    rc = _lib().oracle_evaluate(n, t.shape[0], t.shape[1], t.ctypes.data, w.ctypes.data, e.ctypes.data, N,
                                x.ctypes.data, float(k), beta, mu, lam, gamma, 1 if derivs else 0, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_evaluate: bad arguments")
    return out


def integrand(x, n, k, beta, mu, lam, gamma, diagrams=None, tab=None):
    o = evaluate(x, n, k, beta, mu, lam, gamma, diagrams, tab=tab)
    return o[:, 0, 0] + 1j * o[:, 0, 1]


def fp32_tolerance(x, n, k, beta, mu, lam, gamma, diagrams=None, rel=1e-5, tab=None):
    """(tol, A) as integrand.fp32_tolerance."""
    o = evaluate(x, n, k, beta, mu, lam, gamma, diagrams, tab=tab)
    A = o[:, 0, 2]
    return rel * A + 2.0 * 2.0 ** -24 * o[:, 0, 3] + 1e-30, A
