"""The oracle's C integrand (oracle/evaluate.c) against its numpy integrand, sample by sample: values,
first derivatives, the terms' magnitudes and the exponent-condition weights (orders 1-4, and order 5 on a
few samples), so that the C evaluator can stand in for integrand.py where that is too slow."""
import numpy as np
import pytest

import synth
from oracle import cevaluate as ce
from oracle import integrand as ig
from oracle import physics as ph

from golden_diagrams import oracle_diagrams

BETA, MU = 25.0, 1.0


@pytest.mark.parametrize("n,N", [(1, 400), (2, 400), (3, 300), (4, 120), (5, 6)])
def test_c_evaluator_matches_numpy_oracle(n, N):
    dgs = oracle_diagrams(n)
    x = synth.loop_points(n, N, seed=4200 + n).astype(np.float64)
    for k, lam, rs in [(0.0, 1.0, 1.0), (1.0, 0.5, 2.0), (2.7, 2.0, 1.0)]:
        gamma = ph.coupling(rs)
        o = ce.evaluate(x, n, k, BETA, MU, lam, gamma, dgs, derivs=True)
        vals = ig.diagram_values_dual(x, n, k, BETA, MU, lam, gamma, diagrams=dgs)
        absd = ig.diagram_values_dual(x, n, k, BETA, MU, lam, gamma, diagrams=dgs, absolute=True)
        C = ig.exponent_condition(x, n, k, BETA, MU, diagrams=dgs)
        for q in range(4):
            ref = vals[q].sum(axis=0)
            scale = absd[q].real.sum(axis=0)
            got = o[:, q, 0] + 1j * o[:, q, 1]
            assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300), (n, k, q)
            assert np.allclose(o[:, q, 2], scale, rtol=1e-12, atol=1e-300)
            assert np.allclose(o[:, q, 3], (absd[q].real * C).sum(axis=0), rtol=1e-12, atol=1e-300)
        tol, A = ig.fp32_tolerance(x, n, k, BETA, MU, lam, gamma, diagrams=dgs)
        tc, Ac = ce.fp32_tolerance(x, n, k, BETA, MU, lam, gamma, dgs)
        assert np.allclose(Ac, A, rtol=1e-12, atol=1e-300) and np.allclose(tc, tol, rtol=1e-12, atol=1e-300)
