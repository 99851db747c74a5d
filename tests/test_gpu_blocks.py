"""GPU evaluation with building-block variables (dmc_graph_spec.routing = DMC_ROUTING_BLOCKS) against the oracle
evaluating its own building-block relabelling of the brute-force diagrams."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
import synth
from oracle import blocks
from oracle import integrand as ig
from oracle import physics as ph

from golden_diagrams import oracle_diagrams
from gpu_helpers import BETA, LAM, MU, gpu_integrand, parity_points

pytestmark = pytest.mark.gpu
ALL = dmc.D_MU | dmc.D_LAMBDA | dmc.D_K


@pytest.mark.parametrize("n,N,K", [(1, 300, 3), (2, 600, 5), (3, 400, 4), (4, 300, 3), (5, 200, 2)])
def test_blocks_integrand_per_sample(n, N, K):
    """The per-sample rule (1e-5 A + 2u B + 1e-30) at orders 1-5, several tiles and a ragged tail."""
    x = parity_points(n, N, seed=900 + n)
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, routing=dmc.ROUTING_BLOCKS)
    assert g.info().routing == dmc.ROUTING_BLOCKS
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    x64 = x.astype(np.float64)
    worst = 0.0
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        ref = ig.integrand(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)
        tol, A = ig.fp32_tolerance(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)
        err = np.abs(f[0, 0, j] - ref)
        assert np.all(err <= tol), f"k={k}: worst {np.max(err / (A + 1e-300))}"
        live = A > 1e-30
        if np.any(live):
            worst = max(worst, float(np.max(err[live] / A[live])))
    print(f"order {n} (building blocks): worst |err|/A {worst:.2e}")


def test_blocks_derivative_roots_per_sample():
    """d/dmu, d/dlambda, d/dk with building-block variables at order 3, against the oracle's dual numbers."""
    n, N = 3, 300
    x = parity_points(n, N, seed=931)
    ks = synth.k_grid(3)
    gamma = ph.coupling(1.0)
    f, _, _ = gpu_integrand(dmc.Graph(n, ALL, routing=dmc.ROUTING_BLOCKS), x, ks, [(BETA, MU, LAM, gamma)])
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    x64 = x.astype(np.float64)
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        ref = [a.sum(axis=0) for a in ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)]
        absd = ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs, absolute=True)
        C = ig.exponent_condition(x64, n, kk, BETA, MU, diagrams=dgs)
        for r in range(4):
            err = np.abs(f[0, r, j] - ref[r])
            tol = 1e-5 * absd[r].real.sum(axis=0) + 2 * ig.U32 * (absd[r].real * C).sum(axis=0) + 1e-30
            assert np.all(err <= tol), f"root {r} k={k}"


def test_blocks_order6_per_sample():
    """All 31130 order-6 diagrams with building-block variables (a kernel in parts), against the oracle's C
    evaluator on its own relabelling."""
    from oracle import cevaluate as ce
    n, N = 6, 24
    x = parity_points(n, N, seed=960)
    ks = np.array([1.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, routing=dmc.ROUTING_BLOCKS)
    assert g.info().n_parts > 1
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    o = ce.evaluate(x.astype(np.float64), n, 1.0, BETA, MU, LAM, gamma, dgs)
    ref = o[:, 0, 0] + 1j * o[:, 0, 1]
    tol = 1e-5 * o[:, 0, 2] + 2 * ig.U32 * o[:, 0, 3] + 1e-30
    err = np.abs(f[0, 0, 0] - ref)
    assert np.all(err <= tol), f"worst {np.max(err / (o[:, 0, 2] + 1e-300))}"
    # the shell half is live (line momenta are sums of shell momenta, so some fall off the shell)
    assert np.sum(o[:, 0, 2] > 1e-20) >= N // 3


def test_blocks_taylor_roots_per_sample():
    """Taylor mode (T = 2, mu, lambda and k) with building-block variables at order 3 against the oracle's truncated
    series over its own relabelling.  The rule: the Taylor tests' 2e-5 of the term scale per derivative step, plus
    the per-sample rule's exponent term 2u sum_d scale_d C_d on each root's own term scales (as for the first-order
    derivative roots).  That term decides on the exponentially small samples of the default draw."""
    from oracle import taylor as ty
    n, T, N = 3, 2, 200
    x = parity_points(n, N, seed=941)
    ks = synth.k_grid(2)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, ALL, taylor_order=T, routing=dmc.ROUTING_BLOCKS)
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    x64 = x.astype(np.float64)
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        ref = ty.derivative_roots(x64, n, kk, BETA, MU, LAM, gamma, T, True, True, True, diagrams=dgs)
        scale = ty.derivative_scale(x64, n, kk, BETA, MU, LAM, gamma, T, True, True, True, diagrams=dgs)
        C = ig.exponent_condition(x64, n, kk, BETA, MU, diagrams=dgs)
        per = [ty.derivative_scale(x64, n, kk, BETA, MU, LAM, gamma, T, True, True, True, diagrams=[d]) for d in dgs]
        for r, ((key, rv), (_, sc)) in enumerate(zip(ref, scale)):
            steps = key[0] + key[1] + key[2] + 1
            expo = sum(p[r][1] * C[i] for i, p in enumerate(per))
            err = np.abs(f[0, r, j] - rv)
            assert np.all(err <= 2e-5 * steps * sc + 2 * ig.U32 * steps * expo + 1e-30), (key, k)


def test_blocks_partitioned_order4_per_sample():
    """Order 4 with building-block variables in parts of 40 diagrams, two lambda groups."""
    n, N = 4, 300
    x = parity_points(n, N, seed=944)
    ks = synth.k_grid(3)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, part_size=40, routing=dmc.ROUTING_BLOCKS)
    assert g.info().n_parts == 5
    lams = [0.5, 2.0]
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, lam, gamma) for lam in lams])
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    x64 = x.astype(np.float64)
    for gi, lam in enumerate(lams):
        for j, k in enumerate(ks):
            kk = float(np.float32(k))
            ref = ig.integrand(x64, n, kk, BETA, MU, lam, gamma, diagrams=dgs)
            tol, _ = ig.fp32_tolerance(x64, n, kk, BETA, MU, lam, gamma, diagrams=dgs)
            assert np.all(np.abs(f[gi, 0, j] - ref) <= tol), (lam, k)
