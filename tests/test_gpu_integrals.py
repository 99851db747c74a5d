"""Integral-level parity: GPU estimates against the oracle.

* Independent estimates (orders 2-6): the GPU's VEGAS estimate against the oracle's own estimate (its own
  VEGAS grid or importance proposal, numpy's PCG64, the C integrand), judged in units of the combined error
  by the family rule: with M comparisons (external momenta x Re/Im), the count with |z| > 3 within the
  binomial 99.9 % quantile at p = 0.0027, max |z| <= 4.5, and chi^2/dof within its 99.9 % quantile.  Errors
  on both sides are the scatter of independent batch means (robust to the heavy-tailed weights of orders
  >= 3).  At orders >= 4 the oracle affords few samples and its error is large: these comparisons are weak,
  and the same-sample check below carries the precision.
* Same samples (orders 4-6): the GPU evaluation and FP64 fold of points drawn by the oracle against the
  oracle's FP64 sum over the same points, bounded by the sum of the per-sample FP32 bounds (no sampling
  noise: the whole chain of evaluation, staging, FP64 reduction and estimate at the order's full graph).
* Order 2 against the deterministic quadrature of the rainbow diagram."""
import math

import numpy as np
import pytest
from scipy import stats

import paper_2403_18840_amd as dmc
from oracle import cevaluate as ce
from oracle import mc
from oracle import physics as ph
from oracle import quadrature as qd

from golden_diagrams import oracle_diagrams
from gpu_helpers import BETA, LAM, MU, to_soa, torch_dev

pytestmark = pytest.mark.gpu


def _z(a, ea, b, eb):
    za = (a.real - b.real) / np.sqrt(ea.real ** 2 + eb.real ** 2 + 1e-300)
    zi = (a.imag - b.imag) / np.sqrt(ea.imag ** 2 + eb.imag ** 2 + 1e-300)
    return np.concatenate([np.atleast_1d(za), np.atleast_1d(zi)])


def family_rule(z):
    """The rule for a family of M comparisons; returns (ok, description)."""
    z = z[np.isfinite(z)]
    M = len(z)
    n3 = int(np.sum(np.abs(z) > 3))
    q = int(stats.binom.ppf(0.999, M, 0.0027))
    chi = float(np.mean(z ** 2))
    chi_max = float(stats.chi2.ppf(0.999, M) / M)
    ok = n3 <= q and float(np.max(np.abs(z))) <= 4.5 and chi <= chi_max
    return ok, f"M={M} |z|>3: {n3} (<= {q}) max|z| {np.max(np.abs(z)):.2f} chi2/dof {chi:.2f} (<= {chi_max:.2f})"


def _gpu_batches(g, inst, ks, N, batches, seed, adapt=5):
    """VEGAS: adapt the grid, then `batches` independent estimates of N samples; (mean, scatter error)."""
    import torch
    _, dev = torch_dev()
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, g.order, n_bins=50, beta=BETA, qmax=6.0)
    first = dmc.adapt_grid(g, inst, ks, s, N, adapt, seed=seed)
    X = torch.empty((dmc.dim(g.order), N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    ms = []
    for b in range(batches):
        acc = dmc.Accumulator(1, len(ks), g.n_roots)
        s.sample(seed, first + b * N, X, J)
        dmc.eval_batch(g, inst, ks, X, J, acc)
        dmc.accumulate(acc)
        ms.append(acc.estimate(len(inst))[0][0, 0])
    ms = np.array(ms)
    return ms.mean(axis=0), (ms.real.std(axis=0, ddof=1) + 1j * ms.imag.std(axis=0, ddof=1)) / math.sqrt(batches)


@pytest.mark.parametrize("n,N_gpu,ora", [(2, 1 << 21, ("vegas", 1 << 20)), (3, 1 << 21, ("vegas", 1 << 19)),
                                         (4, 1 << 22, ("vegas", 1 << 18)), (5, 1 << 22, ("vegas", 1 << 14)),
                                         (6, 1 << 21, ("radial", 1 << 11))])
def test_estimates_match_oracle_family_rule(n, N_gpu, ora):
    ks = np.array([0.0, 1.0, 2.0], dtype=np.float32) if n <= 4 else np.array([1.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    inst = [(BETA, MU, LAM, gamma)]
    m, e = _gpu_batches(dmc.Graph(n), inst, ks, N_gpu, 16, seed=11 + n)
    dgs = oracle_diagrams(n)
    kind, N_ora = ora
    if kind == "vegas":
        om, oe = mc.vegas_mc(n, ks.astype(np.float64), BETA, MU, LAM, gamma, dgs, N=N_ora,
                             N_adapt=max(N_ora // 8, 1 << 12), seed=1234 + n)
    else:
        om, oe = mc.importance_mc(n, ks.astype(np.float64), BETA, MU, LAM, gamma, dgs, N=N_ora, seed=1234 + n)
    z = _z(m, e, om, oe)
    ok, msg = family_rule(z)
    print(f"order {n}: {msg}; gpu {m} +- {e}; oracle {om} +- {oe}")
    assert ok, msg


@pytest.mark.parametrize("n,N", [(4, 1 << 15), (5, 1 << 12), (6, 1 << 9)])
def test_same_samples_integral(n, N):
    """Oracle-drawn points (its radial importance proposal) through the GPU (evaluation, staging, FP64 fold,
    estimate) against the oracle's FP64 mean over the same points: |I_gpu - I| <= sum_i (tol_i + u |f_i|) J_i / N
    (tol_i the per-sample rule, u |f_i| J_i the FP32 rounding of the staged weight)."""
    torch, dev = torch_dev()
    rng = np.random.Generator(np.random.PCG64(77 + n))
    x, w = mc.radial_mixture_points(n, N, rng, BETA)
    x = x.astype(np.float32)
    jac = w.astype(np.float32)
    ks = np.array([1.0, 0.3], dtype=np.float32)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n)
    acc = dmc.Accumulator(1, len(ks), 1)
    dmc.eval_batch(g, [(BETA, MU, LAM, gamma)], ks, to_soa(x), torch.from_numpy(jac).to(dev), acc)
    dmc.accumulate(acc)
    m, _, ns, nf = acc.estimate(1)
    assert ns == N and nf == 0
    dgs = oracle_diagrams(n)
    tab = ce.table(dgs, n)
    x64, j64 = x.astype(np.float64), jac.astype(np.float64)
    for j, k in enumerate(ks):
        f = ce.integrand(x64, n, float(k), BETA, MU, LAM, gamma, dgs, tab=tab)
        tol, _ = ce.fp32_tolerance(x64, n, float(k), BETA, MU, LAM, gamma, dgs, tab=tab)
        ref = np.mean(f * j64)
        bound = np.sum((tol + 2.0 ** -24 * np.abs(f)) * j64) / N
        assert abs(m[0, 0, j].real - ref.real) <= bound, (k, m[0, 0, j], ref, bound)
        assert abs(m[0, 0, j].imag - ref.imag) <= bound, (k, m[0, 0, j], ref, bound)
        print(f"order {n} k {k}: gpu {m[0, 0, j]:.6e} oracle {ref:.6e} |diff| {abs(m[0, 0, j] - ref):.2e} bound {bound:.2e}")


@pytest.mark.parametrize("n,N_gpu,N_ora", [(2, 1 << 21, 1 << 20), (3, 1 << 21, 1 << 19)])
def test_blocks_estimates_match_oracle_family_rule(n, N_gpu, N_ora):
    """With building-block variables (DMC_ROUTING_BLOCKS): the GPU's VEGAS estimate against the oracle's own VEGAS
    estimate over its own relabelling of the diagrams, by the family rule."""
    from oracle import blocks
    ks = np.array([0.0, 1.0, 2.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    inst = [(BETA, MU, LAM, gamma)]
    m, e = _gpu_batches(dmc.Graph(n, routing=dmc.ROUTING_BLOCKS), inst, ks, N_gpu, 16, seed=41 + n)
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    om, oe = mc.vegas_mc(n, ks.astype(np.float64), BETA, MU, LAM, gamma, dgs, N=N_ora,
                         N_adapt=max(N_ora // 8, 1 << 12), seed=4321 + n)
    ok, msg = family_rule(_z(m, e, om, oe))
    print(f"order {n} (building blocks): {msg}; gpu {m} +- {e}; oracle {om} +- {oe}")
    assert ok, msg


def test_blocks_same_samples_integral_order5():
    """Oracle-drawn points through the GPU's building-block graph at order 5 against the oracle's FP64 mean over the
    same points with its own relabelling (the bound of test_same_samples_integral)."""
    from oracle import blocks
    torch, dev = torch_dev()
    n, N = 5, 1 << 12
    rng = np.random.Generator(np.random.PCG64(99))
    x, w = mc.radial_mixture_points(n, N, rng, BETA)
    x = x.astype(np.float32)
    jac = w.astype(np.float32)
    ks = np.array([1.0, 0.3], dtype=np.float32)
    gamma = ph.coupling(1.0)
    acc = dmc.Accumulator(1, len(ks), 1)
    dmc.eval_batch(dmc.Graph(n, routing=dmc.ROUTING_BLOCKS), [(BETA, MU, LAM, gamma)], ks, to_soa(x),
                   torch.from_numpy(jac).to(dev), acc)
    dmc.accumulate(acc)
    m, _, ns, nf = acc.estimate(1)
    assert ns == N and nf == 0
    dgs = blocks.block_diagrams(oracle_diagrams(n))
    tab = ce.table(dgs, n)
    x64, j64 = x.astype(np.float64), jac.astype(np.float64)
    for j, k in enumerate(ks):
        f = ce.integrand(x64, n, float(k), BETA, MU, LAM, gamma, dgs, tab=tab)
        tol, _ = ce.fp32_tolerance(x64, n, float(k), BETA, MU, LAM, gamma, dgs, tab=tab)
        ref = np.mean(f * j64)
        bound = np.sum((tol + 2.0 ** -24 * np.abs(f)) * j64) / N
        assert abs(m[0, 0, j].real - ref.real) <= bound and abs(m[0, 0, j].imag - ref.imag) <= bound, (k, m[0, 0, j], ref)


def test_order2_rainbow_matches_quadrature():
    """The rainbow diagram alone (its exported index) by VEGAS on the GPU against the deterministic quadrature of
    the first-order expansion of the Fock term."""
    idx = [i for i, d in enumerate(oracle_diagrams(2)) if d.n_loops_f == 0 and d.ext_line == 0]
    assert len(idx) == 1
    ks = np.array([0.0, 0.5, 1.0, 2.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    m, e = _gpu_batches(dmc.Graph(2, diagram_index=idx[0]), [(BETA, MU, LAM, gamma)], ks, 1 << 21, 16, seed=5)
    ref = np.array([qd.rainbow(float(k), BETA, MU, LAM, gamma) for k in ks])
    z = (m.real - ref) / e.real
    ok, msg = family_rule(z)
    print(f"rainbow: {msg}; gpu {m.real} +- {e.real}; quadrature {ref}")
    assert ok, msg
    assert np.all(m.imag == 0)


def test_proposals_agree_uniform_vs_vegas():
    n = 2
    ks = np.array([0.5, 1.0, 1.5], dtype=np.float32)
    gamma = ph.coupling(2.0)
    inst = [(BETA, MU, LAM, gamma)]
    mv, ev = dmc.integrate(dmc.Graph(n), inst, ks, 1 << 21, iters=6, adapt=5, seed=3)
    mu_, eu = dmc.integrate(dmc.Graph(n), inst, ks, 1 << 22, iters=4, kind=dmc.SAMPLER_UNIFORM, seed=4)
    z = _z(mv[0, 0], ev[0, 0], mu_[0, 0], eu[0, 0])
    ok, msg = family_rule(z)
    print(f"uniform vs VEGAS: {msg}; error ratio {np.round(eu[0, 0].real / ev[0, 0].real, 1)}")
    assert ok, msg
    # VEGAS must actually reduce the variance
    assert np.all(ev[0, 0].real * np.sqrt(6 * 2.0) < eu[0, 0].real * np.sqrt(4 * 4.0))
