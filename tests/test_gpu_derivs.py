"""GPU derivative roots (d/dmu, d/dlambda, d/dk) against the oracle and the closed forms."""
import math

import numpy as np
import pytest

import paper_2403_18840_amd as dmc
import synth
from oracle import integrand as ig
from oracle import physics as ph

from gpu_helpers import BETA, LAM, MU, gpu_integrand, to_soa, torch_dev
from golden_diagrams import oracle_diagrams

pytestmark = pytest.mark.gpu
ALL = dmc.D_MU | dmc.D_LAMBDA | dmc.D_K


@pytest.mark.parametrize("n,N,K", [(1, 600, 3), (2, 600, 5), (3, 400, 3), (4, 300, 3), (5, 100, 2)])
def test_derivative_roots_per_sample(n, N, K):
    """Each derivative against the oracle's dual numbers, judged against the size of the
    derivative's terms before cancellation (the condition-aware reading of 1e-5 relative).
    Orders 4 and 5 run the partitioned kernel (2 and 23 parts)."""
    x = synth.loop_points(n, N, seed=300 + n)
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    f, acc, _ = gpu_integrand(dmc.Graph(n, ALL), x, ks, [(BETA, MU, LAM, gamma)])
    assert f.shape[1] == 4
    x64 = x.astype(np.float64)
    dgs = oracle_diagrams(n)
    worst = [0.0] * 4
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        ref = [a.sum(axis=0) for a in ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)]
        absd = ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs, absolute=True)
        C = ig.exponent_condition(x64, n, kk, BETA, MU, diagrams=dgs)
        scale = [a.real.sum(axis=0) for a in absd]
        for r in range(4):
            err = np.abs(f[0, r, j] - ref[r])
            # the per-sample rule of the value, with the terms' magnitudes of the derivative
            ok = err <= 1e-5 * scale[r] + 2 * ig.U32 * (absd[r].real * C).sum(axis=0) + 1e-30
            assert np.all(ok), f"root {r} k={k}: worst {np.max(err / (scale[r] + 1e-300))}"
            m = scale[r] > 1e-30
            if np.any(m):
                worst[r] = max(worst[r], float(np.max(err[m] / scale[r][m])))
    print(f"order {n}: worst err/scale value {worst[0]:.2e} dmu {worst[1]:.2e} dlam {worst[2]:.2e} dk {worst[3]:.2e}")


def test_order1_derivative_estimates_match_closed_forms():
    torch, dev = torch_dev()
    n, N = 1, 1 << 21
    ks = np.array([0.5, 1.0, 1.6], dtype=np.float32)
    gamma = ph.coupling(1.0)
    s = dmc.Sampler(dmc.SAMPLER_UNIFORM, n)
    X = torch.empty((3, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(77, 0, X, J)
    acc = dmc.Accumulator(1, len(ks), 4)
    dmc.eval_batch(dmc.Graph(n, ALL), [(BETA, MU, LAM, gamma)], ks, X, J, acc)
    dmc.accumulate(acc)
    m, e, ns, nf = acc.estimate(1)
    for j, k in enumerate(ks):
        ref = [ph.fock_finite_T(float(k), BETA, MU, LAM, gamma)] + list(
            ph.fock_derivs_finite_T(float(k), BETA, MU, LAM, gamma))
        for r in range(4):
            z = (m[0, r, j].real - ref[r]) / e[0, r, j].real
            assert abs(z) < 3.5, f"k={k} root {r}: est {m[0, r, j].real} ref {ref[r]} z={z}"


def test_autograd_function_backward_and_finite_differences():
    torch, dev = torch_dev()
    n, N = 2, 1 << 18
    g = dmc.Graph(n, ALL)
    s = dmc.Sampler(dmc.SAMPLER_UNIFORM, n)
    X = torch.empty((dmc.dim(n), N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(5, 0, X, J)
    F = dmc.sigma_function()
    mu = torch.tensor(MU, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(LAM, dtype=torch.float64, requires_grad=True)
    k = torch.tensor([0.7, 1.3], dtype=torch.float64, requires_grad=True)
    gamma = ph.coupling(1.0)
    out = F.apply(mu, lam, k, g, X, J, BETA, gamma)
    wgt = torch.tensor([[1.0, -0.5], [0.3, 2.0]], dtype=torch.float64)
    (out * wgt).sum().backward()
    # same samples (common random numbers): the finite difference of the FP64-summed estimate
    h = 1e-3
    def val(mu_, lam_, k_):
        return (F.apply(torch.tensor(mu_, dtype=torch.float64), torch.tensor(lam_, dtype=torch.float64),
                        torch.tensor(k_, dtype=torch.float64), g, X, J, BETA, gamma) * wgt).sum().item()
    kk = [0.7, 1.3]
    fd_mu = (val(MU + h, LAM, kk) - val(MU - h, LAM, kk)) / (2 * h)
    fd_lam = (val(MU, LAM + h, kk) - val(MU, LAM - h, kk)) / (2 * h)
    fd_k0 = (val(MU, LAM, [kk[0] + h, kk[1]]) - val(MU, LAM, [kk[0] - h, kk[1]])) / (2 * h)
    for got, fd in [(mu.grad.item(), fd_mu), (lam.grad.item(), fd_lam), (k.grad[0].item(), fd_k0)]:
        assert abs(got - fd) <= 5e-3 * max(abs(fd), 1e-6), (got, fd)


def test_k_derivative_order6_per_sample():
    """d Sigma / dk at order 6 (31130 diagrams; a kernel of 221 parts, about a minute of run-time
    compilation) against the oracle's dual numbers at k near k_F."""
    n, N = 6, 24
    x = synth.loop_points(n, N, seed=306)
    ks = np.array([0.0, 1.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    f, acc, _ = gpu_integrand(dmc.Graph(n, dmc.D_K), x, ks, [(BETA, MU, LAM, gamma)])
    assert f.shape[1] == 2
    x64 = x.astype(np.float64)
    dgs = oracle_diagrams(n)
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        vals = ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)
        scales = ig.diagram_values_dual(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs, absolute=True)
        C = ig.exponent_condition(x64, n, kk, BETA, MU, diagrams=dgs)
        for r, src in [(0, 0), (1, 3)]:
            ref = vals[src].sum(axis=0)
            scale = scales[src].real.sum(axis=0)
            err = np.abs(f[0, r, j] - ref)
            tol = 1e-5 * scale + 2 * ig.U32 * (scales[src].real * C).sum(axis=0) + 1e-30
            assert np.all(err <= tol), f"root {r} k={k}: worst {np.max(err / (scale + 1e-300))}"
