"""GPU parity of the evaluation, sampling and reduction kernels against the CPU oracle."""
import math

import numpy as np
import pytest

import paper_2403_18840_amd as dmc
import synth
from oracle import integrand as ig
from oracle import physics as ph
from oracle import sampler as osp

from gpu_helpers import BETA, LAM, MU, gpu_integrand, parity_points, to_soa, torch_dev
from golden_diagrams import oracle_diagrams

pytestmark = pytest.mark.gpu

# Per-sample tolerance (the stated 1e-5 relative, read condition-aware; oracle/integrand.py
# fp32_tolerance): |f_gpu - f| <= 1e-5 A + 2 u B + 1e-30, with A(x) = sum_d |W_d(x)| the size of the
# diagram sum before sign cancellation (FP32 cannot resolve a cancelled sum better than its largest
# terms) and B the first-order error bound of the exponentials' FP32 arguments, which dominates only
# in samples whose every diagram is exponentially small.
REL = 1e-5


def _oracle_f(x, n, k, lam, gamma):
    return ig.integrand(x.astype(np.float64), n, float(np.float32(k)), BETA, MU, lam, gamma,
                        diagrams=oracle_diagrams(n))


@pytest.mark.parametrize("n,N,K,part_size", [(1, 845, 5, 0), (2, 845, 11, 0), (3, 600, 9, 0), (4, 300, 3, 0),
                                             (4, 300, 10, 40), (5, 300, 3, 0), (6, 40, 2, 0)])
def test_integrand_per_sample(n, N, K, part_size):
    """Several 256-sample tiles plus a ragged tail; K spans a partial chunk of k values.  Order 4
    in parts of 40 diagrams and order 6 (31130 diagrams in 20 parts; about
    two minutes of run-time compilation) cover the partitioned kernel."""
    x = parity_points(n, N, seed=100 + n)
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, part_size=part_size)
    f, acc, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    worst = 0.0
    for j, k in enumerate(ks):
        ref = _oracle_f(x, n, k, LAM, gamma)
        tol, A = ig.fp32_tolerance(x.astype(np.float64), n, float(np.float32(k)), BETA, MU, LAM, gamma,
                                   diagrams=oracle_diagrams(n))
        err = np.abs(f[0, 0, j] - ref)
        live = A > 1e-30
        if np.any(live):
            worst = max(worst, float(np.max(err[live] / A[live])))
        bad = np.where(~(err <= tol))[0]
        assert len(bad) == 0, (f"k={k}: {len(bad)} samples out of bounds, e.g. sample {bad[0]}: gpu {f[0, 0, j][bad[0]]}, "
                               f"oracle {ref[bad[0]]}, A {A[bad[0]]}, bound {tol[bad[0]]}")
    print(f"order {n}: worst |f_gpu - f_oracle| / A = {worst:.3e}")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_integrand_seeded_sweep(n):
    """The per-sample rule beyond the parity tests' own seeds: 2^14 samples x 4 external momenta
    (around k_F and at the ends), each sample from a seeded draw of the inputs' distribution.  Prints
    the worst |err| / A and the fractions meeting 1e-5 A and the plain 1e-5 |f|."""
    N = 1 << 14
    x = synth.loop_points(n, N, seed=5000 + n)
    ks = np.array([0.0, 0.95, 1.05, 3.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n)
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    worst, n_live, n_a, n_strict, n_rule = 0.0, 0, 0, 0, 0
    for j, k in enumerate(ks):
        ref = _oracle_f(x, n, k, LAM, gamma)
        tol, A = ig.fp32_tolerance(x.astype(np.float64), n, float(k), BETA, MU, LAM, gamma, diagrams=oracle_diagrams(n))
        err = np.abs(f[0, 0, j] - ref)
        live = A > 1e-30
        worst = max(worst, float(np.max(err[live] / A[live])))
        n_live += int(live.sum())
        n_a += int(np.sum(err[live] <= REL * A[live]))
        n_strict += int(np.sum(err[live] <= REL * np.abs(ref[live])))
        n_rule += int(np.sum(err <= tol))
        bad = np.where(~(err <= tol))[0]
        assert len(bad) == 0, f"k={k}: sample {bad[0]} gpu {f[0, 0, j][bad[0]]} oracle {ref[bad[0]]} bound {tol[bad[0]]}"
    print(f"order {n}: {N} samples x {len(ks)} k: worst |err|/A {worst:.2e}; within 1e-5 A {n_a}/{n_live}; "
          f"within 1e-5 |f| {n_strict}/{n_live}; within the rule {n_rule}/{N * len(ks)}")


@pytest.mark.parametrize("n,N", [(4, 1 << 13), (5, 1 << 11), (6, 1 << 9)])
def test_integrand_seeded_sweep_high_orders(n, N):
    """The sweep at orders 4-6 on the parity inputs' recipe (half the rows on the Fermi shell), seeds outside the
    other tests, 4 external momenta, against the oracle's C evaluator: every sample within the rule; prints the worst
    |err| / A and the fractions meeting 1e-5 A and the plain 1e-5 |f| among samples with A > 1e-20."""
    from oracle import cevaluate as ce
    x = parity_points(n, N, seed=6000 + n)
    ks = np.array([0.0, 0.95, 1.05, 3.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    f, _, _ = gpu_integrand(dmc.Graph(n), x, ks, [(BETA, MU, LAM, gamma)])
    dgs = oracle_diagrams(n)
    tab = ce.table(dgs, n)
    x64 = x.astype(np.float64)
    worst, n_live, n_a, n_strict = 0.0, 0, 0, 0
    for j, k in enumerate(ks):
        o = ce.evaluate(x64, n, float(k), BETA, MU, LAM, gamma, dgs, tab=tab)
        ref = o[:, 0, 0] + 1j * o[:, 0, 1]
        A = o[:, 0, 2]
        tol = 1e-5 * A + 2 * ig.U32 * o[:, 0, 3] + 1e-30
        err = np.abs(f[0, 0, j] - ref)
        bad = np.where(~(err <= tol))[0]
        assert len(bad) == 0, f"k={k}: sample {bad[0]} gpu {f[0, 0, j][bad[0]]} oracle {ref[bad[0]]} bound {tol[bad[0]]}"
        live = A > 1e-20
        worst = max(worst, float(np.max(err[live] / A[live])))
        n_live += int(live.sum())
        n_a += int(np.sum(err[live] <= REL * A[live]))
        n_strict += int(np.sum(err[live] <= REL * np.abs(ref[live])))
    assert n_live >= N * len(ks) // 3
    print(f"order {n}: {N} samples x {len(ks)} k: worst |err|/A {worst:.2e}; within 1e-5 A {n_a}/{n_live}; "
          f"within 1e-5 |f| {n_strict}/{n_live}")


def test_integrand_two_lambda_groups_and_rs_scaling():
    # instances sharing lambda are one evaluation scaled by (r_s'/r_s)^n; distinct lambdas are groups
    n, N = 2, 300
    x = synth.loop_points(n, N, seed=7)
    ks = synth.k_grid(4)
    g1, g2 = ph.coupling(1.0), ph.coupling(2.0)
    inst = [(BETA, MU, 0.5, g1), (BETA, MU, 2.0, g1)]
    f, acc, _ = gpu_integrand(dmc.Graph(n), x, ks, inst)
    for gi, lam in enumerate([0.5, 2.0]):
        for j, k in enumerate(ks):
            ref = _oracle_f(x, n, k, lam, g1)
            tol, _ = ig.fp32_tolerance(x.astype(np.float64), n, float(np.float32(k)), BETA, MU, lam, g1)
            assert np.all(np.abs(f[gi, 0, j] - ref) <= tol)
    # r_s rescaling in the estimate: gamma^n exactly
    torch, dev = torch_dev()
    X = to_soa(x)
    J = torch.ones(N, dtype=torch.float32, device=dev)
    acc = dmc.Accumulator(1, 4, 1)
    dmc.eval_batch(dmc.Graph(n), [(BETA, MU, LAM, g1), (BETA, MU, LAM, g2)], ks, X, J, acc)
    dmc.accumulate(acc)
    m, e, ns, nf = acc.estimate(2)
    assert ns == N and nf == 0
    assert np.allclose(m[1], m[0] * (g2 / g1) ** n, rtol=1e-12, atol=0)


def test_reduction_matches_fsum_and_is_deterministic():
    n, N, K = 2, 3000, 6
    x = synth.loop_points(n, N, seed=11)
    rng = np.random.default_rng(3)
    # powers of two: the kernel folds J into its per-sample phase factors, and scaling by 2^j commutes with
    # FP32 rounding, so the staged weight is exactly fp32(f) J and the FP64 fold can be held to fsum
    jac = (2.0 ** rng.integers(-1, 2, N)).astype(np.float32)
    ks = synth.k_grid(K)
    g = dmc.Graph(n)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    f, acc, imp = gpu_integrand(g, x, ks, inst, jac=jac)
    sums, ns = acc.read()
    assert ns == N
    for j in range(K):
        for c, part in enumerate([f[0, 0, j].real, f[0, 0, j].imag]):
            w = (part.astype(np.float32) * jac).astype(np.float64)  # the kernel's staged weight
            s1 = math.fsum(w)
            s2 = math.fsum(w * w)
            assert abs(sums[0, 0, j, c, 0] - s1) <= 1e-12 * math.fsum(np.abs(w)) + 1e-300
            assert abs(sums[0, 0, j, c, 1] - s2) <= 1e-12 * s2 + 1e-300
    # importance = sum over k, Re/Im of |w|
    w_all = np.abs(np.stack([f[0, 0].real, f[0, 0].imag]).astype(np.float32) * jac).sum(axis=(0, 1))
    assert np.allclose(imp, w_all, rtol=1e-5)
    # bitwise reproducible
    _, acc2, _ = gpu_integrand(g, x, ks, inst, jac=jac)
    sums2, _ = acc2.read()
    assert np.array_equal(sums, sums2)


@pytest.mark.parametrize("path", ["partitioned", "single"])
def test_fold_over_many_tiles_matches_fsum(path):
    """The FP64 fold at production size: 2^20 + 37 samples (thousands of tiles per block's running totals, a
    ragged last tile), two lambda groups, six momenta.  The partitioned kernel stages w = fp32(f J) with f the
    value it writes to f_out, so its weights are known exactly for a general (log-normal) Jacobian; the
    one-part kernel folds J into its per-sample factors, exact for powers of two.  Either way the sums must
    equal math.fsum of the staged weights within the FP64 error of any summation order, (N - 1) u_64 sum |w|,
    and repeat bit for bit."""
    torch, dev = torch_dev()
    n, N = 3, (1 << 20) + 37
    x = synth.loop_points(n, N, seed=29)
    rng = np.random.default_rng(31)
    if path == "partitioned":
        g = dmc.Graph(n, part_size=8)
        assert g.info().n_parts > 1
        jac = np.exp(rng.normal(0.0, 1.5, N)).astype(np.float32)
    else:
        g = dmc.Graph(n)
        assert g.info().n_parts == 1
        jac = (2.0 ** rng.integers(-3, 4, N)).astype(np.float32)
    ks = synth.k_grid(6)
    inst = [(BETA, MU, 0.5, ph.coupling(1.0)), (BETA, MU, 2.0, ph.coupling(1.0))]
    f, acc, imp = gpu_integrand(g, x, ks, inst, jac=jac)
    sums, ns = acc.read()
    assert ns == N
    gamma_n = (N - 1) * 2.0 ** -53 / (1 - (N - 1) * 2.0 ** -53)
    worst = 0.0
    w_abs = np.zeros(N, dtype=np.float64)
    for gi in range(2):
        for j in range(len(ks)):
            for c, part in enumerate([f[gi, 0, j].real, f[gi, 0, j].imag]):
                w32 = part.astype(np.float32) * jac          # the staged weight (RNE product, as on the device)
                w = w32.astype(np.float64)
                w_abs += np.abs(w)
                a1 = math.fsum(np.abs(w))
                s1, s2 = math.fsum(w), math.fsum(w * w)
                e1 = abs(sums[gi, 0, j, c, 0] - s1)
                e2 = abs(sums[gi, 0, j, c, 1] - s2)
                assert e1 <= gamma_n * a1 + 1e-300, (gi, j, c, sums[gi, 0, j, c, 0], s1, e1, gamma_n * a1)
                assert e2 <= gamma_n * s2 + 1e-300, (gi, j, c, sums[gi, 0, j, c, 1], s2, e2, gamma_n * s2)
                worst = max(worst, e1 / max(a1, 1e-300))
    # importance: the FP32 sum over groups, momenta and Re/Im of |w| (24 positive terms); below the smallest
    # normal FP32 number the products and sums round in absolute steps of 2^-149
    assert np.allclose(imp, w_abs, rtol=24 * 2.0 ** -24, atol=2.0 ** -126)
    print(f"{path}: {N} samples, worst |fold - fsum| / sum|w| = {worst:.2e} (bound {gamma_n:.2e})")
    _, acc2, _ = gpu_integrand(g, x, ks, inst, jac=jac)
    assert np.array_equal(sums, acc2.read()[0])


@pytest.mark.parametrize("n,mask,part,N,bad", [(1, 0, 0, 512, [3, 300]), (2, 0, 0, 300, [0, 299]),
                                               (2, 7, 0, 300, [5, 299]), (1, 7, 0, 70, [69]),
                                               (4, 0, 40, 300, [7, 299])])
def test_nonfinite_weights_are_counted_and_dropped(n, mask, part, N, bad):
    # an infinite Jacobian makes every weight of its sample non-finite (inf, or NaN where f = 0): each is
    # dropped and counted once per (root, Re/Im, k), for valid samples only (N = 300 and 70 end in a partial
    # tile whose idle lanes re-read the last sample); the sums and importances are those of the same batch
    # with these Jacobians set to 0.  Derivative roots go through the non-importance check, order 1 through
    # the structurally zero imaginary slots, part size 40 through the partitioned kernel.
    x = synth.loop_points(n, N, seed=5)
    g = dmc.Graph(n, deriv_mask=mask, part_size=part)
    ks = [0.0, 1.0]
    inst = [(BETA, MU, LAM, 0.5)]
    jac = np.ones(N, dtype=np.float32)
    jac[bad] = np.inf
    _, acc, imp = gpu_integrand(g, x, ks, inst, jac=jac)
    jac0 = jac.copy()
    jac0[bad] = 0.0
    _, acc0, imp0 = gpu_integrand(g, x, ks, inst, jac=jac0)
    m, e, ns, nf = acc.estimate(1)
    assert nf == len(bad) * len(ks) * g.n_roots * 2
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(e))
    assert np.array_equal(acc.read()[0], acc0.read()[0])
    assert np.array_equal(imp, imp0) and np.all(imp[bad] == 0.0)


@pytest.mark.parametrize("kind,n", [(dmc.SAMPLER_UNIFORM, 1), (dmc.SAMPLER_VEGAS, 2), (dmc.SAMPLER_VEGAS, 3)])
def test_sampler_matches_oracle(kind, n):
    torch, dev = torch_dev()
    N, seed, first = 1000, 0x2403188400000001, 12345
    s = dmc.Sampler(kind, n, n_bins=50, beta=BETA, qmax=6.0)
    D = dmc.dim(n)
    if kind == dmc.SAMPLER_VEGAS:
        grid = synth.vegas_grid(D, 50, seed=n).astype(np.float64)
        s.set_grid(grid)
    else:
        grid = np.tile(np.linspace(0, 1, 2), (D, 1))
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(seed, first, X, J)
    torch.cuda.synchronize()
    xg = X.cpu().numpy().T.astype(np.float64)
    jg = J.cpu().numpy().astype(np.float64)
    u, m = osp.uniforms(seed, first, N, D)
    if kind == dmc.SAMPLER_VEGAS:
        y, JV, _ = osp.vegas_map_int(m, grid.astype(np.float32).astype(np.float64))
    else:
        y, JV = u, np.ones(N)
    xr, Jp = ig.physical_map(y, n, BETA, 6.0)
    assert np.allclose(xg, xr, rtol=0, atol=6.0 * 4e-6)
    assert np.allclose(jg, JV * Jp, rtol=2e-5 * D, atol=0)


def test_vegas_histogram_matches_numpy():
    torch, dev = torch_dev()
    n, N, seed = 2, 4000, 99
    D = dmc.dim(n)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(seed, 0, X, J)
    acc = dmc.Accumulator(1, 3, 1)
    imp = torch.empty(N, dtype=torch.float32, device=dev)
    dmc.eval_batch(dmc.Graph(n), [(BETA, MU, LAM, 0.5)], [0.0, 1.0, 2.0], X, J, acc, imp_out=imp)
    dmc.accumulate(acc, s, imp)
    h = s.histogram()
    # the importance of each sample from the oracle: sum over k of |Re f J| + |Im f J| at the oracle's own
    # points of the (equal-bin) grid
    _, m = osp.uniforms(seed, 0, N, D)
    y, JV, _ = osp.vegas_map_int(m, np.tile(np.linspace(0.0, 1.0, 51), (D, 1)))
    x, Jp = ig.physical_map(y, n, BETA, 6.0)
    iv = np.zeros(N)
    for k in (0.0, 1.0, 2.0):
        f = ig.integrand(x, n, k, BETA, MU, LAM, 0.5) * (JV * Jp)
        iv += np.abs(f.real) + np.abs(f.imag)
    # FP32 underflows below ~1e-38 and a cancelling diagram sum is resolved to FP32 of its largest terms:
    # relative to the largest importance
    assert np.allclose(imp.cpu().numpy(), iv, rtol=1e-4, atol=1e-6 * iv.max())
    b = ((2 * m.astype(np.int64) + 1) * 50) >> 25
    ref = np.zeros((D, 50))
    for d in range(D):
        np.add.at(ref[d], b[:, d], iv * iv)
    # FP32 importance against FP64 (fixed-point accumulation on top), relative to the largest bin
    assert np.allclose(h, ref, rtol=5e-4, atol=1e-6 * ref.max())
    e0 = s.grid()
    s.refine(0.5)
    e = s.grid()
    assert np.all(np.diff(e, axis=1) > 0) and np.allclose(e[:, 0], 0) and np.allclose(e[:, -1], 1)
    # the sampler refines with the host routine dmc_vegas_refine, pinned to the oracle on the CPU (the
    # refinement weighs bins by their logarithm, so FP32-size differences in tiny bins move the grid)
    assert np.array_equal(e, dmc.vegas_refine(e0, h, 0.5))


def test_order1_estimate_matches_fock_closed_form():
    """16 k in [0, 3], r_s = 1, lambda = 1, beta = 25, 2^20 uniform samples in the ball."""
    torch, dev = torch_dev()
    n, N, K = 1, 1 << 20, 16
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    s = dmc.Sampler(dmc.SAMPLER_UNIFORM, n)
    X = torch.empty((3, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    s.sample(0x2403188400000000, 0, X, J)
    acc = dmc.Accumulator(1, K, 1)
    dmc.eval_batch(dmc.Graph(n), [(BETA, MU, LAM, gamma)], ks, X, J, acc)
    dmc.accumulate(acc)
    m, e, ns, nf = acc.estimate(1)
    assert ns == N and nf == 0
    for j, k in enumerate(ks):
        ref = ph.fock_finite_T(float(k), BETA, MU, LAM, gamma)
        z = (m[0, 0, j].real - ref) / e[0, 0, j].real
        assert abs(z) < 3.0, f"k={k}: z={z}"
        assert m[0, 0, j].imag == 0.0


def test_limits_and_degenerate_batches():
    """The largest observable shape one launch takes (DMC_MAX_K = 64 momenta, DMC_MAX_GROUPS = 8 lambda groups,
    order 2: 2048 staged slots) per sample against the oracle, on a ragged batch (257 samples: one full tile and
    one sample); a batch of one sample; and the refused shapes (no samples, ld < n, no momenta, 65 momenta,
    9 groups), which must leave the accumulator untouched."""
    torch, dev = torch_dev()
    n, N = 2, 257
    x = synth.loop_points(n, N, seed=41)
    ks = synth.k_grid(64)
    lams = [0.25 * (i + 1) for i in range(8)]
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n)
    f, acc, _ = gpu_integrand(g, x, ks, [(BETA, MU, lam, gamma) for lam in lams])
    x64 = x.astype(np.float64)
    for gi, lam in enumerate(lams):
        for j in range(0, 64, 7):
            k = float(np.float32(ks[j]))
            ref = ig.integrand(x64, n, k, BETA, MU, lam, gamma, diagrams=oracle_diagrams(n))
            tol, _ = ig.fp32_tolerance(x64, n, k, BETA, MU, lam, gamma, diagrams=oracle_diagrams(n))
            assert np.all(np.abs(f[gi, 0, j] - ref) <= tol), (lam, k)
    assert acc.read()[1] == N
    # one sample
    f1, acc1, _ = gpu_integrand(g, x[:1], ks[:3], [(BETA, MU, LAM, gamma)])
    for j in range(3):
        k = float(np.float32(ks[j]))
        ref = ig.integrand(x64[:1], n, k, BETA, MU, LAM, gamma, diagrams=oracle_diagrams(n))
        tol, _ = ig.fp32_tolerance(x64[:1], n, k, BETA, MU, LAM, gamma, diagrams=oracle_diagrams(n))
        assert np.all(np.abs(f1[0, 0, j] - ref) <= tol)
    m, e, ns, nf = acc1.estimate(1)
    assert ns == 1 and nf == 0 and np.all(e == 0)
    # refused shapes
    X = to_soa(x)
    J = torch.ones(N, dtype=torch.float32, device=dev)
    a = dmc.Accumulator(1, 4, 1)
    inst = [(BETA, MU, LAM, gamma)]
    bad = [dict(x=X, jac=J[:0], ks=ks[:4], inst=inst),                                   # no samples
           dict(x=X[:, :100].contiguous(), jac=J, ks=ks[:4], inst=inst),                 # ld < n
           dict(x=X, jac=J, ks=ks[:0], inst=inst),                                       # no momenta
           dict(x=X, jac=J, ks=np.linspace(0, 3, 65), inst=inst),                        # 65 momenta
           dict(x=X, jac=J, ks=ks[:4], inst=[(BETA, MU, 0.1 * (i + 1), gamma) for i in range(9)])]  # 9 groups
    for b in bad:
        with pytest.raises(dmc.DmcError) as err:
            dmc.eval_batch(g, b["inst"], b["ks"], b["x"], b["jac"], a)
        assert err.value.status == -1
    torch.cuda.synchronize()
    assert a.read()[1] == 0


def test_partitioned_kernel_at_the_largest_shape():
    """The kernel in parts at DMC_MAX_K = 64 momenta and DMC_MAX_GROUPS = 8 lambda groups (order 2 cut into its
    3 one-diagram parts), per sample against the oracle on a ragged batch of 257 samples: the block's LDS copy of
    the momenta is filled to its last entry, and every part reads the last momentum and the last group."""
    n, N = 2, 257
    x = synth.loop_points(n, N, seed=43)
    ks = synth.k_grid(64)
    lams = [0.25 * (i + 1) for i in range(8)]
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, part_size=1)
    assert g.info().n_parts == 3
    f, acc, _ = gpu_integrand(g, x, ks, [(BETA, MU, lam, gamma) for lam in lams])
    x64 = x.astype(np.float64)
    for gi, lam in enumerate(lams):
        for j in list(range(0, 64, 9)) + [63]:
            k = float(np.float32(ks[j]))
            ref = ig.integrand(x64, n, k, BETA, MU, lam, gamma, diagrams=oracle_diagrams(n))
            tol, _ = ig.fp32_tolerance(x64, n, k, BETA, MU, lam, gamma, diagrams=oracle_diagrams(n))
            assert np.all(np.abs(f[gi, 0, j] - ref) <= tol), (lam, k)
    assert acc.read()[1] == N


@pytest.mark.parametrize("part,kd", [(0, 0), (1, 2)])
def test_importance_roots_setting(part, kd):
    """imp_out sums |f J| over the graph's leading importance roots: the value alone by default, every root after
    set_importance(R); in one part and in parts with derivative roots at the first kd momenta only."""
    torch, dev = torch_dev()
    n, N = 2, 300
    x = synth.loop_points(n, N, seed=17)
    ks = synth.k_grid(4)
    g = dmc.Graph(n, deriv_mask=dmc.D_MU | dmc.D_LAMBDA | dmc.D_K, part_size=part, deriv_k=kd)
    assert (g.info().n_parts > 1) == (part > 0)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    R = g.n_roots
    for nr in (1, R, 2):
        g.set_importance(nr)
        f, _, imp = gpu_integrand(g, x, ks, inst)
        w = np.abs(f[0, :nr].real) + np.abs(f[0, :nr].imag)     # [roots][k][N], J = 1
        ref = w.sum(axis=(0, 1))
        assert np.allclose(imp, ref, rtol=4 * R * len(ks) * 2.0 ** -24, atol=2.0 ** -126), nr
    with pytest.raises(dmc.DmcError):
        g.set_importance(R + 1)
    with pytest.raises(dmc.DmcError):
        g.set_importance(0)


@pytest.mark.parametrize("n,N,K", [(2, 600, 5), (3, 400, 4)])
def test_spinless_integrand_per_sample(n, N, K):
    """spec.spin_deg = 1 (spinless fermions: a closed loop gives its sign only) against the oracle's diagrams with
    the weights (-1)^(n+F) of that definition."""
    import dataclasses
    x = parity_points(n, N, seed=950 + n)
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, spin_deg=1)
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    dgs = [dataclasses.replace(d, weight=float((-1) ** (n + d.n_loops_f))) for d in oracle_diagrams(n)]
    assert any(d.n_loops_f > 0 for d in dgs)
    x64 = x.astype(np.float64)
    for j, k in enumerate(ks):
        kk = float(np.float32(k))
        ref = ig.integrand(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)
        tol, _ = ig.fp32_tolerance(x64, n, kk, BETA, MU, LAM, gamma, diagrams=dgs)
        assert np.all(np.abs(f[0, 0, j] - ref) <= tol), f"k={k}"


@pytest.mark.parametrize("n,N,K", [(3, 400, 4), (5, 200, 2)])
def test_constructed_graph_per_sample(n, N, K):
    """A graph whose diagram list comes from the bottom-up construction (spec.generation = 1, another order of the
    same diagrams, so another kernel) per sample against the oracle."""
    x = parity_points(n, N, seed=970 + n)
    ks = synth.k_grid(K)
    gamma = ph.coupling(1.0)
    g = dmc.Graph(n, generation=dmc.GENERATE_CONSTRUCT)
    f, _, _ = gpu_integrand(g, x, ks, [(BETA, MU, LAM, gamma)])
    x64 = x.astype(np.float64)
    for j, k in enumerate(ks):
        ref = _oracle_f(x, n, k, LAM, gamma)
        tol, _ = ig.fp32_tolerance(x64, n, float(np.float32(k)), BETA, MU, LAM, gamma, diagrams=oracle_diagrams(n))
        assert np.all(np.abs(f[0, 0, j] - ref) <= tol), f"k={k}"
