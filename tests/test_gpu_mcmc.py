"""GPU Markov chains (independent proposals) against the oracle chain and the importance-sampling limit."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
import synth
from oracle import mcmc
from oracle import physics as ph

from gpu_helpers import BETA, LAM, MU, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("alpha,n,batches",
                         [(0.3, 1000, 3), (0.9, 2049, 5), (0.0, 777, 1), (0.5, 9001, 2), (0.7, 20000, 13)])
def test_chain_steps_match_oracle(alpha, n, batches):
    torch, dev = torch_dev()
    G, R, K = 2, 2, 3
    S = G * R * K * 2
    root0 = [s for g in range(G) for s in range(g * R * K * 2, (g * R + 1) * K * 2)]
    seed = 0xC4A1
    ch = dmc.Chains(n, G, K, R, batches)
    state = None
    ref = np.zeros((batches, S + 1, 2))
    taken = 0
    for t in range(4):
        f, jac = synth.chain_proposals(S, n, seed=40 + t, bad=(t < 2))
        off = (t * 7919 + 13) % n
        ch.step(torch.from_numpy(f.ravel()).to(dev), torch.from_numpy(jac).to(dev), alpha, seed, offset=off,
                measure=True)
        state, take = mcmc.step(state, f, jac, alpha, seed, t, root0, offset=off)
        taken += int(take.sum())
        ref += mcmc.measure(state, batches)
        sums, nm, na = ch.read()
        assert na == taken, f"step {t}: accepted {na} vs oracle {taken}"
        assert nm == n * (t + 1)
        # FP64 sums in another order: equal to a few ulps of the sum of magnitudes; a slot that holds
        # an infinite value (a taken proposal may carry one outside root 0) is infinite on both sides
        fin = np.isfinite(ref)
        scale = np.abs(np.where(fin, ref, 0.0)).sum(axis=-1)[..., None]
        with np.errstate(invalid="ignore"):
            close = np.abs(sums - ref) <= 1e-12 * scale + 1e-300
        assert np.all(np.where(fin, close, sums == ref)), f"step {t}"
    assert 0 < taken < 4 * n or alpha == 1.0


def test_alpha_one_equals_importance_sampling():
    torch, dev = torch_dev()
    n = 2
    g = dmc.Graph(n)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    s.set_grid(synth.vegas_grid(dmc.dim(n), 50, seed=3).astype(np.float64))
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    ks = synth.k_grid(5)
    r = dmc.mcmc_integrate(g, inst, ks, s, 1 << 16, steps=4, thermal=0, alpha=1.0, seed=9, n_batches=4)
    assert r.acceptance == 1.0
    # same proposals (rotated among the chains), every one taken: sum (f J) / n in FP64 from FP32 f and J
    # on both paths
    assert np.allclose(r.mean, r.is_mean, rtol=2e-6, atol=1e-7 * np.abs(r.is_mean).max())


def test_chain_estimate_agrees_with_importance_sampling():
    torch, dev = torch_dev()
    n = 2
    g = dmc.Graph(n)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    ks = synth.k_grid(6)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    dmc.adapt_grid(g, inst, ks, s, 1 << 20, 5, seed=2)
    # chains start from the proposal density; with an adapted grid the chain average settles within
    # a few hundred steps (shorter runs read |Sigma| low, the bias of an unthermalised independence
    # sampler), so 400 steps are discarded.  The error is the scatter of 32 independent chain batches.
    r = dmc.mcmc_integrate(g, inst, ks, s, 1 << 16, steps=800, thermal=400, alpha=0.3, seed=7, n_batches=32)
    assert 0.05 < r.acceptance < 1.0
    z = (r.mean[0, 0].real - r.is_mean[0, 0].real) / np.hypot(r.err[0, 0].real, r.is_err[0, 0].real)
    print("acceptance", r.acceptance, "z", z, "halves z", r.halves[2][0, 0].real)
    assert np.all(np.abs(z) < 4.5), z
    assert np.all(np.abs(r.halves[2][0, 0].real) < 4.5)


def test_flow_mixture_chains_agree_with_importance_sampling():
    # proposals from a defensive mixture whose components differ strongly (an untrained flow, the grid
    # and a large uniform share), laid out by component along the sample index: without the per-step
    # rotation the chains fed by one component settle to different distributions and the pooled
    # estimate is biased
    torch, dev = torch_dev()
    n = 1
    g = dmc.Graph(n)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    ks = np.array([1.0], dtype=np.float32)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    dmc.adapt_grid(g, inst, ks, s, 1 << 20, 5, seed=2)
    D = dmc.dim(n)
    masks = synth.flow_masks(D, 8, 5)
    f = dmc.Flow(D, masks)
    f.set_params(synth.flow_params(masks, 11, last_scale=0.3))
    r = dmc.mcmc_integrate(g, inst, ks, s, 1 << 16, steps=400, thermal=200, alpha=0.3, seed=5, n_batches=32,
                           flow=f, flow_alpha=0.5, flow_uniform=0.3)
    z = (r.mean[0, 0].real - r.is_mean[0, 0].real) / np.hypot(r.err[0, 0].real, r.is_err[0, 0].real)
    print("acceptance", r.acceptance, "z", z, "err", r.err[0, 0].real, "IS err", r.is_err[0, 0].real)
    assert np.all(np.abs(z) < 4.5), z


@pytest.mark.parametrize("alpha,n", [(0.0, 1500), (0.4, 5000)])
def test_chain_coordinates_and_training_data_match_oracle(alpha, n):
    torch, dev = torch_dev()
    G, R, K, D = 1, 2, 2, 7
    S = G * R * K * 2
    root0 = list(range(K * 2))
    seed = 0x7D
    ch = dmc.Chains(n, G, K, R, 3, dim_u=D)
    state = None
    rng = np.random.default_rng(17)
    for t in range(3):
        f, jac = synth.chain_proposals(S, n, seed=90 + t, bad=(t == 0))
        u = rng.uniform(size=(D, n)).astype(np.float32)
        off = (t * 131 + 7) % n
        ch.step(torch.from_numpy(f.ravel()).to(dev), torch.from_numpy(jac).to(dev), alpha, seed, offset=off,
                measure=False, u_prop=torch.from_numpy(u).to(dev))
        state, _ = mcmc.step(state, f, jac, alpha, seed, t, root0, offset=off, u_prop=u)
    U = torch.full((D, n + 5), float("nan"), dtype=torch.float32, device=dev)
    W = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
    ch.training_data(U, W)
    u_ref, w_ref = mcmc.training_data(state, root0)
    assert np.array_equal(U.cpu().numpy()[:, :n], u_ref)
    w = W.cpu().numpy().astype(np.float64)
    assert np.allclose(w, w_ref.astype(np.float32).astype(np.float64), rtol=0, atol=0)


def test_flow_trained_on_chain_samples_beats_the_grid():
    # order 2: a flow fitted only to MCMC-generated samples of |f| (alpha = 0) lowers the importance-sampling
    # variance below the adapted grid's and stays unbiased
    torch, dev = torch_dev()
    n = 2
    g = dmc.Graph(n)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    ks = np.array([1.0], dtype=np.float32)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    dmc.adapt_grid(g, inst, ks, s, 1 << 20, 5, seed=2)
    D = dmc.dim(n)
    masks = synth.flow_masks(D, 8, 5)
    f = dmc.Flow(D, masks)
    f.set_params(synth.flow_params(masks, 6, last_scale=0.0))
    losses = dmc.train_flow_mcmc(g, inst, ks, s, f, rounds=3, n_chains=1 << 16, thermal=100, collect=4, stride=10,
                                 steps=48, seed=4)
    assert losses[-1] < losses[0], losses
    N = 1 << 20
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    est = {}
    for name in ("grid", "flow"):
        acc = dmc.Accumulator(1, 1, 1)
        if name == "grid":
            s.sample(50, 0, X, J)
        else:
            f.sample(s, 51, 0, X, J, alpha=0.85, uniform=0.05)
        dmc.eval_batch(g, inst, ks, X, J, acc)
        dmc.accumulate(acc)
        m, e, _, _ = acc.estimate(1)
        est[name] = (m[0, 0, 0].real, e[0, 0, 0].real)
    z = (est["grid"][0] - est["flow"][0]) / np.hypot(est["grid"][1], est["flow"][1])
    ratio = (est["grid"][1] / est["flow"][1]) ** 2
    print("losses", losses, "variance ratio", ratio, "z", z)
    assert abs(z) < 4.5
    assert ratio > 2.0


def _spline_flow(D, seed, scale):
    masks = synth.flow_masks(D, 6, seed)
    f = dmc.Flow(D, masks, kind="spline")
    theta = synth.spline_flow_params(masks, seed + 100, scale)
    f.set_params(theta)
    f.theta32 = np.asarray(theta, dtype=np.float32).astype(np.float64)  # the library keeps FP32 parameters
    return f, [list(m) for m in masks]


def _log_close(got, ref, tight, loose):
    # log weights relative to 1 + |log w| (as for the flow's samples): a weight is a product of FP32 maps of
    # u'', whose own FP32 error a peaked spline magnifies
    lr = np.log(ref)
    r = np.abs(np.log(got) - lr) / (1.0 + np.abs(lr))
    return float(np.quantile(r, 0.99)) <= tight and float(r.max()) <= loose, (float(np.quantile(r, 0.99)),
                                                                               float(r.max()))


@pytest.mark.parametrize("D,n", [(7, 3000), (15, 2049), (23, 700), (3, 1), (11, 67)])
def test_flow_walk_matches_oracle(D, n):
    # base points of the states by the inverse flow, the Box-Muller move on the torus, the flow forward,
    # and the mixture and flow weights at both ends, against the oracle flow in FP64
    from oracle import integrand as ig
    from oracle import nsf
    from oracle import sampler as osp
    torch, dev = torch_dev()
    order = (D + 1) // 4
    # a moderately peaked flow: both traversals of the walk (inverse, forward) magnify FP32 rounding where a
    # spline derivative nears its floor
    f, masks = _spline_flow(D, 9, 0.1)
    th = f.theta32
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, order, n_bins=50)
    edges = synth.vegas_grid(D, 50, seed=4).astype(np.float64)
    s.set_grid(edges)
    us = np.random.default_rng(D).uniform(0.01, 0.99, size=(n, D)).astype(np.float32)
    US = torch.from_numpy(np.ascontiguousarray(us.T)).to(dev)
    X = torch.empty((D, n), dtype=torch.float32, device=dev)
    U = torch.empty((D, n), dtype=torch.float32, device=dev)
    J, JF, JFS = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
    sigma, seed, first, af, au = 0.07, 0xAB17, 55, 0.7, 0.1
    f.walk(s, US, sigma, seed, first, X, J, JF, U, JFS, alpha=af, uniform=au)
    # oracle
    lq_s, z = nsf.log_density(us.astype(np.float64), masks, th)
    zp = mcmc.walk_base(z, mcmc.normals(seed, first, n, D), sigma)
    u2, lq2 = nsf.forward(zp, masks, th)
    y2, jv2, _ = osp.vegas_map_float(u2, edges)
    x2, jp2 = ig.physical_map(y2, order, BETA, 6.0)
    ys, jvs, _ = osp.vegas_map_float(us, edges)
    _, jps = ig.physical_map(ys, order, BETA, 6.0)
    jac_ref = jp2 * jv2 / (af * np.exp(lq2) + (1 - af - au) + au * jv2)
    jf_ref = jp2 * jv2 / np.exp(lq2)
    jfs_ref = jps * jvs / np.exp(lq_s)
    # points whose moved base point lies at the wrap of the torus, or whose u'' lies at a grid bin's edge,
    # may land on the other side in FP32: their comparison says nothing about the arithmetic
    ok = np.all(np.minimum(zp, 1 - zp) > 1e-5, axis=1)
    ok &= np.all(np.abs(u2 * 50 - np.round(u2 * 50)) > 1e-3, axis=1)
    assert ok.mean() > 0.9
    ug = U.cpu().numpy().T.astype(np.float64)
    # two FP32 traversals of the flow (inverse, then forward): the median error is FP32 rounding (a few
    # 1e-7); samples where a spline derivative sits near its floor magnify it, in a tail of about 1 %
    err = np.abs(ug - u2).max(axis=1)[ok]
    assert np.median(err) <= 2e-6, np.median(err)
    assert np.quantile(err, 0.99) <= 1e-4 and err.max() <= 1e-3, (np.quantile(err, 0.99), err.max())
    # x follows u'' through the grid and physical maps: the few points with larger u'' errors (a spline
    # derivative near its floor magnifies FP32 rounding) carry them into x
    rx = (np.abs(X.cpu().numpy().T - x2) / (1 + np.abs(x2))).max(axis=1)[ok]
    assert np.quantile(rx, 0.99) <= 2e-4 and rx.max() <= 5e-2, (np.quantile(rx, 0.99), rx.max())
    # weights compared where FP32 holds them (the flow's own weight 1 / q_T overflows FP32 where q_T is
    # below e^-87); they are functions of u'', so its FP32 error enters them too
    rep = lambda w: (w > 1e-30) & (w < 1e30)
    big = ok & rep(jac_ref) & rep(jf_ref)
    assert big.mean() > 0.5
    for got, ref in ((J, jac_ref), (JF, jf_ref)):
        good, stats = _log_close(got.cpu().numpy().astype(np.float64)[big], ref[big], 1e-4, 2e-3)
        assert good, stats
    good, stats = _log_close(JFS.cpu().numpy().astype(np.float64)[rep(jfs_ref)], jfs_ref[rep(jfs_ref)], 1e-4, 2e-3)
    assert good, stats


@pytest.mark.parametrize("alpha,n", [(0.2, 1500), (0.8, 4099), (0.5, 1)])
def test_walk_step_matches_oracle(alpha, n):
    # the walk's Metropolis-Hastings test and state update on synthetic values, after an independence step
    torch, dev = torch_dev()
    G, R, K, D = 1, 1, 2, 3
    S = G * R * K * 2
    root0 = list(range(K * 2))
    seed = 0x3A1C
    nb = min(2, n)
    ch = dmc.Chains(n, G, K, R, nb, dim_u=D)
    rng = np.random.default_rng(5)
    f, jac = synth.chain_proposals(S, n, seed=70, bad=False)
    u = rng.uniform(size=(D, n)).astype(np.float32)
    tens = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ch.step(tens(f.ravel()), tens(jac), alpha, seed, offset=0, measure=False, u_prop=tens(u))
    state, _ = mcmc.step(None, f, jac, alpha, seed, 0, root0, u_prop=u)
    ref = np.zeros((nb, S + 1, 2))
    taken = 0
    for t in range(1, 4):
        f, jac = synth.chain_proposals(S, n, seed=70 + t, bad=(t == 1))
        _, jf = synth.chain_proposals(S, n, seed=170 + t, bad=(t == 1))
        _, jfs = synth.chain_proposals(S, n, seed=270 + t, bad=False)
        u = rng.uniform(size=(D, n)).astype(np.float32)
        ch.step_walk(tens(f.ravel()), tens(jac), tens(jf), tens(jfs), tens(u), alpha, seed, measure=True)
        state, take = mcmc.step_walk(state, f, jac, jf, jfs, alpha, seed, t, root0, u_prop=u)
        taken += int(take.sum())
        ref += mcmc.measure(state, nb)
        sums, nm, na = ch.read()
        assert na - n == taken, f"step {t}"  # the first (independence) step took every valid proposal
        fin = np.isfinite(ref)
        scale = np.abs(np.where(fin, ref, 0.0)).sum(axis=-1)[..., None]
        with np.errstate(invalid="ignore"):
            close = np.abs(sums - ref) <= 1e-12 * scale + 1e-300
        assert np.all(np.where(fin, close, sums == ref)), f"step {t}"
    assert 0 < taken < 3 * n or n < 10
    U = torch.empty((D, n), dtype=torch.float32, device=dev)
    W = torch.empty(n, dtype=torch.float32, device=dev)
    ch.training_data(U, W)
    assert np.array_equal(U.cpu().numpy(), state["u"])


def test_walk_chains_agree_with_importance_sampling():
    # order 2 with a spline flow's mixture: every other step a base-space walk; the chains' estimate
    # agrees with importance sampling over the independence proposals
    torch, dev = torch_dev()
    n = 2
    g = dmc.Graph(n)
    inst = [(BETA, MU, LAM, ph.coupling(1.0))]
    ks = np.array([1.0], dtype=np.float32)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    dmc.adapt_grid(g, inst, ks, s, 1 << 20, 5, seed=2)
    f, _ = _spline_flow(dmc.dim(n), 7, 0.1)
    r = dmc.mcmc_integrate(g, inst, ks, s, 1 << 16, steps=400, thermal=400, alpha=0.3, seed=6, n_batches=32,
                           flow=f, flow_alpha=0.85, flow_uniform=0.05, walk_every=2, walk_sigma=0.05)
    z = (r.mean[0, 0].real - r.is_mean[0, 0].real) / np.hypot(r.err[0, 0].real, r.is_err[0, 0].real)
    print("acceptance", r.acceptance, "z", z, "err", r.err[0, 0].real, "IS err", r.is_err[0, 0].real,
          "halves z", r.halves[2][0, 0])
    assert 0.05 < r.acceptance < 1.0
    assert abs(z) < 4.5, z
