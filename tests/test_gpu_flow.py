"""GPU affine-coupling flow against the oracle flow: densities, samples, gradients, training."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
import synth
from oracle import flow as ofl
from oracle import integrand as ig
from oracle import sampler as osp

from gpu_helpers import BETA, torch_dev

pytestmark = pytest.mark.gpu
L = 8


def _flow(D, scale=0.03, seed=1):
    m = synth.flow_masks(D, L, seed)
    th = synth.flow_params(m, seed + 1, last_scale=scale)
    f = dmc.Flow(D, m)
    f.set_params(th)
    return f, m, th.astype(np.float64)


def _maps_on_gpu_points(xg, jg, ug, lqg, g32, n, a_f=1.0, a_u=0.0):
    """Every sample, with no selection: the grid and physical maps and the weight applied to the kernel's own u'
    and log q (read back), against the oracle's maps in FP64 after the same FP32 bin decision.  The network is
    compared separately (u' and log q against the oracle flow); this isolates the maps, in the coordinates where
    FP32 is well conditioned: the radius |q| = R y_r (relative), cos(theta) = q_z / |q| = 2 y_c - 1 and
    phi = 2 pi y_phi (absolute; phi only where |q| sin(theta) is not tiny), the times beta y_t, and the weight
    (relative, a few FP32 roundings per dimension)."""
    y, JV, _ = osp.vegas_map_float(ug, g32)
    _, Jp = ig.physical_map(y, n, BETA, 6.0)
    for i in range(n):
        q = xg[:, 3 * i: 3 * i + 3]
        r = np.linalg.norm(q, axis=1)
        assert np.all(np.abs(r - 6.0 * y[:, 3 * i]) <= 2e-6 * (6.0 * y[:, 3 * i]) + 1e-6), i
        ok = r > 1e-5
        c = q[ok, 2] / r[ok]
        assert np.all(np.abs(c - (2.0 * y[ok, 3 * i + 1] - 1.0)) <= 4e-6), i
        rho = np.hypot(q[:, 0], q[:, 1])
        okp = rho > 1e-4
        dphi = np.angle(np.exp(1j * (np.arctan2(q[okp, 1], q[okp, 0]) - 2 * np.pi * y[okp, 3 * i + 2])))
        assert np.all(np.abs(dphi) <= 4e-6 + 2e-7 / rho[okp]), i
    for j in range(n - 1):
        assert np.all(np.abs(xg[:, 3 * n + j] - BETA * y[:, 3 * n + j]) <= 4e-7 * BETA + 2e-6), j
    ref = ofl.mixture_weight(JV * Jp, lqg, a_f, a_u, JV) if a_f < 1.0 else JV * Jp * np.exp(-lqg)
    # a few roundings per dimension in the Jacobians, and the hardware exponential of log q (error ~ |log q| u)
    D = xg.shape[1]
    u = 2.0 ** -24
    assert np.all(np.abs(np.log(jg) - np.log(ref)) <= 4 * D * u + 4 * u * np.abs(lqg) + 1e-6)


@pytest.mark.parametrize("D", [3, 7, 15, 23])
def test_log_density_matches_oracle(D):
    torch, dev = torch_dev()
    f, m, th = _flow(D)
    N = 1000
    u = np.random.default_rng(5).uniform(0.01, 0.99, size=(N, D)).astype(np.float32)
    U = torch.from_numpy(np.ascontiguousarray(u.T)).to(dev)
    lq = torch.empty(N, dtype=torch.float32, device=dev)
    f.log_density(U, lq)
    torch.cuda.synchronize()
    g = lq.cpu().numpy().astype(np.float64)
    ref = ofl.log_q(th, m, u.astype(np.float64))
    err = np.abs(g - ref)
    print(f"D={D}: |log q| median {np.median(np.abs(ref)):.3f}; err median {np.median(err):.2e} max {err.max():.2e}")
    # BF16 rounding of activations may land on the other side of a rounding boundary than the
    # FP64 oracle (FP32 vs FP64 accumulation): a few 2^-8 steps in single activations
    assert np.median(err) < 1e-4 and err.max() < 5e-3


@pytest.mark.parametrize("D,n", [(3, 1), (7, 2), (15, 4), (23, 6)])
def test_flow_samples_match_oracle(D, n):
    torch, dev = torch_dev()
    f, m, th = _flow(D)
    N, seed, first = 777, 0x2403188400000004, 99
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    grid = synth.vegas_grid(D, 50, seed=D).astype(np.float64)
    s.set_grid(grid)
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    Uo = torch.empty((D, N), dtype=torch.float32, device=dev)
    LQ = torch.empty(N, dtype=torch.float32, device=dev)
    f.sample(s, seed, first, X, J, u_out=Uo, lq_out=LQ)
    torch.cuda.synchronize()
    ug = Uo.cpu().numpy().T.astype(np.float64)
    lqg = LQ.cpu().numpy().astype(np.float64)
    u, _ = osp.uniforms(seed, first, N, D)
    up, lq, _ = ofl.sample(th, m, u)
    assert np.max(np.abs(ug - up)) < 2e-3
    assert np.median(np.abs(lqg - lq)) < 1e-4 and np.max(np.abs(lqg - lq)) < 5e-3
    # x and the weight from the oracle's own u' and log q; the grid map jumps at bin edges and BF16 moves u'
    # by up to ~1e-3, so the comparison takes the samples whose u' falls in the same bins on both sides
    y, JV, b_ref = osp.vegas_map_float(up, grid.astype(np.float32).astype(np.float64))
    xr, Jp = ig.physical_map(y, n, BETA, 6.0)
    same = np.all(np.minimum(np.floor(ug * 50), 49) == b_ref, axis=1)
    assert same.mean() > 0.75, same.mean()
    xg = X.cpu().numpy().T.astype(np.float64)
    jg = J.cpu().numpy().astype(np.float64)
    # the maps carry u''s BF16 error (up to ~1e-3, magnified by the grid and by the polar angle near the
    # poles): checked in the median and the 99th percentile
    rx = (np.abs(xg - xr) / (1 + np.abs(xr))).max(axis=1)[same]
    assert np.median(rx) < 5e-4 and np.quantile(rx, 0.99) < 5e-2, (np.median(rx), np.quantile(rx, 0.99))
    lerr = np.abs(np.log(jg) - np.log(JV * Jp * np.exp(-lq)))[same]
    assert np.median(lerr) < 2e-4 and lerr.max() < 2e-2, (np.median(lerr), lerr.max())
    _maps_on_gpu_points(xg, jg, ug, lqg, grid.astype(np.float32).astype(np.float64), n)
    # forward density = inverse density on the GPU
    lq2 = torch.empty(N, dtype=torch.float32, device=dev)
    f.log_density(Uo, lq2)
    torch.cuda.synchronize()
    ok = np.all(np.abs(ug - 0.5) < 0.4999, axis=1)
    assert np.max(np.abs(lq2.cpu().numpy()[ok] - lqg[ok])) < 2e-3


def test_identity_flow_reproduces_vegas_sampler():
    torch, dev = torch_dev()
    D, n, N = 11, 3, 4096
    m = synth.flow_masks(D, L, 3)
    f = dmc.Flow(D, m)
    f.set_params(synth.flow_params(m, 4, last_scale=0.0))
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    s.set_grid(synth.vegas_grid(D, 50, seed=2).astype(np.float64))
    X1 = torch.empty((D, N), dtype=torch.float32, device=dev)
    J1 = torch.empty(N, dtype=torch.float32, device=dev)
    X2 = torch.empty_like(X1)
    J2 = torch.empty_like(J1)
    f.sample(s, 7, 0, X1, J1)
    s.sample(7, 0, X2, J2)
    torch.cuda.synchronize()
    assert torch.allclose(X1, X2, atol=6e-5, rtol=0)
    assert torch.allclose(J1, J2, rtol=1e-4)


@pytest.mark.parametrize("D,N", [(3, 1000), (7, 2048), (15, 3000), (23, 1500)])
def test_gradient_matches_oracle(D, N):
    torch, dev = torch_dev()
    f, m, th = _flow(D, scale=0.03, seed=7)
    seed = 21
    w = np.random.default_rng(8).exponential(size=N).astype(np.float32)
    W = torch.from_numpy(w).to(dev)
    grad = torch.empty(f.n_params, dtype=torch.float32, device=dev)
    loss = f.train_step(W, seed=seed, first=0, lr=0.0, grad_out=grad)
    g = grad.cpu().numpy().astype(np.float64)
    u, _ = osp.uniforms(seed, 0, N, D)
    rl, rg = ofl.loss_and_grad(th, m, u, w.astype(np.float64))
    rel = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"D={D}: loss {loss:.6f} vs {rl:.6f}; |grad - ref| / |ref| = {rel:.2e}")
    assert abs(loss - rl) < 1e-4 * max(1.0, abs(rl))
    assert rel < 1e-2
    # element by element, each layer against its largest entry (none is silently zero): the oracle rounds the
    # same operands to BF16, so what remains is FP32 summation order and the rare rounding flip it causes
    worst = 0.0
    for l in range(L):
        sl = slice(l * ofl.LAYER_SIZE, (l + 1) * ofl.LAYER_SIZE)
        scale = np.max(np.abs(rg[sl]))
        assert scale > 0
        err = np.max(np.abs(g[sl] - rg[sl])) / scale
        worst = max(worst, err)
        assert err <= 1e-3, (l, err)
    print(f"D={D}: worst per-element |grad - ref| / max |ref| of its layer = {worst:.2e}")


def test_training_lowers_the_loss_and_adam_matches_oracle_step():
    torch, dev = torch_dev()
    D, N = 7, 4096
    f, m, th = _flow(D, scale=0.0, seed=11)
    # a peaked target on the unit cube: w = prod_d exp(-(u_d - c_d)^2 / (2 0.1^2)) at Philox points
    u, _ = osp.uniforms(33, 0, N, D)
    c = np.linspace(0.3, 0.7, D)
    w = np.exp(-((u - c) ** 2).sum(axis=1) / (2 * 0.1 ** 2)).astype(np.float32)
    W = torch.from_numpy(w).to(dev)
    # one Adam step equals the oracle's Adam step on the oracle gradient (to BF16/FP32 level)
    grad = torch.empty(f.n_params, dtype=torch.float32, device=dev)
    f.train_step(W, seed=33, first=0, lr=1e-3, grad_out=grad)
    _, rg = ofl.loss_and_grad(th, m, u, w.astype(np.float64))
    th1, _, _ = ofl.adam_step(th, rg, np.zeros_like(th), np.zeros_like(th), 1, 1e-3)
    got = f.params().astype(np.float64)
    moved = np.abs(th1 - th) > 5e-4   # Adam's first step moves every parameter with g != 0 by ~lr
    assert np.mean(np.abs(got - th1)[moved] < 2e-4) > 0.99
    losses = []
    for it in range(60):
        losses.append(f.train_step(W, seed=33, first=0, lr=3e-3))
    print(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < losses[0] - 1.0



def _flow_share_matches(xg, jg, ug, up, lq, g32, n, a_f, a_u):
    """The flow share's points and mixture weights against the oracle's own u' and log q.  The grid map jumps
    at bin edges and BF16 moves u' by up to ~1e-3, so the samples compared are those whose u' falls in the
    same bins on both sides; the maps carry u''s BF16 error (magnified by the grid and, near the poles, by the
    polar angle), so x is checked in the median and the 99th percentile."""
    yv, JV, b_ref = osp.vegas_map_float(up, g32)
    xr, Jp = ig.physical_map(yv, n, BETA, 6.0)
    same = np.all(np.minimum(np.floor(ug * 50), 49) == b_ref, axis=1)
    assert same.mean() > 0.75, same.mean()
    rx = (np.abs(xg - xr) / (1 + np.abs(xr))).max(axis=1)[same]
    assert np.median(rx) < 5e-4 and np.quantile(rx, 0.99) < 5e-2, (np.median(rx), np.quantile(rx, 0.99))
    lerr = np.abs(np.log(jg) - np.log(ofl.mixture_weight(JV * Jp, lq, a_f, a_u, JV)))[same]
    assert np.median(lerr) < 2e-4 and lerr.max() < 2e-2, (np.median(lerr), lerr.max())

@pytest.mark.parametrize("alpha,N", [(0.6, 1000), (0.9, 4099)])
def test_mixture_samples_match_oracle(alpha, N):
    torch, dev = torch_dev()
    D, n = 11, 3
    f, m, th = _flow(D, scale=0.03, seed=2)
    seed, first = 0x51A3, 1 << 33
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    grid = synth.vegas_grid(D, 50, seed=4).astype(np.float64)
    s.set_grid(grid)
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    Uo = torch.empty((D, N), dtype=torch.float32, device=dev)
    LQ = torch.empty(N, dtype=torch.float32, device=dev)
    f.sample(s, seed, first, X, J, u_out=Uo, lq_out=LQ, alpha=alpha)
    n_g = int(np.floor((1 - alpha) * N + 0.5))
    X2 = torch.empty((D, n_g), dtype=torch.float32, device=dev)
    J2 = torch.empty(n_g, dtype=torch.float32, device=dev)
    s.sample(seed, first, X2, J2)
    torch.cuda.synchronize()
    xg, jg = X.cpu().numpy().T.astype(np.float64), J.cpu().numpy().astype(np.float64)
    ug, lqg = Uo.cpu().numpy().T.astype(np.float64), LQ.cpu().numpy().astype(np.float64)
    # the grid's share: the sampler's own points, weighted by the mixture at the flow's density there
    assert np.array_equal(xg[:n_g], X2.cpu().numpy().T)
    u, _ = osp.uniforms(seed, first, n_g, D)
    assert np.max(np.abs(ug[:n_g] - u)) < 1e-7
    lq_ref = ofl.log_q(th, m, u)
    assert np.median(np.abs(lqg[:n_g] - lq_ref)) < 1e-4 and np.max(np.abs(lqg[:n_g] - lq_ref)) < 5e-3
    # the weight from the oracle's grid map and flow density (the BF16 error of log q enters it at most once)
    g32 = grid.astype(np.float32).astype(np.float64)
    _, mw = osp.uniforms(seed, first, n_g, D)
    yg, jv_g, _ = osp.vegas_map_int(mw, g32)
    _, jp_g = ig.physical_map(yg, n, BETA, 6.0)
    lerr = np.abs(np.log(jg[:n_g]) - np.log(ofl.mixture_weight(jp_g * jv_g, lq_ref, alpha)))
    assert np.median(lerr) < 1e-4 and lerr.max() < 6e-3, (np.median(lerr), lerr.max())
    # the flow's share: counters first + n_g onwards through the flow
    uf, _ = osp.uniforms(seed, first + n_g, N - n_g, D)
    up, lq, _ = ofl.sample(th, m, uf)
    assert np.max(np.abs(ug[n_g:] - up)) < 2e-3
    assert np.median(np.abs(lqg[n_g:] - lq)) < 1e-4 and np.max(np.abs(lqg[n_g:] - lq)) < 5e-3
    _flow_share_matches(xg[n_g:], jg[n_g:], ug[n_g:], up, lq, g32, n, alpha, 0.0)
    _maps_on_gpu_points(xg[n_g:], jg[n_g:], ug[n_g:], lqg[n_g:], g32, n, alpha, 0.0)
    # bounded weights: never above the grid's own weight / (1 - alpha)
    assert np.all(jg[:n_g] <= jp_g * jv_g / (1 - alpha) * (1 + 1e-4))


def test_trained_flow_integral_unbiased_and_lower_variance():
    from oracle import physics as ph
    torch, dev = torch_dev()
    n, D = 2, 7
    inst = [(BETA, 1.0, 1.0, ph.coupling(1.0))]
    ks = np.linspace(0.0, 2.0, 8).astype(np.float32)
    g = dmc.Graph(n)
    mv, ev = dmc.integrate(g, inst, ks, 1 << 20, iters=4, adapt=6, seed=21)
    masks = synth.flow_masks(D, L, 5)
    f = dmc.Flow(D, masks)
    f.set_params(synth.flow_params(masks, 6, last_scale=0.0))
    # the flow is kept whatever its cost per point (fallback=None): this checks its estimate, not the choice
    mf, ef = dmc.integrate(g, inst, ks, 1 << 20, iters=4, adapt=6, seed=21, flow=f, flow_alpha=0.9,
                           train=dict(epochs=5, steps=16, minibatch=1 << 16, lr=1e-3), fallback=None)
    z = (mv[0, 0].real - mf[0, 0].real) / np.hypot(ev[0, 0].real, ef[0, 0].real)
    ratio = (ev[0, 0].real / ef[0, 0].real) ** 2
    print("z", np.round(z, 2), "variance ratio", np.round(ratio, 2))
    assert np.all(np.abs(z) < 4.5)
    assert np.mean(ratio) > 2.0


@pytest.mark.parametrize("first", [414480 - 3, 414480 - 12, 2655605 - 12])
def test_extreme_base_words_stay_finite(first):
    # Philox(seed 0x2403) gives the 24-bit word 2^24 - 1 at sample 414480 (dimension 1) and the
    # word 0 at sample 2655605 (dimension 11): u = 1 - 2^-25 rounds to 1 in FP32, but the logit
    # of the base point must stay finite and equal the oracle's; with alpha = 1/2 of 16 samples the
    # first offset puts the sample in the grid's share, the other two in the flow's share
    torch, dev = torch_dev()
    D, n, N, seed = 15, 4, 16, 0x2403
    _, mw = osp.uniforms(seed, first, N, D)
    assert np.any(mw == 0xFFFFFF) or np.any(mw == 0)
    f, m, th = _flow(D, scale=0.03, seed=3)
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    s.set_grid(synth.vegas_grid(D, 50, seed=1).astype(np.float64))
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    LQ = torch.empty(N, dtype=torch.float32, device=dev)
    f.sample(s, seed, first, X, J, lq_out=LQ, alpha=0.5)
    torch.cuda.synchronize()
    lqg = LQ.cpu().numpy().astype(np.float64)
    assert torch.isfinite(X).all() and torch.isfinite(J).all() and np.isfinite(lqg).all()
    u, _ = osp.uniforms(seed, first, N, D)
    lq_grid = ofl.log_q(th, m, u[:8])
    _, lq_flow, _ = ofl.sample(th, m, u[8:])
    assert np.max(np.abs(lqg - np.concatenate([lq_grid, lq_flow]))) < 5e-3


def test_three_way_mixture_matches_oracle():
    torch, dev = torch_dev()
    D, n, N = 11, 3, 3001
    a_f, a_u = 0.7, 0.2
    f, m, th = _flow(D, scale=0.03, seed=2)
    seed, first = 0x7717, 5 << 20
    s = dmc.Sampler(dmc.SAMPLER_VEGAS, n, n_bins=50)
    grid = synth.vegas_grid(D, 50, seed=6).astype(np.float64)
    s.set_grid(grid)
    g32 = grid.astype(np.float32).astype(np.float64)
    X = torch.empty((D, N), dtype=torch.float32, device=dev)
    J = torch.empty(N, dtype=torch.float32, device=dev)
    Uo = torch.empty((D, N), dtype=torch.float32, device=dev)
    LQ = torch.empty(N, dtype=torch.float32, device=dev)
    f.sample(s, seed, first, X, J, u_out=Uo, lq_out=LQ, alpha=a_f, uniform=a_u)
    n_u = int(np.floor(a_u * N + 0.5))
    n_g = int(np.floor((1 - a_f - a_u) * N + 0.5))
    X2 = torch.empty((D, n_g), dtype=torch.float32, device=dev)
    J2 = torch.empty(n_g, dtype=torch.float32, device=dev)
    s.sample(seed, first + n_u, X2, J2)
    torch.cuda.synchronize()
    xg, jg = X.cpu().numpy().T.astype(np.float64), J.cpu().numpy().astype(np.float64)
    ug, lqg = Uo.cpu().numpy().T.astype(np.float64), LQ.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(jg)) and np.all(jg >= 0)
    # uniform share: y = the uniform sampler's points, u' = G^-1(y), weight by the mixture
    y, _ = osp.uniforms(seed, first, n_u, D)
    y32 = y.astype(np.float32).astype(np.float64)
    xr, Jp = ig.physical_map(y32, n, BETA, 6.0)
    assert np.allclose(xg[:n_u], xr, rtol=0, atol=6.0 * 1e-5)
    ur, jv_u = osp.vegas_inverse(y32, g32)
    assert np.max(np.abs(ug[:n_u] - ur)) < 2e-6
    lq_u = ofl.log_q(th, m, ur)
    assert np.median(np.abs(lqg[:n_u] - lq_u)) < 1e-4 and np.max(np.abs(lqg[:n_u] - lq_u)) < 5e-3
    lerr = np.abs(np.log(jg[:n_u]) - np.log(ofl.mixture_weight(Jp * jv_u, lq_u, a_f, a_u, jv_u)))
    assert np.median(lerr) < 1e-4 and lerr.max() < 6e-3, (np.median(lerr), lerr.max())
    assert np.all(jg[:n_u] <= Jp / a_u * (1 + 1e-4))
    # grid share: the sampler's own points, weighted by the mixture
    sl = slice(n_u, n_u + n_g)
    assert np.array_equal(xg[sl], X2.cpu().numpy().T)
    u, mw = osp.uniforms(seed, first + n_u, n_g, D)
    yg, jv_g, _ = osp.vegas_map_int(mw, g32)
    _, jp_g = ig.physical_map(yg, n, BETA, 6.0)
    lq_ref = ofl.log_q(th, m, u)
    assert np.median(np.abs(lqg[sl] - lq_ref)) < 1e-4 and np.max(np.abs(lqg[sl] - lq_ref)) < 5e-3
    lerr = np.abs(np.log(jg[sl]) - np.log(ofl.mixture_weight(jp_g * jv_g, lq_ref, a_f, a_u, jv_g)))
    assert np.median(lerr) < 1e-4 and lerr.max() < 6e-3, (np.median(lerr), lerr.max())
    # flow share
    fs = slice(n_u + n_g, N)
    uf, _ = osp.uniforms(seed, first + n_u + n_g, N - n_u - n_g, D)
    up, lq, _ = ofl.sample(th, m, uf)
    assert np.max(np.abs(ug[fs] - up)) < 2e-3
    assert np.median(np.abs(lqg[fs] - lq)) < 1e-4 and np.max(np.abs(lqg[fs] - lq)) < 5e-3
    _flow_share_matches(xg[fs], jg[fs], ug[fs], up, lq, g32, n, a_f, a_u)


def test_integrate_falls_back_to_vegas():
    """An untrained (identity) flow has the grid's variance at a higher cost per point, so the probe's gain is
    below 1 and integrate() draws from the grid: its estimate is then bit for bit the flow-free one.  With the
    bar at 0 the flow is kept."""
    n = 2
    D = dmc.dim(n)
    ks = [0.5, 1.0]
    inst = [(BETA, 1.0, 1.0, dmc.coupling(1.0))]
    g = dmc.Graph(n)
    f = dmc.Flow(D, synth.flow_masks(D, L, 3))
    rep = {}
    m1, e1 = dmc.integrate(g, inst, ks, 1 << 16, iters=3, adapt=2, seed=9, flow=f, report=rep)
    print(rep)
    assert rep["proposal"] == "vegas" and rep["gain"] < 1 and rep["switched_at"] is None
    m0, e0 = dmc.integrate(g, inst, ks, 1 << 16, iters=3, adapt=2, seed=9)
    assert np.array_equal(m1, m0) and np.array_equal(e1, e0)
    rep = {}
    m2, _ = dmc.integrate(g, inst, ks, 1 << 16, iters=3, adapt=2, seed=9, flow=f, fallback=0.0, report=rep)
    assert rep["proposal"] == "flow" and not np.array_equal(m2, m0)
