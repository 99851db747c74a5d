"""Pins of the oracle flow: invertibility, both density routes, the log-determinant against a
brute-force Jacobian determinant, the hand-written gradient against torch autograd and central
differences, normalisation."""
import contextlib

import numpy as np
import pytest

import synth
from oracle import flow as fl


@contextlib.contextmanager
def smooth():
    old = fl.EMULATE_BF16
    fl.EMULATE_BF16 = False
    try:
        yield
    finally:
        fl.EMULATE_BF16 = old


D, L = 7, 8


def _setup(scale=0.03, seed=1):
    m = synth.flow_masks(D, L, seed)
    th = synth.flow_params(m, seed + 1, last_scale=scale).astype(np.float64)
    return m, th


def test_masks_alternate_and_cover():
    m = synth.flow_masks(15, 8, 3)
    for l in range(0, 8, 2):
        assert np.all(m[l] + m[l + 1] == 1)
    assert np.all((m.sum(axis=1) >= 7) & (m.sum(axis=1) <= 8))


def test_inverse_undoes_forward_and_densities_agree():
    m, th = _setup()
    u = np.random.default_rng(0).uniform(0.02, 0.98, size=(200, D))
    up, lq_fwd, zK = fl.sample(th, m, u)
    z0, _ = fl.inverse(th, m, zK)
    assert np.allclose(z0, fl.logit(u), atol=1e-9)
    ok = np.all(np.abs(zK) < 25, axis=1)           # outputs that do not round to 0 or 1
    assert ok.mean() > 0.9
    assert np.allclose(fl.log_q(th, m, up[ok]), lq_fwd[ok], atol=1e-7)


def test_identity_flow_is_uniform():
    m, th = _setup(scale=0.0)
    u = np.random.default_rng(1).uniform(size=(100, D))
    up, lq, _ = fl.sample(th, m, u)
    assert np.allclose(up, u, atol=1e-12) and np.allclose(lq, 0.0, atol=1e-12)


def test_log_density_is_minus_log_abs_det_jacobian():
    # q(u') = 1 / |det du'/du| for a uniform base: brute-force D x D determinant
    with smooth():
        m, th = _setup()
        rng = np.random.default_rng(2)
        h = 1e-6
        for _ in range(5):
            u = rng.uniform(0.1, 0.9, size=(1, D))
            Jm = np.empty((D, D))
            for c in range(D):
                up_ = u.copy(); up_[0, c] += h
                dn_ = u.copy(); dn_[0, c] -= h
                Jm[:, c] = (fl.sample(th, m, up_)[0][0] - fl.sample(th, m, dn_)[0][0]) / (2 * h)
            lq = fl.sample(th, m, u)[1][0]
            assert abs(lq + np.log(abs(np.linalg.det(Jm)))) < 1e-6


def test_density_normalised():
    with smooth():
        m, th = _setup(scale=0.03)
        up = np.random.default_rng(3).uniform(size=(1 << 16, D))
        q = np.exp(fl.log_q(th, m, up))
        assert abs(q.mean() - 1.0) < 4 * q.std() / np.sqrt(len(q))


def _torch_loss(th, m, up, w):
    import torch
    t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    zK = torch.logit(torch.tensor(up, dtype=torch.float64))
    z = zK.clone()
    ssum = torch.zeros(z.shape[0], dtype=torch.float64)
    o = 0
    lay = []
    for _ in range(len(m)):
        W1t = t[o:o + 2048].view(128, 16); o += 2048
        W2t = t[o:o + 16384].view(128, 128); o += 16384
        b2 = t[o:o + 128]; o += 128
        W3t = t[o:o + 4096].view(32, 128); o += 4096
        b3 = t[o:o + 32]; o += 32
        lay.append((W1t, W2t, b2, W3t, b3))
    for l in reversed(range(len(m))):
        A = np.nonzero(m[l] == 1)[0]; B = np.nonzero(m[l] == 0)[0]
        W1t, W2t, b2, W3t, b3 = lay[l]
        X1 = torch.cat([torch.sigmoid(z[:, A]), torch.ones(z.shape[0], 1, dtype=torch.float64),
                        torch.zeros(z.shape[0], 16 - len(A) - 1, dtype=torch.float64)], dim=1)
        H1 = torch.relu(X1 @ W1t.T)
        H2 = torch.relu(H1 @ W2t.T + b2)
        O = H2 @ W3t.T + b3
        s = 2.0 * torch.tanh(O[:, :len(B)])
        tt = O[:, 16:16 + len(B)]
        zn = z.clone()
        zn[:, B] = (z[:, B] - tt) * torch.exp(-s)
        z = zn
        ssum = ssum + s.sum(dim=1)
    lsp = lambda v: -v.abs() - 2 * torch.log1p(torch.exp(-v.abs()))
    lq = lsp(z).sum(dim=1) - ssum - lsp(zK).sum(dim=1)
    wn = torch.tensor(w / w.sum(), dtype=torch.float64)
    loss = -(wn * lq).sum()
    loss.backward()
    return loss.item(), t.grad.numpy()


def test_hand_written_gradient_matches_autograd_and_differences():
    with smooth():
        m, th = _setup(scale=0.03, seed=5)
        rng = np.random.default_rng(4)
        up = rng.uniform(0.05, 0.95, size=(64, D))
        w = rng.exponential(size=64)
        loss, g = fl.loss_and_grad(th, m, up, w)
        tl, tg = _torch_loss(th, m, up, w)
        assert abs(loss - tl) < 1e-12 * max(1, abs(tl))
        assert np.allclose(g, tg, rtol=1e-9, atol=1e-12 * np.abs(tg).max())
        # and a few central differences of the loss itself
        idx = rng.choice(len(th), size=6, replace=False)
        for i in idx:
            e = np.zeros_like(th); e[i] = 1e-6
            lp, _ = fl.loss_and_grad(th + e, m, up, w)
            lm, _ = fl.loss_and_grad(th - e, m, up, w)
            assert abs((lp - lm) / 2e-6 - g[i]) < 1e-6 * max(1.0, abs(g[i]))


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.14159, 65504.0], dtype=np.float64)
    r = fl.bf16(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties to even -> 1
    assert r[0] == 1.0 and r[1] == 1.0 and r[3] == 1.0078125
    assert r[2] == 1.0078125
    assert abs(r[4] - (-3.140625)) < 1e-12


def test_mixture_estimate_unbiased_and_bounded():
    # integral of prod_d 3 u_d^2 over the cube is 1: points from the grid (uniform) and from a
    # strongly non-uniform flow, in the proportions 1 - alpha : alpha, weighted by the mixture
    with smooth():
        m, th = _setup(scale=0.4, seed=4)
        rng = np.random.default_rng(9)
        alpha, N = 0.7, 1 << 15
        n_g = int(round((1 - alpha) * N))
        ug = rng.uniform(size=(n_g, D))
        uf, lqf, _ = fl.sample(th, m, rng.uniform(size=(N - n_g, D)))
        u = np.concatenate([ug, uf])
        lq = np.concatenate([fl.log_q(th, m, ug), lqf])
        w = fl.mixture_weight(np.ones(N), lq, alpha)
        assert w.max() <= 1.0 / (1.0 - alpha) * (1 + 1e-12)
        assert np.exp(lq).std() > 0.3          # the flow is far from the uniform density
        est = np.prod(3 * u ** 2, axis=1) * w
        assert abs(est.mean() - 1.0) < 4 * est.std() / np.sqrt(N)
        # alpha = 1 is plain flow importance sampling; alpha -> 0 the grid alone
        assert np.allclose(fl.mixture_weight(2.0, lq, 1.0), 2.0 * np.exp(-lq))
        assert np.allclose(fl.mixture_weight(2.0, lq, 0.0), 2.0)


def test_three_way_mixture_unbiased_and_bounded():
    # integral of prod_d 3 y_d^2 over the cube (= 1) with a non-uniform VEGAS grid G: points from the
    # uniform density, from the grid (y = G(u'), u' uniform) and from the flow on the grid, in the
    # proportions a_u : a_g : a_f, weighted by the mixture density in grid coordinates
    import synth as sy
    from oracle import sampler as sp
    with smooth():
        m, th = _setup(scale=0.4, seed=4)
        edges = sy.vegas_grid(D, 50, seed=3).astype(np.float64)
        rng = np.random.default_rng(11)
        a_f, a_u, N = 0.6, 0.15, 1 << 15
        n_u, n_g = int(round(a_u * N)), int(round((1 - a_f - a_u) * N))
        y_u = rng.uniform(size=(n_u, D))
        u_u, jv_u = sp.vegas_inverse(y_u, edges)
        u_g = rng.uniform(size=(n_g, D))
        y_g, jv_g, _ = sp.vegas_map_float(u_g.astype(np.float32), edges)
        u_f, lq_f, _ = fl.sample(th, m, rng.uniform(size=(N - n_u - n_g, D)))
        y_f, jv_f, _ = sp.vegas_map_float(u_f.astype(np.float32), edges)
        u_g32 = u_g.astype(np.float32).astype(np.float64)
        lq = np.concatenate([fl.log_q(th, m, u_u), fl.log_q(th, m, u_g32), lq_f])
        jv = np.concatenate([jv_u, jv_g, jv_f])
        y = np.concatenate([y_u, y_g, y_f])
        w = fl.mixture_weight(jv, lq, a_f, a_u, jv)
        assert w.max() <= 1.0 / a_u * (1 + 1e-12)                          # bounded by the uniform share
        assert np.all(w <= jv / (1 - a_f - a_u) * (1 + 1e-12))              # and by the grid share
        est = np.prod(3 * y ** 2, axis=1) * w
        assert abs(est.mean() - 1.0) < 4 * est.std() / np.sqrt(N)
        # a wrong share in the denominator (the flow's alone) biases the same samples
        bad = np.prod(3 * y ** 2, axis=1) * jv * np.exp(-lq)
        assert abs(bad.mean() - 1.0) > 4 * est.std() / np.sqrt(N)


def test_vegas_inverse_round_trip():
    import synth as sy
    from oracle import sampler as sp
    edges = sy.vegas_grid(7, 50, seed=9).astype(np.float64)
    u = np.random.default_rng(2).uniform(size=(5000, 7))
    y, J, _ = sp.vegas_map_float(u.astype(np.float32), edges)
    u2, J2 = sp.vegas_inverse(y, edges)
    assert np.allclose(u2, u.astype(np.float32), atol=1e-6)
    assert np.allclose(J2, J, rtol=1e-9)
