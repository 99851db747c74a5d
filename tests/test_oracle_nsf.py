"""Pins of the oracle neural spline flow (oracle/nsf.py): spline identities, the flow density against a
brute-force Jacobian determinant and its normalisation, and the autograd gradient against finite
differences."""
import numpy as np
import pytest

from oracle import nsf

K = nsf.K_BINS


def _rand_theta(rng, N, scale=1.5):
    return rng.normal(size=(N, 3 * K - 1)) * scale


def test_spline_endpoints_monotonic_and_inverse():
    rng = np.random.default_rng(1)
    N = 4000
    th = _rand_theta(rng, N)
    v = rng.uniform(size=N)
    y, ld = nsf.spline_forward(v, th)
    x, ld_inv = nsf.spline_inverse(y, th)
    assert np.allclose(x, v, atol=1e-12)
    assert np.allclose(ld, ld_inv, atol=1e-9)
    for e in (0.0, 1.0):
        ye, _ = nsf.spline_forward(np.full(N, e), th)
        assert np.allclose(ye, e, atol=1e-14)
    grid = np.linspace(0, 1, 513)
    th1 = np.repeat(th[:1], len(grid), axis=0)
    yy, _ = nsf.spline_forward(grid, th1)
    assert np.all(np.diff(yy) > 0)


def test_spline_log_derivative_against_finite_differences():
    rng = np.random.default_rng(2)
    N = 500
    th = _rand_theta(rng, N)
    v = rng.uniform(0.01, 0.99, size=N)
    h = 1e-6
    yp, _ = nsf.spline_forward(v + h, th)
    ym, _ = nsf.spline_forward(v - h, th)
    _, ld = nsf.spline_forward(v, th)
    fd = (yp - ym) / (2 * h)
    # a few points sit within h of a knot, where the one-sided pieces differ at second order
    assert np.mean(np.abs(np.exp(ld) - fd) <= 1e-5 * fd) > 0.98


def test_identity_parameters_give_the_identity_flow():
    masks = [[1, 0, 1], [0, 1, 0], [1, 1, 0]]
    params = nsf.identity_params(masks)
    z = np.random.default_rng(3).uniform(size=(200, 3))
    u, lq = nsf.forward(z, masks, params)
    assert np.allclose(u, z, atol=1e-12) and np.allclose(lq, 0.0, atol=1e-12)


def _random_flow(D=3, L=3, seed=4, scale=0.4):
    rng = np.random.default_rng(seed)
    masks = []
    for l in range(L):
        m = np.zeros(D, dtype=int)
        m[rng.permutation(D)[: D // 2 + (l % 2)]] = 1
        if m.all():
            m[0] = 0
        if not m.any():
            m[0] = 1
        masks.append(list(m))
    return masks, nsf.identity_params(masks, rng=rng, scale=scale)


def test_flow_density_against_brute_force_jacobian_and_normalisation():
    # a mild flow: central differences with h = 1e-6 need Jacobian columns well above roundoff / h
    masks, params = _random_flow(scale=0.15)
    rng = np.random.default_rng(5)
    z = rng.uniform(0.05, 0.95, size=(40, 3))
    u, lq = nsf.forward(z, masks, params)
    lq_inv, z_back = nsf.log_density(u, masks, params)
    assert np.allclose(z_back, z, atol=1e-10)
    assert np.allclose(lq_inv, lq, atol=1e-9)
    # log q(u) = -log |det du/dz| by central differences of the whole map
    h = 1e-6
    for i in range(len(z)):
        J = np.zeros((3, 3))
        for d in range(3):
            zp, zm = z[i].copy(), z[i].copy()
            zp[d] += h
            zm[d] -= h
            J[:, d] = (nsf.forward(zp[None], masks, params)[0][0] - nsf.forward(zm[None], masks, params)[0][0]) / (2 * h)
        assert abs(-np.log(abs(np.linalg.det(J))) - lq[i]) < 1e-5
    # q is a density on the unit cube: E_uniform[q(u)] = 1
    uu = rng.uniform(size=(200000, 3))
    q = np.exp(nsf.log_density(uu, masks, params)[0])
    assert abs(q.mean() - 1.0) < 5 * q.std() / np.sqrt(len(q))


def test_torch_gradient_against_finite_differences():
    masks, params = _random_flow(D=4, L=2, seed=6, scale=0.3)
    rng = np.random.default_rng(7)
    u = rng.uniform(0.02, 0.98, size=(64, 4))
    w = rng.uniform(0.1, 2.0, size=64)
    L, g, lq = nsf.loss_and_grad_torch(u, w, masks, params)
    assert np.allclose(lq, nsf.log_density(u, masks, params)[0], atol=1e-10)
    assert np.isclose(L, -(w * lq).sum() / w.sum())
    for trial in range(6):
        dirn = rng.normal(size=params.shape)
        h = 1e-6
        Lp = -(w * nsf.log_density(u, masks, params + h * dirn)[0]).sum() / w.sum()
        Lm = -(w * nsf.log_density(u, masks, params - h * dirn)[0]).sum() / w.sum()
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g @ dirn) <= 1e-5 * (abs(fd) + 1e-3), (trial, fd, g @ dirn)
