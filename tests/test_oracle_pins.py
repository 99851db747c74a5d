"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test targets a plausible mistake in the oracle: a wrong propagator branch or sign, a
dropped prefactor, a wrong diagram filter, a broken routing, a wrong derivative, a wrong
random-number generator or map Jacobian.
"""
import math
import os

import numpy as np
import pytest

from oracle import diagrams as dg
from oracle import integrand as ig
from oracle import physics as ph
from oracle import sampler as sp
import synth

BETA, MU, LAM = 25.0, 1.0, 1.0
GAMMA = ph.coupling(1.0)
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ free propagator
@pytest.mark.parametrize("eps", [-0.9, -0.3, 0.0, 0.2, 1.5, 8.0])
def test_G0_antiperiodic(eps):
    tau = np.linspace(0.01, BETA - 0.01, 57)
    assert np.allclose(ph.G0(eps, tau - BETA, BETA), -ph.G0(eps, tau, BETA), rtol=1e-13, atol=0)


@pytest.mark.parametrize("eps", [-0.5, 0.0, 0.7])
def test_G0_jump_is_one(eps):
    # G0(0^-) - G0(0^+) = 1 (equal-time anticommutator)
    assert abs(ph.G0(eps, 0.0, BETA) - ph.G0(eps, 1e-13, BETA) - 1.0) < 1e-10


@pytest.mark.parametrize("eps,n", [(0.3, 0), (-0.7, 2), (0.0, 1), (2.0, -1)])
def test_G0_matsubara_transform(eps, n):
    # int_0^beta e^{i w_n tau} G0(tau) dtau = 1/(i w_n - eps) (eq. propagator in frequency)
    w = (2 * n + 1) * math.pi / BETA
    assert abs(ph.matsubara_of_G0(eps, BETA, n) - 1.0 / (1j * w - eps)) < 1e-11


def test_dG0_dmu_is_minus_convolution():
    # d/dmu G0 = -G0 * G0 (tau convolution with antiperiodic extension): in frequency
    # d/dmu 1/(i w - k^2 + mu) = -1/(i w - eps)^2.
    eps = 0.35
    x, wt = np.polynomial.legendre.leggauss(200)
    for tau in [0.7, 5.0, 19.0, -3.0]:
        tot = 0.0
        # split [0, beta] at tau (kink of G0(tau - tau'))
        cuts = sorted(set([0.0, BETA] + ([tau] if 0 < tau < BETA else [tau + BETA] if tau < 0 else [])))
        for a, b in zip(cuts[:-1], cuts[1:]):
            t = 0.5 * (b - a) * x + 0.5 * (a + b)
            d = tau - t
            d = np.where(d <= -BETA, d + 2 * BETA, d)
            d = np.where(d > BETA, d - 2 * BETA, d)
            g1 = ph.G0(eps, d, BETA)
            g1 = np.where(np.abs(d) >= BETA, -ph.G0(eps, d - np.sign(d) * BETA, BETA), g1)
            tot += np.sum(0.5 * (b - a) * wt * g1 * ph.G0(eps, t, BETA))
        assert abs(ph.dG0_dmu(eps, tau, BETA) + tot) < 1e-9


# ------------------------------------------------------------------ Fock closed forms
@pytest.mark.parametrize("k", [0.0, 0.3, 0.999, 1.7, 3.0])
def test_fock_T0_limits(k):
    # the finite-T 1D integral at large beta approaches the T = 0 elementary forms
    g = GAMMA
    assert abs(ph.fock_finite_T(k, 4000.0, 1.0, LAM, g) - ph.fock_T0_yukawa(k, LAM, g)) < 2e-6
    assert abs(ph.fock_finite_T(k, 4000.0, 1.0, 1e-10, g) - ph.fock_T0_coulomb(k, g)) < 5e-5


def _tensor_quad_order1(k, nr=96, nc=64, nphi=8):
    """Integrate the oracle's order-1 integrand over the ball |q| <= 6 by tensor Gauss-Legendre
    in (r, cos theta, phi), with r panels split at the Fermi surface."""
    xr, wr = np.polynomial.legendre.leggauss(nr)
    xc, wc = np.polynomial.legendre.leggauss(nc)
    rs, ws = [], []
    for a, b in [(0.0, 0.9), (0.9, 1.0), (1.0, 1.1), (1.1, 2.0), (2.0, 6.0)]:
        rs.append(0.5 * (b - a) * xr + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wr)
    r = np.concatenate(rs)
    w_r = np.concatenate(ws)
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    R, C, P = np.meshgrid(r, xc, phi, indexing="ij")
    W = (w_r[:, None, None] * wc[None, :, None] * (2 * math.pi / nphi)) * R * R
    S = np.sqrt(1 - C * C)
    x = np.stack([R * S * np.cos(P), R * S * np.sin(P), R * C], axis=-1).reshape(-1, 3)
    f = ig.integrand(x, 1, k, BETA, MU, LAM, GAMMA)
    return np.sum(W.reshape(-1) * f)


@pytest.mark.parametrize("k", [0.0, 0.5, 1.0, 2.5])
def test_order1_integrand_matches_fock(k):
    # the oracle's order-1 diagram, integrated deterministically, equals the hand-derived
    # Fock integral: pins the sign (-1)^(n+F), (2 pi)^-3, 8 pi gamma and the equal-time nF.
    val = _tensor_quad_order1(k)
    ref = ph.fock_finite_T(k, BETA, MU, LAM, GAMMA)
    assert abs(val.imag) == 0.0          # Im Sigma^(1) = 0 exactly (instantaneous diagram)
    assert abs(val.real - ref) < 1e-7 * abs(ref)


def test_fock_derivatives_match_quadrature_of_duals():
    # d/dmu, d/dlambda, d/dk of the oracle's dual-number integrand, integrated over the ball,
    # equal the closed-form 1D integrals of the differentiated Fock integrand.
    k = 0.8
    xr, wr = np.polynomial.legendre.leggauss(96)
    xc, wc = np.polynomial.legendre.leggauss(64)
    rs, ws = [], []
    for a, b in [(0.0, 0.9), (0.9, 1.0), (1.0, 1.1), (1.1, 2.0), (2.0, 6.0)]:
        rs.append(0.5 * (b - a) * xr + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * wr)
    r = np.concatenate(rs)
    w_r = np.concatenate(ws)
    R, C = np.meshgrid(r, xc, indexing="ij")
    W = (w_r[:, None] * wc[None, :] * 2 * math.pi) * R * R
    S = np.sqrt(1 - C * C)
    x = np.stack([R * S, 0 * R, R * C], axis=-1).reshape(-1, 3)
    v, dmu, dlam, dk = ig.diagram_values_dual(x, 1, k, BETA, MU, LAM, GAMMA)
    got = [np.sum(W.reshape(-1) * a[0]).real for a in (dmu, dlam, dk)]
    ref = ph.fock_derivs_finite_T(k, BETA, MU, LAM, GAMMA)
    for g_, r_ in zip(got, ref):
        assert abs(g_ - r_) < 2e-6 * max(1.0, abs(r_))


# ------------------------------------------------------------------ diagram set
@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_counts_obey_dyson(n):
    # G = G0 + G0 Sigma G (eq. Dyson): every tadpole-free connected Green's-function diagram
    # is a unique chain of 1PI self-energy insertions, so g_n = sum_i s_i g_{n-i}, g_0 = 1.
    s = [None] + [len(dg.enumerate_topologies(m)[0]) for m in range(1, n + 1)]
    g = [1] + [len(dg.enumerate_topologies(m, dg.is_green_diagram)[0]) for m in range(1, n + 1)]
    assert g[n] == sum(s[i] * g[n - i] for i in range(1, n + 1))


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_labelled_count_is_topologies_times_relabellings(n):
    # fixing the in-vertex leaves no automorphism, so each topology has exactly
    # (n-1)! 2^(n-1) labelled forms (permute lines 1..n-1, swap their ends)
    tops, nlab = dg.enumerate_topologies(n)
    assert nlab == len(tops) * math.factorial(n - 1) * 2 ** (n - 1)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_routing_conserves_momentum_and_no_zero_lines(n):
    for d in dg.sigma_diagrams(n):
        assert dg.check_conservation(d)
        for ln in d.lines:
            assert any(ln.mom), "a line with zero momentum means a tadpole slipped through"
        assert len(d.chords) == n


def test_order2_set_and_signs():
    # n = 2 without tadpoles: rainbow (F=0), second-order exchange (F=0), bubble (F=1)
    ds = dg.sigma_diagrams(2)
    assert sorted((d.n_loops_f, d.weight) for d in ds) == [(0, 1.0), (0, 1.0), (1, -2.0)]


def test_rainbow_time_integral():
    # The n = 2 rainbow (Fock insertion inside Fock) has, at fixed momenta, the time integral
    # int_0^beta dtau G0(p, tau) G0(p, -tau) = d nF / d eps_p = -beta nF (1 - nF), so its
    # integrand integrated over tau_1 equals (2pi)^-6 V(k-p) V(p-q) nF(q) dnF/deps(p): the
    # first-order term of -int V nF(eps + Sigma_x) in Sigma_x.
    rb = [d for d in dg.sigma_diagrams(2)
          if d.n_loops_f == 0 and d.ext_line == 0 and
          any(l.kind == "G" and l.src // 2 == l.dst // 2 for l in d.lines)]
    assert len(rb) == 1
    d = rb[0]
    xg, wg = np.polynomial.legendre.leggauss(120)
    rng = np.random.default_rng(3)
    for trial in range(4):
        q0 = rng.normal(size=3) * 0.6
        q1 = rng.normal(size=3) * 0.6
        k = 0.4 + trial * 0.5
        tot = 0.0
        for a, b in [(0, 1), (1, 5), (5, 25)]:
            t = 0.5 * (b - a) * xg + 0.5 * (a + b)
            x = np.zeros((len(t), 7))
            x[:, 0:3] = q0
            x[:, 3:6] = q1
            x[:, 6] = t
            tot += np.sum(0.5 * (b - a) * wg * ig.diagram_values(x, 2, k, BETA, MU, LAM, GAMMA, [d])[0])
        # the momenta of the lines from the diagram's own routing: both outer propagators carry p,
        # the equal-time one q
        kv = np.array([0.0, 0.0, k])

        def mom(ln):
            return ln.mom[0] * q0 + ln.mom[1] * q1 + ln.mom[2] * kv

        outer = [l for l in d.lines if l.kind == "G" and l.src // 2 != l.dst // 2]
        inner = [l for l in d.lines if l.kind == "G" and l.src // 2 == l.dst // 2]
        assert len(outer) == 2 and len(inner) == 1
        p, q = mom(outer[0]), mom(inner[0])
        assert np.allclose(np.abs(mom(outer[1])), np.abs(p))
        ep = p @ p - MU
        n_p = ph.nF(ep, BETA)
        vv = np.prod([ph.V(np.sum(mom(l) ** 2), LAM, GAMMA) for l in d.lines if l.kind == "V"])
        ref = (2 * math.pi) ** -6 * vv * ph.nF(q @ q - MU, BETA) * (-BETA * n_p * (1 - n_p))
        assert abs(tot - ref) < 1e-10 * abs(ref) + 1e-300


@pytest.mark.parametrize("n", [2, 3])
def test_dual_derivatives_match_central_differences(n):
    x = synth.loop_points(n, 64, seed=7).astype(np.float64)
    # h small enough that the O(h^2) truncation with log-derivatives of order beta is negligible
    k, h = 0.9, 1e-6
    v, dmu, dlam, dk = (a.sum(axis=0) for a in ig.diagram_values_dual(x, n, k, BETA, MU, LAM, GAMMA))
    A = ig.abs_sum(x, n, k, BETA, MU, LAM, GAMMA)
    f = lambda **kw: ig.integrand(x, n, kw.get("k", k), BETA, kw.get("mu", MU), kw.get("lam", LAM), GAMMA)
    fd_mu = (f(mu=MU + h) - f(mu=MU - h)) / (2 * h)
    fd_lam = (f(lam=LAM + h) - f(lam=LAM - h)) / (2 * h)
    fd_k = (f(k=k + h) - f(k=k - h)) / (2 * h)
    for got, fd, scale in [(dmu, fd_mu, BETA), (dlam, fd_lam, 1.0), (dk, fd_k, BETA)]:
        assert np.all(np.abs(got - fd) <= 2e-7 * scale * A + 1e-300)


# ------------------------------------------------------------------ sampler pieces
def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = sp.philox4x32_10(np.array([v[0:4]], dtype=np.uint64), np.array([v[4:6]], dtype=np.uint64))[0]
        assert [int(o) for o in out] == v[6:10]


def test_vegas_map_integrates_one_and_uniform_grid_is_identity():
    D, B = 3, 50
    e = synth.vegas_grid(D, B, seed=1).astype(np.float64)
    # exact: the mean of J_V over one point per (bin, fraction) cell is sum_b (e_{b+1}-e_b) = 1
    m = np.arange(0, 1 << 24, 4099, dtype=np.int64)[:, None].repeat(D, axis=1)
    y, J, b = sp.vegas_map_int(m, e)
    assert np.all((y >= 0) & (y <= 1))
    u = (m + 0.5) * 2.0 ** -24
    assert np.all(b == np.floor(u * B).astype(np.int64))
    assert abs(np.mean(np.sum(np.diff(e, axis=1), axis=1)) - 1.0) < 1e-7
    uni = np.tile(np.linspace(0, 1, B + 1), (D, 1))
    y, J, _ = sp.vegas_map_int(m, uni)
    assert np.allclose(y, u, atol=1e-15) and np.allclose(J, 1.0, atol=1e-12)


def test_vegas_map_jacobian_is_derivative():
    # J_V is dy/du: compare with a difference quotient inside one bin
    D, B = 2, 50
    e = synth.vegas_grid(D, B, seed=4).astype(np.float64)
    m = np.array([[1000, 5_000_000], [9_000_000, 16_000_000]], dtype=np.int64)
    y0, J0, _ = sp.vegas_map_int(m, e)
    y1, _, _ = sp.vegas_map_int(m + 1, e)
    dq = np.prod((y1 - y0) / 2.0 ** -24, axis=1)
    assert np.allclose(dq, J0, rtol=1e-6)


def test_refine_keeps_uniform_on_flat_histogram_and_equalises_weight():
    D, B = 2, 50
    uni = np.tile(np.linspace(0, 1, B + 1), (D, 1))
    new = sp.refine_grid(uni, np.ones((D, B)))
    assert np.allclose(new, uni, atol=1e-14)
    h = synth.histogram(D, B, seed=9)
    e = synth.vegas_grid(D, B, seed=2).astype(np.float64)
    ne = sp.refine_grid(e, h)
    assert np.all(np.diff(ne, axis=1) > 0) and np.all(ne[:, 0] == 0) and np.all(ne[:, -1] == 1)
    # the compressed, smoothed weight, spread uniformly inside each old bin, is equal in every new bin
    for d in range(D):
        s = np.empty(B)
        s[0] = (h[d, 0] + h[d, 1]) / 2
        s[-1] = (h[d, -2] + h[d, -1]) / 2
        s[1:-1] = (h[d, :-2] + h[d, 1:-1] + h[d, 2:]) / 3
        r = s / s.sum()
        w = ((1 - r) / np.log(1 / r)) ** 0.5
        dens = w / np.diff(e[d])
        cdf = lambda z: np.interp(z, e[d], np.concatenate([[0], np.cumsum(w)]))
        mass = np.diff(cdf(ne[d]))
        assert np.allclose(mass, w.sum() / B, rtol=1e-9)


def test_physical_map_jacobian_is_determinant():
    # J of the unit-cube -> (ball x [0,beta)^(n-1)) map equals |det dx/dy| by central differences
    n = 2
    rng = np.random.default_rng(5)
    y = rng.uniform(0.05, 0.95, size=(6, ig.dim(n)))
    x, J = ig.physical_map(y, n, BETA, 6.0)
    h = 1e-6
    for i in range(len(y)):
        M = np.empty((ig.dim(n), ig.dim(n)))
        for c in range(ig.dim(n)):
            yp = y[i:i + 1].copy(); yp[0, c] += h
            ym = y[i:i + 1].copy(); ym[0, c] -= h
            M[:, c] = (ig.physical_map(yp, n, BETA, 6.0)[0][0] - ig.physical_map(ym, n, BETA, 6.0)[0][0]) / (2 * h)
        assert abs(abs(np.linalg.det(M)) - J[i]) < 1e-6 * J[i]


def test_uniform_map_mean_jacobian_is_volume():
    # int_[0,1]^D J dy = ((4/3) pi R^3)^n beta^(n-1)
    n, R = 2, 6.0
    x1, w1 = np.polynomial.legendre.leggauss(8)
    u = 0.5 * (x1 + 1)
    grid = np.stack(np.meshgrid(*([u] * ig.dim(n)), indexing="ij"), -1).reshape(-1, ig.dim(n))
    wt = np.prod(np.stack(np.meshgrid(*([0.5 * w1] * ig.dim(n)), indexing="ij"), -1).reshape(-1, ig.dim(n)), axis=1)
    _, J = ig.physical_map(grid, n, BETA, R)
    assert abs(np.sum(wt * J) / ((4 / 3 * math.pi * R ** 3) ** n * BETA ** (n - 1)) - 1) < 1e-12
