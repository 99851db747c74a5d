"""Pins of the oracle Taylor-mode coefficients (oracle/taylor.py): closed-form derivatives of the leaves,
the first-order coefficients against the dual-number derivatives, and higher and mixed coefficients
of whole diagram sums against finite differences of the plain FP64 integrand."""
import math

import numpy as np
import pytest

from oracle import integrand as ig
from oracle import physics as ph
from oracle import taylor as ty

BETA, MU, LAM = 25.0, 1.0, 1.0
GAMMA = ph.coupling(1.0)


def _series_of(S, v, var=None, dv=1.0):
    s = ty.Series.const(S, np.asarray(v, dtype=np.float64))
    if var is not None:
        s.c[var] = s.c[var] + dv
    return s


def test_index_set_layout():
    S = ty.index_set(2, True, True, True)
    assert S[:6] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 0), (1, 1, 0), (0, 2, 0)]
    assert S[6:] == [(m, l, 1) for (m, l, _) in S[:6]]
    assert ty.index_set(3, True, False, False) == [(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)]
    assert len(ty.index_set(4, True, True, False)) == 15


def test_fermi_function_mu_derivatives_closed_form():
    # equal-time G0 = nF(eps - dmu): d^m/dmu^m nF(p^2 - mu) in closed form for m = 1..3
    S = ty.index_set(3, True, False, False)
    eps0 = np.linspace(-0.9, 0.9, 37)
    eps = _series_of(S, eps0, (1, 0, 0), -1.0)
    g = ty.G0_series(eps, np.zeros_like(eps0), BETA)
    n = ph.nF(eps0, BETA)
    b = BETA
    want = [n, b * n * (1 - n), b ** 2 * n * (1 - n) * (1 - 2 * n), b ** 3 * n * (1 - n) * (1 - 6 * n + 6 * n * n)]
    for m in range(4):
        got = g.c[(m, 0, 0)] * math.factorial(m)
        assert np.allclose(got, want[m], rtol=1e-11, atol=1e-13 * b ** m), m


@pytest.mark.parametrize("tau", [3.7, -11.2, 24.9])
def test_propagator_mu_derivatives_closed_form(tau):
    # G0' = G0 h, G0'' = G0 (h^2 + h'), G0''' = G0 (h^3 + 3 h h' + h'') with h = d ln G0/d mu:
    # h = tau' - beta nF for both branches (tau' = tau or tau + beta), h' = -beta^2 nF (1 - nF),
    # h'' = -beta^3 nF (1 - nF) (1 - 2 nF)
    S = ty.index_set(3, True, False, False)
    eps0 = np.linspace(-0.95, 3.0, 41)
    eps = _series_of(S, eps0, (1, 0, 0), -1.0)
    t = np.full_like(eps0, tau)
    g = ty.G0_series(eps, t, BETA)
    g0 = ph.G0(eps0, t, BETA)
    n = ph.nF(eps0, BETA)
    tp = tau if tau > 0 else tau + BETA
    h = tp - BETA * n
    h1 = -BETA ** 2 * n * (1 - n)
    h2 = -BETA ** 3 * n * (1 - n) * (1 - 2 * n)
    want = [g0, g0 * h, g0 * (h * h + h1), g0 * (h ** 3 + 3 * h * h1 + h2)]
    for m in range(4):
        got = g.c[(m, 0, 0)] * math.factorial(m)
        scale = np.abs(g0) * (abs(tp) + BETA) ** m
        assert np.all(np.abs(got - want[m]) <= 1e-10 * scale + 1e-300), m


def test_interaction_lambda_series_closed_form():
    # V(lambda + dlam) = 8 pi gamma / (p^2 + lambda) sum_l (-dlam / (p^2 + lambda))^l
    S = ty.index_set(4, False, True, False)
    p2v = np.linspace(0.0, 20.0, 33)
    v = ty.V_series(_series_of(S, p2v), LAM, GAMMA)
    base = 8 * math.pi * GAMMA / (p2v + LAM)
    for l in range(5):
        assert np.allclose(v.c[(0, l, 0)], base * (-1.0 / (p2v + LAM)) ** l, rtol=1e-13)


@pytest.mark.parametrize("n", [2, 3])
def test_first_order_coefficients_equal_dual_derivatives(n):
    rng = np.random.default_rng(10 + n)
    x, _ = ig.physical_map(rng.uniform(size=(64, ig.dim(n))), n, BETA, 6.0)
    k = 0.8
    val, dmu, dlam, dk = (a.sum(axis=0) for a in ig.diagram_values_dual(x, n, k, BETA, MU, LAM, GAMMA))
    roots = dict(ty.derivative_roots(x, n, k, BETA, MU, LAM, GAMMA, 1, True, True, True))
    scale = np.abs(ig.diagram_values_dual(x, n, k, BETA, MU, LAM, GAMMA, absolute=True)[0]).sum(axis=0)
    for key, ref, mult in [((0, 0, 0), val, 1.0), ((1, 0, 0), dmu, BETA), ((0, 1, 0), dlam, 1.0),
                           ((0, 0, 1), dk, 10.0)]:
        assert np.all(np.abs(roots[key] - ref) <= 1e-11 * mult * scale), key


def _fd(f, h, order):
    """Central finite-difference derivative of order 1..3 with Richardson extrapolation (h, h/2)."""
    def stencil(hh):
        if order == 1:
            return (f(hh) - f(-hh)) / (2 * hh)
        if order == 2:
            return (f(hh) - 2 * f(0.0) + f(-hh)) / (hh * hh)
        return (f(2 * hh) - 2 * f(hh) + 2 * f(-hh) - f(-2 * hh)) / (2 * hh ** 3)
    return (4 * stencil(h / 2) - stencil(h)) / 3


@pytest.mark.parametrize("n", [2, 3])
def test_higher_and_mixed_coefficients_against_finite_differences(n):
    rng = np.random.default_rng(20 + n)
    x, _ = ig.physical_map(rng.uniform(size=(16, ig.dim(n))), n, BETA, 6.0)
    k = 0.7
    roots = dict(ty.derivative_roots(x, n, k, BETA, MU, LAM, GAMMA, 3, True, True, True))
    scale = dict(ty.derivative_scale(x, n, k, BETA, MU, LAM, GAMMA, 3, True, True, True))

    def F(dmu=0.0, dlam=0.0, dk=0.0):
        return ig.integrand(x, n, k + dk, BETA, MU + dmu, LAM + dlam, GAMMA)

    checks = {
        (2, 0, 0): _fd(lambda h: F(dmu=h), 2e-3, 2),
        (3, 0, 0): _fd(lambda h: F(dmu=h), 1e-3, 3),   # mu varies on the scale 1/beta
        (0, 2, 0): _fd(lambda h: F(dlam=h), 2e-2, 2),
        (0, 3, 0): _fd(lambda h: F(dlam=h), 2e-2, 3),   # truncation ~ (h / (|p|^2 + lambda))^2
        (1, 1, 0): _fd(lambda h: _fd(lambda g: F(dmu=g, dlam=h), 2e-3, 1), 2e-2, 1),
        (2, 1, 0): _fd(lambda h: _fd(lambda g: F(dmu=g, dlam=h), 2e-3, 2), 2e-2, 1),
        (1, 0, 1): _fd(lambda h: _fd(lambda g: F(dmu=g, dk=h), 2e-3, 1), 2e-3, 1),
        (0, 1, 1): _fd(lambda h: _fd(lambda g: F(dlam=g, dk=h), 2e-2, 1), 2e-3, 1),
        (2, 0, 1): _fd(lambda h: _fd(lambda g: F(dmu=g, dk=h), 2e-3, 2), 2e-3, 1),
    }
    for key, ref in checks.items():
        err = np.abs(roots[key] - ref)
        # 1e-300: below it FP64 values are subnormal and lose relative precision
        assert np.all(err <= 2e-5 * scale[key] + 1e-12 * np.abs(ref) + 1e-300), (key, float((err / scale[key]).max()))


def test_fock_taylor_closed_form_against_finite_differences():
    # the 1D closed form for d^m/dmu^m d^l/dlambda^l of the Fock self-energy against finite differences of
    # the value's own quadrature at shifted mu and lambda
    k = 0.9
    F = lambda dmu=0.0, dlam=0.0: ph.fock_finite_T(k, BETA, MU + dmu, LAM + dlam, GAMMA)
    assert np.isclose(ph.fock_taylor_finite_T(k, BETA, MU, LAM, GAMMA, 0, 0), F(), rtol=1e-10)
    d1 = ph.fock_derivs_finite_T(k, BETA, MU, LAM, GAMMA)
    assert np.isclose(ph.fock_taylor_finite_T(k, BETA, MU, LAM, GAMMA, 1, 0), d1[0], rtol=1e-9)
    assert np.isclose(ph.fock_taylor_finite_T(k, BETA, MU, LAM, GAMMA, 0, 1), d1[1], rtol=1e-9)
    for (m, l), ref in {
        (2, 0): _fd(lambda h: F(dmu=h), 2e-3, 2),
        (3, 0): _fd(lambda h: F(dmu=h), 2e-3, 3),
        (0, 2): _fd(lambda h: F(dlam=h), 2e-2, 2),
        (0, 3): _fd(lambda h: F(dlam=h), 4e-2, 3),
        (1, 1): _fd(lambda h: _fd(lambda g: F(dmu=g, dlam=h), 2e-3, 1), 2e-2, 1),
    }.items():
        got = ph.fock_taylor_finite_T(k, BETA, MU, LAM, GAMMA, m, l)
        assert abs(got - ref) <= 1e-5 * abs(ref), (m, l, got, ref)
    # P_m: the closed forms used in the per-leaf pin above
    n = 0.3
    assert np.isclose(ph.nF_mu_derivative_poly(2)(n), n * (1 - n) * (1 - 2 * n))
    assert np.isclose(ph.nF_mu_derivative_poly(3)(n), n * (1 - n) * (1 - 6 * n + 6 * n * n))
