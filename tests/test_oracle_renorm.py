"""Pins of the oracle renormalisation post-processing (oracle/renorm.py): closed-form counterterm series,
the lambda re-expansion, and hand-expanded low orders of m*/m."""
import math

import numpy as np

from oracle import renorm as rn


def test_counterterms_follow_the_tree_function():
    # Sigma^(1)(mu) = c exp(s (mu - mu_R)) and no higher order: delta_mu = xi c exp(s delta_mu), whose
    # solution is s delta_mu = T(xi c s) with the tree function T(z) = sum_j j^(j-1) z^j / j!
    c, s, N = 0.37, -1.3, 7
    sigma = {(1, m, 0): c * s ** m for m in range(N)}
    d = rn.chemical_potential_counterterms(sigma, N, lam_R=0.5)
    want = [0.0] + [c ** j * s ** (j - 1) * j ** (j - 1) / math.factorial(j) for j in range(1, N + 1)]
    assert np.allclose(d, want, rtol=1e-13, atol=0)


def test_lambda_reexpansion_recovers_the_bare_interaction():
    # X^(1)(lambda) = c / (lambda + 1): X^(1,0,l) = c (-1)^l l! / (lambda_R + 1)^(l+1); with
    # dlambda = -xi lambda_R the series is xi c / (lambda_R + 1 - xi lambda_R): coefficient of xi^j is
    # c lambda_R^(j-1) / (lambda_R + 1)^j, and the sum at xi = 1 is X^(1)(0) = c
    c, lam, N = 0.8, 1.375, 40
    X = {(1, 0, l): c * (-1) ** l * math.factorial(l) / (lam + 1) ** (l + 1) for l in range(N)}
    ser = rn.xi_series(X, N, [0.0], lam)
    want = [0.0] + [c * lam ** (j - 1) / (lam + 1) ** j for j in range(1, N + 1)]
    assert np.allclose(ser, want, rtol=1e-12, atol=0)
    assert abs(ser.sum() - c) < 1e-5


def test_second_order_counterterm_by_hand():
    rng = np.random.default_rng(1)
    s100, s200, s110, s101 = rng.normal(size=4)
    lam = 0.7
    sigma = {(1, 0, 0): s100, (2, 0, 0): s200, (1, 1, 0): s110, (1, 0, 1): s101}
    d = rn.chemical_potential_counterterms(sigma, 2, lam)
    assert np.isclose(d[1], s100)
    assert np.isclose(d[2], s200 + s100 * s110 - lam * s101)


def test_effective_mass_series_by_hand():
    # only first-order a and b: m*/m = (1 - xi b1) (1 + xi a1)^-1
    a1, b1 = 0.11, -0.07
    _, A, B, M, part = rn.effective_mass({(1, 0, 0): 0.3}, {(1, 0, 0): a1}, {(1, 0, 0): b1}, 3, 1.0)
    assert np.allclose(A, [0, a1, 0, 0]) and np.allclose(B, [0, b1, 0, 0])
    assert np.allclose(M, [1.0, -a1 - b1, a1 * a1 + a1 * b1, -a1 ** 3 - a1 * a1 * b1], rtol=1e-14)
    assert np.allclose(part, np.cumsum(M))


def test_effective_mass_second_order_with_counterterms_by_hand():
    # a(xi) picks up delta_mu^(1) a^(1,1,0) and -lambda_R a^(1,0,1) at order 2
    lam = 1.2
    sig = {(1, 0, 0): 0.25}
    a = {(1, 0, 0): 0.1, (2, 0, 0): 0.02, (1, 1, 0): 0.3, (1, 0, 1): -0.05}
    b = {(1, 0, 0): 0.0, (2, 0, 0): -0.04}
    d, A, B, M, _ = rn.effective_mass(sig, a, b, 2, lam)
    a2 = 0.02 + 0.25 * 0.3 - lam * (-0.05)
    assert np.allclose(A, [0, 0.1, a2])
    assert np.allclose(B, [0, 0.0, -0.04])
    assert np.allclose(M, [1.0, -0.1, 0.01 - a2 + 0.04])


def test_observables_from_roots_units():
    beta = 25.0
    sig, a, b = rn.observables_from_roots({(1, 0, 0): -0.5}, {(1, 0, 0): 0.2}, {(2, 0, 0): 0.03}, beta)
    assert sig == {(1, 0, 0): -0.5}
    assert np.isclose(a[(1, 0, 0)], 0.1)
    assert np.isclose(b[(2, 0, 0)], 0.03 / (math.pi / beta))
