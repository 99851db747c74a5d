"""Oracle renormalisation post-processing and effective mass (test infrastructure; only tests/, the smoke
check and the bench's CPU leg use it).

Follows Sec. III.B (eq. sigma_xi_dmu: the self-energy as a double series in xi and the chemical-
potential shift dmu = sum_i xi^i delta_mu^(i); eq. counterterm: the counterterms fixed order by order
at the Fermi surface) and Sec. VI.A (eq. sigma_xi_dmu_dlambda with the Yukawa counterterm
dlambda = -xi lambda_R of eq. interaction_ct; eq. dsigma_depsilon_series and its b analogue;
eq. deltam_partitions, eq. deltas_partitions; eq. eff_mass_ratio with Z^-1 = 1 - b).  FP64, plain
truncated polynomial arithmetic in xi.

Inputs are the derivative coefficients X^(n,m,l) = d^m/dmu^m d^l/dlambda^l X^(n) (n >= 1) of one
observable X at the Fermi surface, as a dict {(n, m, l): value}.  The series of X in xi is
    X(xi) = sum_{n,m,l} xi^(n+l) dmu(xi)^m / m! (-lambda_R)^l / l! X^(n,m,l),   truncated at xi^N.

Readings (the paper is terse or garbled here):
  * the counterterm condition: the pole of the full propagator stays at the Fermi surface,
    mu - mu_R - Sigma(k_F, 0) = 0 with mu_R = E_F, so at each order delta_mu^(j) equals the xi^j
    coefficient of Sigma(k_F) (which involves delta_mu^(i) for i < j only: every term carries at
    least one interaction line); the printed condition omits this -dmu term;
  * Sigma(k_F, 0) is taken as Re Sigma(k_F, i w_0) at the lowest Matsubara frequency;
  * a^(n,m,l) = (m_e / k_F) d Re Sigma^(n,m,l) / dk at k_F, with m_e / k_F = 1/2 in units where
    eps_k = k^2 (k_F = E_F = 1); b^(n,m,l) = Im Sigma^(n,m,l)(k_F, i w_0) / w_0 (the finite-temperature
    difference quotient, w_0 = pi / beta);
  * m*/m = (1 - b(xi)) (1 + a(xi))^-1 expanded in xi to order N and evaluated at xi = 1.
"""
from __future__ import annotations

import math

import numpy as np


def _mul(a, b, N):
    out = np.zeros(N + 1)
    for i in range(N + 1):
        for j in range(N + 1 - i):
            out[i + j] += a[i] * b[j]
    return out


def xi_series(coef, N, dmu, lam_R):
    """X(xi) truncated at xi^N: coef {(n, m, l): X^(n,m,l)}, dmu the xi coefficients of the
    chemical-potential shift (dmu[0] = 0)."""
    d = np.zeros(N + 1)
    d[1:min(len(dmu), N + 1)] = np.asarray(dmu, dtype=np.float64)[1:N + 1]
    mmax = max([m for (_, m, _) in coef] + [0])
    pw = [np.eye(1, N + 1, 0).ravel()]
    for m in range(1, mmax + 1):
        pw.append(_mul(pw[-1], d, N))
    out = np.zeros(N + 1)
    for (n, m, l), v in coef.items():
        s = n + l
        if s > N:
            continue
        term = pw[m] * (v / math.factorial(m) * (-lam_R) ** l / math.factorial(l))
        out[s:] += term[:N + 1 - s]
    return out


def chemical_potential_counterterms(sigma_fs, N, lam_R):
    """delta_mu^(j), j = 0..N (index 0 is 0): delta_mu^(j) = [xi^j] Sigma(k_F; xi)."""
    d = np.zeros(N + 1)
    for j in range(1, N + 1):
        d[j] = xi_series(sigma_fs, j, d[:j], lam_R)[j]
    return d


def effective_mass(sigma_fs, a, b, N, lam_R):
    """Returns (delta_mu [N+1], a(xi) [N+1], b(xi) [N+1], m*/m coefficients [N+1], partial sums
    [N+1]: m*/m through order 0, 1, ..., N at xi = 1)."""
    d = chemical_potential_counterterms(sigma_fs, N, lam_R)
    A = xi_series(a, N, d, lam_R)
    B = xi_series(b, N, d, lam_R)
    # 1 / (1 + A(xi)) with A(0) = 0: sum_j (-A)^j
    inv = np.zeros(N + 1)
    inv[0] = 1.0
    p = np.zeros(N + 1)
    p[0] = 1.0
    for _ in range(N):
        p = _mul(p, -A, N)
        inv += p
    one_b = -B
    one_b[0] += 1.0
    M = _mul(one_b, inv, N)
    return d, A, B, M, np.cumsum(M)


def observables_from_roots(re_sigma, dk_re_sigma, im_sigma, beta):
    """(sigma_fs, a, b) from per-(n, m, l) Fermi-surface estimates: Re Sigma(k_F, i w_0), its k
    derivative, and Im Sigma(k_F, i w_0), each a dict {(n, m, l): value}."""
    w0 = math.pi / beta
    a = {key: 0.5 * v for key, v in dk_re_sigma.items()}
    b = {key: v / w0 for key, v in im_sigma.items()}
    return dict(re_sigma), a, b
