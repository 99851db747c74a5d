"""Deterministic second-order results (test infrastructure, FP64): textbook expressions that fix the
signs and factors of the order-2 self-energy diagrams independently of the oracle's own diagram
weights.  Each function restates the physics; the tests compare them with the oracle's diagram
products (integrand.py) and with the GPU.

What is pinned, and from what (Sec. II.A eq. sigma_integration; Sec. VI.A eq. ueg_action, whose
spin-1/2 electrons interact through a spin-independent V):

* The closed fermion loop (the bubble, F = 1).  The screened interaction is W = V + V P V + ...,
  the self-energy at first order in W is Sigma = -int W G (the Fock form), and P is the free
  polarization: both spin states run around the loop, and P(Q, i nu = 0) < 0 (the static
  Lindhard function: screening).  So the bubble diagram equals -int V(Q)^2 G(k - Q) P(Q), and its
  loop (the diagram without the lines outside the loop), integrated over the loop momentum and
  the time difference, equals -P_static(Q), the finite-temperature Lindhard function: a 1D
  integral after the angular integration by hand (lindhard_static).

* The rainbow (a Fock insertion in the Fock diagram).  Expanding the Fock term
  -int V(k - p) nF(eps_p + Sigma_x(p)) to first order in Sigma_x gives
  Sigma_rainbow(k) = -int d^3p/(2 pi)^3 V(k - p) Sigma_x(p) dnF/deps(eps_p)  (static, real).

* The sign of Im Sigma at order 2.  The second-order self-energy is the first whose spectral
  function is non-zero, and it is positive (a sum of squared matrix elements times positive
  occupation factors), so Im Sigma^(2)(k, i w_0) < 0 at w_0 = pi / beta > 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from . import physics as ph


def lindhard_static(Q: float, beta: float, mu: float, qmax: float = 12.0) -> float:
    """P(Q, i nu = 0) = 2 int d^3p/(2 pi)^3 (nF(eps_p) - nF(eps_{p+Q})) / (eps_p - eps_{p+Q}), eps_p = p^2 - mu.

    Shifting p -> p - Q in the second term gives -2 int nF(eps_p) [1/(Q^2 + 2pQc) + 1/(Q^2 - 2pQc)], and the
    angular integral int_{-1}^{1} dc / (Q^2 + 2pQc) = ln|(Q + 2p)/(Q - 2p)| / (2pQ), so
        P = -(1 / (2 pi^2 Q)) int_0^inf p nF(p^2 - mu) ln|(2p + Q)/(2p - Q)| dp.
    At T = 0 and Q -> 0 this is -k_F m / pi^2 (m = 1/2, k_F = 1): -1/(2 pi^2), the density of states."""
    kf = math.sqrt(mu)
    pts = sorted(set(p for p in [0.5 * Q, kf] + [math.sqrt(max(0.0, mu + s * 40.0 / beta)) for s in (-1, 1)]
                     if 0 < p < qmax))

    def f(p):
        return p * float(ph.nF(p * p - mu, beta)) * math.log(abs((2 * p + Q) / (2 * p - Q)))
    val, _ = integrate.quad(f, 0.0, qmax, points=pts, limit=800, epsabs=0, epsrel=1e-11)
    return -val / (2 * math.pi ** 2 * Q)


def rainbow(k: float, beta: float, mu: float, lam: float, gamma: float, qmax: float = 6.0) -> float:
    """Sigma_rainbow(k) = -int d^3p/(2 pi)^3 V(|p + k|) Sigma_x(p) dnF/deps(p^2 - mu), |p| <= qmax.

    The direction of p enters only V(|p + k|): (1/2) int_{-1}^{1} dc 8 pi gamma / (p^2 + k^2 + 2pkc + lam) =
    (2 pi gamma / (p k)) ln[((p + k)^2 + lam) / ((p - k)^2 + lam)] (its k -> 0 limit is V(p)).  Then
    Sigma_rainbow = -(1/(2 pi^2)) int_0^qmax p^2 <V> Sigma_x(p) dnF/deps dp with dnF/deps = -beta nF (1 - nF),
    by composite Gauss-Legendre on panels around the Fermi surface (dnF/deps has width 1/beta)."""
    kf = math.sqrt(mu)
    w = 60.0 / beta
    edges = sorted(set([0.0, qmax] + [math.sqrt(max(0.0, mu + s * w * f)) for s in (-1, 1)
                                      for f in (1.0, 0.5, 0.25, 0.1, 0.03)] + [kf]))
    edges = [e for e in edges if 0 <= e <= qmax]
    x, wt = np.polynomial.legendre.leggauss(24)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        if b <= a:
            continue
        for xi, wi in zip(x, wt):
            p = 0.5 * (b - a) * xi + 0.5 * (a + b)
            n = float(ph.nF(p * p - mu, beta))
            dn = -beta * n * (1.0 - n)
            if dn == 0.0:
                continue
            if k < 1e-12:
                vav = 8 * math.pi * gamma / (p * p + lam)
            else:
                vav = 2 * math.pi * gamma / (p * k) * math.log(((p + k) ** 2 + lam) / ((p - k) ** 2 + lam))
            sx = ph.fock_finite_T(p, beta, mu, lam, gamma)
            tot += 0.5 * (b - a) * wi * p * p * vav * sx * dn
    return -tot / (2 * math.pi ** 2)
