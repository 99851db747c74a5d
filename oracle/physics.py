"""Oracle physics: free propagator, Yukawa interaction, closed forms (test infrastructure, FP64).

Units (a reading; the paper fixes none): lengths in 1/k_F, energies in E_F, so the
dispersion of eq. ueg_action is eps_k = k^2 - mu with mu = mu_R = E_F = 1 (Sec. III.B and
Sec. VI.A set mu_R to the Fermi energy).  The Yukawa interaction of eq. interaction_ct,
4 pi e^2 / (q^2 + lambda_R), written in these units is V(q) = 8 pi gamma / (q^2 + lambda)
with gamma = alpha * r_s, alpha = (4 / (9 pi))^(1/3): e^2 = 2 Ry a_0 and k_F = 1 / (alpha r_s a_0).

Free propagator (eq. propagator, with G = -<T psi psibar> as in eq. ueg_action):
    G0(k, tau) = -exp(-eps tau) (1 - nF(eps))   for 0 < tau < beta
    G0(k, tau) =  exp(-eps tau) nF(eps)         for -beta < tau <= 0
The equal-time value (two ends on one instantaneous interaction line) is taken at 0^-,
the normal-ordered density nF(eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

ALPHA = (4.0 / (9.0 * math.pi)) ** (1.0 / 3.0)


def coupling(rs: float) -> float:
    """gamma = alpha r_s: the Rydberg-unit Yukawa strength in k_F = E_F = 1 units."""
    return ALPHA * rs


def nF(eps, beta):
    """Fermi function 1/(exp(beta eps) + 1), written so neither branch overflows."""
    eps = np.asarray(eps, dtype=np.float64)
    x = beta * eps
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, e / (1.0 + e), 1.0 / (1.0 + e))


def G0(eps, tau, beta):
    """Free propagator at imaginary time tau in (-beta, beta); tau == 0 means 0^-.

    Each branch is the definition above multiplied through by a factor that keeps the
    exponentials bounded: for eps >= 0 use 1 - nF = 1/(1 + e^{-beta eps}); for the negative
    branch with eps > 0 use nF e^{-eps tau} = e^{-eps (tau + beta)} / (1 + e^{-beta eps})."""
    eps = np.asarray(eps, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    eps, tau = np.broadcast_arrays(eps, tau)
    out = np.empty(eps.shape, dtype=np.float64)
    pos = tau > 0
    epos = eps >= 0
    # tau > 0: -exp(-eps tau) (1 - nF)
    m = pos & epos
    out[m] = -np.exp(-eps[m] * tau[m]) / (1.0 + np.exp(-beta * eps[m]))
    m = pos & ~epos
    out[m] = -np.exp(eps[m] * (beta - tau[m])) / (1.0 + np.exp(beta * eps[m]))
    # tau <= 0: exp(-eps tau) nF
    m = ~pos & epos
    out[m] = np.exp(-eps[m] * (tau[m] + beta)) / (1.0 + np.exp(-beta * eps[m]))
    m = ~pos & ~epos
    out[m] = np.exp(-eps[m] * tau[m]) / (1.0 + np.exp(beta * eps[m]))
    return out


def dG0_dmu(eps, tau, beta):
    """d G0 / d mu at fixed k (d eps / d mu = -1), from differentiating the definition:
    tau > 0: G0 (tau - beta nF);  tau <= 0: G0 (tau + beta (1 - nF))."""
    g = G0(eps, tau, beta)
    n = nF(eps, beta)
    tau = np.asarray(tau, dtype=np.float64)
    return np.where(tau > 0, g * (tau - beta * n), g * (tau + beta * (1.0 - n)))


def V(q2, lam, gamma):
    """Yukawa interaction 8 pi gamma / (q^2 + lambda) (eq. interaction_ct in k_F units)."""
    return 8.0 * math.pi * gamma / (np.asarray(q2, dtype=np.float64) + lam)


# ----------------------------------------------------------------------------------------
# First-order (Fock) self-energy: closed forms derived from eq. sigma_integration at n = 1
#   Sigma_x(k) = - int d^3q/(2 pi)^3 V(|k - q|) nF(q^2 - mu)
# Doing the angular integral by hand gives a 1D integral over |q|.
# ----------------------------------------------------------------------------------------

def fock_finite_T(k: float, beta: float, mu: float, lam: float, gamma: float,
                  qmax: float = 12.0) -> float:
    """-(gamma/(pi k)) int_0^qmax q nF(q^2-mu) ln[((k+q)^2+lam)/((k-q)^2+lam)] dq,
    and at k = 0 the limit -(4 gamma/pi) int q^2 nF / (q^2 + lam) dq.  Adaptive Gauss-Kronrod
    with a break point at the Fermi momentum sqrt(mu)."""
    kf = math.sqrt(mu)
    # break points at the Fermi momentum and where nF has fallen by e^{+-40}
    pts = [kf] + [math.sqrt(max(0.0, mu + s * 40.0 / beta)) for s in (-1, 1)]
    pts = [p for p in pts if 0 < p < qmax]
    if k < 1e-12:
        f = lambda q: q * q * float(nF(q * q - mu, beta)) / (q * q + lam)
        val, _ = integrate.quad(f, 0.0, qmax, points=pts, limit=400, epsabs=1e-15, epsrel=1e-12)
        return -4.0 * gamma / math.pi * val

    def f(q):
        return q * float(nF(q * q - mu, beta)) * math.log(((k + q) ** 2 + lam) / ((k - q) ** 2 + lam))
    pts = sorted(set(pts + ([k] if 0 < k < qmax else [])))
    val, _ = integrate.quad(f, 0.0, qmax, points=pts, limit=400, epsabs=1e-15, epsrel=1e-12)
    return -gamma / (math.pi * k) * val


def fock_T0_yukawa(k: float, lam: float, gamma: float) -> float:
    """T = 0, mu = 1 (sharp Fermi sea |q| < 1), elementary antiderivative.

    With u = q + a, an antiderivative of q ln(u^2 + lam) in q is
    F_a(q) = 1/2 [(u^2+lam) ln(u^2+lam) - u^2] - a [u ln(u^2+lam) - 2u + 2 sqrt(lam) atan(u/sqrt(lam))]
    and int_0^1 q ln[((k+q)^2+lam)/((k-q)^2+lam)] dq = [F_k]_0^1 - [F_{-k}]_0^1."""
    s = math.sqrt(lam)

    def F(a, q):
        u = q + a
        L = math.log(u * u + lam)
        return 0.5 * ((u * u + lam) * L - u * u) - a * (u * L - 2 * u + 2 * s * math.atan(u / s))

    if k < 1e-12:
        # -(4 gamma/pi) int_0^1 q^2/(q^2+lam) dq
        return -4.0 * gamma / math.pi * (1.0 - s * math.atan(1.0 / s))
    I = (F(k, 1.0) - F(k, 0.0)) - (F(-k, 1.0) - F(-k, 0.0))
    return -gamma / (math.pi * k) * I


def fock_T0_coulomb(k: float, gamma: float) -> float:
    """lambda -> 0, T = 0: -(2 gamma/pi) [1 + (1-k^2)/(2k) ln|(1+k)/(1-k)|]."""
    if k < 1e-12:
        return -4.0 * gamma / math.pi
    if abs(k - 1.0) < 1e-14:
        return -2.0 * gamma / math.pi
    return -2.0 * gamma / math.pi * (1.0 + (1.0 - k * k) / (2.0 * k) * math.log(abs((1.0 + k) / (1.0 - k))))


def fock_derivs_finite_T(k: float, beta: float, mu: float, lam: float, gamma: float,
                         qmax: float = 12.0):
    """d/dmu, d/dlambda, d/dk of fock_finite_T, each a 1D integral of the differentiated
    integrand (k > 0).  d nF/d mu = beta nF (1 - nF)."""
    kf = math.sqrt(mu)
    pts = [kf, k] + [math.sqrt(max(0.0, mu + s * 40.0 / beta)) for s in (-1, 1)]
    pts = sorted(set(p for p in pts if 0 < p < qmax))

    def n(q):
        return float(nF(q * q - mu, beta))

    def L(q):
        return math.log(((k + q) ** 2 + lam) / ((k - q) ** 2 + lam))

    c = -gamma / (math.pi * k)
    q_ = dict(points=pts, limit=400, epsabs=0, epsrel=1e-12)
    dmu, _ = integrate.quad(lambda q: q * beta * n(q) * (1 - n(q)) * L(q), 0, qmax, **q_)
    dlam, _ = integrate.quad(lambda q: q * n(q) * (1.0 / ((k + q) ** 2 + lam) - 1.0 / ((k - q) ** 2 + lam)),
                             0, qmax, **q_)
    I0, _ = integrate.quad(lambda q: q * n(q) * L(q), 0, qmax, **q_)
    dIk, _ = integrate.quad(lambda q: q * n(q) * (2 * (k + q) / ((k + q) ** 2 + lam)
                                                 - 2 * (k - q) / ((k - q) ** 2 + lam)), 0, qmax, **q_)
    dk = -gamma / math.pi * (dIk / k - I0 / (k * k))
    return c * dmu, c * dlam, dk


def nF_mu_derivative_poly(m: int):
    """Coefficients (ascending powers of n) of P_m with d^m nF(q^2 - mu)/dmu^m = beta^m P_m(nF):
    P_0 = n, P_{m+1}(n) = P_m'(n) n (1 - n), since d nF/d mu = beta nF (1 - nF)."""
    P = np.polynomial.Polynomial([0.0, 1.0])
    w = np.polynomial.Polynomial([0.0, 1.0, -1.0])
    for _ in range(m):
        P = P.deriv() * w
    return P


def fock_taylor_finite_T(k: float, beta: float, mu: float, lam: float, gamma: float, m: int, l: int,
                         qmax: float = 12.0) -> float:
    """d^m/dmu^m d^l/dlambda^l of fock_finite_T (k > 0): the 1D integral of
    -(gamma/(pi k)) q [beta^m P_m(nF)] d^l/dlambda^l ln[((k+q)^2+lam)/((k-q)^2+lam)], with
    d^l/dlambda^l ln(a + lam) = (-1)^(l-1) (l-1)! (a + lam)^(-l) for l >= 1."""
    kf = math.sqrt(mu)
    pts = [kf, k] + [math.sqrt(max(0.0, mu + s * 40.0 / beta)) for s in (-1, 1)]
    pts = sorted(set(p for p in pts if 0 < p < qmax))
    P = nF_mu_derivative_poly(m)

    def L(q):
        ap, am = (k + q) ** 2 + lam, (k - q) ** 2 + lam
        if l == 0:
            return math.log(ap / am)
        return (-1) ** (l - 1) * math.factorial(l - 1) * (ap ** -l - am ** -l)

    def f(q):
        return q * beta ** m * float(P(float(nF(q * q - mu, beta)))) * L(q)
    val, _ = integrate.quad(f, 0.0, qmax, points=pts, limit=400, epsabs=0, epsrel=1e-12)
    return -gamma / (math.pi * k) * val


def matsubara_of_G0(eps: float, beta: float, n: int = 0, nodes: int = 400) -> complex:
    """int_0^beta e^{i w_n tau} G0(eps, tau) dtau by composite Gauss-Legendre (for the pin
    G0(i w_n) = 1 / (i w_n - eps))."""
    w = (2 * n + 1) * math.pi / beta
    x, wt = np.polynomial.legendre.leggauss(nodes)
    panels = 16
    tot = 0j
    for p in range(panels):
        a, b = beta * p / panels, beta * (p + 1) / panels
        t = 0.5 * (b - a) * x + 0.5 * (a + b)
        tot += np.sum(0.5 * (b - a) * wt * np.exp(1j * w * t) * G0(eps, t, beta))
    return complex(tot)
