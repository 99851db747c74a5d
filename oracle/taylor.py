"""Oracle Taylor-mode coefficients of the self-energy integrand (test infrastructure; only tests/, the
smoke check and the bench's CPU leg use it).

Follows Sec. III.B (eq. taylor_node: every node becomes a truncated Taylor series in the
renormalisation parameters) and Sec. VI.A (eq. sigma_xi_dmu_dlambda: Sigma^(n,m,l) is the m-th mu
and l-th lambda derivative of the n-th order self-energy; eq. green_ct and eq. interaction_ct: the
counterterms are the Taylor terms of G0 in mu and of V in lambda).  The momentum derivative of every
coefficient (Sec. VI.A, eq. deltam_partitions) rides along as a first-order tangent.

A series here is a truncated polynomial in (dmu, dlam, dk) over a downward-closed index set
S = {(m, l, e): m + l <= T, m <= T [mu active], l <= T [lambda active], e <= [k active]}; coefficient
c[m, l, e] multiplies dmu^m dlam^l dk^e (normalised Taylor coefficients, not derivatives).  Products
drop every monomial outside S, which is exact because S is downward closed.  Leaves are composed
from the definitions by series arithmetic, not from hand-derived derivative formulas:
  G0(eps, tau) with eps = |p|^2 - (mu + dmu), |p|^2 carrying dk through p = ... + k z-hat
      tau > 0:  -exp(-eps tau) / (1 + exp(-beta eps))   (eps >= 0 at the value; else the same
                 quantity written as -exp(eps (beta - tau)) / (1 + exp(beta eps)))
      tau <= 0:  exp(-eps (tau + beta)) / (1 + exp(-beta eps))  (or exp(-eps tau) / (1 + exp(beta eps)))
  V = 8 pi gamma / (|p|^2 + lam + dlam)
with exp(a) = e^{a_0} sum_j (a - a_0)^j / j! and 1/a = (1/a_0) sum_j (-(a - a_0)/a_0)^j, both exact on S
because (a - a_0)^j vanishes beyond the total degree of S.  Diagrams are plain products of their
lines, as in oracle.integrand.diagram_values, with no sharing between diagrams.

Parity pins (tests/test_oracle_taylor.py): closed-form mu-derivatives of nF and of G0, the lambda
series of V in closed form, first-order coefficients against the dual-number derivatives (which
are pinned to central differences and the Fock closed forms), and higher and mixed coefficients of
whole diagrams against finite differences of the plain FP64 integrand.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import diagrams as dg
from . import integrand as ig
from . import physics as ph


def index_set(T: int, mu: bool = True, lam: bool = True, k: bool = False):
    """The coefficients (m, l, e), graded: e outermost, then total degree m + l, then m descending."""
    out = []
    for e in range(2 if k else 1):
        for d in range(T + 1):
            for m in range(d, -1, -1):
                l = d - m
                if (m and not mu) or (l and not lam):
                    continue
                out.append((m, l, e))
    return out


class Series:
    """Truncated Taylor series over the index set S; coefficients are numpy arrays over samples."""

    def __init__(self, S, c):
        self.S = S
        self.c = c  # dict (m, l, e) -> array

    @staticmethod
    def const(S, v):
        v = np.asarray(v)
        return Series(S, {i: (v if i == (0, 0, 0) else np.zeros_like(v)) for i in S})

    def __add__(self, o):
        return Series(self.S, {i: self.c[i] + o.c[i] for i in self.S})

    def __sub__(self, o):
        return Series(self.S, {i: self.c[i] - o.c[i] for i in self.S})

    def scale(self, s):
        return Series(self.S, {i: self.c[i] * s for i in self.S})

    def __mul__(self, o):
        out = {}
        for i in self.S:
            acc = 0.0
            for a in itertools.product(range(i[0] + 1), range(i[1] + 1), range(i[2] + 1)):
                b = (i[0] - a[0], i[1] - a[1], i[2] - a[2])
                acc = acc + self.c[a] * o.c[b]
            out[i] = acc
        return Series(self.S, out)

    def value(self):
        return self.c[(0, 0, 0)]

    def degree(self):
        return max(i[0] + i[1] + i[2] for i in self.S)


def _nilpotent_power_sum(a, weights):
    """sum_j weights[j] (a - a_0)^j for j = 0..degree (a_0 = the value)."""
    S = a.S
    h = Series(S, dict(a.c))
    h.c[(0, 0, 0)] = np.zeros_like(a.value())
    term = Series.const(S, np.ones_like(a.value()))
    acc = Series.const(S, np.zeros_like(a.value()))
    for j in range(a.degree() + 1):
        acc = acc + term.scale(weights(j))
        term = term * h
    return acc


def s_exp(a):
    """exp of a series: e^{a_0} sum_j (a - a_0)^j / j!."""
    return _nilpotent_power_sum(a, lambda j: 1.0 / math.factorial(j)).scale(np.exp(a.value()))


def s_recip(a):
    """1 / a: (1/a_0) sum_j (-(a - a_0)/a_0)^j."""
    a0 = a.value()
    h = Series(a.S, {i: (a.c[i] / a0 if i != (0, 0, 0) else np.zeros_like(a0)) for i in a.S})
    term = Series.const(a.S, np.ones_like(a0))
    acc = Series.const(a.S, np.zeros_like(a0))
    for j in range(a.degree() + 1):
        acc = acc + term.scale((-1.0) ** j)
        term = term * h
    return acc.scale(1.0 / a0)


def G0_series(eps, tau, beta):
    """G0 at (eps, tau) for a series eps (see the module header for the branch forms)."""
    e0 = eps.value()
    one = Series.const(eps.S, np.ones_like(e0))
    tau = np.asarray(tau, dtype=np.float64)
    pos = tau > 0
    nonneg = e0 >= 0
    # eps >= 0 forms, evaluated where valid (the other lanes use a safe substitute)
    eps_safe_p = Series(eps.S, {i: np.where(nonneg, v, 0.0) for i, v in eps.c.items()})
    eps_safe_n = Series(eps.S, {i: np.where(nonneg, 0.0, v) for i, v in eps.c.items()})
    den_p = s_recip(one + s_exp(eps_safe_p.scale(-beta)))
    den_n = s_recip(one + s_exp(eps_safe_n.scale(beta)))
    tp = np.where(pos, tau, tau + beta)  # tau' in (0, beta]
    # eps >= 0: +-exp(-eps tau') / (1 + exp(-beta eps))
    g_p = s_exp(eps_safe_p * Series.const(eps.S, -tp)) * den_p
    # eps < 0: tau > 0: -exp(eps (beta - tau)) / (1 + exp(beta eps)); tau <= 0: exp(-eps tau) / (...)
    g_n = s_exp(eps_safe_n * Series.const(eps.S, np.where(pos, beta - tau, -tau))) * den_n
    sign = np.where(pos, -1.0, 1.0)
    return Series(eps.S, {i: sign * np.where(nonneg, g_p.c[i], g_n.c[i]) for i in eps.S})


def V_series(p2, lam, gamma):
    """8 pi gamma / (|p|^2 + lam + dlam) for a series |p|^2 (dk part) and the variable dlam."""
    s = p2 + Series.const(p2.S, np.full_like(p2.value(), lam))
    if (0, 1, 0) in s.S:
        s.c[(0, 1, 0)] = s.c[(0, 1, 0)] + 1.0
    return s_recip(s).scale(8.0 * math.pi * gamma)


def diagram_series(x, n, k, beta, mu, lam, gamma, T, use_mu=True, use_lam=True, use_k=False, diagrams=None):
    """Per diagram d, the series of W_d(x) e^{i w_0 tau_ext(d)}: dict index -> complex [Ndiag, N].

    Coefficients are normalised (c[m, l, e]); the paper's Sigma^(n,m,l) derivative is m! l! c[m, l, 0]
    and its k derivative m! l! c[m, l, 1]."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    S = index_set(T, use_mu, use_lam, use_k)
    q, taus = ig._unpack(x, n)
    N = q.shape[0]
    w0 = math.pi / beta
    pref = (2 * math.pi) ** (-3 * n)
    out = {i: np.zeros((len(diagrams), N), dtype=np.complex128) for i in S}
    for di, d in enumerate(diagrams):
        val = Series.const(S, np.full(N, d.weight * pref))
        for ln in d.lines:
            p = ig.line_momentum(q, k, ln.mom)
            p2 = Series.const(S, np.sum(p * p, axis=1))
            if (0, 0, 1) in S:
                p2.c[(0, 0, 1)] = 2.0 * ln.mom[n] * p[:, 2]   # d|p|^2/dk (k enters as c_k k z-hat)
            if ln.kind == "G":
                a, b = ln.src // 2, ln.dst // 2
                tau = np.zeros(N) if a == b else taus[:, b] - taus[:, a]
                eps = p2 - Series.const(S, np.full(N, mu))
                if (1, 0, 0) in S:
                    eps.c[(1, 0, 0)] = eps.c[(1, 0, 0)] - 1.0   # eps = |p|^2 - mu - dmu
                val = val * G0_series(eps, tau, beta)
            else:
                val = val * V_series(p2, lam, gamma)
        phase = np.exp(1j * w0 * taus[:, d.ext_line])
        for i in S:
            out[i][di] = val.c[i] * phase
    return out


def derivative_roots(x, n, k, beta, mu, lam, gamma, T, use_mu=True, use_lam=True, use_k=False, diagrams=None):
    """Summed over diagrams and scaled to derivatives: list of ((m, l, e), complex [N]) in the index
    order, value = m! l! c[m, l, e] (d^m/dmu^m d^l/dlam^l (d/dk)^e of the integrand)."""
    ser = diagram_series(x, n, k, beta, mu, lam, gamma, T, use_mu, use_lam, use_k, diagrams)
    out = []
    for i in index_set(T, use_mu, use_lam, use_k):
        out.append((i, ser[i].sum(axis=0) * math.factorial(i[0]) * math.factorial(i[1])))
    return out


def _leaf_majorants(S, p2, dp2, tau, beta, lam, gamma, kind, mu):
    """Positive series bounding the terms a leaf's own series adds up (the scale of an FP32 evaluation,
    cancellation inside the leaf included): G: |G0| (tau' + beta)^m / m! (tau' + beta bounds the log-
    derivatives of exp(-eps tau') and of 1 / (1 + exp(-beta eps)) together); V: r^(l+1), r = 1 / (p^2 + lam);
    the k tangent of coefficient j: (j + 1) |coefficient j + 1| |d|p|^2/dk|."""
    N = p2.shape[0]
    out = {i: np.zeros(N) for i in S}
    if kind == "G":
        tp = np.where(tau > 0, tau, tau + beta)
        g0 = np.abs(ph.G0(p2 - mu, tau, beta))
        c = lambda m: g0 * (tp + beta) ** m / math.factorial(m)
        for (m, l, e) in S:
            if l:
                continue
            out[(m, l, e)] = c(m) if e == 0 else (m + 1) * c(m + 1) * np.abs(dp2)
    else:
        r = 1.0 / (p2 + lam)
        c = lambda l: 8.0 * math.pi * gamma * r ** (l + 1)
        for (m, l, e) in S:
            if m:
                continue
            out[(m, l, e)] = c(l) if e == 0 else (l + 1) * c(l + 1) * np.abs(dp2)
    return Series(S, out)


def derivative_scale(x, n, k, beta, mu, lam, gamma, T, use_mu=True, use_lam=True, use_k=False, diagrams=None):
    """The scale against which an FP32 evaluation of each derivative root is judged: the sum over
    diagrams of the product of the leaves' majorant series (_leaf_majorants) times |weight|, scaled to
    derivatives (m! l!).  It bounds the magnitude of every term the evaluation adds, before cancellation
    between diagrams and inside each leaf's series."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    S = index_set(T, use_mu, use_lam, use_k)
    q, taus = ig._unpack(x, n)
    N = q.shape[0]
    pref = (2 * math.pi) ** (-3 * n)
    tot = {i: np.zeros(N) for i in S}
    for d in diagrams:
        val = Series.const(S, np.full(N, abs(d.weight) * pref))
        for ln in d.lines:
            p = ig.line_momentum(q, k, ln.mom)
            p2 = np.sum(p * p, axis=1)
            dp2 = 2.0 * ln.mom[n] * p[:, 2]
            if ln.kind == "G":
                a, b = ln.src // 2, ln.dst // 2
                tau = np.zeros(N) if a == b else taus[:, b] - taus[:, a]
            else:
                tau = None
            val = val * _leaf_majorants(S, p2, dp2, tau, beta, lam, gamma, ln.kind, mu)
        for i in S:
            tot[i] += val.c[i]
    return [(i, tot[i] * math.factorial(i[0]) * math.factorial(i[1])) for i in S]
