"""Oracle integrand: naive FP64 diagram-by-diagram evaluation (test infrastructure).

Follows eq. sigma_integration: Sigma^(n) = int dV sum_t W_t(V), with the Feynman rules of the
UEG action (eq. ueg_action): one free propagator G0 (eq. propagator) per fermion line, one
Yukawa interaction V (eq. interaction_ct) per interaction line, momentum conserved at every
vertex, int d^3q/(2 pi)^3 per loop, and the diagram weight (-1)^(n+F) 2^F (F closed fermion
loops, spin 1/2, spin-independent V; the paper prints no sign rule, so this is the textbook
rule for the expansion of exp(-S) with G = -<T psi psibar>).

Observable (a reading): Sigma^(n)(k, i w_0) = int_0^beta dtau e^{i w_0 tau} Sigma^(n)(k, tau) at the
lowest fermionic Matsubara frequency w_0 = pi/beta (the frequency that Sec. VI.A's b
coefficients use), with the in-vertex at tau_0 = 0 and the out-vertex at the time of the
interaction line that holds it.

Sample layout x[N, D], D = 4n - 1: loop momenta q_0..q_{n-1} as Cartesian (x, y, z)
triples, then the times tau_1..tau_{n-1} of interaction lines 1..n-1.  External momentum
k z-hat.  No hoisting, no common-subexpression elimination, no fusion: every diagram is a
plain product of its lines.
"""
from __future__ import annotations

import math

import numpy as np

from . import diagrams as dg
from . import physics as ph


def dim(n: int) -> int:
    return 4 * n - 1


def _unpack(x, n):
    x = np.asarray(x, dtype=np.float64)
    q = x[:, : 3 * n].reshape(-1, n, 3)
    taus = np.concatenate([np.zeros((x.shape[0], 1)), x[:, 3 * n:]], axis=1)
    return q, taus


def line_momentum(q, k, mom):
    """p = sum_j c_j q_j + c_k k z-hat for one line; q[N, n, 3], returns p[N, 3]."""
    n = q.shape[1]
    p = np.zeros((q.shape[0], 3))
    for j in range(n):
        if mom[j]:
            p += mom[j] * q[:, j, :]
    if mom[n]:
        p[:, 2] += mom[n] * k
    return p


def diagram_values(x, n, k, beta, mu, lam, gamma, diagrams=None):
    """W_d(x) e^{i w_0 tau_ext(d)} for every diagram d: complex array [Ndiag, N]."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    q, taus = _unpack(x, n)
    N = q.shape[0]
    w0 = math.pi / beta
    pref = (2 * math.pi) ** (-3 * n)
    out = np.zeros((len(diagrams), N), dtype=np.complex128)
    for di, d in enumerate(diagrams):
        val = np.full(N, d.weight * pref)
        for ln in d.lines:
            p = line_momentum(q, k, ln.mom)
            p2 = np.sum(p * p, axis=1)
            if ln.kind == "G":
                a, b = ln.src // 2, ln.dst // 2
                if a == b:
                    tau = np.zeros(N)          # equal time: 0^-
                else:
                    tau = taus[:, b] - taus[:, a]
                val = val * ph.G0(p2 - mu, tau, beta)
            else:
                val = val * ph.V(p2, lam, gamma)
        phase = np.exp(1j * w0 * taus[:, d.ext_line])
        out[di] = val * phase
    return out


def integrand(x, n, k, beta, mu, lam, gamma, diagrams=None):
    """f(x) = sum_d W_d(x) e^{i w_0 tau_ext(d)}: complex array [N]."""
    return diagram_values(x, n, k, beta, mu, lam, gamma, diagrams).sum(axis=0)


def abs_sum(x, n, k, beta, mu, lam, gamma, diagrams=None):
    """A(x) = sum_d |W_d(x)|: the scale of the sum before sign cancellation."""
    return np.abs(diagram_values(x, n, k, beta, mu, lam, gamma, diagrams)).sum(axis=0)


# ----------------------------------------------------------------------------------------
# The per-sample tolerance an FP32 evaluation is held to.  A diagram is a product of leaves; a
# propagator's leaf is exp(-|eps| S) / (1 + exp(-beta |eps|)), S = tau' for eps >= 0 and
# beta - tau' for eps < 0 (tau' in (0, beta], the time shifted into that interval), written so
# that no factor exceeds 1.  In FP32 every operation rounds with relative error u = 2^-24, so a
# diagram carries a relative error of a few u per leaf, plus the error of each exponential's
# argument, which is absolute: rounding eps = |p|^2 - mu (|p|^2 summed from the rounded components
# of p, each the sum of rounded terms of size m_p = sum_j |c_j| |q_j| + |c_k| k) and S (times of size
# up to beta) gives at first order
#     |delta arg| <= u (|eps| (S + beta) + S (|p|^2 + 2 |p| m_p)) = u c_G.
# The rule: |f_FP32 - f| <= 1e-5 A + 2 u B + 1e-30, A = sum_d |W_d|, B = sum_d |W_d| sum_{G in d} c_G.
# The 1e-5 A term is the stated relative tolerance taken against the terms before cancellation
# (FP32 cannot resolve a cancelled sum better than its largest terms); the 2 u B term is the
# first-order error of the exponentials, which dominates only in samples whose every diagram is
# exponentially small.
# ----------------------------------------------------------------------------------------
U32 = 2.0 ** -24


def exponent_condition(x, n, k, beta, mu, diagrams=None):
    """C_d(x) = sum over the propagators G of diagram d of c_G (above): real [Ndiag, N]."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    q, taus = _unpack(x, n)
    N = q.shape[0]
    qn = np.linalg.norm(q, axis=2)                     # |q_j| [N, n]
    out = np.zeros((len(diagrams), N))
    for di, d in enumerate(diagrams):
        for ln in d.lines:
            if ln.kind != "G":
                continue
            p = line_momentum(q, k, ln.mom)
            p2 = np.sum(p * p, axis=1)
            eps = p2 - mu
            a, b = ln.src // 2, ln.dst // 2
            tp = np.full(N, beta) if a == b else taus[:, b] - taus[:, a]
            tp = np.where(tp > 0, tp, tp + beta)
            S = np.where(eps >= 0, tp, beta - tp)
            mp = sum(abs(ln.mom[j]) * qn[:, j] for j in range(n)) + abs(ln.mom[n]) * abs(k)
            out[di] += np.abs(eps) * (S + beta) + S * (p2 + 2.0 * np.sqrt(p2) * mp)
    return out


def fp32_tolerance(x, n, k, beta, mu, lam, gamma, diagrams=None, rel=1e-5):
    """(tol, A): the per-sample bound rel A + 2 u B + 1e-30 of the FP32 integrand, and A."""
    W = np.abs(diagram_values(x, n, k, beta, mu, lam, gamma, diagrams))
    C = exponent_condition(x, n, k, beta, mu, diagrams)
    A = W.sum(axis=0)
    return rel * A + 2.0 * U32 * (W * C).sum(axis=0) + 1e-30, A


# ----------------------------------------------------------------------------------------
# Derivatives by forward-mode dual numbers on the plain product of each diagram: every line
# value carries its value and its derivatives with respect to (mu, lambda, k); products follow
# the Leibniz rule.  Pinned by central differences and by the Fock closed forms.
# ----------------------------------------------------------------------------------------

def _G0_dual(eps, deps_dk, tau, beta):
    """(G0, dG0/dmu, dG0/dk) from d G0/d eps: tau > 0: G0 (beta nF - tau);
    tau <= 0: G0 (-tau - beta (1 - nF)); d eps/d mu = -1."""
    g = ph.G0(eps, tau, beta)
    n = ph.nF(eps, beta)
    dge = np.where(tau > 0, g * (beta * n - tau), g * (-tau - beta * (1.0 - n)))
    return g, -dge, dge * deps_dk


def diagram_values_dual(x, n, k, beta, mu, lam, gamma, diagrams=None, absolute=False):
    """Returns (value, d/dmu, d/dlambda, d/dk), each complex [Ndiag, N].

    With absolute=True each derivative is replaced by the sum of the magnitudes of its terms
    before any cancellation: |W| sum_l (tau'_l + beta nF_l) for mu (the two terms of
    d ln G0 / d mu = tau' - beta nF, tau' the time shifted into (0, beta]), |W| sum_l 1/(p_l^2 + lam)
    for lambda, and the same times |d|p_l|^2/dk| for k: the scale against which an FP32
    evaluation is judged."""
    if diagrams is None:
        diagrams = dg.sigma_diagrams(n)
    q, taus = _unpack(x, n)
    N = q.shape[0]
    w0 = math.pi / beta
    pref = (2 * math.pi) ** (-3 * n)
    outs = [np.zeros((len(diagrams), N), dtype=np.complex128) for _ in range(4)]
    for di, d in enumerate(diagrams):
        v = np.full(N, d.weight * pref)
        dmu = np.zeros(N)
        dlam = np.zeros(N)
        dk = np.zeros(N)
        for ln in d.lines:
            p = line_momentum(q, k, ln.mom)
            p2 = np.sum(p * p, axis=1)
            dp2_dk = 2.0 * ln.mom[n] * p[:, 2]
            if ln.kind == "G":
                a, b = ln.src // 2, ln.dst // 2
                tau = np.zeros(N) if a == b else taus[:, b] - taus[:, a]
                f, fmu, fk = _G0_dual(p2 - mu, dp2_dk, tau, beta)
                flam = np.zeros(N)
            else:
                f = ph.V(p2, lam, gamma)
                flam = -f / (p2 + lam)
                fk = flam * dp2_dk
                fmu = np.zeros(N)
            if absolute:
                if ln.kind == "G":
                    tp = np.where(tau > 0, tau, tau + beta)
                    lmu = tp + beta * ph.nF(p2 - mu, beta)
                    fmu = np.abs(f) * lmu
                    fk = np.abs(f) * lmu * np.abs(dp2_dk)
                else:
                    flam = np.abs(f) / (p2 + lam)
                    fk = flam * np.abs(dp2_dk)
                f = np.abs(f)
                v = np.abs(v)
            dmu = dmu * f + v * fmu
            dlam = dlam * f + v * flam
            dk = dk * f + v * fk
            v = v * f
        phase = np.ones(N) if absolute else np.exp(1j * w0 * taus[:, d.ext_line])
        for o, val in zip(outs, (v, dmu, dlam, dk)):
            o[di] = val * phase
    return tuple(outs)


# ----------------------------------------------------------------------------------------
# Physical map of the unit cube (a reading of "uniform in a ball |q| <= R (spherical coords)"):
# r = R y, cos(theta) = 2y - 1, phi = 2 pi y per loop, tau_j = beta y.  Jacobian
# prod_i (4 pi R r_i^2) beta^(n-1).
# ----------------------------------------------------------------------------------------

def physical_map(y, n, beta, R):
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    x = np.empty((N, dim(n)))
    J = np.ones(N)
    for i in range(n):
        r = R * y[:, 3 * i]
        c = 2.0 * y[:, 3 * i + 1] - 1.0
        s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
        phi = 2 * math.pi * y[:, 3 * i + 2]
        x[:, 3 * i] = r * s * np.cos(phi)
        x[:, 3 * i + 1] = r * s * np.sin(phi)
        x[:, 3 * i + 2] = r * c
        J *= 4 * math.pi * R * r * r
    for j in range(n - 1):
        x[:, 3 * n + j] = beta * y[:, 3 * n + j]
    J *= beta ** (n - 1)
    return x, J
