"""Second-order pins of the oracle (orders 1-2 are where the paper's method has closed forms): the
fermion-loop factor of the bubble against the finite-temperature Lindhard function, the rainbow
against the first-order expansion of the Fock term, and the sign of Im Sigma^(2).  Each reference
comes from oracle/quadrature.py, which restates the physics and shares no diagram weight with
integrand.py, so a dropped spin factor, a wrong loop sign or a wrong Matsubara phase fails here."""
import math

import numpy as np
import pytest

from oracle import diagrams as dg
from oracle import integrand as ig
from oracle import mc
from oracle import physics as ph
from oracle import quadrature as qd

BETA, MU, LAM = 25.0, 1.0, 1.0
GAMMA = ph.coupling(1.0)


def test_lindhard_static_limits():
    # T -> 0 (beta = 4000): the closed form -N(0) [1/2 + (1 - x^2)/(4x) ln|(1 + x)/(1 - x)|], x = Q / (2 k_F),
    # N(0) = m k_F / pi^2 = 1 / (2 pi^2) with m = 1/2; Q -> 0 gives -N(0) (the compressibility)
    N0 = 1.0 / (2 * math.pi ** 2)
    for Q in (0.2, 1.0, 1.7, 3.0):
        x = Q / 2
        ref = -N0 * (0.5 + (1 - x * x) / (4 * x) * math.log(abs((1 + x) / (1 - x))))
        assert abs(qd.lindhard_static(Q, 4000.0, MU) - ref) < 2e-3 * abs(ref)
    assert abs(qd.lindhard_static(1e-3, 4000.0, MU) + N0) < 1e-3 * N0
    # finite T: dn/dmu of the free gas, n = 2 int nF d^3p/(2 pi)^3, equals -P(Q -> 0)
    from scipy import integrate
    dn = 2 * BETA / (2 * math.pi ** 2) * integrate.quad(
        lambda p: p * p * float(ph.nF(p * p - MU, BETA)) * (1 - float(ph.nF(p * p - MU, BETA))), 0, 3,
        points=[0.9, 1.0, 1.1], limit=400, epsabs=0, epsrel=1e-12)[0]
    assert abs(qd.lindhard_static(1e-4, BETA, MU) + dn) < 1e-5 * dn


def _bubble():
    ds = [d for d in dg.sigma_diagrams(2) if d.n_loops_f == 1]
    assert len(ds) == 1
    return ds[0]


def _chords_for(d, targets, k):
    """Loop momenta (q0, q1) that give line targets[i][0] the momentum targets[i][1] (vectors [M, 3])."""
    rows = [d.lines[i].mom for i, _ in targets]
    A = np.array([[r[0], r[1]] for r in rows], dtype=float)
    kz = np.array([0.0, 0.0, k])
    rhs = [np.asarray(v, float) - rows[j][2] * kz for j, (_, v) in enumerate(targets)]
    Ai = np.linalg.inv(A)
    q0 = Ai[0, 0] * rhs[0] + Ai[0, 1] * rhs[1]
    q1 = Ai[1, 0] * rhs[0] + Ai[1, 1] * rhs[1]
    return q0, q1


@pytest.mark.parametrize("Qn", [0.35, 1.0, 1.5, 2.6])
def test_bubble_loop_is_minus_the_static_polarization(Qn):
    """The bubble diagram divided by its lines outside the closed loop (the two interactions, the open
    propagator and the phase), integrated over the loop momentum and the time between the two interaction
    lines, equals -P(Q, 0): loop sign -1 and spin factor 2 (a weight of -1 or +2 fails)."""
    d = _bubble()
    n, k = 2, 0.7
    # the closed loop is the cycle of sigma that does not hold the in-vertex
    main = {0}
    v = d.sigma[0]
    while v != 0:
        main.add(v)
        v = d.sigma[v]
    loop = [i for i, ln in enumerate(d.lines) if ln.kind == "G" and ln.src not in main]
    outside_g = [i for i, ln in enumerate(d.lines) if ln.kind == "G" and ln.src in main]
    vl = [i for i, ln in enumerate(d.lines) if ln.kind == "V"]
    assert len(loop) == 2 and len(outside_g) == 1 and len(vl) == 2
    Qv = Qn * np.array([0.36, 0.48, 0.8])
    e1 = np.array([0.8, -0.6, 0.0])
    e2 = np.cross(Qv / Qn, e1)
    # nodes: |p| (panels around the Fermi surface), |p + Q| (panels around 1), tau
    xg, wg = np.polynomial.legendre.leggauss(24)

    def nodes(edges):
        t, w = [], []
        for a, b in zip(edges[:-1], edges[1:]):
            if b > a:
                t.append(0.5 * (b - a) * xg + 0.5 * (a + b))
                w.append(0.5 * (b - a) * wg)
        return np.concatenate(t), np.concatenate(w)

    # |p| also breaks where |p - Q| = 1 (there the range of |p + Q| first reaches the Fermi surface)
    pe = [0, 0.8, 0.93, 0.98, 1.0, 1.02, 1.07, 1.2, 1.5, Qn + 1.6]
    for c in (abs(Qn - 1), Qn + 1):
        pe += [c - 0.05, c - 0.01, c, c + 0.01, c + 0.05]
    pr, pw = nodes(sorted(set(v for v in pe if 0 <= v <= Qn + 1.6)))
    tr, tw = nodes([0, 0.02, 0.1, 0.4, 1.5, 5, 12, BETA])
    total = 0.0
    for p, wp in zip(pr, pw):
        # the angle through s = |p + Q| (dc = s ds / (p Q)), with panels around the Fermi surface s = 1
        lo, hi = abs(p - Qn), p + Qn
        se = sorted(set([lo, hi] + [v for v in (0.85, 0.96, 1.0, 1.04, 1.15) if lo < v < hi]))
        sr, sw = nodes(se)
        cr = np.clip((sr * sr - p * p - Qn * Qn) / (2 * p * Qn), -1.0, 1.0)
        cw = sw * sr / (p * Qn)
        P = p * (cr[:, None] * Qv / Qn + np.sqrt(1 - cr[:, None] ** 2) * e1)
        # every (c, tau) pair
        Pm = np.repeat(P, len(tr), axis=0)
        T = np.tile(tr, len(cr))
        W = np.repeat(cw, len(tr)) * np.tile(tw, len(cr))
        # the interaction line carries +Q or -Q so that the loop's other propagator carries p + Q
        for sq in (1.0, -1.0):
            q0, q1 = _chords_for(d, [(vl[0], np.broadcast_to(sq * Qv, Pm.shape)), (loop[0], Pm)], k)
            other = ig.line_momentum(np.stack([q0, q1], axis=1), k, d.lines[loop[1]].mom)
            if np.allclose(np.sum(other ** 2, axis=1), np.sum((Pm + Qv) ** 2, axis=1)):
                break
        else:
            raise AssertionError("the bubble's loop does not carry p and p + Q")
        x = np.concatenate([q0, q1, T[:, None]], axis=1)
        full = ig.diagram_values(x, n, k, BETA, MU, LAM, GAMMA, [d])[0]
        q, taus = ig._unpack(x, n)
        out = (2 * math.pi) ** (-3 * n) * np.exp(1j * math.pi / BETA * taus[:, d.ext_line])
        for i in vl + outside_g:
            ln = d.lines[i]
            pv = ig.line_momentum(q, k, ln.mom)
            p2 = np.sum(pv * pv, axis=1)
            if ln.kind == "V":
                out = out * ph.V(p2, LAM, GAMMA)
            else:
                a, b = ln.src // 2, ln.dst // 2
                out = out * ph.G0(p2 - MU, taus[:, b] - taus[:, a], BETA)
        R = full / out
        assert np.max(np.abs(R.imag)) <= 1e-9 * np.max(np.abs(R.real)) + 1e-300
        total += wp * p * p * np.sum(W * R.real)
    total /= 4 * math.pi ** 2
    ref = -qd.lindhard_static(Qn, BETA, MU)
    assert ref > 0
    assert abs(total - ref) < 1e-6 * ref, (total, ref)


def test_rainbow_matches_the_expanded_fock_term():
    """The rainbow diagram's integral (the oracle's product, by importance sampling through the C integrand)
    against -int V(k - p) Sigma_x(p) dnF/deps by quadrature; it is static, so its Im part is 0."""
    rb = [d for d in dg.sigma_diagrams(2) if d.n_loops_f == 0 and d.ext_line == 0]
    assert len(rb) == 1
    ks = [0.0, 0.5, 1.0, 2.0]
    m, e = mc.importance_mc(2, ks, BETA, MU, LAM, GAMMA, rb, N=1 << 22, seed=2024)
    for a, k in enumerate(ks):
        ref = qd.rainbow(k, BETA, MU, LAM, GAMMA)
        assert ref < 0
        assert abs(m[a].real - ref) < 3.5 * e[a].real, (k, m[a], e[a], ref)
        assert m[a].imag == 0.0


def test_second_order_imaginary_part_is_negative():
    """Im Sigma^(2)(k, i pi / beta) < 0 (positive spectral function of the second-order self-energy): pins
    the phase e^{i w_0 tau_out} and the relative signs of the dynamic diagrams (bubble and exchange)."""
    ks = [0.3, 1.0, 1.6, 2.5]
    m, e = mc.importance_mc(2, ks, BETA, MU, LAM, GAMMA, dg.sigma_diagrams(2), N=1 << 21, seed=99)
    for a, k in enumerate(ks):
        assert m[a].imag < -5 * e[a].imag, (k, m[a], e[a])
