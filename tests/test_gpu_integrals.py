"""Integral-level parity: GPU estimates against the oracle's plain Monte Carlo (and against each
other under different proposals).  Both sides are unbiased estimators of the same integral, so
their difference is judged in units of the combined standard error."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
from oracle import mc
from oracle import physics as ph

from gpu_helpers import BETA, LAM, MU

pytestmark = pytest.mark.gpu


def _z(a, ea, b, eb):
    za = (a.real - b.real) / np.sqrt(ea.real ** 2 + eb.real ** 2 + 1e-300)
    zi = (a.imag - b.imag) / np.sqrt(ea.imag ** 2 + eb.imag ** 2 + 1e-300)
    return np.concatenate([np.atleast_1d(za), np.atleast_1d(zi)])


@pytest.mark.parametrize("n,N_ora", [(2, 1 << 21), (3, 1 << 17)])
def test_vegas_estimate_matches_oracle_mc(n, N_ora):
    ks = np.array([0.0, 1.0, 2.0], dtype=np.float32)
    gamma = ph.coupling(1.0)
    m, e = dmc.integrate(dmc.Graph(n), [(BETA, MU, LAM, gamma)], ks, 1 << 21, iters=8, adapt=5, seed=11 + n)
    om, oe = mc.plain_mc(n, ks.astype(np.float64), BETA, MU, LAM, gamma, N=N_ora, seed=1234 + n)
    z = _z(m[0, 0], e[0, 0], om, oe)
    # Im at k where the estimate is exactly 0 on both sides is excluded by its zero error
    z = z[np.isfinite(z)]
    print(f"order {n}: z = {np.round(z, 2)}; gpu {m[0, 0]} +- {e[0, 0]}; oracle {om} +- {oe}")
    # the three k share samples on each side, so the six z are correlated: bound their mean square loosely
    assert np.all(np.abs(z) < 4.0)
    assert np.mean(z ** 2) < 4.0


def test_proposals_agree_uniform_vs_vegas():
    n = 2
    ks = np.array([0.5, 1.0, 1.5], dtype=np.float32)
    gamma = ph.coupling(2.0)
    inst = [(BETA, MU, LAM, gamma)]
    mv, ev = dmc.integrate(dmc.Graph(n), inst, ks, 1 << 21, iters=6, adapt=5, seed=3)
    mu_, eu = dmc.integrate(dmc.Graph(n), inst, ks, 1 << 22, iters=4, kind=dmc.SAMPLER_UNIFORM, seed=4)
    z = _z(mv[0, 0], ev[0, 0], mu_[0, 0], eu[0, 0])
    print(f"uniform vs VEGAS z = {np.round(z, 2)}; error ratio {np.round(eu[0, 0].real / ev[0, 0].real, 1)}")
    assert np.all(np.abs(z) < 4.0)
    # VEGAS must actually reduce the variance
    assert np.all(ev[0, 0].real * np.sqrt(6 * 2.0) < eu[0, 0].real * np.sqrt(4 * 4.0))
