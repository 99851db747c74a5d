"""The effective-mass pipeline on the GPU (Taylor-mode coefficients at k_F, counterterms, xi series)
against the first-order closed forms, and its consistency at higher order."""
import math

import numpy as np
import pytest

import paper_2403_18840_amd as dmc
from oracle import physics as ph

from gpu_helpers import BETA, MU

pytestmark = pytest.mark.gpu


def test_first_order_mass_and_counterterm_match_fock():
    # N = 1: delta_mu^(1) = Re Sigma_x(k_F); m*/m through order 1 = 1 - a^(1,0,0) - b^(1,0,0) with
    # a = (1/2) d Sigma_x / dk at k_F and b = 0 (the exchange term is static)
    lam, rs = 1.0, 1.0
    gamma = ph.coupling(rs)
    assert math.isclose(dmc.coupling(rs), gamma, rel_tol=1e-15)
    mp, me, dm, de = dmc.effective_mass_estimate(1, rs, lam, beta=BETA, mu=MU, n_samples=1 << 21, batches=8)
    sx = ph.fock_finite_T(1.0, BETA, MU, lam, gamma)
    dk = ph.fock_derivs_finite_T(1.0, BETA, MU, lam, gamma)[2]
    assert mp[0] == 1.0 and dm[0] == 0.0
    assert abs(dm[1] - sx) < 4 * de[1] + 1e-6 * abs(sx), (dm[1], de[1], sx)
    want = 1.0 - 0.5 * dk
    assert abs(mp[1] - want) < 4 * me[1] + 1e-6, (mp[1], me[1], want)


def test_third_order_series_is_finite_and_consistent():
    mp, me, dm, de = dmc.effective_mass_estimate(3, 1.0, 1.0, beta=BETA, mu=MU, n_samples=1 << 20, batches=6)
    assert np.all(np.isfinite(mp)) and np.all(np.isfinite(me)) and np.all(np.isfinite(dm))
    assert mp[0] == 1.0
    # the partial sums are what dmc_effective_mass returns for the same tables (cumulative)
    assert np.all(me[1:] > 0)
    print("m*/m partial sums", mp, "+-", me, "delta_mu", dm, "+-", de)
