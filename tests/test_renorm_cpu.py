"""The library's renormalisation post-processing (dmc_effective_mass, host FP64) against the oracle's."""
import numpy as np
import pytest

import paper_2403_18840_amd as dmc
from oracle import renorm as rn


def _table(rng, N, scale=0.3):
    return {(n, m, l): float(rng.normal() * scale ** (n + m + l))
            for n in range(1, N + 1) for m in range(0, N - n + 1) for l in range(0, N - n - m + 1)}


@pytest.mark.parametrize("N,lam", [(1, 0.5), (2, 1.0), (4, 1.375), (6, 2.0)])
def test_effective_mass_matches_oracle(N, lam):
    rng = np.random.default_rng(N)
    sig, a, b = _table(rng, N), _table(rng, N, 0.2), _table(rng, N, 0.1)
    out = dmc.effective_mass(N, lam, sig, a, b)
    d, A, B, M, part = rn.effective_mass(sig, a, b, N, lam)
    for name, ref in [("delta_mu", d), ("a_xi", A), ("b_xi", B), ("mass", M), ("mass_partial", part)]:
        assert np.allclose(out[name], ref, rtol=1e-12, atol=1e-15), name


def test_effective_mass_argument_errors():
    with pytest.raises(dmc.DmcError):
        dmc.effective_mass(0, 1.0, {}, {}, {})
    with pytest.raises(dmc.DmcError):
        dmc.effective_mass(2, -1.0, {}, {}, {})
    with pytest.raises(dmc.DmcError):
        dmc.effective_mass(2, 1.0, {(0, 1, 0): 1.0}, {}, {})
    out = dmc.effective_mass(3, 1.0, {}, {}, {})   # free electrons: m*/m = 1
    assert np.allclose(out["mass"], [1, 0, 0, 0]) and np.allclose(out["mass_partial"], 1.0)
