"""Host FP64 calls of the estimators (no device): the equal-weight combination of iterations with chi^2/dof,
the Markov-chain ratio estimator from batch sums (against the oracle's ratio), the effective-mass coefficient
tables, and the checkpoint format's parsing and errors."""
import math

import numpy as np
import pytest

import paper_2403_18840_amd as dmc
from oracle import mcmc as omc


def test_combine_iterations_mean_error_and_chi2():
    rng = np.random.default_rng(5)
    n_iter, nv = 400, 6
    truth = rng.normal(size=nv)
    errs = np.abs(rng.normal(size=(n_iter, nv))) * 0.1 + 0.05
    means = truth + errs * rng.normal(size=(n_iter, nv))
    m, e, c = dmc.combine_iterations(means, errs)
    assert np.allclose(m, means.mean(axis=0), rtol=1e-14)
    assert np.allclose(e, np.sqrt((errs ** 2).sum(axis=0)) / n_iter, rtol=1e-14)
    ref = ((means - means.mean(axis=0)) ** 2 / errs ** 2).sum(axis=0) / (n_iter - 1)
    assert np.allclose(c, ref, rtol=1e-12)
    # consistent iterations: chi^2/dof near 1; inconsistent (errors understated 3x): near 9
    assert np.all(np.abs(c - 1) < 0.3)
    _, _, c3 = dmc.combine_iterations(means, errs / 3)
    assert np.all(c3 > 6)
    _, _, c1 = dmc.combine_iterations(means[:1], errs[:1])
    assert np.all(np.isnan(c1))
    with pytest.raises(dmc.DmcError):
        dmc.combine_iterations(means[:0], errs[:0])


def test_proposal_select_rule():
    ef = np.array([1.0, 2.0, 0.5])
    eg = 3.0 * ef                               # the grid's variance is 9x the flow's
    use, gain = dmc.proposal_select(ef, eg, 3.0, 1.0, 0)
    assert use and gain == pytest.approx(3.0, rel=1e-15)        # 9 x (1 / 3)
    assert dmc.proposal_select(ef, eg, 3.0, 1.0, 0, min_gain=3.5) == (False, pytest.approx(3.0))
    assert not dmc.proposal_select(ef, eg, 1.0, 1.0, 1)[0]       # a dropped weight rules the flow out
    assert dmc.proposal_select(np.zeros(3), eg, 1.0, 1.0, 0) == (True, math.inf)
    assert dmc.proposal_select(np.full(3, np.nan), eg, 1.0, 1.0, 0) == (False, 0.0)
    for bad in [dict(t_flow=0.0), dict(t_grid=-1.0), dict(min_gain=-1.0), dict(t_flow=math.inf)]:
        args = dict(err_flow=ef, err_grid=eg, t_flow=1.0, t_grid=1.0, nonfinite_flow=0, min_gain=1.0)
        args.update(bad)
        with pytest.raises(dmc.DmcError):
            dmc.proposal_select(**args)


def test_chains_ratio_matches_oracle_and_rescales_rs():
    rng = np.random.default_rng(9)
    B, G, R, K = 8, 2, 2, 3
    S = G * R * K * 2
    sums = rng.normal(size=(B, S + 1, 2))
    sums[:, S, 0] = 5.0 + rng.random(B)      # positive sum q/pi per batch
    sums[:, :, 1] = np.abs(sums[:, :, 1])
    order = 3
    g1, g2 = dmc.coupling(1.0), dmc.coupling(2.0)
    inst = [(25.0, 1.0, 0.5, g1), (25.0, 1.0, 2.0, g1), (25.0, 1.0, 0.5, g2)]
    m, e = dmc.chains_ratio(sums, G, R, K, order, inst)
    tot = omc.ratio_estimate(sums.sum(axis=0))            # [S]
    per = omc.ratio_estimate(sums)                         # [B][S]
    err = per.std(axis=0, ddof=1) / math.sqrt(B)
    for i, (g, fac) in enumerate([(0, 1.0), (1, 1.0), (0, (g2 / g1) ** order)]):
        ref = tot.reshape(G, R, K, 2)[g]
        assert np.allclose(m[i].real, fac * ref[..., 0], rtol=1e-12)
        assert np.allclose(m[i].imag, fac * ref[..., 1], rtol=1e-12)
        er = err.reshape(G, R, K, 2)[g]
        assert np.allclose(e[i].real, fac * er[..., 0], rtol=1e-10)
        assert np.allclose(e[i].imag, fac * er[..., 1], rtol=1e-10)
    with pytest.raises(dmc.DmcError):
        dmc.chains_ratio(sums[:1], G, R, K, order, inst)        # one batch: no scatter
    with pytest.raises(dmc.DmcError):
        dmc.chains_ratio(sums, 3, R, K, order, inst)            # two lambdas, three groups


def test_mass_table_assembles_a_and_b():
    beta = 25.0
    w0 = math.pi / beta
    # first-order roots of a d/dk graph: value then d/dk; and a Taylor set with (1, 0) and its k tangent
    orders = [(0, 0, 0), (0, 0, 1)]
    est = np.array([-0.3 + 0.02j, 0.8 - 0.1j])
    s, a, b = dmc.mass_table(4, orders, est, beta)
    assert s == {(4, 0, 0): -0.3} and a == {(4, 0, 0): 0.4} and abs(b[(4, 0, 0)] - 0.02 / w0) < 1e-15
    orders = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)]
    est = np.arange(6) * (1 + 0.5j)
    s, a, b = dmc.mass_table(2, orders, est, beta)
    assert s == {(2, 0, 0): 0.0, (2, 1, 0): 1.0, (2, 0, 1): 2.0}
    assert a == {(2, 0, 0): 1.5, (2, 1, 0): 2.0, (2, 0, 1): 2.5}
    assert all(abs(b[k] - 0.5 * s[k] / w0) < 1e-14 for k in s)


def test_checkpoint_position_roundtrip_and_errors():
    # without handles the checkpoint holds the Philox position only (no device needed)
    blob = dmc.checkpoint_save(seed=0x2403188400000001, next_index=123456789)
    assert blob[:8] == b"DMCCKPT1"
    assert dmc.checkpoint_load(blob) == (0x2403188400000001, 123456789)
    for bad in (b"", b"NOTACKPT" + blob[8:], blob[:12]):
        with pytest.raises(dmc.DmcError) as e:
            dmc.checkpoint_load(bad)
        assert e.value.status == -1
