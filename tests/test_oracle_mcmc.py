"""Pins of the oracle Markov-chain estimator: the importance-sampling limit alpha = 1, a closed-form
sign-changing integral, and the stationary distribution of the chain."""
import numpy as np

from oracle import mcmc


def _toy(alpha, n=4096, steps=60, thermal=10, seed=5, batches=16):
    # integral over (0, 1) of f(x) = cos(6 x) (= sin(6) / 6, sign-changing), uniform proposals q = 1;
    # per chain batch, the ratio estimate over all measured steps (batches are independent)
    rng = np.random.default_rng(seed)
    state = None
    cur = np.zeros((batches, 2, 2))
    xs = np.zeros(n)
    for t in range(thermal + steps):
        xp = rng.uniform(size=n)
        f = np.cos(6 * xp).astype(np.float32)[None, :]
        state, take = mcmc.step(state, f, np.ones(n, dtype=np.float32), alpha, seed, t, [0])
        xs = np.where(take, xp, xs)
        if t >= thermal:
            cur += mcmc.measure(state, batches)
    sizes = np.array([c1 - c0 for c0, c1 in mcmc.batch_bounds(n, batches)])
    return mcmc.ratio_estimate(cur)[:, 0], xs, cur[:, 0, 0] / (sizes * steps)


def test_alpha_one_is_importance_sampling():
    # pi = q: every proposal is taken and the estimate is the plain mean of f / q
    rng = np.random.default_rng(1)
    n = 1000
    f = rng.normal(size=(4, n)).astype(np.float32)
    jac = rng.uniform(0.5, 2.0, size=n).astype(np.float32)
    state, take = mcmc.step(None, f, jac, 1.0, 3, 0, [0, 1])
    state, take = mcmc.step(state, f[::-1].copy(), jac, 1.0, 3, 1, [0, 1])
    assert take.all()
    est = mcmc.ratio_estimate(mcmc.measure(state)[0])
    ref = (f[::-1].astype(np.float64) * jac.astype(np.float64)).mean(axis=1)
    assert np.allclose(est, ref, rtol=1e-12)


def test_sign_changing_integral_and_target():
    exact = np.sin(6.0) / 6.0
    for alpha in [0.2, 0.6]:
        blocks, xs, _ = _toy(alpha)
        m, e = blocks.mean(), blocks.std(ddof=1) / np.sqrt(len(blocks))
        assert abs(m - exact) < 5 * e, (alpha, m, e, exact)
        # the chain samples pi = alpha + (1 - alpha) |cos 6x|, normalised over (0, 1)
        edges = np.linspace(0, 1, 21)
        h, _ = np.histogram(xs, edges)
        xm = np.linspace(0, 1, 20001)
        dens = alpha + (1 - alpha) * np.abs(np.cos(6 * xm))
        cdf = np.concatenate([[0], np.cumsum((dens[1:] + dens[:-1]) / 2 * np.diff(xm))])
        cdf /= cdf[-1]
        expect = np.diff(np.interp(edges, xm, cdf)) * len(xs)
        chi2 = np.sum((h - expect) ** 2 / expect)
        assert chi2 < 60, (alpha, chi2)   # 19 degrees of freedom (chains are independent)
    # the plain mean of f / pi over the chain states is I / Z_pi, not the integral: the ratio with
    # the mean of q / pi is what removes the unknown normalisation of pi
    blocks, _, naive = _toy(0.2)
    z_pi = 0.2 + 0.8 * np.mean(np.abs(np.cos(6 * np.linspace(0, 1, 200001))))
    assert abs(naive.mean() - exact / z_pi) < 5 * naive.std(ddof=1) / np.sqrt(len(naive))
    assert abs(naive.mean() - exact) > 10 * naive.std(ddof=1) / np.sqrt(len(naive))


def test_rotation_hands_every_chain_the_whole_mixture():
    # proposals laid out by component: alternate runs of 256 indices from q1 = 1 and from q2 = 2x, both
    # on (0, 1) (every chain batch holds both); the acceptance test uses the mixture q = (q1 + q2) / 2.  A chain always
    # fed by component i settles to q_i pi / q / Z_i, and Z_1 != Z_2, so without rotation the pooled
    # ratio estimate converges to int f w / int q w, w = (q1 / Z_1 + q2 / Z_2) / q, not to int f.
    alpha, n, steps, thermal = 0.2, 8192, 120, 30
    exact = np.sin(6.0) / 6.0
    xm = (np.arange(200000) + 0.5) / 200000
    q1, q2 = np.ones_like(xm), 2 * xm
    q = (q1 + q2) / 2
    pi = alpha * q + (1 - alpha) * np.abs(np.cos(6 * xm))
    z1, z2 = np.mean(q1 * pi / q), np.mean(q2 * pi / q)
    w = (q1 / z1 + q2 / z2) / q
    biased = np.mean(np.cos(6 * xm) * w) / np.mean(q * w)
    assert abs(biased - exact) > 0.005   # the two limits are apart (16 %)
    for rotate in (False, True):
        rng = np.random.default_rng(8)
        state, cur = None, np.zeros((16, 2, 2))
        for t in range(thermal + steps):
            u = rng.uniform(size=n)
            x = np.where((np.arange(n) // 256) % 2 == 0, u, np.sqrt(u))
            f = np.cos(6 * x).astype(np.float32)[None, :]
            jac = (1.0 / ((1.0 + 2.0 * x) / 2.0)).astype(np.float32)
            off = int(rng.integers(n)) if rotate else 0
            state, _ = mcmc.step(state, f, jac, alpha, 11, t, [0], offset=off)
            if t >= thermal:
                cur += mcmc.measure(state, 16)
        est = mcmc.ratio_estimate(cur)[:, 0]
        m = mcmc.ratio_estimate(cur.sum(axis=0))[0]
        e = est.std(ddof=1) / np.sqrt(len(est))
        target = exact if rotate else biased
        assert abs(m - target) < 5 * e, (rotate, m, e, target)
        assert abs(m - (biased if rotate else exact)) > 5 * e, (rotate, m, e)


def test_offset_rotates_the_proposals():
    rng = np.random.default_rng(2)
    f = rng.normal(size=(2, 10)).astype(np.float32)
    jac = rng.uniform(0.5, 2.0, size=10).astype(np.float32)
    state, take = mcmc.step(None, f, jac, 0.5, 1, 0, [0, 1], offset=3)
    assert take.all()
    assert np.array_equal(state["f"], np.roll(f, -3, axis=1))
    assert np.allclose(state["q"], 1.0 / np.roll(jac, -3).astype(np.float64))


def test_batches_partition_the_chains():
    rng = np.random.default_rng(4)
    n = 1001
    f = rng.normal(size=(3, n)).astype(np.float32)
    jac = rng.uniform(0.5, 2.0, size=n).astype(np.float32)
    state, _ = mcmc.step(None, f, jac, 0.4, 3, 0, [0, 1])
    bounds = mcmc.batch_bounds(n, 7)
    assert bounds[0][0] == 0 and bounds[-1][1] == n
    assert all(a[1] == b[0] for a, b in zip(bounds, bounds[1:]))
    assert {c1 - c0 for c0, c1 in bounds} <= {n // 7, n // 7 + 1}
    per = mcmc.measure(state, 7)
    whole = mcmc.measure(state)[0]
    assert np.allclose(per.sum(axis=0), whole, rtol=1e-12)
    c0, c1 = bounds[3]
    v = f[1, c0:c1].astype(np.float64) / state["pi"][c0:c1]
    assert np.isclose(per[3, 1, 0], v.sum(), rtol=1e-12) and np.isclose(per[3, 1, 1], (v * v).sum(), rtol=1e-12)


def test_invalid_proposals_are_never_taken():
    f = np.array([[1.0, 2.0, np.nan, 1.0]], dtype=np.float32)
    jac = np.array([1.0, 0.0, 1.0, 1.0], dtype=np.float32)
    state, take = mcmc.step(None, f, jac, 0.5, 1, 0, [0])
    assert list(take) == [True, False, False, True]
    assert list(state["pi"] > 0) == [True, False, False, True]
    # a chain without a valid state takes its next valid proposal
    state, take = mcmc.step(state, np.ones((1, 4), dtype=np.float32), np.ones(4, dtype=np.float32), 0.5, 1, 1, [0])
    assert take[1] and take[2]


def test_chains_carry_coordinates_and_training_weights():
    # the state's coordinates follow the taken proposals; at alpha = 0 every valid chain weighs 1
    rng = np.random.default_rng(6)
    n, D = 64, 3
    f = rng.normal(size=(2, n)).astype(np.float32)
    jac = rng.uniform(0.5, 2.0, size=n).astype(np.float32)
    u = rng.uniform(size=(D, n)).astype(np.float32)
    state, take = mcmc.step(None, f, jac, 0.0, 1, 0, [0, 1], offset=5, u_prop=u)
    assert np.array_equal(state["u"], np.roll(u, -5, axis=1))
    f2 = rng.normal(size=(2, n)).astype(np.float32)
    u2 = rng.uniform(size=(D, n)).astype(np.float32)
    state2, take2 = mcmc.step(state, f2, jac, 0.0, 1, 1, [0, 1], u_prop=u2)
    assert 0 < take2.sum() < n
    assert np.array_equal(state2["u"][:, take2], u2[:, take2])
    assert np.array_equal(state2["u"][:, ~take2], state["u"][:, ~take2])
    uu, w = mcmc.training_data(state2, [0, 1])
    assert np.allclose(w, 1.0)
    s3, _ = mcmc.step(state2, f2, jac, 0.6, 1, 2, [0, 1], u_prop=u2)
    _, w3 = mcmc.training_data(s3, [0, 1])
    p = np.abs(s3["f"].astype(np.float64)).sum(axis=0)
    assert np.allclose(w3, p / s3["pi"])


def test_walk_normals_are_standard_and_follow_the_counter():
    # Box-Muller of the documented Philox stream: moments of a standard normal, independent pair members,
    # and point i's draws do not depend on where a batch starts
    x = mcmc.normals(11, 0, 400000, 3)
    se = 1.0 / np.sqrt(len(x))
    assert np.all(np.abs(x.mean(axis=0)) < 5 * se)
    assert np.all(np.abs(x.var(axis=0) - 1.0) < 5 * np.sqrt(2.0) * se)
    assert np.all(np.abs(np.mean(x ** 4, axis=0) - 3.0) < 5 * np.sqrt(96.0) * se)
    assert abs(np.corrcoef(x[:, 0], x[:, 1])[0, 1]) < 5 * se
    assert np.array_equal(mcmc.normals(11, 1000, 50, 3), x[1000:1050])
    # the move wraps onto the torus
    z = mcmc.walk_base([[0.95, 0.02]], [[1.0, -1.0]], 0.1)
    assert np.allclose(z, [[0.05, 0.92]])


def _toy_walk(use_flow_density=True, n=4000, thermal=150, steps=300, batches=20, sigma=0.25, alpha=0.5, seed=9):
    # 2D toy: flow T(z) = (z0^2, z1), so q_T(x) = 1 / (2 sqrt(x0)); the sampler's mixture is
    # q = 0.5 q_T + 0.5 (uniform); f(x) = (3 x0^2 - 1/2)(1 + x1) changes sign, integral 0.75.  One
    # independence step from q, then base-space walks only: the ratio estimate converges to the integral
    # only if the walk samples pi.  use_flow_density=False plants the mistake of testing with q for q_T.
    rng = np.random.default_rng(seed)
    f_of = lambda x: ((3 * x[:, 0] ** 2 - 0.5) * (1 + x[:, 1])).astype(np.float32)[None, :]
    qT = lambda x: 1.0 / (2.0 * np.sqrt(x[:, 0]))
    q = lambda x: 0.5 * qT(x) + 0.5
    flow = rng.uniform(size=n) < 0.5
    z0 = rng.uniform(size=(n, 2))
    x = np.where(flow[:, None], np.stack([z0[:, 0] ** 2, z0[:, 1]], axis=1), rng.uniform(size=(n, 2)))
    state, _ = mcmc.step(None, f_of(x), (1.0 / q(x)).astype(np.float32), alpha, seed, 0, [0])
    cur = np.zeros((batches, 2, 2))
    for t in range(1, thermal + steps):
        z = np.stack([np.sqrt(x[:, 0]), x[:, 1]], axis=1)
        zp = mcmc.walk_base(z, mcmc.normals(seed + 1, t * n, n, 2), sigma)
        xp = np.stack([zp[:, 0] ** 2, zp[:, 1]], axis=1)
        g = qT if use_flow_density else q
        state, take = mcmc.step_walk(state, f_of(xp), (1.0 / q(xp)).astype(np.float32),
                                     (1.0 / g(xp)).astype(np.float32), (1.0 / g(x)).astype(np.float32),
                                     alpha, seed, t, [0])
        x = np.where(take[:, None], xp, x)
        if t >= thermal:
            cur += mcmc.measure(state, batches)
    est = mcmc.ratio_estimate(cur)[:, 0]
    return est.mean(), est.std(ddof=1) / np.sqrt(batches)


def test_base_space_walk_samples_the_target():
    m, e = _toy_walk()
    assert abs(m - 0.75) < 5 * e, (m, e)
    assert e < 0.02
    # testing with the sampler's mixture density in place of the flow's own one biases the chain
    m_bad, e_bad = _toy_walk(use_flow_density=False)
    assert abs(m_bad - 0.75) > 5 * max(e, e_bad), (m_bad, e_bad)


def test_walk_step_keeps_invalid_chains():
    # a chain without a valid state, or with a non-positive flow density on either side, does not move
    n = 6
    f = np.ones((1, n), dtype=np.float32)
    state, _ = mcmc.step(None, f, np.ones(n, dtype=np.float32), 0.5, 1, 0, [0])
    state["pi"][0] = 0.0
    jfp = np.ones(n, dtype=np.float32)
    jfs = np.ones(n, dtype=np.float32)
    jfp[1] = 0.0
    jfs[2] = np.inf
    new, take = mcmc.step_walk(state, 2 * f, np.ones(n, dtype=np.float32), jfp, jfs, 0.5, 1, 1, [0])
    assert not take[:3].any() and take[3:].all()  # pi' > pi with equal q_T: always taken
