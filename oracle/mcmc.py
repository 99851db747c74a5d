"""Oracle Markov-chain estimator with independent proposals and random-walk moves in a flow's base space
(test infrastructure; only tests/, the smoke check and the bench's CPU leg use it).

Follows Sec. IV: the target pi = alpha q + (1 - alpha) p with p = |f| (eq.
target_distr_nf_mcmc_qft_revised), the Metropolis-Hastings acceptance
min(1, pi(x') Q(x | x') / (pi(x) Q(x' | x))), which for independent proposals Q(x' | x) = q(x')
reads min(1, pi(x') q(x) / (pi(x) q(x'))), and the ratio estimator
I = sum_i f(x_i)/pi(x_i) / sum_i q(x_i)/pi(x_i) over the chain states x_i (eq.
nf_mcmc_estimator_qft_final_revised).

Conventions shared with the library (data, each side with its own code): p sums |f| over the
root-0 observable slots in slot order, in FP64; the test is u pi(x) q(x') < pi(x') q(x) in FP64
with u = ((w >> 8) + 1/2) 2^-24, w the first Philox4x32-10 word of key `seed`, counter
(chain mod 2^32, chain div 2^32, step mod 2^32, step div 2^32); a proposal whose q or pi is not
finite and positive is never taken, a chain without a valid state takes its next valid proposal,
and the first step takes every valid proposal.
"""
from __future__ import annotations

import numpy as np

from oracle import sampler as osp

MASK = 0xFFFFFFFF


def uniforms(seed: int, step: int, n: int):
    c = np.arange(n, dtype=np.uint64)
    ctr = np.stack([c & np.uint64(MASK), c >> np.uint64(32),
                    np.full(n, step & MASK, dtype=np.uint64), np.full(n, step >> 32, dtype=np.uint64)], axis=-1)
    key = np.broadcast_to(np.array([seed & MASK, (seed >> 32) & MASK], dtype=np.uint64), (n, 2))
    w = osp.philox4x32_10(ctr, key)[:, 0]
    return ((w >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def step(state, f_prop, jac_prop, alpha, seed, step_index, root0_slots, offset=0, u_prop=None):
    """One Metropolis-Hastings step of every chain.  state: dict f [S][n] (float32 values), q, pi
    [n] float64 (and u [D][n] float32 when proposals carry coordinates), or None before the first step.
    f_prop [S][n] float32, jac_prop [n] float32, u_prop [D][n] float32 or None; chain c proposes column
    (c + offset) mod n (a uniform offset per step makes every chain's proposal a draw from the whole
    proposal density when the sampler orders its draws by mixture component).
    Returns (new state, taken [n] bool)."""
    n = np.asarray(f_prop).shape[1]
    cols = (np.arange(n) + offset) % n
    f_prop = np.asarray(f_prop, dtype=np.float32)[:, cols]
    jac_prop = np.asarray(jac_prop)[cols]
    if u_prop is not None:
        u_prop = np.asarray(u_prop, dtype=np.float32)[:, cols]
    p = np.zeros(n)
    for s in root0_slots:
        p = p + np.abs(f_prop[s].astype(np.float64))
    jp = np.asarray(jac_prop, dtype=np.float32).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        qp = 1.0 / jp
        pip = alpha * qp + (1.0 - alpha) * p
        vp = (jp > 0) & np.isfinite(qp) & np.isfinite(pip) & (pip > 0)
        if state is None:
            pis = np.zeros(n)
            qs = np.zeros(n)
        else:
            pis, qs = state["pi"], state["q"]
        vs = (pis > 0) & np.isfinite(pis)
        u = uniforms(seed, step_index, n)
        test = u * pis * qp < pip * qs
    take = vp & (~vs | test)
    if state is None:
        new = {"f": np.zeros_like(f_prop), "q": np.zeros(n), "pi": np.zeros(n)}
        if u_prop is not None:
            new["u"] = np.zeros_like(u_prop)
    else:
        new = {k: v.copy() for k, v in state.items()}
    if u_prop is not None:
        new["u"][:, take] = u_prop[:, take]
    new["f"][:, take] = f_prop[:, take]
    new["q"][take] = qp[take]
    new["pi"][take] = pip[take]
    return new, take


def normals(seed: int, first: int, n: int, D: int):
    """Standard normals [n][D] of the base-space walk (a reading: the paper names no generator).
    Coordinates (2j, 2j + 1) of point i = first + index take the first two Philox4x32-10 words w0, w1 of
    counter (i mod 2^32, i div 2^32, j, 1), key (seed mod 2^32, seed div 2^32); with
    u_k = ((w_k >> 8) + 1/2) 2^-24 and r = sqrt(-2 log u0) they are r cos(2 pi u1), r sin(2 pi u1)
    (the Box-Muller transform)."""
    i = np.arange(first, first + n, dtype=np.uint64)
    key = np.broadcast_to(np.array([seed & MASK, (seed >> 32) & MASK], dtype=np.uint64), (n, 2))
    out = np.empty((n, 2 * ((D + 1) // 2)))
    for j in range((D + 1) // 2):
        ctr = np.stack([i & np.uint64(MASK), i >> np.uint64(32), np.full(n, j, dtype=np.uint64),
                        np.ones(n, dtype=np.uint64)], axis=-1)
        w = osp.philox4x32_10(ctr, key)
        u0 = ((w[:, 0] >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
        u1 = ((w[:, 1] >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
        r = np.sqrt(-2.0 * np.log(u0))
        out[:, 2 * j] = r * np.cos(2.0 * np.pi * u1)
        out[:, 2 * j + 1] = r * np.sin(2.0 * np.pi * u1)
    return out[:, :D]


def walk_base(z, xi, sigma):
    """The symmetric move of base points on the unit torus: z' = (z + sigma xi) mod 1."""
    return np.mod(np.asarray(z, dtype=np.float64) + sigma * np.asarray(xi, dtype=np.float64), 1.0)


def step_walk(state, f_prop, jac_prop, jflow_prop, jflow_state, alpha, seed, step_index, root0_slots, u_prop=None):
    """One random-walk step in the base space of the flow T (Sec. IV: the optional base-space proposals
    of NF-MCMC).  Chain c proposes column c, reached from its own state by a symmetric move of the base
    point z = T^-1(x).  In base coordinates the target is pi(T(z)) |det dT/dz| = pi(x) / q_T(x) for the
    uniform base (q_T: the flow's own density, 1 / jflow in x), so Metropolis-Hastings takes x' with
    probability min(1, [pi(x') / q_T(x')] / [pi(x) / q_T(x)]): the test u pi(x) q_T(x') < pi(x') q_T(x),
    with the uniform u of step().  pi = alpha q + (1 - alpha) p keeps the sampler's mixture q = 1 / jac.
    A chain without a valid state, or with a q_T that is not finite and positive on either side, stays.
    Returns (new state, taken)."""
    f_prop = np.asarray(f_prop, dtype=np.float32)
    n = f_prop.shape[1]
    p = np.zeros(n)
    for s in root0_slots:
        p = p + np.abs(f_prop[s].astype(np.float64))
    jp = np.asarray(jac_prop, dtype=np.float32).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        qp = 1.0 / jp
        pip = alpha * qp + (1.0 - alpha) * p
        vp = (jp > 0) & np.isfinite(qp) & np.isfinite(pip) & (pip > 0)
        gp = 1.0 / np.asarray(jflow_prop, dtype=np.float32).astype(np.float64)
        gs = 1.0 / np.asarray(jflow_state, dtype=np.float32).astype(np.float64)
        vg = np.isfinite(gp) & (gp > 0) & np.isfinite(gs) & (gs > 0)
        pis = state["pi"]
        vs = (pis > 0) & np.isfinite(pis)
        u = uniforms(seed, step_index, n)
        test = u * pis * gp < pip * gs
    take = vp & vs & vg & test
    new = {k: v.copy() for k, v in state.items()}
    if u_prop is not None and "u" in new:
        new["u"][:, take] = np.asarray(u_prop, dtype=np.float32)[:, take]
    new["f"][:, take] = f_prop[:, take]
    new["q"][take] = qp[take]
    new["pi"][take] = pip[take]
    return new, take


def training_data(state, root0_slots):
    """The chains' states as forward-KL training data for a proposal density (Appendix A: samples that
    represent |f|): the coordinates u [D][n] and weights w = p / pi [n], p = sum of |f| over the root-0
    slots (so w = 1 at alpha = 0: the chains sample |f| itself); 0 for a chain without a valid state."""
    pi = state["pi"]
    p = np.zeros(len(pi))
    for s in root0_slots:
        p = p + np.abs(state["f"][s].astype(np.float64))
    ok = pi > 0
    w = np.where(ok, p / np.where(ok, pi, 1.0), 0.0)
    return state["u"].copy(), w


def batch_bounds(n: int, n_batches: int):
    """Chain batch b holds chains [b n // B, (b + 1) n // B)."""
    return [(b * n // n_batches, (b + 1) * n // n_batches) for b in range(n_batches)]


def measure(state, n_batches: int = 1):
    """Per chain batch and slot, the sum over the batch's chains of f/pi and of (f/pi)^2, and the same
    for q/pi: [n_batches][S + 1][2] (a chain without a valid state adds zero)."""
    pi = state["pi"]
    ok = pi > 0
    rows = [state["f"][s].astype(np.float64) for s in range(state["f"].shape[0])] + [state["q"]]
    out = np.zeros((n_batches, len(rows), 2))
    for b, (c0, c1) in enumerate(batch_bounds(len(pi), n_batches)):
        for i, r in enumerate(rows):
            v = np.where(ok[c0:c1], r[c0:c1] / np.where(ok[c0:c1], pi[c0:c1], 1.0), 0.0)
            out[b, i, 0] = np.sum(v)
            out[b, i, 1] = np.sum(v * v)
    return out


def ratio_estimate(sums):
    """I_s = sum f_s/pi / sum q/pi, over the last two axes [S + 1][2] (any leading batch axes)."""
    sums = np.asarray(sums, dtype=np.float64)
    return sums[..., :-1, 0] / sums[..., -1:, 0]
