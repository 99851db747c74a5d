"""Seeded synthetic inputs shared by the tests, the bench and the oracle's timing leg.

Nothing here computes any part of the method: it only draws points of the integration domain
(loop momenta in the ball |q| <= R, imaginary times in [0, beta)), external momenta, VEGAS
grids and histograms with the shapes and value ranges of the workloads, from numpy's
seeded PCG64 stream.
"""
from __future__ import annotations

import numpy as np

R_BALL = 6.0
BETA = 25.0


def dim(n: int) -> int:
    """Integration dimension 3n + (n - 1): n loop momenta, n - 1 free interaction times."""
    return 4 * n - 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def loop_points(n: int, N: int, seed: int, R: float = R_BALL, beta: float = BETA,
                fermi_fraction: float = 0.25, special: bool = True) -> np.ndarray:
    """x[N, D] float32: momenta Cartesian (r uniform in [0, R], direction uniform on the sphere),
    a fraction of them placed within 0.05 of the Fermi surface |q| = 1, and times uniform in
    [0, beta).  With `special`, the first rows hold edge cases: q = 0, equal times on two lines,
    a time at exactly 0 and times at the top of the range."""
    g = rng(seed)
    D = dim(n)
    x = np.empty((N, D), dtype=np.float64)
    for i in range(n):
        r = R * g.random(N)
        near = g.random(N) < fermi_fraction
        r[near] = 1.0 + 0.1 * (g.random(near.sum()) - 0.5)
        c = 2.0 * g.random(N) - 1.0
        s = np.sqrt(1.0 - c * c)
        ph = 2.0 * np.pi * g.random(N)
        x[:, 3 * i] = r * s * np.cos(ph)
        x[:, 3 * i + 1] = r * s * np.sin(ph)
        x[:, 3 * i + 2] = r * c
    x[:, 3 * n:] = beta * g.random((N, n - 1))
    x = x.astype(np.float32)
    if special and N >= 8:
        x[0, 0:3] = 0.0                     # a loop momentum at the origin
        if n >= 2:
            x[1, 3 * n] = 0.0               # tau_1 exactly at the in-vertex time
            x[2, 3 * n] = np.float32(beta) * np.float32(0.999999)
        if n >= 3:
            x[3, 3 * n + 1] = x[3, 3 * n]   # two lines at the same time
        x[4, 0:3] = np.array([0.0, 0.0, 1.0], dtype=np.float32)   # on the Fermi surface
    return x


def k_grid(K: int, kmax: float = 3.0) -> np.ndarray:
    """K external momenta evenly in [0, kmax] (both ends included), float32."""
    return np.linspace(0.0, kmax, K).astype(np.float32)


def vegas_grid(D: int, B: int, seed: int, jitter: float = 0.8) -> np.ndarray:
    """A non-uniform, strictly increasing grid of B bins per dimension: edges[D, B+1] float32
    with edges[:, 0] = 0 and edges[:, B] = 1."""
    g = rng(seed)
    w = 1.0 + jitter * (g.random((D, B)) * 2 - 1)
    w = w / w.sum(axis=1, keepdims=True)
    e = np.zeros((D, B + 1))
    e[:, 1:] = np.cumsum(w, axis=1)
    e[:, B] = 1.0
    return e.astype(np.float32)


def histogram(D: int, B: int, seed: int) -> np.ndarray:
    """A positive per-bin importance histogram [D, B] float64 with a peaked profile."""
    g = rng(seed)
    xb = (np.arange(B) + 0.5) / B
    h = np.empty((D, B))
    for d in range(D):
        c = g.random()
        h[d] = np.exp(-((xb - c) ** 2) / (2 * 0.05 ** 2)) + 0.01 + 0.01 * g.random(B)
    return h


def flow_masks(D: int, n_layers: int, seed: int) -> np.ndarray:
    """Coupling masks int8[n_layers][D] (1 = conditioning, 0 = transformed): a seeded permutation
    of the dimensions, split in halves that alternate roles, a new permutation every two layers."""
    g = rng(seed)
    m = np.zeros((n_layers, D), dtype=np.int8)
    perm = None
    for l in range(n_layers):
        if l % 2 == 0:
            perm = g.permutation(D)
        half = perm[: D // 2] if l % 2 == 0 else perm[D // 2:]
        m[l, half] = 1
    return m


def flow_params(masks: np.ndarray, seed: int, last_scale: float = 0.0) -> np.ndarray:
    """Initial flat FP32 parameters of the coupling networks (per layer W1t[128][16], W2t[128][128],
    b2[128], W3t[32][128], b3[32]).  Hidden weights He-normal; the output layer is scaled by
    `last_scale` (0 gives the identity flow)."""
    g = rng(seed)
    out = []
    for m in masks:
        dA = int(m.sum())
        W1t = np.zeros((128, 16))
        W1t[:, : dA + 1] = g.normal(size=(128, dA + 1)) * np.sqrt(2.0 / (dA + 1))
        W2t = g.normal(size=(128, 128)) * np.sqrt(2.0 / 128)
        b2 = np.zeros(128)
        dB = m.size - dA
        W3t = np.zeros((32, 128))
        W3t[:dB] = g.normal(size=(dB, 128)) * last_scale / np.sqrt(128)
        W3t[16:16 + dB] = g.normal(size=(dB, 128)) * last_scale / np.sqrt(128)
        b3 = np.zeros(32)
        out.append(np.concatenate([W1t.ravel(), W2t.ravel(), b2, W3t.ravel(), b3]))
    return np.concatenate(out).astype(np.float32)


def spline_flow_params(masks: np.ndarray, seed: int, scale: float = 0.0) -> np.ndarray:
    """Flat FP32 parameters of a spline-coupling flow (per layer W1 [32][dA], b1 [32], W2 [32][32], b2 [32],
    W3 [23 dB][32], b3 [23 dB]): He-normal hidden weights, zero hidden biases, output weights normal of
    std `scale`, output biases `scale`-normal around the values whose spline is the identity (width and
    height logits 0, interior-derivative logits log(exp(1 - 1e-3) - 1)).  scale = 0: the identity flow."""
    g = rng(seed)
    ident = np.log(np.exp(1.0 - 1e-3) - 1.0)
    out = []
    for m in masks:
        dA = int(np.sum(m))
        dB = len(m) - dA
        P = 23 * dB
        W1 = g.normal(size=(32, dA)) * np.sqrt(2.0 / dA)
        W2 = g.normal(size=(32, 32)) * np.sqrt(2.0 / 32)
        W3 = g.normal(size=(P, 32)) * scale
        b3 = np.zeros(P)
        for j in range(dB):
            b3[j * 23 + 16:(j + 1) * 23] = ident
        b3 = b3 + g.normal(size=P) * scale
        out += [W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3.ravel(), b3]
    return np.concatenate(out).astype(np.float32)


def chain_proposals(S: int, n: int, seed: int, bad: bool = True):
    """Integrand values f[S][n] float32 (signed, log-uniform magnitudes over six decades) and proposal
    Jacobians jac[n] float32 (log-uniform in [1e-3, 1e3]) for the Markov-chain step; with `bad`, a few
    chains carry a NaN value, an infinite value or a zero Jacobian."""
    g = rng(seed)
    f = (np.sign(g.random((S, n)) - 0.5) * 10.0 ** (6 * g.random((S, n)) - 6)).astype(np.float32)
    jac = (10.0 ** (6 * g.random(n) - 3)).astype(np.float32)
    if bad and n >= 8:
        f[0, 3] = np.nan
        f[S - 1, 5] = np.inf
        jac[6] = 0.0
    return f, jac
