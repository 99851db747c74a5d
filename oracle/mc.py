"""Oracle plain Monte Carlo integrator (test infrastructure, FP64).

The estimator is eq. nf_mcmc_estimator_qft_final_revised with alpha = 1 (pi = q, every
proposal accepted), which is plain importance sampling: I = (1/N) sum_i f(x_i) / q(x_i).
Here q is the uniform physical map of the unit cube (1/q = Jacobian), and the standard error
is the FP64 sample standard deviation over sqrt(N).  Random numbers come from numpy's
PCG64 stream, seeded; nothing is shared with the library's Philox sampler.
"""
from __future__ import annotations

import numpy as np

from . import integrand as ig


def plain_mc(n, ks, beta, mu, lam, gamma, R=6.0, N=1 << 16, seed=12345, chunk=1 << 14,
             diagrams=None):
    """Estimate Sigma^(n)(k, i w_0) for each k in ks; returns (mean[K], stderr[K]) complex."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = np.atleast_1d(np.asarray(ks, dtype=np.float64))
    s1 = np.zeros(len(ks), dtype=np.complex128)
    s2r = np.zeros(len(ks))
    s2i = np.zeros(len(ks))
    done = 0
    while done < N:
        m = min(chunk, N - done)
        y = rng.random((m, ig.dim(n)))
        x, J = ig.physical_map(y, n, beta, R)
        for a, k in enumerate(ks):
            w = ig.integrand(x, n, k, beta, mu, lam, gamma, diagrams) * J
            s1[a] += w.sum()
            s2r[a] += (w.real ** 2).sum()
            s2i[a] += (w.imag ** 2).sum()
        done += m
    mean = s1 / N
    var_r = (s2r / N - mean.real ** 2) / (N - 1)
    var_i = (s2i / N - mean.imag ** 2) / (N - 1)
    err = np.sqrt(np.maximum(var_r, 0)) + 1j * np.sqrt(np.maximum(var_i, 0))
    return mean, err


def radial_mixture_points(n, N, rng, beta, R=6.0, shell=(0.85, 1.15), p_shell=0.5):
    """Proposal for the oracle's importance sampling: each loop momentum's length is drawn with probability
    p_shell uniformly from the shell around the Fermi momentum, else uniformly from [0, R]; its direction is
    isotropic; times are uniform in [0, beta).  Returns (x [N, 4n - 1], 1/q [N]) with q the proposal density
    (per loop: (p_shell [r in shell] / (shell width) + (1 - p_shell) / R) / (4 pi r^2); per time 1/beta)."""
    a, b = shell
    x = np.empty((N, ig.dim(n)))
    invq = np.ones(N)
    for j in range(n):
        u = rng.random(N)
        in_shell = rng.random(N) < p_shell
        r = np.where(in_shell, a + (b - a) * u, R * u)
        dens = (p_shell * ((r >= a) & (r <= b)) / (b - a) + (1 - p_shell) / R) / (4 * np.pi * r * r)
        c = 2 * rng.random(N) - 1
        s = np.sqrt(np.maximum(0.0, 1 - c * c))
        ph = 2 * np.pi * rng.random(N)
        x[:, 3 * j] = r * s * np.cos(ph)
        x[:, 3 * j + 1] = r * s * np.sin(ph)
        x[:, 3 * j + 2] = r * c
        invq /= dens
    for j in range(n - 1):
        x[:, 3 * n + j] = beta * rng.random(N)
    invq *= beta ** (n - 1)
    return x, invq


def importance_mc(n, ks, beta, mu, lam, gamma, diagrams, N=1 << 20, seed=777, chunk=1 << 16, R=6.0, batches=32):
    """Sigma^(n)(k, i w_0) for each k by importance sampling from radial_mixture_points, every sample through
    the C integrand (cevaluate.py: the same products as integrand.py).  The error is the scatter of `batches`
    independent batch means (robust to heavy tails of the weights).  Returns (mean[K], stderr[K]) complex."""
    from . import cevaluate as ce
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = np.atleast_1d(np.asarray(ks, dtype=np.float64))
    tab = ce.table(diagrams, n)
    per = N // batches
    means = np.zeros((batches, len(ks)), dtype=np.complex128)
    for b in range(batches):
        s = np.zeros(len(ks), dtype=np.complex128)
        done = 0
        while done < per:
            m = min(chunk, per - done)
            x, w = radial_mixture_points(n, m, rng, beta, R)
            for a, k in enumerate(ks):
                s[a] += np.sum(ce.integrand(x, n, k, beta, mu, lam, gamma, diagrams, tab=tab) * w)
            done += m
        means[b] = s / per
    mean = means.mean(axis=0)
    err = (means.real.std(axis=0, ddof=1) + 1j * means.imag.std(axis=0, ddof=1)) / np.sqrt(batches)
    return mean, err


def vegas_mc(n, ks, beta, mu, lam, gamma, diagrams, N=1 << 18, adapt=5, N_adapt=1 << 16, bins=50, batches=32,
             seed=4321, R=6.0, chunk=1 << 15, alpha=0.5):
    """Sigma^(n)(k, i w_0) by VEGAS importance sampling with the oracle's own grid (sampler.py's map and
    refinement, numpy PCG64 uniforms, every sample through the C integrand): `adapt` refinements on N_adapt
    points each (importance sum_k |Re f| + |Im f| times the Jacobian; histogram of its square per bin), then N
    points from the frozen grid in `batches` independent batches; the error is the scatter of the batch means.
    Returns (mean[K], stderr[K]) complex."""
    from . import cevaluate as ce
    from . import sampler as osp
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = np.atleast_1d(np.asarray(ks, dtype=np.float64))
    D = ig.dim(n)
    tab = ce.table(diagrams, n)
    edges = np.tile(np.linspace(0.0, 1.0, bins + 1), (D, 1))

    def weights(m):
        u = rng.random((m, D)).astype(np.float32).astype(np.float64)
        y, JV, b = osp.vegas_map_float(u, edges)
        x, JP = ig.physical_map(y, n, beta, R)
        w = [ce.integrand(x, n, k, beta, mu, lam, gamma, diagrams, tab=tab) * (JV * JP) for k in ks]
        return np.array(w), b

    for _ in range(adapt):
        hist = np.zeros((D, bins))
        done = 0
        while done < N_adapt:
            m = min(chunk, N_adapt - done)
            w, b = weights(m)
            imp2 = (np.abs(w.real) + np.abs(w.imag)).sum(axis=0) ** 2
            for d in range(D):
                hist[d] += np.bincount(b[:, d], weights=imp2, minlength=bins)
            done += m
        edges = osp.refine_grid(edges, hist, alpha)
    per = N // batches
    means = np.zeros((batches, len(ks)), dtype=np.complex128)
    for bi in range(batches):
        s = np.zeros(len(ks), dtype=np.complex128)
        done = 0
        while done < per:
            m = min(chunk, per - done)
            w, _ = weights(m)
            s += w.sum(axis=1)
            done += m
        means[bi] = s / per
    mean = means.mean(axis=0)
    err = (means.real.std(axis=0, ddof=1) + 1j * means.imag.std(axis=0, ddof=1)) / np.sqrt(batches)
    return mean, err
