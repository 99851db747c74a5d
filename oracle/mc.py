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
