"""Oracle sampler: Philox4x32-10, the VEGAS map and its refinement (test infrastructure).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key, ten rounds
of two 32 x 32 -> 64 multiplies with the multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped
by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

Counter convention (a reading; the paper names no generator): draw d of sample i uses counter
(i mod 2^32, i div 2^32, d div 4, 0) and word d mod 4, with key (seed mod 2^32, seed div 2^32).
A 32-bit word w becomes the 24-bit integer m = w >> 8 and the open-interval uniform
u = (m + 1/2) 2^-24.

VEGAS map (Lepage, J. Comput. Phys. 27 (1978), which the paper cites in Sec. IV): per dimension
B bins with edges e_0 = 0 < e_1 < ... < e_B = 1; u falls in bin b = floor(u B) at fraction
t = u B - b and maps to y = e_b + t (e_{b+1} - e_b) with Jacobian B (e_{b+1} - e_b).  For a
Philox uniform, b and t come from the integer (2m + 1) B so the bin choice is exact.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: uint64 array [..., 4] (values < 2^32); key: [..., 2].  Returns uint64 [..., 4]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def raw_words(seed: int, first: int, N: int, D: int):
    """32-bit words [N, D] for samples first..first+N-1."""
    i = np.arange(first, first + N, dtype=np.uint64)
    nblk = (D + 3) // 4
    key = np.array([seed & MASK, (seed >> 32) & MASK], dtype=np.uint64)
    out = np.empty((N, nblk * 4), dtype=np.uint64)
    for b in range(nblk):
        ctr = np.stack([i & np.uint64(MASK), i >> np.uint64(32),
                        np.full(N, b, dtype=np.uint64), np.zeros(N, dtype=np.uint64)], axis=-1)
        out[:, 4 * b: 4 * b + 4] = philox4x32_10(ctr, np.broadcast_to(key, (N, 2)))
    return out[:, :D]


def uniforms(seed: int, first: int, N: int, D: int):
    m = raw_words(seed, first, N, D) >> np.uint64(8)
    return (m.astype(np.float64) + 0.5) * 2.0 ** -24, m


def vegas_map_int(m, edges):
    """Map 24-bit integers m[N, D] through the grid edges[D, B+1] (FP64): returns y, J_V."""
    edges = np.asarray(edges, dtype=np.float64)
    D, B1 = edges.shape
    B = B1 - 1
    t = (2 * m.astype(np.int64) + 1) * B
    b = (t >> 25).astype(np.int64)
    frac = (t & ((1 << 25) - 1)).astype(np.float64) * 2.0 ** -25
    y = np.empty(m.shape)
    J = np.ones(m.shape[0])
    for d in range(D):
        lo = edges[d, b[:, d]]
        hi = edges[d, b[:, d] + 1]
        y[:, d] = lo + frac[:, d] * (hi - lo)
        J *= B * (hi - lo)
    return y, J, b


def vegas_map_float(u, edges):
    """Map continuous uniforms u[N, D] (float32, e.g. from a flow): the bin index is taken in
    float32 as floor(u * B), as a float32 kernel takes it, clamped to B - 1."""
    edges = np.asarray(edges, dtype=np.float64)
    D, B1 = edges.shape
    B = B1 - 1
    u32 = np.asarray(u, dtype=np.float32)
    ub = u32 * np.float32(B)
    b = np.minimum(np.floor(ub).astype(np.int64), B - 1)
    frac = ub.astype(np.float64) - b
    y = np.empty(u32.shape)
    J = np.ones(u32.shape[0])
    for d in range(D):
        lo = edges[d, b[:, d]]
        hi = edges[d, b[:, d] + 1]
        y[:, d] = lo + frac[:, d] * (hi - lo)
        J *= B * (hi - lo)
    return y, J, b


def vegas_inverse(y, edges):
    """Inverse of the VEGAS map: for points y[N, D] in the unit cube, the bin b with
    e_b <= y < e_{b+1} (clamped to the grid), the grid coordinate u' = (b + (y - e_b) / (e_{b+1} - e_b)) / B
    and the Jacobian J_V = prod_d B (e_{b+1} - e_b) of the forward map at u'."""
    edges = np.asarray(edges, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    D, B1 = edges.shape
    B = B1 - 1
    u = np.empty(y.shape)
    J = np.ones(y.shape[0])
    for d in range(D):
        b = np.clip(np.searchsorted(edges[d], y[:, d], side="right") - 1, 0, B - 1)
        lo, hi = edges[d, b], edges[d, b + 1]
        u[:, d] = (b + np.minimum((y[:, d] - lo) / (hi - lo), 1.0)) / B
        J *= B * (hi - lo)
    return u, J


def refine_grid(edges, hist, alpha=0.5):
    """One VEGAS grid refinement (Lepage 1978), FP64.

    hist[D, B] holds per-bin sums of (integrand x Jacobian)^2.  Per dimension: smooth with
    the neighbours (interior (h_{b-1} + h_b + h_{b+1})/3, ends (h_0 + h_1)/2 and
    (h_{B-2} + h_{B-1})/2), normalise to sum 1, compress each r_b to ((1 - r_b)/ln(1/r_b))^alpha
    (r_b = 0 -> 0, r_b = 1 -> 1), then place new edges so that every new bin holds an equal
    share of the compressed weight, assuming the weight is uniform inside each old bin."""
    edges = np.asarray(edges, dtype=np.float64)
    D, B1 = edges.shape
    B = B1 - 1
    new = np.empty_like(edges)
    for d in range(D):
        h = np.asarray(hist[d], dtype=np.float64)
        s = np.empty(B)
        s[0] = (h[0] + h[1]) / 2
        s[B - 1] = (h[B - 2] + h[B - 1]) / 2
        s[1:B - 1] = (h[:-2] + h[1:-1] + h[2:]) / 3
        tot = s.sum()
        if not (tot > 0):
            new[d] = edges[d]
            continue
        r = s / tot
        w = np.zeros(B)
        for b in range(B):
            if r[b] >= 1.0:
                w[b] = 1.0
            elif r[b] > 0:
                w[b] = ((1.0 - r[b]) / math.log(1.0 / r[b])) ** alpha
        per = w.sum() / B
        ne = np.empty(B + 1)
        ne[0] = 0.0
        ne[B] = 1.0
        acc = 0.0
        ob = 0
        for j in range(1, B):
            target = j * per
            while ob < B and acc + w[ob] < target:
                acc += w[ob]
                ob += 1
            lo, hi = edges[d, ob], edges[d, ob + 1]
            ne[j] = lo + (target - acc) / w[ob] * (hi - lo)
        new[d] = ne
    return new


def physical_map_f64(y, n, beta, R):
    """Same map as integrand.physical_map, returning Cartesian x and the Jacobian (FP64)."""
    from .integrand import physical_map
    return physical_map(y, n, beta, R)
