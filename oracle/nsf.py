"""Oracle neural spline flow (test infrastructure; only tests/, the smoke check and the bench's CPU leg use it).

Appendix A: coupling layers (eq. coupling_layer) whose transformed half goes through monotonic rational-
quadratic splines with 8 bins (Durkan et al. 2019), parameters from a residual network with two hidden
layers of 32 ReLU units, and a uniform base distribution.  The flow acts on the VEGAS coordinates
u in [0, 1]^D, so the spline covers [0, 1] in both directions.

Readings (the paper names the parts, not their exact form):
  * residual network: a1 = relu(W1 z_A + b1), a2 = relu(W2 a1 + b2) + a1, theta = W3 a2 + b3 (z_A: the
    coordinates the layer keeps, theta: 3K - 1 values per transformed coordinate);
  * spline parameters of one coordinate, in this order: K width logits, K height logits, K - 1 interior
    derivative logits; widths w = m_w + (1 - K m_w) softmax, heights likewise, interior derivatives
    d = m_d + softplus, boundary derivatives 1; m_w = m_h = m_d = 1e-3 (Durkan et al.'s defaults);
  * the forward map of one coordinate in bin k (knots x_k, y_k, width W, height H, s = H / W,
    derivatives d_k, d_{k+1}, xi = (x - x_k) / W):
        y = y_k + H (s xi^2 + d_k xi (1 - xi)) / (s + (d_{k+1} + d_k - 2 s) xi (1 - xi)),
        dy/dx = s^2 (d_{k+1} xi^2 + 2 s xi (1 - xi) + d_k (1 - xi)^2) / (s + (d_{k+1} + d_k - 2 s) xi (1 - xi))^2;
    the inverse solves the quadratic for xi (the root in [0, 1]);
  * bin search: the last knot <= the argument (clamped to 0..K-1);
  * log q(u) = -sum over layers of log dy/dx along the forward path from the base point z (uniform base:
    log p(z) = 0).
Layer parameters are a flat FP32 vector per layer: W1 [H][dA], b1 [H], W2 [H][H], b2 [H], W3 [P][H],
b3 [P] (H = 32, P = (3K - 1) dB, row-major), layers concatenated.
"""
from __future__ import annotations

import math

import numpy as np

K_BINS = 8
HIDDEN = 32
MIN_W = MIN_H = MIN_D = 1e-3
IDENTITY_D = math.log(math.exp(1.0 - MIN_D) - 1.0)   # softplus^-1(1 - MIN_D): interior derivatives 1


def layer_dims(mask):
    """mask[D]: 1 = kept (conditioner input), 0 = transformed."""
    a = [i for i, m in enumerate(mask) if m]
    b = [i for i, m in enumerate(mask) if not m]
    return a, b


def layer_param_count(dA, dB, K=K_BINS, H=HIDDEN):
    P = (3 * K - 1) * dB
    return H * dA + H + H * H + H + P * H + P


def unpack_layer(theta, dA, dB, K=K_BINS, H=HIDDEN):
    P = (3 * K - 1) * dB
    o = 0
    out = {}
    for name, shape in [("W1", (H, dA)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (P, H)), ("b3", (P,))]:
        sz = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + sz], dtype=np.float64).reshape(shape)
        o += sz
    return out


def identity_params(masks, rng=None, scale=0.0, K=K_BINS, H=HIDDEN):
    """Parameters of the identity flow (W3 = 0, derivative biases at the identity value); with rng and
    scale > 0 the first two layers of every conditioner are random (He-like) and W3, b3 get noise of
    that scale, so the flow is a nearby, non-trivial map."""
    parts = []
    for mask in masks:
        a, b = layer_dims(mask)
        dA, dB = len(a), len(b)
        P = (3 * K - 1) * dB
        W1 = np.zeros((H, dA)) if rng is None else rng.normal(size=(H, dA)) * math.sqrt(2.0 / max(dA, 1))
        W2 = np.zeros((H, H)) if rng is None else rng.normal(size=(H, H)) * math.sqrt(2.0 / H)
        b1 = np.zeros(H)
        b2 = np.zeros(H)
        W3 = np.zeros((P, H)) if rng is None or scale == 0 else rng.normal(size=(P, H)) * scale
        b3 = np.zeros(P)
        for j in range(dB):
            b3[j * (3 * K - 1) + 2 * K: (j + 1) * (3 * K - 1)] = IDENTITY_D
        if rng is not None and scale:
            b3 = b3 + rng.normal(size=P) * scale
        parts += [W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3]
    return np.concatenate(parts)


def conditioner(zA, p):
    """zA [N, dA] -> (theta [N, P], a1, a2, pre1, pre2)."""
    pre1 = zA @ p["W1"].T + p["b1"]
    a1 = np.maximum(pre1, 0.0)
    pre2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(pre2, 0.0) + a1
    theta = a2 @ p["W3"].T + p["b3"]
    return theta, a1, a2, pre1, pre2


def _softmax(t):
    m = t.max(axis=-1, keepdims=True)
    e = np.exp(t - m)
    return e / e.sum(axis=-1, keepdims=True)


def _softplus(t):
    return np.log1p(np.exp(-np.abs(t))) + np.maximum(t, 0.0)


def spline_knots(th, K=K_BINS):
    """th [N, 3K - 1] -> knots x [N, K + 1], y [N, K + 1], derivatives d [N, K + 1]."""
    w = MIN_W + (1 - K * MIN_W) * _softmax(th[:, :K])
    h = MIN_H + (1 - K * MIN_H) * _softmax(th[:, K:2 * K])
    d_in = MIN_D + _softplus(th[:, 2 * K:])
    N = th.shape[0]
    x = np.concatenate([np.zeros((N, 1)), np.cumsum(w, axis=1)], axis=1)
    y = np.concatenate([np.zeros((N, 1)), np.cumsum(h, axis=1)], axis=1)
    x[:, -1] = 1.0
    y[:, -1] = 1.0
    d = np.concatenate([np.ones((N, 1)), d_in, np.ones((N, 1))], axis=1)
    return x, y, d


def _bin(knots, v, K):
    k = np.sum(knots[:, 1:K] <= v[:, None], axis=1)
    return np.clip(k, 0, K - 1)


def spline_forward(v, th, K=K_BINS):
    """v [N] in [0, 1] -> (y [N], log dy/dx [N])."""
    x, y, d = spline_knots(th, K)
    k = _bin(x, v, K)
    r = np.arange(len(v))
    xk, W = x[r, k], x[r, k + 1] - x[r, k]
    yk, Hh = y[r, k], y[r, k + 1] - y[r, k]
    dk, dk1 = d[r, k], d[r, k + 1]
    s = Hh / W
    xi = (v - xk) / W
    t = xi * (1 - xi)
    den = s + (dk1 + dk - 2 * s) * t
    out = yk + Hh * (s * xi * xi + dk * t) / den
    dydx = s * s * (dk1 * xi * xi + 2 * s * t + dk * (1 - xi) ** 2) / (den * den)
    return out, np.log(dydx)


def spline_inverse(v, th, K=K_BINS):
    """v [N] in [0, 1] (a spline output) -> (x [N], log dy/dx [N] at x)."""
    x, y, d = spline_knots(th, K)
    k = _bin(y, v, K)
    r = np.arange(len(v))
    xk, W = x[r, k], x[r, k + 1] - x[r, k]
    yk, Hh = y[r, k], y[r, k + 1] - y[r, k]
    dk, dk1 = d[r, k], d[r, k + 1]
    s = Hh / W
    dy = v - yk
    g = dk1 + dk - 2 * s
    a = Hh * (s - dk) + dy * g
    b = Hh * dk - dy * g
    c = -s * dy
    disc = np.maximum(b * b - 4 * a * c, 0.0)
    xi = 2 * c / (-b - np.sqrt(disc))
    xo = xk + xi * W
    t = xi * (1 - xi)
    den = s + g * t
    dydx = s * s * (dk1 * xi * xi + 2 * s * t + dk * (1 - xi) ** 2) / (den * den)
    return xo, np.log(dydx)


def forward(z, masks, params, K=K_BINS, H=HIDDEN):
    """Base points z [N, D] -> (u [N, D], log q(u) [N])."""
    u = np.array(z, dtype=np.float64)
    lq = np.zeros(u.shape[0])
    o = 0
    for mask in masks:
        a, b = layer_dims(mask)
        n_p = layer_param_count(len(a), len(b), K, H)
        p = unpack_layer(params[o:o + n_p], len(a), len(b), K, H)
        o += n_p
        theta = conditioner(u[:, a], p)[0]
        for j, col in enumerate(b):
            u[:, col], ld = spline_forward(u[:, col], theta[:, j * (3 * K - 1):(j + 1) * (3 * K - 1)], K)
            lq -= ld
    return u, lq


def log_density(u, masks, params, K=K_BINS, H=HIDDEN):
    """log q(u) [N] by the inverse layers; also returns the base points z [N, D]."""
    z = np.array(u, dtype=np.float64)
    lq = np.zeros(z.shape[0])
    offs = []
    o = 0
    for mask in masks:
        a, b = layer_dims(mask)
        n_p = layer_param_count(len(a), len(b), K, H)
        offs.append((o, n_p))
        o += n_p
    for mask, (o, n_p) in reversed(list(zip(masks, offs))):
        a, b = layer_dims(mask)
        p = unpack_layer(params[o:o + n_p], len(a), len(b), K, H)
        theta = conditioner(z[:, a], p)[0]
        for j, col in enumerate(b):
            z[:, col], ld = spline_inverse(z[:, col], theta[:, j * (3 * K - 1):(j + 1) * (3 * K - 1)], K)
            lq -= ld
    return lq, z


def loss_and_grad_torch(u, w, masks, params, K=K_BINS, H=HIDDEN):
    """L = -sum w log q(u) / sum w and dL/dparams by torch autograd on the CPU in FP64 (the reference
    for the library's hand-written reverse sweep)."""
    import torch
    th = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    z = torch.tensor(np.asarray(u, dtype=np.float64))
    lq = torch.zeros(z.shape[0], dtype=torch.float64)
    offs = []
    o = 0
    for mask in masks:
        a, b = layer_dims(mask)
        n_p = layer_param_count(len(a), len(b), K, H)
        offs.append((o, n_p))
        o += n_p
    cols = [z[:, i] for i in range(z.shape[1])]
    for mask, (o, n_p) in reversed(list(zip(masks, offs))):
        a, b = layer_dims(mask)
        dA, dB = len(a), len(b)
        P = (3 * K - 1) * dB
        q = 0
        W1 = th[o + q:o + q + H * dA].reshape(H, dA); q += H * dA
        b1 = th[o + q:o + q + H]; q += H
        W2 = th[o + q:o + q + H * H].reshape(H, H); q += H * H
        b2 = th[o + q:o + q + H]; q += H
        W3 = th[o + q:o + q + P * H].reshape(P, H); q += P * H
        b3 = th[o + q:o + q + P]
        zA = torch.stack([cols[i] for i in a], dim=1)
        a1 = torch.relu(zA @ W1.T + b1)
        a2 = torch.relu(a1 @ W2.T + b2) + a1
        theta = a2 @ W3.T + b3
        for j, col in enumerate(b):
            t = theta[:, j * (3 * K - 1):(j + 1) * (3 * K - 1)]
            wdt = MIN_W + (1 - K * MIN_W) * torch.softmax(t[:, :K], dim=1)
            hgt = MIN_H + (1 - K * MIN_H) * torch.softmax(t[:, K:2 * K], dim=1)
            din = MIN_D + torch.nn.functional.softplus(t[:, 2 * K:])
            N = t.shape[0]
            xk_all = torch.cat([torch.zeros(N, 1, dtype=t.dtype), torch.cumsum(wdt, 1)[:, :-1]], 1)
            yk_all = torch.cat([torch.zeros(N, 1, dtype=t.dtype), torch.cumsum(hgt, 1)[:, :-1]], 1)
            dd = torch.cat([torch.ones(N, 1, dtype=t.dtype), din, torch.ones(N, 1, dtype=t.dtype)], 1)
            v = cols[col]
            # the bin (a discrete choice, no gradient) from the same knots as the numpy oracle
            ycum = torch.cumsum(hgt, 1).detach().numpy()
            k = np.clip(np.sum(ycum[:, :K - 1] <= v.detach().numpy()[:, None], axis=1), 0, K - 1)
            r = torch.arange(N)
            kk = torch.tensor(k)
            W = wdt[r, kk]
            Hh = hgt[r, kk]
            xk = xk_all[r, kk]
            yk = yk_all[r, kk]
            dk = dd[r, kk]
            dk1 = dd[r, kk + 1]
            s = Hh / W
            dy = v - yk
            g = dk1 + dk - 2 * s
            aa = Hh * (s - dk) + dy * g
            bb = Hh * dk - dy * g
            cc = -s * dy
            xi = 2 * cc / (-bb - torch.sqrt(torch.clamp(bb * bb - 4 * aa * cc, min=0.0)))
            tt = xi * (1 - xi)
            den = s + g * tt
            dydx = s * s * (dk1 * xi * xi + 2 * s * tt + dk * (1 - xi) ** 2) / (den * den)
            cols[col] = xk + xi * W
            lq = lq - torch.log(dydx)
    wt = torch.tensor(np.asarray(w, dtype=np.float64))
    L = -(wt * lq).sum() / wt.sum()
    L.backward()
    return float(L.detach()), th.grad.numpy().copy(), lq.detach().numpy()
