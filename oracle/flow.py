"""Oracle affine-coupling normalizing flow (test infrastructure, FP64 with BF16 emulation).

Follows the coupling transform of Appendix A (eq. coupling_layer): the dimensions are split by a
mask into a conditioning part z_A, left unchanged, and a transformed part z_B, mapped by a
function whose parameters a network computes from z_A.  Here the function is affine,
z_B' = z_B exp(s) + t, with (s_hat, t) = MLP(z_A) and s = S_MAX tanh(s_hat) (a reading: the
workload asks for affine couplings; the paper's own flow uses rational-quadratic splines).
The density follows the change of variables of eq. NFtransform.  Training minimises the forward
KL of Appendix A in its weighted form: L = -sum_i w_i log q(u_i) / sum_i w_i.

Conventions (shared with the library as data, each side with its own code):
  base: u uniform in (0,1)^D, z_0 = logit(u) (a uniform base seen through the logit);
  output: u' = sigmoid(z_K); the flow density of u' is
      log q(u') = sum_d log sig'(z_0,d) - sum_l sum_b s_{l,b} - sum_d log sig'(z_K,d),
  with log sig'(z) = -|z| - 2 log(1 + e^{-|z|}).
  MLP per layer: X1 = [sigmoid(z_A), 1, 0...] (16 wide: the conditioning variables enter in the
  bounded coordinates u_A = sigmoid(z_A) so that the network never sees the logit tails),
  H1 = relu(X1 W1t^T) (the bias of the first layer
  is W1t's column d_A), H2 = relu(H1 W2t^T + b2), O = H2 W3t^T + b3 (32 wide): s_hat_b = O[b],
  t_b = O[16 + b] for b < d_B.
  BF16: every matmul input (weights and activations) is rounded to bfloat16 (round to nearest
  even); products are exact and accumulate in high precision; biases, activations and the
  coupling arithmetic stay in full precision.
  Flat parameter vector, per layer: W1t[128][16], W2t[128][128], b2[128], W3t[32][128], b3[32].
"""
from __future__ import annotations

import numpy as np

H = 128
KIN = 16
NOUT = 32
S_MAX = 2.0
LAYER_SIZE = H * KIN + H * H + H + NOUT * H + NOUT


EMULATE_BF16 = True  # tests of the smooth map (Jacobian determinants, autograd) switch it off


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    if not EMULATE_BF16:
        return np.asarray(x, dtype=np.float64)
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta, n_layers):
    theta = np.asarray(theta, dtype=np.float64)
    layers = []
    o = 0
    for _ in range(n_layers):
        p = {}
        for name, shape in [("W1t", (H, KIN)), ("W2t", (H, H)), ("b2", (H,)), ("W3t", (NOUT, H)), ("b3", (NOUT,))]:
            sz = int(np.prod(shape))
            p[name] = theta[o:o + sz].reshape(shape)
            o += sz
        layers.append(p)
    return layers


def split(mask):
    mask = np.asarray(mask)
    return np.nonzero(mask == 1)[0], np.nonzero(mask == 0)[0]


def mlp(p, zA, dB):
    N, dA = zA.shape
    X1 = np.zeros((N, KIN))
    X1[:, :dA] = sigmoid(zA)
    X1[:, dA] = 1.0
    pre1 = bf16(X1) @ bf16(p["W1t"]).T
    H1 = np.maximum(pre1, 0.0)
    pre2 = bf16(H1) @ bf16(p["W2t"]).T + p["b2"]
    H2 = np.maximum(pre2, 0.0)
    O = bf16(H2) @ bf16(p["W3t"]).T + p["b3"]
    shat = O[:, :dB]
    t = O[:, 16:16 + dB]
    s = S_MAX * np.tanh(shat)
    return s, t, dict(X1=X1, pre1=pre1, H1=H1, pre2=pre2, H2=H2, shat=shat)


def log_sig_prime(z):
    a = np.abs(z)
    return -a - 2.0 * np.log1p(np.exp(-a))


def logit(u):
    u = np.asarray(u, dtype=np.float64)
    return np.log(u) - np.log1p(-u)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(theta, masks, z0):
    """z_0 -> z_K and sum over layers of sum_b s."""
    layers = unpack(theta, len(masks))
    z = np.array(z0, dtype=np.float64)
    ssum = np.zeros(z.shape[0])
    for p, m in zip(layers, masks):
        A, B = split(m)
        s, t, _ = mlp(p, z[:, A], len(B))
        z[:, B] = z[:, B] * np.exp(s) + t
        ssum += s.sum(axis=1)
    return z, ssum


def inverse(theta, masks, zK):
    layers = unpack(theta, len(masks))
    z = np.array(zK, dtype=np.float64)
    ssum = np.zeros(z.shape[0])
    for p, m in reversed(list(zip(layers, masks))):
        A, B = split(m)
        s, t, _ = mlp(p, z[:, A], len(B))
        z[:, B] = (z[:, B] - t) * np.exp(-s)
        ssum += s.sum(axis=1)
    return z, ssum


def sample(theta, masks, u):
    """Base uniforms u -> flow output u' and log q(u')."""
    z0 = logit(u)
    zK, ssum = forward(theta, masks, z0)
    lq = log_sig_prime(z0).sum(axis=1) - ssum - log_sig_prime(zK).sum(axis=1)
    return sigmoid(zK), lq, zK


def log_q(theta, masks, uprime):
    zK = logit(uprime)
    z0, ssum = inverse(theta, masks, zK)
    return log_sig_prime(z0).sum(axis=1) - ssum - log_sig_prime(zK).sum(axis=1)


def loss_and_grad(theta, masks, uprime, w):
    """L = -sum_i w_i log q(u'_i) / sum_i w_i and dL/dtheta, by a hand-written reverse sweep.

    The inverse pass runs layers K..1; the reverse sweep revisits them in order 1..K, recomputing
    each layer's network from the stored states.  Per layer (inverse z_B <- (z_B - t) e^{-s}):
      G_B(in) = G_B(out) e^{-s},  G_t = -G_B(out) e^{-s},  G_s = -G_B(out) z_B(out) + w,
      G_shat = G_s S_MAX (1 - tanh^2), then back through the network; G_A(in) += dL/dz_A.
    BF16 rounding of the gradient operands mirrors the forward: the output gradient and the hidden
    gradients are rounded before every product they feed, and the bias gradients are the sums of
    those rounded values (a convention shared with the library)."""
    L_ = len(masks)
    layers = unpack(theta, L_)
    w = np.asarray(w, dtype=np.float64)
    wn = w / w.sum()
    zK = logit(uprime)
    states = [None] * (L_ + 1)
    z = zK.copy()
    states[L_] = z.copy()
    ssum = np.zeros(z.shape[0])
    for l in reversed(range(L_)):
        A, B = split(masks[l])
        s, t, _ = mlp(layers[l], z[:, A], len(B))
        z[:, B] = (z[:, B] - t) * np.exp(-s)
        ssum += s.sum(axis=1)
        states[l] = z.copy()
    z0 = z
    lq = log_sig_prime(z0).sum(axis=1) - ssum - log_sig_prime(zK).sum(axis=1)
    loss = -(wn * lq).sum()
    grads = []
    G = -wn[:, None] * (1.0 - 2.0 * sigmoid(z0))   # d(-w lq)/dz_0
    for l in range(L_):
        p = layers[l]
        A, B = split(masks[l])
        dA, dB = len(A), len(B)
        zin = states[l]
        s, t, c = mlp(p, zin[:, A], dB)
        zB_out = zin[:, B]                 # state after the inverse layer (= its output)
        GB = G[:, B]
        e = np.exp(-s)
        G_t = -GB * e
        G_s = -GB * zB_out + wn[:, None]
        G_shat = G_s * S_MAX * (1.0 - np.tanh(c["shat"]) ** 2)
        N = zin.shape[0]
        dO = np.zeros((N, NOUT))
        dO[:, :dB] = G_shat
        dO[:, 16:16 + dB] = G_t
        dOb = bf16(dO)
        g = {}
        g["W3t"] = dOb.T @ bf16(c["H2"])
        g["b3"] = dOb.sum(axis=0)
        dH2 = dOb @ bf16(p["W3t"])
        dpre2 = dH2 * (c["pre2"] > 0)
        dpre2b = bf16(dpre2)
        g["W2t"] = dpre2b.T @ bf16(c["H1"])
        g["b2"] = dpre2b.sum(axis=0)
        dH1 = dpre2b @ bf16(p["W2t"])
        dpre1 = dH1 * (c["pre1"] > 0)
        dpre1b = bf16(dpre1)
        g["W1t"] = dpre1b.T @ bf16(c["X1"])
        dX1 = dpre1b @ bf16(p["W1t"])
        Gn = G.copy()
        Gn[:, B] = GB * e
        sA = sigmoid(zin[:, A])
        Gn[:, A] += dX1[:, :dA] * sA * (1.0 - sA)
        G = Gn
        grads.append(np.concatenate([g["W1t"].ravel(), g["W2t"].ravel(), g["b2"], g["W3t"].ravel(), g["b3"]]))
    return loss, np.concatenate(grads)


def mixture_weight(jac, lq, alpha, uniform=0.0, jv=None):
    """Weight of a point drawn from the defensive mixture alpha q + (1 - alpha - uniform) g + uniform u,
    where g is the VEGAS grid's density (1 / J_V in the cube of its outputs) and u the uniform density
    of that cube: jac (the point's physical Jacobian times J_V at its grid coordinates) divided by the
    mixture density in grid coordinates, alpha q + (1 - alpha - uniform) + uniform J_V.  This is the
    balance heuristic of multiple importance sampling (Veach and Guibas 1995); the mixture mirrors the
    alpha-mixed target of eq. target_distr_nf_mcmc_qft_revised.  Unbiased for any split of the samples
    in the proportions of the shares, never above jac / (1 - alpha - uniform) nor above
    (jac / J_V) / uniform."""
    lq = np.asarray(lq, dtype=np.float64)
    jv = np.zeros_like(lq) if jv is None else np.asarray(jv, dtype=np.float64)
    return np.asarray(jac, dtype=np.float64) / (alpha * np.exp(lq) + ((1.0 - alpha - uniform) + uniform * jv))


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma and Ba, 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
