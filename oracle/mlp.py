"""Oracle for the sketch-rank model: features, MLP forward/backward, loss, Adam.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  FP64 throughout, written
out by hand (no autograd).

Model: x (35) -> Linear(35,128) -> GELU -> Linear(128,128) -> GELU -> Linear(128,1)
with the exact GELU(x) = x/2 (1 + erf(x / sqrt 2)).

Features of one bond (35 values):
    [log2(chi_max)/11, d/4, -log10(eps)/16,
     q_0 .. q_31 with q_t = clamp(log10(s_j / s_0) / 16, -1, 0),
     j = floor((t + 1/2) / 32 * (len(s) - 1))]
where s is the previous (descending) spectrum of the bond.
Target: log2 chi*(eps) of the bond after the update.
Loss: pinball (quantile) loss with tau = 0.9, averaged over the batch:
    rho(u) = max(tau u, (tau - 1) u),  u = target - prediction.
Sketch rank from a prediction y: k = 32 * ceil((1.5 * 2^y + 32) / 32); the
plain truncated SVD is used instead when y > log2(chi_max) or k > n / 4.  (The
oversampling follows the randomized-SVD error bound of Halko, Martinsson and
Tropp: with q power iterations the residual of the kept triplet j scales like
(s_{k+1}/s_j)^(2q+1), so a slowly decaying spectrum needs k well above chi*.)
Parameters are stored flat in the order W1 (128x35, row-major), b1, W2
(128x128), b2, W3 (1x128), b3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_H = 35, 128
SIZES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (1, N_H), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)
TAU = 0.9


def features(s, chi_max: int, d: int, eps: float) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(N_IN)
    out[0] = math.log2(chi_max) / 11.0
    out[1] = d / 4.0
    out[2] = -math.log10(eps) / 16.0
    L = len(s)
    for t in range(32):
        j = int(math.floor((t + 0.5) / 32.0 * (L - 1))) if L > 1 else 0
        if s[0] > 0 and s[j] > 0:
            q = math.log10(s[j] / s[0]) / 16.0
        else:
            q = -1.0
        out[3 + t] = min(0.0, max(-1.0, q))
    return out


def sketch_rank(y: float, n: int, chi_max: int):
    """Returns the sketch rank, or None for 'plain truncated SVD'."""
    if y > math.log2(chi_max):
        return None
    k = 32 * math.ceil((2.0 ** y * 1.5 + 32.0) / 32.0)
    if 4 * k > n:
        return None
    return k


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[off:off + n].reshape(s))
        off += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights: U(-sqrt(6/fan_in), +sqrt(6/fan_in)); zero biases.
    Uniforms come from the Philox stream (seed, stream 7), u = (x + 0.5) 2^-32."""
    from . import philox_blocks
    nw = N_H * N_IN + N_H * N_H + N_H
    blocks = philox_blocks(seed, 7, 0, (nw + 3) // 4).astype(np.float64)
    u = (blocks[:nw] + 0.5) * 2.0 ** -32
    w1 = (2 * u[: N_H * N_IN] - 1) * math.sqrt(6.0 / N_IN)
    w2 = (2 * u[N_H * N_IN: N_H * N_IN + N_H * N_H] - 1) * math.sqrt(6.0 / N_H)
    w3 = (2 * u[N_H * N_IN + N_H * N_H:] - 1) * math.sqrt(6.0 / N_H)
    return pack([w1.reshape(N_H, N_IN), np.zeros(N_H), w2.reshape(N_H, N_H), np.zeros(N_H),
                 w3.reshape(1, N_H), np.zeros(1)])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, x):
    """x: (batch, 35).  Returns prediction (batch,) and the cache for backward."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ w1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ w2.T + b2
    h2 = gelu(z2)
    y = (h2 @ w3.T + b3)[:, 0]
    return y, (x, z1, h1, z2, h2)


def pinball(y, t, tau=TAU):
    u = np.asarray(t, dtype=np.float64) - y
    return float(np.mean(np.maximum(tau * u, (tau - 1.0) * u)))


def loss_and_grad(theta, x, t, tau=TAU):
    """Mean pinball loss and its gradient w.r.t. the flat parameters.
    At u = 0 the subgradient -tau / batch is used (u < 0 gives (1 - tau) / batch)."""
    w1, b1, w2, b2, w3, b3 = unpack(theta)
    y, (x, z1, h1, z2, h2) = forward(theta, x)
    nb = len(y)
    u = np.asarray(t, dtype=np.float64) - y
    g_y = np.where(u < 0, (1.0 - tau), -tau) / nb            # d loss / d y
    gw3 = g_y[None, :] @ h2                                 # (1, 128)
    gb3 = np.array([g_y.sum()])
    g_h2 = g_y[:, None] * w3                                 # (batch, 128)
    g_z2 = g_h2 * gelu_grad(z2)
    gw2 = g_z2.T @ h1
    gb2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ w2
    g_z1 = g_h1 * gelu_grad(z1)
    gw1 = g_z1.T @ x
    gb1 = g_z1.sum(axis=0)
    return pinball(y, t, tau), pack([gw1, gb1, gw2, gb2, gw3, gb3])


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); step counts from 1.  Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
