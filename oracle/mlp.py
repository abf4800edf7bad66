"""Fitness-surrogate network in float64: a multilayer perceptron with GELU
hidden layers, its loss, analytic gradients, Adam update, parameter
initialisation, the per-gene standardisation of its inputs and the
Spearman rank correlation used to assess it.

Test infrastructure (see ``oracle/__init__.py``).  The network maps a
chromosome's genes to a standardised log error:

    Z1 = X W1^T + b1,  H1 = gelu(Z1)
    Z2 = H1 W2^T + b2, H2 = gelu(Z2)
    y  = H2 w3^T + b3
    loss = mean((y - target)^2)

with gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.  Parameter order
everywhere: W1 [H1 x In], b1, W2 [H2 x H1], b2, w3 [1 x H2], b3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .philox import block

STREAM_SURROGATE = 3
_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + special.erf(z * _SQRT1_2))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + special.erf(z * _SQRT1_2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def shapes(n_in: int, hidden=(256, 256)):
    h1, h2 = hidden
    return [(h1, n_in), (h1,), (h2, h1), (h2,), (1, h2), (1,)]


def init_params(n_in: int, seed: int, hidden=(256, 256)):
    """Weights uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero.

    Draws: Philox key (seed, 3), counter (0, tensor, element, 0); the uniform
    is u = (lo32(o0) >> 8) 2^-24 in [0, 1) and the weight
    float32(2u - 1) * float32(1/sqrt(fan_in)), one float32 rounding per
    step (2u - 1 is exact)."""
    params = []
    for ti, shp in enumerate(shapes(n_in, hidden)):
        if len(shp) == 1:
            params.append(np.zeros(shp, dtype=np.float32))
            continue
        n = shp[0] * shp[1]
        b = block(seed, STREAM_SURROGATE, 0, ti, np.arange(n, dtype=np.uint64))
        u = ((b[:, 0] & np.uint64(0xFFFFFFFF)) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
        scale = np.float32(1.0 / math.sqrt(shp[1]))
        w = (np.float32(1.0) * (2.0 * u - 1.0).astype(np.float32)) * scale
        params.append(w.astype(np.float32).reshape(shp))
    return params


def forward(params, X):
    """Returns (y [B], cache) with every intermediate in float64."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, dtype=np.float64) for p in params)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    y = H2 @ w3.T[:, 0] + b3[0]
    return y, (X, Z1, H1, Z2, H2)


def loss(params, X, target):
    y, _ = forward(params, X)
    r = y - np.asarray(target, dtype=np.float64)
    return float(np.mean(r * r))


def backward(params, X, target):
    """Analytic gradients of `loss` with respect to every parameter."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, dtype=np.float64) for p in params)
    y, (X, Z1, H1, Z2, H2) = forward(params, X)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(target, dtype=np.float64)) / B        # [B]
    dw3 = dy[None, :] @ H2                                            # [1, H2]
    db3 = np.array([dy.sum()])
    dZ2 = (dy[:, None] * w3[0][None, :]) * gelu_grad(Z2)              # [B, H2]
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)                                  # [B, H1]
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return [dW1, db1, dW2, db2, dw3, db3]


def adam_step(params, grads, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; step counts from
    1.  Returns new (params, m, v) in float64."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        g = np.asarray(g, dtype=np.float64)
        mm = beta1 * np.asarray(mm, dtype=np.float64) + (1 - beta1) * g
        vv = beta2 * np.asarray(vv, dtype=np.float64) + (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** step)
        vh = vv / (1 - beta2 ** step)
        out_p.append(np.asarray(p, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


INPUT_STD_FLOOR = 1e-3


def input_stats(genes, floor=INPUT_STD_FLOOR):
    """Per-gene mean and inverse standard deviation of archived chromosomes
    [rows x K]: float64 moments, population form (divide by the row count),
    the deviation floored at `floor`, each rounded once to float32."""
    G = np.asarray(genes, dtype=np.float64)
    mean = G.mean(axis=0)
    var = np.maximum((G * G).mean(axis=0) - mean * mean, 0.0)
    inv = 1.0 / np.maximum(np.sqrt(var), floor)
    return mean.astype(np.float32), inv.astype(np.float32)


def standardize(genes, mean, inv_std):
    """The network's inputs: (g - mean) * inv_std per gene, each step one
    float32 rounding."""
    G = np.asarray(genes, dtype=np.float32)
    return ((G - np.asarray(mean, np.float32)).astype(np.float32) *
            np.asarray(inv_std, np.float32)).astype(np.float32)


def ranks(a):
    """Ranks 0..n-1 by (value, index): ties take distinct ranks by index."""
    a = np.asarray(a)
    order = np.lexsort((np.arange(a.size), a))
    r = np.empty(a.size, dtype=np.float64)
    r[order] = np.arange(a.size)
    return r


def spearman(a, b):
    """Pearson correlation of the rank vectors (ties broken by index)."""
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = math.sqrt(float(ra @ ra) * float(rb @ rb))
    return float(ra @ rb) / den if den > 0 else 0.0
