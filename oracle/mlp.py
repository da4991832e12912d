"""FP64 reference of the learned initialiser's network (forward, loss, backward, Adam).

TEST INFRASTRUCTURE ONLY (oracle).  NumPy, no GPU code.

Network: 4 standardised inputs (a, T/T_c, R, nu_g/nu_l) -> three hidden layers of
256 units with the exact (erf) GELU -> 128 linear outputs (log-density samples
across the droplet interface).  Loss: mean squared error over batch and outputs.

Parameter vector layout (FP32 on the device, FP64 here), in this order:
  W1[256][4], b1[256], W2[256][256], b2[256], W3[256][256], b3[256], W4[128][256], b4[128]
(165,760 values).

`bf16=True` rounds every operand of a matrix product to bfloat16 (round to
nearest even) exactly where the GPU feeds its BF16 matrix cores: the weights,
the layer inputs (hidden activations and the input vector), the output
gradient and the pre-activation gradients.  Everything else stays FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = [4, 256, 256, 256, 128]
SHAPES = []
for _i in range(4):
    SHAPES.append(("W", (SIZES[_i + 1], SIZES[_i])))
    SHAPES.append(("b", (SIZES[_i + 1],)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(x):
    """Round to bfloat16 (RNE), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def unpack(theta):
    """Flat parameter vector -> list of (W, b) per layer."""
    out, off = [], 0
    for i in range(4):
        n_out, n_in = SIZES[i + 1], SIZES[i]
        W = theta[off: off + n_out * n_in].reshape(n_out, n_in)
        off += n_out * n_in
        b = theta[off: off + n_out]
        off += n_out
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(seed=0):
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(4):
        n_out, n_in = SIZES[i + 1], SIZES[i]
        parts.append(rng.standard_normal(n_out * n_in) * math.sqrt(2.0 / n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def forward(theta, X, bf16=False, base=None):
    """Returns (Y, cache), Y = network(X) + base.  X: [B][4] standardised inputs;
    base: [B][128] or None (a known profile the network corrects)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(np.asarray(theta, dtype=np.float64))
    H = r(X)
    cache = {"H": [H], "Z": []}
    for i, (W, b) in enumerate(layers):
        Z = H @ r(W).T + b
        cache["Z"].append(Z)
        if i < 3:
            H = r(gelu(Z))
            cache["H"].append(H)
        else:
            H = Z if base is None else Z + np.asarray(base, dtype=np.float64)
    return H, cache


def loss_and_grad(theta, X, T, bf16=False, base=None):
    """MSE loss of network(X) + base against T and its gradient with respect to the
    flat parameter vector (base does not depend on the parameters)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    theta = np.asarray(theta, dtype=np.float64)
    layers = unpack(theta)
    Y, cache = forward(theta, X, bf16, base)
    B, n_out = Y.shape
    diff = Y - T
    loss = float((diff ** 2).sum() / (B * n_out))
    dZ = r(2.0 * diff / (B * n_out))
    grads = [None] * 4
    for i in (3, 2, 1, 0):
        W, _ = layers[i]
        H_in = cache["H"][i]
        dW = dZ.T @ H_in
        db = dZ.sum(axis=0)
        grads[i] = (dW, db)
        if i > 0:
            dH = dZ @ r(W)
            dZ = r(dH * gelu_prime(cache["Z"][i - 1]))
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    return loss, flat


def adam_step(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
