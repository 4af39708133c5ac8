"""FP64 reference of the surrogate MLP (test infrastructure; not in the paper).

Network: x (7) -> Linear(7,256) -> GELU -> Linear(256,256) -> GELU ->
Linear(256,1), GELU in its erf form gelu(z) = z * Phi(z).  Loss is the mean
squared error over the batch, L = (1/B) sum (yhat - y)^2.  The optimiser is
Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.

The GPU keeps FP32 master weights and multiplies with BF16 copies of the
weights and of the hidden activations.  ``quantize=True`` makes this oracle
take the same BF16 roundings of weights and layer inputs (round to nearest
even from FP32), while every product and sum stays FP64.

Weights are lists [(W0, b0), (W1, b1), (W2, b2)], W of shape (fan_in, fan_out).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * _SQRT1_2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z * _SQRT1_2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(params, x, quantize=False):
    """Returns (yhat, cache) for input x (B, 7)."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    (W0, b0), (W1, b1), (W2, b2) = params
    x = np.asarray(x, dtype=np.float64)
    a0 = q(x)
    z1 = a0 @ q(W0) + b0
    h1 = gelu(z1)
    a1 = q(h1)
    z2 = a1 @ q(W1) + b1
    h2 = gelu(z2)
    a2 = q(h2)
    y = (a2 @ q(W2) + b2).reshape(-1)
    return y, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2)


def loss_and_grads(params, x, y, quantize=False):
    """MSE loss and gradients w.r.t. every weight and bias (chain rule)."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    (W0, b0), (W1, b1), (W2, b2) = params
    yhat, c = forward(params, x, quantize)
    B = yhat.size
    diff = yhat - np.asarray(y, dtype=np.float64).reshape(-1)
    loss = float((diff * diff).mean())
    g3 = (2.0 / B) * diff.reshape(-1, 1)              # dL/dy, (B, 1)
    gW2 = c["a2"].T @ g3
    gb2 = g3.sum(axis=0)
    dh2 = g3 @ q(W2).T                                  # (B, 256)
    dz2 = dh2 * gelu_grad(c["z2"])
    gW1 = c["a1"].T @ dz2
    gb1 = dz2.sum(axis=0)
    dh1 = dz2 @ q(W1).T
    dz1 = dh1 * gelu_grad(c["z1"])
    gW0 = c["a0"].T @ dz1
    gb0 = dz1.sum(axis=0)
    return loss, [(gW0, gb0), (gW1, gb1), (gW2, gb2)]


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    newp, newm, newv = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for P, G, Mm, Vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            Mn = beta1 * Mm + (1 - beta1) * G
            Vn = beta2 * Vv + (1 - beta2) * G * G
            mh = Mn / (1 - beta1 ** t)
            vh = Vn / (1 - beta2 ** t)
            out.append((P - lr * mh / (np.sqrt(vh) + eps), Mn, Vn))
        newp.append((out[0][0], out[1][0]))
        newm.append((out[0][1], out[1][1]))
        newv.append((out[0][2], out[1][2]))
    return newp, newm, newv


def zeros_like(params):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
