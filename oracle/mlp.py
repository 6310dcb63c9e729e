"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE.

A 2 -> 64 -> 64 -> 1 perceptron with SiLU activations, silu(z) = z / (1 + e^-z),
trained with the mean squared error.  Parameters are one flat vector in the
order W1 [64, 2], b1 [64], W2 [64, 64] (out, in), b2 [64], w3 [64], b3 [1]
(4417 numbers).  Plain numpy forward and backward (chain rule written out);
the tests pin the backward to the forward by finite differences.

bf16=True rounds the operands of the BF16 matrix products to bfloat16 and
keeps everything else in FP64: in the forward pass W2 is rounded and each
layer-1 activation h enters layer 2 as hi + lo with hi = bf16(h),
lo = bf16(h - hi) (about 16 significant bits); in the backward pass the
operands of W2^T dz2 and of the weight gradients (dz2, dz1, hi, h2, the
inputs, dy) are rounded.  This is the arithmetic of a BF16-weight network
with wide accumulation; the gradient is then the one of the rounded forward
with rounding treated as the identity.
"""
from __future__ import annotations

import numpy as np

H = 64
N_PARAMS = H * 2 + H + H * H + H + H + 1


def unpack(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + 2 * H].reshape(H, 2); o += 2 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, np.atleast_1d(b3)]).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, X, bf16=False):
    """X [n, 2] -> y [n] and the intermediate values."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    z1 = X @ W1.T + b1
    h1 = silu(z1)
    if bf16:
        hi = bf16_round(h1)
        W2 = bf16_round(W2)
        z2 = (hi + bf16_round(h1 - hi)) @ W2.T + b2
        h1 = hi
    else:
        z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss_grad(p, X, t, bf16=False):
    """Mean squared error over the batch and its gradient (flat, same order as p)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X, bf16)
    rd = bf16_round if bf16 else (lambda a: a)  # noqa: E731
    n = X.shape[0]
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / n                      # dL/dy
    g_w3 = rd(h2).T @ rd(dy)
    g_b3 = dy.sum()
    dz2 = (dy[:, None] * w3[None, :]) * dsilu(z2)
    g_W2 = rd(dz2).T @ h1                 # h1 is its leading bfloat16 part when bf16
    g_b2 = rd(dz2).sum(axis=0)
    dz1 = (rd(dz2) @ rd(W2)) * dsilu(z1)
    g_W1 = rd(dz1).T @ rd(X)
    g_b1 = rd(dz1).sum(axis=0)
    return L, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32).copy()
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(chi, r=None, logit_r=None):
    """Network inputs: ln(chi)/ln(100) and logit(r)/10."""
    chi = np.asarray(chi, dtype=np.float64)
    if logit_r is None:
        r = np.asarray(r, dtype=np.float64)
        logit_r = np.log(r) - np.log1p(-r)
    return np.stack([np.log(chi) / np.log(100.0), np.asarray(logit_r) / 10.0], axis=1)
