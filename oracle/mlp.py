"""FP64 reference of the warm-start MLP -- TEST INFRASTRUCTURE ONLY.

Network: h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), out = W3 h2 + b3,
GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2; loss = weighted mean of
squared errors on standardized targets; gradients by back-propagation.

With ``emulate=True`` every GEMM operand (standardized input, weights,
activations, back-propagated output / pre-activation gradients) is rounded
to BF16 (through FP32, round to nearest even) exactly where the GPU kernels
round; everything else is FP64.  ``emulate=False`` is the plain FP64
network (used to pin the backward pass by finite differences).
Parameter layout: W1 (h1 x n_in, row-major), b1, W2 (h2 x h1), b2, W3, b3.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def bf16(x) -> np.ndarray:
    """float64 -> float32 (RNE) -> bfloat16 (RNE) -> float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def num_params(dims) -> int:
    n_in, h1, h2, n_out = dims
    return h1 * n_in + h1 + h2 * h1 + h2 + n_out * h2 + n_out


def unpack(p, dims):
    n_in, h1, h2, n_out = dims
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for rows, cols in ((h1, n_in), (h2, h1), (n_out, h2)):
        W = p[o:o + rows * cols].reshape(rows, cols); o += rows * cols
        b = p[o:o + rows]; o += rows
        out += [W, b]
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def _scale(v, mean, std):
    if mean is None:
        return v
    inv = np.where(std > 1e-12, 1.0 / np.maximum(std, 1e-300), 0.0)
    return (v - mean) * inv


def forward(p, X, dims, emulate=True, in_mean=None, in_std=None):
    """Network output in standardized units and the cache of the backward pass."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, dims)
    Xs = r(_scale(np.asarray(X, dtype=np.float64), in_mean, in_std))
    W1r, W2r, W3r = r(W1), r(W2), r(W3)
    Z1 = Xs @ W1r.T + b1
    A1 = r(gelu(Z1))
    Z2 = A1 @ W2r.T + b2
    A2 = r(gelu(Z2))
    Y = A2 @ W3r.T + b3
    return Y, dict(Xs=Xs, W1r=W1r, W2r=W2r, W3r=W3r, Z1=Z1, A1=A1, Z2=Z2, A2=A2)


def loss_grad(p, X, T, dims, w=None, emulate=True, in_mean=None, in_std=None, out_mean=None, out_std=None):
    """(loss, gradient) of sum_j w_j (Y - T_std)^2 / (B n_out)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    Y, c = forward(p, X, dims, emulate, in_mean, in_std)
    Ts = _scale(np.asarray(T, dtype=np.float64), out_mean, out_std)
    B, N = Y.shape
    wv = np.ones(N) if w is None else np.asarray(w, dtype=np.float64)
    R = Y - Ts
    loss = float(np.sum(wv * R * R) / (B * N))
    dY = 2.0 * wv * R / (B * N)
    dYr = r(dY)
    dW3 = dYr.T @ c["A2"]
    db3 = dY.sum(axis=0)
    dA2 = dYr @ c["W3r"]
    dZ2 = dA2 * gelu_d(c["Z2"])
    dZ2r = r(dZ2)
    dW2 = dZ2r.T @ c["A1"]
    db2 = dZ2.sum(axis=0)
    dA1 = dZ2r @ c["W2r"]
    dZ1 = dA1 * gelu_d(c["Z1"])
    dZ1r = r(dZ1)
    dW1 = dZ1r.T @ c["Xs"]
    db1 = dZ1.sum(axis=0)
    return loss, pack([dW1, db1, dW2, db2, dW3, db3])
