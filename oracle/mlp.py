"""FP64 reference of the sigma-surrogate network (TEST INFRASTRUCTURE ONLY).

A 3-64-64-2 multilayer perceptron with exact (erf) GELU, mapping the
standardised inputs (T/Tc, tau, sigma) to the standardised outputs
(log rho_l, log rho_g).  Every matrix product optionally rounds both operands
to bfloat16 (round to nearest even, via float32) before multiplying, and
accumulates in FP64; biases, activations, the loss and Adam stay in FP64.

Loss: L = sum over rows and outputs of (y - t)^2 / (2 B), on standardised
outputs.  Parameter layout (one vector): W1 (64x3, row = output unit), b1,
W2 (64x64), b2, W3 (2x64), b3 -- 4546 numbers.
"""
from __future__ import annotations

import math

import numpy as np

SHAPES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
          ("W3", (2, 64)), ("b3", (2,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)

_erf = np.vectorize(math.erf)


def unpack(theta):
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest even), going through float32 first."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, norm, emulate_bf16=True):
    """Standardised outputs y (B x 2) and the intermediate values."""
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(theta)
    x = (np.asarray(X, dtype=np.float64) - norm["in_mean"]) / norm["in_std"]
    z1 = q(x) @ q(P["W1"]).T + P["b1"]
    h1 = gelu(z1)
    z2 = q(h1) @ q(P["W2"]).T + P["b2"]
    h2 = gelu(z2)
    y = q(h2) @ q(P["W3"]).T + P["b3"]
    return y, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2)


def predict(theta, X, norm, emulate_bf16=True):
    """Outputs in the original units (log rho_l, log rho_g)."""
    y, _ = forward(theta, X, norm, emulate_bf16)
    return y * norm["out_std"] + norm["out_mean"]


def loss_and_grad(theta, X, T, norm, emulate_bf16=True):
    """Loss and its gradient (same layout as theta) for raw targets T (log rho)."""
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(theta)
    B = X.shape[0]
    y, c = forward(theta, X, norm, emulate_bf16)
    t = (np.asarray(T, dtype=np.float64) - norm["out_mean"]) / norm["out_std"]
    d = y - t
    loss = float((d * d).sum() / (2.0 * B))
    dy = d / B
    g = {}
    g["W3"] = q(dy).T @ q(c["h2"])
    g["b3"] = dy.sum(0)
    dz2 = (q(dy) @ q(P["W3"])) * gelu_prime(c["z2"])
    g["W2"] = q(dz2).T @ q(c["h1"])
    g["b2"] = dz2.sum(0)
    dz1 = (q(dz2) @ q(P["W2"])) * gelu_prime(c["z1"])
    g["W1"] = q(dz1).T @ q(c["x"])
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015); t is the 1-based step count."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def norm_from(X, T):
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    return dict(in_mean=X.mean(0), in_std=X.std(0) + 1e-12, out_mean=T.mean(0), out_std=T.std(0) + 1e-12)
