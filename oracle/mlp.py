"""FP64 reference of the surrogate MLP (TEST INFRASTRUCTURE ONLY).

The search's learned pruning ranks candidate masks with a small MLP,
F -> 256 -> 256 -> 1 with GELU activations, that predicts
y = ln(e_loc + 1e-12) from per-mask features, trained by mean-squared error
with Adam.  This module is the plain FP64 NumPy version of the forward pass,
the gradient of the loss and one Adam step, written from their definitions;
the GPU kernels (BF16 operands, FP32 accumulation) are compared against it.

GELU is the exact (erf) form: gelu(x) = x * Phi(x), Phi the standard normal
CDF, so gelu'(x) = Phi(x) + x * phi(x).

Parity status: pinned by central finite differences of the loss
(tests/test_mlp_oracle.py).
"""
import math

import numpy as np

_erf = np.vectorize(math.erf)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def init_params(F, H=256, seed=0):
    """Weights in [out][in] layout: W1[H][F], W2[H][H], w3[H]; biases."""
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, math.sqrt(2.0 / F), (H, F)), b1=np.zeros(H),
                W2=rng.normal(0, math.sqrt(2.0 / H), (H, H)), b2=np.zeros(H),
                w3=rng.normal(0, math.sqrt(1.0 / H), H), b3=np.zeros(1))


def forward(p, X):
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = gelu(Z2)
    y = H2 @ p["w3"] + p["b3"][0]
    return y, (X, Z1, H1, Z2, H2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def grads(p, X, t):
    """Gradient of mean((y - t)^2) with respect to every parameter."""
    y, (X, Z1, H1, Z2, H2) = forward(p, X)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B
    g = {}
    g["w3"] = H2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dZ2 = np.outer(dy, p["w3"]) * gelu_grad(Z2)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * gelu_grad(Z1)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; step counts from 1."""
    for key in p:
        m[key] = beta1 * m[key] + (1 - beta1) * g[key]
        v[key] = beta2 * v[key] + (1 - beta2) * g[key] ** 2
        mh = m[key] / (1 - beta1 ** step)
        vh = v[key] / (1 - beta2 ** step)
        p[key] = p[key] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
