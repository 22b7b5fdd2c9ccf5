"""Pins of the FP64 surrogate-MLP reference: its analytic gradient against
central finite differences of the loss, GELU against its defining integral
form, and one Adam step against the update written out by hand."""
import math

import numpy as np

from oracle import mlp


def test_gelu_matches_definition():
    x = np.linspace(-5, 5, 41)
    # x * Phi(x), Phi via the complementary error function
    want = x * 0.5 * np.array([math.erfc(-v / math.sqrt(2)) for v in x])
    np.testing.assert_allclose(mlp.gelu(x), want, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    F, H, B = 5, 8, 7
    p = mlp.init_params(F, H, seed=3)
    for k in p:
        p[k] = p[k] + 0.1 * rng.normal(size=p[k].shape)
    X = rng.normal(size=(B, F))
    t = rng.normal(size=B)
    g = mlp.grads(p, X, t)
    h = 1e-6
    for key in p:
        flat = p[key].reshape(-1)
        for idx in range(min(flat.size, 12)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(p, X, t)
            flat[idx] = old - h
            lm = mlp.loss(p, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[key].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (key, idx)


def test_adam_step_by_hand():
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.5, 0.25])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    mlp.adam_step(p, g, m, v, step=1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * sign(g) (up to eps)
    np.testing.assert_allclose(p["w"], [1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 - 0.1 * 0.25 / (0.25 + 1e-8)],
                               rtol=1e-15)
