"""Pins of the FP64 surrogate-network oracle: finite differences, bfloat16
rounding, GELU and Adam against their definitions."""
import math

import numpy as np
import pytest

import synth
from oracle import mlp


def _data(B=24, seed=3):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0.5, 0.95, B), rng.uniform(0.6, 1.5, B), rng.uniform(0, 0.2, B)])
    T = np.column_stack([np.log(rng.uniform(0.2, 0.4, B)), np.log(rng.uniform(0.005, 0.06, B))])
    return X, T


def test_layout_and_init():
    th = synth.mlp_init()
    assert th.dtype == np.float32 and th.size == mlp.NPARAMS == 4546 == synth.MLP_NPARAMS
    P = mlp.unpack(th)
    assert np.all(np.abs(P["W1"]) <= 1 / math.sqrt(3)) and np.all(np.abs(P["W2"]) <= 1 / 8)
    assert np.all(P["b1"] == 0) and np.all(P["b3"] == 0)
    assert np.array_equal(mlp.pack(P).astype(np.float32), th)


def test_gradient_matches_finite_differences():
    X, T = _data()
    norm = mlp.norm_from(X, T)
    th = synth.mlp_init().astype(np.float64)
    rng = np.random.default_rng(0)
    th = th + 0.05 * rng.standard_normal(th.size)     # away from zero biases
    _, g = mlp.loss_and_grad(th, X, T, norm, emulate_bf16=False)
    idx = rng.choice(th.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th); e[i] = h
        lp, _ = mlp.loss_and_grad(th + e, X, T, norm, emulate_bf16=False)
        lm, _ = mlp.loss_and_grad(th - e, X, T, norm, emulate_bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding():
    # exact cases of round-to-nearest-even at 8 significand bits
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.0e-5, 0.0])
    r = mlp.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == 1.0
    assert r[4] == -2.5 and r[6] == 0.0
    assert abs(r[5] / 3.0e-5 - 1) < 2 ** -8
    x = np.random.default_rng(1).standard_normal(1000)
    assert np.all(np.abs(mlp.bf16(x) - x) <= np.abs(x) * 2 ** -8)


def test_gelu_closed_form():
    z = np.linspace(-6, 6, 41)
    assert np.allclose(mlp.gelu(z), z * 0.5 * (1 + np.array([math.erf(v / math.sqrt(2)) for v in z])))
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    h = 1e-6
    assert np.allclose(mlp.gelu_prime(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)
    assert np.allclose(mlp.gelu(np.array([10.0])), 10.0) and abs(mlp.gelu(np.array([-10.0]))[0]) < 1e-20


def test_adam_first_step_is_signed_lr():
    # with m0 = v0 = 0 the bias-corrected first step is lr * g / (|g| + eps)
    th = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -1e-3])
    new, m, v = mlp.adam(th, np.zeros(5), np.zeros(5), g, 1, lr=0.01)
    assert np.allclose(new, -0.01 * g / (np.abs(g) + 1e-8))


def test_training_decreases_loss():
    X, T = _data(B=64, seed=5)
    norm = mlp.norm_from(X, T)
    th = synth.mlp_init().astype(np.float64)
    m = np.zeros_like(th); v = np.zeros_like(th)
    l0, _ = mlp.loss_and_grad(th, X, T, norm)
    for t in range(1, 201):
        l, g = mlp.loss_and_grad(th, X, T, norm)
        th, m, v = mlp.adam(th, m, v, g, t, lr=3e-3)
    assert l < 0.2 * l0


@pytest.mark.parametrize("t", [2, 3, 10])
def test_adam_bias_correction_beyond_the_first_step(t):
    # with a constant gradient g, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected step is lr * g / (|g| + eps) at every t.  A bias correction with
    # t - 1, or b1 and b2 swapped, or without the square root, fails at t >= 2.
    g = np.array([1.0, -2.0, 0.5, 1e-3, -1e-3])
    th = np.zeros(5)
    m = np.zeros(5)
    v = np.zeros(5)
    for k in range(1, t + 1):
        new, m, v = mlp.adam(th, m, v, g, k, lr=0.01)
        assert np.allclose(new - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        th = new
    assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-14)
    assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-14)
