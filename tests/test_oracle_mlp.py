"""Pins of the FP64 MLP oracle (learned warm start): identities of GELU and
softplus, bfloat16 rounding on representable neighbours, the analytic
gradient against central finite differences, the first Adam step in closed
form, and that plain training lowers the loss."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_gelu_and_softplus_identities():
    t = np.linspace(-6, 6, 241)
    # x Phi(x) with Phi(x) + Phi(-x) = 1  =>  GELU(x) - GELU(-x) = x
    np.testing.assert_allclose(M.gelu(t) - M.gelu(-t), t, atol=1e-14)
    assert M.gelu(0.0) == 0.0
    assert abs(M.gelu_prime(0.0) - 0.5) < 1e-15
    assert abs(M.gelu(40.0) - 40.0) < 1e-12 and abs(M.gelu(-40.0)) < 1e-12
    # derivative against central differences
    h = 1e-6
    np.testing.assert_allclose(M.gelu_prime(t), (M.gelu(t + h) - M.gelu(t - h)) / (2 * h), atol=1e-8)
    z = np.linspace(-30, 30, 61)
    np.testing.assert_allclose(M.softplus(z) - M.softplus(-z), z, atol=1e-12)
    np.testing.assert_allclose(M.sigmoid(z), np.exp(-np.logaddexp(0, -z)), atol=1e-15)


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7
    assert M.bf16(one) == one
    assert M.bf16(one + ulp / 2) == one                     # tie -> even
    assert M.bf16(one + 3 * ulp / 2) == one + 2 * ulp       # tie -> even (up)
    assert M.bf16(one + 0.75 * ulp) == one + ulp
    assert M.bf16(math.pi) == 3.140625
    assert M.bf16(-2.0) == -2.0


def _batch(seed, B=40):
    rng = np.random.default_rng(seed)
    flat = M.init_params(seed)
    flat = flat + 0.05 * rng.normal(size=flat.size)  # nonzero biases
    X = rng.normal(size=(B, M.F))
    y = np.abs(rng.normal(size=B))
    return flat, X, y


def test_gradient_matches_finite_differences():
    flat, X, y = _batch(0)
    g = M.grad(flat, X, y)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.arange(0, 1024), 30, replace=False),     # W1
                          rng.choice(np.arange(1024, 1152), 10, replace=False),  # b1
                          rng.choice(np.arange(1152, 17536), 40, replace=False),  # W2
                          rng.choice(np.arange(17536, 17664), 10, replace=False),  # b2
                          rng.choice(np.arange(17664, 17792), 10, replace=False),  # w3
                          [17792]])                                                # b3
    h = 1e-6
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = h
        fd = (M.loss(flat + e, X, y) - M.loss(flat - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-10, (k, fd, g[k])
    assert M.NPARAM == 17793 and g.size == 17793


def test_emulated_gradient_is_close_to_exact():
    flat, X, y = _batch(2)
    g0 = M.grad(flat, X, y)
    g1 = M.grad(flat, X, y, emulate=True)
    assert np.linalg.norm(g1 - g0) < 3e-2 * np.linalg.norm(g0)


def test_first_adam_step_closed_form():
    flat = np.zeros(5)
    g = np.array([0.3, -2.0, 1e-3, -1e-5, 7.0])
    new, m, v = M.adam(flat, g, np.zeros(5), np.zeros(5), 1, 0.01)
    # bias-corrected moments are g and g^2 on the first step: update = -lr g/(|g| + eps)
    np.testing.assert_allclose(new, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_lowers_loss():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(256, M.F))
    y = np.log1p(np.exp(0.5 * X[:, 0] - 0.3 * X[:, 2]))  # a smooth positive target
    flat = M.init_params(4)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    l0 = M.loss(flat, X, y)
    for t in range(1, 151):
        flat, m, v = M.adam(flat, M.grad(flat, X, y), m, v, t, 3e-3)
    assert M.loss(flat, X, y) < 0.2 * l0
