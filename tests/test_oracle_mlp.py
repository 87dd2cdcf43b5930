"""Pins of the FP64 surrogate-network oracle: central finite differences for every gradient,
GELU against its exact (erf) form and its own derivative, bfloat16 rounding against known
encodings, and properties of Adam (first step of size lr along -sign(g); convergence on a
convex quadratic)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1.0; just above -> 1 + 2^-7
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp.bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie, rounds to the even neighbour
    assert mlp.bf16(-3.0) == -3.0 and mlp.bf16(0.1) == pytest.approx(0.1, rel=2 ** -8)


def test_gelu_against_exact_form_and_derivative():
    z = np.linspace(-6, 6, 2001)
    exact = 0.5 * z * (1 + erf(z / math.sqrt(2)))
    assert np.abs(mlp.gelu(z) - exact).max() < 1e-3  # tanh approximation error bound
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=0, atol=1e-8)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    x = rng.normal(size=(5, 6))
    t = rng.normal(size=(5, 6))
    y, cache = mlp.forward(p, x)
    L, dy = mlp.loss_and_grad_y(y, t)
    g = mlp.flatten(mlp.backward(p, cache, dy))
    v = mlp.flatten(p)
    idx = np.concatenate([rng.choice(len(v), 60, replace=False),
                          [0, 1535, 1536, 1791, len(v) - 7, len(v) - 1]])  # W1, b1, W5, b5 edges
    h = 1e-5
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        Lp = mlp.loss_and_grad_y(mlp.forward(mlp.unflatten(vp), x)[0], t)[0]
        Lm = mlp.loss_and_grad_y(mlp.forward(mlp.unflatten(vm), x)[0], t)[0]
        fd = (Lp - Lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10), i


def test_parameter_count():
    assert len(mlp.flatten(mlp.init_params())) == 200710


def test_adam_first_step_and_convergence():
    v = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.01, 1e-3])
    v1, m, s = mlp.adam_step(v, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(v1 - v, -0.01 * np.sign(g), rtol=1e-4)
    # convex quadratic 0.5 |v - c|^2: Adam reaches the minimum
    c = np.array([0.3, -0.7, 2.0])
    v, m, s = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        v, m, s = mlp.adam_step(v, v - c, m, s, t, lr=0.01)
    np.testing.assert_allclose(v, c, atol=1e-3)
