"""Pins for the FP64 reference of the mobility-correction network.

* bfloat16 rounding: round-to-nearest-even on the 16 dropped bits, checked on
  values whose rounding is fixed by that definition.
* Backpropagation against central finite differences (weights not rounded,
  so that the loss is smooth).
* One Adam step from zero moments moves every weight by lr * sign(grad)
  (up to eps), the closed form of the bias-corrected update at t = 1.
* Training on a smooth target reduces the loss.
"""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.NPARAM == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4545


@pytest.mark.parametrize("x,exp", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                           # tie -> even (mantissa 0)
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),           # tie -> even (mantissa 2)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above the tie -> up
    (-(1.0 + 2.0 ** -8 + 2.0 ** -20), -(1.0 + 2.0 ** -7)),
    (3.0e-3, 0.0030059814453125),
    (0.0, 0.0),
])
def test_bf16_round_to_nearest_even(x, exp):
    assert mlp.bf16_round(np.float32(x)) == exp


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init_params(1).astype(np.float64)
    theta += rng.normal(scale=0.05, size=theta.shape)
    X = rng.normal(size=(17, 4))
    y = rng.normal(size=17)
    loss, grad = mlp.loss_and_grad(theta, X, y, round_bf16=False)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 256, 320]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, y, False)[0] - mlp.loss_and_grad(tm, X, y, False)[0]) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-6, abs=1e-10)


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(1)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    assert np.allclose(theta - new, 1e-3 * np.sign(g), rtol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(256, 4))
    y = 0.02 * np.cos(np.pi * X[:, 0]) * np.cos(np.pi * X[:, 1]) + 0.01 * X[:, 3]
    theta = mlp.init_params(3).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, y)[0]
    for t in range(1, 301):
        loss, g = mlp.loss_and_grad(theta, X, y)
        theta, m, v = mlp.adam_step(theta, m, v, g, t, lr=3e-3)
    assert loss < 0.2 * l0
