"""Pins of the FP64 surrogate-network reference (oracle/mlp.py), CPU only.

Each pin comes from outside the reference itself: torch's own bfloat16
conversion, central finite differences of the loss, the closed form of the
first Adam step, and the layer sizes of the network.
"""

import numpy as np
import pytest
import torch

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 4 * 128 + 128 + 128 * 128 + 128 + 2 * 128 + 2 == 17410


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125, 3.0e38, 1e-40, -2.5]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(mlp.bf16(x), ref)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    flat = mlp.init_params(3).astype(np.float64)
    x = rng.standard_normal((16, 4))
    t = rng.uniform(0.0, 1.0, (16, 2))
    _, g = mlp.loss_and_grad(flat, x, t, mixed=False)
    idx = np.concatenate([rng.choice(512, 40, replace=False),                  # W1
                          512 + rng.choice(128, 10, replace=False),            # b1
                          640 + rng.choice(16384, 80, replace=False),          # W2
                          17024 + rng.choice(128, 10, replace=False),          # b2
                          17152 + rng.choice(258, 30, replace=False)])         # W3, b3
    h = 1e-6
    for k in idx:
        e = np.zeros_like(flat)
        e[k] = h
        fd = (mlp.loss(flat + e, x, t, mixed=False) - mlp.loss(flat - e, x, t, mixed=False)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_mixed_precision_gradient_is_close_to_exact():
    rng = np.random.default_rng(4)
    flat = mlp.init_params(5).astype(np.float64)
    x = rng.standard_normal((64, 4))
    t = rng.uniform(0.0, 1.0, (64, 2))
    _, g_exact = mlp.loss_and_grad(flat, x, t, mixed=False)
    _, g_mixed = mlp.loss_and_grad(flat, x, t, mixed=True)
    # bf16 keeps 8 significant bits: the gradient moves by ~1 % of its scale
    assert np.max(np.abs(g_mixed - g_exact)) < 0.05 * np.max(np.abs(g_exact))


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(6)
    w = rng.standard_normal(100)
    g = rng.standard_normal(100)
    lr, eps = 1e-3, 1e-8
    w1, m, v = mlp.adam_step(w, g, np.zeros(100), np.zeros(100), 1, lr, eps=eps)
    assert np.allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_outputs_are_probabilities_and_silu_limits():
    flat = mlp.init_params(7)
    y, _ = mlp.forward(flat, np.random.default_rng(8).standard_normal((50, 4)) * 5)
    assert np.all((y > 0) & (y < 1))
    z = np.array([-50.0, 0.0, 50.0])
    assert np.allclose(mlp.silu(z), [0.0, 0.0, 50.0], atol=1e-18)
    assert np.allclose(mlp.dsilu(z), [0.0, 0.5, 1.0], atol=1e-18)


@pytest.mark.parametrize("seed", [1, 2])
def test_loss_decreases_under_adam(seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (256, 4))
    t = np.stack([1 / (1 + np.exp(-3 * x[:, 0])), 0.5 + 0.4 * np.tanh(x[:, 1] - x[:, 2])], axis=1)
    flat = mlp.init_params(seed).astype(np.float64)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    l0 = mlp.loss(flat, x, t)
    for k in range(1, 61):
        _, g = mlp.loss_and_grad(flat, x, t)
        flat, m, v = mlp.adam_step(flat, g, m, v, k, 3e-3)
    assert mlp.loss(flat, x, t) < 0.5 * l0
