"""Pins of the FP64 surrogate-MLP reference (forward, backward, Adam)."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_parameter_count():
    assert mlp.n_params() == 34819


def test_bf16_rounding_matches_torch_converter():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-5, 5, 20000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -1 - 2 ** -8, 0.0, 65504.0, 1e-30]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1 + 2 ** -8]))[0] == 1.0            # tie -> even
    assert mlp.bf16(np.array([1 + 3 * 2 ** -9]))[0] == 1 + 2 ** -7


def test_dsilu_is_the_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = mlp.init_params(3).astype(np.float64) * 0.5
    theta += rng.standard_normal(theta.size) * 0.01     # non-zero biases
    X = rng.standard_normal((7, 10))
    Y = rng.standard_normal((7, 3))
    L, g = mlp.loss_and_grad(theta, X, Y, quant=False)
    idx = np.concatenate([rng.choice(theta.size, 60, replace=False), [0, 1280 + 3, theta.size - 1, theta.size - 4]])
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (mlp.loss_and_grad(theta + e, X, Y, False)[0] - mlp.loss_and_grad(theta - e, X, Y, False)[0]) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_forward_special_cases():
    theta = np.zeros(mlp.n_params())
    theta[-3:] = [0.5, -1.0, 2.0]                       # only the output bias
    Y, _ = mlp.forward(theta, np.ones((4, 10)))
    np.testing.assert_array_equal(Y, np.tile([0.5, -1.0, 2.0], (4, 1)))
    # quantised forward equals the unquantised network evaluated on BF16-exact data
    rng = np.random.default_rng(2)
    th = mlp.bf16(mlp.init_params(5))
    X = mlp.bf16(rng.standard_normal((5, 10)))
    Yq, cq = mlp.forward(th, X, quant=True)
    assert np.all(mlp.bf16(cq[1][0]) == cq[1][0])       # layer inputs are BF16 values


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = mlp.adam(th, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2, update = lr g / (|g| + eps)
    np.testing.assert_allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)
