"""Pins of the FP64 surrogate-network oracle: bfloat16 rounding against a
library conversion and hand values, SiLU and its derivative in closed form,
gradients against central finite differences, and Adam's first step."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def test_bf16_rounding_matches_library_conversion():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 65504.0, 1e-40]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(x), ref)
    # ties go to the even significand: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_silu_closed_forms():
    z = np.array([-3.0, -0.5, 0.0, 0.5, 3.0])
    s = 1.0 / (1.0 + np.exp(-z))
    assert np.allclose(M.silu(z), z * s, rtol=1e-15, atol=0)
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert M.silu_grad(np.array([0.0]))[0] == 0.5
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.allclose(M.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("bf16", [False])
def test_gradients_match_finite_differences(bf16):
    sizes = [6, 9, 7, 3]
    params = M.init_params(sizes, seed=4)
    params = [(W, np.random.default_rng(5 + k).standard_normal(b.shape) * 0.1) for k, (W, b) in enumerate(params)]
    rng = np.random.default_rng(6)
    x = rng.standard_normal((11, sizes[0]))
    t = rng.standard_normal((11, sizes[-1]))
    grads = M.backward(params, x, t)
    h = 1e-6
    for k, (W, b) in enumerate(params):
        for arr, g in ((W, grads[k][0]), (b, grads[k][1])):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + h
                lp = M.loss(params, x, t)
                flat[idx] = old - h
                lm = M.loss(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(g.reshape(-1)[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_forward_of_a_linear_network_is_a_matrix_product():
    # one layer: no activation, y = x W + b exactly
    rng = np.random.default_rng(1)
    W, b = rng.standard_normal((4, 3)), rng.standard_normal(3)
    x = rng.standard_normal((5, 4))
    y, _ = M.forward([(W, b)], x)
    assert np.allclose(y, x @ W + b, rtol=1e-15, atol=1e-15)


def test_adam_first_step_moves_each_weight_by_lr_times_sign():
    # at step 1 the bias-corrected update is lr * g / (|g| + eps) ~= lr sign(g)
    params = [(np.array([[1.0, -2.0]]), np.array([0.5, 0.0]))]
    grads = [(np.array([[3.0, -1e-3]]), np.array([-2.0, 0.0]))]
    new, state = M.adam(params, grads, None, step=1, lr=0.1)
    assert np.allclose(new[0][0], [[0.9, -1.9]], atol=1e-6)
    assert np.allclose(new[0][1], [0.6, 0.0], atol=1e-6)
    assert np.allclose(state[0][0], [[0.3, -1e-4]])


def test_training_reduces_the_loss():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((256, 5))
    t = np.stack([np.sin(x[:, 0]) + x[:, 1] * x[:, 2], x[:, 3] - x[:, 4] ** 2], axis=1)
    params = M.init_params([5, 32, 32, 2], seed=2)
    state = None
    l0 = M.loss(params, x, t)
    for step in range(1, 301):
        params, state = M.adam(params, M.backward(params, x, t), state, step, lr=3e-3)
    assert M.loss(params, x, t) < 0.25 * l0
