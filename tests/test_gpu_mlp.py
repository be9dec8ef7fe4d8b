"""Parity of the surrogate network's HIP kernels (through the C-ABI) with the
FP64 network oracle.

Like-for-like: the oracle rounds every matrix-product operand to bfloat16 at
the same points as the matrix cores, so the remaining difference is FP32
accumulation and FP32 SiLU (bar: relative L2 <= 1e-3 for outputs, 5e-3 for
gradients).  Against the unrounded FP64 network the BF16 path stays within
relative L2 2e-2 and cosine >= 0.999.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1911_13255_amd import mlp

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_case(rows, in_dim=24, out_dim=4, seed=0):
    params = M.init_params([in_dim, 128, 128, 128, out_dim], seed=seed)
    rng = np.random.default_rng(seed + 100)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    x = rng.standard_normal((rows, in_dim))
    t = rng.standard_normal((rows, out_dim))
    return params, x, t


def to_dev(a):
    import torch

    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def fp32_params(params):
    return [(np.float32(W).astype(np.float64), np.float32(b).astype(np.float64)) for W, b in params]


@pytest.mark.parametrize("rows", [1, 63, 64, 1000, 4099])
def test_forward_matches_oracle(gpu, rows):
    params, x, _ = make_case(rows)
    net = mlp.Network(24, 4, max(rows, 64))
    net.set_params(params)
    y = net.forward(to_dev(x)).cpu().numpy().astype(np.float64)
    p32 = fp32_params(params)
    x32 = np.float32(x).astype(np.float64)
    ref, _ = M.forward(p32, x32, bf16=True)
    exact, _ = M.forward(p32, x32, bf16=False)
    assert rel_l2(y, ref) <= 1e-3, rel_l2(y, ref)
    assert rel_l2(y, exact) <= 2e-2
    cos = float(np.sum(y * exact) / (np.linalg.norm(y) * np.linalg.norm(exact)))
    assert cos >= 0.999
    net.close()


@pytest.mark.parametrize("rows", [100, 1031])
def test_gradients_and_loss_match_oracle(gpu, rows):
    params, x, t = make_case(rows, seed=3)
    net = mlp.Network(24, 4, rows)
    net.set_params(params)
    loss = net.backward(to_dev(x), to_dev(t))
    g = net.grads()
    p32 = fp32_params(params)
    x32, t32 = np.float32(x).astype(np.float64), np.float32(t).astype(np.float64)
    ref = M.backward(p32, x32, t32, bf16=True)
    ref_loss = M.loss(p32, x32, t32, bf16=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    for k in range(4):
        assert rel_l2(g[k][0], ref[k][0]) <= 5e-3, (k, rel_l2(g[k][0], ref[k][0]))
        assert rel_l2(g[k][1], ref[k][1]) <= 5e-3, (k, rel_l2(g[k][1], ref[k][1]))
    net.close()


def test_adam_step_matches_oracle(gpu):
    params, x, t = make_case(200, seed=5)
    net = mlp.Network(24, 4, 256)
    net.set_params(params)
    net.backward(to_dev(x), to_dev(t))
    g = [(gw.astype(np.float64), gb.astype(np.float64)) for gw, gb in net.grads()]
    net.adam(lr=1e-3)
    new = net.get_params()
    ref, _ = M.adam(fp32_params(params), g, None, step=1, lr=1e-3)
    for k in range(4):
        assert np.abs(new[k][0] - ref[k][0]).max() <= 1e-6
        assert np.abs(new[k][1] - ref[k][1]).max() <= 1e-6
    net.close()


def test_parameters_round_trip(gpu):
    params, _, _ = make_case(8, seed=7)
    net = mlp.Network(24, 4, 64)
    net.set_params(params)
    back = net.get_params()
    for (W, b), (W2, b2) in zip(params, back):
        assert np.array_equal(np.float32(W), W2) and np.array_equal(np.float32(b), b2)
    net.close()


def test_training_on_the_gpu_reduces_the_loss(gpu):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((4096, 24))
    t = np.stack([np.sin(x[:, 0]) + x[:, 1] * x[:, 2], x[:, 3] - 0.5 * x[:, 4] ** 2,
                  np.tanh(x[:, 5] + x[:, 6]), x[:, 7] * x[:, 8]], axis=1)
    net = mlp.Network(24, 4, 4096)
    net.set_params(M.init_params([24, 128, 128, 128, 4], seed=1))
    xd, td = to_dev(x), to_dev(t)
    l0 = net.backward(xd, td)
    for _ in range(300):
        net.train_step(xd, td, lr=2e-3)
    l1 = net.backward(xd, td)
    assert l1 < 0.1 * l0, (l0, l1)
    net.close()
