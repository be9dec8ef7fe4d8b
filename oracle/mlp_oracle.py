"""FP64 reference of the sub-step surrogate network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: the plain, slow reference that the GPU network
kernels are checked against.  Only the tests, the smoke check and the
benchmark's CPU baseline may import it; the product path never does.  It
shares no code with the GPU library.

The network is a per-solid-particle multilayer perceptron with SiLU hidden
activations, z -> z sigmoid(z), and a linear output layer:
    h_0 = x,  h_k = SiLU(h_{k-1} W_k + b_k)  (k < L),  y = h_{L-1} W_L + b_L,
trained on the mean squared error 0.5 mean_rows sum_cols (y - t)^2 with Adam.
The paper has no learned component; this follows the definitions of the
multilayer perceptron, SiLU and Adam (Kingma & Ba, 2015) written out.

Precision switch: with ``bf16=True`` the operands of every matrix product
(the layer input and the weights) are rounded to bfloat16 before an exact
FP64 product, which is the arithmetic the GPU's BF16 matrix cores perform
with FP32 accumulation, so both sides round at the same points.
"""
import numpy as np


def round_bf16(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64.

    bfloat16 keeps the top 16 bits of an IEEE binary32: round to binary32
    first, then to 8 significant bits by adding half of the dropped range
    plus the parity of the kept bit and truncating."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    keep = (u >> 16) & 1
    u = (u + 0x7FFF + keep) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    """d/dz [z sigmoid(z)] = sigmoid(z) (1 + z (1 - sigmoid(z)))."""
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, seed=0):
    """Layer weights W_k (fan_in x fan_out) and biases b_k, uniform in
    +-sqrt(6 / (fan_in + fan_out)) (Glorot), biases zero; from a seeded
    numpy generator (inputs of both sides, not method arithmetic)."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        params.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
    return params


def forward(params, x, bf16=False):
    """Returns the output and the cache (layer inputs and pre-activations)."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    L = len(params)
    for k, (W, b) in enumerate(params):
        hin = round_bf16(h) if bf16 else h
        Wq = round_bf16(W) if bf16 else W
        z = hin @ Wq + b
        cache.append((hin, z))
        h = silu(z) if k < L - 1 else z
    return h, cache


def loss(params, x, t, bf16=False):
    y, _ = forward(params, x, bf16)
    return 0.5 * np.mean(np.sum((y - t) ** 2, axis=1))


def backward(params, x, t, bf16=False):
    """Gradients of ``loss`` with respect to every W_k and b_k (chain rule,
    layer by layer from the output)."""
    y, cache = forward(params, x, bf16)
    n = y.shape[0]
    delta = (y - t) / n  # d loss / d y
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        hin, z = cache[k]
        if k < len(params) - 1:
            delta = delta * silu_grad(z)
        W = params[k][0]
        Wq = round_bf16(W) if bf16 else W
        dq = round_bf16(delta) if bf16 else delta
        grads[k] = (hin.T @ dq, delta.sum(axis=0))
        delta = dq @ Wq.T
    return grads


def adam(params, grads, state, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected first and second moments)."""
    if state is None:
        state = [(np.zeros_like(W), np.zeros_like(b), np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    new_p, new_s = [], []
    c1, c2 = 1.0 - b1 ** step, 1.0 - b2 ** step
    for (W, b), (gW, gb), (mW, mb, vW, vb) in zip(params, grads, state):
        mW = b1 * mW + (1 - b1) * gW
        mb = b1 * mb + (1 - b1) * gb
        vW = b2 * vW + (1 - b2) * gW * gW
        vb = b2 * vb + (1 - b2) * gb * gb
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        new_p.append((W, b))
        new_s.append((mW, mb, vW, vb))
    return new_p, new_s
