"""FP64 reference of the surrogate MLP (6 -> 256 -> 256 -> 256 -> 256 -> 5, SiLU).

TEST INFRASTRUCTURE: the GPU surrogate kernels are checked against this.
The surrogate is not part of the paper; this module is pinned by finite
differences (backward against forward) and by torch.nn on the CPU (forward).

Precision model of the GPU path, reproduced here when bf16=True:
  layer 1 (6 inputs) in FP32 on the vector units: z1 = x W1 + b1
  layers 2..5 on BF16 matrix cores with FP32 accumulation: the activations
  and weights are rounded to BF16 (round to nearest even) before each
  product, products and sums are exact here (FP64) and only the final FP32
  rounding order differs from the GPU.
Backward uses the same rounding points: the incoming gradient of a BF16
product is rounded to BF16, weight gradients are accumulated in FP64 here.
"""
from __future__ import annotations

import numpy as np

SIZES = [6, 256, 256, 256, 256, 5]


def to_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed: int):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (for tests)."""
    rng = np.random.default_rng(seed)
    p = []
    for i in range(5):
        k = 1.0 / np.sqrt(SIZES[i])
        p.append(rng.uniform(-k, k, (SIZES[i], SIZES[i + 1])))
        p.append(rng.uniform(-k, k, SIZES[i + 1]))
    return p


def forward(params, x, bf16=False):
    """Returns (y, cache). x: (n, 6). params: [W1, b1, ..., W5, b5]."""
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    zs, acts = [], [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for i in range(5):
        W, b = params[2 * i], params[2 * i + 1]
        if i == 0:
            z = h @ W + b  # FP32 vector layer on the GPU
        else:
            z = r(h) @ r(W) + b
        zs.append(z)
        if i < 4:
            h = silu(z)
            acts.append(h)
        else:
            h = z
    return h, (zs, acts)


def loss_and_grads(params, x, t, w=None, bf16=False):
    """Mean over the batch of sum_o w_o (y_o - t_o)^2 and its gradients."""
    n = x.shape[0]
    w = np.ones(5) if w is None else np.asarray(w, dtype=np.float64)
    y, (zs, acts) = forward(params, x, bf16)
    d = y - t
    loss = float((w * d * d).sum() / n)
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * 10
    g = 2.0 * w * d / n  # dL/dz5
    for i in range(4, -1, -1):
        W = params[2 * i]
        a_in = acts[i]
        if i == 0:
            grads[0] = a_in.T @ g
        else:
            grads[2 * i] = r(a_in).T @ r(g)
        grads[2 * i + 1] = g.sum(axis=0)
        if i > 0:
            da = r(g) @ r(W).T
            g = da * silu_grad(zs[i - 1])
    return loss, grads
