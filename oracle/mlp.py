"""FP64 reference of the surrogate MLP (6 -> 256 -> 256 -> 256 -> 256 -> 5, SiLU).

TEST INFRASTRUCTURE: the GPU surrogate kernels are checked against this.
The surrogate is not part of the paper; this module is pinned by finite
differences (backward against forward), by torch.nn on the CPU (forward)
and by torch.optim.AdamW on the CPU (the optimizer step).

Precision model of the GPU path, reproduced here when bf16=True:
  layers 1 (6 -> 256) and 5 (256 -> 5) in FP32 on the vector units: no
  rounding of operands (FP64 here),
  layers 2..4 (256 -> 256) on BF16 matrix cores with FP32 accumulation: the
  activations and weights are rounded to BF16 (round to nearest even)
  before each product; products and sums are exact here (FP64).
Backward uses the same rounding points: the gradient entering a BF16
product is rounded to BF16; weight gradients are accumulated in FP64 here.
"""
from __future__ import annotations

import numpy as np

SIZES = [6, 256, 256, 256, 256, 5]
BF16_LAYERS = (1, 2, 3)  # 0-based: the three 256 x 256 layers


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


def features(x6):
    """Network input features of entries x6 (6, n): the tangential wave
    numbers k_theta = cos(beta) sin(alpha) and k_z = sin(beta) in place of
    the azimuth and height (which the transit of the infinite cylinder does
    not depend on), then alpha, beta and the two bits. Returns (n, 6)."""
    x6 = np.asarray(x6, dtype=np.float64)
    al, be = x6[2], x6[3]
    return np.stack([np.cos(be) * np.sin(al), np.sin(be), al, be, x6[4], x6[5]], axis=1)


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
        if i in BF16_LAYERS:
            z = r(h) @ r(W) + b
        else:
            z = h @ W + b  # FP32 vector layer on the GPU
        zs.append(z)
        if i < 4:
            h = silu(z)
            acts.append(h)
        else:
            h = z
    return h, (zs, acts)


def loss_and_grads(params, x, t, w=None, bf16=False, huber=0.0):
    """Mean over the batch of sum_o w_o rho(y_o - t_o) and its gradients,
    rho(d) = d^2, or the Huber function for huber = delta > 0 (d^2 for
    |d| <= delta, 2 delta |d| - delta^2 beyond)."""
    n = x.shape[0]
    w = np.ones(5) if w is None else np.asarray(w, dtype=np.float64)
    y, (zs, acts) = forward(params, x, bf16)
    d = y - t
    big = (huber > 0) & (np.abs(d) > huber)
    rho = np.where(big, 2.0 * huber * np.abs(d) - huber * huber, d * d)
    drho = np.where(big, 2.0 * huber * np.sign(d), 2.0 * d)
    loss = float((w * rho).sum() / n)
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * 10
    g = w * drho / n  # dL/dz5
    for i in range(4, -1, -1):
        W = params[2 * i]
        a_in = acts[i]
        q = r if i in BF16_LAYERS else (lambda a: a)
        grads[2 * i] = q(a_in).T @ q(g)
        grads[2 * i + 1] = g.sum(axis=0)
        if i > 0:
            da = q(g) @ q(W).T
            g = da * silu_grad(zs[i - 1])
    return loss, grads


def is_bias_index(nparam_layout=SIZES):
    """Boolean mask over the flat parameter vector (W1, b1, ..., W5, b5, each
    weight (fan_in, fan_out) row-major): True for bias entries."""
    mask = []
    for i in range(5):
        mask.append(np.zeros(nparam_layout[i] * nparam_layout[i + 1], dtype=bool))
        mask.append(np.ones(nparam_layout[i + 1], dtype=bool))
    return np.concatenate(mask)


def adamw_step(p, g, m, v, step, lr, beta1, beta2, eps, weight_decay, decay_mask):
    """One AdamW step (Loshchilov & Hutter, decoupled weight decay) in FP64
    on flat arrays; `step` is the index t >= 1 of this step. Returns
    (p', m', v'):
      m' = beta1 m + (1 - beta1) g,   v' = beta2 v + (1 - beta2) g^2,
      p  <- p - lr wd p  where decay_mask (the weights, not the biases),
      p' = p - lr (m' / (1 - beta1^t)) / (sqrt(v' / (1 - beta2^t)) + eps)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m1 = beta1 * m + (1.0 - beta1) * g
    v1 = beta2 * v + (1.0 - beta2) * g * g
    pd = np.where(decay_mask, p - lr * weight_decay * p, p)
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    p1 = pd - lr * (m1 / c1) / (np.sqrt(v1 / c2) + eps)
    return p1, m1, v1


def grad_term_magnitudes(params, x, t, bf16=False, huber=0.0):
    """For each gradient tensor of loss_and_grads (same order), the sum S of
    the absolute values of the terms it adds up (over rows, and for weights
    of the products a_rk g_rj) and the largest single term Mx. Rounding
    error bounds of the gradient are combinations of the two: accumulation
    in a working precision u errs by at most ~ (terms) u S, and one operand
    rounded to the other side of a BF16 rounding boundary moves a sum by at
    most 2^-8 Mx."""
    n = x.shape[0]
    y, (zs, acts) = forward(params, x, bf16)
    d = y - t
    big = (huber > 0) & (np.abs(d) > huber)
    drho = np.where(big, 2.0 * huber * np.sign(d), 2.0 * d)
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    S, Mx = [None] * 10, [None] * 10
    g = drho / n
    for i in range(4, -1, -1):
        W = params[2 * i]
        q = r if i in BF16_LAYERS else (lambda a: a)
        A, G = np.abs(q(acts[i])), np.abs(q(g))
        S[2 * i] = A.T @ G
        mx = np.zeros((A.shape[1], G.shape[1]))
        for row in range(n):
            np.maximum(mx, np.outer(A[row], G[row]), out=mx)
        Mx[2 * i] = mx
        S[2 * i + 1] = np.abs(g).sum(axis=0)
        Mx[2 * i + 1] = np.abs(g).max(axis=0)
        if i > 0:
            g = (q(g) @ q(W).T) * silu_grad(zs[i - 1])
    return S, Mx
