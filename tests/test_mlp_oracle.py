"""Pins of the FP64 MLP reference used to check the GPU surrogate kernels."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_definition():
    # exactly representable values stay; halfway cases round to even
    x = np.array([1.0, -2.5, 0.15625, 2.0 ** 127, 0.0], dtype=np.float32)
    np.testing.assert_array_equal(mlp.to_bf16(x), x.astype(np.float64))
    one_plus = np.float32(1.0) + np.float32(2.0 ** -8)   # halfway between 1 and 1+2^-7: ties to even (1)
    assert mlp.to_bf16(np.array([one_plus]))[0] == 1.0
    three_q = np.float32(1.0) + np.float32(3 * 2.0 ** -8)  # halfway, rounds up to even 1+2^-6
    assert mlp.to_bf16(np.array([three_q]))[0] == 1.0 + 2.0 ** -6
    assert mlp.to_bf16(np.array([1.0 + 2.0 ** -9], dtype=np.float32))[0] == 1.0


def test_forward_matches_torch_cpu():
    import torch
    p = mlp.init_params(3)
    x = np.random.default_rng(4).normal(size=(17, 6))
    y, _ = mlp.forward(p, x)
    layers = []
    for i in range(5):
        lin = torch.nn.Linear(mlp.SIZES[i], mlp.SIZES[i + 1], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(p[2 * i].T))
            lin.bias.copy_(torch.from_numpy(p[2 * i + 1]))
        layers.append(lin)
        if i < 4:
            layers.append(torch.nn.SiLU())
    net = torch.nn.Sequential(*layers)
    with torch.no_grad():
        yt = net(torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(y, yt, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("huber", [0.0, 0.3])
def test_backward_matches_finite_differences(huber):
    p = mlp.init_params(5)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(9, 6))
    t = rng.normal(size=(9, 5))
    w = np.array([1.0, 2.0, 0.5, 1.0, 3.0])
    loss, g = mlp.loss_and_grads(p, x, t, w, huber=huber)
    eps = 1e-6
    for li in range(10):
        P = p[li]
        flat_idx = rng.choice(P.size, 4, replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, P.shape)
            old = P[idx]
            P[idx] = old + eps
            lp, _ = mlp.loss_and_grads(p, x, t, w, huber=huber)
            P[idx] = old - eps
            lm, _ = mlp.loss_and_grads(p, x, t, w, huber=huber)
            P[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert g[li][idx] == pytest.approx(fd, rel=2e-5, abs=1e-8), (li, idx)


def test_silu_derivative():
    z = np.linspace(-8, 8, 33)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(mlp.silu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_huber_limits():
    """Huber with a delta above every residual is the squared error; with a
    small delta every residual is on the linear branch, whose value is
    2 delta |d| - delta^2 summed (a closed form checked directly)."""
    p = mlp.init_params(11)
    rng = np.random.default_rng(12)
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=(7, 5)) + 3.0
    l2, g2 = mlp.loss_and_grads(p, x, t)
    lh, gh = mlp.loss_and_grads(p, x, t, huber=1e3)
    assert lh == pytest.approx(l2, rel=1e-14)
    for a, b in zip(g2, gh):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)
    y, _ = mlp.forward(p, x)
    d = np.abs(y - t)
    delta = 1e-3
    assert d.min() > delta
    ls, _ = mlp.loss_and_grads(p, x, t, huber=delta)
    assert ls == pytest.approx((2 * delta * d - delta * delta).sum() / 7, rel=1e-13)


def test_features_are_the_tangential_wave_numbers():
    """k_theta and k_z are the components of the unit entry direction
    d = cos(beta) (cos(alpha) (-r) + sin(alpha) theta) + sin(beta) z along
    theta and z (built here from the vectors, not the formula)."""
    rng = np.random.default_rng(3)
    x6 = np.stack([rng.uniform(0, 6.28, 50), rng.uniform(0, 4, 50), rng.uniform(-1.5, 1.5, 50),
                   rng.uniform(-1.5, 1.5, 50), rng.integers(0, 2, 50), rng.integers(0, 2, 50)])
    f = mlp.features(x6)
    for i in range(50):
        phi, al, be = x6[0, i], x6[2, i], x6[3, i]
        rh = np.array([np.cos(phi), np.sin(phi), 0.0])
        th = np.array([-np.sin(phi), np.cos(phi), 0.0])
        ez = np.array([0.0, 0.0, 1.0])
        d = np.cos(be) * (np.cos(al) * -rh + np.sin(al) * th) + np.sin(be) * ez
        assert abs(np.linalg.norm(d) - 1) < 1e-12
        assert f[i, 0] == pytest.approx(d @ th, abs=1e-13)
        assert f[i, 1] == pytest.approx(d @ ez, abs=1e-13)
        assert list(f[i, 2:]) == [al, be, x6[4, i], x6[5, i]]


def test_adamw_matches_torch_cpu():
    """Three AdamW steps of the reference against torch.optim.AdamW in
    float64, weights decayed and biases not (two parameter groups)."""
    import torch
    rng = np.random.default_rng(11)
    shapes = [(3, 4), (4,), (4, 2), (2,)]  # a small layout of the same kind: W, b, W, b
    p0 = [rng.normal(size=s_) for s_ in shapes]
    hp = dict(lr=3e-3, betas=(0.85, 0.99), eps=1e-7, weight_decay=0.05)
    tw = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in p0]
    opt = torch.optim.AdamW([{"params": [tw[0], tw[2]], "weight_decay": hp["weight_decay"]},
                             {"params": [tw[1], tw[3]], "weight_decay": 0.0}],
                            lr=hp["lr"], betas=hp["betas"], eps=hp["eps"])
    flat = np.concatenate([a.ravel() for a in p0])
    mask = np.concatenate([np.full(a.size, len(a.shape) == 2) for a in p0])
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    for t in range(1, 4):
        grads = [rng.normal(size=s_) for s_ in shapes]
        for tt, gg in zip(tw, grads):
            tt.grad = torch.tensor(gg, dtype=torch.float64)
        opt.step()
        gflat = np.concatenate([a.ravel() for a in grads])
        flat, m, v = mlp.adamw_step(flat, gflat, m, v, t, hp["lr"], hp["betas"][0], hp["betas"][1],
                                    hp["eps"], hp["weight_decay"], mask)
        ref = np.concatenate([tt.detach().numpy().ravel() for tt in tw])
        np.testing.assert_allclose(flat, ref, rtol=0, atol=1e-14)


def test_bias_mask_layout():
    mask = mlp.is_bias_index()
    assert mask.size == 200453
    assert mask.sum() == 256 * 4 + 5
    assert not mask[:6 * 256].any() and mask[6 * 256:6 * 256 + 256].all()
