"""GPU tests of the transit in entry/exit parameters (rt_transit_exact, parity
with the FP64 oracle) and of the surrogate MLP kernels (forward and gradients
against the FP64 reference with BF16 emulation, training, gated inference
with exact fallback)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1209_6038_amd import workloads as W
from tests.gpu_helpers import say
from tests.oracle_transit import oracle_exit_params

pytestmark = pytest.mark.gpu


def _angle_diff(a, b):
    return np.abs(np.angle(np.exp(1j * (a - b))))


@pytest.mark.parametrize("height", [None, W.HEIGHT])
def test_transit_exact_matches_oracle(height):
    """rt_transit_exact (all four (axis, branch) pairs in one launch) against
    the oracle per pair. Outputs are float32: ulp(2 pi) = 4.8e-7, ulp(8) =
    9.5e-7, so the bar is 4e-6 on angles and heights and 4e-6 relative on T
    (the FP64 integration itself agrees to 1e-6 of R2, rt_trace_batch tests)."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    n = 2000
    x6 = W.surrogate_features(n, seed=17)
    cloaks = S.make_cloaks(height)
    opts = S.exact_opts()
    # a few entries that cannot enter: grazing at |alpha| = pi/2, non-finite
    x6[2, :4] = np.float32(0.5 * math.pi)
    x6[0, 4:8] = np.nan
    say(f"case transit_exact height={height} n={n}")
    y5, st, hr = rt.transit_exact(cloaks, opts, torch.from_numpy(x6).cuda(), hres=True)
    torch.cuda.synchronize()
    y5, st, hr = y5.cpu().numpy(), st.cpu().numpy(), hr.cpu().numpy()
    assert (st[:8] == 6).all() and np.isnan(hr[:8]).all()
    for axis in (0, 1):
        for pol in (0, 1):
            sel = np.flatnonzero((x6[4] == pol) & (x6[5] == axis))
            sel = sel[sel >= 8]
            yo, so, ho = oracle_exit_params(W.cloak(axis, height=height), opts, x6[:, sel])
            assert (st[sel] == so).all(), (axis, pol, np.flatnonzero(st[sel] != so)[:5])
            ok = so == 0
            say(f"  axis {axis} pol {pol}: {sel.size} rays, {ok.sum()} exited, "
                f"statuses {np.bincount(so, minlength=8)}")
            g, o = y5[:, sel][:, ok], yo[:, ok]
            assert _angle_diff(g[0], o[0]).max() <= 4e-6
            assert (np.abs(g[1] - o[1]) <= 4e-6 * np.maximum(1.0, np.abs(o[1]))).all()
            assert np.abs(g[2] - o[2]).max() <= 4e-6
            assert np.abs(g[3] - o[3]).max() <= 4e-6
            assert (np.abs(g[4] - o[4]) <= 4e-6 * np.abs(o[4]) + 1e-6).all()
            assert np.isnan(y5[:, sel][:, ~ok]).all()
            # Hamiltonian drift at the exit: the same quantity of the same
            # scheme. It depends on the exact step sequence, and one
            # accept/reject decision taken differently by a rounding (which
            # moves the exit far less than 1e-6) changes it by tens of
            # percent: same magnitude, both sides of the 1e-6 threshold alike
            assert np.allclose(hr[sel][ok], ho[ok], rtol=0.5, atol=1e-9)
            assert ((hr[sel][ok] > 1e-6) == (ho[ok] > 1e-6)).all()
    # masked call: only the masked rays are written
    mask = torch.from_numpy((np.arange(n) % 3 == 0).astype(np.uint8)).cuda()
    x6t = torch.from_numpy(x6).cuda()
    y5m = torch.full((5, n), -7.0, device="cuda")
    stm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    rt.transit_exact(cloaks, opts, x6t, mask=mask, y5=y5m, status=stm)
    torch.cuda.synchronize()
    m = mask.cpu().numpy().astype(bool)
    assert (stm.cpu().numpy()[m] == st[m]).all() and (stm.cpu().numpy()[~m] == -1).all()
    assert np.array_equal(y5m.cpu().numpy()[:, m], y5[:, m], equal_nan=True)
    assert (y5m.cpu().numpy()[:, ~m] == -7.0).all()


def test_transit_conserves_tangential_wave_numbers():
    """Side-to-side transits of the infinite cloak leave with the tangential
    wave numbers they entered with, k_theta = cos(beta) sin(alpha) and
    k_z = sin(beta) (Sect. 3 refraction conserves the tangential wave vector
    at both interfaces; p_theta = r k_theta and p_z are conserved in
    between). The angles themselves are ill-conditioned at grazing
    incidence (d alpha = d k_theta / (cos beta cos alpha)), so the check is
    on the wave numbers, at the float32 resolution of the outputs."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    x6 = torch.from_numpy(W.surrogate_features(20000, seed=5)).cuda()
    y5, st = rt.transit_exact(S.make_cloaks(None), S.exact_opts(), x6)
    ok = st == 0
    say(f"exited {int(ok.sum())} of {ok.numel()}")
    assert ok.float().mean() > 0.98
    kt = torch.cos(x6[3].double()) * torch.sin(x6[2].double())
    kt2 = torch.cos(y5[3].double()) * torch.sin(y5[2].double())
    dkt = float((kt2 - kt)[ok].abs().max())
    dkz = float((torch.sin(y5[3].double()) - torch.sin(x6[3].double()))[ok].abs().max())
    say(f"max |dk_theta| {dkt:.2e}, max |dk_z| {dkz:.2e}")
    assert dkt < 1e-6 and dkz < 1e-6


def _oracle_params(p):
    out, off = [], 0
    for i in range(5):
        a, b = mlp.SIZES[i], mlp.SIZES[i + 1]
        out.append(p[off:off + a * b].astype(np.float64).reshape(a, b)); off += a * b
        out.append(p[off:off + b].astype(np.float64)); off += b
    assert off == p.size
    return out


def test_forward_matches_bf16_reference():
    """Forward on 300 rows (4 full 64-row tiles and a ragged tail) against
    the FP64 reference with BF16 rounding of layers 2-4. Remaining
    differences: FP32 accumulation order and FP32 SiLU, which flip a BF16
    rounding now and then (measured 2e-6 on outputs of size 6e-2; the bar
    leaves 10x room), against 8e-5 between the kernel and the unrounded
    FP64 network."""
    import torch
    from paper_1209_6038_amd import rt
    m = rt.Surrogate(seed=3)
    p = _oracle_params(m.get_params())
    x = np.random.default_rng(4).normal(size=(6, 300)).astype(np.float32)
    y = m.forward(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy().T.astype(np.float64)
    f = mlp.features(x)
    yo, _ = mlp.forward(p, f, bf16=True)
    y64, _ = mlp.forward(p, f, bf16=False)
    err, err64 = np.abs(y - yo).max(), np.abs(y - y64).max()
    say(f"forward: max |gpu - bf16 ref| {err:.2e}, |gpu - fp64 ref| {err64:.2e}, |y| {np.abs(yo).max():.2e}")
    assert err <= 2e-5
    assert err64 > 2 * err  # the rounding is where the reference puts it


@pytest.mark.parametrize("masked,huber", [(False, 0.0), (True, 0.0), (False, 0.5)])
def test_gradients_match_bf16_reference(masked, huber):
    """Gradients of the batch loss against the FP64 reference's (BF16
    rounding at the same points), element by element. Masked rows (weight
    0) must not contribute.

    Per-element bar, from the rounding the reference models. With S the sum
    of the absolute values of the terms an entry adds up and Mx its largest
    term (oracle.mlp.grad_term_magnitudes): the GPU's values before each
    BF16 rounding differ from the reference's FP64 ones by FP32 accumulation
    (~1e-7 relative); now and then such a value lies on the other side of a
    BF16 rounding boundary, and the rounded operand differs by one BF16 unit
    (2^-8 relative), which moves the values downstream, which flips further
    roundings in the layers below (the backward pass crosses three BF16
    layers). An entry then moves by a few BF16 units of its largest terms:
    |gpu - ref| <= 2^-3 Mx + 1e-4 S, 32 units, or 1e-4 of the summed
    magnitudes for the FP32 accumulation over up to 300 rows x 256 terms and
    the propagated differences. A CPU simulation of this cascade (relative
    noise up to 1e-6 before every rounding of the reference) stays within
    0.4 of the bar. The bar still resolves single rows: the test checks that
    dropping one row from the reference breaks it (in the simulation 40-87%
    of each weight tensor's entries then exceed it)."""
    import torch
    from paper_1209_6038_amd import rt
    m = rt.Surrogate(seed=8)
    p = _oracle_params(m.get_params())
    rng = np.random.default_rng(9)
    n = 300
    x = rng.normal(size=(6, n)).astype(np.float32)
    t = rng.normal(size=(5, n)).astype(np.float32)
    w = (rng.random(n) < 0.7).astype(np.float32) if masked else np.ones(n, np.float32)
    g, loss = m.grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), torch.from_numpy(w).cuda(),
                     huber=huber)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    keep = w > 0
    f, tt = mlp.features(x)[keep], t.T[keep].astype(np.float64)
    lo, go = mlp.loss_and_grads(p, f, tt, bf16=True, huber=huber)
    scale = keep.sum() / n  # the GPU loss is a mean over all n rows
    lo *= scale
    go = [gg * scale for gg in go]
    say(f"loss gpu {loss.item():.6e} ref {lo:.6e}")
    assert abs(loss.item() - lo) <= 1e-5 * lo
    S, Mx = mlp.grad_term_magnitudes(p, f, tt, bf16=True, huber=huber)
    bars = [(1e-4 * S[i] + 2.0 ** -3 * Mx[i]) * scale for i in range(10)]
    off = 0
    gpu_t = []
    for i, gg in enumerate(go):
        gpu = g[off:off + gg.size].reshape(gg.shape)
        gpu_t.append(gpu)
        off += gg.size
        ratio = np.abs(gpu - gg) / bars[i]
        worst = np.unravel_index(np.argmax(ratio), ratio.shape)
        say(f"  tensor {i} (layer {i // 2 + 1}): max |gpu - ref| / bar = {ratio.max():.3f} at {worst}, "
            f"max |gpu - ref| {np.abs(gpu - gg).max():.2e}, max |ref| {np.abs(gg).max():.2e}")
        assert (ratio <= 1.0).all(), (i, worst, gpu[worst], gg[worst])
    # the bar resolves one row: without the kept row with the largest loss
    # term, the reference's weight gradients leave it in every layer
    yk, _ = mlp.forward(p, f, bf16=True)
    drop = int(np.argmax(((yk - tt) ** 2).sum(axis=1)))
    sel = np.ones(len(f), bool)
    sel[drop] = False
    _, gd = mlp.loss_and_grads(p, f[sel], tt[sel], bf16=True, huber=huber)
    sd = (len(f) - 1) / n
    for i in range(0, 10, 2):
        over = (np.abs(gpu_t[i] - gd[i] * sd) > bars[i]).mean()
        say(f"  one row dropped: tensor {i}: {over:.1%} of the entries over the bar")
        assert over > 0.01, i


def test_closed_form_baselines_match_the_exact_transit():
    """The residual baselines are exact transits of the infinite cylinder
    for all four branches (radial cloak: homogeneous index sqrt(kappa) with
    the mirror for the ordinary branch, the elementary quadrature for the
    extraordinary one; azimuthal cloak: the elementary quadrature for the
    ordinary branch, a straight line in (sqrt(kappa)(r - a), theta,
    sqrt(kappa) z) for the extraordinary one): a network with zero output
    decodes to them, they match the integrator's exits, and the encoded
    targets of exact transits vanish, to float32 resolution. This includes
    the radial-o rays whose chord only just dips into the metal cylinder
    (near-grazing entries), which the integrator finds inside a step by the
    chord's closest approach."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cloaks = S.make_cloaks(None)
    opts = S.exact_opts()
    x = S.features(20000, seed=41)
    y_ex, st_ex = rt.transit_exact(cloaks, opts, x)
    t5, w = rt.surrogate_encode(cloaks, x, y_ex, st_ex)
    m = rt.Surrogate(seed=0)
    m.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    m.calibrate(cloaks, x, y_ex, st_ex, tol=1e30, min_count=1)
    y_s, st_s, fb = m.infer(cloaks, opts, x)
    torch.cuda.synchronize()
    kind = (x[5] * 2 + x[4]).long()
    err, operr = S.exit_error(y_s, y_ex)
    for k in range(4):
        sel = (kind == k) & (fb == 0) & (w > 0)
        assert sel.sum() > 4000
        e = S.summarize_errors(err, sel)
        say(f"kind {k}: baseline exit error {e}, max opl rel err {float(operr[sel].max()):.2e}")
        # float32 formulas vs the FP64 integrator: p99 at float32 resolution;
        # the max allows the few rays with p_theta -> 0 that pass close to
        # r = a, where the integrator's own tolerance-1e-8 error grows
        assert e["p99"] < 2e-6 and e["max"] < 1e-4
        assert float(operr[sel].max()) < 1e-4
        for o in (0, 1, 4):
            assert float(t5[o][sel].abs().max()) < 1e-4, o


def test_training_reduces_loss_and_save_load():
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    rng = np.random.default_rng(2)
    n = 32768
    x = rng.uniform(-1, 1, size=(6, n)).astype(np.float32)
    # a smooth map to fit, of inputs the network sees (entries 0 and 1 enter
    # only through k_theta = cos(x3) sin(x2) and k_z = sin(x3))
    t = np.stack([np.sin(2 * x[2]) * x[3], x[4] ** 2 - x[5], np.cos(x[2] + x[5]), x[4] * x[5], np.tanh(x[3] + x[4])])
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t.astype(np.float32)).cuda()
    m = rt.Surrogate(seed=1)
    m.fit_scaling(xt, tt)
    _, l0 = m.grad(xt, tt)
    last = S.train(m, xt, tt, torch.ones(n, device="cuda"), steps=600, batch=4096, lr=2e-3, warmup=50)
    say(f"loss {l0.item():.3e} -> {last:.3e}")
    assert last < 0.02 * l0.item()
    import os
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        m.save(path)
        m2 = rt.Surrogate(path=path)
        assert np.array_equal(m2.get_params(), m.get_params())
        assert np.array_equal(m2.get_scaling(), m.get_scaling())
        assert torch.equal(m2.forward(xt), m.forward(xt))


def test_surrogate_pipeline_small():
    """Small version of the surrogate workload: label entries with the exact
    transit, train briefly, calibrate the trust map on separate rays (about
    30 per cell) at half the tolerance, then infer on held-out rays. The
    integrator is the reference only where it resolves the path: exits whose
    Hamiltonian drift |H - 1| exceeds 1e-6 (entries with p_theta -> 0 that
    pass next to the singular r = a) and totally reflected exits (drift at
    grazing entries) are no reference, in calibration and here. The
    calibration bound is empirical (a cell is judged on its calibration
    rays), so accepted held-out rays with a resolved reference are checked
    at p99 and with at most 1e-4 of them over tol; rejected rays must carry
    exactly the exact transit's result."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cloaks = S.make_cloaks(None)
    opts = S.exact_opts()
    x_tr = S.features(1_000_000, seed=101)
    _, _, t_tr, w_tr = S.label(cloaks, x_tr, opts)
    m = rt.Surrogate(seed=0)
    m.fit_scaling(x_tr, t_tr, w_tr)
    last = S.train(m, x_tr, t_tr, w_tr, steps=3000, batch=8192, lr=2e-3, huber=0.01)
    say(f"train loss {last:.3e}")
    x_cal = S.features(2_000_000, seed=202)
    y_cal, st_cal, h_cal = rt.transit_exact(cloaks, opts, x_cal, hres=True)
    tol = 1e-3
    frac = m.calibrate(cloaks, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=16, dilate=1,
                       hres_exact=h_cal, unresolved=1e-6)
    say(f"trusted cells {frac:.4f}")
    x_ev = S.features(200_000, seed=303)
    y_ex, st_ex, h_ex = rt.transit_exact(cloaks, opts, x_ev, hres=True)
    y_s, st_s, fb = m.infer(cloaks, opts, x_ev)
    torch.cuda.synchronize()
    acc = fb == 0
    say(f"accepted {acc.float().mean().item():.4f}")
    assert acc.float().mean().item() > 0.95
    err, _ = S.exit_error(y_s, y_ex)
    # an accepted ray the integrator did not carry across: a ray aimed at
    # the axis (p_theta ~ 0) that the integrator brings to the singular
    # r = a and absorbs (the measure-zero case of the inner-cylinder
    # reading), in a cell whose calibration rays all passed
    odd = acc & (st_ex != 0) & (st_ex != 5)
    say(f"accepted but not exited by the integrator: {int(odd.sum())}, statuses "
        f"{torch.bincount(st_ex[odd].long(), minlength=8).tolist()}")
    assert int(odd.sum()) <= max(1, int(1e-4 * int(acc.sum())))
    # unresolved references: a drifted Hamiltonian, or total internal
    # reflection at the exit of a side entry into the infinite cylinder
    # (impossible in exact arithmetic: the tangential wave numbers are
    # conserved)
    resolved = (st_ex == 0) & (h_ex <= 1e-6)
    unres = acc & ~resolved & ((st_ex == 0) | (st_ex == 5))
    ux = unres & (st_ex == 0)
    say(f"accepted with an unresolved reference: {int(unres.sum())} ({int((unres & (st_ex == 5)).sum())} "
        f"totally reflected)" + (f", max difference of the exited {float(err[ux].max()):.2e}" if bool(ux.any()) else ""))
    acc = acc & resolved
    e = S.summarize_errors(err, acc)
    say(f"accepted exit error (resolved references) {e}")
    over = float((err[acc] > tol).float().mean())
    say(f"accepted over tol: {over:.2e}")
    assert e["p99"] <= 1e-5 and over <= 1e-4
    rej = fb == 1
    assert torch.equal(st_s[rej], st_ex[rej])
    assert torch.equal(torch.nan_to_num(y_s[:, rej]), torch.nan_to_num(y_ex[:, rej]))


def test_infer_with_nothing_trusted_is_exact():
    """With every cell untrusted the surrogate path is the exact transit."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cloaks = S.make_cloaks(W.HEIGHT)
    opts = S.exact_opts()
    m = rt.Surrogate(seed=0)
    x = S.features(5000, seed=7)
    y_ex, st_ex = rt.transit_exact(cloaks, opts, x)
    m.calibrate(cloaks, x, y_ex, st_ex, tol=1e-30)
    assert m.trust_map().sum() == 0
    y_s, st_s, fb = m.infer(cloaks, opts, x)
    torch.cuda.synchronize()
    assert bool((fb == 1).all())
    assert torch.equal(st_s, st_ex)
    assert torch.equal(torch.nan_to_num(y_s), torch.nan_to_num(y_ex))


def test_infer_rows_do_not_depend_on_the_batch():
    """Every row of rt_surrogate_infer gets what it would get alone: rows of
    a strided subset equal the full batch's bit for bit (accepted
    predictions, flags, statuses), and the rejected rows equal the exact
    transit's."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cloaks = S.make_cloaks(None)
    opts = S.exact_opts()
    m = rt.Surrogate(seed=0)
    m.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    x_cal = S.features(40000, seed=8)
    y_cal, st_cal = rt.transit_exact(cloaks, opts, x_cal)
    m.calibrate(cloaks, x_cal, y_cal, st_cal, tol=5e-4, min_count=4)
    x = S.features(60000, seed=9)
    y_s, st_s, fb = m.infer(cloaks, opts, x)
    y_ex, st_ex = rt.transit_exact(cloaks, opts, x)
    torch.cuda.synchronize()
    rej = fb == 1
    say(f"rejected {int(rej.sum())} of {x.shape[1]}")
    assert 0 < int(rej.sum()) < x.shape[1]
    assert torch.equal(st_s[rej], st_ex[rej])
    assert torch.equal(torch.nan_to_num(y_s[:, rej]), torch.nan_to_num(y_ex[:, rej]))
    sub = torch.arange(1, x.shape[1], 3, device=x.device)
    xs = x[:, sub].contiguous()
    y2, st2, fb2 = m.infer(cloaks, opts, xs)
    torch.cuda.synchronize()
    assert torch.equal(fb2, fb[sub])
    assert torch.equal(st2, st_s[sub])
    assert torch.equal(torch.nan_to_num(y2), torch.nan_to_num(y_s[:, sub]))


def test_adamw_step_matches_reference():
    """Two AdamW steps (rt_surrogate_step, the optimizer of
    rt_surrogate_train) from a seeded state (parameters, moments, step
    count 7) with seeded gradients, against the FP64 AdamW of the reference,
    element by element: parameters, first and second moments. The GPU works
    in FP32 on FP32 inputs (the reference takes the same FP32 values), a
    handful of roundings per entry: |m - ref| <= 2^-21 (beta1 |m| +
    (1 - beta1) |g|), likewise v, and |p - ref| <= 2^-21 (|p| + lr |m^| /
    (sqrt(v^) + eps)). Biases are not decayed."""
    import torch
    from paper_1209_6038_amd import rt
    n = rt.Surrogate.NPARAM
    rng = np.random.default_rng(12)
    m = rt.Surrogate(seed=13)
    p0 = m.get_params().astype(np.float64)
    m0 = rng.normal(scale=1e-3, size=n).astype(np.float32)
    v0 = (rng.normal(scale=1e-3, size=n) ** 2).astype(np.float32)
    m.set_state(m0, v0, 7)
    hp = dict(lr=np.float32(2e-3), beta1=np.float32(0.9), beta2=np.float32(0.995), eps=np.float32(1e-8),
              weight_decay=np.float32(0.01))
    mask = ~mlp.is_bias_index()
    pr, mr, vr = p0, m0.astype(np.float64), v0.astype(np.float64)
    for k in range(2):
        g = rng.normal(scale=1e-3, size=n).astype(np.float32)
        g[:50] = 0.0  # zero gradients: the update is the decay and the old moments alone
        m.step(torch.from_numpy(g).cuda(), **{a: float(b) for a, b in hp.items()})
        torch.cuda.synchronize()
        b1, b2 = float(hp["beta1"]), float(hp["beta2"])
        m_prev, v_prev = mr, vr
        pr, mr, vr = mlp.adamw_step(pr, g, mr, vr, 8 + k, float(hp["lr"]), b1, b2, float(hp["eps"]),
                                    float(hp["weight_decay"]), mask)
        pg = m.get_params().astype(np.float64)
        mg, vg, step = m.get_state()
        assert step == 8 + k
        gg = g.astype(np.float64)
        tol_m = 2.0 ** -21 * (b1 * np.abs(m_prev) + (1 - b1) * np.abs(gg)) + 1e-30
        tol_v = 2.0 ** -21 * (b2 * v_prev + (1 - b2) * gg * gg) + 1e-30
        upd = float(hp["lr"]) * np.abs(mr / (1 - b1 ** (8 + k))) / (np.sqrt(vr / (1 - b2 ** (8 + k))) +
                                                                     float(hp["eps"]))
        tol_p = 2.0 ** -21 * (np.abs(pr) + upd)
        say(f"step {k}: max |dm|/tol {np.max(np.abs(mg - mr) / tol_m):.3f}, "
            f"|dv|/tol {np.max(np.abs(vg - vr) / tol_v):.3f}, |dp|/tol {np.max(np.abs(pg - pr) / tol_p):.3f}")
        assert (np.abs(mg - mr) <= tol_m).all()
        assert (np.abs(vg - vr) <= tol_v).all()
        assert (np.abs(pg - pr) <= tol_p).all()
        # the next step starts from the GPU's FP32 state, as the GPU does
        pr, mr, vr = pg, mg.astype(np.float64), vg.astype(np.float64)
    m.close()


def test_train_step_counts_steps_and_reports_the_gradient_loss():
    """rt_surrogate_train evaluates the loss of rt_surrogate_grad (same
    forward; the reduction order of its atomics may differ, ~1e-7) and
    advances the step count that sets AdamW's bias corrections."""
    import torch
    from paper_1209_6038_amd import rt
    rng = np.random.default_rng(14)
    x = torch.from_numpy(rng.normal(size=(6, 700)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=(5, 700)).astype(np.float32)).cuda()
    a = rt.Surrogate(seed=15)
    _, lg = a.grad(x, t)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    a.train_step(x, t, lr=1e-3, weight_decay=0.01, loss=loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - lg.item()) <= 1e-6 * abs(lg.item())
    a.train_step(x, t, lr=1e-3, weight_decay=0.01)
    assert a.get_state()[2] == 2
    a.close()
