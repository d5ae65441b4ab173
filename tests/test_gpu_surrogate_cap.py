"""GPU tests of the surrogate's cap job: side entries of a cloak of finite
height whose path meets an end cap, which the closed-form transits of the
infinite cylinder cannot give. The encoding is compared with the FP64
cap-state geometry (tests/cap_geometry.py) on the oracle's exits; a
trained and calibrated cap model's accepted predictions with the exact
transit; the closed-form-only model must reject every cap exit; chaining
the two keeps each one's accepted rows."""
import math

import numpy as np
import pytest

from paper_1209_6038_amd import workloads as W
from tests import cap_geometry as G
from tests.gpu_helpers import say
from tests.oracle_transit import oracle_exits

pytestmark = pytest.mark.gpu

B, Z0, Z1 = W.R2, 0.0, W.HEIGHT
TOL = 1e-3  # exit error bar of an accepted prediction (units of r2, radians)


def _unwrap(s, a):
    """Signed sweep with the sign s: s * ((s a) mod 2 pi)."""
    return s * np.mod(s * a, 2.0 * math.pi)


def test_cap_targets_match_fp64_geometry():
    """rt_surrogate_encode_job(RT_SUR_CAP) on the oracle's exits (FP64,
    rounded to FP32 as the GPU's inputs) against the FP64 geometry: which
    rows get w = 1 (leave through the cap they head for, u < 1 with the
    rise dz_0 of the oracle's infinite-cylinder transit) and their targets
    (the cap state against the chord model, tests/cap_geometry.chord_state:
    t0 = dtheta_c - frac dtheta_0, r_c, d_r and |d_z| less the chord's,
    t3 = T_c - u T_0). FP32
    inputs: the exit point and direction carry ~1e-7 relative error, which
    the vacuum leg of length tb back to the cap multiplies."""
    import torch
    from paper_1209_6038_amd import rt
    x6 = W.surrogate_features(20000, seed=41)
    opts = W.opts_dp45(1e-10, r_out=B)
    y5, st, _ = oracle_exits([W.cloak(0, height=W.HEIGHT), W.cloak(1, height=W.HEIGHT)], opts, x6)
    yi, sti, _ = oracle_exits([W.cloak(0), W.cloak(1)], opts, x6)
    xd = x6.astype(np.float64)
    s = np.where(xd[2] < 0, -1.0, 1.0)
    dz0 = yi[1] - xd[1]
    dth0 = _unwrap(s, yi[0] - xd[0])
    T0 = yi[4]
    up = xd[3] >= 0
    u = np.where(up, Z1 - xd[1], xd[1] - Z0) / np.abs(dz0)
    beyond = np.where(up, y5[1] > Z1, y5[1] < Z0)
    w_ref = (st == 0) & (sti == 0) & beyond & (u < 1)
    # borderline rows that FP32 rounding may put on either side
    border = (np.abs(u - 1) < 1e-4) | (np.abs(y5[1] - Z1) < 1e-4) | (np.abs(y5[1] - Z0) < 1e-4)
    say(f"case cap encoding n={x6.shape[1]}: {int(w_ref.sum())} cap exits, {int(border.sum())} borderline")
    cl = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    xg = torch.from_numpy(x6).cuda()
    yg = torch.from_numpy(np.nan_to_num(y5, nan=0.0).astype(np.float32)).cuda()
    sg = torch.from_numpy(st.astype(np.int32)).cuda()
    t5, w = rt.surrogate_encode(cl, xg, yg, sg, job=rt.CAP)
    t5, w = t5.cpu().numpy().astype(np.float64), w.cpu().numpy()
    assert ((w == 1) | (w == 0)).all()
    # the reference terms need the infinite-cylinder transit to exit
    cmp = ~border & (sti == 0)
    assert ((w == 1) == w_ref)[cmp].all(), np.flatnonzero(((w == 1) != w_ref) & cmp)[:5]
    sel = w_ref & (w == 1) & ~border
    assert sel.sum() > 1000
    cs = G.cap_state(xd[:, sel], y5[:, sel], B, Z0, Z1)
    frac, rch, drh, adzh = (np.empty(int(sel.sum())) for _ in range(4))
    idx = np.flatnonzero(sel)
    for axis in (0, 1):
        for branch in (0, 1):
            k = (xd[5, idx] == axis) & (xd[4, idx] == branch)
            if k.any():
                j = idx[k]
                frac[k], rch[k], drh[k], adzh[k] = G.chord_state(
                    axis, branch, np.cos(xd[3, j]) * np.sin(xd[2, j]), np.sin(xd[3, j]), u[j], W.R1, B)
    ref = [cs["dth"] - frac * dth0[sel], cs["rc"] - rch, cs["dr"] - drh, cs["Tc"] - u[sel] * T0[sel],
           np.abs(cs["dz"]) - adzh]
    # the chord's radial wave number is a square root of a difference that
    # cancels next to the turning point: in FP32 (the GPU's encoding and
    # decoding share it) it is good to ~1e-7 / |d_r|, hence the t2 and t4 bars
    lead = 1.0 + cs["tb"]
    bars = (1e-5, 5e-6, 5e-5, 2e-5, 5e-5)
    for o in range(5):
        d = np.abs(t5[o, sel] - ref[o]) / lead
        say(f"  t{o}: max |gpu - fp64| / (1 + tb) = {d.max():.2e}")
        assert d.max() <= bars[o], (o, d.max())
    for c in cl:
        c.close()


@pytest.fixture(scope="module")
def cap_setup():
    """A cap model trained on the cap exits of 8 M uniform side entries of
    the height-4 cloaks and calibrated (tol / 2, cells of >= 8 rays, the
    neighbours of failing cells distrusted) on 16 M others, the
    closed-form-only side model (zero network, every cell trusted), and 1 M
    held-out entries with their exact transits."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cl = S.make_cloaks(W.HEIGHT)
    op = S.exact_opts()
    x_tr, t_tr, w_tr = S.cap_training_set(8_000_000, seed=501, opts=op)
    m = rt.Surrogate(seed=0)
    m.set_job(rt.CAP, cl[0])
    assert m.job == rt.CAP
    m.fit_scaling(x_tr, t_tr, w_tr)
    last = S.train(m, x_tr, t_tr, w_tr, steps=20000, batch=16384, lr=1e-3, lr_end=1e-5, huber=0.01)
    say(f"cap model: {x_tr.shape[1]} training rows, loss {last:.3e}")
    del x_tr, t_tr, w_tr
    x_cal = S.features(16_000_000, seed=502)
    y_cal, st_cal, h_cal = rt.transit_exact(cl, op, x_cal, hres=True)
    frac = m.calibrate(cl, x_cal, y_cal, st_cal, tol=0.5 * TOL, min_count=8, dilate=1, hres_exact=h_cal,
                       unresolved=1e-6, p_min=0.0)
    say(f"trusted cells {frac:.4f}")
    del x_cal, y_cal, st_cal, h_cal
    base = rt.Surrogate(seed=0)
    base.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    sc = base.get_scaling()
    sc[12:22] = np.concatenate([np.zeros(5, np.float32), np.ones(5, np.float32)])
    base.set_scaling(sc)
    x_ev = S.features(1_000_000, seed=503)
    y_ex, st_ex, h_ex = rt.transit_exact(cl, op, x_ev, hres=True)
    base.calibrate(cl, x_ev, y_ex, st_ex, tol=1e30, min_count=1, p_min=0.0)
    torch.cuda.synchronize()
    yield m, base, cl, op, x_ev, y_ex, st_ex, h_ex
    base.close()
    m.close()


def _cap_exits(x_ev, y_ex, st_ex):
    up = x_ev[3] >= 0
    return (st_ex == 0) & (((y_ex[1] > Z1) & up) | ((y_ex[1] < Z0) & ~up))


def _resolved(x_ev, h_ex):
    """Exact transits the integrator resolves: Hamiltonian drift |H - 1| at
    the exit below 1e-6 and below the entry's squared normal wave number
    (cos alpha cos beta)^2, which the exit refraction keeps (the tangential
    wave numbers are conserved). A side entry at grazing incidence has a
    tiny one; a drift above it turns the side exit into a total reflection,
    and the ray runs on to a cap."""
    import torch
    kn = torch.cos(x_ev[2]) * torch.cos(x_ev[3])
    return (h_ex <= 1e-6) & (h_ex < kn * kn)


def test_cap_model_accepts_cap_exits_within_tolerance(cap_setup):
    """Accepted predictions of the cap model alone: each is a cap exit of
    the exact transit, within TOL of it where the integrator resolves the
    path (_resolved); the calibration bound is empirical,
    so at most 1e-4 of them may exceed TOL. A real share of the cap exits is
    accepted, and every rejected row carries the exact transit's result."""
    import torch
    from paper_1209_6038_amd import surrogate as S
    m, base, cl, op, x_ev, y_ex, st_ex, h_ex = cap_setup
    say("case cap model alone on 1 M held-out entries")
    y_s, st_s, fb = m.infer(cl, op, x_ev)
    torch.cuda.synchronize()
    acc = fb == 0
    cap = _cap_exits(x_ev, y_ex, st_ex)
    resolved = _resolved(x_ev, h_ex)
    share = float(acc[cap].float().mean())
    say(f"cap exits {int(cap.sum())}, accepted {int(acc.sum())} ({share:.3f} of the cap exits)")
    assert share > 0.1
    assert int((acc & ~cap).sum()) <= max(1, int(1e-4 * int(acc.sum())))
    err, _ = S.exit_error(y_s, y_ex)
    a = acc & cap & resolved
    over = int((err[a] > TOL).sum())
    say(f"accepted exit error: p50 {float(err[a].median()):.2e}, max {float(err[a].max()):.2e}, over TOL {over}")
    assert over <= max(1, int(1e-4 * int(a.sum())))
    rej = ~acc
    assert torch.equal(st_s[rej], st_ex[rej])
    assert torch.equal(torch.nan_to_num(y_s[:, rej]), torch.nan_to_num(y_ex[:, rej]))


def test_closed_forms_reject_every_cap_exit_and_the_chain_adds_them(cap_setup):
    """The side model with its network output zeroed (the closed-form
    transits alone) and every cell trusted rejects every entry that leaves
    through a cap where the integrator resolves the path (_resolved: a
    drifted reference can leave through a cap that the path does not
    reach); chained to the cap
    model, its accepted rows stay as they were, the rows it rejects that the
    cap model accepts take the cap model's prediction, and the rest take the
    exact transit."""
    import torch
    m, base, cl, op, x_ev, y_ex, st_ex, h_ex = cap_setup
    cap = _cap_exits(x_ev, y_ex, st_ex) & _resolved(x_ev, h_ex)
    say("case closed forms alone, then chained to the cap model")
    y_b, st_b, fb_b = base.infer(cl, op, x_ev)
    y_c, st_c, fb_c = m.infer(cl, op, x_ev)
    base.chain(m)
    try:
        y_k, st_k, fb_k = base.infer(cl, op, x_ev)
    finally:
        base.chain(None)
    torch.cuda.synchronize()
    assert bool((fb_b[cap] == 1).all())
    ab, ac = fb_b == 0, fb_c == 0
    assert torch.equal(fb_k == 0, ab | (ac & ~ab))
    assert torch.equal(torch.nan_to_num(y_k[:, ab]), torch.nan_to_num(y_b[:, ab]))
    only_c = ac & ~ab
    assert torch.equal(torch.nan_to_num(y_k[:, only_c]), torch.nan_to_num(y_c[:, only_c]))
    rej = fb_k == 1
    assert torch.equal(torch.nan_to_num(y_k[:, rej]), torch.nan_to_num(y_ex[:, rej]))
    assert torch.equal(st_k[rej], st_ex[rej])
    say(f"accepted: closed forms {float(ab.float().mean()):.4f}, chained {float((fb_k == 0).float().mean()):.4f}; "
        f"cap exits accepted: {float((fb_k[cap] == 0).float().mean()):.4f} (closed forms 0)")
    assert float((fb_k[cap] == 0).float().mean()) > 0.1


def test_cap_model_save_load_and_job_errors(cap_setup, tmp_path):
    """The model file keeps the job and the geometry; a cap model refuses
    cloaks of another geometry."""
    import torch
    from paper_1209_6038_amd import rt
    m, base, cl, op, x_ev, y_ex, st_ex, h_ex = cap_setup
    p = str(tmp_path / "cap.bin")
    m.save(p)
    m2 = rt.Surrogate(path=p)
    assert m2.job == rt.CAP
    x = x_ev[:, :4096].contiguous()
    assert torch.equal(m2.forward(x), m.forward(x))
    assert np.array_equal(m2.trust_map(), m.trust_map()) and m.trust_map().shape == (4, 32, 16, 32)
    other = [rt.Cloak(W.cloak(a, height=2.0)) for a in (0, 1)]
    with pytest.raises(rt.RtError) as ex:
        m2.infer(other, op, x)
    assert "geometry" in str(ex.value)
    inf = [rt.Cloak(W.cloak(0))]
    with pytest.raises(rt.RtError):
        m2.set_job(rt.CAP, inf[0])
    m2.set_job(rt.SIDE)
    assert m2.job == rt.SIDE and m2.trust_map().shape == (4, 128, 128)
    m2.close()


def _forward_to_r2(rec):
    """Exit points (records (7, n): point, direction, ...) moved along their
    direction to r = R2 where they lie inside it (cap points)."""
    x, d = rec[:3], rec[3:6]
    qa = d[0] ** 2 + d[1] ** 2
    qb = x[0] * d[0] + x[1] * d[1]
    qc = x[0] ** 2 + x[1] ** 2 - B * B
    s = np.where(qc < -1e-9, (-qb + np.sqrt(np.maximum(qb * qb - qa * qc, 0.0))) / np.maximum(qa, 1e-30), 0.0)
    return x + s * d


def test_chained_render_matches_the_plain_render(cap_setup):
    """rt_render_surrogate with the closed-form side model (calibrated as in
    the side job's render tests) chained to the cap model: the same side
    entries are offered, more of them are accepted than by the side model
    alone (cap exits), accepted samples leave where the integrator's rays
    leave (within TOL), the others are the plain render's bit for bit, and no
    pixel differs from the plain render by more than 1/255 (tile-edge gate
    with the chain's tolerance)."""
    import torch
    from paper_1209_6038_amd import rt
    from tests.gpu_helpers import R2, angle_between
    from tests.test_gpu_surrogate_render import closed_form_model
    m = cap_setup[0]
    side = closed_form_model()
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    cams = [W.orbit_camera(0.3, 20.0, 96, 96, spp=4, seed=11), W.orbit_camera(2.5, 45.0, 96, 96, spp=4, seed=11),
            W.orbit_camera(4.0, 60.0, 96, 96, spp=4, seed=11)]
    opts = W.render_opts()
    say("case chained render: 3 views 96 x 96 x 4 spp")
    rgb_p, aux_p = rt.render_multi(cls, opts, W.room(), cams, 3, aux=True)
    _, _, c_side = rt.render_surrogate(side, cls, opts, W.room(), cams, 3, aux=True, counts=True)
    side.chain(m)
    try:
        rgb_s, aux_s, c_chain = rt.render_surrogate(side, cls, opts, W.room(), cams, 3, aux=True, counts=True)
    finally:
        side.chain(None)
    torch.cuda.synchronize()
    say(f"offered {c_side[0]}, accepted by the side model {c_side[1]}, chained {c_chain[1]}")
    assert c_chain[0] == c_side[0] and c_chain[1] > c_side[1]
    st_p, st_s = aux_p["status"], aux_s["status"]
    acc = (st_s == 0) & (aux_s["nsteps"] == 0) & (aux_p["nsteps"] > 0)
    assert int(acc.sum()) == c_chain[1]
    same = ~acc
    assert torch.equal(st_p[same], st_s[same]) and torch.equal(aux_p["code"][same], aux_s["code"][same])
    assert torch.equal(torch.nan_to_num(aux_p["rec"].transpose(3, 4)[same]),
                       torch.nan_to_num(aux_s["rec"].transpose(3, 4)[same]))
    ok = acc & (st_p == 0)
    assert int((acc & (st_p != 0)).sum()) <= max(1, int(1e-4 * c_chain[1]))
    rp = aux_p["rec"].transpose(3, 4)[ok].cpu().numpy().T.astype(np.float64)
    rs = aux_s["rec"].transpose(3, 4)[ok].cpu().numpy().T.astype(np.float64)
    # both record where the ray left the crystal (a cap point for a cap
    # exit); the calibration bounds the exit ray where it crosses r = r2
    err = np.maximum(np.linalg.norm(_forward_to_r2(rs) - _forward_to_r2(rp), axis=0) / R2,
                     angle_between(rs[3:6], rp[3:6]))
    say(f"accepted exit error: p50 {np.median(err):.2e} max {err.max():.2e}")
    assert err.max() <= TOL
    d = (rgb_s - rgb_p).abs().amax(dim=-1)
    say(f"max pixel difference {float(d.max()):.3e}")
    assert float(d.max()) <= 1.0 / 255.0
    side.close()


def test_chain_rules_and_freeing_a_chained_model():
    """A chain holds two models: a model cannot follow itself, a chained
    model cannot start or extend another chain, and freeing either model
    unchains the other (its next calls work alone, with no reference to the
    freed one)."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    a, b, c = rt.Surrogate(seed=1), rt.Surrogate(seed=2), rt.Surrogate(seed=3)
    cl = S.make_cloaks(None)
    x = S.features(4096, seed=9)
    y, st = rt.transit_exact(cl, S.exact_opts(), x)
    for m in (a, b, c):
        m.calibrate(cl, x, y, st, tol=1e-30)
    with pytest.raises(rt.RtError):
        a.chain(a)
    a.chain(b)
    with pytest.raises(rt.RtError):
        b.chain(c)  # b follows a: it cannot start a chain
    with pytest.raises(rt.RtError):
        c.chain(a)  # a leads a chain: it cannot follow
    with pytest.raises(rt.RtError):
        c.chain(b)  # b already follows a
    y1, st1, fb1 = a.infer(cl, S.exact_opts(), x)
    b.close()  # unchains a
    y2, st2, fb2 = a.infer(cl, S.exact_opts(), x)
    torch.cuda.synchronize()
    assert bool((fb1 == 1).all()) and bool((fb2 == 1).all())
    assert torch.equal(torch.nan_to_num(y1), torch.nan_to_num(y2)) and torch.equal(st1, st2)
    a.chain(c)
    a.close()  # unchains c, which can now lead a chain of its own
    c.chain(rt.Surrogate(seed=4))
    c.chain(None)
    c.close()
