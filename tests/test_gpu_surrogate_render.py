"""GPU tests of rt_render_surrogate (through the C ABI): the render with the
side-to-side transits taken from the surrogate where its gate accepts them,
against the plain render rt_render_multi of the same views."""
import numpy as np
import pytest

from paper_1209_6038_amd import workloads as W
from tests.gpu_helpers import R2, angle_between, say
from tests.test_gpu_render import edge_distance

pytestmark = pytest.mark.gpu


def closed_form_model(calibrate_n=3_000_000, seed=77):
    """A model whose network outputs zero: its predictions are the closed-form
    transits of the infinite cylinder, calibrated like the trained one (half
    of the 1e-3 tolerance, resolved references only)."""
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    m = rt.Surrogate(seed=0)
    m.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    sc = m.get_scaling()
    sc[12:17] = 0.0
    sc[17:22] = 1.0
    m.set_scaling(sc)
    cl = S.make_cloaks(None)
    x = S.features(calibrate_n, seed)
    y, st, h = rt.transit_exact(cl, S.exact_opts(), x, hres=True)
    frac = m.calibrate(cl, x, y, st, tol=5e-4, min_count=16, dilate=1, hres_exact=h, unresolved=1e-6)
    say(f"trusted cells {frac:.4f}")
    return m


def trained_model(n_train=4_000_000, steps=1500, calibrate_n=3_000_000, seed=78):
    """A network trained like the benchmark's (AdamW on residuals of exact
    transits of the infinite cylinders, Huber loss, BF16 MFMA), on fewer rays
    and steps, then calibrated at half of the 1e-3 tolerance."""
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    cl = S.make_cloaks(None)
    x = S.features(n_train, seed)
    _, _, t, w = S.label(cl, x)
    m = rt.Surrogate(seed=seed)
    m.fit_scaling(x, t, w)
    loss = S.train(m, x, t, w, steps=steps, batch=65536, lr=2e-3, lr_end=2e-5, warmup=100, huber=0.01)
    say(f"trained {steps} steps, loss {loss:.3e}")
    del x, t, w
    xc = S.features(calibrate_n, seed + 1)
    y, st, h = rt.transit_exact(cl, S.exact_opts(), xc, hres=True)
    frac = m.calibrate(cl, xc, y, st, tol=5e-4, min_count=16, dilate=1, hres_exact=h, unresolved=1e-6)
    say(f"trusted cells {frac:.4f}")
    return m


@pytest.fixture(scope="module")
def models():
    return {"closed_form": closed_form_model(), "trained": trained_model()}


def both_renders(model, cams, opts, min_difficulty=0):
    import torch
    from paper_1209_6038_amd import rt
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    rgb_p, aux_p = rt.render_multi(cls, opts, W.room(), cams, 3, aux=True)
    rgb_s, aux_s, counts = rt.render_surrogate(model, cls, opts, W.room(), cams, 3, aux=True, counts=True,
                                               min_difficulty=min_difficulty)
    torch.cuda.synchronize()
    return rgb_p, aux_p, rgb_s, aux_s, counts


def test_surrogate_render_with_nothing_trusted_is_the_plain_render():
    """Every side entry rejected: each is generated again from its camera
    sample and integrated, so images, records and step counts equal the
    plain render's bit for bit, in one chunk and in many."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    m = rt.Surrogate(seed=0)
    x = S.features(4096, seed=5)
    y, st = rt.transit_exact(S.make_cloaks(None), S.exact_opts(), x)
    m.calibrate(S.make_cloaks(None), x, y, st, tol=1e-30)
    assert m.trust_map().sum() == 0
    cams = [W.orbit_camera(0.3, 20.0, 64, 64, spp=4, seed=3), W.orbit_camera(2.0, 40.0, 64, 64, spp=4, seed=3)]
    for opts in (W.render_opts(), W.render_opts(max_chunk=5000)):
        rgb_p, aux_p, rgb_s, aux_s, counts = both_renders(m, cams, opts)
        say(f"max_chunk {opts.get('max_chunk', 0)}: side entries {counts[0]}, accepted {counts[1]}")
        assert counts[0] > 1000 and counts[1] == 0
        assert torch.equal(rgb_p, rgb_s)
        for key in ("status", "code", "nsteps"):
            assert torch.equal(aux_p[key], aux_s[key]), key
        assert torch.equal(torch.nan_to_num(aux_p["rec"]), torch.nan_to_num(aux_s["rec"]))
        assert torch.equal(torch.nan_to_num(aux_p["tof"]), torch.nan_to_num(aux_s["tof"]))


@pytest.mark.parametrize("kind,min_difficulty", [("trained", 0), ("trained", 2), ("closed_form", 0)])
def test_surrogate_render_matches_the_plain_render(models, kind, min_difficulty):
    """With a calibrated model (the trained network, or its closed-form
    baselines alone) most offered side entries take the surrogate's exit
    ray. Samples it does not take are the plain render's bit for bit; the
    accepted ones leave where the integrator's rays leave (exit position and
    direction within the calibration tolerance, p99 at float32 resolution),
    and, with the tile-edge gate sending every accepted sample whose room
    point lies within twice its propagated exit-error bound of a tile edge
    to the integrator, they see the same tile: no pixel differs by more than
    1/255 in any channel. A difficulty threshold offers fewer entries (only
    those whose paths pass close to r = a)."""
    import torch
    model = models[kind]
    cams = [W.orbit_camera(0.3, 20.0, 96, 96, spp=4, seed=11), W.orbit_camera(2.5, 45.0, 96, 96, spp=4, seed=11),
            W.orbit_camera(4.0, 0.0, 96, 96, spp=4, seed=11)]
    rgb_p, aux_p, rgb_s, aux_s, counts = both_renders(model, cams, W.render_opts(), min_difficulty)
    say(f"min difficulty {min_difficulty}: side entries offered {counts[0]}, accepted {counts[1]} "
        f"({counts[1] / max(counts[0], 1):.4f})")
    # the rest exit through an end cap (or within the gate's margin of one)
    # or sit in untrusted cells
    assert counts[1] > 0.5 * counts[0]
    if min_difficulty == 0:
        assert counts[0] > 80000
    else:
        assert 1000 < counts[0] < 40000
    st_p, st_s = aux_p["status"], aux_s["status"]
    acc = (st_s == 0) & (aux_s["nsteps"] == 0) & (aux_p["nsteps"] > 0)
    assert int(acc.sum()) == counts[1]
    same = ~acc
    assert torch.equal(st_p[same], st_s[same])
    assert torch.equal(aux_p["code"][same], aux_s["code"][same])
    assert torch.equal(aux_p["nsteps"][same], aux_s["nsteps"][same])
    assert torch.equal(torch.nan_to_num(aux_p["rec"].transpose(3, 4)[same]),
                      torch.nan_to_num(aux_s["rec"].transpose(3, 4)[same]))
    # accepted samples: the integrator's ray left too (rays aimed at the
    # axis that it absorbs at the singular r = a are measure-zero)
    odd = acc & (st_p != 0)
    say(f"accepted but not exited by the integrator: {int(odd.sum())}")
    assert int(odd.sum()) <= max(1, int(1e-4 * counts[1]))
    ok = acc & (st_p == 0)
    rp = aux_p["rec"].transpose(3, 4)[ok].cpu().numpy().T  # (7, n)
    rs = aux_s["rec"].transpose(3, 4)[ok].cpu().numpy().T
    dpos = np.linalg.norm(rs[:3] - rp[:3], axis=0) / R2
    ddir = angle_between(rs[3:6], rp[3:6])
    err = np.maximum(dpos, ddir)
    say(f"accepted exit error: p50 {np.median(err):.2e} p99 {np.quantile(err, 0.99):.2e} max {err.max():.2e}")
    assert np.quantile(err, 0.99) <= 1e-5 and err.max() <= 1e-3
    # colours: the edge gate keeps every accepted room point away from tile
    # edges by more than the exit error can move it
    cp, cs = aux_p["code"][ok].cpu().numpy(), aux_s["code"][ok].cpu().numpy()
    diff = cp != cs
    dist, sroom = edge_distance(W.room(), rs[:6])
    say(f"accepted samples with another colour code: {int(diff.sum())} of {diff.size}; "
        f"closest accepted room point to a tile edge {dist.min():.2e}")
    assert not diff.any()
    d = (rgb_s - rgb_p).abs().amax(dim=-1)
    over = float((d > 1.0 / 255.0).float().mean())
    say(f"pixels differing by more than 1/255: {over:.2e} (max {float(d.max()):.3e})")
    assert float(d.max()) <= 1.0 / 255.0


def test_surrogate_render_argument_errors():
    from paper_1209_6038_amd import rt
    cams = [W.orbit_camera(0.3, 20.0, 8, 8)]
    cls = [rt.Cloak(W.cloak(0, height=W.HEIGHT))]
    m = rt.Surrogate(seed=0)
    with pytest.raises(rt.RtError):  # not calibrated
        rt.render_surrogate(m, cls, W.render_opts(), W.room(), cams, 3)
    with pytest.raises(rt.RtError):  # no cloak
        rt.render_surrogate(m, [], W.render_opts(), W.room(), cams, 3)
    with pytest.raises(rt.RtError):  # difficulty outside [0, 16]
        rt.render_surrogate(m, cls, W.render_opts(), W.room(), cams, 3, min_difficulty=17)
