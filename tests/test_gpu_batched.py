"""Batched workload: 64 seeded views x 512^2 x both cloaks x both branches,
recorded once into a HIP graph (rt_render_plan_*) and replayed; and the
3-D render replayed from plans overlapping on several streams."""
import numpy as np
import pytest

import oracle
from paper_1209_6038_amd import workloads as W
from tests.gpu_helpers import say
from tests.test_gpu_render import compare_samples

pytestmark = pytest.mark.gpu


def _cloaks():
    from paper_1209_6038_amd import rt
    return [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]


def test_plan_replays_match_eager_render():
    """Every replay of the captured graph gives the eager render bit for bit,
    with unrelated eager work and synchronizations between the replays."""
    import torch
    from paper_1209_6038_amd import rt
    cams = W.batched_views(64, 512)
    cls = _cloaks()
    opts = W.render_opts()
    say("case batched: eager render of 64 views x 512^2")
    rgb_e, aux_e = rt.render_multi(cls, opts, W.room(), cams, 3, aux=True)
    torch.cuda.synchronize()
    st = aux_e["status"]
    miss = (st == 1).float().mean().item()
    say(f"  miss fraction {miss:.3f}, entering rays {int((st != 1).sum())}")
    plan = rt.RenderPlan(cls, opts, W.room(), cams, 3, aux=True)
    small = [W.orbit_camera(1.0, 5.0, 32, 32)]
    for rep in range(3):
        say(f"  replay {rep}")
        plan.launch()
        # unrelated eager work between replays
        rt.render_multi(cls, opts, W.room(), small, 2)
        torch.cuda.synchronize()
        assert torch.equal(plan.rgb, rgb_e)
        for key in ("status", "code", "nsteps"):
            assert torch.equal(plan.aux[key], aux_e[key]), key
        assert torch.equal(torch.nan_to_num(plan.aux["rec"]), torch.nan_to_num(aux_e["rec"]))
        plan.rgb.zero_()
    plan.close()


def test_batched_full_size_sampled():
    """Sampled pixels of the full batched workload (through the graph)
    re-traced by the oracle."""
    import torch
    from paper_1209_6038_amd import rt
    cams = W.batched_views(64, 512)
    descs = [W.cloak(a, height=W.HEIGHT) for a in (0, 1)]
    cls = [rt.Cloak(d) for d in descs]
    plan = rt.RenderPlan(cls, W.render_opts(), W.room(), cams, 3, aux=True)
    plan.launch()
    torch.cuda.synchronize()
    aux = {k: v.cpu().numpy() for k, v in plan.aux.items()}
    plan.close()
    rng = np.random.default_rng(11)
    room = W.room()
    for k in rng.choice(64, 4, replace=False):
        for ci, c in enumerate(descs):
            for pi in range(2):
                st = aux["status"][ci, k, pi]
                hits = np.flatnonzero(st != 1)
                ids = np.unique(np.concatenate([rng.choice(st.size, 32, replace=False),
                                                rng.choice(hits, min(48, hits.size), replace=False)]))
                o = oracle.render_samples(c, W.opts_dp45(), room, cams[k], int(k), pi, ids)
                compare_samples(aux["code"][ci, k, pi][ids], aux["rec"][ci, k, pi][:, ids],
                                aux["status"][ci, k, pi][ids], o, room,
                                f"batched a{c['axis']} view{k} b{pi}")


def test_autotuner_choice_does_not_change_results():
    import torch
    from paper_1209_6038_amd import rt
    cams = W.batched_views(8, 128, seed=5)
    cls = _cloaks()
    tuned, ms = rt.autotune_render(cls, W.render_opts(), W.room(), cams, 3)
    say(f"autotuned block {tuned['block']} refill {tuned['refill_period']}: {ms:.3f} ms")
    assert tuned["block"] in (64, 128, 256) and tuned["refill_period"] in (1, 2, 4, 8, 12, 16)
    assert ms > 0
    a = rt.render_multi(cls, W.render_opts(), W.room(), cams, 3)
    b = rt.render_multi(cls, tuned, W.room(), cams, 3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("n_streams", [3, 4])
def test_overlapped_plans_match_eager_render(n_streams):
    """The benchmark's step loop (3 streams by default): the 3-D render
    (4 views x 1024^2, both cloaks and branches) recorded into one plan per
    stream, step k replayed from plan k mod S on stream k mod S so that
    consecutive steps overlap. Each plan owns its workspace: every replay
    gives the eager render bit for bit."""
    import torch
    from paper_1209_6038_amd import rt
    cams = W.render_views(res=1024)
    cls = _cloaks()
    opts = W.render_opts()
    say(f"case render3d: eager render, then {n_streams} plans x 3 overlapped replays")
    rgb_e, aux_e = rt.render_multi(cls, opts, W.room(), cams, 3, aux=True)
    torch.cuda.synchronize()
    plans = [rt.RenderPlan(cls, opts, W.room(), cams, 3, aux=True) for _ in range(n_streams)]
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    for rnd in range(3):
        for k in range(n_streams):
            with torch.cuda.stream(streams[k]):
                plans[k].launch()
        torch.cuda.synchronize()
        for k, p in enumerate(plans):
            assert torch.equal(p.rgb, rgb_e), (rnd, k)
            for key in ("status", "code", "nsteps"):
                assert torch.equal(p.aux[key], aux_e[key]), (rnd, k, key)
            assert torch.equal(torch.nan_to_num(p.aux["rec"]), torch.nan_to_num(aux_e["rec"])), (rnd, k)
            p.rgb.zero_()
        say(f"  round {rnd}: {n_streams} plans equal to the eager render")
    for p in plans:
        p.close()
