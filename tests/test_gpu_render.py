"""GPU parity of rt_render against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1209_6038_amd import workloads as W
from tests.gpu_helpers import R2, angle_between, say

pytestmark = pytest.mark.gpu


def gpu_render(cloak_d, opts, cams, pol_mask):
    import torch
    from paper_1209_6038_amd import rt
    cl = rt.Cloak(cloak_d) if cloak_d is not None else None
    rgb, aux = rt.render(cl, opts, W.room(), cams, pol_mask, aux=True)
    torch.cuda.synchronize()
    res = rgb.cpu().numpy(), {k: v.cpu().numpy() for k, v in aux.items()}
    if cl is not None:
        cl.close()
    return res


def edge_distance(room, rec):
    """Distance of the room point seen by each record to the nearest tile edge."""
    o, d = rec[:3], rec[3:6]
    lo, hi, tile = np.array(room["lo"]), np.array(room["hi"]), room["tile"]
    s = np.full(o.shape[1], np.inf)
    face_ax = np.zeros(o.shape[1], int)
    for ax in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            plane = np.where(d[ax] > 0, hi[ax], lo[ax])
            sa = np.where(d[ax] != 0, (plane - o[ax]) / d[ax], np.inf)
        better = sa < s
        s = np.where(better, sa, s)
        face_ax = np.where(better, ax, face_ax)
    p = o + s * d
    dist = np.full(o.shape[1], np.inf)
    for ax in range(3):
        fr = p[ax] / tile - np.floor(p[ax] / tile)
        dd = np.minimum(fr, 1 - fr) * tile
        dist = np.where(face_ax != ax, np.minimum(dist, dd), dist)
    return dist, s


def compare_samples(g_code, g_rec, g_st, o, room, label, pos_tol=1e-6, dir_tol=1e-6):
    st_same = g_st == o["status"]
    assert st_same.all(), f"{label}: status differs at {np.flatnonzero(~st_same)[:10]}"
    ok = np.isin(o["status"], (0, 1, 7))
    dpos = np.linalg.norm(g_rec[:3] - o["rec"][:3], axis=0) / R2
    ddir = angle_between(g_rec[3:6], o["rec"][3:6])
    dopl = np.abs(g_rec[6] - o["rec"][6])
    say(f"{label}: n={ok.sum()} max pos/R2={dpos[ok].max(initial=0):.3e} "
        f"dir={ddir[ok].max(initial=0):.3e} opl={dopl[ok].max(initial=0):.3e}")
    assert dpos[ok].max(initial=0) <= pos_tol
    assert ddir[ok].max(initial=0) <= dir_tol
    # tile parity is decided from the hit point: a differing code is only
    # acceptable within the propagated error of a tile edge
    diff = g_code != o["code"]
    if diff.any():
        dist, s = edge_distance(room, o["rec"])
        allowed = dist <= (pos_tol * R2 + s * dir_tol) * 4 + 1e-12
        assert allowed[diff].all(), f"{label}: code differs away from tile edges at {np.flatnonzero(diff & ~allowed)[:10]}"
    say(f"  codes differing at tile edges: {diff.sum()} of {len(diff)}")


def compare_tof(g_tof, o, spp):
    """Per-pixel time of flight against the oracle's samples: the mean optical
    path of the samples that reach the room (black ones left out), NaN where
    none does. float32 output: 4e-6 relative."""
    L = np.where(o["code"] < 12, o["rec"][6], np.nan).reshape(-1, spp)
    cnt = np.isfinite(L).sum(axis=1)
    want = np.where(cnt > 0, np.nansum(L, axis=1) / np.maximum(cnt, 1), np.nan)
    g = g_tof.reshape(-1)
    assert np.array_equal(np.isnan(g), np.isnan(want))
    ok = np.isfinite(want)
    assert (np.abs(g[ok] - want[ok]) <= 4e-6 * np.abs(want[ok]) + 1e-6).all()


@pytest.mark.parametrize("axis", [0, 1])
def test_render_small_parity(axis):
    cams = W.render_views(res=48)
    c = W.cloak(axis, height=W.HEIGHT)
    op = W.render_opts()
    say(f"case render small axis={axis}")
    rgb, aux = gpu_render(c, op, cams, 3)
    room = W.room()
    table = np.zeros((13, 3))
    table[:12] = room["rgb"].reshape(12, 3)
    ns = 48 * 48
    for k, cam in enumerate(cams):
        for pi, branch in enumerate((0, 1)):
            o = oracle.render_samples(c, W.opts_dp45(), room, cam, k, branch, np.arange(ns))
            compare_samples(aux["code"][k, pi], aux["rec"][k, pi], aux["status"][k, pi], o, room,
                            f"small a{axis} cam{k} b{branch}")
            want = table[aux["code"][k, pi]].reshape(48, 48, 3)
            np.testing.assert_allclose(rgb[k, pi], want, atol=1e-7)
            compare_tof(aux["tof"][k, pi], o, 1)


@pytest.mark.parametrize("axis", [0, 1])
def test_render_hamiltonian_form_parity(axis):
    """The 3-D render with the Hamiltonian form (RK4 in tau, step 2e-3) on
    both branches, against the oracle's Hamiltonian tracer sample by sample:
    statuses, exit rays within the 1e-6 bar, colour codes and the time of
    flight (from dt/dtau = 2 f). The step limit bounds the rays aimed at the
    axis, which stall in tau; both sides stop them the same way."""
    cams = W.render_views(res=32)
    c = W.cloak(axis, height=W.HEIGHT)
    op = W.opts_rk4_ham(h=2e-3, max_steps=100_000)
    say(f"case render hamiltonian axis={axis}")
    rgb, aux = gpu_render(c, op, cams, 3)
    room = W.room()
    for k, cam in enumerate(cams):
        for pi, branch in enumerate((0, 1)):
            o = oracle.render_samples(c, op, room, cam, k, branch, np.arange(32 * 32))
            compare_samples(aux["code"][k, pi], aux["rec"][k, pi], aux["status"][k, pi], o, room,
                            f"ham a{axis} cam{k} b{branch}")
            compare_tof(aux["tof"][k, pi], o, 1)


def test_render_empty_room():
    """No cloak: camera rays hit the room directly. Codes agree except where a
    ray lands exactly on a tile edge (the elevation-0 camera sits at z = 2, a
    tile boundary, so symmetric rays produce exact ties)."""
    cams = W.render_views(res=32)
    rgb, aux = gpu_render(None, W.render_opts(), cams, 2)
    room = W.room()
    for k, cam in enumerate(cams):
        o = oracle.render_samples(None, W.opts_dp45(), room, cam, k, 1, np.arange(32 * 32))
        assert (aux["status"][k, 0] == 1).all()
        compare_samples(aux["code"][k, 0], aux["rec"][k, 0], aux["status"][k, 0], o, room,
                        f"empty cam{k}", pos_tol=1e-13, dir_tol=1e-13)


@pytest.mark.parametrize("axis", [0, 1])
def test_render_jittered_samples(axis):
    """4 stratified samples per pixel (SplitMix64 jitter) and their mean."""
    cams = [W.orbit_camera(0.9, 30.0, 24, 24, spp=4, seed=11),
            W.orbit_camera(2.1, 10.0, 24, 24, spp=4, seed=11)]
    c = W.cloak(axis, height=W.HEIGHT)
    say(f"case render spp4 axis={axis}")
    rgb, aux = gpu_render(c, W.render_opts(), cams, 1)
    room = W.room()
    for k, cam in enumerate(cams):
        o = oracle.render_samples(c, W.opts_dp45(), room, cam, k, 0, np.arange(24 * 24 * 4))
        compare_samples(aux["code"][k, 0], aux["rec"][k, 0], aux["status"][k, 0], o, room,
                        f"spp4 a{axis} cam{k}")
        col, _ = oracle.render_pixels(c, W.opts_dp45(), room, cam, k, 0, np.arange(24 * 24))
        same = (aux["code"][k, 0] == o["code"]).reshape(-1, 4).all(axis=1)
        np.testing.assert_allclose(rgb[k, 0].reshape(-1, 3)[same], col[same], atol=1e-6)
        compare_tof(aux["tof"][k, 0], o, 4)


def test_render_full_size_sampled():
    """The 3-D render workload at full size (both cloaks in one pass, 4
    elevations, 1024 x 1024, both branches) in the launch configuration the
    benchmark times; sampled pixels re-traced by the oracle."""
    import torch
    from paper_1209_6038_amd import rt
    cams = W.render_views(res=1024)
    descs = [W.cloak(a, height=W.HEIGHT) for a in (0, 1)]
    cls = [rt.Cloak(d) for d in descs]
    say("case render full size, both cloaks")
    rgb, aux = rt.render_multi(cls, W.render_opts(), W.room(), cams, 3, aux=True)
    torch.cuda.synchronize()
    aux = {k: v.cpu().numpy() for k, v in aux.items()}
    room = W.room()
    rng = np.random.default_rng(3)
    for ci, c in enumerate(descs):
        for k, cam in enumerate(cams):
            for pi, branch in enumerate((0, 1)):
                st = aux["status"][ci, k, pi]
                hits = np.flatnonzero(st != 1)
                ids = np.unique(np.concatenate([rng.choice(st.size, 64, replace=False),
                                                rng.choice(hits, min(96, hits.size), replace=False)]))
                o = oracle.render_samples(c, W.opts_dp45(), room, cam, k, branch, ids)
                compare_samples(aux["code"][ci, k, pi][ids], aux["rec"][ci, k, pi][:, ids],
                                aux["status"][ci, k, pi][ids], o, room,
                                f"full a{c['axis']} cam{k} b{branch}")


def test_render_multi_equals_single_calls():
    """One pass over both cloaks gives bit-identical images, records and step
    counts to one call per cloak (per-ray work does not depend on batching)."""
    import torch
    from paper_1209_6038_amd import rt
    cams = [W.orbit_camera(0.3, 20.0, 64, 64), W.orbit_camera(2.0, 40.0, 64, 64)]
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    rgb_m, aux_m = rt.render_multi(cls, W.render_opts(), W.room(), cams, 3, aux=True)
    for ci, cl in enumerate(cls):
        rgb_s, aux_s = rt.render(cl, W.render_opts(), W.room(), cams, 3, aux=True)
        torch.cuda.synchronize()
        assert torch.equal(rgb_m[ci], rgb_s)
        for key in ("status", "code", "nsteps"):
            assert torch.equal(aux_m[key][ci], aux_s[key]), key
        assert torch.equal(torch.nan_to_num(aux_m["rec"][ci]), torch.nan_to_num(aux_s["rec"]))
        assert torch.equal(torch.nan_to_num(aux_m["tof"][ci]), torch.nan_to_num(aux_s["tof"]))


def test_render_multi_rejects_mismatched_geometry():
    from paper_1209_6038_amd import rt
    cls = [rt.Cloak(W.cloak(0, height=4.0)), rt.Cloak(W.cloak(1, height=3.0))]
    with pytest.raises(rt.RtError):
        rt.render_multi(cls, W.render_opts(), W.room(), [W.orbit_camera(0.0, 10.0, 8, 8)], 3)


def test_render_in_small_chunks_equals_one_launch():
    """A render split into many chunks (one integrator launch each, chunk
    boundaries inside images and between samples of a pixel's stratum run)
    gives the single-launch render bit for bit."""
    import torch
    from paper_1209_6038_amd import rt
    cams = [W.orbit_camera(0.3, 25.0, 96, 96, spp=4, seed=9), W.orbit_camera(2.0, 40.0, 96, 96, spp=4, seed=9)]
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    say("case chunked render: 2 views x 96^2 x 4 spp, chunks of 5000 samples vs one launch")
    a, aux_a = rt.render_multi(cls, W.render_opts(), W.room(), cams, 3, aux=True)
    b, aux_b = rt.render_multi(cls, W.render_opts(max_chunk=5000), W.room(), cams, 3, aux=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for key in ("status", "code", "nsteps"):
        assert torch.equal(aux_a[key], aux_b[key]), key
    assert torch.equal(torch.nan_to_num(aux_a["tof"]), torch.nan_to_num(aux_b["tof"]))


def test_orbit_frames_full_size_sampled():
    """Two frames of the large-render workload at full size (4096^2 x 4
    jittered spp, both cloaks, both branches) in the launch configuration
    the benchmark times (two frames per integrator launch, the launch shape
    from the autotuner on these frames): per image, 256
    random samples and 256 samples that enter the cloak re-traced by the
    oracle, compared sample by sample as the 1024^2 render is: equal
    statuses, exit rays within the 1e-6 bar (position / R2 and direction),
    colour codes equal except within the propagated error of a tile edge."""
    import torch
    from paper_1209_6038_amd import rt
    frames = W.orbit_frames(36, 4096, 4)[5:7]
    descs = [W.cloak(a, height=W.HEIGHT) for a in (0, 1)]
    cls = [rt.Cloak(d) for d in descs]
    say("case orbit frames 5-6: 4096^2 x 4 spp, 2 cloaks x 2 branches, one launch")
    opts, _ = rt.autotune_render(cls, W.render_opts(max_chunk=2 * 4096 * 4096 * 4), W.room(), frames, 3)
    say(f"launch shape: block {opts['block']}, refill period {opts['refill_period']}")
    _, aux = rt.render_multi(cls, opts, W.room(), frames, 3, aux=("rec", "status", "code"))
    torch.cuda.synchronize()
    room = W.room()
    gen = torch.Generator(device="cpu").manual_seed(5)
    ns = 4096 * 4096 * 4
    for ci, c in enumerate(descs):
        for k, frame in enumerate(frames):
            for pi in range(2):
                st = aux["status"][ci, k, pi]
                hits = torch.nonzero(st != 1).flatten().cpu()
                ids = torch.cat([torch.randint(0, ns, (256,), generator=gen),
                                 hits[torch.randint(0, hits.numel(), (256,), generator=gen)]])
                ids = torch.unique(ids).numpy().astype(np.int64)
                it = torch.from_numpy(ids).cuda()
                g_code = aux["code"][ci, k, pi][it].cpu().numpy()
                g_rec = aux["rec"][ci, k, pi][:, it].cpu().numpy()
                g_st = st[it].cpu().numpy()
                # camera index k within the launch: the jitter is keyed by it
                o = oracle.render_samples(c, W.opts_dp45(), room, frame, k, pi, ids)
                compare_samples(g_code, g_rec, g_st, o, room, f"orbit a{c['axis']} frame{5 + k} b{pi}")


def test_two_large_frames_in_one_launch_equal_one_launch_each():
    """Two 4096^2 x 4 spp frames (2^27 samples) in one integrator launch give
    the same images as one launch per frame: work-table slots past 2^28 and
    the codes of the second frame stay in range, and per-ray work does not
    depend on the batching."""
    import torch
    from paper_1209_6038_amd import rt
    frames = W.orbit_frames(36, 4096, 4)[:2]
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    one = rt.render_multi(cls, W.render_opts(max_chunk=2 * 4096 * 4096 * 4), W.room(), frames, 3)
    each = rt.render_multi(cls, W.render_opts(), W.room(), frames, 3)
    torch.cuda.synchronize()
    say(f"max |difference| {float((one - each).abs().max()):.3e}")
    assert torch.equal(one, each)
    del one, each
    rt.release_workspace()


@pytest.mark.parametrize("spp", [1, 4])
def test_unpolarized_image_parity(spp):
    """Eq. (12) unpolarized images (rt_render_aux.unpol) of both cloaks in one
    rt_render_multi call against the oracle's composition of the two branch
    images with its per-sample weights; the branch images stay as without."""
    import torch
    from paper_1209_6038_amd import rt
    n = 32
    cams = [W.orbit_camera(az, el, n, n, spp=spp, seed=5) for az, el in ((0.0, 0.0), (0.7, 30.0))]
    room = W.room()
    ds = [W.cloak(0, height=W.HEIGHT), W.cloak(1, height=W.HEIGHT)]
    cls = [rt.Cloak(d) for d in ds]
    say(f"case unpolarized spp={spp}")
    rgb, aux = rt.render_multi(cls, W.opts_dp45(), room, cams, 3, unpolarized=True)
    rgb0 = rt.render_multi(cls, W.opts_dp45(), room, cams, 3)
    torch.cuda.synchronize()
    assert torch.equal(rgb, rgb0)
    u = aux["unpol"].cpu().numpy()
    for ci, d in enumerate(ds):
        for k, cam in enumerate(cams):
            o = oracle.render_unpolarized_pixels(d, W.opts_dp45(), room, cam, k, np.arange(n * n))
            err = np.abs(u[ci, k].reshape(-1, 3) - o).max()
            say(f"  cloak {ci} cam {k}: max |unpol - oracle| = {err:.3e}, mean {u[ci, k].mean():.4f}")
            assert err <= 1e-5
    # without a cloak the unpolarized image is the room
    e_rgb, e_aux = rt.render_multi([], W.opts_dp45(), room, cams, 3, unpolarized=True)
    torch.cuda.synchronize()
    assert torch.allclose(e_aux["unpol"][0], e_rgb[0, :, 1], rtol=0, atol=1e-6)
    for c in cls:
        c.close()


def test_renders_on_two_streams_equal_renders_on_one():
    """Direct render calls alternating between two streams (the library then
    uses a workspace per stream and lets them overlap), with traces on a third
    stream in between (ordered after the renders that share their workspace),
    give the images and exits of the same calls issued one after another on
    one stream, bit for bit."""
    import torch
    from paper_1209_6038_amd import rt
    cls = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    groups = [[W.orbit_camera(0.4 * k + 0.1 * j, 10.0 * k, 96, 64, spp=4, seed=k) for j in range(2)]
              for k in range(6)]
    rays = torch.from_numpy(W.random_rays(4096, seed=21, z_range=(-1.0, 5.0))).cuda()
    say("case two streams")

    def run(streams):
        imgs, exits = [], []
        for k, g in enumerate(groups):
            with torch.cuda.stream(streams[k % len(streams)]):
                imgs.append(rt.render_multi(cls, W.render_opts(), room, g, 3))
            if k % 2 == 1:
                with torch.cuda.stream(streams[-1]):
                    exits.append(rt.trace_batch(cls[k % 2], W.opts_dp45(), 1, rays)["out"])
        torch.cuda.synchronize()
        return imgs, exits

    one = torch.cuda.current_stream()
    ref_i, ref_e = run([one])
    alt_i, alt_e = run([one, torch.cuda.Stream(), torch.cuda.Stream()])
    for a, b in zip(ref_i, alt_i):
        assert torch.equal(a, b)
    for a, b in zip(ref_e, alt_e):
        assert torch.equal(a, b)
    for c in cls:
        c.close()
    rt.release_workspace()


@pytest.mark.parametrize("spp", [1, 4])
def test_goggle_image_parity(spp):
    """The images through the in-plane and the axial polarizer
    (rt_render_aux.goggle_inplane / goggle_axial, Figs. 1d,e and 2d,e) of both
    cloaks in one call against the oracle's per-sample goggle weights; the
    branch images and the unpolarized image are those of the call without
    goggles, the two goggles add up to the unpolarized image, and without a
    cloak each goggle sees half of the room."""
    import torch
    from paper_1209_6038_amd import rt
    n = 32
    cams = [W.orbit_camera(az, el, n, n, spp=spp, seed=7) for az, el in ((0.2, 0.0), (1.1, 35.0))]
    room = W.room()
    ds = [W.cloak(0, height=W.HEIGHT), W.cloak(1, height=W.HEIGHT)]
    cls = [rt.Cloak(d) for d in ds]
    say(f"case goggles spp={spp}")
    rgb, aux = rt.render_multi(cls, W.opts_dp45(), room, cams, 3, unpolarized=True, goggles=True)
    rgb0, aux0 = rt.render_multi(cls, W.opts_dp45(), room, cams, 3, unpolarized=True)
    torch.cuda.synchronize()
    assert torch.equal(rgb, rgb0)
    assert torch.equal(aux["unpol"], aux0["unpol"])
    g_in, g_ax = aux["goggle_inplane"], aux["goggle_axial"]
    assert float((g_in + g_ax - aux["unpol"]).abs().max()) <= 1e-6
    for gi, img in enumerate((g_in.cpu().numpy(), g_ax.cpu().numpy())):
        for ci, d in enumerate(ds):
            for k, cam in enumerate(cams):
                o = oracle.render_goggle_pixels(d, W.opts_dp45(), room, cam, k, np.arange(n * n), gi)
                err = np.abs(img[ci, k].reshape(-1, 3) - o).max()
                say(f"  goggle {gi} cloak {ci} cam {k}: max |image - oracle| = {err:.3e}, mean {img[ci, k].mean():.4f}")
                assert err <= 1e-5
    e_rgb, e_aux = rt.render_multi([], W.opts_dp45(), room, cams, 3, goggles=True)
    torch.cuda.synchronize()
    for name in ("goggle_inplane", "goggle_axial"):
        assert torch.allclose(e_aux[name][0], 0.5 * e_rgb[0, :, 1], rtol=0, atol=1e-6)
    for c in cls:
        c.close()


@pytest.mark.parametrize("spp", [1, 4])
def test_first_order_reflection_parity(spp):
    """First-order reflections (rt_render_aux.reflections, Sect. 4) in the
    unpolarized and both goggle images of both cloaks, against the oracle's
    primary images plus its reflection contributions (the entry's reflected
    ray and the two waves reflected at each branch's exit, followed to their
    own exits); the branch images stay as without; the goggles still add up
    to the unpolarized image; chunking does not change the images."""
    import torch
    from paper_1209_6038_amd import rt
    n = 24
    cams = [W.orbit_camera(az, el, n, n, spp=spp, seed=9) for az, el in ((0.2, 0.0), (1.1, 35.0))]
    room = W.room()
    ds = [W.cloak(0, height=W.HEIGHT), W.cloak(1, height=W.HEIGHT)]
    cls = [rt.Cloak(d) for d in ds]
    say(f"case reflections spp={spp}")
    kw = {"unpolarized": True, "goggles": True}
    rgb, aux = rt.render_multi(cls, W.opts_dp45(), room, cams, 3, reflections=True, **kw)
    rgb0, aux0 = rt.render_multi(cls, W.opts_dp45(), room, cams, 3, **kw)
    rgb1, aux1 = rt.render_multi(cls, W.opts_dp45(max_chunk=n * n * spp // 3 // spp * spp), room, cams, 3,
                                 reflections=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(rgb, rgb0)
    added = aux["unpol"] - aux0["unpol"]
    say(f"  reflections add mean {float(added.mean()):.4e}, max {float(added.max()):.4e}")
    assert float(added.min()) >= -1e-6 and float(added.max()) > 1e-3
    for name in ("unpol", "goggle_inplane", "goggle_axial"):
        assert torch.equal(aux[name], aux1[name]), name
    assert float((aux["goggle_inplane"] + aux["goggle_axial"] - aux["unpol"]).abs().max()) <= 1e-6
    for gi, name in ((-1, "unpol"), (0, "goggle_inplane"), (1, "goggle_axial")):
        img = aux[name].cpu().numpy()
        for ci, d in enumerate(ds):
            for k, cam in enumerate(cams):
                px = np.arange(n * n)
                base = (oracle.render_unpolarized_pixels(d, W.opts_dp45(), room, cam, k, px) if gi < 0 else
                        oracle.render_goggle_pixels(d, W.opts_dp45(), room, cam, k, px, gi))
                ref = base + oracle.render_reflection_pixels(d, W.opts_dp45(), room, cam, k, px, gi)
                err = np.abs(img[ci, k].reshape(-1, 3) - ref).max()
                say(f"  {name} cloak {ci} cam {k}: max |image - oracle| = {err:.3e}")
                assert err <= 1e-5
    for c in cls:
        c.close()


def test_unpolarized_image_needs_both_branches_and_fp64():
    from paper_1209_6038_amd import rt
    cam = W.orbit_camera(0.0, 0.0, 8, 8)
    cl = rt.Cloak(W.cloak(0, height=W.HEIGHT))
    for pol_mask, op in ((1, W.opts_dp45()),):
        for kw in ({"unpolarized": True}, {"goggles": True}):
            with pytest.raises(rt.RtError) as e:
                rt.render_multi([cl], op, W.room(), [cam], pol_mask, **kw)
            assert e.value.code == rt.RT_E_UNSUPPORTED
    cl.close()
