#!/usr/bin/env python3
"""Benchmark of the cloak ray tracer on one MI355X.

Workload (one step): the photorealistic-render workload -- radial and
azimuthal uniaxial cloaks (R1 = 1, R2 = 2, height 4) in the checkerboard room
[-10,10]^2 x [0,10] (0.5 tiles), pinhole camera at distance 8 from (0,0,2),
60 deg field of view, elevations 0/15/30/45 deg, 1024 x 1024 pixels,
ordinary and extraordinary branch traced separately, Dormand-Prince 5(4) at
tolerance 1e-8. One step renders both cloaks (16.8 M camera rays, one
integrator launch), with the integrator's launch shape (block size, refill
period) chosen by rt_autotune_render on the batch beforehand (--block /
--refill fix it instead). The batch is recorded into --streams render plans (default 3; the GPU
runs 4 hardware queues, and a fourth stream can share one)
(rt_render_plan_*, each with its own workspace and output images), and step k
replays plan k mod S on stream k mod S: consecutive steps overlap, so one
step's last rays and small kernels share the chip with the next step's bulk.
The integrator's launch time for the roofline is measured on eager,
one-at-a-time launches of the same batch (HIP events on the launch stream).

Metric: Mrays/s traced through the cloak = rays that enter the cloak material
per second of step time (all camera rays per second are reported too).

--workload batched times the batched workload instead: 64 seeded views
(azimuth U[0, 2 pi), elevation U[0, 60] deg) at 512 x 512, both cloaks, both
branches, replayed from render plans in the same way, with the integrator's
launch shape chosen by rt_autotune_render.

Surrogate leg (the "surrogate vs plain speedup at 1e-3" half of the metric,
skipped with --no-surrogate): 10 M seeded entries on the outer cylinder of the
infinite radial and azimuthal cloaks (both branches) are labelled by the exact
transit (DP45 1e-8, FP64) and train the BF16 MFMA surrogate (residuals on the
closed-form transits); a trust map is calibrated at half the 1e-3 exit-error
tolerance on 3 M separate entries; then 1 M held-out entries are traced by the
plain exact transit and by surrogate + exact fallback (both timed with HIP
events, inputs resident), and the accepted predictions' exit errors are
measured against the exact exits. Last, four frames of the large render are
timed plain and with the surrogate (rt_render_surrogate) for several
difficulty thresholds, with the image difference.

Prints one JSON line. --gpus N with N > 1 exits: the implementation runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix (MFMA)
# surrogate MLP per ray: MFMA flops of the three 256 x 256 layers
MLP_MFMA_FLOPS = 2 * 3 * 256 * 256
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 with packed instructions

# Algorithmic flops (FMA = 2; add, mul, div, sqrt, rcp = 1) of one evaluation
# of dv/dt (Eq. (8), reduced cylindrical form, radial terms reduced with
# 1 - s = a w (1 + q)) per branch kind (radial-o, radial-e, azimuthal-o,
# azimuthal-e).
ACCEL_FLOPS = {0: 0, 1: 35, 2: 37, 3: 31}
# One Dormand-Prince 5(4) attempt on the 6-component state: stage inputs
# (20 non-zero a_sj per component, 2 flops each, + 2 per stage) 312, embedded
# error 78, scaled RMS norm 42, controller 5.
DP45_COMBINE_FLOPS = 312 + 78 + 42 + 5
DP45_STAGES = 6
# RK4: stage inputs 3 x 6 FMA + 3, final combination 6 x 8.
RK4_COMBINE_FLOPS = 75 + 48
RK4_STAGES = 4
# The Hamiltonian form (scheme 2): one evaluation of (dx/dtau, dk/dtau,
# dt/dtau) in the reduced cylindrical form per branch kind, and the RK4
# combination of the 7-component state (x, k, t).
HAM_RHS_FLOPS = {0: 3, 1: 48, 2: 18, 3: 51}
HAM_COMBINE_FLOPS = 78


def attempt_flops(kind: int, scheme: int) -> int:
    if scheme == 1:
        return DP45_COMBINE_FLOPS + DP45_STAGES * ACCEL_FLOPS[kind]
    return RK4_COMBINE_FLOPS + RK4_STAGES * ACCEL_FLOPS[kind]


# Hamiltonian drift |v^T M v - 1| above which an exact exit is taken as not
# resolved by the integrator (the surrogate is then judged elsewhere)
UNRESOLVED = 1e-6

# HBM traffic of one integrator launch from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) of this benchmark, scaled by the same counters on a
# plain device copy of known size (bench.py --copy-probe). Valid only for the
# integrator source it was measured on; reported as null otherwise. Keyed by
# the launch shape (block, refill period) of the measured run: the figure moves
# by about 1% between shapes, and the one nearest the run's shape is reported
# together with the shape it was taken at.
TRAFFIC = {"source_sha256": "d163277e576ce36582d5f0afd8748092ebcd51e73416e61189a8948ef1517944",
           "bytes_per_launch": {(256, 2): 783520288, (256, 4): 785148896, (256, 8): 794267648,
                                (128, 4): 769098592, (128, 8): 777473856}}


def traffic_for(block, refill):
    """(bytes per integrator launch, shape it was measured at) or (None, None)."""
    if TRAFFIC["source_sha256"] != integrator_source_hash():
        return None, None
    shapes = TRAFFIC["bytes_per_launch"]
    key = min(shapes, key=lambda k: (k[0] != block, abs(k[1] - refill)))
    return shapes[key], list(key)


def finite_json(obj):
    """obj with non-finite floats replaced by None (strict JSON)."""
    if isinstance(obj, float):
        return obj if math.isfinite(obj) else None
    if isinstance(obj, dict):
        return {k: finite_json(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [finite_json(v) for v in obj]
    return obj


def integrator_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in ("paper_1209_6038_amd/csrc/rt_cloak.hip", "paper_1209_6038_amd/csrc/device.h"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def copy_probe(nbytes: int = 1 << 30) -> None:
    """One plain device-to-device copy of nbytes (for counter calibration)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(finite_json({"copy_probe_bytes": nbytes})), flush=True)


def cpu_baseline(opts, cams, stride, entered_only=True):
    """Time the oracle on every `stride`-th pixel of every image."""
    import numpy as np

    import oracle
    from paper_1209_6038_amd import workloads as W
    room = W.room()
    n_entered = 0
    n_rays = 0
    t0 = time.perf_counter()
    for axis in (0, 1):
        c = W.cloak(axis, height=W.HEIGHT)
        for k, cam in enumerate(cams):
            ids = np.arange(0, cam["w"] * cam["h"], stride, dtype=np.int64)
            for branch in (0, 1):
                r = oracle.render_samples(c, opts, room, cam, k, branch, ids)
                n_entered += int(np.isin(r["status"], (0, 2, 3, 4, 5)).sum())
                n_rays += len(ids)
    dt = time.perf_counter() - t0
    return {"value": n_entered / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"every {stride}th pixel of the 16 images ({n_rays} camera rays, "
                      f"{n_entered} entering the cloak), FP64 C oracle with OpenMP, {dt:.1f} s",
            "all_rays_per_s": n_rays / dt}


def mixed_precision_leg(cloaks, room, cams, ms_fp64, out, opts, steps: int = 10):
    """The same render with the derivative of Eq. (8) evaluated in FP32 away
    from the inner radius (FP64 within 0.05 of r = a, and for every event and
    refraction): time per step and the exit error of each sample against the
    FP64 render, stated as it is (it does not meet the 1e-6 bar)."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    om = dict(opts, precision=1)  # the FP64 run's launch shape
    rgb_f, aux_f = rt.render_multi(cloaks, opts, room, cams, 3, aux=True)
    rgb_m, aux_m = rt.render_multi(cloaks, om, room, cams, 3, aux=True)
    torch.cuda.synchronize()
    both = (aux_f["status"] == 0) & (aux_m["status"] == 0)
    rf = aux_f["rec"].transpose(3, 4)[both]
    rm = aux_m["rec"].transpose(3, 4)[both]
    dpos = (rf[:, :3] - rm[:, :3]).norm(dim=1) / W.R2
    cosang = (rf[:, 3:6] * rm[:, 3:6]).sum(dim=1).clamp(-1.0, 1.0)
    sinang = torch.cross(rf[:, 3:6], rm[:, 3:6], dim=1).norm(dim=1)
    err = torch.maximum(dpos, torch.atan2(sinang, cosang))
    q = torch.quantile(err.float()[:: max(1, err.numel() // 4_000_000)], torch.tensor([0.5, 0.99], device=err.device))
    stat_mismatch = int((aux_f["status"] != aux_m["status"]).sum())
    code_diff = float((aux_f["code"] != aux_m["code"]).float().mean())
    d = (rgb_m - rgb_f).abs().amax(dim=-1)
    over = float((d > 1.0 / 255.0).float().mean())
    n_both = int(both.sum())
    over_bar = float((err > 1e-6).float().mean())
    emax = float(err.max())
    del aux_f, aux_m, rf, rm, dpos, err, rgb_f, rgb_m
    for _ in range(2):
        rt.render_multi(cloaks, om, room, cams, 3, out=out)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        rt.render_multi(cloaks, om, room, cams, 3, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {
        "note": ("dv/dt of Eq. (8) in FP32 outside r < r1 + 0.05, FP64 there and for events and refraction; "
                 "exit error of each sample against the FP64 render (both exited)"),
        "ms_per_step": round(ms, 4), "speedup_vs_fp64": round(ms_fp64 / ms, 3),
        "exit_error_vs_fp64": {"n": n_both, "p50": float(f"{float(q[0]):.3e}"), "p99": float(f"{float(q[1]):.3e}"),
                               "max": float(f"{emax:.3e}"), "fraction_over_1e-6": float(f"{over_bar:.3e}")},
        "status_mismatches": stat_mismatch, "colour_code_differences": float(f"{code_diff:.3e}"),
        "pixels_over_1_255": float(f"{over:.3e}"),
    }


def surrogate_render_leg(model, log, n_frames: int = 4, fpl: int = 2, difficulties=(0, 2, 3, 4)):
    """The large render (4096^2 px x 4 jittered spp, radial + azimuthal
    cloaks, both branches) of n_frames frames of the 36-frame orbit at 30 deg,
    fpl frames per launch, plain (rt_render_multi) and with the surrogate
    (rt_render_surrogate) for each threshold of difficulty (side entries of
    at least that difficulty bucket go to the network): time per frame, share
    of the offered side entries the gate accepts, and the image difference."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    frames = W.orbit_frames(36, 4096, 4)[:: 36 // n_frames][:n_frames]
    groups = [frames[i:i + fpl] for i in range(0, len(frames), fpl)]
    opts = W.render_opts(max_chunk=fpl * 4096 * 4096 * 4)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    dev = torch.device("cuda", 0)
    out_p = torch.empty((len(groups), 2, fpl, 2, 4096, 4096, 3), dtype=torch.float32, device=dev)
    out_s = torch.empty_like(out_p)

    def timed(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for k, g in enumerate(groups):
            fn(k, g)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / len(frames)

    def plain(k, g):
        rt.render_multi(cloaks, opts, room, g, 3, out=out_p[k, :, :len(g)])

    for k, g in enumerate(groups):  # warm-up
        plain(k, g)
    ms_p = timed(plain)
    sweep = []
    for dmin in difficulties:
        offered = accepted = 0
        for k, g in enumerate(groups):  # untimed pass: counts
            _, (c0, c1) = rt.render_surrogate(model, cloaks, opts, room, g, 3, out=out_s[k, :, :len(g)],
                                              counts=True, min_difficulty=dmin)
            offered += c0
            accepted += c1
        torch.cuda.synchronize()
        d = (out_s - out_p).abs().amax(dim=-1)
        over = float((d > 1.0 / 255.0).float().mean())
        dmax = float(d.max())
        del d
        ms_s = timed(lambda k, g: rt.render_surrogate(model, cloaks, opts, room, g, 3, out=out_s[k, :, :len(g)],
                                                      min_difficulty=dmin))
        log(f"surrogate render, min difficulty {dmin}: {ms_s:.1f} ms/frame (plain {ms_p:.1f}), "
            f"accepted {accepted}/{offered} offered side entries, pixels over 1/255: {over:.2e}")
        sweep.append({"min_difficulty": dmin, "surrogate_ms_per_frame": round(ms_s, 2),
                      "speedup": round(ms_p / ms_s, 3), "offered_per_frame": offered // len(frames),
                      "accepted_per_frame": accepted // len(frames),
                      "pixels_over_1_255": over, "max_pixel_difference": round(dmax, 4)})
    del out_p, out_s
    best = max(sweep, key=lambda r: r["speedup"])
    return {
        "workload": (f"{len(frames)} frames of the 36-frame orbit at 30 deg elevation, 4096^2 px x 4 jittered spp, "
                     f"radial + azimuthal cloaks (height 4), ordinary + extraordinary, {fpl} frames per launch"),
        "plain_ms_per_frame": round(ms_p, 2), "speedup": best["speedup"], "best": best, "sweep": sweep,
    }


def surrogate_leg(steps: int, n_train: int, log, fpl: int = 2):
    """Train, calibrate and time the transit surrogate (see the module doc)."""
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S

    def sync():
        torch.cuda.synchronize()

    cl = S.make_cloaks(None)
    op = S.exact_opts()
    x_tr = S.features(n_train, 1001)
    sync()
    t0 = time.perf_counter()
    _, _, t_tr, w_tr = S.label(cl, x_tr, op)
    sync()
    t_label = time.perf_counter() - t0
    m = rt.Surrogate(seed=0)
    m.fit_scaling(x_tr, t_tr, w_tr)
    batch = 65536
    t0 = time.perf_counter()
    loss = S.train(m, x_tr, t_tr, w_tr, steps=steps, batch=batch, lr=2e-3, lr_end=2e-5, huber=0.01)
    sync()
    t_train = time.perf_counter() - t0
    log(f"surrogate: labelled {n_train} in {t_label:.2f} s, trained {steps} steps in {t_train:.1f} s "
        f"(loss {loss:.2e})")
    del x_tr, t_tr, w_tr
    x_cal = S.features(3_000_000, 2002)
    y_cal, st_cal, h_cal = rt.transit_exact(cl, op, x_cal, hres=True)
    tol = 1e-3
    # cells are judged on their calibration rays: calibrate at half the
    # target, distrusting the neighbours of failing cells; exits the
    # integrator did not resolve (Hamiltonian drift > UNRESOLVED) are no
    # reference
    trusted = m.calibrate(cl, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=16, dilate=1,
                          hres_exact=h_cal, unresolved=UNRESOLVED)
    del x_cal, y_cal, st_cal, h_cal
    n = 1_000_000
    x_ev = S.features(n, 3003)
    y_ex, st_ex, h_ex = rt.transit_exact(cl, op, x_ev, hres=True)
    y_s, st_s, fb = m.infer(cl, op, x_ev)
    sync()
    resolved = (st_ex == 0) & (h_ex <= UNRESOLVED)
    acc_all = fb == 0
    acc = acc_all & resolved
    err, operr = S.exit_error(y_s, y_ex)
    e = S.summarize_errors(err, acc)
    # a totally reflected exit of a side entry into the infinite cylinder is
    # drift at a grazing entry (the tangential wave numbers are conserved):
    # no reference either
    unres = acc_all & ~resolved & ((st_ex == 0) | (st_ex == 5))
    ux = unres & (st_ex == 0)
    unres_max = float(err[ux].max()) if bool(ux.any()) else 0.0
    kind = (x_ev[5] * 2 + x_ev[4]).long()

    def timed(fn, reps=5):
        for _ in range(2):
            fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        sync()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        sync()
        return a.elapsed_time(b) / reps

    # the same gate with the network's output zeroed: the closed-form
    # baselines alone, for comparison
    base = rt.Surrogate(seed=0)
    base.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    sc = m.get_scaling()
    sc[12:22] = np.concatenate([np.zeros(5, np.float32), np.ones(5, np.float32)])
    base.set_scaling(sc)
    base.calibrate(cl, x_ev, y_ex, st_ex, tol=1e30, min_count=1)
    y_b, _, fb_b = base.infer(cl, op, x_ev)
    err_b, _ = S.exit_error(y_b, y_ex)
    sel_b = (fb_b == 0) & resolved
    e_base = S.summarize_errors(err_b, sel_b)
    e_net = S.summarize_errors(err, sel_b & (fb == 0))
    del y_b, fb_b, err_b
    # the plain transit's launch is set by its longest rays (near-singular
    # entries with p_theta -> 0 take thousands of steps): also time it
    # without the 0.1 % of rays with the most steps
    _, _, ns = rt.transit_exact(cl, op, x_ev, nsteps=True)
    bulk = torch.ones(n, dtype=torch.uint8, device=x_ev.device)
    bulk[torch.argsort(ns, descending=True)[: n // 1000]] = 0
    ms_plain_bulk = timed(lambda: rt.transit_exact(cl, op, x_ev, mask=bulk, y5=y_ex, status=st_ex))
    ms_plain = timed(lambda: rt.transit_exact(cl, op, x_ev, y5=y_ex, status=st_ex))
    ms_sur = timed(lambda: m.infer(cl, op, x_ev, y5=y_s, fallback=fb, status=st_s))
    ms_fwd = timed(lambda: m.forward(x_ev))
    mlp_tflops = MLP_MFMA_FLOPS * n / (ms_fwd * 1e-3) / 1e12
    rec = {
        "speedup": round(ms_plain / ms_sur, 3),
        "plain_Mrays_s": round(n / (ms_plain * 1e-3) / 1e6, 2),
        "surrogate_Mrays_s": round(n / (ms_sur * 1e-3) / 1e6, 2),
        "tolerance": tol,
        "accepted_fraction": round(acc_all.float().mean().item(), 4),
        "accepted_by_branch": {name: round(acc_all[kind == k].float().mean().item(), 4)
                               for k, name in enumerate(("radial_o", "radial_e", "azimuthal_o",
                                                         "azimuthal_e"))},
        "trusted_cells": round(trusted, 4),
        "accepted_exit_error": {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in e.items()},
        "accepted_over_tolerance": int((err[acc] > tol).sum()),
        "accepted_not_left_in_reference": int((acc_all & (st_ex != 0) & (st_ex != 5)).sum()),
        "reference": (f"exact transit where it resolves the path (|H - 1| <= {UNRESOLVED:g} at the exit, "
                      "not totally reflected)"),
        "accepted_with_unresolved_reference": {
            "n": int(unres.sum()), "totally_reflected": int((unres & (st_ex == 5)).sum()),
            "max_difference_of_exited": float(f"{unres_max:.3e}")},
        "accepted_opl_rel_error_p99": float(f"{S.summarize_errors(operr, acc).get('p99', 0.0):.3e}"),
        "network_vs_closed_form": {
            "note": "exit error vs the exact transit on the rays both accept: baselines + network, baselines alone",
            "with_network": {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in e_net.items()},
            "closed_form_only": {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in e_base.items()}},
        "plain_steps": {"max": int(ns.max()), "mean": round(float(ns.double().mean()), 1),
                        "ms_all": round(ms_plain, 3), "ms_without_longest_0.1pct": round(ms_plain_bulk, 3)},
        "workload": ("1 M held-out entries (phi U[0,2pi), z U[0,4], alpha, beta U(-pi/2,pi/2), branch and "
                     "axis bits uniform) on r = 2 of the infinite radial and azimuthal cloaks, DP45 1e-8 FP64 "
                     "exact transit vs MLP 6-256x4-5 (BF16 MFMA) + gate + exact fallback"),
        "train": {"rays": n_train, "steps": steps, "batch": batch, "seconds": round(t_train, 2),
                  "samples_per_s_M": round(steps * batch / t_train / 1e6, 2), "final_loss": float(f"{loss:.3e}"),
                  "label_seconds": round(t_label, 2)},
        "mlp_roofline": {"bound": "mfma", "kernel": "k_mlp_fused", "achieved": round(mlp_tflops, 1),
                         "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(mlp_tflops / PEAK_BF16_TFLOPS, 4), "ms_per_1M_rays": round(ms_fwd, 4)},
    }
    del x_ev, y_ex, st_ex, h_ex, y_s, st_s, fb, err, operr
    rec["render"] = surrogate_render_leg(m, log, fpl=fpl)
    return rec


# MFMA flops of one training sample: the forward products of the three
# 256 x 256 layers, and in backward the data gradient through them and the
# weight gradient of each (the 6 -> 256 and 256 -> 5 layers run in FP32 on
# the vector units and are not counted)
TRAIN_MFMA_FLOPS = 3 * MLP_MFMA_FLOPS


def train_workload(args):
    """Surrogate training alone: AdamW steps of 65,536 rows (BF16 MFMA forward
    and backward, FP32 master weights) over the 10 M labelled entries of the
    surrogate leg, timed with HIP events on the launch stream, inputs
    resident."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S

    cl = S.make_cloaks(None)
    x_tr = S.features(args.surrogate_train, 1001)
    _, _, t_tr, w_tr = S.label(cl, x_tr, S.exact_opts())
    m = rt.Surrogate(seed=0)
    m.fit_scaling(x_tr, t_tr, w_tr)
    batch = 65536
    nb = x_tr.shape[1] // batch
    steps = args.surrogate_steps
    loss = torch.zeros(1, dtype=torch.float32, device=x_tr.device)

    def run(k0, k1):
        for k in range(k0, k1):
            j = (k % nb) * batch
            m.train_step(x_tr[:, j:j + batch], t_tr[:, j:j + batch], w_tr[j:j + batch], lr=1e-3,
                         huber=0.01, loss=loss)

    run(0, 20)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    run(20, 20 + steps)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    tflops = TRAIN_MFMA_FLOPS * batch / (ms * 1e-3) / 1e12
    return {"metric": "surrogate training samples/s", "unit": "M samples/s",
            "value": round(batch / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4), "steps": steps,
            "dtype": "bf16 x bf16 -> f32 (layers 2-4), f32 (layers 1, 5)", "data": "synthetic",
            "config": {"workload": "surrogate training: AdamW steps of 65,536 rows of the 10 M labelled "
                                   "entries, MLP 6-256x4-5", "final_loss": float(loss.item())},
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": PEAK_BF16_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / PEAK_BF16_TFLOPS, 4),
                         "note": "MFMA flops of forward and backward per sample x batch / step time"}}


def inplane_workload(args):
    """The 2-D workload: radial cloak, extraordinary branch, 16,384 parallel
    in-plane rays (impact parameters on the midpoint grid of [-3, 3]) at each
    of 8 incidence angles, RK4 h = 1e-3 (the paper's fixed-step scheme),
    FP64, exits reported at r = 3. One step = one rt_trace_batch call."""
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    rays = torch.from_numpy(W.inplane_bundle(16384, 8)).cuda()
    opts = W.opts_rk4(1e-3)
    cl = rt.Cloak(W.cloak(W.RADIAL))
    r = rt.trace_batch(cl, opts, W.EXTRAORDINARY, rays)
    torch.cuda.synchronize()
    st = r["status"].cpu().numpy()
    entered = int((st != 1).sum())
    attempts = int(r["nsteps"].cpu().numpy().astype(np.int64).sum())
    for _ in range(args.warmup):
        rt.trace_batch(cl, opts, W.EXTRAORDINARY, rays, with_aux=False)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    rt.profile_enable(True)
    rt.profile_read()
    a.record()
    for _ in range(args.steps):
        rt.trace_batch(cl, opts, W.EXTRAORDINARY, rays, with_aux=False)
    b.record()
    torch.cuda.synchronize()
    transit_ms, launches = rt.profile_read()
    rt.profile_enable(False)
    ms = a.elapsed_time(b) / args.steps
    launch_ms = transit_ms / max(1, launches)
    flops = attempts * attempt_flops(1, 0)
    achieved = flops / (launch_ms * 1e-3) / 1e12
    return {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error", "unit": "Mrays/s",
        "value": round(entered / (ms * 1e-3) / 1e6, 3), "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2-D in-plane: radial cloak, extraordinary branch, 16384 rays x 8 angles, "
                               "RK4 h=1e-3, FP64, exits at r=3",
                   "rays": int(rays.shape[1]), "entering": entered, "rk4_steps": attempts},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "k_transit (integrator)", "avg_launch_ms": round(launch_ms, 4)},
    }


def hamiltonian_workload(args):
    """The comparison of Sect. 4: the ray equation Eq. (8) with fixed RK4
    steps in the optical path t against the Hamiltonian form (state (x, k),
    H = k^T eps k - eps_o eps_e, fixed RK4 steps in the ray parameter tau),
    on rays for which perfect cloaking is expected: the in-plane workload's
    extraordinary rays through the radial cloak (16,384 impact parameters x 8
    angles), whose exact exit is the incident line continued (CF1). Two sets
    of entering rays: impact parameter 0.3 <= |p| < 1.999 ("wide"), and
    1e-3 <= |p| < 0.3 ("near axis"; closer in, both forms stall). For each
    form and set, a sweep of step sizes gives the largest exit error
    (position / R2 and direction; a ray that does not exit counts as
    infinite) and the time per rt_trace_batch call on that set (HIP events);
    the forms are compared at the largest step that meets 1e-8."""
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    bundle = W.inplane_bundle(16384, 8)
    pb = bundle[0] * (-bundle[4]) + bundle[1] * bundle[3]
    sets = {"wide": (np.abs(pb) >= 0.3) & (np.abs(pb) < 1.999),
            "near_axis": (np.abs(pb) >= 1e-3) & (np.abs(pb) < 0.3)}
    cl = rt.Cloak(W.cloak(W.RADIAL))
    target = 1e-8

    def sweep(make, steps, sel):
        rays_np = np.ascontiguousarray(bundle[:, sel])
        rays = torch.from_numpy(rays_np).cuda()
        o, d, p = rays_np[:3], rays_np[3:], pb[sel]
        want = o + 2.0 * np.sqrt(9.0 - p ** 2) * d
        rows = []
        for h in steps:
            opts = make(h)
            r = rt.trace_batch(cl, opts, W.EXTRAORDINARY, rays)
            torch.cuda.synchronize()
            st = r["status"].cpu().numpy()
            out = r["out"].cpu().numpy()
            err = np.maximum(np.linalg.norm(out[:3] - want, axis=0) / W.R2, np.linalg.norm(out[3:] - d, axis=0))
            err = np.where(st == 0, err, np.inf)
            ns = r["nsteps"].cpu().numpy().astype(np.int64)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            rt.profile_enable(True)
            rt.profile_read()
            a.record()
            for _ in range(3):
                rt.trace_batch(cl, opts, W.EXTRAORDINARY, rays, with_aux=False)
            b.record()
            torch.cuda.synchronize()
            transit_ms, launches = rt.profile_read()
            rt.profile_enable(False)
            launch_ms = transit_ms / max(1, launches)
            per_step = (HAM_COMBINE_FLOPS + 4 * HAM_RHS_FLOPS[1] if opts["scheme"] == 2
                        else attempt_flops(1, 0))
            tflops = float(ns.sum()) * per_step / (launch_ms * 1e-3) / 1e12
            rows.append({"step": h, "ms_per_call": round(a.elapsed_time(b) / 3, 4),
                         "integrator_launch_ms": round(launch_ms, 4),
                         "integrator_fp64_frac": round(tflops / PEAK_FP64_TFLOPS, 4),
                         "steps_per_ray": round(float(ns.mean()), 1), "max_steps_of_a_ray": int(ns.max()),
                         "max_exit_err": float(f"{err.max():.3e}"), "not_exited": int((st != 0).sum())})
        return rows

    res = {}
    for name, sel in sets.items():
        eq8 = sweep(lambda h: W.opts_rk4(h, max_steps=200_000), (4e-3, 2e-3, 1e-3, 5e-4, 2.5e-4), sel)
        ham = sweep(lambda h: W.opts_rk4_ham(h, max_steps=200_000), (1.6e-2, 8e-3, 4e-3, 2e-3, 1e-3), sel)
        ok_e = [r for r in eq8 if r["max_exit_err"] <= target]
        ok_h = [r for r in ham if r["max_exit_err"] <= target]
        e = max(ok_e, key=lambda r: r["step"]) if ok_e else None
        h = max(ok_h, key=lambda r: r["step"]) if ok_h else None
        res[name] = {"rays": int(sel.sum()), "eq8_rk4_in_t": eq8, "hamiltonian_rk4_in_tau": ham,
                     "at_target": {"eq8": e and {"step": e["step"], "ms_per_call": e["ms_per_call"]},
                                   "hamiltonian": h and {"step": h["step"], "ms_per_call": h["ms_per_call"]},
                                   "time_ratio_hamiltonian_over_eq8": (round(h["ms_per_call"] / e["ms_per_call"], 3)
                                                                       if e and h else None)}}
    return {"config": {"workload": "Sect. 4 comparison: Eq. (8) vs the Hamiltonian form, fixed-step RK4, "
                                   "in-plane radial cloak, extraordinary rays, exact exit = incident line (CF1), "
                                   "FP64", "target_exit_error": target, "max_steps": 200_000},
            **res}


def weights_workload(args):
    """Eq. (12) weights: 2^20 random 3-D rays (uniform over azimuth, height
    [-1, 5], in-plane angle and elevation within 60 deg, starting on r = 3)
    against the finite radial and azimuthal cloaks, each traced in both
    branches, DP45 at 1e-8, FP64: one step = four rt_trace_batch calls with
    the weights; the same four calls without them are timed beside."""
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    n = 1 << 20
    rays = torch.from_numpy(W.random_rays(n, seed=11, z_range=(-1.0, 5.0))).cuda()
    opts = W.opts_dp45()
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (W.RADIAL, W.AZIMUTHAL)]
    cases = [(ax, br) for ax in (0, 1) for br in (0, 1)]
    entered, flops, summary = 0, 0, {}
    for ax, br in cases:
        r = rt.trace_batch(cloaks[ax], opts, br, rays, with_trans=True)
        torch.cuda.synchronize()
        st = r["status"].cpu().numpy()
        w = r["trans"].cpu().numpy()
        entered += int((st != 1).sum())
        flops += int(r["nsteps"].cpu().numpy().astype(np.int64).sum()) * attempt_flops(2 * ax + br, 1)
        ex = st == 0
        summary[f"{'radial' if ax == 0 else 'azimuthal'}_{'o' if br == 0 else 'e'}"] = {
            "exited": int(ex.sum()), "mean_weight_exited": round(float(w[ex].mean()), 5),
            "entering_intensity_delivered": round(float(w[ex].sum() / max(1, (st != 1).sum())), 5)}

    def run(trans, steps):
        for _ in range(steps):
            for ax, br in cases:
                rt.trace_batch(cloaks[ax], opts, br, rays, with_aux=False, with_trans=trans)

    timing = {}
    for trans in (False, True):
        run(trans, args.warmup)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        rt.profile_enable(True)
        rt.profile_read()
        a.record()
        run(trans, args.steps)
        b.record()
        torch.cuda.synchronize()
        transit_ms, launches = rt.profile_read()
        rt.profile_enable(False)
        timing[trans] = (a.elapsed_time(b) / args.steps, transit_ms / max(1, launches))
    ms, launch_ms = timing[True]
    achieved = flops / len(cases) / (launch_ms * 1e-3) / 1e12
    return {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error, with Eq. (12) weights",
        "unit": "Mrays/s", "value": round(entered / (ms * 1e-3) / 1e6, 3), "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D random rays with Eq. (12) weights: 2^20 rays from r=3 (z in [-1,5], "
                               "elevation <= 60 deg), radial + azimuthal cloaks (height 4), ordinary + "
                               "extraordinary, DP45 tol 1e-8, FP64",
                   "entering_per_step": entered, "ms_per_step_without_weights": round(timing[False][0], 4),
                   "weights_cost": round(ms / timing[False][0], 4), "per_branch": summary},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "k_transit (integrator, weighted)", "avg_launch_ms": round(launch_ms, 4),
                     "avg_launch_ms_without_weights": round(timing[False][1], 4),
                     "note": "integration flops only; the Fresnel solves at the events are not counted"},
    }


def unpolarized_workload(args):
    """The headline render (both cloaks, 4 views of 1024^2, both branches,
    DP45 1e-8, FP64) with the Eq. (12) unpolarized images, timed beside the
    same render without them; one step = one rt_render_multi call."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    cams = W.render_views(res=args.res)
    opts = W.render_opts(block=args.block, refill_period=args.refill)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    _, aux = rt.render_multi(cloaks, opts, room, cams, 3, aux=True, unpolarized=True)
    torch.cuda.synchronize()
    dev = aux["status"].device
    entered = int(torch.isin(aux["status"], torch.tensor([0, 2, 3, 4, 5], device=dev, dtype=torch.int32)).sum())
    mean_unpol = float(aux["unpol"].mean())
    del aux
    timing = {}
    for unpol in (False, True):
        for _ in range(args.warmup):
            rt.render_multi(cloaks, opts, room, cams, 3, unpolarized=unpol)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        rt.profile_enable(True)
        rt.profile_read()
        a.record()
        for _ in range(args.steps):
            rt.render_multi(cloaks, opts, room, cams, 3, unpolarized=unpol)
        b.record()
        torch.cuda.synchronize()
        transit_ms, launches = rt.profile_read()
        rt.profile_enable(False)
        timing[unpol] = (a.elapsed_time(b) / args.steps, transit_ms / max(1, launches))
    ms, launch_ms = timing[True]
    return {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error, with Eq. (12) unpolarized images",
        "unit": "Mrays/s", "value": round(entered / (ms * 1e-3) / 1e6, 3), "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D render with unpolarized images: radial + azimuthal cloaks (height 4), "
                               "4 elevations x 1024^2 px, ordinary + extraordinary, DP45 tol 1e-8, FP64, "
                               "eager calls",
                   "entering_per_step": entered, "ms_per_step_without_images": round(timing[False][0], 4),
                   "images_cost": round(ms / timing[False][0], 4), "mean_unpolarized_value": round(mean_unpol, 5)},
        "roofline": {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": None, "traffic": None, "kernel": "k_transit (integrator, weighted)",
                     "avg_launch_ms": round(launch_ms, 4),
                     "avg_launch_ms_without_images": round(timing[False][1], 4)},
    }


def orbit_workload(args):
    """The large-render workload timed plain: 36-frame orbit at 30 deg
    elevation, 4096 x 4096 px, 4 jittered samples per pixel, radial and
    azimuthal cloaks, both branches; `frames_per_launch` frames per
    rt_render_multi call, one integrator launch each (a launch lasts at least
    as long as its longest ray, so frames rendered together overlap one
    frame's longest rays with the others' bulk)."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    fpl = args.frames_per_launch
    frames = W.orbit_frames(36, 4096, 4)
    groups = [frames[i:i + fpl] for i in range(0, len(frames), fpl)]
    opts = W.render_opts(max_chunk=fpl * 4096 * 4096 * 4)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    dev = torch.device("cuda", 0)
    out = torch.empty((2, fpl, 2, 4096, 4096, 3), dtype=torch.float32, device=dev)
    # entering rays per frame (untimed counting pass, status only)
    # the orbit is symmetric up to the jitter: every 9th frame is counted
    entered = 0
    counted = frames[::9]
    for f in counted:
        _, aux = rt.render_multi(cloaks, W.render_opts(), room, [f], 3, aux=True)
        torch.cuda.synchronize()
        entered += int(torch.isin(aux["status"], torch.tensor([0, 2, 3, 4, 5], device=dev,
                                                                dtype=torch.int32)).sum())
        del aux
    entered_per_frame = entered / len(counted)
    rt.render_multi(cloaks, opts, room, groups[0], 3, out=out[:, :len(groups[0])])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for g in groups:
        rt.render_multi(cloaks, opts, room, g, 3, out=out[:, :len(g)])
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    samples = 36 * 4096 * 4096 * 4 * 2 * 2
    return {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error", "unit": "Mrays/s",
        "value": round(entered_per_frame * 36 / (ms * 1e-3) / 1e6, 3), "n_gpus": 1,
        "ms_per_step": round(ms, 2), "steps": 1, "warmup": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "large render: 36-frame orbit at 30 deg elevation, 4096^2 px x 4 jittered spp, "
                               "radial + azimuthal cloaks, ordinary + extraordinary, DP45 tol 1e-8, plain tracer",
                   "frames_per_launch": fpl,
                   "ray_branch_samples": samples, "ms_per_frame": round(ms / 36, 2),
                   "all_samples_per_s_M": round(samples / (ms * 1e-3) / 1e6, 1),
                   "entered_per_frame_estimate": int(entered_per_frame),
                   "frames_counted_for_entered": len(counted)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--frames-per-launch", type=int, default=2,
                    help="orbit workload and surrogate render: 4096^2 x 4 spp frames per integrator launch (1-4)")
    ap.add_argument("--workload", choices=("render3d", "batched", "orbit", "surrogate", "inplane", "hamiltonian",
                                           "weights", "unpolarized", "train"),
                    default="render3d")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 mixed")
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--streams", type=int, default=3,
                    help="render plans replayed on this many streams, consecutive steps overlapping")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-steps", type=int, default=10000,
                    help="AdamW steps of 65,536 rows (10,000 = 65 epochs of the 10 M labelled rays)")
    ap.add_argument("--surrogate-train", type=int, default=10_000_000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if not 1 <= args.streams <= 4:
        ap.error("--streams must be in 1..4")
    if not 1 <= args.frames_per_launch <= 4:
        ap.error("--frames-per-launch must be in 1..4 (at most 2^28 samples per launch)")
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; across GPUs the render would shard by camera or image "
              "tile (no exchange but the image gather), which is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1209_6038_amd import build as B
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    if not os.path.exists(rt.LIB_PATH):
        B.build()
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.workload == "orbit":
        print(json.dumps(finite_json(orbit_workload(args))), flush=True)
        return
    if args.workload == "inplane":
        print(json.dumps(finite_json(inplane_workload(args))), flush=True)
        return
    if args.workload == "hamiltonian":
        print(json.dumps(finite_json(hamiltonian_workload(args))), flush=True)
        return
    if args.workload == "weights":
        print(json.dumps(finite_json(weights_workload(args))), flush=True)
        return
    if args.workload == "unpolarized":
        print(json.dumps(finite_json(unpolarized_workload(args))), flush=True)
        return
    if args.workload == "train":
        print(json.dumps(finite_json(train_workload(args))), flush=True)
        return
    if args.workload == "surrogate":
        torch.cuda.set_device(0)
        rec = surrogate_leg(args.surrogate_steps, args.surrogate_train,
                            lambda msg: print(msg, file=sys.stderr, flush=True), args.frames_per_launch)
        print(json.dumps(finite_json({"config": {"workload": "surrogate leg only"}, "surrogate": rec})), flush=True)
        return
    batched = args.workload == "batched"
    cams = W.batched_views(64, 512) if batched else W.render_views(res=args.res)
    res = int(cams[0]["w"])
    opts = W.render_opts(precision=args.precision, refill_period=args.refill, block=args.block)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    out = torch.empty((2, len(cams), 2, res, res, 3), dtype=torch.float32, device=dev)
    tuned_ms = None
    if not (args.refill or args.block):
        # launch shape (block size, refill period) from the autotuner on this
        # batch; per-ray results do not depend on it
        opts, tuned_ms = rt.autotune_render(cloaks, opts, room, cams, 3)
    # one plan per stream (own workspace and images); step k replays plan
    # k mod S on stream k mod S: all cloaks, views and branches of the batch
    # in one pass (one integrator launch)
    plans = [rt.RenderPlan(cloaks, opts, room, cams, 3) for _ in range(args.streams)]
    streams = [torch.cuda.Stream() for _ in range(args.streams)]

    def step(k):
        with torch.cuda.stream(streams[k % args.streams]):
            plans[k % args.streams].launch()

    # untimed counting pass: entering rays and integrator step attempts
    entered = 0
    flops = 0
    _, aux = rt.render_multi(cloaks, opts, room, cams, 3, aux=True)
    torch.cuda.synchronize()
    st = aux["status"].cpu().numpy()
    ns = aux["nsteps"].cpu().numpy().astype(np.int64)
    del aux
    entered += int(np.isin(st, (0, 2, 3, 4, 5)).sum())
    for ci in range(2):
        for pi, pol in enumerate((0, 1)):
            kind = ci * 2 + pol
            flops += int(ns[ci, :, pi].sum()) * attempt_flops(kind, opts["scheme"])
    camera_rays = 2 * len(cams) * 2 * res * res

    for k in range(max(args.warmup, args.streams)):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # every plan rendered the batch: the images agree with an eager render
    rt.render_multi(cloaks, opts, room, cams, 3, out=out)
    torch.cuda.synchronize()
    images_equal = all(torch.equal(p.rgb, out) for p in plans)
    for p in plans:
        p.close()
    del plans
    # graph replays carry no timing events, and overlapped launches share the
    # chip: time the integrator on eager, one-at-a-time launches of the same
    # batch (same kernels, same launch shape), HIP events on the launch stream
    rt.render_multi(cloaks, opts, room, cams, 3, out=out)
    torch.cuda.synchronize()
    rt.profile_enable(True)
    rt.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        rt.render_multi(cloaks, opts, room, cams, 3, out=out)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / args.steps
    transit_ms, launches = rt.profile_read()
    launches_per_step = launches / args.steps
    rt.profile_enable(False)

    avg_launch_ms = transit_ms / max(launches, 1)
    flops_per_launch = flops / launches_per_step
    achieved = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if args.precision == 0 else PEAK_FP32_TFLOPS
    value = entered / (ms * 1e-3) / 1e6
    shape = (opts.get("block") or 256, opts.get("refill_period") or 2)
    traffic, traffic_shape = traffic_for(*shape) if not batched else (None, None)
    rec = {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error; surrogate vs plain speedup at 1e-3",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": ("batched: 64 seeded views x 512^2 px (azimuth U[0,2pi), elevation "
                                "U[0,60] deg), radial + azimuthal cloaks, ordinary + extraordinary, "
                                "DP45 tol 1e-8, one HIP-graph replay per step" if batched else
                                "3-D render: radial + azimuthal uniaxial cloaks (R1=1, R2=2, "
                                "height 4), checkerboard room 20x20x10, 4 elevations x 1024^2 px, "
                                "ordinary + extraordinary, DP45 tol 1e-8"),
                   "streams": args.streams,
                   "eager_ms_per_step": round(eager_ms, 4),
                   "images_equal_across_streams": images_equal,
                   "launch_shape": {"block": shape[0],
                                    "refill_period": shape[1],
                                    "autotuned_ms": tuned_ms},
                   "miss_fraction": round(1.0 - entered / camera_rays, 4),
                   "camera_rays_per_step": camera_rays,
                   "rays_entering_cloak_per_step": entered,
                   "all_camera_rays_per_s_M": round(camera_rays / (ms * 1e-3) / 1e6, 3),
                   "precision": "fp64" if args.precision == 0 else "mixed",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic,
                     "traffic_launch_shape": traffic_shape,
                     "kernel": "k_transit (integrator)",
                     "avg_launch_ms": round(avg_launch_ms, 4),
                     "launches_per_step": launches_per_step,
                     "integrator_share_of_eager_step": round(transit_ms / args.steps / eager_ms, 4)},
    }
    if not batched and args.precision == 0:
        rec["mixed_precision"] = mixed_precision_leg(cloaks, room, cams, eager_ms, out, opts)
    if not args.no_cpu_baseline and not batched:
        rec["cpu_baseline"] = cpu_baseline(W.opts_dp45(), cams, args.cpu_stride)
    if not args.no_surrogate:
        del out
        rt.release_workspace()
        rec["surrogate"] = surrogate_leg(args.surrogate_steps, args.surrogate_train,
                                         lambda msg: print(msg, file=sys.stderr, flush=True),
                                         args.frames_per_launch)
    print(json.dumps(finite_json(rec)), flush=True)


if __name__ == "__main__":
    main()
