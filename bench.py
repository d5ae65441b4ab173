#!/usr/bin/env python3
"""Benchmark of the cloak ray tracer on one MI355X.

Headline (one step): the large-render workload -- a 36-frame camera orbit at
30 deg elevation around the radial and the azimuthal uniaxial cloaks (R1 = 1,
R2 = 2, height 4, standing in the checkerboard room [-10,10]^2 x [0,10] with
0.5 tiles), pinhole camera at distance 8 from (0,0,2), 60 deg field of view,
4096 x 4096 pixels, 4 jittered samples per pixel, ordinary and extraordinary
branch traced separately, Dormand-Prince 5(4) at tolerance 1e-8, FP64: 9.66e9
ray-branch samples per step, rendered two frames per integrator launch
(rt_render_multi). Inputs (cameras, room, cloaks) are resident before the
timed region; W orbits warm up, K orbits are timed between device
synchronizations.

Metric: Mrays/s traced through the cloak = samples that refract into the
cloak material per second of step time (all samples per second are reported
too); the exit error of this tracer against the FP64 oracle is <= 1e-6 (the
GPU parity tests).

Roofline: algorithmic FP64 flops of the integrator (step attempts x flops per
attempt, counted in an untimed pass) per launch over the launch time measured
with HIP events on the launch stream, against the 78.6 TFLOP/s FP64 vector
peak; HBM traffic per launch from rocprofv3 counters (see TRAFFIC).

Reported beside it: the FP64 C oracle on a strided sample of the first frame
on the host cores (cpu_baseline); the surrogate (the "surrogate vs plain
speedup at 1e-3" half of the metric: a BF16 MFMA network trained on 10 M
exact transits, gated and calibrated at the 1e-3 exit-error tolerance, as a
transit replacement on 1 M held-out entries and inside the orbit render, with
the per-pixel difference from the plain render); and sub-records for the
other workloads (the 1024^2 four-elevation render on overlapping streams, the
64-view batched render in HIP graphs, the 2-D in-plane set, surrogate
training throughput).

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

# statuses of rays that refracted into the crystal (exited, absorbed, step
# limit, diverged, totally reflected): the "rays traced through the cloak"
ENTERED = (0, 2, 3, 4, 5)

# HBM traffic of one integrator launch from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) of `bench.py --workload <w> --block B --refill R
# --profile-launches N`, scaled by the same counters on a plain device copy of
# known size (bench.py --copy-probe), per workload and launch shape (block,
# refill period). Valid only for the integrator source it was measured on;
# reported as null otherwise, or for a shape that was not measured.
TRAFFIC = {"source_sha256": "a9a9495366d70c26cce4b56bb0ce7d971ef1e55ade0358be616ac5afc396e310",
           "bytes_per_launch": {
               "orbit": {(64, 4): 16_367_264_853, (64, 8): 16_602_244_747, (64, 12): 16_738_936_565,
                         (64, 16): 16_740_058_976, (128, 4): 16_492_896_405, (128, 8): 16_727_920_267,
                         (128, 12): 16_840_027_520, (128, 16): 16_883_521_525, (256, 4): 16_535_520_341,
                         (256, 8): 16_765_989_120, (256, 12): 16_876_966_368, (256, 16): 16_928_693_867},
               "render_1024": {(64, 1): 576_314_856, (64, 2): 578_478_216, (64, 4): 581_150_584,
                               (64, 8): 585_980_760, (64, 12): 589_803_952, (64, 16): 585_261_208,
                               (128, 1): 577_334_288, (128, 2): 579_538_424, (128, 4): 582_954_576,
                               (128, 8): 587_826_800, (128, 12): 591_496_336, (128, 16): 588_082_776,
                               (256, 1): 582_124_096, (256, 2): 585_049_584, (256, 4): 589_310_288,
                               (256, 8): 595_968_472, (256, 12): 598_821_816, (256, 16): 594_912_168},
               "batched": {(64, 1): 2_575_599_168, (64, 2): 2_588_529_816, (64, 4): 2_599_886_416,
                           (64, 8): 2_611_125_984, (64, 12): 2_614_895_840, (64, 16): 2_602_135_272,
                           (128, 1): 2_580_383_632, (128, 2): 2_599_642_352, (128, 4): 2_614_251_952,
                           (128, 8): 2_624_741_968, (128, 12): 2_625_039_016, (128, 16): 2_610_439_112,
                           (256, 1): 2_593_232_352, (256, 2): 2_614_858_856, (256, 4): 2_633_913_808,
                           (256, 8): 2_642_026_480, (256, 12): 2_640_291_072, (256, 16): 2_626_358_272}}}


def traffic_for(workload, shape=None):
    """(bytes per integrator launch) of the workload at launch shape
    (block, refill_period), or None where it was not measured."""
    if TRAFFIC["source_sha256"] != integrator_source_hash():
        return None
    v = TRAFFIC["bytes_per_launch"].get(workload)
    return v.get(tuple(shape)) if isinstance(v, dict) and shape is not None else None


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
                n_entered += int(np.isin(r["status"], ENTERED).sum())
                n_rays += len(ids)
    dt = time.perf_counter() - t0
    return {"value": n_entered / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"every {stride}th pixel of the 16 images ({n_rays} camera rays, "
                      f"{n_entered} entering the cloak), FP64 C oracle with OpenMP, {dt:.1f} s",
            "all_rays_per_s": n_rays / dt}


def surrogate_leg(steps: int, n_train: int, log, keep: bool = False):
    """Train, calibrate and time the transit surrogate (see the module doc).
    The transit speedup is measured with the gate's near-singular band off
    (p_min = 0: entries whose paths pass within ~1e-4 of r = r1 are accepted
    like the others; the error statistics leave out references the
    integrator did not resolve) and with it on (p_min = 1e-4: those entries
    go to the exact transit, which is where its longest rays are).
    keep=True also returns the model and the calibration data."""
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
                          hres_exact=h_cal, unresolved=UNRESOLVED, p_min=0.0)
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
    m.calibrate(cl, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=16, dilate=1, hres_exact=h_cal,
                unresolved=UNRESOLVED, p_min=1e-4)
    y_b2, st_b2, fb_b2 = m.infer(cl, op, x_ev)
    acc_band = float((fb_b2 == 0).float().mean())
    ms_sur_band = timed(lambda: m.infer(cl, op, x_ev, y5=y_b2, fallback=fb_b2, status=st_b2))
    del y_b2, st_b2, fb_b2
    ms_fwd = timed(lambda: m.forward(x_ev))
    mlp_tflops = MLP_MFMA_FLOPS * n / (ms_fwd * 1e-3) / 1e12
    rec = {
        "speedup": round(ms_plain / ms_sur, 3),
        "plain_Mrays_s": round(n / (ms_plain * 1e-3) / 1e6, 2),
        "surrogate_Mrays_s": round(n / (ms_sur * 1e-3) / 1e6, 2),
        "near_singular_band": {"p_min": 1e-4, "speedup": round(ms_plain / ms_sur_band, 3),
                               "accepted_fraction": round(acc_band, 4)},
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
    if keep:
        return rec, m, (x_cal, y_cal, st_cal, h_cal, cl, tol)
    m.close()
    return rec


def cap_leg(side_model, log, steps: int = 60000, n_train: int = 8_000_000, n_cal: int = 16_000_000):
    """The surrogate's cap job: a second model learns the side entries of the
    height-4 cloaks whose path leaves through an end cap (the closed-form
    transits are those of the infinite cylinder, and the side job's gate
    rejects every entry that meets a cap). Trained on the cap exits of
    n_train uniform side entries, calibrated on n_cal others, measured on
    1 M held-out entries against the exact transit: the share of cap exits
    accepted with the network and with the closed forms alone (a side model
    whose network output is zeroed, every cell trusted), the accepted exit
    errors, and the side model alone against the side model chained to the
    cap model (rows the first rejects go to the second), with times."""
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import surrogate as S
    from paper_1209_6038_amd import workloads as W

    def sync():
        torch.cuda.synchronize()

    def timed(fn, reps=3):
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

    tol = 1e-3
    cl = S.make_cloaks(W.HEIGHT)
    op = S.exact_opts()
    sync()
    t0 = time.perf_counter()
    x_tr, t_tr, w_tr = S.cap_training_set(n_train, 1101, op)
    sync()
    t_label = time.perf_counter() - t0
    rows = x_tr.shape[1]
    m = rt.Surrogate(seed=0)
    m.set_job(rt.CAP, cl[0])
    m.fit_scaling(x_tr, t_tr, w_tr)
    batch = 16384
    t0 = time.perf_counter()
    loss = S.train(m, x_tr, t_tr, w_tr, steps=steps, batch=batch, lr=1e-3, lr_end=1e-5, huber=0.01)
    sync()
    t_train = time.perf_counter() - t0
    del x_tr, t_tr, w_tr
    log(f"cap model: {rows} cap exits of {n_train} entries labelled in {t_label:.2f} s, trained {steps} steps in "
        f"{t_train:.1f} s (loss {loss:.2e})")
    x_cal = S.features(n_cal, 1102)
    y_cal, st_cal, h_cal = rt.transit_exact(cl, op, x_cal, hres=True)
    trusted = m.calibrate(cl, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=CAP_MIN_COUNT, dilate=CAP_DILATE,
                          hres_exact=h_cal, unresolved=UNRESOLVED, p_min=0.0)
    del x_cal, y_cal, st_cal, h_cal
    n = 1_000_000
    x_ev = S.features(n, 1103)
    y_ex, st_ex, h_ex = rt.transit_exact(cl, op, x_ev, hres=True)
    up = x_ev[3] >= 0
    cap = (st_ex == 0) & (((y_ex[1] > W.HEIGHT) & up) | ((y_ex[1] < 0.0) & ~up))
    # references the integrator resolves: drift below UNRESOLVED and below
    # the squared normal wave number (cos alpha cos beta)^2 that the exit
    # keeps (a grazing side entry's drift above it turns the side exit into
    # a total reflection, and the ray runs on to a cap)
    kn = torch.cos(x_ev[2]) * torch.cos(x_ev[3])
    resolved = (h_ex <= UNRESOLVED) & (h_ex < kn * kn)
    cap = cap & resolved
    y_c, _, fb_c = m.infer(cl, op, x_ev)
    acc_c = fb_c == 0
    err, operr = S.exit_error(y_c, y_ex)
    a = acc_c & cap
    e = S.summarize_errors(err, a)
    base = rt.Surrogate(seed=0)
    base.set_params(np.zeros(rt.Surrogate.NPARAM, np.float32))
    sc = base.get_scaling()
    sc[12:22] = np.concatenate([np.zeros(5, np.float32), np.ones(5, np.float32)])
    base.set_scaling(sc)
    base.calibrate(cl, x_ev, y_ex, st_ex, tol=1e30, min_count=1, p_min=0.0)
    _, _, fb_b = base.infer(cl, op, x_ev)
    base.close()
    _, _, fb_s = side_model.infer(cl, op, x_ev)
    side_model.chain(m)
    try:
        _, _, fb_k = side_model.infer(cl, op, x_ev)
        ms_chain = timed(lambda: side_model.infer(cl, op, x_ev))
    finally:
        side_model.chain(None)
    ms_side = timed(lambda: side_model.infer(cl, op, x_ev))
    ms_plain = timed(lambda: rt.transit_exact(cl, op, x_ev))
    ncap = int(cap.sum())

    def share(mask):
        return round(float(mask.float().mean()), 4)

    rec = {
        "workload": ("1 M held-out uniform side entries (phi, z in [0, 4], alpha, beta, branch and axis bits as the "
                     "side job's) of the height-4 radial and azimuthal cloaks, DP45 1e-8 FP64 exact transit"),
        "cap_exits": ncap,
        "accepted_of_cap_exits": {"with_network": share(acc_c[cap]), "closed_forms_only": share(fb_b[cap] == 0)},
        "accepted_exit_error": {k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in e.items()},
        "accepted_over_tolerance": int((err[a] > tol).sum()),
        "accepted_not_cap_exits": int((acc_c & ~cap & resolved).sum()),
        "reference": ("cap exits of the exact transit where it resolves the path: |H - 1| <= 1e-6 at the exit and "
                      "below the entry's squared normal wave number"),
        "accepted_opl_rel_error_p99": float(f"{S.summarize_errors(operr, a).get('p99', 0.0):.3e}"),
        "tolerance": tol,
        "trusted_cells": round(trusted, 4),
        "calibration": {"entries": n_cal, "tol": 0.5 * tol, "min_count": CAP_MIN_COUNT, "dilate": CAP_DILATE},
        "side_entries_accepted": {"side_model": share(fb_s == 0), "side_then_cap_model": share(fb_k == 0)},
        "ms_per_1M_entries": {"plain": round(ms_plain, 3), "side_model": round(ms_side, 3),
                              "side_then_cap_model": round(ms_chain, 3)},
        "train": {"entries": n_train, "cap_exit_rows": rows, "steps": steps, "batch": batch,
                  "seconds": round(t_train, 2), "final_loss": float(f"{loss:.3e}")},
    }
    log(f"cap model: accepts {rec['accepted_of_cap_exits']['with_network']} of the cap exits (closed forms "
        f"{rec['accepted_of_cap_exits']['closed_forms_only']}), exit error p50 {e.get('p50', 0):.2e} max "
        f"{e.get('max', 0):.2e}, over tol {rec['accepted_over_tolerance']}")
    del x_ev, y_ex, st_ex, h_ex, y_c, fb_c, err, operr
    return rec, m


# calibration of the cap model's trust map (cells of (axis, branch) x alpha x
# |beta| x u, 32 x 16 x 32)
CAP_MIN_COUNT, CAP_DILATE = 8, 1


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
    steps = args.train_steps
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
    entered = int(np.isin(st, ENTERED).sum())
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
    # the same impact parameters 16 times denser: the "wide" rays fill the
    # chip's resident lanes several times over, so the comparison is one of
    # throughput rather than of the longest ray's latency
    big = W.inplane_bundle(16384 * 16, 8)
    pbig = big[0] * (-big[4]) + big[1] * big[3]
    sets = {"wide": (bundle, pb, (np.abs(pb) >= 0.3) & (np.abs(pb) < 1.999)),
            "near_axis": (bundle, pb, (np.abs(pb) >= 1e-3) & (np.abs(pb) < 0.3)),
            "wide_full_chip": (big, pbig, (np.abs(pbig) >= 0.3) & (np.abs(pbig) < 1.999))}
    steps = {"wide": ((4e-3, 2e-3, 1e-3, 5e-4, 2.5e-4), (1.6e-2, 8e-3, 4e-3, 2e-3, 1e-3)),
             "near_axis": ((4e-3, 2e-3, 1e-3, 5e-4, 2.5e-4), (1.6e-2, 8e-3, 4e-3, 2e-3, 1e-3)),
             "wide_full_chip": ((2e-3, 1e-3), (4e-3, 2e-3))}
    cl = rt.Cloak(W.cloak(W.RADIAL))
    target = 1e-8

    def sweep(make, steps, bundle, pb, sel):
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
            per_step = (HAM_COMBINE_FLOPS + 4 * HAM_RHS_FLOPS[1] if opts["scheme"] in (2, 3)
                        else attempt_flops(1, 0))
            tflops = float(ns.sum()) * per_step / (launch_ms * 1e-3) / 1e12
            rows.append({"step": h, "ms_per_call": round(a.elapsed_time(b) / 3, 4),
                         "integrator_launch_ms": round(launch_ms, 4),
                         "integrator_fp64_frac": round(tflops / PEAK_FP64_TFLOPS, 4),
                         "steps_per_ray": round(float(ns.mean()), 1), "max_steps_of_a_ray": int(ns.max()),
                         "max_exit_err": float(f"{err.max():.3e}"), "not_exited": int((st != 0).sum())})
        return rows

    res = {}
    for name, (bnd, pbb, sel) in sets.items():
        eq8 = sweep(lambda h: W.opts_rk4(h, max_steps=200_000), steps[name][0], bnd, pbb, sel)
        ham = sweep(lambda h: W.opts_rk4_ham(h, max_steps=200_000), steps[name][1], bnd, pbb, sel)
        # the canonical normalization: tau steps of h are optical-path steps of 2 h
        hamc = sweep(lambda h: W.opts_rk4_hamc(h, max_steps=200_000), tuple(0.5 * h for h in steps[name][0]),
                     bnd, pbb, sel)
        ok_e = [r for r in eq8 if r["max_exit_err"] <= target]
        ok_h = [r for r in ham if r["max_exit_err"] <= target]
        ok_c = [r for r in hamc if r["max_exit_err"] <= target]
        e = max(ok_e, key=lambda r: r["step"]) if ok_e else None
        h = max(ok_h, key=lambda r: r["step"]) if ok_h else None
        cc = max(ok_c, key=lambda r: r["step"]) if ok_c else None
        res[name] = {"rays": int(sel.sum()), "eq8_rk4_in_t": eq8, "hamiltonian_rk4_in_tau": ham,
                     "canonical_hamiltonian_rk4_in_tau": hamc,
                     "at_target": {"eq8": e and {"step": e["step"], "ms_per_call": e["ms_per_call"]},
                                   "hamiltonian": h and {"step": h["step"], "ms_per_call": h["ms_per_call"]},
                                   "canonical_hamiltonian": cc and {"step": cc["step"],
                                                                    "ms_per_call": cc["ms_per_call"]},
                                   "time_ratio_hamiltonian_over_eq8": (round(h["ms_per_call"] / e["ms_per_call"], 3)
                                                                       if e and h else None),
                                   "time_ratio_canonical_over_eq8": (round(cc["ms_per_call"] / e["ms_per_call"], 3)
                                                                     if e and cc else None)}}
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
        entered += int(np.isin(st, ENTERED).sum())
        flops += int(r["nsteps"].cpu().numpy().astype(np.int64).sum()) * attempt_flops(2 * ax + br, 1)
        ex = st == 0
        summary[f"{'radial' if ax == 0 else 'azimuthal'}_{'o' if br == 0 else 'e'}"] = {
            "exited": int(ex.sum()), "mean_weight_exited": round(float(w[ex].mean()), 5),
            "entering_intensity_delivered": round(float(w[ex].sum() / max(1, np.isin(st, ENTERED).sum())), 5)}

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
    DP45 1e-8, FP64) with the Eq. (12) unpolarized images and the two
    polarizer-goggle images, timed beside the same render without images,
    with the unpolarized images only, and with first-order reflections added
    to the images; one step = one rt_render_multi call."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W

    cams = W.render_views(res=args.res)
    opts = W.render_opts(block=args.block, refill_period=args.refill)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    _, aux = rt.render_multi(cloaks, opts, room, cams, 3, aux=True, unpolarized=True, goggles=True)
    _, aux_r = rt.render_multi(cloaks, opts, room, cams, 3, unpolarized=True, goggles=True, reflections=True)
    torch.cuda.synchronize()
    dev = aux["status"].device
    entered = int(torch.isin(aux["status"], torch.tensor(ENTERED, device=dev, dtype=torch.int32)).sum())
    means = {k: round(float(aux[k].mean()), 5) for k in ("unpol", "goggle_inplane", "goggle_axial")}
    means["unpol_with_reflections"] = round(float(aux_r["unpol"].mean()), 5)
    del aux, aux_r
    modes = {"none": {}, "unpolarized": {"unpolarized": True}, "goggles": {"unpolarized": True, "goggles": True},
             "reflections": {"unpolarized": True, "goggles": True, "reflections": True}}
    timing = {}
    for mode, kw in modes.items():
        for _ in range(args.warmup):
            rt.render_multi(cloaks, opts, room, cams, 3, **kw)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        rt.profile_enable(True)
        rt.profile_read()
        a.record()
        for _ in range(args.steps):
            rt.render_multi(cloaks, opts, room, cams, 3, **kw)
        b.record()
        torch.cuda.synchronize()
        transit_ms, launches = rt.profile_read()
        rt.profile_enable(False)
        timing[mode] = (a.elapsed_time(b) / args.steps, transit_ms / max(1, launches))
    ms, launch_ms = timing["goggles"]
    return {
        "metric": "Mrays/s traced through cloak at <=1e-6 exit error, with Eq. (12) unpolarized and goggle images",
        "unit": "Mrays/s", "value": round(entered / (ms * 1e-3) / 1e6, 3), "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D render with unpolarized and in-plane / axial goggle images: radial + "
                               "azimuthal cloaks (height 4), 4 elevations x 1024^2 px, ordinary + extraordinary, "
                               "DP45 tol 1e-8, FP64, eager calls",
                   "entering_per_step": entered, "ms_per_step_without_images": round(timing["none"][0], 4),
                   "ms_per_step_unpolarized_only": round(timing["unpolarized"][0], 4),
                   "images_cost": round(ms / timing["none"][0], 4),
                   "goggles_cost_over_unpolarized": round(ms / timing["unpolarized"][0], 4),
                   "ms_per_step_with_first_order_reflections": round(timing["reflections"][0], 4),
                   "reflections_cost_over_goggles": round(timing["reflections"][0] / ms, 4),
                   "mean_image_values": means},
        "roofline": {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": None, "traffic": None, "kernel": "k_transit (integrator, weighted)",
                     "avg_launch_ms": round(launch_ms, 4),
                     "avg_launch_ms_without_images": round(timing["none"][1], 4)},
    }


def _entered_tensor(dev):
    import torch
    return torch.tensor(ENTERED, device=dev, dtype=torch.int32)


def orbit_counts(cloaks, room, frames, log):
    """Untimed pass over the orbit, one frame per call with per-sample status
    and step counts only: samples that enter the cloak, and the integrator's
    algorithmic FP64 flops (step attempts x flops per attempt of each
    (cloak, branch) kind). Both are per-ray quantities, independent of how
    frames are grouped into launches."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    entered, flops = 0, 0
    dev = torch.device("cuda", torch.cuda.current_device())
    ent = _entered_tensor(dev)
    for k, f in enumerate(frames):
        _, aux = rt.render_multi(cloaks, W.render_opts(), room, [f], 3, aux=("status", "nsteps"))
        entered += int(torch.isin(aux["status"], ent).sum())
        for ci in range(2):
            for pi in range(2):
                flops += int(aux["nsteps"][ci, 0, pi].sum(dtype=torch.int64)) * attempt_flops(2 * ci + pi, 1)
        del aux
    torch.cuda.synchronize()
    log(f"orbit: {len(frames)} frames counted, {entered} entering samples, {flops / 1e12:.2f} TFLOP of integration")
    return entered, flops


def orbit_cpu_baseline(frame, stride):
    """The FP64 C oracle (OpenMP, all host threads) on every `stride`-th
    sample of the first orbit frame, both cloaks and both branches."""
    import numpy as np

    import oracle
    from paper_1209_6038_amd import workloads as W
    room = W.room()
    ids = np.arange(0, frame["w"] * frame["h"] * frame["spp"], stride, dtype=np.int64)
    n_entered = 0
    t0 = time.perf_counter()
    for axis in (0, 1):
        c = W.cloak(axis, height=W.HEIGHT)
        for branch in (0, 1):
            r = oracle.render_samples(c, W.opts_dp45(), room, frame, 0, branch, ids)
            n_entered += int(np.isin(r["status"], ENTERED).sum())
    dt = time.perf_counter() - t0
    return {"value": n_entered / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"every {stride}th sample of orbit frame 0 ({len(ids)} samples x 2 cloaks x 2 branches, "
                       f"{n_entered} entering the cloak), FP64 C oracle with OpenMP, {dt:.1f} s"),
            "all_samples_per_s": 4 * len(ids) / dt}


def orbit_setup(args):
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    fpl = args.frames_per_launch
    frames = W.orbit_frames(36, 4096, 4)[:args.frames]
    groups = [frames[i:i + fpl] for i in range(0, len(frames), fpl)]
    opts = W.render_opts(max_chunk=fpl * 4096 * 4096 * 4, block=args.block, refill_period=args.refill)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    return frames, groups, opts, cloaks, W.room()


def orbit_headline(args, log):
    """The headline: the 36-frame orbit (see the module doc), plain tracer."""
    import torch
    from paper_1209_6038_amd import rt

    frames, groups, opts, cloaks, room = orbit_setup(args)
    fpl = args.frames_per_launch
    dev = torch.device("cuda", 0)
    entered, flops = orbit_counts(cloaks, room, frames, log)
    # launch shape (block size, refill period) from the autotuner on the first
    # launch group, unless given; untimed
    tuned_ms = None
    if not (args.block or args.refill):
        opts, tuned_ms = rt.autotune_render(cloaks, opts, room, groups[0], 3)
        torch.cuda.synchronize()
        log(f"orbit launch shape: block {opts['block']}, refill period {opts['refill_period']} "
            f"({tuned_ms:.1f} ms per launch group)")
    shape = (opts.get("block") or 256, opts.get("refill_period") or 2)
    # images per launch group, each a dense [cloak][frame][branch][h][w][3] block
    out = torch.empty((len(groups), 2, fpl, 2, 4096, 4096, 3), dtype=torch.float32, device=dev)
    # consecutive launch groups alternate between streams: the library keeps
    # a workspace per stream, so one group's camera rays, sort and finish run
    # beside the previous group's integrator and its drain
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(args.orbit_streams - 1)]

    def step(overlap=True):
        for k, g in enumerate(groups):
            with torch.cuda.stream(streams[k % len(streams)] if overlap else streams[0]):
                rt.render_multi(cloaks, opts, room, g, 3, out=out[k])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"orbit: {ms:.1f} ms per orbit ({ms / len(frames):.2f} ms per frame)")
    # integrator launches timed with HIP events on the launch stream, one
    # stream (overlapped launches would share the chip)
    rt.profile_enable(True)
    rt.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    step(overlap=False)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1)
    transit_ms, launches = rt.profile_read()
    rt.profile_enable(False)
    avg_launch_ms = transit_ms / max(launches, 1)
    achieved = flops / max(launches, 1) / (avg_launch_ms * 1e-3) / 1e12
    samples = len(frames) * 4096 * 4096 * 4 * 2 * 2
    rec = {
        "metric": "Mrays/s traced through cloak at ≤1e-6 exit error; surrogate vs plain speedup at 1e-3",
        "value": round(entered / (ms * 1e-3) / 1e6, 3),
        "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"large render: {len(frames)}-frame orbit at 30 deg elevation, 4096^2 px x 4 "
                                "jittered spp, radial + azimuthal uniaxial cloaks (R1=1, R2=2, height 4) in the "
                                "checkerboard room 20x20x10, ordinary + extraordinary, DP45 tol 1e-8, FP64, plain "
                                "tracer"),
                   "frames": len(frames), "frames_per_launch": fpl, "ray_branch_samples_per_step": samples,
                   "rays_entering_cloak_per_step": entered, "miss_fraction": round(1.0 - entered / samples, 4),
                   "all_samples_per_s_M": round(samples / (ms * 1e-3) / 1e6, 1),
                   "ms_per_frame": round(ms / len(frames), 3), "parallelism": "single GPU",
                   "streams": len(streams), "ms_per_step_one_stream": round(eager_ms, 3),
                   "launch_shape": {"block": shape[0], "refill_period": shape[1], "autotuned_ms": tuned_ms}},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic_for("orbit", shape),
                     "kernel": "k_transit (integrator)", "avg_launch_ms": round(avg_launch_ms, 3),
                     "launches_per_step": launches, "flops_per_launch": round(flops / max(launches, 1)),
                     "integrator_share_of_step": round(transit_ms / eager_ms, 4)},
    }
    torch.cuda.synchronize()
    rt.release_workspace()  # the other streams' workspaces (~70 GB each) are not needed further on
    return rec, out, (frames, groups, opts, cloaks, room)


def orbit_surrogate(model, orbit, out_plain, ms_plain, log, cal, sweep_frames=4,
                    difficulties=(0, 2, 3, 4), p_mins=(1e-4, 0.0), cap_model=None):
    """The surrogate inside the orbit render (rt_render_surrogate): a sweep of
    the difficulty threshold (side entries of at least that bucket go to the
    network) and of the near-singular band p_min on `sweep_frames` frames,
    then the fastest setting whose images stay within 1/255 of the plain
    render on every pixel runs the whole orbit: time per orbit against the
    plain orbit, and the per-pixel difference over all of its frames. With
    cap_model, the same setting also runs with the side model chained to the
    cap model (side entries the first rejects that meet a cap go to the
    second): accepted entries, time and pixel difference with and without it,
    on the sweep frames (every side entry offered) and on the whole orbit."""
    import torch
    from paper_1209_6038_amd import rt
    frames, groups, opts, cloaks, room = orbit
    fpl = max(len(g) for g in groups)
    sub = [k for k in range(len(groups))][:: max(1, len(groups) // max(1, sweep_frames // fpl))][:max(1, sweep_frames // fpl)]
    out_s = torch.empty_like(out_plain)
    x_cal, y_cal, st_cal, h_cal, cl_inf, tol = cal

    def run_groups(ks, dmin):
        for k in ks:
            g = groups[k]
            rt.render_surrogate(model, cloaks, opts, room, g, 3, out=out_s[k], min_difficulty=dmin)

    def plain_groups(ks):
        for k in ks:
            g = groups[k]
            rt.render_multi(cloaks, opts, room, g, 3, out=out_plain[k])

    def timed(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    nf_sub = sum(len(groups[k]) for k in sub)
    ms_plain_sub = timed(lambda: plain_groups(sub)) / nf_sub
    sweep = []
    for p_min in p_mins:
        model.calibrate(cl_inf, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=16, dilate=1, hres_exact=h_cal,
                        unresolved=UNRESOLVED, p_min=p_min)
        for dmin in difficulties:
            offered = accepted = 0
            for k in sub:
                g = groups[k]
                _, (c0, c1) = rt.render_surrogate(model, cloaks, opts, room, g, 3, out=out_s[k], counts=True,
                                                  min_difficulty=dmin)
                offered += c0
                accepted += c1
            torch.cuda.synchronize()
            dmax = 0.0
            over = 0
            npix = 0
            for k in sub:
                d = (out_s[k] - out_plain[k]).abs().amax(dim=-1)
                dmax = max(dmax, float(d.max()))
                over += int((d > 1.0 / 255.0).sum())
                npix += d.numel()
                del d
            ms_s = timed(lambda: run_groups(sub, dmin)) / nf_sub
            log(f"surrogate render p_min {p_min:g}, min difficulty {dmin}: {ms_s:.1f} ms/frame "
                f"(plain {ms_plain_sub:.1f}), accepted {accepted}/{offered}, max pixel difference {dmax:.4f}")
            sweep.append({"p_min": p_min, "min_difficulty": dmin, "surrogate_ms_per_frame": round(ms_s, 2),
                          "speedup": round(ms_plain_sub / ms_s, 3), "offered_per_frame": offered // nf_sub,
                          "accepted_per_frame": accepted // nf_sub, "pixels_over_1_255": over / npix,
                          "max_pixel_difference": round(dmax, 4)})
    valid = [r for r in sweep if r["max_pixel_difference"] <= 1.0 / 255.0]
    best = max(valid, key=lambda r: r["speedup"]) if valid else None
    full = None
    if best is not None:
        model.calibrate(cl_inf, x_cal, y_cal, st_cal, tol=0.5 * tol, min_count=16, dilate=1, hres_exact=h_cal,
                        unresolved=UNRESOLVED, p_min=best["p_min"])
        allk = list(range(len(groups)))
        run_groups(allk[:1], best["min_difficulty"])  # warm-up
        ms_orbit = timed(lambda: run_groups(allk, best["min_difficulty"]))
        dmax, over, npix = 0.0, 0, 0
        for k in range(len(groups)):
            d = (out_s[k] - out_plain[k]).abs().amax(dim=-1)
            dmax = max(dmax, float(d.max()))
            over += int((d > 1.0 / 255.0).sum())
            npix += d.numel()
            del d
        full = {"p_min": best["p_min"], "min_difficulty": best["min_difficulty"],
                "surrogate_ms_per_orbit": round(ms_orbit, 2), "plain_ms_per_orbit": round(ms_plain, 2),
                "speedup": round(ms_plain / ms_orbit, 3), "max_pixel_difference": round(dmax, 5),
                "pixels_over_1_255": over / npix}
        log(f"surrogate orbit: {ms_orbit:.0f} ms vs plain {ms_plain:.0f} ms, max pixel difference "
            f"{full['max_pixel_difference']}")
    chained = None
    if best is not None and cap_model is not None:
        def frames_rec(ks, dmin, chain):
            model.chain(cap_model if chain else None)
            try:
                offered = accepted = 0
                for k in ks:
                    _, (c0, c1) = rt.render_surrogate(model, cloaks, opts, room, groups[k], 3, out=out_s[k],
                                                      counts=True, min_difficulty=dmin)
                    offered += c0
                    accepted += c1
                torch.cuda.synchronize()
                dmax = max(float((out_s[k] - out_plain[k]).abs().max()) for k in ks)
                ms = timed(lambda: run_groups(ks, dmin))
            finally:
                model.chain(None)
            nf = sum(len(groups[k]) for k in ks)
            return {"ms_per_frame": round(ms / nf, 2), "offered_per_frame": offered // nf,
                    "accepted_per_frame": accepted // nf, "max_pixel_difference": round(dmax, 5)}

        chained = {"note": ("side model alone vs chained to the cap model, same calibration; min_difficulty 0 offers "
                            "every side entry, the best setting only the hard ones"),
                   "every_side_entry": {"without_cap_model": frames_rec(sub, 0, False),
                                        "with_cap_model": frames_rec(sub, 0, True)},
                   "best_setting": {"without_cap_model": frames_rec(sub, best["min_difficulty"], False),
                                    "with_cap_model": frames_rec(sub, best["min_difficulty"], True)}}
        allk = list(range(len(groups)))
        model.chain(cap_model)
        try:
            ms_orbit_c = timed(lambda: run_groups(allk, best["min_difficulty"]))
            dmax = max(float((out_s[k] - out_plain[k]).abs().max()) for k in allk)
        finally:
            model.chain(None)
        chained["orbit_with_cap_model"] = {"surrogate_ms_per_orbit": round(ms_orbit_c, 2),
                                           "speedup": round(ms_plain / ms_orbit_c, 3),
                                           "max_pixel_difference": round(dmax, 5)}
        e0, e1 = chained["every_side_entry"]["without_cap_model"], chained["every_side_entry"]["with_cap_model"]
        log(f"surrogate render with the cap model (every side entry offered): accepted {e1['accepted_per_frame']} "
            f"vs {e0['accepted_per_frame']} per frame, {e1['ms_per_frame']} vs {e0['ms_per_frame']} ms/frame; "
            f"orbit at the best setting {ms_orbit_c:.0f} ms, max pixel difference {dmax:.5f}")
    del out_s
    return {"workload": (f"the orbit render with rt_render_surrogate; sweep on {nf_sub} frames, then the whole "
                         f"orbit with the fastest setting within 1/255 per pixel of the plain render"),
            "plain_ms_per_frame_sweep_frames": round(ms_plain_sub, 2), "sweep": sweep, "best": best,
            "orbit": full, "chained_cap_model": chained}


def render1024_record(args, log):
    """Sub-record: the 1024^2 render (both cloaks, elevations 0/15/30/45 deg,
    1 sample per pixel, both branches) replayed from render plans on 3
    overlapping streams, launch shape from the autotuner."""
    from paper_1209_6038_amd import workloads as W
    return _plan_record(args, log, W.render_views(res=1024), "render_1024",
                        ("3-D render: radial + azimuthal cloaks (height 4), 4 elevations x 1024^2 px, 1 spp, "
                         "ordinary + extraordinary, DP45 tol 1e-8, FP64, render plans on 3 streams"),
                        cpu_stride=4)


def batched_record(args, log):
    """Sub-record: 64 seeded views x 512^2 (azimuth U[0, 2 pi), elevation
    U[0, 60] deg), both cloaks and branches, one HIP-graph replay per step."""
    from paper_1209_6038_amd import workloads as W
    return _plan_record(args, log, W.batched_views(64, 512), "batched",
                        ("batched: 64 seeded views x 512^2 px (azimuth U[0,2pi), elevation U[0,60] deg), radial + "
                         "azimuthal cloaks, ordinary + extraordinary, DP45 tol 1e-8, FP64, one HIP-graph replay "
                         "per step, plans on 3 streams"),
                        cpu_stride=64)


def _plan_record(args, log, cams, name, desc, cpu_stride):
    import numpy as np
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    dev = torch.device("cuda", 0)
    res = int(cams[0]["w"])
    opts = W.render_opts(block=args.block, refill_period=args.refill)
    cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
    room = W.room()
    out = torch.empty((2, len(cams), 2, res, res, 3), dtype=torch.float32, device=dev)
    # launch shape from the autotuner, unless given
    tuned_ms = None
    if not (args.block or args.refill):
        opts, tuned_ms = rt.autotune_render(cloaks, opts, room, cams, 3)
    opts["block"], opts["refill_period"] = opts.get("block") or 256, opts.get("refill_period") or 2
    nstreams = 3
    plans = [rt.RenderPlan(cloaks, opts, room, cams, 3) for _ in range(nstreams)]
    streams = [torch.cuda.Stream() for _ in range(nstreams)]

    def step(k):
        with torch.cuda.stream(streams[k % nstreams]):
            plans[k % nstreams].launch()

    _, aux = rt.render_multi(cloaks, opts, room, cams, 3, aux=("status", "nsteps"))
    torch.cuda.synchronize()
    st = aux["status"].cpu().numpy()
    ns = aux["nsteps"].cpu().numpy().astype(np.int64)
    del aux
    entered = int(np.isin(st, ENTERED).sum())
    flops = sum(int(ns[ci, :, pi].sum()) * attempt_flops(2 * ci + pi, 1) for ci in range(2) for pi in range(2))
    camera_rays = 2 * len(cams) * 2 * res * res
    steps = max(5, args.steps // 2)
    for k in range(nstreams + 2):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    rt.render_multi(cloaks, opts, room, cams, 3, out=out)
    torch.cuda.synchronize()
    images_equal = all(torch.equal(p.rgb, out) for p in plans)
    for p in plans:
        p.close()
    del plans
    rt.profile_enable(True)
    rt.profile_read()
    for _ in range(3):
        rt.render_multi(cloaks, opts, room, cams, 3, out=out)
    torch.cuda.synchronize()
    transit_ms, launches = rt.profile_read()
    rt.profile_enable(False)
    avg = transit_ms / max(1, launches)
    achieved = flops / (avg * 1e-3) / 1e12
    rec = {"metric": "Mrays/s traced through cloak at ≤1e-6 exit error", "unit": "Mrays/s",
           "value": round(entered / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4), "steps": steps,
           "config": {"workload": desc, "launch_shape": {"block": opts.get("block"),
                                                         "refill_period": opts.get("refill_period"),
                                                         "autotuned_ms": tuned_ms},
                      "miss_fraction": round(1.0 - entered / camera_rays, 4), "camera_rays_per_step": camera_rays,
                      "rays_entering_cloak_per_step": entered, "images_equal_across_streams": images_equal},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                        "traffic": traffic_for(name, (opts.get("block"), opts.get("refill_period"))),
                        "kernel": "k_transit (integrator)",
                        "avg_launch_ms": round(avg, 4)}}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(W.opts_dp45(), cams, cpu_stride)
    log(f"{name}: {ms:.2f} ms per step, {rec['value']} M entering rays/s, FP64 roofline {rec['roofline']['frac']}")
    for c in cloaks:
        c.close()
    return rec


def profile_launches(args):
    """Only `--profile-launches N` integrator launches of the workload (after
    one warm-up launch), for rocprofv3 counter runs."""
    import torch
    from paper_1209_6038_amd import rt
    from paper_1209_6038_amd import workloads as W
    n = args.profile_launches
    if args.workload == "orbit":
        frames, groups, opts, cloaks, room = orbit_setup(args)
        fpl = args.frames_per_launch
        out = torch.empty((2, fpl, 2, 4096, 4096, 3), dtype=torch.float32, device="cuda")
        for k in range(n + 1):
            rt.render_multi(cloaks, opts, room, groups[k % len(groups)], 3, out=out)
    else:
        cams = W.render_views(res=1024) if args.workload == "render_1024" else W.batched_views(64, 512)
        cloaks = [rt.Cloak(W.cloak(a, height=W.HEIGHT)) for a in (0, 1)]
        opts = W.render_opts(block=args.block, refill_period=args.refill)
        for _ in range(n + 1):
            rt.render_multi(cloaks, opts, W.room(), cams, 3)
    torch.cuda.synchronize()
    return {"profile_launches": n, "workload": args.workload}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed orbits (steps of the headline)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=36, help="orbit frames per step (the workload has 36)")
    ap.add_argument("--orbit-streams", type=int, default=2, choices=(1, 2, 3, 4),
                    help="streams the orbit's launch groups rotate over (the library keeps a workspace for each "
                         "of up to four)")
    ap.add_argument("--frames-per-launch", type=int, default=2,
                    help="4096^2 x 4 spp frames per integrator launch (1-4)")
    ap.add_argument("--workload", choices=("orbit", "render_1024", "batched", "inplane",
                                           "hamiltonian", "weights", "unpolarized", "train", "surrogate"),
                    default="orbit")
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-stride", type=int, default=64, help="oracle sample stride on orbit frame 0")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="headline only, no sub-records")
    ap.add_argument("--profile-launches", type=int, default=0,
                    help="only run this many integrator launches of --workload (orbit, render_1024, batched)")
    ap.add_argument("--surrogate-steps", type=int, default=10000,
                    help="AdamW steps of 65,536 rows (10,000 = 65 epochs of the 10 M labelled rays)")
    ap.add_argument("--surrogate-train", type=int, default=10_000_000)
    ap.add_argument("--train-steps", type=int, default=300, help="timed AdamW steps of --workload train")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if not 1 <= args.frames_per_launch <= 4:
        ap.error("--frames-per-launch must be in 1..4 (at most 2^28 samples per launch)")
    if not 1 <= args.frames <= 36 or args.frames % args.frames_per_launch:
        ap.error("--frames must be in 1..36 and a multiple of --frames-per-launch")
    if args.orbit_streams * args.frames_per_launch > 6:
        ap.error("--orbit-streams x --frames-per-launch must be at most 6: each stream's workspace takes "
                 "~35 GB per frame of a launch, and the orbit's pixels another ~29 GB of the 288 GB")
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; across GPUs the render would shard by camera or image "
              "tile (no exchange but the image gather), which is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1209_6038_amd import build as B
    from paper_1209_6038_amd import rt

    if not os.path.exists(rt.LIB_PATH):
        B.build()
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.profile_launches:
        print(json.dumps(profile_launches(args)), flush=True)
        return
    single = {"inplane": inplane_workload, "hamiltonian": hamiltonian_workload, "weights": weights_workload,
              "unpolarized": unpolarized_workload, "train": train_workload,
              "surrogate": lambda a: surrogate_leg(a.surrogate_steps, a.surrogate_train, log)}
    if args.workload in single:
        print(json.dumps(finite_json(single[args.workload](args))), flush=True)
        return
    if args.workload in ("render_1024", "batched"):
        fn = render1024_record if args.workload == "render_1024" else batched_record
        print(json.dumps(finite_json(fn(args, log))), flush=True)
        return

    rec, out_plain, orbit = orbit_headline(args, log)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = orbit_cpu_baseline(orbit[0][0], args.cpu_stride)
        log(f"cpu baseline: {rec['cpu_baseline']['value']:.4f} Mrays/s on {rec['cpu_baseline']['cores']} threads")
    if not args.no_surrogate:
        sur, model, cal = surrogate_leg(args.surrogate_steps, args.surrogate_train, log, keep=True)
        sur["cap_job"], cap_model = cap_leg(model, log)
        sur["render"] = orbit_surrogate(model, orbit, out_plain, rec["ms_per_step"], log, cal, cap_model=cap_model)
        rec["surrogate"] = sur
        cap_model.close()
        model.close()
        del cal
    del out_plain, orbit
    rt.release_workspace()
    torch.cuda.empty_cache()
    if not args.no_sub:
        rec["sub"] = {"render_1024": render1024_record(args, log), "batched": batched_record(args, log),
                      "inplane": inplane_workload(args), "train": train_workload(args)}
    print(json.dumps(finite_json(rec)), flush=True)


if __name__ == "__main__":
    main()
