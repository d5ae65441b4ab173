"""Training, calibration and evaluation of the transit surrogate.

Orchestration only: the exact transits (rt_transit_exact), the target
encoding, every forward/backward/optimizer step, the calibration of the
trust map and the gated inference run in the HIP library; this module
chooses batches and the learning-rate schedule and measures errors.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import rt
from . import workloads as W


def exact_opts(**kw) -> dict:
    """Integration options of the surrogate workload: Dormand-Prince 5(4) at
    tolerance 1e-8 in FP64."""
    return W.opts_dp45(1e-8, r_out=W.R2, **kw)


def make_cloaks(height=None) -> list:
    """The radial and the azimuthal cloak (axis bit 0 and 1) sharing geometry."""
    return [rt.Cloak(W.cloak(a, height=height)) for a in (W.RADIAL, W.AZIMUTHAL)]


def features(n: int, seed: int, device="cuda"):
    import torch
    return torch.from_numpy(W.surrogate_features(n, seed)).to(device)


def label(cloaks, x6, opts=None, job=rt.SIDE):
    """Exact transits and training targets of entries x6 for the side or the
    cap job: (y5, status, t5, w)."""
    y5, st = rt.transit_exact(cloaks, opts or exact_opts(), x6)
    t5, w = rt.surrogate_encode(cloaks, x6, y5, st, job=job)
    return y5, st, t5, w


def compact(x6, t5, w):
    """The rows with w > 0 (contiguous SoA copies) and unit weights: for a
    job whose targets exist on few rows (the cap job's side entries that
    leave through a cap), so that every training batch is full."""
    import torch
    idx = torch.nonzero(w > 0).flatten()
    ones = torch.ones(idx.numel(), dtype=torch.float32, device=w.device)
    return x6[:, idx].contiguous(), t5[:, idx].contiguous(), ones


def cap_training_set(n: int, seed: int, opts=None):
    """Cap-job training rows from n side entries (uniform, as features) of
    the radial and azimuthal cloaks of height W.HEIGHT: (x6, t5, w) of the
    entries that leave through the cap they head for, compacted."""
    cl = make_cloaks(W.HEIGHT)
    x6 = features(n, seed)
    _, _, t5, w = label(cl, x6, opts, job=rt.CAP)
    return compact(x6, t5, w)


def exit_points(y5, b: float):
    """Exit point (3, n) and unit direction (3, n) from exit parameters."""
    import torch
    phi, z, al, be = y5[0].double(), y5[1].double(), y5[2].double(), y5[3].double()
    cp, sp = torch.cos(phi), torch.sin(phi)
    x = torch.stack([b * cp, b * sp, z])
    cb = torch.cos(be)
    d = torch.stack([cb * (torch.cos(al) * cp - torch.sin(al) * sp),
                     cb * (torch.cos(al) * sp + torch.sin(al) * cp), torch.sin(be)])
    return x, d


def exit_error(y5, y5_ref, b: float = W.R2):
    """Per-ray exit error max(|x - x_ref| / b, angle(d, d_ref)) and relative
    optical-path error."""
    import torch
    x, d = exit_points(y5, b)
    xr, dr = exit_points(y5_ref, b)
    pos = torch.linalg.vector_norm(x - xr, dim=0) / b
    ang = 2.0 * torch.asin(torch.clamp(0.5 * torch.linalg.vector_norm(d - dr, dim=0), max=1.0))
    opl = (y5[4].double() - y5_ref[4].double()).abs() / y5_ref[4].double().abs().clamp(min=1e-30)
    return torch.maximum(pos, ang), opl


def train(model, x6, t5, w, steps: int, batch: int = 8192, lr: float = 2e-3, lr_end: float = 2e-5,
          warmup: int = 200, weight_decay: float = 0.0, huber: float = 0.0, log_every: int = 0,
          log=print):
    """AdamW over contiguous batches of the (already shuffled) data set with
    linear warm-up and cosine decay of the learning rate. Returns the mean
    loss of the last 100 steps."""
    import torch
    n = x6.shape[1]
    nb = max(1, n // batch)
    loss = torch.zeros(1, dtype=torch.float32, device=x6.device)
    hist = []
    t0 = time.perf_counter()
    for k in range(steps):
        if k < warmup:
            cur = lr * (k + 1) / warmup
        else:
            f = (k - warmup) / max(1, steps - warmup)
            cur = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * f))
        j = (k % nb) * batch
        model.train_step(x6[:, j:j + batch], t5[:, j:j + batch], w[j:j + batch], lr=cur,
                         weight_decay=weight_decay, huber=huber, loss=loss)
        if k >= steps - 100 or (log_every and k % log_every == 0):
            lv = loss.item()
            if k >= steps - 100:
                hist.append(lv)
            if log_every and k % log_every == 0:
                log(f"  step {k:6d} lr {cur:.2e} loss {lv:.3e} ({time.perf_counter() - t0:.1f} s)")
    return float(np.mean(hist)) if hist else float("nan")


def summarize_errors(err, mask=None) -> dict:
    import torch
    e = err if mask is None else err[mask]
    e = e[torch.isfinite(e)]
    if e.numel() == 0:
        return {"n": 0}
    q = torch.quantile(e.float(), torch.tensor([0.5, 0.99], device=e.device)).tolist()
    return {"n": int(e.numel()), "p50": q[0], "p99": q[1], "max": float(e.max())}
