"""Shared helpers of the GPU parity tests (GPU side through the C ABI binding,
reference side through the oracle)."""
from __future__ import annotations

import math
import sys

import numpy as np

POS_TOL = 1e-6   # exit position error in units of R2
DIR_TOL = 1e-6   # exit direction error in radians
R2 = 2.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_trace(cloak_d, opts, branch, rays, with_trans=False):
    import torch
    from paper_1209_6038_amd import rt
    c = rt.Cloak(cloak_d)
    t = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    r = rt.trace_batch(c, opts, branch, t, with_trans=with_trans)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    c.close()
    return out


def angle_between(a, b):
    """Angle (rad) between direction columns of (3, n) arrays."""
    cr = np.linalg.norm(np.cross(a.T, b.T), axis=1)
    dt = np.einsum("ij,ij->j", a, b)
    return np.arctan2(cr, dt)


def trace_errors(g, o):
    dpos = np.linalg.norm(g["out"][:3] - o["out"][:3], axis=0) / R2
    ddir = angle_between(g["out"][3:], o["out"][3:])
    dopl = np.abs(g["opl"] - o["opl"])
    return dpos, ddir, dopl


def check_trace(g, o, mask=None, pos_tol=POS_TOL, dir_tol=DIR_TOL, opl_tol=None, label=""):
    """Status equal on `mask` (default all) and exit rays within tolerance."""
    n = len(o["status"])
    mask = np.ones(n, bool) if mask is None else mask
    same = g["status"] == o["status"]
    bad = np.flatnonzero(mask & ~same)
    assert bad.size == 0, f"{label}: status differs at {bad[:10]}: gpu {g['status'][bad[:10]]} oracle {o['status'][bad[:10]]}"
    ok = mask & np.isin(o["status"], (0, 1, 7))
    dpos, ddir, dopl = trace_errors(g, o)
    say(f"{label}: n={ok.sum()} max pos/R2={dpos[ok].max(initial=0):.3e} "
        f"max dir={ddir[ok].max(initial=0):.3e} rad max opl={dopl[ok].max(initial=0):.3e}")
    assert dpos[ok].max(initial=0) <= pos_tol, label
    assert ddir[ok].max(initial=0) <= dir_tol, label
    if opl_tol is not None:
        assert dopl[ok].max(initial=0) <= opl_tol, label
    return dpos, ddir, dopl
