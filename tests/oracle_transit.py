"""The oracle's transit in the surrogate's entry/exit parameters (test
infrastructure)."""
import math

import numpy as np

import oracle


def oracle_exit_params(cloak_d, opts, x6):
    """Oracle transit of entries x6 (float32 (6, n), one (axis, branch) pair
    per call): vacuum rays starting one unit outside the entry point, traced
    to r = r2, converted to exit parameters (phi', z', alpha', beta', T)."""
    b = cloak_d["r2"]
    phi, z, al, be = (x6[k].astype(np.float64) for k in range(4))
    cp, sp = np.cos(phi), np.sin(phi)
    d = np.stack([np.cos(be) * (-np.cos(al) * cp - np.sin(al) * sp),
                  np.cos(be) * (-np.cos(al) * sp + np.sin(al) * cp), np.sin(be)])
    p = np.stack([b * cp, b * sp, z])
    rays = np.concatenate([p - d, d])
    o = oracle.trace(cloak_d, dict(opts, r_out=b), int(x6[4, 0]), rays)
    out = o["out"]
    ph = np.mod(np.arctan2(out[1], out[0]), 2 * math.pi)
    rl = np.hypot(out[0], out[1])
    vr = (out[0] * out[3] + out[1] * out[4]) / rl
    vt = (out[0] * out[4] - out[1] * out[3]) / rl
    y5 = np.stack([ph, out[2], np.arctan2(vt, vr), np.arcsin(np.clip(out[5], -1, 1)), o["opl"] - 1.0])
    return y5, o["status"], o["hres"]


def oracle_exits(cloaks_d, opts, x6):
    """oracle_exit_params over mixed (axis, branch) rows: cloaks_d[axis]."""
    n = x6.shape[1]
    y5 = np.full((5, n), np.nan)
    st = np.full(n, -1, dtype=np.int64)
    hr = np.full(n, np.nan)
    for axis in (0, 1):
        for pol in (0, 1):
            idx = np.flatnonzero((x6[4] == pol) & (x6[5] == axis))
            if idx.size:
                y5[:, idx], st[idx], hr[idx] = oracle_exit_params(cloaks_d[axis], opts, x6[:, idx])
    return y5, st, hr
