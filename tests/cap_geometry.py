"""FP64 geometry of the cap job's targets (test infrastructure, shares no
code with the HIP path): the state where a side entry's path leaves a cloak
of finite height through an end cap, recovered from its exit on r = b, and
the way back from that state to the exit on r = b.

Between the cap point and r = b the ray is a straight vacuum line, so the
cap point is the exit point moved back along the exit direction to the cap
plane. The cap's refraction keeps the tangential wave vector (k_r, k_theta)
of Sect. 3, and the vacuum direction's azimuthal component there is the
conserved angular momentum over the radius."""
import math

import numpy as np


def exit_rays(y5, b):
    """Exit point and unit direction (3, n) from exit parameters
    (phi', z', alpha', beta', T) on r = b."""
    phi, z, al, be = (np.asarray(y5[k], float) for k in range(4))
    cp, sp = np.cos(phi), np.sin(phi)
    x = np.stack([b * cp, b * sp, z])
    d = np.stack([np.cos(be) * (np.cos(al) * cp - np.sin(al) * sp),
                  np.cos(be) * (np.cos(al) * sp + np.sin(al) * cp), np.sin(be)])
    return x, d


def cap_state(x6, y5, b, z0, z1):
    """Cap state of exits beyond a cap (z' > z1 or z' < z0): dict of the
    swept azimuth dth from the entry azimuth to the cap point (the sign of
    alpha, unwrapped), radius rc, vacuum direction components dr, dt, dz
    (cylindrical at the cap point), optical path Tc up to the cap point, the
    cap height zc and the vacuum leg tb from the cap point to r = b."""
    x, d = exit_rays(y5, b)
    zc = np.where(np.asarray(y5[1], float) > z1, z1, z0)
    tb = (x[2] - zc) / d[2]
    c = x - tb * d
    rc = np.hypot(c[0], c[1])
    th = np.arctan2(c[1], c[0])
    s = np.where(np.asarray(x6[2]) < 0, -1.0, 1.0)
    dth = s * np.mod(s * (th - np.asarray(x6[0], float)), 2.0 * math.pi)
    dth = np.where(s * dth > 2.0 * math.pi - 1e-3, dth - s * 2.0 * math.pi, dth)
    dr = (c[0] * d[0] + c[1] * d[1]) / rc
    dt = (c[0] * d[1] - c[1] * d[0]) / rc
    return {"dth": dth, "rc": rc, "dr": dr, "dt": dt, "dz": d[2], "Tc": np.asarray(y5[4], float) - tb,
            "zc": zc, "tb": tb}


def exit_from_cap(phi, st, b):
    """Exit parameters on r = b of the vacuum ray leaving the cap point of
    state st (cap_state's keys) for an entry at azimuth phi."""
    th = np.asarray(phi, float) + st["dth"]
    rc = st["rc"]
    c = np.stack([rc * np.cos(th), rc * np.sin(th), st["zc"]])
    d = np.stack([st["dr"] * np.cos(th) - st["dt"] * np.sin(th),
                  st["dr"] * np.sin(th) + st["dt"] * np.cos(th), st["dz"]])
    qa = d[0] ** 2 + d[1] ** 2
    qb = c[0] * d[0] + c[1] * d[1]
    qc = rc ** 2 - b * b
    s = (-qb + np.sqrt(qb * qb - qa * qc)) / qa
    p = c + s * d
    ph = np.mod(np.arctan2(p[1], p[0]), 2.0 * math.pi)
    vr = d[0] * np.cos(ph) + d[1] * np.sin(ph)
    vt = d[1] * np.cos(ph) - d[0] * np.sin(ph)
    return np.stack([ph, p[2], np.arctan2(vt, vr), np.arcsin(np.clip(d[2], -1.0, 1.0)), st["Tc"] + s])


def chord_state(axis, branch, kt, kz, u, a, b):
    """Chord model of the infinite-cylinder path up to rise fraction u (the
    cap job's baselines): the straight chord through the entry with the
    path's impact parameter, traversed to u; returns (frac, rc, dr, adz):
    the share of the whole sweep, the radius, the radial wave number from
    the dispersion relation there (sign of the leg: inwards for u < 1/2)
    and |d_z| of the vacuum direction after the cap. For the azimuthal
    cloak's extraordinary branch the chord lives in rho = sqrt(kappa)(r - a),
    where the path is straight (Eq. (15)); for the radial extraordinary and
    azimuthal ordinary branches the impact parameter is the turning radius,
    the larger root of kappa (r - a)^2 - p^2 - k_z^2 r^2 (p = b k_theta)."""
    from tests.closed_forms import AZIMUTHAL, EXTRAORDINARY, cyl_metric, kappa
    kap = kappa(a, b)
    kt = np.abs(np.asarray(kt, float))
    kz = np.asarray(kz, float)
    u = np.asarray(u, float)
    p = b * kt
    straight = axis == AZIMUTHAL and branch == EXTRAORDINARY
    if straight:
        w = b * kt / np.sqrt(1.0 - kz * kz / kap)
    else:
        w = np.empty_like(kt)
        for i in range(kt.size):  # larger root of the quadratic, numerically
            roots = np.roots([kap - kz[i] ** 2, -2.0 * kap * a, kap * a * a - p[i] ** 2])
            w[i] = np.max(roots.real)
    w = np.minimum(w, b)
    wb = np.sqrt(np.maximum(b * b - w * w, 0.0))
    rr = np.sqrt(w * w + wb * wb * (1.0 - 2.0 * u) ** 2)
    rc = a + rr / math.sqrt(kap) if straight else rr
    half = np.arctan2(wb, w)
    frac = (np.arctan2(wb * (2.0 * u - 1.0), w) + half) / (2.0 * half)
    mr, mt, mz = np.empty_like(rc), np.empty_like(rc), np.empty_like(rc)
    for i in range(rc.size):
        (mr[i], mt[i], mz[i]), _ = cyl_metric(axis, branch, rc[i], a, b)
    kth = p / rc
    kr2 = mr * (1.0 - kth * kth / mt - kz * kz / mz)
    dr = np.where(u < 0.5, -1.0, 1.0) * np.sqrt(np.maximum(kr2, 0.0))
    adz = np.sqrt(np.maximum(1.0 - dr * dr - kth * kth, 0.0))
    return frac, rc, dr, adz
