"""Pins of the FP64 cap-state geometry (tests/cap_geometry.py) that the cap
job's GPU tests compare against: the way from an exit on r = b back to the
cap point and forward again is the identity on the oracle's exits, the exit
line keeps the entry's angular momentum (tangential continuity at the cap,
Sect. 3), and for the azimuthal cloak's extraordinary branch the recovered
cap point, direction and optical path are those of the closed-form transit
of the finite cloak (tests/closed_forms.py), as is the chord model of the
path up to the cap (exact for that branch)."""
import math

import numpy as np
import pytest

from paper_1209_6038_amd import workloads as W
from tests import cap_geometry as G
from tests import closed_forms as CF
from tests.oracle_transit import oracle_exits

B, Z0, Z1 = W.R2, 0.0, W.HEIGHT


@pytest.fixture(scope="module")
def exits():
    x6 = W.surrogate_features(6000, seed=91)
    opts = W.opts_dp45(1e-10, r_out=B)
    y5, st, _ = oracle_exits([W.cloak(0, height=W.HEIGHT), W.cloak(1, height=W.HEIGHT)], opts, x6)
    cap = (st == 0) & ((y5[1] > Z1) | (y5[1] < Z0))
    return x6.astype(np.float64), y5, st, cap


def test_some_side_entries_leave_through_a_cap(exits):
    x6, y5, st, cap = exits
    kind = (x6[5] * 2 + x6[4]).astype(int)
    assert 0.05 < cap.mean() < 0.3
    # the radial cloak's ordinary branch (n = 2, |k_z| <= 1/2 inside) is
    # totally reflected at every cap it meets
    assert not cap[kind == 0].any()
    for k in (1, 2, 3):
        assert cap[kind == k].sum() > 20


def test_round_trip_and_angular_momentum(exits):
    x6, y5, _, cap = exits
    s = G.cap_state(x6[:, cap], y5[:, cap], B, Z0, Z1)
    assert (s["tb"] > 0).all()
    assert (s["rc"] >= W.R1 - 1e-9).all() and (s["rc"] <= B + 1e-9).all()
    y = G.exit_from_cap(x6[0, cap], s, B)
    xa, da = G.exit_rays(y, B)
    xb, db = G.exit_rays(y5[:, cap], B)
    assert np.abs(xa - xb).max() < 1e-9 and np.abs(da - db).max() < 1e-9
    assert np.abs(y[4] - y5[4, cap]).max() < 1e-9
    kt = np.cos(x6[3, cap]) * np.sin(x6[2, cap])
    assert np.abs(s["rc"] * s["dt"] - B * kt).max() < 1e-7


def test_azimuthal_e_cap_state_matches_the_closed_form(exits):
    x6, y5, _, cap = exits
    sel = np.flatnonzero(cap & (x6[5] == 1) & (x6[4] == 1))[:200]
    s = G.cap_state(x6[:, sel], y5[:, sel], B, Z0, Z1)
    worst = 0.0
    for j, i in enumerate(sel):
        phi, z, al, be = x6[:4, i]
        cp, sp = math.cos(phi), math.sin(phi)
        d = np.array([math.cos(be) * (-math.cos(al) * cp - math.sin(al) * sp),
                      math.cos(be) * (-math.cos(al) * sp + math.sin(al) * cp), math.sin(be)])
        o = np.array([B * cp, B * sp, z]) - d
        ev = []
        stat, p, dout, opl, _ = CF.finite_azimuthal_e(o, d, z0=Z0, z1=Z1, events=ev)
        assert stat == CF.S_EXITED and ev[-1][0] == "exit" and ev[-1][1] in (CF.TOP, CF.BOTTOM)
        zc = Z1 if ev[-1][1] == CF.TOP else Z0
        back = (p[2] - zc) / dout[2]
        xc = p - back * dout
        rc = math.hypot(xc[0], xc[1])
        th = math.atan2(xc[1], xc[0])
        dr = (xc[0] * dout[0] + xc[1] * dout[1]) / rc
        dt = (xc[0] * dout[1] - xc[1] * dout[0]) / rc
        Tc = opl - 1.0 - back
        dth = math.remainder(th - phi - s["dth"][j], 2 * math.pi)
        worst = max(worst, abs(rc - s["rc"][j]), abs(dth), abs(dr - s["dr"][j]), abs(dt - s["dt"][j]),
                    abs(abs(dout[2]) - abs(s["dz"][j])), abs(Tc - s["Tc"][j]) / max(1.0, Tc))
    assert worst < 1e-6, worst


def test_chord_model_is_exact_for_the_azimuthal_e_branch(exits):
    """For the azimuthal cloak's extraordinary branch the path is a straight
    line in (sqrt(kappa)(r - a), theta, sqrt(kappa) z) (Eq. (15)), so the
    chord model at the rise fraction u = h / |dz_0| (dz_0 from the oracle's
    infinite-cylinder transit) gives the cap state of the oracle's finite
    transit; for the other branches it is only a model (residuals of a few
    per cent of r_c)."""
    from tests.closed_forms import AZIMUTHAL, EXTRAORDINARY, ORDINARY, RADIAL
    from tests.oracle_transit import oracle_exits as ox
    x6, y5, st, cap = exits
    opts = W.opts_dp45(1e-10, r_out=B)
    for axis, branch, exact in ((AZIMUTHAL, EXTRAORDINARY, True), (RADIAL, EXTRAORDINARY, False),
                                (AZIMUTHAL, ORDINARY, False)):
        sel = np.flatnonzero(cap & (x6[5] == axis) & (x6[4] == branch))[:100]
        yi, sti, _ = ox([W.cloak(0), W.cloak(1)], opts, x6[:, sel].astype(np.float32))
        assert (sti == 0).all()
        up = x6[3, sel] >= 0
        u = np.where(up, Z1 - x6[1, sel], x6[1, sel] - Z0) / np.abs(yi[1] - x6[1, sel])
        assert (u < 1).all()
        kt = np.cos(x6[3, sel]) * np.sin(x6[2, sel])
        frac, rc, dr, adz = G.chord_state(axis, branch, kt, np.sin(x6[3, sel]), u, W.R1, B)
        s = G.cap_state(x6[:, sel], y5[:, sel], B, Z0, Z1)
        sw = np.where(x6[2, sel] < 0, -1.0, 1.0) * np.mod(np.where(x6[2, sel] < 0, -1.0, 1.0) * (yi[0] - x6[0, sel]),
                                                          2 * math.pi)
        dev = max(np.abs(rc - s["rc"]).max(), np.abs(dr - s["dr"]).max(), np.abs(adz - np.abs(s["dz"])).max(),
                  np.abs(frac * sw - s["dth"]).max())
        if exact:
            assert dev < 1e-6, dev
        else:
            assert 1e-4 < np.abs(rc - s["rc"]).max() < 0.2, np.abs(rc - s["rc"]).max()
