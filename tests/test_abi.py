"""Host-side checks of the C ABI (no GPU needed, no compute calls)."""
import ctypes
import math
import os
import re
import subprocess
import tempfile

import pytest

from paper_1209_6038_amd import build as B
from paper_1209_6038_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


@pytest.fixture(scope="module")
def lib():
    if B.is_stale():
        B.build()
    return rt.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rt_build_cloak", "rt_trace_batch", "rt_render", "rt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", rt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(rt_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_struct_layouts_match_header():
    """Compile the header with gcc and compare sizeof/offsetof with ctypes."""
    fields = {
        "rt_cloak_desc": (rt.CloakDesc, ["r1", "z0", "axis", "inner_mirror"]),
        "rt_trace_opts": (rt.TraceOpts, ["scheme", "h", "fp64_band", "r_out", "max_steps",
                                         "max_bounces", "refill_period", "max_chunk"]),
        "rt_camera": (rt.Camera, ["eye", "fov_deg", "w", "spp", "seed"]),
        "rt_room": (rt.Room, ["lo", "tile", "rgb"]),
        "rt_render_aux": (rt.RenderAux, ["rec", "status", "code", "nsteps", "tof", "unpol", "goggle_inplane",
                                         "goggle_axial", "reflections"]),
        "rt_train_opts": (rt.TrainOpts, ["lr", "eps", "weight_decay"]),
        "rt_gate_opts": (rt.GateOpts, ["tol", "hres_max", "cap_margin", "min_count", "dilate", "unresolved", "p_min"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for s, (_, fs) in fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-o", exe, c], check=True)
        got = dict(l.split() for l in subprocess.run([exe], capture_output=True, text=True,
                                                     check=True).stdout.splitlines())
    for s, (cls, fs) in fields.items():
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fs:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, f"{s}.{f}"


def test_argument_validation_needs_no_gpu(lib):
    """Invalid descriptions are rejected synchronously before any device use."""
    h = ctypes.c_void_p()
    bad = rt.CloakDesc(2.0, 1.0, -1e300, 1e300, 0, 1)
    assert lib.rt_build_cloak(ctypes.byref(bad), ctypes.byref(h)) == rt.RT_E_INVALID
    assert b"r1 < r2" in lib.rt_last_error()
    bad = rt.CloakDesc(1.0, 2.0, 0.0, 4.0, 7, 1)
    assert lib.rt_build_cloak(ctypes.byref(bad), ctypes.byref(h)) == rt.RT_E_INVALID
    good = rt.CloakDesc(1.0, 2.0, 0.0, 4.0, 1, 1)
    assert lib.rt_build_cloak(ctypes.byref(good), ctypes.byref(h)) == rt.RT_OK
    o = rt.trace_opts({"scheme": 1, "h": 1e-2, "hmax": 1e-3})
    assert lib.rt_trace_batch(h, ctypes.byref(o), 1, 10, None, None, None, None, None, None,
                              None, None) == rt.RT_E_INVALID
    o = rt.trace_opts({"scheme": 0, "h": 1e-3, "r_out": 1.5})
    assert lib.rt_trace_batch(h, ctypes.byref(o), 1, 10, ctypes.c_void_p(8), ctypes.c_void_p(8),
                              ctypes.c_void_p(8), ctypes.c_void_p(8), None, None, None, None) == rt.RT_E_INVALID
    assert b"r_out" in lib.rt_last_error()
    o = rt.trace_opts({"scheme": 0, "h": 1e-3})
    assert lib.rt_trace_batch(h, ctypes.byref(o), 5, 10, ctypes.c_void_p(8), ctypes.c_void_p(8),
                              ctypes.c_void_p(8), ctypes.c_void_p(8), None, None, None, None) == rt.RT_E_INVALID
    assert lib.rt_trace_batch(h, ctypes.byref(o), 1, 0, None, None, None, None, None, None,
                              None, None) == rt.RT_OK  # n = 0 is a no-op
    # an FP32 derivative (RT_PREC_MIXED) is rejected for every scheme, with
    # or without the Eq. (12) weights, and in the allocation-free variant;
    # scheme 4 does not exist
    for scheme, h0 in ((rt.RK4_HAM, 1e-3), (rt.DP45, 1e-2), (rt.RK4, 1e-3)):
        o = rt.trace_opts({"scheme": scheme, "precision": rt.MIXED, "h": h0, "fp64_band": 0.05})
        for trans in (None, ctypes.c_void_p(8)):
            for fn in (lib.rt_trace_batch, lib.rt_trace_batch_noalloc):
                assert fn(h, ctypes.byref(o), 1, 10, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), None, None, trans, None) == rt.RT_E_UNSUPPORTED
                assert b"RT_PREC_FP64" in lib.rt_last_error()
    # the allocation-free variant holds at most RT_NOALLOC_MAX_RAYS rays
    o = rt.trace_opts({"scheme": rt.DP45, "h": 1e-2})
    assert lib.rt_trace_batch_noalloc(h, ctypes.byref(o), 1, rt.NOALLOC_MAX_RAYS + 1, ctypes.c_void_p(8),
                                      ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), None, None,
                                      None, None) == rt.RT_E_INVALID
    assert b"at most" in lib.rt_last_error()
    o = rt.trace_opts({"scheme": 4, "h": 1e-3})
    assert lib.rt_trace_batch(h, ctypes.byref(o), 1, 10, ctypes.c_void_p(8), ctypes.c_void_p(8),
                              ctypes.c_void_p(8), ctypes.c_void_p(8), None, None, None, None) == rt.RT_E_INVALID
    assert lib.rt_free_cloak(h) == rt.RT_OK


def test_product_path_has_no_oracle_dependency():
    """The package never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1209_6038_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "cloak_oracle" not in txt, f


def test_render_argument_validation_needs_no_gpu(lib):
    """Render arguments are checked on the host before any device use: the
    number of cloaks, the branch mask, the stratified sample count, the
    chunk limit (2^28 samples) and the surrogate model."""
    from paper_1209_6038_amd import workloads as W
    h = ctypes.c_void_p()
    good = rt.CloakDesc(1.0, 2.0, 0.0, 4.0, 0, 1)
    assert lib.rt_build_cloak(ctypes.byref(good), ctypes.byref(h)) == rt.RT_OK
    harr = (ctypes.c_void_p * 3)(h, h, h)
    room = rt.room(W.room())
    fake_rgb = ctypes.c_void_p(8)  # never dereferenced on these paths

    def render(ncl=1, cams=None, pol_mask=3, **opts):
        cams = cams or [W.orbit_camera(0.3, 20.0, 8, 8)]
        carr = (rt.Camera * len(cams))(*[rt.camera(c) for c in cams])
        o = rt.trace_opts(W.render_opts(**opts))
        return lib.rt_render_multi(harr, ncl, ctypes.byref(o), ctypes.byref(room), carr, len(cams), pol_mask,
                                   fake_rgb, None, None)

    assert render(ncl=3) == rt.RT_E_INVALID
    assert render(pol_mask=0) == rt.RT_E_INVALID
    assert render(cams=[W.orbit_camera(0.3, 20.0, 8, 8, spp=3)]) == rt.RT_E_INVALID
    assert render(max_chunk=(1 << 28) + 1) == rt.RT_E_INVALID
    assert b"max_chunk" in lib.rt_last_error()
    cams = (rt.Camera * 1)(rt.camera(W.orbit_camera(0.3, 20.0, 8, 8)))
    o = rt.trace_opts(W.render_opts())
    # first-order reflections need an image they add to, and render plans
    # do not take them
    aux = rt.RenderAux()
    aux.reflections = 1
    assert lib.rt_render_multi(harr, 1, ctypes.byref(o), ctypes.byref(room), cams, 1, 3, fake_rgb,
                               ctypes.byref(aux), None) == rt.RT_E_INVALID
    assert b"reflections" in lib.rt_last_error()
    aux.unpol = 8
    plan = ctypes.c_void_p()
    assert lib.rt_render_plan_create(harr, 1, ctypes.byref(o), ctypes.byref(room), cams, 1, 3, fake_rgb,
                                     ctypes.byref(aux), ctypes.byref(plan)) == rt.RT_E_UNSUPPORTED
    assert b"reflections" in lib.rt_last_error()
    assert lib.rt_render_surrogate(None, harr, 1, ctypes.byref(o), ctypes.byref(room), cams, 1, 3, 0, fake_rgb,
                                   None, None, None, None) == rt.RT_E_INVALID
    assert b"model" in lib.rt_last_error()
    assert lib.rt_free_cloak(h) == rt.RT_OK


def test_cap_job_argument_validation_needs_no_gpu(lib):
    """The cap job's encoding is checked on the host: a job that does not
    exist, and cloaks of infinite height (the cap job needs end caps), are
    rejected before any device use; chaining and job changes need a model."""
    h_inf, h_fin = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.rt_build_cloak(ctypes.byref(rt.CloakDesc(1.0, 2.0, -math.inf, math.inf, 0, 1)),
                              ctypes.byref(h_inf)) == rt.RT_OK
    assert lib.rt_build_cloak(ctypes.byref(rt.CloakDesc(1.0, 2.0, 0.0, 4.0, 0, 1)), ctypes.byref(h_fin)) == rt.RT_OK
    fake = ctypes.c_void_p(8)  # never dereferenced on these paths
    for h, job, msg in ((h_fin, 2, b"RT_SUR_SIDE or RT_SUR_CAP"), (h_inf, rt.CAP, b"finite height")):
        arr = (ctypes.c_void_p * 1)(h)
        assert lib.rt_surrogate_encode_job(job, arr, 1, 10, 10, fake, fake, fake, fake, fake, None) == rt.RT_E_INVALID
        assert msg in lib.rt_last_error()
    arr = (ctypes.c_void_p * 1)(h_fin)
    assert lib.rt_surrogate_encode_job(rt.CAP, arr, 1, 0, 0, None, None, None, None, None, None) == rt.RT_OK
    assert lib.rt_surrogate_chain(None, None) == rt.RT_E_INVALID
    assert lib.rt_surrogate_set_job(None, rt.CAP, h_fin) == rt.RT_E_INVALID
    assert lib.rt_free_cloak(h_inf) == rt.RT_OK and lib.rt_free_cloak(h_fin) == rt.RT_OK
