"""ctypes binding of the C ABI in include/rt.h (argument marshalling only).

Device memory comes from torch tensors on the current HIP device and work is
enqueued on torch's current stream; every step of the computation runs in the
HIP library. There is no fallback: if the library is missing or no GPU is
present, calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_cloak.so")

RT_OK, RT_E_INVALID, RT_E_NOMEM, RT_E_DEVICE, RT_E_UNSUPPORTED = range(5)
RADIAL, AZIMUTHAL = 0, 1
ORDINARY, EXTRAORDINARY = 0, 1
RK4, DP45 = 0, 1
FP64, MIXED = 0, 1
STATUS_NAMES = ["EXITED", "MISSED", "ABSORBED", "MAXSTEPS", "DIVERGED", "TIR", "INVALID", "REFLECTED"]

EXPORTED = ["rt_build_cloak", "rt_free_cloak", "rt_trace_batch", "rt_render", "rt_render_multi",
            "rt_render_plan_create", "rt_render_plan_launch", "rt_render_plan_destroy",
            "rt_autotune_render", "rt_profile_enable", "rt_profile_read", "rt_release_workspace",
            "rt_last_error"]


class RtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


class CloakDesc(ctypes.Structure):
    _fields_ = [("r1", ctypes.c_double), ("r2", ctypes.c_double),
                ("z0", ctypes.c_double), ("z1", ctypes.c_double),
                ("axis", ctypes.c_int32), ("inner_mirror", ctypes.c_int32)]


class TraceOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("h", ctypes.c_double), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("hmax", ctypes.c_double), ("fp64_band", ctypes.c_double),
                ("r_out", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("max_bounces", ctypes.c_int32), ("block", ctypes.c_int32),
                ("refill_period", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("look", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_deg", ctypes.c_double),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class Room(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("tile", ctypes.c_double), ("rgb", ctypes.c_float * 36)]


class RenderAux(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_void_p), ("status", ctypes.c_void_p), ("code", ctypes.c_void_p),
                ("nsteps", ctypes.c_void_p)]


_lib = None


def lib():
    """Load librt_cloak.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1209_6038_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.rt_build_cloak.argtypes = [ctypes.POINTER(CloakDesc), ctypes.POINTER(vp)]
        L.rt_free_cloak.argtypes = [vp]
        L.rt_trace_batch.argtypes = [vp, ctypes.POINTER(TraceOpts), i32, i64, vp, vp, vp, vp, vp, vp, vp]
        L.rt_render.argtypes = [vp, ctypes.POINTER(TraceOpts), ctypes.POINTER(Room),
                                ctypes.POINTER(Camera), i32, i32, vp, ctypes.POINTER(RenderAux), vp]
        L.rt_render_multi.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts),
                                      ctypes.POINTER(Room), ctypes.POINTER(Camera), i32, i32, vp,
                                      ctypes.POINTER(RenderAux), vp]
        L.rt_render_plan_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts),
                                            ctypes.POINTER(Room), ctypes.POINTER(Camera), i32, i32, vp,
                                            ctypes.POINTER(RenderAux), ctypes.POINTER(vp)]
        L.rt_render_plan_launch.argtypes = [vp, vp]
        L.rt_render_plan_destroy.argtypes = [vp]
        L.rt_autotune_render.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts),
                                         ctypes.POINTER(Room), ctypes.POINTER(Camera), i32, i32, vp,
                                         ctypes.POINTER(TraceOpts), ctypes.POINTER(ctypes.c_double)]
        L.rt_release_workspace.argtypes = []
        L.rt_profile_enable.argtypes = [i32]
        L.rt_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.rt_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            getattr(L, name).restype = ctypes.c_char_p if name == "rt_last_error" else ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code != RT_OK:
        raise RtError(code, lib().rt_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def cloak_desc(d: dict) -> CloakDesc:
    return CloakDesc(float(d["r1"]), float(d["r2"]), float(d.get("z0", -math.inf)),
                     float(d.get("z1", math.inf)), int(d["axis"]), int(d.get("inner_mirror", 1)))


def trace_opts(d: dict) -> TraceOpts:
    return TraceOpts(int(d.get("scheme", RK4)), int(d.get("precision", FP64)),
                     float(d.get("h", 1e-3)), float(d.get("rtol", 1e-8)), float(d.get("atol", 1e-8)),
                     float(d.get("hmax", 0.5)), float(d.get("fp64_band", 0.05)),
                     float(d.get("r_out", 3.0)), int(d.get("max_steps", 1_000_000)),
                     int(d.get("max_bounces", 4)), int(d.get("block", 0)),
                     int(d.get("refill_period", 0)), 0)


def camera(d: dict) -> Camera:
    c = Camera()
    c.eye[:] = [float(v) for v in d["eye"]]
    c.look[:] = [float(v) for v in d["look"]]
    c.up[:] = [float(v) for v in d["up"]]
    c.fov_deg = float(d["fov_deg"])
    c.w, c.h, c.spp = int(d["w"]), int(d["h"]), int(d.get("spp", 1))
    c.seed = int(d.get("seed", 0)) & ((1 << 64) - 1)
    return c


def room(d: dict) -> Room:
    r = Room()
    r.lo[:] = [float(v) for v in d["lo"]]
    r.hi[:] = [float(v) for v in d["hi"]]
    r.tile = float(d["tile"])
    r.rgb[:] = [float(v) for v in np.asarray(d["rgb"], dtype=np.float32).reshape(-1)]
    return r


class Cloak:
    """Owning wrapper of an rt_cloak handle."""

    def __init__(self, desc: dict):
        self.desc = dict(desc)
        h = ctypes.c_void_p()
        _check(lib().rt_build_cloak(ctypes.byref(cloak_desc(desc)), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().rt_free_cloak(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_batch(cloak: Cloak, opts: dict, pol: int, in6, with_aux: bool = True):
    """rt_trace_batch on a float64 CUDA tensor in6 of shape (6, n).

    Returns dict(out=(6, n) float64, opl, status int32[, hres, nsteps]) of
    device tensors (asynchronous on the current stream)."""
    import torch
    assert in6.is_cuda and in6.dtype == torch.float64 and in6.dim() == 2 and in6.shape[0] == 6
    in6 = in6.contiguous()
    n = in6.shape[1]
    dev = in6.device
    out = torch.empty((6, n), dtype=torch.float64, device=dev)
    opl = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    hres = torch.empty(n, dtype=torch.float64, device=dev) if with_aux else None
    ns = torch.empty(n, dtype=torch.int32, device=dev) if with_aux else None
    o = trace_opts(opts)
    _check(lib().rt_trace_batch(cloak.handle, ctypes.byref(o), int(pol), int(n), _ptr(in6), _ptr(out),
                                _ptr(opl), _ptr(st), _ptr(hres), _ptr(ns), _stream()))
    r = {"out": out, "opl": opl, "status": st}
    if with_aux:
        r["hres"] = hres
        r["nsteps"] = ns
    return r


def render_multi(cloaks: list, opts: dict, room_d: dict, cams: list, pol_mask: int,
                 aux: bool = False, out=None):
    """rt_render_multi: the same views for several cloaks (sharing geometry) in
    one pass. Returns rgb float32 (n_cloaks, n_cams, npol, h, w, 3) and, with
    aux=True, dict(rec, status, code, nsteps) in the same image order."""
    import torch
    n = len(cams)
    ncl = max(len(cloaks), 1)
    w, h, spp = int(cams[0]["w"]), int(cams[0]["h"]), int(cams[0].get("spp", 1))
    npol = 2 if pol_mask == 3 else 1
    dev = torch.device("cuda", torch.cuda.current_device())
    rgb = out if out is not None else torch.empty((ncl, n, npol, h, w, 3), dtype=torch.float32,
                                                  device=dev)
    carr = (Camera * n)(*[camera(c) for c in cams])
    harr = (ctypes.c_void_p * max(len(cloaks), 1))(*[c.handle for c in cloaks])
    rm = room(room_d)
    o = trace_opts(opts)
    aux_s = None
    aux_t = None
    if aux:
        ns = w * h * spp
        aux_t = {"rec": torch.empty((ncl, n, npol, 7, ns), dtype=torch.float64, device=dev),
                 "status": torch.empty((ncl, n, npol, ns), dtype=torch.int32, device=dev),
                 "code": torch.empty((ncl, n, npol, ns), dtype=torch.uint8, device=dev),
                 "nsteps": torch.empty((ncl, n, npol, ns), dtype=torch.int32, device=dev)}
        aux_s = RenderAux(aux_t["rec"].data_ptr(), aux_t["status"].data_ptr(), aux_t["code"].data_ptr(),
                          aux_t["nsteps"].data_ptr())
    _check(lib().rt_render_multi(harr, len(cloaks), ctypes.byref(o), ctypes.byref(rm), carr, n,
                                 int(pol_mask), _ptr(rgb),
                                 ctypes.byref(aux_s) if aux_s is not None else None, _stream()))
    return (rgb, aux_t) if aux else rgb


def render(cloak, opts: dict, room_d: dict, cams: list, pol_mask: int, aux: bool = False,
           out=None):
    """rt_render. cloak: Cloak or None (empty room). Returns rgb float32
    (n_cams, npol, h, w, 3) and, with aux=True, dict(rec, status, code, nsteps)."""
    import torch
    n = len(cams)
    w, h, spp = int(cams[0]["w"]), int(cams[0]["h"]), int(cams[0].get("spp", 1))
    npol = 2 if pol_mask == 3 else 1
    dev = torch.device("cuda", torch.cuda.current_device())
    rgb = out if out is not None else torch.empty((n, npol, h, w, 3), dtype=torch.float32, device=dev)
    carr = (Camera * n)(*[camera(c) for c in cams])
    rm = room(room_d)
    o = trace_opts(opts)
    aux_s = None
    aux_t = None
    if aux:
        ns = w * h * spp
        aux_t = {"rec": torch.empty((n, npol, 7, ns), dtype=torch.float64, device=dev),
                 "status": torch.empty((n, npol, ns), dtype=torch.int32, device=dev),
                 "code": torch.empty((n, npol, ns), dtype=torch.uint8, device=dev),
                 "nsteps": torch.empty((n, npol, ns), dtype=torch.int32, device=dev)}
        aux_s = RenderAux(aux_t["rec"].data_ptr(), aux_t["status"].data_ptr(), aux_t["code"].data_ptr(),
                          aux_t["nsteps"].data_ptr())
    _check(lib().rt_render(cloak.handle if cloak is not None else None, ctypes.byref(o),
                           ctypes.byref(rm), carr, n, int(pol_mask), _ptr(rgb),
                           ctypes.byref(aux_s) if aux_s is not None else None, _stream()))
    return (rgb, aux_t) if aux else rgb


def _alloc_render_outputs(ncl, cams, pol_mask, aux, out=None):
    import torch
    n = len(cams)
    w, h, spp = int(cams[0]["w"]), int(cams[0]["h"]), int(cams[0].get("spp", 1))
    npol = 2 if pol_mask == 3 else 1
    dev = torch.device("cuda", torch.cuda.current_device())
    rgb = out if out is not None else torch.empty((ncl, n, npol, h, w, 3), dtype=torch.float32,
                                                  device=dev)
    aux_t = aux_s = None
    if aux:
        ns = w * h * spp
        aux_t = {"rec": torch.empty((ncl, n, npol, 7, ns), dtype=torch.float64, device=dev),
                 "status": torch.empty((ncl, n, npol, ns), dtype=torch.int32, device=dev),
                 "code": torch.empty((ncl, n, npol, ns), dtype=torch.uint8, device=dev),
                 "nsteps": torch.empty((ncl, n, npol, ns), dtype=torch.int32, device=dev)}
        aux_s = RenderAux(aux_t["rec"].data_ptr(), aux_t["status"].data_ptr(), aux_t["code"].data_ptr(),
                          aux_t["nsteps"].data_ptr())
    return rgb, aux_t, aux_s


class RenderPlan:
    """rt_render_plan_*: a batch of views captured once into a HIP graph.

    Owns its output tensors (rgb, and aux if requested); launch() replays the
    graph on torch's current stream and overwrites them."""

    def __init__(self, cloaks: list, opts: dict, room_d: dict, cams: list, pol_mask: int,
                 aux: bool = False):
        self.rgb, self.aux, aux_s = _alloc_render_outputs(max(len(cloaks), 1), cams, pol_mask, aux)
        carr = (Camera * len(cams))(*[camera(c) for c in cams])
        harr = (ctypes.c_void_p * max(len(cloaks), 1))(*[c.handle for c in cloaks])
        self._cloaks = list(cloaks)  # keep the handles alive with the plan
        h = ctypes.c_void_p()
        _check(lib().rt_render_plan_create(harr, len(cloaks), ctypes.byref(trace_opts(opts)),
                                           ctypes.byref(room(room_d)), carr, len(cams), int(pol_mask),
                                           _ptr(self.rgb),
                                           ctypes.byref(aux_s) if aux_s is not None else None,
                                           ctypes.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().rt_render_plan_launch(self.handle, _stream()))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().rt_render_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_render(cloaks: list, opts: dict, room_d: dict, cams: list, pol_mask: int):
    """rt_autotune_render: returns (opts with the fastest block/refill_period,
    best milliseconds per render)."""
    rgb, _, _ = _alloc_render_outputs(max(len(cloaks), 1), cams, pol_mask, False)
    carr = (Camera * len(cams))(*[camera(c) for c in cams])
    harr = (ctypes.c_void_p * max(len(cloaks), 1))(*[c.handle for c in cloaks])
    tuned = TraceOpts()
    ms = ctypes.c_double()
    _check(lib().rt_autotune_render(harr, len(cloaks), ctypes.byref(trace_opts(opts)),
                                    ctypes.byref(room(room_d)), carr, len(cams), int(pol_mask),
                                    _ptr(rgb), ctypes.byref(tuned), ctypes.byref(ms)))
    out = dict(opts)
    out["block"] = tuned.block
    out["refill_period"] = tuned.refill_period
    return out, ms.value


def profile_enable(on: bool = True):
    _check(lib().rt_profile_enable(1 if on else 0))


def profile_read():
    """(summed integrator milliseconds, launches) since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().rt_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def release_workspace():
    _check(lib().rt_release_workspace())
