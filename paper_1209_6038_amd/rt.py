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
RK4, DP45, RK4_HAM, RK4_HAMC = 0, 1, 2, 3
FP64, MIXED = 0, 1
STATUS_NAMES = ["EXITED", "MISSED", "ABSORBED", "MAXSTEPS", "DIVERGED", "TIR", "INVALID", "REFLECTED"]

EXPORTED = ["rt_build_cloak", "rt_free_cloak", "rt_trace_batch", "rt_render", "rt_render_multi",
            "rt_render_plan_create", "rt_render_plan_launch", "rt_render_plan_destroy",
            "rt_autotune_render", "rt_profile_enable", "rt_profile_read", "rt_release_workspace",
            "rt_last_error", "rt_cloak_get_desc", "rt_transit_exact",
            "rt_surrogate_create", "rt_surrogate_free", "rt_surrogate_nparams",
            "rt_surrogate_get_params", "rt_surrogate_set_params", "rt_surrogate_get_scaling",
            "rt_surrogate_set_scaling", "rt_surrogate_fit_scaling", "rt_surrogate_encode",
            "rt_surrogate_grad", "rt_surrogate_train", "rt_surrogate_forward",
            "rt_surrogate_calibrate", "rt_surrogate_get_map", "rt_surrogate_infer",
            "rt_surrogate_save", "rt_surrogate_load", "rt_render_surrogate", "rt_surrogate_step",
            "rt_surrogate_get_state", "rt_surrogate_set_state", "rt_trace_batch_noalloc",
            "rt_surrogate_encode_job", "rt_surrogate_set_job", "rt_surrogate_get_job", "rt_surrogate_chain"]


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
                ("refill_period", ctypes.c_int32), ("max_chunk", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("look", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_deg", ctypes.c_double),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class Room(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("tile", ctypes.c_double), ("rgb", ctypes.c_float * 36)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float), ("huber", ctypes.c_float)]


class GateOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("hres_max", ctypes.c_double),
                ("cap_margin", ctypes.c_double), ("min_count", ctypes.c_int32),
                ("dilate", ctypes.c_int32), ("unresolved", ctypes.c_double), ("p_min", ctypes.c_double)]


class RenderAux(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_void_p), ("status", ctypes.c_void_p), ("code", ctypes.c_void_p),
                ("nsteps", ctypes.c_void_p), ("tof", ctypes.c_void_p), ("unpol", ctypes.c_void_p),
                ("goggle_inplane", ctypes.c_void_p), ("goggle_axial", ctypes.c_void_p),
                ("reflections", ctypes.c_int32)]


AUX_FIELDS = ("rec", "status", "code", "nsteps", "tof")


def _render_aux(lead: tuple, w: int, h: int, spp: int, dev, fields=True):
    """Per-sample (rec, status, code, nsteps) and per-pixel (tof) render
    outputs for images of leading shape `lead`, and their rt_render_aux.
    fields: True for all of them, or the names of the ones to produce."""
    import torch
    ns = w * h * spp
    want = AUX_FIELDS if fields is True else tuple(fields)
    make = {"rec": lambda: torch.empty(lead + (7, ns), dtype=torch.float64, device=dev),
            "status": lambda: torch.empty(lead + (ns,), dtype=torch.int32, device=dev),
            "code": lambda: torch.empty(lead + (ns,), dtype=torch.uint8, device=dev),
            "nsteps": lambda: torch.empty(lead + (ns,), dtype=torch.int32, device=dev),
            "tof": lambda: torch.empty(lead + (h, w), dtype=torch.float32, device=dev)}
    aux_t = {k: make[k]() for k in want}
    aux_s = RenderAux(*(aux_t[k].data_ptr() if k in aux_t else None for k in AUX_FIELDS))
    return aux_t, aux_s


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
        L.rt_trace_batch.argtypes = [vp, ctypes.POINTER(TraceOpts), i32, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rt_trace_batch_noalloc.argtypes = [vp, ctypes.POINTER(TraceOpts), i32, i64, vp, vp, vp, vp, vp, vp,
                                             vp, vp]
        L.rt_render.argtypes = [vp, ctypes.POINTER(TraceOpts), ctypes.POINTER(Room),
                                ctypes.POINTER(Camera), i32, i32, vp, ctypes.POINTER(RenderAux), vp]
        L.rt_render_multi.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts),
                                      ctypes.POINTER(Room), ctypes.POINTER(Camera), i32, i32, vp,
                                      ctypes.POINTER(RenderAux), vp]
        L.rt_render_surrogate.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts),
                                          ctypes.POINTER(Room), ctypes.POINTER(Camera), i32, i32, i32, vp,
                                          ctypes.POINTER(RenderAux), ctypes.POINTER(i64), vp]
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
        L.rt_cloak_get_desc.argtypes = [vp, ctypes.POINTER(CloakDesc)]
        L.rt_transit_exact.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts), i64, i64,
                                       vp, vp, vp, vp, vp, vp, vp]
        L.rt_surrogate_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
        L.rt_surrogate_free.argtypes = [vp]
        L.rt_surrogate_nparams.argtypes = [ctypes.POINTER(i64)]
        L.rt_surrogate_get_params.argtypes = [vp, vp]
        L.rt_surrogate_set_params.argtypes = [vp, vp]
        L.rt_surrogate_get_scaling.argtypes = [vp, vp]
        L.rt_surrogate_set_scaling.argtypes = [vp, vp]
        L.rt_surrogate_fit_scaling.argtypes = [vp, i64, i64, vp, vp, vp, vp]
        L.rt_surrogate_encode.argtypes = [ctypes.POINTER(vp), i32, i64, i64, vp, vp, vp, vp, vp, vp]
        L.rt_surrogate_grad.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.c_float, vp, vp, vp]
        L.rt_surrogate_train.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(TrainOpts), vp, vp]
        L.rt_surrogate_forward.argtypes = [vp, i64, i64, vp, vp, vp]
        L.rt_surrogate_step.argtypes = [vp, vp, ctypes.POINTER(TrainOpts), vp]
        L.rt_surrogate_get_state.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
        L.rt_surrogate_set_state.argtypes = [vp, vp, vp, i64]
        L.rt_surrogate_calibrate.argtypes = [vp, ctypes.POINTER(vp), i32, i64, i64, vp, vp, vp, vp,
                                             ctypes.POINTER(GateOpts), ctypes.POINTER(ctypes.c_double),
                                             vp]
        L.rt_surrogate_get_map.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.rt_surrogate_encode_job.argtypes = [i32, ctypes.POINTER(vp), i32, i64, i64, vp, vp, vp, vp, vp, vp]
        L.rt_surrogate_set_job.argtypes = [vp, i32, vp]
        L.rt_surrogate_get_job.argtypes = [vp, ctypes.POINTER(i32)]
        L.rt_surrogate_chain.argtypes = [vp, vp]
        L.rt_surrogate_infer.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(TraceOpts), i64,
                                         i64, vp, vp, vp, vp, vp]
        L.rt_surrogate_save.argtypes = [vp, ctypes.c_char_p]
        L.rt_surrogate_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
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
                     int(d.get("refill_period", 0)), int(d.get("max_chunk", 0)))


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


NOALLOC_MAX_RAYS = 65536


def trace_batch(cloak: Cloak, opts: dict, pol: int, in6, with_aux: bool = True,
                with_trans: bool = False, out=None, noalloc: bool = False):
    """rt_trace_batch on a float64 CUDA tensor in6 of shape (6, n).

    Returns dict(out=(6, n) float64, opl, status int32[, hres, nsteps][, trans])
    of device tensors (asynchronous on the current stream). `trans` is the
    Eq. (12) intensity weight of each ray (FP64 options only). `out`: a dict
    of preallocated tensors of those names to write into instead.
    noalloc=True calls rt_trace_batch_noalloc (at most NOALLOC_MAX_RAYS rays;
    the library allocates nothing)."""
    import torch
    assert in6.is_cuda and in6.dtype == torch.float64 and in6.dim() == 2 and in6.shape[0] == 6
    in6 = in6.contiguous()
    n = in6.shape[1]
    dev = in6.device
    pre = out or {}
    out = pre.get("out", torch.empty((6, n), dtype=torch.float64, device=dev))
    opl = pre.get("opl", torch.empty(n, dtype=torch.float64, device=dev))
    st = pre.get("status", torch.empty(n, dtype=torch.int32, device=dev))
    hres = pre.get("hres", torch.empty(n, dtype=torch.float64, device=dev)) if with_aux else None
    ns = pre.get("nsteps", torch.empty(n, dtype=torch.int32, device=dev)) if with_aux else None
    tr = pre.get("trans", torch.empty(n, dtype=torch.float64, device=dev)) if with_trans else None
    o = trace_opts(opts)
    fn = lib().rt_trace_batch_noalloc if noalloc else lib().rt_trace_batch
    _check(fn(cloak.handle, ctypes.byref(o), int(pol), int(n), _ptr(in6), _ptr(out),
              _ptr(opl), _ptr(st), _ptr(hres), _ptr(ns), _ptr(tr), _stream()))
    r = {"out": out, "opl": opl, "status": st}
    if with_aux:
        r["hres"] = hres
        r["nsteps"] = ns
    if with_trans:
        r["trans"] = tr
    return r


def _check_out(rgb, shape):
    """The library writes the images densely from the tensor's first element."""
    import torch
    if rgb.dtype != torch.float32 or not rgb.is_cuda or not rgb.is_contiguous() or rgb.numel() != int(np.prod(shape)):
        raise ValueError(f"out must be a contiguous float32 CUDA tensor of {int(np.prod(shape))} elements "
                         f"({shape}); got {tuple(rgb.shape)}, contiguous={rgb.is_contiguous()}")


def render_multi(cloaks: list, opts: dict, room_d: dict, cams: list, pol_mask: int,
                 aux: bool = False, out=None, unpolarized: bool = False, goggles: bool = False,
                 reflections: bool = False):
    """rt_render_multi: the same views for several cloaks (sharing geometry) in
    one pass. Returns rgb float32 (n_cloaks, n_cams, npol, h, w, 3) and, with
    aux=True, dict(rec, status, code, nsteps, tof) in the same image order
    (aux = a tuple of those names: only these); with
    unpolarized=True (pol_mask 3, FP64) the dict also holds "unpol", the
    Eq. (12) unpolarized images, float32 (n_cloaks, n_cams, h, w, 3), and
    with goggles=True "goggle_inplane" and "goggle_axial", the images through
    the in-plane and the axial polarizer (same shape); reflections=True adds
    first-order reflections to those images."""
    import torch
    n = len(cams)
    ncl = max(len(cloaks), 1)
    w, h, spp = int(cams[0]["w"]), int(cams[0]["h"]), int(cams[0].get("spp", 1))
    npol = 2 if pol_mask == 3 else 1
    dev = torch.device("cuda", torch.cuda.current_device())
    rgb = out if out is not None else torch.empty((ncl, n, npol, h, w, 3), dtype=torch.float32,
                                                  device=dev)
    _check_out(rgb, (ncl, n, npol, h, w, 3))
    carr = (Camera * n)(*[camera(c) for c in cams])
    harr = (ctypes.c_void_p * max(len(cloaks), 1))(*[c.handle for c in cloaks])
    rm = room(room_d)
    o = trace_opts(opts)
    aux_s = None
    aux_t = None
    if aux:
        aux_t, aux_s = _render_aux((ncl, n, npol,), w, h, spp, dev, aux)
    for on, names in ((unpolarized, ("unpol",)), (goggles, ("goggle_inplane", "goggle_axial"))):
        if not on:
            continue
        if aux_s is None:
            aux_t, aux_s = {}, RenderAux()
        for name in names:
            aux_t[name] = torch.empty((ncl, n, h, w, 3), dtype=torch.float32, device=dev)
            setattr(aux_s, name, aux_t[name].data_ptr())
    if reflections:
        if aux_s is None:
            aux_t, aux_s = {}, RenderAux()
        aux_s.reflections = 1
    _check(lib().rt_render_multi(harr, len(cloaks), ctypes.byref(o), ctypes.byref(rm), carr, n,
                                 int(pol_mask), _ptr(rgb),
                                 ctypes.byref(aux_s) if aux_s is not None else None, _stream()))
    return (rgb, aux_t) if (aux or unpolarized or goggles or reflections) else rgb


def render_surrogate(model, cloaks: list, opts: dict, room_d: dict, cams: list, pol_mask: int,
                     aux: bool = False, out=None, counts: bool = False, min_difficulty: int = 0):
    """rt_render_surrogate: render_multi with the side-to-side transits of
    entries of difficulty >= min_difficulty taken from the calibrated
    surrogate `model` (a Surrogate) where its gate accepts them. Returns rgb
    as render_multi (then the aux dict if aux, then (candidates, accepted) if
    counts)."""
    import torch
    n = len(cams)
    ncl = len(cloaks)
    w, h, spp = int(cams[0]["w"]), int(cams[0]["h"]), int(cams[0].get("spp", 1))
    npol = 2 if pol_mask == 3 else 1
    dev = torch.device("cuda", torch.cuda.current_device())
    rgb = out if out is not None else torch.empty((ncl, n, npol, h, w, 3), dtype=torch.float32,
                                                  device=dev)
    _check_out(rgb, (ncl, n, npol, h, w, 3))
    carr = (Camera * n)(*[camera(c) for c in cams])
    harr = (ctypes.c_void_p * max(ncl, 1))(*[c.handle for c in cloaks])
    rm = room(room_d)
    o = trace_opts(opts)
    aux_s = None
    aux_t = None
    if aux:
        aux_t, aux_s = _render_aux((ncl, n, npol,), w, h, spp, dev)
    c2 = (ctypes.c_int64 * 2)(0, 0)
    _check(lib().rt_render_surrogate(model.handle, harr, ncl, ctypes.byref(o), ctypes.byref(rm), carr, n,
                                     int(pol_mask), int(min_difficulty), _ptr(rgb),
                                     ctypes.byref(aux_s) if aux_s is not None else None,
                                     c2 if counts else None, _stream()))
    out_t = (rgb,)
    if aux:
        out_t += (aux_t,)
    if counts:
        out_t += ((int(c2[0]), int(c2[1])),)
    return out_t if len(out_t) > 1 else rgb


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
    _check_out(rgb, (n, npol, h, w, 3))
    carr = (Camera * n)(*[camera(c) for c in cams])
    rm = room(room_d)
    o = trace_opts(opts)
    aux_s = None
    aux_t = None
    if aux:
        aux_t, aux_s = _render_aux((n, npol,), w, h, spp, dev)
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
    _check_out(rgb, (ncl, n, npol, h, w, 3))
    aux_t = aux_s = None
    if aux:
        aux_t, aux_s = _render_aux((ncl, n, npol,), w, h, spp, dev)
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


# ---------------------------------------------------------------------------
# transit in entry/exit parameters and the learned surrogate
# ---------------------------------------------------------------------------
def _handles(cloaks):
    return (ctypes.c_void_p * len(cloaks))(*[c.handle for c in cloaks])


def _check_soa(x, rows, dtype):
    import torch
    assert x.is_cuda and x.dtype == dtype and x.dim() == 2 and x.shape[0] == rows, (x.shape, x.dtype)
    assert x.stride(1) == 1, "SoA rows must be contiguous"
    return x.stride(0)


def transit_exact(cloaks: list, opts: dict, x6, mask=None, y5=None, status=None, nsteps=False, hres=False):
    """rt_transit_exact on float32 CUDA x6 (6, n) (entry phi, z, alpha, beta,
    branch bit, axis bit). Returns (y5 (5, n) float32, status int32), then
    hres float32 (|H - 1| at the exit) if hres, then nsteps int32 if nsteps."""
    import torch
    ld = _check_soa(x6, 6, torch.float32)
    n = x6.shape[1]
    dev = x6.device
    if y5 is None:
        y5 = torch.empty((5, ld), dtype=torch.float32, device=dev)[:, :n]
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=dev)
    assert y5.stride(0) == ld and y5.stride(1) == 1
    hr = torch.empty(n, dtype=torch.float32, device=dev) if hres else None
    ns = torch.empty(n, dtype=torch.int32, device=dev) if nsteps else None
    _check(lib().rt_transit_exact(_handles(cloaks), len(cloaks), ctypes.byref(trace_opts(opts)), n, ld,
                                  _ptr(x6), _ptr(mask), _ptr(y5), _ptr(status), _ptr(hr), _ptr(ns), _stream()))
    out = (y5, status)
    if hres:
        out += (hr,)
    if nsteps:
        out += (ns,)
    return out


SIDE, CAP = 0, 1  # surrogate jobs (RT_SUR_SIDE, RT_SUR_CAP)


def surrogate_encode(cloaks: list, x6, y5, status, job: int = SIDE):
    """Training targets t5 (5, n) and row weights w (n) of exact transits
    for the side or the cap job."""
    import torch
    ld = _check_soa(x6, 6, torch.float32)
    assert y5.stride(0) == ld
    n = x6.shape[1]
    t5 = torch.empty((5, ld), dtype=torch.float32, device=x6.device)[:, :n]
    w = torch.empty(n, dtype=torch.float32, device=x6.device)
    _check(lib().rt_surrogate_encode_job(int(job), _handles(cloaks), len(cloaks), n, ld, _ptr(x6), _ptr(y5),
                                         _ptr(status), _ptr(t5), _ptr(w), _stream()))
    return t5, w


class Surrogate:
    """Owning wrapper of an rt_model (the transit MLP)."""

    NPARAM = 200453

    def __init__(self, seed: int = 0, path: str | None = None):
        h = ctypes.c_void_p()
        if path is not None:
            _check(lib().rt_surrogate_load(path.encode(), ctypes.byref(h)))
        else:
            _check(lib().rt_surrogate_create(int(seed), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().rt_surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.NPARAM, dtype=np.float32)
        _check(lib().rt_surrogate_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.NPARAM
        _check(lib().rt_surrogate_set_params(self.handle, p.ctypes.data))

    def get_scaling(self) -> np.ndarray:
        out = np.empty(22, dtype=np.float32)
        _check(lib().rt_surrogate_get_scaling(self.handle, out.ctypes.data))
        return out

    def set_scaling(self, sc: np.ndarray):
        sc = np.ascontiguousarray(sc, dtype=np.float32)
        _check(lib().rt_surrogate_set_scaling(self.handle, sc.ctypes.data))

    def fit_scaling(self, x6, t5, w=None):
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        _check(lib().rt_surrogate_fit_scaling(self.handle, x6.shape[1], ld, _ptr(x6), _ptr(t5), _ptr(w),
                                              _stream()))

    def grad(self, x6, t5, w=None, huber=0.0):
        """(gradient (NPARAM,) float32 tensor, loss (1,) tensor) of one batch."""
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        g = torch.empty(self.NPARAM, dtype=torch.float32, device=x6.device)
        loss = torch.empty(1, dtype=torch.float32, device=x6.device)
        _check(lib().rt_surrogate_grad(self.handle, x6.shape[1], ld, _ptr(x6), _ptr(t5), _ptr(w),
                                       float(huber), _ptr(g), _ptr(loss), _stream()))
        return g, loss

    def train_step(self, x6, t5, w=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   weight_decay=0.0, huber=0.0, loss=None):
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        o = TrainOpts(lr, beta1, beta2, eps, weight_decay, huber)
        _check(lib().rt_surrogate_train(self.handle, x6.shape[1], ld, _ptr(x6), _ptr(t5), _ptr(w),
                                        ctypes.byref(o), _ptr(loss), _stream()))

    def step(self, grads, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        """One AdamW step with a caller-supplied gradient (NPARAM float32 device tensor)."""
        import torch
        assert grads.dtype == torch.float32 and grads.is_contiguous() and grads.numel() == self.NPARAM
        o = TrainOpts(lr, beta1, beta2, eps, weight_decay, 0.0)
        _check(lib().rt_surrogate_step(self.handle, _ptr(grads), ctypes.byref(o), _stream()))

    def get_state(self):
        """(m, v, step): AdamW moments (float32 host arrays) and the step count."""
        m = np.empty(self.NPARAM, dtype=np.float32)
        v = np.empty(self.NPARAM, dtype=np.float32)
        k = ctypes.c_int64()
        _check(lib().rt_surrogate_get_state(self.handle, m.ctypes.data, v.ctypes.data, ctypes.byref(k)))
        return m, v, k.value

    def set_state(self, m, v, step: int):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        assert m.size == self.NPARAM and v.size == self.NPARAM
        _check(lib().rt_surrogate_set_state(self.handle, m.ctypes.data, v.ctypes.data, int(step)))

    def forward(self, x6):
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        n = x6.shape[1]
        t5 = torch.empty((5, ld), dtype=torch.float32, device=x6.device)[:, :n]
        _check(lib().rt_surrogate_forward(self.handle, n, ld, _ptr(x6), _ptr(t5), _stream()))
        return t5

    def calibrate(self, cloaks, x6, y5_exact, status_exact, tol=1e-3, hres_max=1e-4,
                  cap_margin=1e-2, min_count=8, dilate=0, hres_exact=None, unresolved=1e-6,
                  p_min=1e-4) -> float:
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        g = GateOpts(tol, hres_max, cap_margin, min_count, dilate, unresolved, p_min)
        frac = ctypes.c_double()
        _check(lib().rt_surrogate_calibrate(self.handle, _handles(cloaks), len(cloaks), x6.shape[1], ld,
                                            _ptr(x6), _ptr(y5_exact), _ptr(status_exact), _ptr(hres_exact),
                                            ctypes.byref(g), ctypes.byref(frac), _stream()))
        return frac.value

    def trust_map(self) -> np.ndarray:
        """(4, alpha cells, beta cells) for the side job, (4, alpha, |beta|, u
        cells) for the cap job."""
        na, nb, nu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().rt_surrogate_get_map(self.handle, None, ctypes.byref(na), ctypes.byref(nb), ctypes.byref(nu)))
        out = np.empty((4, na.value, nb.value, nu.value), dtype=np.uint8)
        _check(lib().rt_surrogate_get_map(self.handle, out.ctypes.data, None, None, None))
        return out if nu.value > 1 else out[..., 0]

    def set_job(self, job: int, cloak=None):
        """Side job (SIDE) or cap job (CAP, with the geometry of `cloak`);
        clears the trust map."""
        _check(lib().rt_surrogate_set_job(self.handle, int(job), cloak.handle if cloak is not None else None))

    @property
    def job(self) -> int:
        j = ctypes.c_int32()
        _check(lib().rt_surrogate_get_job(self.handle, ctypes.byref(j)))
        return j.value

    def chain(self, nxt: "Surrogate | None"):
        """Offer the rows this model's gate rejects to `nxt` (None unchains).
        Keeps a reference so that `nxt` lives as long as the chain."""
        _check(lib().rt_surrogate_chain(self.handle, nxt.handle if nxt is not None else None))
        self._next = nxt

    def infer(self, cloaks, opts: dict, x6, y5=None, fallback=None, status=None):
        """Surrogate transit with exact fallback: (y5, status, fallback)."""
        import torch
        ld = _check_soa(x6, 6, torch.float32)
        n = x6.shape[1]
        dev = x6.device
        if y5 is None:
            y5 = torch.empty((5, ld), dtype=torch.float32, device=dev)[:, :n]
        if fallback is None:
            fallback = torch.empty(n, dtype=torch.uint8, device=dev)
        if status is None:
            status = torch.empty(n, dtype=torch.int32, device=dev)
        _check(lib().rt_surrogate_infer(self.handle, _handles(cloaks), len(cloaks),
                                        ctypes.byref(trace_opts(opts)), n, ld, _ptr(x6), _ptr(y5),
                                        _ptr(fallback), _ptr(status), _stream()))
        return y5, status, fallback

    def save(self, path: str):
        _check(lib().rt_surrogate_save(self.handle, path.encode()))
