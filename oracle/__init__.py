"""FP64 CPU oracle for ray tracing through uniaxial-dielectric cylindrical cloaks.

TEST INFRASTRUCTURE. This package is the independent reference that the GPU
library is checked against (Halimeh & Wegener, Sects. 2-4). Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
import it; the product package never does. It shares no code with the GPU
library: the C source ``cloak_oracle.c`` is compiled with gcc, loaded here
with ctypes, and fed plain numpy arrays.

Descriptions are plain dicts (the same keys the GPU binding accepts):
  cloak:  r1, r2, z0, z1, axis (0 radial Eq. (14), 1 azimuthal Eq. (15)), inner_mirror
  opts:   scheme (0 RK4, 1 DP45, 2 RK4 on the Hamiltonian form), h, rtol, atol, hmax, r_out, max_steps, max_bounces
  camera: eye, look, up, fov_deg, w, h, spp, seed
  room:   lo, hi, tile, rgb (6 faces x 2 parities x 3)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cloak_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libcloak_oracle.so")
_lib = None

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)


def build() -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP, no SIMD intrinsics)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", "-Wall",
           "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Cloak(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double),
                ("z0", ctypes.c_double), ("z1", ctypes.c_double),
                ("axis", ctypes.c_int32), ("inner_mirror", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("max_bounces", ctypes.c_int32),
                ("h", ctypes.c_double), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double), ("hmax", ctypes.c_double),
                ("r_out", ctypes.c_double), ("max_steps", ctypes.c_int64)]


class _Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("look", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_deg", ctypes.c_double),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class _Room(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("tile", ctypes.c_double), ("rgb", ctypes.c_float * 36)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = _load(_LIB_PATH)
    return _lib


class use_library:
    """Context manager: route every call of this module to another build of
    the oracle (a copy of cloak_oracle.c compiled elsewhere, e.g. with a
    deliberate mistake planted by a test), then restore the default."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(src_text: str, out_dir: str) -> str:
    """Compile oracle source text (same flags as build()) into out_dir."""
    src = os.path.join(out_dir, "cloak_oracle_variant.c")
    with open(src, "w") as f:
        f.write(src_text)
    out = os.path.join(out_dir, "libcloak_oracle_variant.so")
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", "-I" + _HERE,
                    "-o", out, src, "-lm"], check=True)
    return out


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _load(path):
    L = ctypes.CDLL(path)
    L.orc_trace.argtypes = [ctypes.POINTER(_Cloak), ctypes.POINTER(_Opts), ctypes.c_int32,
                            ctypes.c_int64, c_double_p, c_double_p, c_double_p, c_int32_p,
                            c_double_p, c_int64_p, c_double_p]
    L.orc_render_samples.argtypes = [ctypes.POINTER(_Cloak), ctypes.POINTER(_Opts),
                                     ctypes.POINTER(_Room), ctypes.POINTER(_Camera),
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                     c_int64_p, c_uint8_p, c_double_p, c_int32_p, c_double_p]
    L.orc_eps_cyl.argtypes = [ctypes.POINTER(_Cloak), ctypes.c_double, c_double_p]
    L.orc_metric.argtypes = [ctypes.POINTER(_Cloak), c_double_p, c_double_p]
    L.orc_metric_det_form.argtypes = [ctypes.POINTER(_Cloak), c_double_p, c_double_p]
    L.orc_rhs.argtypes = [ctypes.POINTER(_Cloak), ctypes.c_int32, c_double_p, c_double_p]
    L.orc_rhs_eq8_isotropic.argtypes = [ctypes.POINTER(_Cloak), c_double_p, c_double_p]
    L.orc_refract_in.argtypes = [ctypes.c_double, ctypes.c_double, c_double_p, c_double_p,
                                 c_double_p, ctypes.c_int32, c_double_p, c_double_p]
    L.orc_refract_in.restype = ctypes.c_int32
    L.orc_refract_out.argtypes = [ctypes.c_double, ctypes.c_double, c_double_p, c_double_p,
                                  c_double_p, ctypes.c_int32, c_double_p]
    L.orc_refract_out.restype = ctypes.c_int32
    L.orc_fresnel_in.argtypes = [ctypes.c_double, ctypes.c_double, c_double_p, c_double_p,
                                 c_double_p, c_double_p, c_double_p]
    L.orc_fresnel_in.restype = ctypes.c_int32
    L.orc_fresnel_out.argtypes = [ctypes.c_double, ctypes.c_double, c_double_p, c_double_p,
                                  c_double_p, ctypes.c_int32, c_double_p, c_double_p]
    L.orc_fresnel_out.restype = ctypes.c_int32
    L.orc_fresnel_in_pol.argtypes = [ctypes.c_double, ctypes.c_double, c_double_p, c_double_p,
                                     c_double_p, c_double_p, c_double_p, c_double_p]
    L.orc_fresnel_in_pol.restype = ctypes.c_int32
    L.orc_goggle_axis.argtypes = [ctypes.POINTER(_Camera), c_double_p, ctypes.c_int32, c_double_p]
    L.orc_goggle_axis.restype = ctypes.c_int32
    L.orc_render_goggle.argtypes = [ctypes.POINTER(_Cloak), ctypes.POINTER(_Opts), ctypes.POINTER(_Camera),
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    c_int64_p, c_double_p]
    L.orc_trace_reflections.argtypes = [ctypes.POINTER(_Cloak), ctypes.POINTER(_Opts), ctypes.c_int32,
                                        ctypes.c_int64, c_double_p, c_double_p, c_double_p]
    L.orc_render_reflections.argtypes = [ctypes.POINTER(_Cloak), ctypes.POINTER(_Opts), ctypes.POINTER(_Room),
                                         ctypes.POINTER(_Camera), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, c_int64_p, c_double_p, c_uint8_p]
    L.orc_camera_ray.argtypes = [ctypes.POINTER(_Camera), ctypes.c_int32, ctypes.c_int64,
                                 c_double_p, c_double_p]
    L.orc_room_code.argtypes = [ctypes.POINTER(_Room), c_double_p, c_double_p, c_double_p]
    L.orc_room_code.restype = ctypes.c_int32
    L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.orc_splitmix64.restype = ctypes.c_uint64
    L.orc_test_oscillator.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, c_double_p, c_int64_p]
    L.orc_test_oscillator.restype = ctypes.c_double
    L.orc_num_threads.restype = ctypes.c_int32
    return L


def _ptr(a, t=c_double_p):
    return a.ctypes.data_as(t) if a is not None else None


def _cloak(d):
    if d is None:
        return None
    return _Cloak(float(d["r1"]), float(d["r2"]), float(d.get("z0", -np.inf)),
                  float(d.get("z1", np.inf)), int(d["axis"]), int(d.get("inner_mirror", 1)))


def _opts(d):
    return _Opts(int(d.get("scheme", 0)), int(d.get("max_bounces", 4)), float(d.get("h", 1e-3)),
                 float(d.get("rtol", 1e-8)), float(d.get("atol", 1e-8)),
                 float(d.get("hmax", 0.5)), float(d.get("r_out", 3.0)),
                 int(d.get("max_steps", 1_000_000)))


def _camera(d):
    c = _Camera()
    for k in ("eye", "look", "up"):
        getattr(c, k)[:] = [float(v) for v in d[k]]
    c.fov_deg = float(d["fov_deg"])
    c.w, c.h, c.spp = int(d["w"]), int(d["h"]), int(d.get("spp", 1))
    c.seed = int(d.get("seed", 0)) & ((1 << 64) - 1)
    return c


def _room(d):
    r = _Room()
    r.lo[:] = [float(v) for v in d["lo"]]
    r.hi[:] = [float(v) for v in d["hi"]]
    r.tile = float(d["tile"])
    r.rgb[:] = [float(v) for v in np.asarray(d["rgb"], dtype=np.float32).reshape(-1)]
    return r


def trace(cloak, opts, branch, rays6):
    """Trace vacuum rays (SoA array 6 x n: origin, direction) through the cloak.

    Returns a dict with out (6 x n: point on r = r_out, unit direction), opl,
    status, hres (|H-1| at the last interface), nsteps (step attempts) and
    trans (the Eq. (12) weight of the reported ray: unpolarized entry
    transmission x same-mode internal reflectances x exit transmission; 1 for
    a miss or a reflection off the metal end disk, 0 when the ray does not
    exit).
    """
    rays6 = np.ascontiguousarray(rays6, dtype=np.float64)
    n = rays6.shape[1]
    out = np.empty((6, n))
    opl = np.empty(n)
    st = np.empty(n, dtype=np.int32)
    hr = np.empty(n)
    ns = np.empty(n, dtype=np.int64)
    tr = np.empty(n)
    c, o = _cloak(cloak), _opts(opts)
    lib().orc_trace(ctypes.byref(c), ctypes.byref(o), int(branch), n, _ptr(rays6), _ptr(out),
                    _ptr(opl), _ptr(st, c_int32_p), _ptr(hr), _ptr(ns, c_int64_p), _ptr(tr))
    return {"out": out, "opl": opl, "status": st, "hres": hr, "nsteps": ns, "trans": tr}


def render_samples(cloak, opts, room, camera, cam_index, branch, ids, weights=False):
    """Codes (face*2+parity, 12 = black), records (7 x n), status and image
    weight (the share of the sample's unpolarized light this branch carries to
    the room: 1/2 for a ray that stays in vacuum, the Eq. (12) trace weight
    for one that crosses the crystal, 0 otherwise; with weights=True) of
    samples."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = ids.shape[0]
    code = np.empty(n, dtype=np.uint8)
    rec = np.empty((7, n))
    st = np.empty(n, dtype=np.int32)
    wimg = np.empty(n) if weights else None
    c = _cloak(cloak)
    o, rm, cm = _opts(opts), _room(room), _camera(camera)
    lib().orc_render_samples(ctypes.byref(c) if c is not None else None, ctypes.byref(o),
                             ctypes.byref(rm), ctypes.byref(cm), int(cam_index), int(branch), n,
                             _ptr(ids, c_int64_p), _ptr(code, c_uint8_p), _ptr(rec),
                             _ptr(st, c_int32_p), None if wimg is None else _ptr(wimg))
    out = {"code": code, "rec": rec, "status": st}
    if weights:
        out["wimg"] = wimg
    return out


def render_pixels(cloak, opts, room, camera, cam_index, branch, pixels):
    """Mean RGB (float64, n x 3) of the given pixels over their samples."""
    pixels = np.asarray(pixels, dtype=np.int64)
    spp = int(camera.get("spp", 1))
    ids = (pixels[:, None] * spp + np.arange(spp)[None, :]).reshape(-1)
    r = render_samples(cloak, opts, room, camera, cam_index, branch, ids)
    table = np.zeros((13, 3))
    table[:12] = np.asarray(room["rgb"], dtype=np.float32).reshape(12, 3)
    col = table[r["code"]].reshape(len(pixels), spp, 3).mean(axis=1)
    return col, r


def render_unpolarized_pixels(cloak, opts, room, camera, cam_index, pixels):
    """Unpolarized RGB (float64, n x 3) of the given pixels: per sample, the
    sum over the ordinary and extraordinary branch of its image weight times
    the colour it sees, averaged over the pixel's samples (Eq. (12), Fig. 1c)."""
    pixels = np.asarray(pixels, dtype=np.int64)
    spp = int(camera.get("spp", 1))
    ids = (pixels[:, None] * spp + np.arange(spp)[None, :]).reshape(-1)
    table = np.zeros((13, 3))
    table[:12] = np.asarray(room["rgb"], dtype=np.float32).reshape(12, 3)
    col = np.zeros((len(ids), 3))
    for branch in (0, 1):
        r = render_samples(cloak, opts, room, camera, cam_index, branch, ids, weights=True)
        col += r["wimg"][:, None] * table[r["code"]]
    return col.reshape(len(pixels), spp, 3).mean(axis=1)


def render_goggle_pixels(cloak, opts, room, camera, cam_index, pixels, goggle):
    """RGB (float64, n x 3) of the given pixels seen through goggle `goggle`
    (0 in-plane, 1 axial; Figs. 1d,e and 2d,e): per sample, the sum over the
    two branches of its goggle weight times the colour it sees, averaged
    over the pixel's samples."""
    pixels = np.asarray(pixels, dtype=np.int64)
    spp = int(camera.get("spp", 1))
    ids = (pixels[:, None] * spp + np.arange(spp)[None, :]).reshape(-1)
    table = np.zeros((13, 3))
    table[:12] = np.asarray(room["rgb"], dtype=np.float32).reshape(12, 3)
    col = np.zeros((len(ids), 3))
    for branch in (0, 1):
        r = render_samples(cloak, opts, room, camera, cam_index, branch, ids)
        wg = render_goggle_weights(cloak, opts, camera, cam_index, branch, goggle, ids)
        col += wg[:, None] * table[r["code"]]
    return col.reshape(len(pixels), spp, 3).mean(axis=1)


def trace_reflections(cloak, opts, branch, rays):
    """First-order reflections of vacuum rays (6 x n) through `branch`:
    weights (3, n) and vacuum rays (3, 6, n) of the entry's reflected ray
    (row 0) and the ordinary (1) and extraordinary (2) waves reflected at the
    exit, each where it leaves the crystal."""
    rays = np.ascontiguousarray(rays, dtype=np.float64)
    n = rays.shape[1]
    w = np.empty((3, n))
    ray = np.empty((3, 6, n))
    c = _cloak(cloak)
    o = _opts(opts)
    lib().orc_trace_reflections(ctypes.byref(c), ctypes.byref(o), int(branch), n, _ptr(rays), _ptr(w), _ptr(ray))
    return w, ray


def render_reflections(cloak, opts, room, camera, cam_index, branch, ids, goggle=-1):
    """First-order reflections of samples through `branch`: weights (3, n)
    and room codes (3, n) of the entry's reflected vacuum ray (row 0) and the
    ordinary (1) and extraordinary (2) waves reflected at the exit; goggle -1
    for the unpolarized image, 0 / 1 for the in-plane / axial goggle."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = ids.shape[0]
    w = np.empty((3, n))
    code = np.empty((3, n), dtype=np.uint8)
    c = _cloak(cloak)
    o, rm, cm = _opts(opts), _room(room), _camera(camera)
    lib().orc_render_reflections(ctypes.byref(c) if c is not None else None, ctypes.byref(o), ctypes.byref(rm),
                                 ctypes.byref(cm), int(cam_index), int(branch), int(goggle), n,
                                 _ptr(ids, c_int64_p), _ptr(w), _ptr(code, c_uint8_p))
    return w, code


def render_reflection_pixels(cloak, opts, room, camera, cam_index, pixels, goggle=-1):
    """RGB (float64, n x 3) that first-order reflections add to the given
    pixels of the unpolarized image (goggle -1) or a goggle image (0 / 1):
    per sample, the sum over both branches and the three contributions of
    weight times colour, averaged over the pixel's samples."""
    pixels = np.asarray(pixels, dtype=np.int64)
    spp = int(camera.get("spp", 1))
    ids = (pixels[:, None] * spp + np.arange(spp)[None, :]).reshape(-1)
    table = np.zeros((13, 3))
    table[:12] = np.asarray(room["rgb"], dtype=np.float32).reshape(12, 3)
    col = np.zeros((len(ids), 3))
    for branch in (0, 1):
        w, code = render_reflections(cloak, opts, room, camera, cam_index, branch, ids, goggle)
        for j in range(3):
            col += w[j][:, None] * table[code[j]]
    return col.reshape(len(pixels), spp, 3).mean(axis=1)


def eps_cyl(cloak, r):
    out = np.empty(3)
    c = _cloak(cloak)
    lib().orc_eps_cyl(ctypes.byref(c), float(r), _ptr(out))
    return out


def metric(cloak, x, det_form=False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    M = np.empty(9)
    c = _cloak(cloak)
    f = lib().orc_metric_det_form if det_form else lib().orc_metric
    f(ctypes.byref(c), _ptr(x), _ptr(M))
    return M.reshape(3, 3)


def rhs(cloak, branch, y, eq8_isotropic=False):
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.empty(6)
    c = _cloak(cloak)
    if eq8_isotropic:
        lib().orc_rhs_eq8_isotropic(ctypes.byref(c), _ptr(y), _ptr(dy))
    else:
        lib().orc_rhs(ctypes.byref(c), int(branch), _ptr(y), _ptr(dy))
    return dy


def refract_in(eps_o, eps_e, chat, nhat, kin, branch):
    """Entry refraction (Sect. 3). Returns (status, k, v); status 1 = evanescent."""
    chat, nhat, kin = (np.ascontiguousarray(a, dtype=np.float64) for a in (chat, nhat, kin))
    k = np.empty(3)
    v = np.empty(3)
    st = lib().orc_refract_in(float(eps_o), float(eps_e), _ptr(chat), _ptr(nhat), _ptr(kin),
                              int(branch), _ptr(k), _ptr(v))
    return st, k, v


def refract_out(eps_o, eps_e, chat, nhat, v_in, branch):
    """Exit refraction into vacuum. Returns (status, d_out); status 1 = TIR."""
    chat, nhat, v_in = (np.ascontiguousarray(a, dtype=np.float64) for a in (chat, nhat, v_in))
    d = np.empty(3)
    st = lib().orc_refract_out(float(eps_o), float(eps_e), _ptr(chat), _ptr(nhat), _ptr(v_in),
                               int(branch), _ptr(d))
    return st, d


def fresnel_in(eps_o, eps_e, chat, nhat, kin):
    """Eq. (12) at the entry, unpolarized: ((T_o, T_e), R)."""
    chat, nhat, kin = (np.ascontiguousarray(a, dtype=np.float64) for a in (chat, nhat, kin))
    T = np.empty(2)
    R = np.empty(1)
    st = lib().orc_fresnel_in(float(eps_o), float(eps_e), _ptr(chat), _ptr(nhat), _ptr(kin), _ptr(T), _ptr(R))
    assert st == 0
    return T, float(R[0])


def fresnel_out(eps_o, eps_e, chat, nhat, k_in, branch):
    """Eq. (12) at the exit for an incident wave of `branch` with wave
    vector k_in: (T, (R_o, R_e))."""
    chat, nhat, k_in = (np.ascontiguousarray(a, dtype=np.float64) for a in (chat, nhat, k_in))
    T = np.empty(1)
    R = np.empty(2)
    st = lib().orc_fresnel_out(float(eps_o), float(eps_e), _ptr(chat), _ptr(nhat), _ptr(k_in), int(branch),
                               _ptr(T), _ptr(R))
    assert st == 0
    return float(T[0]), R


def fresnel_in_pol(eps_o, eps_e, chat, nhat, kin, e_in):
    """Eq. (12) at the entry for the incident vacuum field along e_in:
    ((T_o, T_e), R)."""
    chat, nhat, kin, e_in = (np.ascontiguousarray(a, dtype=np.float64) for a in (chat, nhat, kin, e_in))
    T = np.empty(2)
    R = np.empty(1)
    st = lib().orc_fresnel_in_pol(float(eps_o), float(eps_e), _ptr(chat), _ptr(nhat), _ptr(kin), _ptr(e_in),
                                  _ptr(T), _ptr(R))
    assert st == 0
    return T, float(R[0])


def goggle_axis(camera, d, goggle):
    """Transmission axis of goggle 0 (in-plane) or 1 (axial) for the unit ray
    direction d of `camera`."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.empty(3)
    cm = _camera(camera)
    assert lib().orc_goggle_axis(ctypes.byref(cm), _ptr(d), int(goggle), _ptr(e)) == 0
    return e


def render_goggle_weights(cloak, opts, camera, cam_index, branch, goggle, ids):
    """Per sample, the share of its light that reaches the camera through
    goggle `goggle` (0 in-plane, 1 axial) by way of `branch`."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = ids.shape[0]
    wg = np.empty(n)
    c = _cloak(cloak)
    o, cm = _opts(opts), _camera(camera)
    lib().orc_render_goggle(ctypes.byref(c) if c is not None else None, ctypes.byref(o), ctypes.byref(cm),
                            int(cam_index), int(branch), int(goggle), n, _ptr(ids, c_int64_p), _ptr(wg))
    return wg


def camera_ray(camera, cam_index, sample_id):
    o = np.empty(3)
    d = np.empty(3)
    cm = _camera(camera)
    lib().orc_camera_ray(ctypes.byref(cm), int(cam_index), int(sample_id), _ptr(o), _ptr(d))
    return o, d


def room_code(room, o, d):
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    s = np.empty(1)
    rm = _room(room)
    code = lib().orc_room_code(ctypes.byref(rm), _ptr(o), _ptr(d), _ptr(s))
    return int(code), float(s[0])


def splitmix64(seed, n):
    return int(lib().orc_splitmix64(int(seed) & ((1 << 64) - 1), int(n) & ((1 << 64) - 1)))


def test_oscillator(scheme, h, rtol, T):
    y = np.empty(6)
    ns = np.empty(1, dtype=np.int64)
    e = lib().orc_test_oscillator(int(scheme), float(h), float(rtol), float(T), _ptr(y),
                                  _ptr(ns, c_int64_p))
    return float(e), y, int(ns[0])


def num_threads():
    return int(lib().orc_num_threads())
