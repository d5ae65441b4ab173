"""Seeded synthetic workloads shared by the GPU binding's callers and the oracle.

This module only builds inputs: cloak/option/camera/room descriptions and ray
bundles. It holds none of the method's arithmetic and imports neither the GPU
binding nor the oracle, so both sides can be fed the same inputs.

Geometry: the paper's cloak has b/a = 2 (a = 5 cm, b = 10 cm, Sect. 4); here
the radii are R1 = 1, R2 = 2. For 3-D scenes the cloak and the metal cylinder
it hides stand on the floor of a checkerboard room, z in [0, 4].
"""
from __future__ import annotations

import math

import numpy as np

R1, R2, HEIGHT = 1.0, 2.0, 4.0
ROOM_LO, ROOM_HI, TILE = (-10.0, -10.0, 0.0), (10.0, 10.0, 10.0), 0.5
CAM_TARGET, CAM_DIST, FOV_DEG = (0.0, 0.0, 2.0), 8.0, 60.0

RADIAL, AZIMUTHAL = 0, 1
ORDINARY, EXTRAORDINARY = 0, 1


def cloak(axis: int, height: float | None = None, inner_mirror: int = 1) -> dict:
    """Cloak description. height=None: infinitely long cylinder (2-D runs)."""
    if height is None:
        z0, z1 = -math.inf, math.inf
    else:
        z0, z1 = 0.0, float(height)
    return {"r1": R1, "r2": R2, "z0": z0, "z1": z1, "axis": int(axis),
            "inner_mirror": int(inner_mirror)}


def opts_rk4(h: float = 1e-3, r_out: float = 3.0, **kw) -> dict:
    d = {"scheme": 0, "precision": 0, "h": h, "rtol": 1e-8, "atol": 1e-8, "hmax": 0.5,
         "r_out": r_out, "max_steps": 1_000_000, "max_bounces": 4}
    d.update(kw)
    return d


def opts_rk4_hamc(h: float = 1e-3, r_out: float = 3.0, **kw) -> dict:
    """Classical RK4 with the fixed step h in the ray parameter of the
    canonically normalized Hamiltonian k^T M^-1 k - 1 (scheme 3); dt/dtau = 2
    everywhere, so h = 1e-3 is a step of 0.002 in optical path."""
    d = opts_rk4_ham(h, r_out, **kw)
    d["scheme"] = 3
    return d


def opts_rk4_ham(h: float = 3e-3, r_out: float = 3.0, **kw) -> dict:
    """Classical RK4 with the fixed step h in the ray parameter tau of the
    Hamiltonian form (scheme 2); dt/dtau = 2 eps_o eps_e = 8 at r = 2 of the
    R1 = 1, R2 = 2 cloak, so h = 3e-3 is a step of 0.024 in optical path
    there, shrinking towards r = R1."""
    d = {"scheme": 2, "precision": 0, "h": h, "rtol": 1e-8, "atol": 1e-8, "hmax": 0.5,
         "r_out": r_out, "max_steps": 1_000_000, "max_bounces": 4}
    d.update(kw)
    return d


def opts_dp45(tol: float = 1e-8, h0: float = 1e-2, r_out: float = 3.0, **kw) -> dict:
    d = {"scheme": 1, "precision": 0, "h": h0, "rtol": tol, "atol": tol, "hmax": 0.5,
         "r_out": r_out, "max_steps": 1_000_000, "max_bounces": 4}
    d.update(kw)
    return d


def inplane_bundle(n_per_angle: int = 16384, n_angles: int = 8, r_start: float = 3.0,
                   p_max: float = 3.0) -> np.ndarray:
    """Parallel in-plane rays: impact parameters on the midpoint grid of
    [-p_max, p_max] (which avoids the singular p = 0), directions at angles
    2 pi j / n_angles, origins on the circle r = r_start upstream.
    Returns SoA float64 (6, n_per_angle * n_angles), angle-major."""
    p = -p_max + 2.0 * p_max * (np.arange(n_per_angle) + 0.5) / n_per_angle
    out = np.empty((6, n_angles * n_per_angle))
    for j in range(n_angles):
        a = 2.0 * math.pi * j / n_angles
        d = np.array([math.cos(a), math.sin(a)])
        nperp = np.array([-math.sin(a), math.cos(a)])
        back = np.sqrt(np.maximum(r_start * r_start - p * p, 0.0))
        sl = slice(j * n_per_angle, (j + 1) * n_per_angle)
        out[0, sl] = p * nperp[0] - back * d[0]
        out[1, sl] = p * nperp[1] - back * d[1]
        out[2, sl] = 0.0
        out[3, sl] = d[0]
        out[4, sl] = d[1]
        out[5, sl] = 0.0
    return out


def random_rays(n: int, seed: int, r_start: float = 3.0, z_range=(0.5, 3.5),
                elev_max_deg: float = 60.0) -> np.ndarray:
    """Random 3-D vacuum rays starting on the cylinder r = r_start and aimed
    inwards (azimuth, height, in-plane angle, elevation uniform). SoA (6, n)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    z = rng.uniform(z_range[0], z_range[1], n)
    alpha = rng.uniform(-0.5 * math.pi, 0.5 * math.pi, n)
    beta = np.deg2rad(rng.uniform(-elev_max_deg, elev_max_deg, n))
    out = np.empty((6, n))
    out[0] = r_start * np.cos(phi)
    out[1] = r_start * np.sin(phi)
    out[2] = z
    inward = phi + math.pi
    hor = inward + alpha
    out[3] = np.cos(beta) * np.cos(hor)
    out[4] = np.cos(beta) * np.sin(hor)
    out[5] = np.sin(beta)
    return out


def room() -> dict:
    """Checkerboard room [-10,10]^2 x [0,10], 0.5-unit tiles, one colour pair
    per face (faces x-, x+, y-, y+, z- (floor), z+ (ceiling))."""
    rgb = np.array([
        [[0.90, 0.20, 0.20], [0.35, 0.05, 0.05]],
        [[0.20, 0.80, 0.25], [0.05, 0.30, 0.08]],
        [[0.20, 0.35, 0.90], [0.05, 0.10, 0.35]],
        [[0.95, 0.85, 0.20], [0.40, 0.30, 0.05]],
        [[0.85, 0.85, 0.85], [0.15, 0.15, 0.15]],
        [[0.80, 0.30, 0.85], [0.30, 0.08, 0.35]],
    ], dtype=np.float32)
    return {"lo": ROOM_LO, "hi": ROOM_HI, "tile": TILE, "rgb": rgb}


def orbit_camera(azimuth: float, elevation_deg: float, w: int, h: int, spp: int = 1,
                 seed: int = 0, dist: float = CAM_DIST, fov_deg: float = FOV_DEG) -> dict:
    """Pinhole camera on a sphere of radius `dist` about (0, 0, 2), looking at
    it, up = +z."""
    el = math.radians(elevation_deg)
    t = CAM_TARGET
    eye = (t[0] + dist * math.cos(el) * math.cos(azimuth),
           t[1] + dist * math.cos(el) * math.sin(azimuth),
           t[2] + dist * math.sin(el))
    return {"eye": eye, "look": t, "up": (0.0, 0.0, 1.0), "fov_deg": fov_deg,
            "w": int(w), "h": int(h), "spp": int(spp), "seed": int(seed)}


def render_views(res: int = 1024, elevations=(0.0, 15.0, 30.0, 45.0)) -> list:
    """3-D render workload: azimuth 0, the given elevations, 1 sample/pixel."""
    return [orbit_camera(0.0, e, res, res) for e in elevations]


def batched_views(n_views: int = 64, res: int = 512, seed: int = 20120926) -> list:
    """Batched workload: azimuth U[0, 2 pi), elevation U[0, 60] deg, seeded."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0.0, 2.0 * math.pi, n_views)
    el = rng.uniform(0.0, 60.0, n_views)
    return [orbit_camera(float(a), float(e), res, res) for a, e in zip(az, el)]


def orbit_frames(n_frames: int = 36, res: int = 4096, spp: int = 4,
                 elevation_deg: float = 30.0, seed: int = 7) -> list:
    """Large-render workload: an orbit of n_frames views at fixed elevation,
    jittered spp samples per pixel."""
    return [orbit_camera(2.0 * math.pi * k / n_frames, elevation_deg, res, res, spp, seed)
            for k in range(n_frames)]


def surrogate_entries(n: int, seed: int, height: float = HEIGHT) -> np.ndarray:
    """Entry parameters on the outer cylinder, uniform: azimuth phi in
    [0, 2 pi), height z in [0, height], horizontal angle alpha to the inward
    normal and elevation beta in (-pi/2, pi/2). float64 (n, 4)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, 4))
    out[:, 0] = rng.uniform(0.0, 2.0 * math.pi, n)
    out[:, 1] = rng.uniform(0.0, height, n)
    out[:, 2] = rng.uniform(-0.5 * math.pi, 0.5 * math.pi, n)
    out[:, 3] = rng.uniform(-0.5 * math.pi, 0.5 * math.pi, n)
    return out


def surrogate_features(n: int, seed: int, height: float = HEIGHT) -> np.ndarray:
    """Surrogate inputs: the entry parameters of surrogate_entries plus a
    branch bit (0 ordinary, 1 extraordinary) and an optic-axis bit (0 radial,
    1 azimuthal), each uniform. float32 SoA (6, n)."""
    e = surrogate_entries(n, seed, height)
    rng = np.random.default_rng(seed + 0x5EED)
    out = np.empty((6, n), dtype=np.float32)
    out[:4] = e.T
    out[4] = rng.integers(0, 2, n)
    out[5] = rng.integers(0, 2, n)
    # keep |alpha|, |beta| < pi/2 after rounding to float32
    lim = np.nextafter(np.float32(0.5 * math.pi), np.float32(0.0))
    out[2:4] = np.clip(out[2:4], -lim, lim)
    return out


def render_opts(precision: int = 0, **kw) -> dict:
    """Integration options of the 3-D render workload: Dormand-Prince 5(4) at
    tolerance 1e-8, FP64 band 0.05 next to the inner radius in mixed mode."""
    return opts_dp45(1e-8, precision=precision, fp64_band=0.05, **kw)
