"""Closed forms and quadratures that pin the oracle (no code shared with it).

Everything here is derived by hand from the paper's equations, independently
of the oracle's Cartesian formulation:

* For the uniaxial cloaks of Eq. (14) and Eq. (15), the auxiliary matrix of
  Eq. (7) is diagonal in the cylindrical frame: the components across the
  optic axis are eps_e and the one along it is eps_o (extraordinary ray), or
  n_o^2 times the identity (ordinary ray, Eq. (2) is Eq. (8) with M = n_o^2 I).
* Eq. (8) is the Euler-Lagrange equation of L = v^T M v / 2 (Fermat's
  principle, Sect. 2); in cylindrical coordinates this gives the reduced
  right-hand side below, and the conserved p_theta = r m_theta v_theta,
  p_z = m_z v_z and H = v^T M v = 1.
* Extraordinary in-plane rays of both cloaks, and azimuthal-cloak
  extraordinary rays in 3-D, see a flat metric in the coordinates
  rho = sqrt(kappa) (r - a), zeta = sqrt(kappa) z: straight lines at unit
  speed (the design of Sect. 4 keeps the ideal cloak's index distribution
  for in-plane polarized light).
* Radial-cloak ordinary rays: constant index n_o = sqrt(kappa) (Sect. 4),
  straight lines, Snell refraction, specular inner mirror.
* Radial-cloak extraordinary and azimuthal-cloak ordinary rays in 3-D:
  integrable, exit angle and height by one-dimensional quadrature.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

RADIAL, AZIMUTHAL = 0, 1
ORDINARY, EXTRAORDINARY = 0, 1


def kappa(a, b):
    return (b / (b - a)) ** 2


def cyl_metric(axis, branch, r, a=1.0, b=2.0):
    """(m_r, m_theta, m_z) and their r-derivatives."""
    k = kappa(a, b)
    s = ((r - a) / r) ** 2
    sp = 2.0 * a * (r - a) / r ** 3
    if branch == EXTRAORDINARY:
        if axis == RADIAL:   # c = r_hat: eps_e = k s along r, eps_o = k across
            return (k, k * s, k * s), (0.0, k * sp, k * sp)
        return (k, k * s, k), (0.0, k * sp, 0.0)   # c = theta_hat
    if axis == RADIAL:
        return (k, k, k), (0.0, 0.0, 0.0)
    return (k * s, k * s, k * s), (k * sp, k * sp, k * sp)


def reduced_rhs(axis, branch, y, a=1.0, b=2.0):
    """Euler-Lagrange equations of L = (m_r rdot^2 + m_theta r^2 thetadot^2 +
    m_z zdot^2)/2, written back in Cartesian components."""
    x, yy, z, vx, vy, vz = y
    r = math.hypot(x, yy)
    rh = (x / r, yy / r)
    th = (-yy / r, x / r)
    vr = vx * rh[0] + vy * rh[1]
    vt = vx * th[0] + vy * th[1]
    m, dm = cyl_metric(axis, branch, r, a, b)
    ar = (-dm[0] * vr ** 2 + dm[1] * vt ** 2 + dm[2] * vz ** 2
          - 2.0 * (m[0] - m[1]) * vt ** 2 / r) / (2.0 * m[0])
    at = -(dm[1] / m[1]) * vr * vt
    az = -(dm[2] / m[2]) * vr * vz
    return np.array([vx, vy, vz, ar * rh[0] + at * th[0], ar * rh[1] + at * th[1], az])


def side_entry(o, d, b=2.0):
    """Vacuum leg to the outer cylinder: entry distance, point, local frame and
    the incident direction's components (k_n, k_theta, k_z) there."""
    A = d[0] ** 2 + d[1] ** 2
    B = o[0] * d[0] + o[1] * d[1]
    C = o[0] ** 2 + o[1] ** 2 - b * b
    s = (-B - math.sqrt(B * B - A * C)) / A
    p = o + s * d
    r = math.hypot(p[0], p[1])
    rh = np.array([p[0] / r, p[1] / r, 0.0])
    th = np.array([-p[1] / r, p[0] / r, 0.0])
    return s, p, rh, th, (d @ rh, d @ th, d[2])


def frame_at(p):
    r = math.hypot(p[0], p[1])
    return np.array([p[0] / r, p[1] / r, 0.0]), np.array([-p[1] / r, p[0] / r, 0.0])


def exit_direction(p, kt, kz):
    """Vacuum direction leaving r = b at p with conserved tangential k."""
    rh, th = frame_at(p)
    kn = math.sqrt(max(0.0, 1.0 - kt * kt - kz * kz))
    return kn * rh + kt * th + kz * np.array([0.0, 0.0, 1.0])


def cf2_azimuthal_e(o, d, a=1.0, b=2.0):
    """Azimuthal cloak, extraordinary ray, infinite cylinder: straight line in
    (rho cos theta, rho sin theta, sqrt(kappa) z) at unit speed; rho(b) = b."""
    k = kappa(a, b)
    sk = math.sqrt(k)
    s_in, p, rh, th, (kn, kt, kz) = side_entry(o, d, b)
    q = math.sqrt(k - k * kt * kt - kz * kz)  # normal wave-vector component inside
    X0 = np.array([p[0], p[1], sk * p[2]])
    V = -(q / sk) * rh + kt * th + np.array([0.0, 0.0, kz / sk])
    Vxy = V[:2]
    s = -2.0 * (X0[:2] @ Vxy) / (Vxy @ Vxy)
    X1 = X0 + s * V
    pe = np.array([X1[0], X1[1], X1[2] / sk])
    return pe, exit_direction(pe, kt, kz), s_in + s


def cf3_radial_o(o, d, a=1.0, b=2.0):
    """Radial cloak, ordinary ray: Snell at r = b with n = sqrt(kappa),
    straight line, specular reflection at the metal cylinder r = a."""
    k = kappa(a, b)
    s_in, p, rh, th, (kn, kt, kz) = side_entry(o, d, b)
    kvec = kt * th + np.array([0.0, 0.0, kz]) - math.sqrt(k - kt * kt - kz * kz) * rh
    v = kvec / k
    x = p.copy()
    t = 0.0
    A = v[0] ** 2 + v[1] ** 2
    B = x[0] * v[0] + x[1] * v[1]
    C = x[0] ** 2 + x[1] ** 2 - a * a
    disc = B * B - A * C
    if disc >= 0.0:
        tm = (-B - math.sqrt(disc)) / A
        if tm > 0.0:
            x = x + tm * v
            t += tm
            n = np.array([x[0], x[1], 0.0]) / math.hypot(x[0], x[1])
            v = v - 2.0 * (v @ n) * n
    B = x[0] * v[0] + x[1] * v[1]
    C = x[0] ** 2 + x[1] ** 2 - b * b
    tb = (-B + math.sqrt(B * B - A * C)) / A
    x = x + tb * v
    t += tb
    rh1, th1 = frame_at(x)
    kout = k * v
    return x, exit_direction(x, kout @ th1, kout[2]), s_in + t


def cf4_quadrature(axis, branch, o, d, a=1.0, b=2.0):
    """Integrable 3-D cases (radial extraordinary, azimuthal ordinary): the
    exit angle, height and optical path by quadrature between the turning
    point and r = b, with r = r_min + (b - r_min) u^2."""
    k = kappa(a, b)
    s_in, p, rh, th, (kn, kt, kz) = side_entry(o, d, b)
    # entry velocity at r = b where k s(b) = 1: p_theta = b k_theta, p_z = k_z
    pth, pz = b * kt, kz

    def F(r):
        m, _ = cyl_metric(axis, branch, r, a, b)
        return 1.0 - pth * pth / (r * r * m[1]) - pz * pz / m[2]

    rmin = optimize.brentq(F, a * (1.0 + 1e-15) + 1e-15, b, xtol=1e-16, rtol=1e-15, maxiter=500)

    def parts(u):
        r = rmin + (b - rmin) * u * u
        m, _ = cyl_metric(axis, branch, r, a, b)
        rdot = math.sqrt(max(F(r), 0.0) / m[0])
        jac = 2.0 * (b - rmin) * u
        return r, m, rdot, jac

    def f_theta(u):
        r, m, rdot, jac = parts(u)
        return pth / (r * r * m[1]) * jac / rdot if u > 0 else _limit(f_theta)

    def f_z(u):
        r, m, rdot, jac = parts(u)
        return (pz / m[2]) * jac / rdot if u > 0 else _limit(f_z)

    def f_t(u):
        r, m, rdot, jac = parts(u)
        return jac / rdot if u > 0 else _limit(f_t)

    def _limit(f):
        return f(1e-9)

    opt = dict(epsabs=1e-14, epsrel=1e-13, limit=200)
    dth = 2.0 * integrate.quad(f_theta, 0.0, 1.0, **opt)[0]
    dz = 2.0 * integrate.quad(f_z, 0.0, 1.0, **opt)[0]
    T = 2.0 * integrate.quad(f_t, 0.0, 1.0, **opt)[0]
    th0 = math.atan2(p[1], p[0])
    pe = np.array([b * math.cos(th0 + dth), b * math.sin(th0 + dth), p[2] + dz])
    return pe, exit_direction(pe, kt, kz), s_in + T


def _asinh_ratio(x):
    """asinh(sqrt(x))/sqrt(x) for x >= 0 and asin(sqrt(-x))/sqrt(-x) for
    x < 0: one analytic function of x, 1 - x/6 + 3x^2/40 - ... near 0."""
    if abs(x) < 1e-6:
        return 1.0 - x / 6.0
    if x > 0.0:
        return math.asinh(math.sqrt(x)) / math.sqrt(x)
    return math.asin(math.sqrt(-x)) / math.sqrt(-x)


def cf4_elementary(axis, kt, kz, a=1.0, b=2.0):
    """The integrable 3-D cases in closed form: (dtheta, dz, T) of the
    side-to-side transit of the infinite cylinder for an entry with
    tangential wave numbers (k_theta, k_z) on r = b.

    With m_theta = m_z = kappa s in both cases, H = 1 gives
    m_r rdot^2 = Q(r) / (kappa (r - a)^2) with the quadratic
    Q(r) = kappa (r - a)^2 - p^2 - k_z^2 r^2 (p = b k_theta), Q(b) =
    b^2 k_n^2 since kappa (b - a)^2 = b^2. The turning point is the larger
    root of Q. Per unit r:
      radial e    (m_r = kappa):   dtheta = p / (u sqrt Q),
                  dz = k_z r^2 / (u sqrt Q), dt = kappa u / sqrt Q, u = r - a;
      azimuthal o (m_r = kappa s): dtheta = p / (r sqrt Q),
                  dz = k_z r / sqrt Q, dt = kappa u^2 / (r sqrt Q).
    Each integrand is a combination of 1/sqrt Q, x/sqrt Q and 1/(x sqrt Q)
    for a quadratic Q in x, whose integrals from a root are elementary."""
    k = kappa(a, b)
    p = b * kt
    A = k - kz * kz                      # leading coefficient of Q
    S = math.sqrt(A * p * p + k * kz * kz * a * a)   # sqrt(discriminant) / 2
    Qb = b * b * max(0.0, 1.0 - kt * kt - kz * kz)
    sq = math.sqrt(Qb)
    J0 = math.asinh(math.sqrt(A * Qb) / S) / math.sqrt(A)     # int dx / sqrt Q
    if axis == RADIAL:   # in u = r - a: Q = A u^2 - 2 a k_z^2 u - (p^2 + k_z^2 a^2)
        mC = p * p + kz * kz * a * a
        J1 = sq / A + a * kz * kz / A * J0                      # int u du / sqrt Q
        Jm = math.atan2(math.sqrt(mC) * sq, a * kz * kz * (b - a) + mC) / math.sqrt(mC)
        return 2.0 * p * Jm, 2.0 * kz * (J1 + 2.0 * a * J0 + a * a * Jm), 2.0 * k * J1
    C = k * a * a - p * p  # in r: Q = A r^2 - 2 kappa a r + C
    J1 = sq / A + k * a / A * J0                                # int r dr / sqrt Q
    Jm = sq / (b * S) * _asinh_ratio(C * Qb / (b * b * S * S))  # int dr / (r sqrt Q)
    return 2.0 * p * Jm, 2.0 * kz * J1, 2.0 * k * (J1 - 2.0 * a * J0 + a * a * Jm)


def aimed_rays(n, seed, r_start=3.0, b=2.0, min_tangential=0.25, elev=True, min_ktheta=0.0):
    """Vacuum rays from r = r_start that hit the side of the infinite cylinder
    with tangential wave-vector (k_theta, k_z) of norm >= min_tangential
    (away from the singular set p_theta = p_z = 0) and |k_theta| >= min_ktheta
    (azimuthal-cloak extraordinary rays: only p_theta keeps them off r = a).
    SoA (6, n)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        phi = rng.uniform(0, 2 * math.pi)
        o = np.array([r_start * math.cos(phi), r_start * math.sin(phi), rng.uniform(-1, 1)])
        target = np.array([rng.uniform(-b, b), rng.uniform(-b, b), rng.uniform(-1, 1)])
        if not elev:
            o[2] = 0.0
            target[2] = 0.0
        dd = target - o
        dd /= np.linalg.norm(dd)
        A = dd[0] ** 2 + dd[1] ** 2
        B = o[0] * dd[0] + o[1] * dd[1]
        C = o[0] ** 2 + o[1] ** 2 - b * b
        if B * B - A * C <= 0:
            continue
        s, p, rh, th, (kn, kt, kz) = side_entry(o, dd, b)
        if math.hypot(kt, kz) < min_tangential or abs(kn) < 0.05 or abs(kt) < min_ktheta:
            continue
        out.append(np.concatenate([o, dd]))
    return np.array(out).T.copy()


# --------------------------------------------------------------------------
# finite cloak (end caps z = z0, z1): the two branches whose paths are
# straight lines, in physical space (radial cloak, ordinary ray) or in the
# virtual space (rho, theta, sqrt(kappa) z) (azimuthal cloak, extraordinary
# ray). The caps are interfaces of Sect. 3 with normal +-z; an evanescent
# transmitted wave means same-mode specular reflection inside (entry: the
# ray is reflected into vacuum), and after max_bounces internal reflections
# (caps, side or inner mirror) the ray stops.
# --------------------------------------------------------------------------
S_EXITED, S_MISSED, S_ABSORBED, S_TIR, S_REFLECTED = 0, 1, 2, 5, 7
SIDE, TOP, BOTTOM = "side", "top", "bottom"


def body_entry(o, d, b, z0, z1):
    """First point where o + s d (s > 0) enters r <= b, z0 <= z <= z1:
    (s, surface) or None. Written out case by case: the side (smaller root of
    the quadratic, if its height lies between the caps) and each cap plane
    (if the ray comes from its outside and meets it within r <= b)."""
    best = None
    A = d[0] ** 2 + d[1] ** 2
    B = o[0] * d[0] + o[1] * d[1]
    C = o[0] ** 2 + o[1] ** 2 - b * b
    if A > 0.0 and C > 0.0 and B * B - A * C >= 0.0:
        s = (-B - math.sqrt(B * B - A * C)) / A
        if s > 0.0 and z0 <= o[2] + s * d[2] <= z1:
            best = (s, SIDE)
    for plane, surf, sign in ((z1, TOP, 1.0), (z0, BOTTOM, -1.0)):
        if sign * d[2] < 0.0 and sign * (o[2] - plane) > 0.0:
            s = (plane - o[2]) / d[2]
            q = o + s * d
            if q[0] ** 2 + q[1] ** 2 <= b * b and (best is None or s < best[0]):
                best = (s, surf)
    return best


def _outward(surf, x):
    if surf == TOP:
        return np.array([0.0, 0.0, 1.0])
    if surf == BOTTOM:
        return np.array([0.0, 0.0, -1.0])
    r = math.hypot(x[0], x[1])
    return np.array([x[0] / r, x[1] / r, 0.0])


def _leave_cylinder(x, d, R):
    """Vacuum leg from x along d to the outgoing crossing of r = R."""
    A = d[0] ** 2 + d[1] ** 2
    if A <= 0.0:
        return x, 0.0
    B = x[0] * d[0] + x[1] * d[1]
    C = x[0] ** 2 + x[1] ** 2 - R * R
    disc = B * B - A * C
    if disc < 0.0:
        return x, 0.0
    s = max((-B + math.sqrt(disc)) / A, 0.0)
    return x + s * d, s


def finite_radial_o(o, d, a=1.0, b=2.0, z0=0.0, z1=4.0, max_bounces=4, r_out=3.0, events=None):
    """Radial cloak, ordinary ray, cloak of finite height (Sect. 4: n_o =
    sqrt(kappa) constant, straight rays; metal cylinder r < a with its end
    disks). Snell's law at every interface with n = sqrt(kappa): the wave
    vector's tangential part is continuous and |k| = n inside, 1 outside; a
    tangential part longer than the index of the far side reflects totally.
    Returns (status, point on r = r_out or the last point, unit direction,
    optical path, bounces); `events` (a list) receives (kind, surface) of
    every interface the ray meets."""
    ev = events if events is not None else []
    n = math.sqrt(kappa(a, b))
    d = np.asarray(d, float) / np.linalg.norm(d)
    o = np.asarray(o, float)
    hit = body_entry(o, d, b, z0, z1)
    if hit is None:
        p, s = _leave_cylinder(o, d, r_out)
        return S_MISSED, p, d, s, 0
    s_in, surf = hit
    ev.append(("enter", surf))
    x = o + s_in * d
    if surf != SIDE:
        x[2] = z1 if surf == TOP else z0
    nrm = _outward(surf, x)
    if surf != SIDE and x[0] ** 2 + x[1] ** 2 <= a * a:  # the metal end disk
        dr = d - 2.0 * (d @ nrm) * nrm
        p, s = _leave_cylinder(x, dr, r_out)
        return S_REFLECTED, p, dr, s_in + s, 0
    kt = d - (d @ nrm) * nrm
    k = kt - math.sqrt(n * n - kt @ kt) * nrm      # inward normal component
    v = k / (n * n)                                # |v| = 1/n: t is the optical path
    t, bounces = 0.0, 0
    while True:
        # earliest of: inner mirror r = a (entering it), side r = b, caps
        cands = []
        A = v[0] ** 2 + v[1] ** 2
        B = x[0] * v[0] + x[1] * v[1]
        if A > 0.0:
            Ca = x[0] ** 2 + x[1] ** 2 - a * a
            disc = B * B - A * Ca
            if disc > 0.0:
                tm = (-B - math.sqrt(disc)) / A
                if tm > 1e-12:
                    cands.append((tm, "inner"))
            Cb = x[0] ** 2 + x[1] ** 2 - b * b
            tb = (-B + math.sqrt(B * B - A * Cb)) / A
            if tb > 1e-12:
                cands.append((tb, SIDE))
        if v[2] > 0.0:
            cands.append(((z1 - x[2]) / v[2], TOP))
        elif v[2] < 0.0:
            cands.append(((z0 - x[2]) / v[2], BOTTOM))
        tc, surf = min(cands, key=lambda c: c[0])
        x = x + tc * v
        t += tc
        if surf == "inner":
            ev.append(("mirror", surf))
            if bounces >= max_bounces:
                return S_ABSORBED, x, v / np.linalg.norm(v), s_in + t, bounces
            m = np.array([x[0], x[1], 0.0]) / math.hypot(x[0], x[1])
            v = v - 2.0 * (v @ m) * m
            bounces += 1
            continue
        nrm = _outward(surf, x)
        k = n * n * v
        kt = k - (k @ nrm) * nrm
        ev.append(("exit" if kt @ kt <= 1.0 else "tir", surf))
        if kt @ kt <= 1.0:
            dout = kt + math.sqrt(1.0 - kt @ kt) * nrm
            p, s = _leave_cylinder(x, dout, r_out)
            return S_EXITED, p, dout, s_in + t + s, bounces
        if bounces >= max_bounces:
            return S_TIR, x, v / np.linalg.norm(v), s_in + t, bounces
        v = v - 2.0 * (v @ nrm) * nrm
        bounces += 1


def finite_azimuthal_e(o, d, a=1.0, b=2.0, z0=0.0, z1=4.0, max_bounces=4, r_out=3.0, events=None):
    """Azimuthal cloak, extraordinary ray, cloak of finite height. With
    M = diag(kappa, kappa s, kappa) in (r, theta, z) (Eq. (15), Eq. (7)) the
    line element is that of flat space in X = rho cos(theta),
    Y = rho sin(theta), Z = sqrt(kappa) z, rho = sqrt(kappa) (r - a): the ray
    is a straight line there at unit speed, its parameter the optical path.
    The wave vector k = M v, v the physical velocity, meets each interface
    as in Sect. 3: its tangential part is continuous, the normal part solves
    k^T M^-1 k = 1 inside (evanescent: same-mode reflection, i.e. the
    virtual velocity's normal component flips) or |k| = 1 outside.
    Returns (status, point, unit direction, optical path, bounces); `events`
    as for finite_radial_o."""
    ev = events if events is not None else []
    kap = kappa(a, b)
    sk = math.sqrt(kap)
    d = np.asarray(d, float) / np.linalg.norm(d)
    o = np.asarray(o, float)
    hit = body_entry(o, d, b, z0, z1)
    if hit is None:
        p, s = _leave_cylinder(o, d, r_out)
        return S_MISSED, p, d, s, 0
    s_in, surf = hit
    ev.append(("enter", surf))
    x = o + s_in * d
    if surf != SIDE:
        x[2] = z1 if surf == TOP else z0
    r = math.hypot(x[0], x[1])
    nrm = _outward(surf, x)
    if surf != SIDE and r <= a:
        dr = d - 2.0 * (d @ nrm) * nrm
        p, s = _leave_cylinder(x, dr, r_out)
        return S_REFLECTED, p, dr, s_in + s, 0
    rh, th = frame_at(x)
    sq = (r - a) / r                      # sqrt(s)
    kr, kth, kz = d @ rh, d @ th, d[2]
    if surf == SIDE:
        q2 = kap - kap * kth * kth / (kap * sq * sq) - kz * kz   # m_r (1 - kt^2/m_t - kz^2/m_z)
        if q2 < 0.0:
            dr = d - 2.0 * (d @ nrm) * nrm
            p, s = _leave_cylinder(x, dr, r_out)
            return S_REFLECTED, p, dr, s_in + s, 0
        kr = -math.sqrt(q2)
    else:
        q2 = kap - kr * kr - kth * kth / (sq * sq)
        if q2 < 0.0:
            dr = d - 2.0 * (d @ nrm) * nrm
            p, s = _leave_cylinder(x, dr, r_out)
            return S_REFLECTED, p, dr, s_in + s, 0
        kz = -math.sqrt(q2) if surf == TOP else math.sqrt(q2)
    # virtual state: position and unit velocity (V_rho, V_theta, V_Z)
    theta = math.atan2(x[1], x[0])
    rho = sk * (r - a)
    X = np.array([rho * math.cos(theta), rho * math.sin(theta), sk * x[2]])
    Vr, Vt, Vz = kr / sk, kth / (sk * sq), kz / sk
    V = Vr * np.array([math.cos(theta), math.sin(theta), 0.0]) + \
        Vt * np.array([-math.sin(theta), math.cos(theta), 0.0]) + np.array([0.0, 0.0, Vz])
    t, bounces = 0.0, 0
    Zlo, Zhi = sk * z0, sk * z1
    while True:
        cands = []
        A = V[0] ** 2 + V[1] ** 2
        if A > 0.0:
            B = X[0] * V[0] + X[1] * V[1]
            C = X[0] ** 2 + X[1] ** 2 - b * b
            tb = (-B + math.sqrt(max(B * B - A * C, 0.0))) / A
            if tb > 1e-12:
                cands.append((tb, SIDE))
        if V[2] > 0.0:
            cands.append(((Zhi - X[2]) / V[2], TOP))
        elif V[2] < 0.0:
            cands.append(((Zlo - X[2]) / V[2], BOTTOM))
        tc, surf = min(cands, key=lambda c: c[0])
        X = X + tc * V
        t += tc
        theta = math.atan2(X[1], X[0])
        rho = math.hypot(X[0], X[1])
        rhv = np.array([math.cos(theta), math.sin(theta), 0.0])
        thv = np.array([-math.sin(theta), math.cos(theta), 0.0])
        r = a + rho / sk
        sq = (r - a) / r
        xp = np.array([r * math.cos(theta), r * math.sin(theta), X[2] / sk])
        Vr, Vt, Vz = V @ rhv, V @ thv, V[2]
        # physical velocity and k = M v
        vr, vt, vz = Vr / sk, Vt / (sk * sq), Vz / sk
        kr, kth, kz = kap * vr, kap * sq * sq * vt, kap * vz
        tan2 = kth * kth + kz * kz if surf == SIDE else kr * kr + kth * kth
        ev.append(("exit" if tan2 <= 1.0 else "tir", surf))
        if surf == SIDE:
            if tan2 <= 1.0:
                dout = math.sqrt(1.0 - tan2) * rhv + kth * thv + np.array([0.0, 0.0, kz])
                p, s = _leave_cylinder(xp, dout, r_out)
                return S_EXITED, p, dout, s_in + t + s, bounces
            if bounces >= max_bounces:
                vv = vr * rhv + vt * thv + np.array([0.0, 0.0, vz])
                return S_TIR, xp, vv / np.linalg.norm(vv), s_in + t, bounces
            V = V - 2.0 * Vr * rhv
        else:
            if tan2 <= 1.0:
                sgn = 1.0 if surf == TOP else -1.0
                dout = kr * rhv + kth * thv + np.array([0.0, 0.0, sgn * math.sqrt(1.0 - tan2)])
                p, s = _leave_cylinder(xp, dout, r_out)
                return S_EXITED, p, dout, s_in + t + s, bounces
            if bounces >= max_bounces:
                vv = vr * rhv + vt * thv + np.array([0.0, 0.0, vz])
                return S_TIR, xp, vv / np.linalg.norm(vv), s_in + t, bounces
            V = V * np.array([1.0, 1.0, -1.0])
        bounces += 1


def cap_rays(n, seed, a=1.0, b=2.0, z0=0.0, z1=4.0, polar_max_deg=75.0, side_share=0.5):
    """Vacuum rays that meet the finite cloak: a share through the annulus of
    a cap (aimed at a uniform point of a < r < b on the top or bottom cap,
    from outside, at polar angles up to polar_max_deg to the cap's normal),
    the rest through the side at steep elevations (so that inside they reach
    the caps). SoA (6, n), origins 6 units before the aim point."""
    rng = np.random.default_rng(seed)
    out = np.empty((6, n))
    for i in range(n):
        if rng.uniform() >= side_share:
            top = rng.uniform() < 0.5
            r = math.sqrt(rng.uniform(a * a, b * b))
            ph = rng.uniform(0, 2 * math.pi)
            tgt = np.array([r * math.cos(ph), r * math.sin(ph), z1 if top else z0])
            pol = math.radians(rng.uniform(0.0, polar_max_deg))
            az = rng.uniform(0, 2 * math.pi)
            d = np.array([math.sin(pol) * math.cos(az), math.sin(pol) * math.sin(az),
                          -math.cos(pol) if top else math.cos(pol)])
        else:
            ph = rng.uniform(0, 2 * math.pi)
            tgt = np.array([b * math.cos(ph), b * math.sin(ph), rng.uniform(z0 + 0.3, z1 - 0.3)])
            al = rng.uniform(-1.3, 1.3)
            be = rng.uniform(0.5, 1.3) * (1 if rng.uniform() < 0.5 else -1)
            inward = ph + math.pi + al
            d = np.array([math.cos(be) * math.cos(inward), math.cos(be) * math.sin(inward), math.sin(be)])
        out[:3, i] = tgt - 6.0 * d
        out[3:, i] = d
    return out


def _fresnel_s(kt2, n):
    """Intensity reflectance of the s wave (field across the plane of
    incidence) between vacuum and index n for the tangential wave number^2
    kt2 (the same from either side); 1 beyond the critical angle."""
    if kt2 >= 1.0:
        return 1.0
    cv, cn = math.sqrt(1.0 - kt2), math.sqrt(n * n - kt2)
    r = (cv - cn) / (cv + cn)
    return r * r


def radial_o_first_reflection(o, d, a=1.0, b=2.0, max_bounces=4):
    """Radial cloak, ordinary ray, side surface only (an infinitely long
    cylinder): the primary ray and the ordinary wave it reflects into at its
    exit (R27). At the side the optic axis is the normal, so the ordinary
    wave is the s wave of index n = sqrt(kappa) on both sides of every
    interface: the entry takes (1 - R_s)/2 of unpolarized light, total
    internal reflection keeps all of it, the exit reflects R_s back into the
    ordinary wave, and the child leaves with 1 - R_s, each R_s at that
    interface's tangential wave number. Rays are straight inside and reflect
    specularly off the metal at r = a. Returns None if the ray misses, else
    (primary exit point, primary vacuum direction, child status, child exit
    point, child vacuum direction, child weight)."""
    n = math.sqrt(kappa(a, b))
    d = np.asarray(d, float) / np.linalg.norm(d)
    o = np.asarray(o, float)
    A = d[0] ** 2 + d[1] ** 2
    B = o[0] * d[0] + o[1] * d[1]
    if A <= 0.0 or B * B - A * (o[0] ** 2 + o[1] ** 2 - b * b) <= 0.0:
        return None
    _, x, nrm, _, _ = side_entry(o, d, b)
    kt = d - (d @ nrm) * nrm
    w = 0.5 * (1.0 - _fresnel_s(kt @ kt, n))
    v = (kt - math.sqrt(n * n - kt @ kt) * nrm) / (n * n)

    def walk(x, v, w):
        """straight legs to the next side exit; returns (status, x, v, kt2, w)"""
        bounces = 0
        while True:
            A = v[0] ** 2 + v[1] ** 2
            B = x[0] * v[0] + x[1] * v[1]
            cands = []
            Ca = x[0] ** 2 + x[1] ** 2 - a * a
            disc = B * B - A * Ca
            if disc > 0.0:
                tm = (-B - math.sqrt(disc)) / A
                if tm > 1e-12:
                    cands.append((tm, "inner"))
            Cb = x[0] ** 2 + x[1] ** 2 - b * b
            tb = (-B + math.sqrt(B * B - A * Cb)) / A
            cands.append((tb, "side"))
            tc, surf = min(cands, key=lambda c: c[0])
            x = x + tc * v
            m = np.array([x[0], x[1], 0.0]) / math.hypot(x[0], x[1])
            if surf == "inner":
                if bounces >= max_bounces:
                    return S_ABSORBED, x, v, 0.0, 0.0
                v = v - 2.0 * (v @ m) * m
                bounces += 1
                continue
            k = n * n * v
            ktt = k - (k @ m) * m
            if ktt @ ktt <= 1.0:
                return S_EXITED, x, v, ktt @ ktt, w
            if bounces >= max_bounces:
                return S_TIR, x, v, 0.0, 0.0
            v = v - 2.0 * (v @ m) * m
            bounces += 1

    st, xe, ve, kt2, w = walk(x, v, w)
    if st != S_EXITED:
        return None
    m = np.array([xe[0], xe[1], 0.0]) / math.hypot(xe[0], xe[1])
    k = n * n * ve
    ktt = k - (k @ m) * m
    dout = ktt + math.sqrt(1.0 - kt2) * m
    wc = w * _fresnel_s(kt2, n)
    vc = ve - 2.0 * (ve @ m) * m  # the same-mode reflected wave: the mirror image
    stc, xc, vcc, kt2c, wc = walk(xe, vc, wc)
    if stc != S_EXITED:
        return xe, dout, stc, xc, None, 0.0
    mc = np.array([xc[0], xc[1], 0.0]) / math.hypot(xc[0], xc[1])
    kc = n * n * vcc
    kttc = kc - (kc @ mc) * mc
    doutc = kttc + math.sqrt(1.0 - kt2c) * mc
    return xe, dout, S_EXITED, xc, doutc, wc * (1.0 - _fresnel_s(kt2c, n))
