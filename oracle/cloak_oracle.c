/*
 * cloak_oracle.c -- plain, slow FP64 CPU reference tracer.
 *
 * TEST INFRASTRUCTURE: the oracle the GPU library is checked against. Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark load
 * it. It shares nothing with the GPU library.
 *
 * Source: J. C. Halimeh and M. Wegener, "Photorealistic ray tracing of
 * free-space invisibility cloaks made of uniaxial dielectrics".
 *   - material law:        Eq. (1) local uniaxial tensor, Eq. (14) radial and
 *                           Eq. (15) azimuthal cloak, optic axis r or theta
 *   - auxiliary matrix:     Eq. (7), M = n_o^2 n_e^2 eps^-1
 *   - ray equations:        Eq. (2) ordinary ray, Eq. (8) extraordinary ray,
 *                           written in Cartesian form; the gradient of M and
 *                           of n_o comes from forward-mode dual numbers
 *   - vacuum <-> crystal:   Sect. 3, phase matching Eq. (11) with the
 *                           extraordinary index of Eq. (9) and the angle of
 *                           Eq. (10), solved for the refraction angle by
 *                           bisection; ray velocity from Eq. (6)
 *   - integrator:           classical fourth-order Runge-Kutta (Sect. 4), and
 *                           the Dormand-Prince 5(4) pair for adaptive runs
 *   - Hamiltonian form:     the alternative tracer Sect. 4 compares against:
 *                           H(x, k) = k^T A k - f from the Cartesian tensor
 *                           of Eq. (1) (A = eps, f = eps_o eps_e, or A = I,
 *                           f = eps_o), gradient by dual numbers, RK4 in the
 *                           ray parameter
 *   - inner metal cylinder: single specular reflection (Sect. 4)
 * Units: c0 = omega = 1, so |k| is the phase index and the ODE time is the
 * optical path length. Everything is FP64, plain loops, no SIMD intrinsics.
 */
#include "cloak_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* dual numbers: value and one directional derivative                  */
/* ------------------------------------------------------------------ */
typedef struct { double v, d; } dual;

static dual mkd(double v, double d) { dual r; r.v = v; r.d = d; return r; }
static dual dk(double v) { return mkd(v, 0.0); }
static dual dadd(dual a, dual b) { return mkd(a.v + b.v, a.d + b.d); }
static dual dsub(dual a, dual b) { return mkd(a.v - b.v, a.d - b.d); }
static dual dmul(dual a, dual b) { return mkd(a.v * b.v, a.d * b.v + a.v * b.d); }
static dual ddiv(dual a, dual b) {
    return mkd(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
static dual dsqrt(dual a) { double s = sqrt(a.v); return mkd(s, a.d / (2.0 * s)); }
static dual dscale(dual a, double k) { return mkd(a.v * k, a.d * k); }
static dual dneg(dual a) { return mkd(-a.v, -a.d); }

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* 3x3 inverse by adjugate / determinant (plain doubles). */
static void inv3(const double A[3][3], double R[3][3]) {
    double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    R[0][0] = c00 / det;
    R[1][0] = c01 / det;
    R[2][0] = c02 / det;
    R[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    R[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    R[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    R[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    R[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    R[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

/* ------------------------------------------------------------------ */
/* material: Eq. (14) / Eq. (15), Eq. (1), Eq. (7)                     */
/* ------------------------------------------------------------------ */
static double kappa_of(const orc_cloak *c) {
    double q = c->b / (c->b - c->a);
    return q * q;
}

/* Cylindrical permittivity components (eps_r, eps_theta, eps_z) at radius r.
   Radial cloak, Eq. (14): eps_r = ((r-a)/r)^2 (b/(b-a))^2,
   eps_theta = eps_z = (b/(b-a))^2.  Azimuthal cloak, Eq. (15): eps_r and
   eps_z = ((r-a)/r)^2 (b/(b-a))^2, eps_theta = (b/(b-a))^2. */
static void eps_cyl(const orc_cloak *c, dual r, dual *er, dual *et, dual *ez) {
    double kap = kappa_of(c);
    dual q = ddiv(dsub(r, dk(c->a)), r);
    dual ks = dscale(dmul(q, q), kap);
    if (c->axis == ORC_AXIS_RADIAL) {
        *er = ks; *et = dk(kap); *ez = dk(kap);
    } else {
        *er = ks; *et = dk(kap); *ez = ks;
    }
}

/* Eq. (1): eps_o is the doubly degenerate principal value, eps_e the one
   along the optic axis. Radial cloak: c = r_hat, eps_theta = eps_z = eps_o.
   Azimuthal cloak: c = theta_hat, eps_r = eps_z = eps_o. */
static void uniaxial_split(const orc_cloak *c, dual er, dual et, dual ez,
                           dual *eo, dual *ee) {
    (void)ez;
    if (c->axis == ORC_AXIS_RADIAL) { *ee = er; *eo = et; }
    else { *ee = et; *eo = er; }
}

/* Principal frame at x: r_hat, theta_hat, z_hat, and the principal
   permittivities (eps_r, eps_theta, eps_z) of Eq. (14)/(15). */
static void principal(const orc_cloak *c, const dual x[3], dual ax[3][3], dual ev[3],
                      dual *eo, dual *ee) {
    dual r = dsqrt(dadd(dmul(x[0], x[0]), dmul(x[1], x[1])));
    ax[0][0] = ddiv(x[0], r); ax[0][1] = ddiv(x[1], r); ax[0][2] = dk(0.0);
    ax[1][0] = dneg(ddiv(x[1], r)); ax[1][1] = ddiv(x[0], r); ax[1][2] = dk(0.0);
    ax[2][0] = dk(0.0); ax[2][1] = dk(0.0); ax[2][2] = dk(1.0);
    eps_cyl(c, r, &ev[0], &ev[1], &ev[2]);
    uniaxial_split(c, ev[0], ev[1], ev[2], eo, ee);
}

/* sum_p w_p a_p a_p^T for the three principal axes a_p */
static void spectral(const dual ax[3][3], const dual w[3], dual T[3][3]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            dual t = dk(0.0);
            for (int p = 0; p < 3; p++) t = dadd(t, dmul(w[p], dmul(ax[p][i], ax[p][j])));
            T[i][j] = t;
        }
}

/* Cartesian permittivity tensor eps = eps_r r r^T + eps_theta t t^T + eps_z z z^T. */
static void eps_cart(const orc_cloak *c, const dual x[3], dual E[3][3],
                     dual *eo, dual *ee) {
    dual ax[3][3], ev[3];
    principal(c, x, ax, ev, eo, ee);
    spectral(ax, ev, E);
}

/* Eq. (7), right-hand form: M = n_o^2 n_e^2 eps^-1 = eps_o eps_e eps^-1, with
   eps^-1 taken in the principal frame (1/eps_p on each axis) so that no
   cancellation occurs where a principal value goes to zero at r = a. */
static void metric_dual(const orc_cloak *c, const dual x[3], dual M[3][3]) {
    dual ax[3][3], ev[3], eo, ee, w[3];
    principal(c, x, ax, ev, &eo, &ee);
    dual f = dmul(eo, ee);
    for (int p = 0; p < 3; p++) w[p] = ddiv(f, ev[p]);
    spectral(ax, w, M);
}

/* inverse of Eq. (7): M^-1 = eps / (n_o^2 n_e^2) */
static void metric_inv(const orc_cloak *c, const double *x, double Mi[3][3]) {
    dual xd[3] = { dk(x[0]), dk(x[1]), dk(x[2]) }, ax[3][3], ev[3], eo, ee, w[3], T[3][3];
    principal(c, xd, ax, ev, &eo, &ee);
    dual f = dmul(eo, ee);
    for (int p = 0; p < 3; p++) w[p] = ddiv(ev[p], f);
    spectral(ax, w, T);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Mi[i][j] = T[i][j].v;
}

static void material_at(const orc_cloak *c, const double *x, double *eo,
                        double *ee, double chat[3]) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    dual er, et, ez, o, e;
    eps_cyl(c, dk(r), &er, &et, &ez);
    uniaxial_split(c, er, et, ez, &o, &e);
    *eo = o.v;
    *ee = e.v;
    if (c->axis == ORC_AXIS_RADIAL) {
        chat[0] = x[0] / r; chat[1] = x[1] / r; chat[2] = 0.0;
    } else {
        chat[0] = -x[1] / r; chat[1] = x[0] / r; chat[2] = 0.0;
    }
}

/* Eq. (1) rotated to Cartesian axes from (eps_o, eps_e, c), then Eq. (7). */
static void metric_from_axis(double eo, double ee, const double chat[3], double M[3][3]) {
    double E[3][3], Ei[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double cc = chat[i] * chat[j];
            E[i][j] = eo * ((i == j ? 1.0 : 0.0) - cc) + ee * cc;
        }
    inv3(E, Ei);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i][j] = eo * ee * Ei[i][j];
}

/* ------------------------------------------------------------------ */
/* ray equations of motion                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    const orc_cloak *c;
    int branch;
} rhs_ctx;

/* Eq. (8): dv/dt = 1/2 M^-1 [ v (grad M) v - 2 ((grad M) . v) v ], with
   [v (grad M) v]_k = v^T (d_k M) v and ((grad M) . v) = sum_k v_k d_k M. */
static void rhs_eq8_with(void (*mfun)(const orc_cloak *, const dual *, dual (*)[3]),
                         void (*minv)(const orc_cloak *, const double *, double (*)[3]),
                         const orc_cloak *c, const double *y, double *dy) {
    double M[3][3], dM[3][3][3];
    for (int k = 0; k < 3; k++) {
        dual x[3];
        for (int i = 0; i < 3; i++) x[i] = mkd(y[i], i == k ? 1.0 : 0.0);
        dual Md[3][3];
        mfun(c, x, Md);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                M[i][j] = Md[i][j].v;
                dM[k][i][j] = Md[i][j].d;
            }
    }
    double Mi[3][3];
    if (minv) minv(c, y, Mi);
    else inv3(M, Mi);
    const double *v = y + 3;
    double w[3], gv[3], rhs[3];
    for (int k = 0; k < 3; k++) {
        double s = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) s += v[i] * dM[k][i][j] * v[j];
        w[k] = s;
    }
    for (int i = 0; i < 3; i++) {
        double s = 0.0;
        for (int k = 0; k < 3; k++)
            for (int j = 0; j < 3; j++) s += v[k] * dM[k][i][j] * v[j];
        gv[i] = s;
    }
    for (int i = 0; i < 3; i++) {
        double s = 0.0;
        for (int j = 0; j < 3; j++) s += Mi[i][j] * (w[j] - 2.0 * gv[j]);
        rhs[i] = 0.5 * s;
    }
    dy[0] = v[0]; dy[1] = v[1]; dy[2] = v[2];
    dy[3] = rhs[0]; dy[4] = rhs[1]; dy[5] = rhs[2];
}

static void metric_e_cb(const orc_cloak *c, const dual *x, dual (*M)[3]) {
    metric_dual(c, x, M);
}

/* isotropic test metric n_o^2 I (used to check Eq. (8) against Eq. (2)) */
static void metric_iso_cb(const orc_cloak *c, const dual *x, dual (*M)[3]) {
    dual E[3][3], eo, ee;
    eps_cart(c, x, E, &eo, &ee);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[i][j] = (i == j) ? eo : dk(0.0);
}

/* Eq. (2): dv/dt = (|v|^2 grad n_o - 2 (grad n_o . v) v) / n_o. */
static void rhs_eq2(const orc_cloak *c, const double *y, double *dy) {
    double g[3], n = 0.0;
    for (int k = 0; k < 3; k++) {
        dual x[3];
        for (int i = 0; i < 3; i++) x[i] = mkd(y[i], i == k ? 1.0 : 0.0);
        dual E[3][3], eo, ee;
        eps_cart(c, x, E, &eo, &ee);
        dual no = dsqrt(eo);
        g[k] = no.d;
        n = no.v;
    }
    const double *v = y + 3;
    double vv = dot3(v, v), gv = dot3(g, v);
    dy[0] = v[0]; dy[1] = v[1]; dy[2] = v[2];
    for (int i = 0; i < 3; i++) dy[3 + i] = (vv * g[i] - 2.0 * gv * v[i]) / n;
}

static void rhs_fn(const rhs_ctx *ctx, const double *y, double *dy) {
    if (ctx->branch == ORC_EXTRAORDINARY) rhs_eq8_with(metric_e_cb, metric_inv, ctx->c, y, dy);
    else rhs_eq2(ctx->c, y, dy);
}

/* Ray Hamiltonian: v^T M v (extraordinary) or n_o^2 |v|^2 (ordinary); 1 on
   every exact ray because k^T M^-1 k = 1 (Eq. (6) with the dispersion
   relation of the uniaxial medium). */
static double hamiltonian(const orc_cloak *c, int branch, const double *y) {
    double eo, ee, ch[3];
    material_at(c, y, &eo, &ee, ch);
    const double *v = y + 3;
    if (branch == ORC_ORDINARY) return eo * dot3(v, v);
    double M[3][3];
    metric_from_axis(eo, ee, ch, M);
    double s = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) s += v[i] * M[i][j] * v[j];
    return s;
}

/* ------------------------------------------------------------------ */
/* steppers                                                            */
/* ------------------------------------------------------------------ */
typedef void (*ode_fn)(const void *ctx, const double *y, double *dy);

static void rk4_step(ode_fn f, const void *ctx, const double *y, double h, double *out) {
    double k1[6], k2[6], k3[6], k4[6], t[6];
    f(ctx, y, k1);
    for (int i = 0; i < 6; i++) t[i] = y[i] + 0.5 * h * k1[i];
    f(ctx, t, k2);
    for (int i = 0; i < 6; i++) t[i] = y[i] + 0.5 * h * k2[i];
    f(ctx, t, k3);
    for (int i = 0; i < 6; i++) t[i] = y[i] + h * k3[i];
    f(ctx, t, k4);
    for (int i = 0; i < 6; i++)
        out[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* Dormand & Prince (1980), RK5(4)7M: fifth-order propagation, embedded
   fourth-order error estimate, first-same-as-last. */
static const double DP_A[7][6] = {
    { 0, 0, 0, 0, 0, 0 },
    { 1.0 / 5, 0, 0, 0, 0, 0 },
    { 3.0 / 40, 9.0 / 40, 0, 0, 0, 0 },
    { 44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0 },
    { 19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0 },
    { 9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0 },
    { 35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84 },
};
static const double DP_B5[7] = { 35.0 / 384, 0, 500.0 / 1113, 125.0 / 192,
                                 -2187.0 / 6784, 11.0 / 84, 0 };
static const double DP_B4[7] = { 5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                 -92097.0 / 339200, 187.0 / 2100, 1.0 / 40 };

/* One DP45 attempt from y with f(y) = k1. out = fifth-order solution, k7 =
   f(out). Returns the RMS error norm over the six components scaled by
   atol + rtol max(|y_i|, |out_i|). */
static double dp45_step(ode_fn f, const void *ctx, const double *y, const double *k1,
                        double h, double rtol, double atol, double *out, double *k7) {
    double k[7][6], t[6];
    memcpy(k[0], k1, sizeof(double) * 6);
    for (int s = 1; s < 7; s++) {
        for (int i = 0; i < 6; i++) {
            double acc = 0.0;
            for (int j = 0; j < s; j++) acc += DP_A[s][j] * k[j][i];
            t[i] = y[i] + h * acc;
        }
        if (s == 6) memcpy(out, t, sizeof(double) * 6);
        f(ctx, t, k[s]);
    }
    memcpy(k7, k[6], sizeof(double) * 6);
    double sum = 0.0;
    for (int i = 0; i < 6; i++) {
        double e = 0.0;
        for (int j = 0; j < 7; j++) e += (DP_B5[j] - DP_B4[j]) * k[j][i];
        e *= h;
        double sc = atol + rtol * fmax(fabs(y[i]), fabs(out[i]));
        sum += (e / sc) * (e / sc);
    }
    return sqrt(sum / 6.0);
}

/* Step-size update of the adaptive runs: safety 0.9, exponent -1/5,
   factor clipped to [0.2, 5], no growth right after a rejection. */
static double dp45_factor(double err, int after_reject) {
    double fac;
    if (err == 0.0) fac = 5.0;
    else if (!(err == err)) fac = 0.2;
    else fac = fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    if (after_reject && fac > 1.0) fac = 1.0;
    return fac;
}

/* ------------------------------------------------------------------ */
/* integration inside the cloak with boundary events                   */
/* ------------------------------------------------------------------ */
enum { EV_SIDE = 0, EV_INNER = 1, EV_TOP = 2, EV_BOTTOM = 3, EV_MAXSTEPS = 10, EV_DIVERGED = 11 };

static void ode_cb(const void *ctx, const double *y, double *dy) {
    rhs_fn((const rhs_ctx *)ctx, y, dy);
}

static double gfun(const orc_cloak *c, int id, const double *y) {
    double r = sqrt(y[0] * y[0] + y[1] * y[1]);
    switch (id) {
    case EV_SIDE: return r - c->b;
    case EV_INNER: return c->a - r;
    case EV_TOP: return y[2] - c->z1;
    default: return c->z0 - y[2];
    }
}

static int all_finite(const double *y) {
    for (int i = 0; i < 6; i++)
        if (!isfinite(y[i])) return 0;
    return 1;
}

/* the single-step map of the active scheme */
static void step_map(const orc_opts *o, const rhs_ctx *ctx, const double *y,
                     const double *k1, double h, double *out) {
    if (o->scheme == ORC_RK4) {
        rk4_step(ode_cb, ctx, y, h, out);
    } else {
        double k7[6];
        (void)dp45_step(ode_cb, ctx, y, k1, h, o->rtol, o->atol, out, k7);
    }
}

/* Bisection for the step length hs in (0, h] at which the step map puts the
   state on boundary `id`, to |g| <= 1e-13 b; g < 0 at 0 and g >= 0 at h. */
static double crossing(const orc_cloak *c, const orc_opts *o, const rhs_ctx *ctx,
                       const double *y, const double *k1, double h, int id, double *yout) {
    double lo = 0.0, hi = h, mid = h, tol = 1e-13 * c->b;
    double ym[6];
    for (int it = 0; it < 400; it++) {
        double m = 0.5 * (lo + hi);
        if (!(m > lo && m < hi)) break; /* bracket at machine resolution */
        mid = m;
        step_map(o, ctx, y, k1, mid, ym);
        double g = gfun(c, id, ym);
        if (fabs(g) <= tol) break;
        if (g < 0.0) lo = mid; else hi = mid;
    }
    step_map(o, ctx, y, k1, mid, yout);
    return mid;
}

/* Integrate from y until the state leaves a < r < b, z0 < z < z1. On an
   event, y is the state on the boundary, *t is advanced and the event id is
   returned. */
static int integrate(const orc_cloak *c, int branch, const orc_opts *o, double *y,
                     double *t, int64_t *nsteps) {
    rhs_ctx ctx = { c, branch };
    double h = o->h, k1[6], k7[6], yn[6];
    int after_reject = 0;
    if (o->scheme == ORC_DP45) ode_cb(&ctx, y, k1);
    for (;;) {
        if (*nsteps >= o->max_steps) return EV_MAXSTEPS;
        (*nsteps)++;
        double h_next = h;
        if (o->scheme == ORC_RK4) {
            rk4_step(ode_cb, &ctx, y, h, yn);
        } else {
            double err = dp45_step(ode_cb, &ctx, y, k1, h, o->rtol, o->atol, yn, k7);
            if (!(err <= 1.0)) {
                h *= dp45_factor(err, 0);
                after_reject = 1;
                if (!(h >= 1e-12)) return EV_DIVERGED;
                continue;
            }
            h_next = fmin(h * dp45_factor(err, after_reject), o->hmax);
            after_reject = 0;
        }
        if (!all_finite(yn)) return EV_DIVERGED;
        int first = -1;
        double hfirst = 0.0, yfirst[6];
        for (int id = 0; id < 4; id++) {
            if (gfun(c, id, yn) >= 0.0) {
                double yc[6];
                double hc = crossing(c, o, &ctx, y, k1, h, id, yc);
                if (first < 0 || hc < hfirst) {
                    first = id; hfirst = hc;
                    memcpy(yfirst, yc, sizeof(yc));
                }
            }
        }
        /* The radial cloak's ordinary branch moves in a homogeneous medium
           (Eq. (14): eps_o = kappa constant), so a step is a straight chord,
           and a chord can dip into r < a and come back out within one step
           with both ends outside: its point of closest approach to the axis
           then lies inside, and the crossing is searched before it. */
        if (first < 0 && c->axis == ORC_AXIS_RADIAL && branch == ORC_ORDINARY) {
            double dx = yn[0] - y[0], dy = yn[1] - y[1];
            double dd = dx * dx + dy * dy;
            if (dd > 0.0) {
                double f = -(y[0] * dx + y[1] * dy) / dd;
                double px = y[0] + f * dx, py = y[1] + f * dy;
                if (f > 0.0 && f < 1.0 && px * px + py * py < c->a * c->a) {
                    double yc[6];
                    hfirst = crossing(c, o, &ctx, y, k1, f * h, EV_INNER, yc);
                    first = EV_INNER;
                    memcpy(yfirst, yc, sizeof(yc));
                }
            }
        }
        if (first >= 0) {
            memcpy(y, yfirst, sizeof(yfirst));
            *t += hfirst;
            return first;
        }
        memcpy(y, yn, sizeof(yn));
        *t += h;
        if (o->scheme == ORC_DP45) memcpy(k1, k7, sizeof(k7));
        h = h_next;
    }
}

/* ------------------------------------------------------------------ */
/* Hamiltonian form of the ray equations (Sect. 4: the alternative the  */
/* paper compares its Eq. (8) tracer against)                          */
/* ------------------------------------------------------------------ */
/* H(x, k) = k^T A(x) k - f(x) vanishes on every ray. Extraordinary wave:
   A = eps, f = eps_o eps_e, since k^T eps k = eps_o eps_e is the uniaxial
   dispersion relation (Eq. (6) with M = eps_o eps_e eps^-1, Eq. (7)).
   Ordinary wave: A = I, f = eps_o. With the ray parameter tau,
   dx/dtau = dH/dk = 2 A k and dk/dtau = -dH/dx; because the ray velocity is
   v = dx/dt = M^-1 k = A k / f, the optical path advances as dt/dtau = 2 f.
   The canonical normalization (canon) is H' = H / f = k^T M^-1 k - 1, the
   same form with A / f in place of A and 1 in place of f: the same rays, the
   ray parameter proportional to the optical path (dt/dtau = 2). */
static void ham_parts(const orc_cloak *c, int branch, const dual x[3], dual A[3][3], dual *f, int canon) {
    dual E[3][3], eo, ee;
    eps_cart(c, x, E, &eo, &ee);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            A[i][j] = branch == ORC_EXTRAORDINARY ? E[i][j] : dk(i == j ? 1.0 : 0.0);
    *f = branch == ORC_EXTRAORDINARY ? dmul(eo, ee) : eo;
    if (canon) {
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) A[i][j] = ddiv(A[i][j], *f);
        *f = dk(1.0);
    }
}

/* y = (x, k, t): dy/dtau, the gradient of H by forward-mode duals */
static void rhs_ham(const orc_cloak *c, int branch, const double *y, double *dy, int canon) {
    const double *k = y + 3;
    double A[3][3], dH[3], f = 0.0;
    for (int m = 0; m < 3; m++) {
        dual x[3], Ad[3][3], fd;
        for (int i = 0; i < 3; i++) x[i] = mkd(y[i], i == m ? 1.0 : 0.0);
        ham_parts(c, branch, x, Ad, &fd, canon);
        double s = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                A[i][j] = Ad[i][j].v;
                s += k[i] * Ad[i][j].d * k[j];
            }
        dH[m] = s - fd.d;
        f = fd.v;
    }
    for (int i = 0; i < 3; i++) {
        double s = 0.0;
        for (int j = 0; j < 3; j++) s += A[i][j] * k[j];
        dy[i] = 2.0 * s;
        dy[3 + i] = -dH[i];
    }
    dy[6] = 2.0 * f;
}

/* classical RK4 in tau on the 7-component state (x, k, t) */
static void rk4_ham(const orc_cloak *c, int branch, const double *y, double h, double *out, int canon) {
    double k1[7], k2[7], k3[7], k4[7], t[7];
    rhs_ham(c, branch, y, k1, canon);
    for (int i = 0; i < 7; i++) t[i] = y[i] + 0.5 * h * k1[i];
    rhs_ham(c, branch, t, k2, canon);
    for (int i = 0; i < 7; i++) t[i] = y[i] + 0.5 * h * k2[i];
    rhs_ham(c, branch, t, k3, canon);
    for (int i = 0; i < 7; i++) t[i] = y[i] + h * k3[i];
    rhs_ham(c, branch, t, k4, canon);
    for (int i = 0; i < 7; i++)
        out[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

/* k = M v = f A^-1 v, and back v = A k / f, at the point x */
static void ham_v_to_k(const orc_cloak *c, int branch, const double *x, const double *v, double *k) {
    dual xd[3] = { dk(x[0]), dk(x[1]), dk(x[2]) }, Ad[3][3], fd;
    ham_parts(c, branch, xd, Ad, &fd, 0);
    double A[3][3], Ai[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) A[i][j] = Ad[i][j].v;
    inv3(A, Ai);
    for (int i = 0; i < 3; i++) k[i] = fd.v * (Ai[i][0] * v[0] + Ai[i][1] * v[1] + Ai[i][2] * v[2]);
}

static void ham_k_to_v(const orc_cloak *c, int branch, const double *x, const double *k, double *v) {
    dual xd[3] = { dk(x[0]), dk(x[1]), dk(x[2]) }, Ad[3][3], fd;
    ham_parts(c, branch, xd, Ad, &fd, 0);
    for (int i = 0; i < 3; i++)
        v[i] = (Ad[i][0].v * k[0] + Ad[i][1].v * k[1] + Ad[i][2].v * k[2]) / fd.v;
}

/* bisection on the tau step for boundary `id`, as crossing() */
static double crossing_ham(const orc_cloak *c, int branch, const double *y, double h, int id,
                           double *yout, int canon) {
    double lo = 0.0, hi = h, mid = h, tol = 1e-13 * c->b;
    double ym[7];
    for (int it = 0; it < 400; it++) {
        double m = 0.5 * (lo + hi);
        if (!(m > lo && m < hi)) break;
        mid = m;
        rk4_ham(c, branch, y, mid, ym, canon);
        double g = gfun(c, id, ym);
        if (fabs(g) <= tol) break;
        if (g < 0.0) lo = mid; else hi = mid;
    }
    rk4_ham(c, branch, y, mid, yout, canon);
    return mid;
}

/* integrate() for the Hamiltonian form with fixed RK4 steps in tau. y holds
   (x, v) on entry and return (converted to and from k at the ends); *t
   advances by the optical path. */
static int integrate_ham(const orc_cloak *c, int branch, const orc_opts *o, double *y,
                         double *t, int64_t *nsteps) {
    const int canon = o->scheme == ORC_RK4_HAMC;
    double z[7], zn[7], h = o->h;
    memcpy(z, y, 3 * sizeof(double));
    ham_v_to_k(c, branch, y, y + 3, z + 3);
    z[6] = 0.0;
    int ev = -1;
    for (;;) {
        if (*nsteps >= o->max_steps) { ev = EV_MAXSTEPS; break; }
        (*nsteps)++;
        rk4_ham(c, branch, z, h, zn, canon);
        int fin = 1;
        for (int i = 0; i < 7; i++) fin &= isfinite(zn[i]) ? 1 : 0;
        if (!fin) { ev = EV_DIVERGED; break; }
        int first = -1;
        double hfirst = 0.0, zfirst[7];
        for (int id = 0; id < 4; id++) {
            if (gfun(c, id, zn) >= 0.0) {
                double zc[7];
                double hc = crossing_ham(c, branch, z, h, id, zc, canon);
                if (first < 0 || hc < hfirst) {
                    first = id; hfirst = hc;
                    memcpy(zfirst, zc, sizeof(zc));
                }
            }
        }
        /* radial-o: straight chords (A = I, f constant); a chord can dip
           into r < a and leave it again within one step */
        if (first < 0 && c->axis == ORC_AXIS_RADIAL && branch == ORC_ORDINARY) {
            double dx = zn[0] - z[0], dy = zn[1] - z[1];
            double dd = dx * dx + dy * dy;
            if (dd > 0.0) {
                double f = -(z[0] * dx + z[1] * dy) / dd;
                double px = z[0] + f * dx, py = z[1] + f * dy;
                if (f > 0.0 && f < 1.0 && px * px + py * py < c->a * c->a) {
                    crossing_ham(c, branch, z, f * h, EV_INNER, zfirst, canon);
                    first = EV_INNER;
                }
            }
        }
        if (first >= 0) {
            memcpy(z, zfirst, sizeof(zfirst));
            ev = first;
            break;
        }
        memcpy(z, zn, sizeof(zn));
    }
    memcpy(y, z, 3 * sizeof(double));
    ham_k_to_v(c, branch, z, z + 3, y + 3);
    *t += z[6];
    return ev;
}

/* ------------------------------------------------------------------ */
/* Sect. 3: refraction at the vacuum/crystal interface                 */
/* ------------------------------------------------------------------ */

/* Eq. (9): index seen by the extraordinary wave whose polarization makes the
   angle phi with the optic axis. */
static double n_of_phi(double no, double ne, double phi) {
    double cp = cos(phi), sp = sin(phi);
    return no * ne / sqrt(no * no * cp * cp + ne * ne * sp * sp);
}

/* Eq. (10): polarization angle for refraction angle vphi; k_hat =
   sin(vphi) t_hat - cos(vphi) n_hat with n_hat the outward normal. */
static double phi_of(double ct, double cn, double vphi) {
    double s = ct * sin(vphi) - cn * cos(vphi);
    if (s > 1.0) s = 1.0;
    if (s < -1.0) s = -1.0;
    return asin(s);
}

/* a unit tangent for normal incidence (any direction perpendicular to n) */
static void any_tangent(const double *n, double *t) {
    double a[3] = { 1.0, 0.0, 0.0 };
    if (fabs(n[0]) > 0.9) { a[0] = 0.0; a[1] = 1.0; }
    double d = dot3(a, n);
    for (int i = 0; i < 3; i++) t[i] = a[i] - d * n[i];
    double l = norm3(t);
    for (int i = 0; i < 3; i++) t[i] /= l;
}

int32_t orc_refract_in(double eps_o, double eps_e, const double chat[3],
                       const double nhat[3], const double kin[3], int32_t branch,
                       double k_out[3], double v_out[3]) {
    double cos_i = -dot3(kin, nhat);
    double kt[3], th[3];
    for (int i = 0; i < 3; i++) kt[i] = kin[i] + cos_i * nhat[i];
    double sin_i = norm3(kt);
    if (sin_i > 1e-300) {
        for (int i = 0; i < 3; i++) th[i] = kt[i] / sin_i;
    } else {
        sin_i = 0.0;
        any_tangent(nhat, th);
    }
    double no = sqrt(eps_o), ne = sqrt(eps_e);
    double vphi, n;
    if (branch == ORC_ORDINARY) {
        /* Eq. (11), ordinary part: sin(phi_i) = n_o sin(phi_o) */
        double s = sin_i / no;
        if (s > 1.0) return 1;
        vphi = asin(s);
        n = no;
        for (int i = 0; i < 3; i++) k_out[i] = n * (sin(vphi) * th[i] - cos(vphi) * nhat[i]);
        for (int i = 0; i < 3; i++) v_out[i] = k_out[i] / eps_o;
        return 0;
    }
    /* Eq. (11), extraordinary part: sin(phi_i) = n(phi_e(vphi)) sin(vphi),
       one root in [0, pi/2]; bisection on F(vphi) = n sin(vphi) - sin(phi_i). */
    double ct = dot3(chat, th), cn = dot3(chat, nhat);
    double lo = 0.0, hi = 0.5 * M_PI;
    double Fhi = n_of_phi(no, ne, phi_of(ct, cn, hi)) - sin_i;
    if (Fhi < 0.0) return 1;
    if (sin_i == 0.0) {
        vphi = 0.0;
    } else {
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (lo + hi);
            double F = n_of_phi(no, ne, phi_of(ct, cn, mid)) * sin(mid) - sin_i;
            if (F < 0.0) lo = mid; else hi = mid;
            if (!(hi - lo > 1e-17)) break;
        }
        vphi = 0.5 * (lo + hi);
    }
    n = n_of_phi(no, ne, phi_of(ct, cn, vphi));
    for (int i = 0; i < 3; i++) k_out[i] = n * (sin(vphi) * th[i] - cos(vphi) * nhat[i]);
    /* Eq. (6) with c0 = omega = 1: v = M^-1 k */
    double M[3][3], Mi[3][3];
    metric_from_axis(eps_o, eps_e, chat, M);
    inv3(M, Mi);
    for (int i = 0; i < 3; i++)
        v_out[i] = Mi[i][0] * k_out[0] + Mi[i][1] * k_out[1] + Mi[i][2] * k_out[2];
    return 0;
}

int32_t orc_refract_out(double eps_o, double eps_e, const double chat[3],
                        const double nhat[3], const double v_in[3], int32_t branch,
                        double d_out[3]) {
    double k[3];
    if (branch == ORC_ORDINARY) {
        for (int i = 0; i < 3; i++) k[i] = eps_o * v_in[i];
    } else {
        /* Eq. (6) inverted: k = M v */
        double M[3][3];
        metric_from_axis(eps_o, eps_e, chat, M);
        for (int i = 0; i < 3; i++) k[i] = M[i][0] * v_in[0] + M[i][1] * v_in[1] + M[i][2] * v_in[2];
    }
    /* Eq. (11) towards air: sin(phi_t) = n(phi_e) sin(phi_e) with n = |k| and
       phi_e the angle of k to the normal. */
    double kn = dot3(k, nhat), kt[3], th[3];
    for (int i = 0; i < 3; i++) kt[i] = k[i] - kn * nhat[i];
    double ktl = norm3(kt);
    double n_in = norm3(k);
    double phi_e = atan2(ktl, fabs(kn));
    double sin_t = n_in * sin(phi_e);
    if (sin_t > 1.0) return 1;
    if (ktl > 0.0) {
        for (int i = 0; i < 3; i++) th[i] = kt[i] / ktl;
    } else {
        any_tangent(nhat, th);
    }
    double cos_t = sqrt(1.0 - sin_t * sin_t);
    for (int i = 0; i < 3; i++) d_out[i] = sin_t * th[i] + cos_t * nhat[i];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sect. 3, Eq. (12): intensity transmission at the interface          */
/* ------------------------------------------------------------------ */
/* Plane waves exp(i k.x) with omega = c0 = 1 and mu = 1: H = k x E and
   D = -k x H = eps E. Crystal: eps = eps_o (I - c c^T) + eps_e c c^T.
   Ordinary wave: E = k x c, k.k = eps_o. Extraordinary wave: D in the plane
   of k and c and perpendicular to k, D = (k.k) c - (c.k) k, E = eps^-1 D,
   k^T eps k = eps_o eps_e. Normal components q of k = kt + q n come from the
   dispersion relations; complex q (evanescent waves) are allowed. The
   boundary conditions are continuity of tangential E and H; the powers are
   the normal components of Re(E x H*) / 2 (Eq. (12)). */
typedef double complex zc;

static void zcross(const zc a[3], const zc b[3], zc r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static zc zdot(const zc a[3], const zc b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double zflux(const zc E[3], const zc H[3], const double n[3]) {
    zc Hc[3] = { conj(H[0]), conj(H[1]), conj(H[2]) }, S[3];
    zcross(E, Hc, S);
    return 0.5 * creal(S[0] * n[0] + S[1] * n[1] + S[2] * n[2]);
}

/* normal component of the wave vector: dir = +1 for a wave that carries
   power towards +n (or decays towards +n), -1 towards -n */
static zc q_iso(double eps, double ktt, int dir) {
    double d = eps - ktt;
    return d >= 0.0 ? dir * sqrt(d) : dir * I * sqrt(-d);
}

static zc q_extra(double eo, double ee, const double c[3], const double n[3], const double kt[3], int dir) {
    /* (n^T eps n) q^2 + 2 (n^T eps kt) q + kt^T eps kt - eo ee = 0; the ray
       direction eps k has normal component (n^T eps kt) + q (n^T eps n) */
    double cn = dot3(c, n), ck = dot3(c, kt);
    double a = eo + (ee - eo) * cn * cn;
    double b = eo * dot3(n, kt) + (ee - eo) * cn * ck;
    double c0 = eo * dot3(kt, kt) + (ee - eo) * ck * ck - eo * ee;
    double disc = b * b - a * c0;
    return disc >= 0.0 ? (-b + dir * sqrt(disc)) / a : (-b + dir * I * sqrt(-disc)) / a;
}

/* fields of a crystal mode with wave vector k; t1 is a tangent used where
   k is along c (ordinary and extraordinary waves then coincide) */
static void crystal_mode(double eo, double ee, const double c[3], int ordinary, const zc k[3],
                         const double t1[3], zc E[3], zc H[3]) {
    zc cz[3] = { c[0], c[1], c[2] };
    zc kc[3];
    zcross(k, cz, kc);
    double kk = creal(zdot(k, (const zc[3]){ conj(k[0]), conj(k[1]), conj(k[2]) }));
    double deg = creal(zdot(kc, (const zc[3]){ conj(kc[0]), conj(kc[1]), conj(kc[2]) }));
    if (deg <= 1e-24 * kk) {
        zc u[3] = { t1[0], t1[1], t1[2] };
        if (ordinary) {
            for (int i = 0; i < 3; i++) E[i] = u[i];
        } else {
            zcross(k, u, E);
        }
    } else if (ordinary) {
        for (int i = 0; i < 3; i++) E[i] = kc[i];
    } else {
        zc kkz = zdot(k, k), ckz = zdot(cz, k), D[3];
        for (int i = 0; i < 3; i++) D[i] = kkz * cz[i] - ckz * k[i];
        zc cd = zdot(cz, D);
        for (int i = 0; i < 3; i++) E[i] = (D[i] - cd * cz[i]) / eo + cd * cz[i] / ee;
    }
    zcross(k, E, H);
}

/* complex Gaussian elimination with partial pivoting, 4 x 4 */
static int zsolve4(zc A[4][4], zc b[4], zc x[4]) {
    for (int col = 0; col < 4; col++) {
        int piv = col;
        for (int r = col + 1; r < 4; r++)
            if (cabs(A[r][col]) > cabs(A[piv][col])) piv = r;
        if (cabs(A[piv][col]) == 0.0) return 1;
        if (piv != col) {
            for (int j = 0; j < 4; j++) { zc t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
            zc t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < 4; r++) {
            zc f = A[r][col] / A[col][col];
            for (int j = col; j < 4; j++) A[r][j] -= f * A[col][j];
            b[r] -= f * b[col];
        }
    }
    for (int r = 3; r >= 0; r--) {
        zc s = b[r];
        for (int j = r + 1; j < 4; j++) s -= A[r][j] * x[j];
        x[r] = s / A[r][r];
    }
    return 0;
}

static void tangent_basis(const double n[3], const double kt[3], double t1[3], double t2[3]) {
    double l = norm3(kt);
    if (l > 1e-12) {
        for (int i = 0; i < 3; i++) t1[i] = kt[i] / l;
    } else {
        any_tangent(n, t1);
    }
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

/* rows: tangential E (t1, t2), tangential H (t1, t2) of a field pair */
static void tangential(const zc E[3], const zc H[3], const double t1[3], const double t2[3], zc col[4]) {
    col[0] = E[0] * t1[0] + E[1] * t1[1] + E[2] * t1[2];
    col[1] = E[0] * t2[0] + E[1] * t2[1] + E[2] * t2[2];
    col[2] = H[0] * t1[0] + H[1] * t1[1] + H[2] * t1[2];
    col[3] = H[0] * t2[0] + H[1] * t2[1] + H[2] * t2[2];
}

/* the waves of an entry: the two reflected vacuum polarizations (s along
   t2, perpendicular to the plane of incidence, and p) and the two
   refracted crystal waves, as field pairs */
typedef struct {
    double t1[3], t2[3];
    zc s[3], ki[3];
    zc Es[3], Hs[3], Ep[3], Hp[3], Eo[3], Ho[3], Ee[3], He[3];
} entry_waves;

static void entry_setup(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                        const double kin[3], entry_waves *w) {
    double kn = dot3(kin, nhat), kt[3];
    for (int i = 0; i < 3; i++) kt[i] = kin[i] - kn * nhat[i];
    tangent_basis(nhat, kt, w->t1, w->t2);
    double ktt = dot3(kt, kt);
    zc qr = q_iso(1.0, ktt, +1), qo = q_iso(eps_o, ktt, -1), qe = q_extra(eps_o, eps_e, chat, nhat, kt, -1);
    zc kr[3], ko[3], ke[3];
    for (int i = 0; i < 3; i++) {
        kr[i] = kt[i] + qr * nhat[i];
        ko[i] = kt[i] + qo * nhat[i];
        ke[i] = kt[i] + qe * nhat[i];
        w->ki[i] = kin[i];
        w->s[i] = w->t2[i];
    }
    for (int i = 0; i < 3; i++) w->Es[i] = w->s[i];
    zcross(kr, w->Es, w->Hs);
    zcross(kr, w->Es, w->Ep);
    zcross(kr, w->Ep, w->Hp);
    crystal_mode(eps_o, eps_e, chat, 1, ko, w->t1, w->Eo, w->Ho);
    crystal_mode(eps_o, eps_e, chat, 0, ke, w->t1, w->Ee, w->He);
}

/* continuity of tangential E and H for the incident field Ei (transverse to
   kin): the flux into each wave over the incident flux */
static int entry_solve(const entry_waves *w, const double nhat[3], const zc Ei[3], double *To, double *Te,
                       double *Rr) {
    zc Hi[3];
    zcross(w->ki, Ei, Hi);
    zc cols[4][4], A[4][4], b[4], x[4];
    tangential(w->Es, w->Hs, w->t1, w->t2, cols[0]);
    tangential(w->Ep, w->Hp, w->t1, w->t2, cols[1]);
    tangential(w->Eo, w->Ho, w->t1, w->t2, cols[2]);
    tangential(w->Ee, w->He, w->t1, w->t2, cols[3]);
    zc inc[4];
    tangential(Ei, Hi, w->t1, w->t2, inc);
    for (int r = 0; r < 4; r++) {
        A[r][0] = cols[0][r];
        A[r][1] = cols[1][r];
        A[r][2] = -cols[2][r];
        A[r][3] = -cols[3][r];
        b[r] = -inc[r];
    }
    if (zsolve4(A, b, x)) return 1;
    double si = fabs(zflux(Ei, Hi, nhat));
    zc E1[3], H1[3];
    for (int i = 0; i < 3; i++) { E1[i] = x[2] * w->Eo[i]; H1[i] = x[2] * w->Ho[i]; }
    *To = fabs(zflux(E1, H1, nhat)) / si;
    for (int i = 0; i < 3; i++) { E1[i] = x[3] * w->Ee[i]; H1[i] = x[3] * w->He[i]; }
    *Te = fabs(zflux(E1, H1, nhat)) / si;
    for (int i = 0; i < 3; i++) { E1[i] = x[0] * w->Es[i] + x[1] * w->Ep[i]; H1[i] = x[0] * w->Hs[i] + x[1] * w->Hp[i]; }
    *Rr = fabs(zflux(E1, H1, nhat)) / si;
    return 0;
}

int32_t orc_fresnel_in(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                       const double kin[3], double T[2], double *R) {
    entry_waves w;
    entry_setup(eps_o, eps_e, chat, nhat, kin, &w);
    double To = 0.0, Te = 0.0, Rr = 0.0;
    for (int pol = 0; pol < 2; pol++) {
        zc Ei[3];
        if (pol == 0) {
            for (int i = 0; i < 3; i++) Ei[i] = w.s[i];
        } else {
            zcross(w.ki, w.s, Ei);
        }
        double to, te, rr;
        if (entry_solve(&w, nhat, Ei, &to, &te, &rr)) return 1;
        To += to;
        Te += te;
        Rr += rr;
    }
    T[0] = 0.5 * To;
    T[1] = 0.5 * Te;
    if (R) *R = 0.5 * Rr;
    return 0;
}

int32_t orc_fresnel_in_pol(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                           const double kin[3], const double e_in[3], double T[2], double *R) {
    /* the transverse part of e_in, normalized */
    double ek = dot3(e_in, kin), e[3];
    for (int i = 0; i < 3; i++) e[i] = e_in[i] - ek * kin[i];
    double l = norm3(e);
    if (!(l > 1e-12)) return 1;
    entry_waves w;
    entry_setup(eps_o, eps_e, chat, nhat, kin, &w);
    zc Ei[3] = { e[0] / l, e[1] / l, e[2] / l };
    double rr;
    if (entry_solve(&w, nhat, Ei, &T[0], &T[1], &rr)) return 1;
    if (R) *R = rr;
    return 0;
}

int32_t orc_fresnel_out(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                        const double k_in[3], int32_t branch, double *T, double R[2]) {
    double kn = dot3(k_in, nhat), kt[3], t1[3], t2[3];
    for (int i = 0; i < 3; i++) kt[i] = k_in[i] - kn * nhat[i];
    tangent_basis(nhat, kt, t1, t2);
    double ktt = dot3(kt, kt);
    zc qo = q_iso(eps_o, ktt, -1), qe = q_extra(eps_o, eps_e, chat, nhat, kt, -1), qv = q_iso(1.0, ktt, +1);
    zc km[3], ko[3], ke[3], kv[3];
    for (int i = 0; i < 3; i++) {
        km[i] = k_in[i];
        ko[i] = kt[i] + qo * nhat[i];
        ke[i] = kt[i] + qe * nhat[i];
        kv[i] = kt[i] + qv * nhat[i];
    }
    zc Em[3], Hm[3], Eo[3], Ho[3], Ee[3], He[3], Es[3], Hs[3], Ep[3], Hp[3];
    crystal_mode(eps_o, eps_e, chat, branch == ORC_ORDINARY, km, t1, Em, Hm);
    crystal_mode(eps_o, eps_e, chat, 1, ko, t1, Eo, Ho);
    crystal_mode(eps_o, eps_e, chat, 0, ke, t1, Ee, He);
    for (int i = 0; i < 3; i++) Es[i] = t2[i];
    zcross(kv, Es, Hs);
    zcross(kv, Es, Ep);
    zcross(kv, Ep, Hp);
    zc cols[4][4], A[4][4], b[4], x[4], inc[4];
    tangential(Eo, Ho, t1, t2, cols[0]);
    tangential(Ee, He, t1, t2, cols[1]);
    tangential(Es, Hs, t1, t2, cols[2]);
    tangential(Ep, Hp, t1, t2, cols[3]);
    tangential(Em, Hm, t1, t2, inc);
    for (int r = 0; r < 4; r++) {
        A[r][0] = cols[0][r];
        A[r][1] = cols[1][r];
        A[r][2] = -cols[2][r];
        A[r][3] = -cols[3][r];
        b[r] = -inc[r];
    }
    if (zsolve4(A, b, x)) return 1;
    double si = fabs(zflux(Em, Hm, nhat));
    zc E1[3], H1[3];
    for (int i = 0; i < 3; i++) { E1[i] = x[0] * Eo[i]; H1[i] = x[0] * Ho[i]; }
    R[0] = fabs(zflux(E1, H1, nhat)) / si;
    for (int i = 0; i < 3; i++) { E1[i] = x[1] * Ee[i]; H1[i] = x[1] * He[i]; }
    R[1] = fabs(zflux(E1, H1, nhat)) / si;
    for (int i = 0; i < 3; i++) { E1[i] = x[2] * Es[i] + x[3] * Ep[i]; H1[i] = x[2] * Hs[i] + x[3] * Hp[i]; }
    *T = fabs(zflux(E1, H1, nhat)) / si;
    return 0;
}

/* ------------------------------------------------------------------ */
/* vacuum geometry                                                     */
/* ------------------------------------------------------------------ */
enum { SURF_SIDE = 0, SURF_TOP = 2, SURF_BOTTOM = 3 };

/* First entry of the ray o + s d (s > 0) into the cloak body r <= b,
   z0 <= z <= z1. */
static int first_entry(const orc_cloak *c, const double *o, const double *d,
                       double *s_out, int *surf) {
    int found = 0;
    double best = INFINITY;
    double A = d[0] * d[0] + d[1] * d[1];
    double B = o[0] * d[0] + o[1] * d[1];
    double C = o[0] * o[0] + o[1] * o[1] - c->b * c->b;
    if (A > 0.0 && C > 0.0) {
        double disc = B * B - A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -(B + (B >= 0.0 ? sq : -sq));
            double s1 = q / A, s2 = C / q;
            double s = fmin(s1, s2);
            double z = o[2] + s * d[2];
            if (s > 0.0 && z >= c->z0 && z <= c->z1 && s < best) {
                best = s; *surf = SURF_SIDE; found = 1;
            }
        }
    }
    if (d[2] < 0.0 && o[2] > c->z1 && isfinite(c->z1)) {
        double s = (c->z1 - o[2]) / d[2];
        double x = o[0] + s * d[0], y = o[1] + s * d[1];
        if (s > 0.0 && x * x + y * y <= c->b * c->b && s < best) {
            best = s; *surf = SURF_TOP; found = 1;
        }
    }
    if (d[2] > 0.0 && o[2] < c->z0 && isfinite(c->z0)) {
        double s = (c->z0 - o[2]) / d[2];
        double x = o[0] + s * d[0], y = o[1] + s * d[1];
        if (s > 0.0 && x * x + y * y <= c->b * c->b && s < best) {
            best = s; *surf = SURF_BOTTOM; found = 1;
        }
    }
    *s_out = best;
    return found;
}

static void outward_normal(int surf, const double *x, double *n) {
    if (surf == SURF_TOP || surf == EV_TOP) { n[0] = 0; n[1] = 0; n[2] = 1; return; }
    if (surf == SURF_BOTTOM || surf == EV_BOTTOM) { n[0] = 0; n[1] = 0; n[2] = -1; return; }
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    n[0] = x[0] / r; n[1] = x[1] / r; n[2] = 0.0;
}

static void reflect(double *v, const double *n) {
    double d = dot3(v, n);
    for (int i = 0; i < 3; i++) v[i] -= 2.0 * d * n[i];
}

/* A crystal ray where it leaves: the wave met at the exit and what the
   interface reflects of it (Sect. 3: two reflected waves in the crystal,
   one refracted into vacuum). */
typedef struct {
    double x[3], n[3], k[3];  /* exit point, outward normal, wave vector k = M v met */
    double eo, ee, ch[3];     /* material at the exit */
    double Rref[2];           /* fractions reflected into the ordinary and extraordinary waves */
    double w_pre;             /* the ray's weight before the exit transmission */
} exit_state;

/* Follow a crystal ray of `branch` from y = (x, v) (inside the cloak or on
   its boundary heading in) until it leaves: specular reflection at the inner
   metal cylinder (radial cloak), same-mode specular reflection under total
   internal reflection (weight x that mode's reflectance), refraction into
   vacuum at the exit (Sect. 3). Returns the status; p/dout get the exit ray
   (or the last state), *t the optical path. With w, *w is multiplied by the
   reflectances and the exit transmission (0 unless the ray exits); with ex,
   an exit fills it. */
static int crystal_walk(const orc_cloak *c, int branch, const orc_opts *o, double *y, double *t,
                        int64_t *nsteps, double *w, exit_state *ex, double *p, double *dout, double *hres) {
    int bounces = 0, status;
    for (;;) {
        int ev = o->scheme == ORC_RK4_HAM || o->scheme == ORC_RK4_HAMC ? integrate_ham(c, branch, o, y, t, nsteps)
                                                                       : integrate(c, branch, o, y, t, nsteps);
        if (ev == EV_MAXSTEPS) { status = ORC_MAXSTEPS; break; }
        if (ev == EV_DIVERGED) { status = ORC_DIVERGED; break; }
        double nn[3];
        if (ev == EV_INNER) {
            if (c->inner_mirror && c->axis == ORC_AXIS_RADIAL && bounces < o->max_bounces) {
                /* optic axis along the mirror normal: one specular reflection
                   for either ray (Sect. 4) */
                outward_normal(SURF_SIDE, y, nn);
                reflect(y + 3, nn);
                bounces++;
                continue;
            }
            status = ORC_ABSORBED;
            break;
        }
        outward_normal(ev, y, nn);
        /* a ray whose Hamiltonian v^T M v has drifted from 1 by more than
           1e-3 at an outer interface is no longer a ray of the medium: its
           direction there is not a solution of the dispersion relation, and
           the refraction of Sect. 3 would act on an arbitrary vector */
        if (!(fabs(hamiltonian(c, branch, y) - 1.0) <= 1e-3)) { status = ORC_DIVERGED; break; }
        double eo2, ee2, ch2[3], dd[3], k[3];
        material_at(c, y, &eo2, &ee2, ch2);
        double Tout = 0.0, Rref[2] = { 0.0, 0.0 };
        if (w || ex) {
            /* k = M v of the wave meeting the interface */
            double M[3][3];
            if (branch == ORC_ORDINARY) {
                for (int i = 0; i < 3; i++) k[i] = eo2 * y[3 + i];
            } else {
                metric_from_axis(eo2, ee2, ch2, M);
                for (int i = 0; i < 3; i++) k[i] = M[i][0] * y[3] + M[i][1] * y[4] + M[i][2] * y[5];
            }
            if (orc_fresnel_out(eo2, ee2, ch2, nn, k, branch, &Tout, Rref) != 0) Tout = Rref[0] = Rref[1] = 0.0;
        }
        if (orc_refract_out(eo2, ee2, ch2, nn, y + 3, branch, dd) == 0) {
            *hres = fabs(hamiltonian(c, branch, y) - 1.0);
            memcpy(p, y, 3 * sizeof(double));
            memcpy(dout, dd, sizeof(dd));
            status = ORC_EXITED;
            if (ex) {
                memcpy(ex->x, y, 3 * sizeof(double));
                memcpy(ex->n, nn, sizeof(nn));
                memcpy(ex->k, k, sizeof(k));
                ex->eo = eo2;
                ex->ee = ee2;
                memcpy(ex->ch, ch2, sizeof(ch2));
                ex->Rref[0] = Rref[0];
                ex->Rref[1] = Rref[1];
                ex->w_pre = w ? *w : 0.0;
            }
            if (w) *w *= Tout;
            break;
        }
        /* total internal reflection: same-mode specular reflection */
        if (bounces >= o->max_bounces) { status = ORC_TIR; break; }
        if (w) *w *= Rref[branch];
        reflect(y + 3, nn);
        bounces++;
    }
    if (status != ORC_EXITED) {
        *hres = fabs(hamiltonian(c, branch, y) - 1.0);
        memcpy(p, y, 3 * sizeof(double));
        double l = norm3(y + 3);
        for (int i = 0; i < 3; i++) dout[i] = y[3 + i] / l;
        if (w) *w = 0.0;
    }
    return status;
}

/* First-order reflections of one camera ray through one branch (R27):
   the vacuum ray reflected at its first crystal interface, and the two
   waves the branch's ray reflects into at its exit, each followed to its
   own exit (their own reflections are of second order and not followed). */
typedef struct {
    double w_ext, p_ext[3], d_ext[3];          /* reflected flux fraction R at the entry (0: none) */
    double w_child[2], p_child[2][3], d_child[2][3];  /* weight and exit ray of the ordinary / extraordinary child */
} orc_refl;

/* Trace one vacuum ray through the cloak. On return p/dout hold the last
   vacuum ray (for MISSED the input ray), opl the optical path up to p. */
static int trace_vacuum(const orc_cloak *c, int branch, const orc_opts *o,
                        const double *o_in, const double *d_in, double *p, double *dout,
                        double *opl, double *hres, int64_t *nsteps, double *wt, const double *e_pol,
                        orc_refl *rf) {
    memcpy(p, o_in, 3 * sizeof(double));
    memcpy(dout, d_in, 3 * sizeof(double));
    *opl = 0.0;
    *hres = NAN;
    if (rf) memset(rf, 0, sizeof(*rf));
    /* Eq. (12) weight of the reported ray: 1 for a miss or a reflection off
       the metal end disk, the product of the entry transmission, the same-mode reflectances of internal reflections
       and the exit transmission for an exit, 0 otherwise. The entry takes
       unpolarized light, or with e_pol the vacuum field along e_pol. */
    if (wt) *wt = 0.0;
    if (!c) {
        if (wt) *wt = 1.0;
        return ORC_MISSED;
    }
    double s;
    int surf;
    if (!first_entry(c, o_in, d_in, &s, &surf)) {
        if (wt) *wt = 1.0;
        return ORC_MISSED;
    }
    double x[3];
    for (int i = 0; i < 3; i++) x[i] = o_in[i] + s * d_in[i];
    if (surf == SURF_TOP) x[2] = c->z1;
    if (surf == SURF_BOTTOM) x[2] = c->z0;
    *opl = s;
    double n[3];
    outward_normal(surf, x, n);
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    if (surf != SURF_SIDE && r <= c->a) {
        /* end disk of the inner metal cylinder */
        memcpy(p, x, sizeof(x));
        if (!c->inner_mirror) return ORC_ABSORBED;
        /* the perfect metal reflects every polarization: all of the light */
        reflect(dout, n);
        if (wt) *wt = 1.0;
        return ORC_REFLECTED;
    }
    double eo, ee, ch[3], k[3], v[3];
    material_at(c, x, &eo, &ee, ch);
    double w = 0.0;
    if (wt || rf) {
        double Tin[2], Rin = 0.0;
        int bad = e_pol ? orc_fresnel_in_pol(eo, ee, ch, n, d_in, e_pol, Tin, &Rin)
                        : orc_fresnel_in(eo, ee, ch, n, d_in, Tin, &Rin);
        if (!bad) w = Tin[branch];
        if (rf && !bad) {
            rf->w_ext = Rin;
            memcpy(rf->p_ext, x, sizeof(x));
            memcpy(rf->d_ext, d_in, 3 * sizeof(double));
            reflect(rf->d_ext, n);
        }
    }
    if (orc_refract_in(eo, ee, ch, n, d_in, branch, k, v)) {
        memcpy(p, x, sizeof(x));
        reflect(dout, n);
        if (wt) *wt = 0.0;
        return ORC_REFLECTED;
    }
    double y[6] = { x[0], x[1], x[2], v[0], v[1], v[2] };
    double t = 0.0;
    exit_state ex;
    int status = crystal_walk(c, branch, o, y, &t, nsteps, &w, rf ? &ex : NULL, p, dout, hres);
    *opl += t;
    if (wt) *wt = w;
    if (rf && status == ORC_EXITED) {
        /* the two reflected waves: the tangential wave vector of the wave met
           and each mode's dispersion relation, the root that carries power
           back into the crystal (the refraction of Sect. 3 read with the
           reflected wave vectors) */
        double kt[3], kn = dot3(ex.k, ex.n), kin[3];
        for (int i = 0; i < 3; i++) {
            kt[i] = ex.k[i] - kn * ex.n[i];
            kin[i] = kt[i] - ex.n[i];
        }
        for (int bp = 0; bp < 2; bp++) {
            double kc[3], vc[3];
            if (!(ex.Rref[bp] > 0.0) || orc_refract_in(ex.eo, ex.ee, ex.ch, ex.n, kin, bp, kc, vc)) continue;
            double yc[6] = { ex.x[0], ex.x[1], ex.x[2], vc[0], vc[1], vc[2] };
            double tc = 0.0, hc, wc = ex.w_pre * ex.Rref[bp];
            int64_t nc = 0;
            int sc = crystal_walk(c, bp, o, yc, &tc, &nc, &wc, NULL, rf->p_child[bp], rf->d_child[bp], &hc);
            rf->w_child[bp] = sc == ORC_EXITED ? wc : 0.0;
        }
    }
    return status;
}

/* larger root of |p + s d|_xy = R (the outgoing crossing), 0 if none */
static double leave_radius(const double *p, const double *d, double R) {
    double A = d[0] * d[0] + d[1] * d[1];
    if (!(A > 0.0)) return 0.0;
    double B = p[0] * d[0] + p[1] * d[1];
    double C = p[0] * p[0] + p[1] * p[1] - R * R;
    double disc = B * B - A * C;
    if (disc < 0.0) return 0.0;
    double sq = sqrt(disc);
    double s = (B <= 0.0) ? (-B + sq) / A : -C / (B + sq);
    return s > 0.0 ? s : 0.0;
}

static int origin_inside(const orc_cloak *c, const double *o) {
    double r2 = o[0] * o[0] + o[1] * o[1];
    return r2 < c->b * c->b && o[2] > c->z0 && o[2] < c->z1;
}

void orc_trace(const orc_cloak *c, const orc_opts *o, int32_t branch, int64_t n,
               const double *in6, double *out6, double *opl, int32_t *status,
               double *hres, int64_t *nsteps, double *trans) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double org[3], d[3], p[3], dout[3], L = 0.0, hr = NAN, w = 0.0;
        int64_t ns = 0;
        int st;
        for (int j = 0; j < 3; j++) { org[j] = in6[j * n + i]; d[j] = in6[(3 + j) * n + i]; }
        double dl = norm3(d);
        int ok = isfinite(org[0]) && isfinite(org[1]) && isfinite(org[2]) && isfinite(dl) && dl > 0.0;
        if (ok) {
            for (int j = 0; j < 3; j++) d[j] /= dl;
            ok = !origin_inside(c, org);
        }
        if (!ok) {
            st = ORC_INVALID;
            memcpy(p, org, sizeof(p));
            memcpy(dout, d, sizeof(dout));
        } else {
            st = trace_vacuum(c, branch, o, org, d, p, dout, &L, &hr, &ns, trans ? &w : NULL, NULL, NULL);
            if (st == ORC_EXITED || st == ORC_MISSED || st == ORC_REFLECTED) {
                double s = leave_radius(p, dout, o->r_out);
                for (int j = 0; j < 3; j++) p[j] += s * dout[j];
                L += s;
            }
        }
        for (int j = 0; j < 3; j++) { out6[j * n + i] = p[j]; out6[(3 + j) * n + i] = dout[j]; }
        if (opl) opl[i] = L;
        if (status) status[i] = st;
        if (hres) hres[i] = hr;
        if (nsteps) nsteps[i] = ns;
        if (trans) trans[i] = w;
    }
}

/* ------------------------------------------------------------------ */
/* camera, room and shading                                            */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea & Flood 2014): the n-th output of the generator
   seeded with `seed`, i.e. the mixing function applied to seed + n * gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void normalize3(double *a) {
    double l = norm3(a);
    for (int i = 0; i < 3; i++) a[i] /= l;
}

static void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

/* Pinhole camera: square-pixel image plane at unit distance, vertical full
   field of view fov_deg, row 0 at the top. With spp = m*m samples the pixel
   is split into m x m strata and each sample is jittered inside its stratum
   by two SplitMix64 outputs; spp = 1 takes the pixel centre. */
void orc_camera_ray(const orc_camera *cam, int32_t cam_index, int64_t id,
                    double o[3], double d[3]) {
    int64_t spp = cam->spp;
    int64_t pix = id / spp, smp = id % spp;
    int64_t row = pix / cam->w, col = pix % cam->w;
    double ox = 0.5, oy = 0.5;
    if (spp > 1) {
        int m = (int)llround(sqrt((double)spp));
        uint64_t key = ((uint64_t)cam_index << 40) ^ ((uint64_t)pix << 8) ^ (uint64_t)smp;
        double x1 = (double)(orc_splitmix64(cam->seed, 2 * key + 1) >> 11) * 0x1.0p-53;
        double x2 = (double)(orc_splitmix64(cam->seed, 2 * key + 2) >> 11) * 0x1.0p-53;
        ox = ((double)(smp % m) + x1) / m;
        oy = ((double)(smp / m) + x2) / m;
    }
    double F[3], R[3], U[3];
    for (int i = 0; i < 3; i++) F[i] = cam->look[i] - cam->eye[i];
    normalize3(F);
    cross3(F, cam->up, R);
    normalize3(R);
    cross3(R, F, U);
    double tn = tan(0.5 * cam->fov_deg * M_PI / 180.0);
    double u = ((col + ox) / cam->w * 2.0 - 1.0) * tn * ((double)cam->w / cam->h);
    double v = (1.0 - (row + oy) / cam->h * 2.0) * tn;
    for (int i = 0; i < 3; i++) {
        o[i] = cam->eye[i];
        d[i] = F[i] + u * R[i] + v * U[i];
    }
    normalize3(d);
}

/* Room box seen from inside: the face the ray leaves through and the tile
   parity floor(u/tile) + floor(v/tile) of the two in-face coordinates. */
int32_t orc_room_code(const orc_room *room, const double o[3], const double d[3],
                      double *s_hit) {
    double best = INFINITY;
    int face = -1;
    for (int ax = 0; ax < 3; ax++) {
        if (d[ax] == 0.0) continue;
        double plane = d[ax] > 0.0 ? room->hi[ax] : room->lo[ax];
        double s = (plane - o[ax]) / d[ax];
        if (s < best) { best = s; face = 2 * ax + (d[ax] > 0.0 ? 1 : 0); }
    }
    if (face < 0) { *s_hit = 0.0; return 12; }
    if (best < 0.0) best = 0.0;
    *s_hit = best;
    double p[3];
    for (int i = 0; i < 3; i++) p[i] = o[i] + best * d[i];
    int ax = face / 2;
    int u_ax = ax == 0 ? 1 : 0;
    int v_ax = ax == 2 ? 1 : 2;
    double fu = floor(p[u_ax] / room->tile), fv = floor(p[v_ax] / room->tile);
    int64_t par = ((int64_t)fu + (int64_t)fv) & 1;
    return face * 2 + (int32_t)par;
}

void orc_render_samples(const orc_cloak *c, const orc_opts *o, const orc_room *room,
                        const orc_camera *cam, int32_t cam_index, int32_t branch,
                        int64_t n, const int64_t *ids, uint8_t *code,
                        double *rec, int32_t *status, double *wimg) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double org[3], d[3], p[3], dout[3], L = 0.0, hr, w = 0.0;
        int64_t ns = 0;
        orc_camera_ray(cam, cam_index, ids[i], org, d);
        int st = trace_vacuum(c, branch, o, org, d, p, dout, &L, &hr, &ns, wimg ? &w : NULL, NULL, NULL);
        if (wimg) {
            /* share of the sample's unpolarized light that this branch carries
               to the room (Eq. (12)): a ray that stays in vacuum (a miss, or
               the metal end disk, which reflects every polarization) splits
               evenly over the two branch images; a ray through the crystal
               carries its trace weight; light reflected at the crystal's
               surface is not imaged */
            double wi = 0.0;
            if (st == ORC_MISSED) wi = 0.5;
            else if (st == ORC_EXITED) wi = w;
            else if (st == ORC_REFLECTED && c && sqrt(p[0] * p[0] + p[1] * p[1]) <= c->a) wi = 0.5;
            wimg[i] = wi;
        }
        int cd = 12;
        if (st == ORC_EXITED || st == ORC_MISSED || st == ORC_REFLECTED) {
            double s;
            cd = orc_room_code(room, p, dout, &s);
            L += s;
        }
        code[i] = (uint8_t)cd;
        if (status) status[i] = st;
        if (rec) {
            for (int j = 0; j < 3; j++) { rec[j * n + i] = p[j]; rec[(3 + j) * n + i] = dout[j]; }
            rec[6 * n + i] = L;
        }
    }
}

/* First-order reflections of arbitrary vacuum rays (in6 as orc_trace)
   through branch `branch`, unpolarized: w[j * n + i] the flux fraction of
   contribution j (0 the entry's reflected vacuum ray, 1 / 2 the ordinary /
   extraordinary wave reflected at the exit and followed to its own exit;
   0 if absent) and ray[(j * 6 + q) * n + i] its vacuum ray where it leaves
   the interface (point q < 3, unit direction q >= 3). */
void orc_trace_reflections(const orc_cloak *c, const orc_opts *o, int32_t branch, int64_t n, const double *in6,
                           double *w, double *ray) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double org[3], d[3], p[3], dout[3], L = 0.0, hr, wt = 0.0;
        int64_t ns = 0;
        orc_refl rf;
        memset(&rf, 0, sizeof(rf));
        for (int j = 0; j < 3; j++) { org[j] = in6[j * n + i]; d[j] = in6[(3 + j) * n + i]; }
        double dl = norm3(d);
        for (int j = 0; j < 3; j++) d[j] /= dl;
        trace_vacuum(c, branch, o, org, d, p, dout, &L, &hr, &ns, &wt, NULL, &rf);
        const double wj[3] = { rf.w_ext, rf.w_child[0], rf.w_child[1] };
        const double *pj[3] = { rf.p_ext, rf.p_child[0], rf.p_child[1] };
        const double *dj[3] = { rf.d_ext, rf.d_child[0], rf.d_child[1] };
        for (int j = 0; j < 3; j++) {
            w[j * n + i] = wj[j];
            for (int q = 0; q < 3; q++) {
                ray[(j * 6 + q) * n + i] = pj[j][q];
                ray[(j * 6 + 3 + q) * n + i] = dj[j][q];
            }
        }
    }
}

/* First-order reflections of camera samples through branch `branch`
   (R27). For each sample three contributions j: 0 the vacuum ray reflected
   at its first crystal interface, 1 and 2 the ordinary and extraordinary
   waves the branch's ray reflects into at its exit, each followed to its
   own exit. w[j * n + i] is the contribution's image weight and
   code[j * n + i] the room code it sees (12: no light, weight 0). goggle
   -1: the unpolarized image (the reflected fraction R of the entry split
   evenly over the two branches, R / 2 each; a child carries the trace
   weight of its path); 0, 1: that goggle's image (entry with the goggle's
   field, and half of it, as orc_render_goggle). */
void orc_render_reflections(const orc_cloak *c, const orc_opts *o, const orc_room *room, const orc_camera *cam,
                            int32_t cam_index, int32_t branch, int32_t goggle, int64_t n, const int64_t *ids,
                            double *w, uint8_t *code) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double org[3], d[3], p[3], dout[3], L = 0.0, hr, wt = 0.0, e[3];
        int64_t ns = 0;
        orc_refl rf;
        memset(&rf, 0, sizeof(rf));
        orc_camera_ray(cam, cam_index, ids[i], org, d);
        int ok = goggle < 0 || orc_goggle_axis(cam, d, goggle, e) == 0;
        if (ok) trace_vacuum(c, branch, o, org, d, p, dout, &L, &hr, &ns, &wt, goggle < 0 ? NULL : e, &rf);
        double half = goggle < 0 ? 1.0 : 0.5, s;
        double wj[3] = { ok ? 0.5 * half * rf.w_ext : 0.0, ok ? half * rf.w_child[0] : 0.0,
                         ok ? half * rf.w_child[1] : 0.0 };
        const double *pj[3] = { rf.p_ext, rf.p_child[0], rf.p_child[1] };
        const double *dj[3] = { rf.d_ext, rf.d_child[0], rf.d_child[1] };
        for (int j = 0; j < 3; j++) {
            int cd = 12;
            if (wj[j] > 0.0) cd = orc_room_code(room, pj[j], dj[j], &s);
            w[j * n + i] = cd < 12 ? wj[j] : 0.0;
            code[j * n + i] = (uint8_t)cd;
        }
    }
}

/* Polarizer goggles in front of the camera (Sect. 4, Figs. 1d,e and 2d,e).
   The in-plane goggle transmits the field along the camera's horizontal axis
   R = F x up / |F x up| (at elevation 0 the horizontal is the cross-section
   plane of the upright cylinder, the cloaking plane), the axial goggle the
   orthogonal one; for a ray of unit direction d the axes are the projection
   of R on the plane normal to d and d x that projection, an orthonormal pair
   transverse to d. */
int32_t orc_goggle_axis(const orc_camera *cam, const double d[3], int32_t goggle, double e[3]) {
    double F[3], R[3];
    for (int i = 0; i < 3; i++) F[i] = cam->look[i] - cam->eye[i];
    normalize3(F);
    cross3(F, cam->up, R);
    normalize3(R);
    double rd = dot3(R, d), a[3];
    for (int i = 0; i < 3; i++) a[i] = R[i] - rd * d[i];
    double l = norm3(a);
    if (!(l > 1e-12)) return 1;
    for (int i = 0; i < 3; i++) a[i] /= l;
    if (goggle == 0) {
        memcpy(e, a, sizeof(a));
    } else {
        cross3(d, a, e);
    }
    return 0;
}

/* Share of each sample's light that reaches the camera through goggle
   `goggle` (0 in-plane, 1 axial) by way of this branch. Unpolarized light
   from the room behind a polarizer keeps half its intensity: a ray that stays
   in vacuum (a miss, or the metal end disk, which reflects every
   polarization) gives each of the two branch images 1/4. For a ray through
   the crystal, reciprocity turns the polarizer into the polarization of the
   camera ray: the light of the room enters the crystal unpolarized at the
   far side and leaves towards the camera, and the flux it carries into the
   goggle's polarization equals 1/2 (the unpolarized room light's share of
   one polarization) times the transmission of the reversed path, which
   enters with the goggle's field: 1/2 x (entry transmission of the goggle's
   field into the branch) x (internal reflectances) x (exit transmission).
   The two goggles' weights add up to the unpolarized image weight. */
void orc_render_goggle(const orc_cloak *c, const orc_opts *o, const orc_camera *cam, int32_t cam_index,
                       int32_t branch, int32_t goggle, int64_t n, const int64_t *ids, double *wg) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double org[3], d[3], p[3], dout[3], L = 0.0, hr, w = 0.0, e[3];
        int64_t ns = 0;
        orc_camera_ray(cam, cam_index, ids[i], org, d);
        double wi = 0.0;
        if (orc_goggle_axis(cam, d, goggle, e) == 0) {
            int st = trace_vacuum(c, branch, o, org, d, p, dout, &L, &hr, &ns, &w, e, NULL);
            if (st == ORC_MISSED) wi = 0.25;
            else if (st == ORC_EXITED) wi = 0.5 * w;
            else if (st == ORC_REFLECTED && c && sqrt(p[0] * p[0] + p[1] * p[1]) <= c->a) wi = 0.25;
        }
        wg[i] = wi;
    }
}

/* ------------------------------------------------------------------ */
/* pieces exposed for the pin tests                                    */
/* ------------------------------------------------------------------ */
void orc_eps_cyl(const orc_cloak *c, double r, double out3[3]) {
    dual er, et, ez;
    eps_cyl(c, dk(r), &er, &et, &ez);
    out3[0] = er.v; out3[1] = et.v; out3[2] = ez.v;
}

void orc_metric(const orc_cloak *c, const double x[3], double M[9]) {
    dual xd[3] = { dk(x[0]), dk(x[1]), dk(x[2]) }, Md[3][3];
    metric_dual(c, xd, Md);
    for (int i = 0; i < 9; i++) M[i] = Md[i / 3][i % 3].v;
}

/* Eq. (7), left-hand form: M = |eps| eps^-1 / n_o^2. */
void orc_metric_det_form(const orc_cloak *c, const double x[3], double M[9]) {
    dual xd[3] = { dk(x[0]), dk(x[1]), dk(x[2]) }, ax[3][3], ev[3], eo, ee, w[3], T[3][3];
    principal(c, xd, ax, ev, &eo, &ee);
    dual det = dmul(dmul(ev[0], ev[1]), ev[2]);
    for (int p = 0; p < 3; p++) w[p] = ddiv(det, dmul(ev[p], eo));
    spectral(ax, w, T);
    for (int i = 0; i < 9; i++) M[i] = T[i / 3][i % 3].v;
}

void orc_rhs(const orc_cloak *c, int32_t branch, const double y[6], double dy[6]) {
    rhs_ctx ctx = { c, branch };
    rhs_fn(&ctx, y, dy);
}

void orc_rhs_eq8_isotropic(const orc_cloak *c, const double y[6], double dy[6]) {
    rhs_eq8_with(metric_iso_cb, NULL, c, y, dy);
}

/* harmonic oscillator x'' = -x in 3-D, integrated by the same steppers and
   controller (scheme 0 RK4 fixed h, 1 DP45 adaptive, 2 DP45 fixed h);
   returns the max-norm error against the exact solution at T */
static void osc_rhs(const void *ctx, const double *y, double *dy) {
    (void)ctx;
    for (int i = 0; i < 3; i++) { dy[i] = y[3 + i]; dy[3 + i] = -y[i]; }
}

double orc_test_oscillator(int32_t scheme, double h, double rtol, double T,
                           double y_out[6], int64_t *nsteps) {
    double y[6] = { 1.0, 0.0, 0.5, 0.0, 1.0, -0.25 }, yn[6], k1[6], k7[6];
    double t = 0.0;
    int after_reject = 0;
    int64_t ns = 0;
    osc_rhs(NULL, y, k1);
    while (t < T) {
        double hh = fmin(h, T - t);
        ns++;
        if (scheme == ORC_RK4) {
            rk4_step(osc_rhs, NULL, y, hh, yn);
            t += hh;
            memcpy(y, yn, sizeof(yn));
            continue;
        }
        if (scheme == 2) { /* DP45 fifth-order solution at fixed h */
            (void)dp45_step(osc_rhs, NULL, y, k1, hh, 1.0, 1.0, yn, k7);
            t += hh;
            memcpy(y, yn, sizeof(yn));
            memcpy(k1, k7, sizeof(k7));
            continue;
        }
        double err = dp45_step(osc_rhs, NULL, y, k1, hh, rtol, rtol, yn, k7);
        if (!(err <= 1.0)) {
            h = hh * dp45_factor(err, 0);
            after_reject = 1;
            continue;
        }
        double hnext = hh * dp45_factor(err, after_reject);
        after_reject = 0;
        t += hh;
        memcpy(y, yn, sizeof(yn));
        memcpy(k1, k7, sizeof(k7));
        h = hnext;
    }
    /* x(t) = x0 cos t + v0 sin t with x0 = (1, 0, 1/2), v0 = (0, 1, -1/4) */
    double ex[6] = { cos(T), sin(T), 0.5 * cos(T) - 0.25 * sin(T),
                     -sin(T), cos(T), -0.5 * sin(T) - 0.25 * cos(T) };
    double e = 0.0;
    for (int i = 0; i < 6; i++) e = fmax(e, fabs(y[i] - ex[i]));
    if (y_out) memcpy(y_out, y, sizeof(y));
    if (nsteps) *nsteps = ns;
    return e;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
