// device.h -- device-side math of the cloak tracer for gfx950.
//
// Halimeh & Wegener, "Photorealistic ray tracing of free-space invisibility
// cloaks made of uniaxial dielectrics":
//   material      Eq. (14) radial / Eq. (15) azimuthal cloak, optic axis r or
//                 theta, mu = 1 (Sect. 2)
//   metric        Eq. (7): in the cylindrical frame M = diag(m_r, m_theta, m_z)
//                 with eps_e across the optic axis and eps_o along it (the
//                 extraordinary ray), or n_o^2 I (the ordinary ray, for which
//                 Eq. (2) is Eq. (8) with M = n_o^2 I)
//   ray equation  Eq. (8) (Eq. (2) as its isotropic case), evaluated as the
//                 Euler-Lagrange equations of L = v^T M v / 2 in cylindrical
//                 coordinates, which is the same vector field with no 3x3
//                 tensor algebra
//   refraction    Sect. 3: tangential k continuous (Eq. (11)); the normal
//                 component solves k^T M^-1 k = 1, the dispersion relation
//                 behind Eq. (9); ray velocity v = M^-1 k (Eq. (6))
//   stepping      classical RK4 (Sect. 4) and Dormand-Prince 5(4)
// Units: c0 = omega = 1, so the ODE time is the optical path length.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

// ---------------------------------------------------------------------------
// parameters passed by value to every kernel
// ---------------------------------------------------------------------------
struct CloakP {
  double a, b, z0, z1;  // radii and axial extent
  double kappa;         // (b / (b - a))^2
  double a2, b2;        // a^2, b^2
  double inv_a, inv_b;  // 1/a, 1/b
  int axis, mirror;     // 0 radial / 1 azimuthal; inner metal cylinder
};

struct OptsP {
  double h0, rtol, atol, hmax, r_out;
  long long max_steps;
  int scheme, precision, max_bounces, pad;
};

// branch kind = axis * 2 + pol
enum { K_RO = 0, K_RE = 1, K_AO = 2, K_AE = 3 };

// boundary ids
enum { B_SIDE = 0, B_INNER = 1, B_TOP = 2, B_BOTTOM = 3 };

// ---------------------------------------------------------------------------
// fast FP64 reciprocal and reciprocal square root: hardware estimate refined
// by two Newton steps (quadratic convergence to full double precision)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// ---------------------------------------------------------------------------
// metric diag(m_r, m_theta, m_z) at radius r for a branch kind
// ---------------------------------------------------------------------------
__device__ __forceinline__ void metric_diag(int kind, double kappa, double a, double w,
                                            double& mr, double& mt, double& mz) {
  double q = fma(-a, w, 1.0);  // (r - a) / r with w = 1/r
  double ks = kappa * q * q;
  switch (kind) {
    case K_RO: mr = kappa; mt = kappa; mz = kappa; break;
    case K_RE: mr = kappa; mt = ks; mz = ks; break;
    case K_AO: mr = ks; mt = ks; mz = ks; break;
    default:   mr = kappa; mt = ks; mz = kappa; break;
  }
}

// one Newton step on the hardware estimate: relative error ~4e-15 (rsq) and
// ~2e-15 (rcp) on gfx950, used inside the derivative evaluation
__device__ __forceinline__ double rcp64_1(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsq64_1(double x) {
  double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// ---------------------------------------------------------------------------
// acceleration dv/dt of Eq. (8)/(2) at (p, v), FP64.
// With w = 1/r, q = (r-a)/r, s = q^2, s' = ds/dr = 2 a q w^2, g = s'/s:
//   a_r     = [-m_r' v_r^2 + m_t' v_t^2 + m_z' v_z^2 - 2 (m_r - m_t) v_t^2 / r] / (2 m_r)
//   a_theta = -(m_t'/m_t) v_r v_t,   a_z = -(m_z'/m_z) v_r v_z
// which for the three non-trivial branches is
//   radial-e    (k, k s, k s): a_r = s'/2 (v_t^2 + v_z^2) - (1 - s) v_t^2 / r,
//                              a_t = -g v_r v_t, a_z = -g v_r v_z
//   azimuthal-e (k, k s, k):   a_r = s'/2 v_t^2 - (1 - s) v_t^2 / r,
//                              a_t = -g v_r v_t, a_z = 0
//   azimuthal-o  k s I:        a_r = g/2 (v_t^2 + v_z^2 - v_r^2),
//                              a_t = -g v_r v_t, a_z = -g v_r v_z
// (radial-o: k I, zero). s'/2 = a q w^2 needs no division; g = 2 a w^2 / q.
// Since 1 - q = a w, (1 - s) / r = a w^2 (1 + q), and the radial terms reduce
// to a_r = a w^2 (q v_z^2 - v_t^2) (radial-e) and a_r = -a w^2 v_t^2
// (azimuthal-e).
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void accel64(double a, double px, double py, double vx, double vy,
                                        double vz, double& ax, double& ay, double& az) {
  if constexpr (KIND == K_RO) {
    ax = 0.0; ay = 0.0; az = 0.0;
    return;
  } else {
    double r2 = fma(px, px, py * py);
    double w = rsq64_1(r2);
    double w2 = w * w;
    double q = fma(-a, w, 1.0);
    double P = fma(px, vx, py * vy);   // r v_r
    double Q = fma(px, vy, -py * vx);  // r v_t
    double vt = Q * w;
    double vt2 = vt * vt;
    double gvr = (2.0 * a) * w2 * rcp64_1(q) * (P * w);  // g v_r
    double ar, at;
    if constexpr (KIND == K_RE) {
      ar = a * w2 * fma(q * vz, vz, -vt2);
      at = -gvr * vt;
      az = -gvr * vz;
    } else if constexpr (KIND == K_AE) {
      ar = -a * w2 * vt2;
      at = -gvr * vt;
      az = 0.0;
    } else {
      // g/2 (v_t^2 + v_z^2 - v_r^2) with g v_r known: g = gvr / v_r is not
      // safe at v_r = 0, so form g directly
      double g = (2.0 * a) * w2 * rcp64_1(q);
      double vr = P * w;
      ar = 0.5 * g * fma(vz, vz, fma(-vr, vr, vt2));
      at = -g * vr * vt;
      az = -g * vr * vz;
      (void)gvr;
    }
    ar *= w;
    at *= w;
    ax = fma(ar, px, -at * py);
    ay = fma(ar, py, at * px);
  }
}

// the acceleration of branch KIND (FP64)
template <int KIND>
__device__ __forceinline__ void accel(double a, double px, double py, double vx, double vy, double vz,
                                      double& ax, double& ay, double& az) {
  accel64<KIND>(a, px, py, vx, vy, vz, ax, ay, az);
}

// ---------------------------------------------------------------------------
// Dormand & Prince (1980) RK5(4)7M tableau and the products used below.
// For y = (x, v) with dx/dt = v the stage inputs only need the stage
// accelerations A_l:
//   V_s = v + h sum_l a_sl A_l
//   X_s = x + h (c_s v + h sum_l (a a)_sl A_l),   (a a)_sl = sum_j a_sj a_jl
// The seventh stage input is the fifth-order solution (first same as last);
// the embedded error is h^2 sum_l (e a)_l A_l for x (the weights e = b - b*
// sum to zero) and h sum_j e_j A_j for v.
// ---------------------------------------------------------------------------
struct DP {
  static constexpr double A[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {1.0 / 5, 0, 0, 0, 0, 0, 0},
      {3.0 / 40, 9.0 / 40, 0, 0, 0, 0, 0},
      {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0, 0},
      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0, 0},
      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0, 0},
      {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0}};
  static constexpr double E[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920,
                                  -17253.0 / 339200, 22.0 / 525, -1.0 / 40};
};

constexpr double dp_c(int s) {
  double c = 0;
  for (int j = 0; j < 7; ++j) c += DP::A[s][j];
  return c;
}
constexpr double dp_aa(int s, int l) {
  double t = 0;
  for (int j = 0; j < 7; ++j) t += DP::A[s][j] * DP::A[j][l];
  return t;
}
constexpr double dp_ea(int l) {
  double t = 0;
  for (int j = 0; j < 7; ++j) t += DP::E[j] * DP::A[j][l];
  return t;
}

// One DP45 attempt. Inputs: state (x, v), A[0] = acceleration at the state.
// Outputs: fifth-order state (xn, vn), A[6] = acceleration there, and the sum
// of squared scaled errors (accept when <= 6, i.e. RMS <= 1).
template <int KIND>
__device__ __forceinline__ double dp45_attempt(double a, const double x[3],
                                               const double v[3], double A[7][3], double h,
                                               double rtol, double atol, double xn[3],
                                               double vn[3]) {
#pragma unroll
  for (int s = 1; s < 7; ++s) {
    double X[3], V[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double ax = 0.0, av = 0.0;
#pragma unroll
      for (int l = 0; l < s; ++l) {
        if (dp_aa(s, l) != 0.0) ax = fma(dp_aa(s, l), A[l][i], ax);
        if (DP::A[s][l] != 0.0) av = fma(DP::A[s][l], A[l][i], av);
      }
      V[i] = fma(h, av, v[i]);
      X[i] = fma(h, fma(h, ax, dp_c(s) * v[i]), x[i]);
    }
    accel<KIND>(a, X[0], X[1], V[0], V[1], V[2], A[s][0], A[s][1], A[s][2]);
    if (s == 6) {
#pragma unroll
      for (int i = 0; i < 3; ++i) { xn[i] = X[i]; vn[i] = V[i]; }
    }
  }
  double e6[6], s6[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double ex = 0.0, ev = 0.0;
#pragma unroll
    for (int l = 0; l < 7; ++l) {
      if (dp_ea(l) != 0.0) ex = fma(dp_ea(l), A[l][i], ex);
      if (DP::E[l] != 0.0) ev = fma(DP::E[l], A[l][i], ev);
    }
    e6[2 * i] = ex * (h * h);
    e6[2 * i + 1] = ev * h;
    s6[2 * i] = fma(rtol, fmax(fabs(x[i]), fabs(xn[i])), atol);
    s6[2 * i + 1] = fma(rtol, fmax(fabs(v[i]), fabs(vn[i])), atol);
  }
  double sum = 0.0;
  if (atol >= 1e-40) {
    // every scale is at least atol >= 1e-40, so the product of the six stays
    // above 1e-240 (and overflows only for states beyond 1e50), and
    // 1/s_k = (prod_{j != k} s_j) / prod_j s_j takes one reciprocal instead
    // of six
    double pre[6], suf[6];
    pre[0] = 1.0;
    suf[5] = 1.0;
#pragma unroll
    for (int k = 1; k < 6; ++k) pre[k] = pre[k - 1] * s6[k - 1];
#pragma unroll
    for (int k = 4; k >= 0; --k) suf[k] = suf[k + 1] * s6[k + 1];
    const double r = rcp64(pre[5] * s6[5]);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double q = e6[k] * (pre[k] * suf[k]) * r;
      sum = fma(q, q, sum);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double q = e6[k] * rcp64(s6[k]);
      sum = fma(q, q, sum);
    }
  }
  return sum;
}

// step-size factor from the summed squared error: 0.9 * RMS^(-1/5) clipped
// to [0.2, 5]; evaluated in FP32 (a controller heuristic, not part of the
// solution's accuracy)
__device__ __forceinline__ double dp45_factor(double sum, bool after_reject) {
  float fac;
  if (sum == 0.0) fac = 5.0f;
  else if (!(sum == sum)) fac = 0.2f;
  else {
    float rms2 = (float)(sum * (1.0 / 6.0));
    fac = 0.9f * exp2f(-0.1f * log2f(rms2));
    fac = fminf(5.0f, fmaxf(0.2f, fac));
  }
  if (after_reject && fac > 1.0f) fac = 1.0f;
  return (double)fac;
}

// classical RK4 step for y = (x, v); A1 = acceleration at the state
template <int KIND>
__device__ __forceinline__ void rk4_step(double a, const double x[3],
                                         const double v[3], const double A1[3], double h,
                                         double xn[3], double vn[3]) {
  double hh = 0.5 * h;
  double V2[3], V3[3], V4[3], A2[3], A3[3], A4[3], X[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(hh, v[i], x[i]); V2[i] = fma(hh, A1[i], v[i]); }
  accel<KIND>(a, X[0], X[1], V2[0], V2[1], V2[2], A2[0], A2[1], A2[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(hh, V2[i], x[i]); V3[i] = fma(hh, A2[i], v[i]); }
  accel<KIND>(a, X[0], X[1], V3[0], V3[1], V3[2], A3[0], A3[1], A3[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(h, V3[i], x[i]); V4[i] = fma(h, A3[i], v[i]); }
  accel<KIND>(a, X[0], X[1], V4[0], V4[1], V4[2], A4[0], A4[1], A4[2]);
  double h6 = h * (1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    xn[i] = fma(h6, v[i] + 2.0 * (V2[i] + V3[i]) + V4[i], x[i]);
    vn[i] = fma(h6, A1[i] + 2.0 * (A2[i] + A3[i]) + A4[i], v[i]);
  }
}

// ---------------------------------------------------------------------------
// Hamiltonian form of the ray equations (the alternative of Sect. 4):
// H(x, k) = k^T A k - f with A = diag(A_r, A_t, A_z) in (r_hat, theta_hat,
// z_hat); A = eps, f = eps_o eps_e = kappa^2 s for the extraordinary branches,
// A = I, f = eps_o for the ordinary ones. H = f (k^T M^-1 k - 1), so A = f M^-1:
//   radial-e    A = kappa (s, 1, 1),    f = kappa^2 s
//   azimuthal-e A = kappa (s, 1, s),    f = kappa^2 s
//   azimuthal-o A = I,                  f = kappa s
//   radial-o    A = I,                  f = kappa
// dx/dtau = 2 A k; with k_r = k . r_hat, k_t = k . theta_hat,
//   dk/dtau = -r_hat [A_t' |k_xy|^2 + (A_r' - A_t') k_r^2 + A_z' k_z^2 - f']
//             - 2 (A_r - A_t) k_r k_t theta_hat / r,
// and the optical path advances as dt/dtau = 2 f (v = M^-1 k = A k / f).
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void ham_rhs(double a, double kappa, const double x[3], const double k[3],
                                        double dx[3], double dk[3], double& dt) {
  if constexpr (KIND == K_RO) {
#pragma unroll
    for (int i = 0; i < 3; ++i) { dx[i] = 2.0 * k[i]; dk[i] = 0.0; }
    dt = 2.0 * kappa;
  } else {
    const double r2 = fma(x[0], x[0], x[1] * x[1]);
    const double w = rsq64_1(r2);
    const double q = fma(-a, w, 1.0);
    const double s = q * q;
    const double sp = 2.0 * a * q * w * w;  // ds/dr
    if constexpr (KIND == K_AO) {
#pragma unroll
      for (int i = 0; i < 3; ++i) dx[i] = 2.0 * k[i];
      const double g = kappa * sp * w;  // f' along r_hat, r_hat = w x
      dk[0] = g * x[0];
      dk[1] = g * x[1];
      dk[2] = 0.0;
      dt = 2.0 * kappa * s;
    } else {
      const double kr = fma(x[0], k[0], x[1] * k[1]) * w;
      const double kt = fma(x[0], k[1], -x[1] * k[0]) * w;
      // dx/dtau = 2 kappa (s k_r r_hat + k_t theta_hat, (1 or s) k_z)
      const double ur = 2.0 * kappa * s * kr * w, ut = 2.0 * kappa * kt * w;
      dx[0] = fma(ur, x[0], -ut * x[1]);
      dx[1] = fma(ur, x[1], ut * x[0]);
      double P;  // radial component of dk/dtau
      if constexpr (KIND == K_RE) {
        dx[2] = 2.0 * kappa * k[2];
        P = -kappa * sp * fma(kr, kr, -kappa);
      } else {
        dx[2] = 2.0 * kappa * s * k[2];
        P = -kappa * sp * (fma(kr, kr, k[2] * k[2]) - kappa);
      }
      const double Qt = 2.0 * kappa * (1.0 - s) * kr * kt * w;  // theta component
      dk[0] = fma(P * w, x[0], -Qt * w * x[1]);
      dk[1] = fma(P * w, x[1], Qt * w * x[0]);
      dk[2] = 0.0;
      dt = 2.0 * kappa * kappa * s;
    }
  }
}

// The canonically normalized Hamiltonian H' = H / f = k^T M^-1 k - 1 with
// M^-1 = A / f = diag(a_r, a_t, a_z) in (r_hat, theta_hat, z_hat):
// dx/dtau = 2 (a_r k_r r_hat + a_t k_t theta_hat + a_z k_z z_hat),
// dk/dtau = -(a_r' k_r^2 + a_t' k_t^2 + a_z' k_z^2) r_hat
//           - 2 (a_r - a_t) k_r k_t / r theta_hat,
// dt/dtau = 2. Per branch (s = (1 - a/r)^2, f = kappa^2 s or eps_o):
// radial-o a = 1/kappa; azimuthal-o a = 1/(kappa s); radial-e (a_r, a_t,
// a_z) = (1/kappa, 1/(kappa s), 1/(kappa s)); azimuthal-e (1/kappa,
// 1/(kappa s), 1/kappa). The derivative of 1/(kappa s) is -s'/(kappa s^2).
template <int KIND>
__device__ __forceinline__ void ham_rhs_canon(double a, double kappa, const double x[3], const double k[3],
                                              double dx[3], double dk[3], double& dt) {
  dt = 2.0;
  const double ik = 1.0 / kappa;
  if constexpr (KIND == K_RO) {
#pragma unroll
    for (int i = 0; i < 3; ++i) { dx[i] = 2.0 * ik * k[i]; dk[i] = 0.0; }
  } else {
    const double r2 = fma(x[0], x[0], x[1] * x[1]);
    const double w = rsq64_1(r2);
    const double q = fma(-a, w, 1.0);
    const double s = q * q;
    const double sp = 2.0 * a * q * w * w;  // ds/dr
    const double is = rcp64(s);
    const double g = ik * is;              // 1 / (kappa s)
    const double gp = -g * sp * is;        // its r-derivative
    const double kr = fma(x[0], k[0], x[1] * k[1]) * w;
    const double kt = fma(x[0], k[1], -x[1] * k[0]) * w;
    double ar, at, az, arp, atp, azp;
    if constexpr (KIND == K_AO) {
      ar = at = az = g; arp = atp = azp = gp;
    } else if constexpr (KIND == K_RE) {
      ar = ik; at = az = g; arp = 0.0; atp = azp = gp;
    } else {  // K_AE
      ar = az = ik; at = g; arp = azp = 0.0; atp = gp;
    }
    const double ur = 2.0 * ar * kr * w, ut = 2.0 * at * kt * w;
    dx[0] = fma(ur, x[0], -ut * x[1]);
    dx[1] = fma(ur, x[1], ut * x[0]);
    dx[2] = 2.0 * az * k[2];
    const double P = -(arp * kr * kr + atp * kt * kt + azp * k[2] * k[2]);
    const double Qt = -2.0 * (ar - at) * kr * kt * w;
    dk[0] = fma(P * w, x[0], -Qt * w * x[1]);
    dk[1] = fma(P * w, x[1], Qt * w * x[0]);
    dk[2] = 0.0;
  }
}

template <int KIND, bool CANON>
__device__ __forceinline__ void ham_rhs_any(double a, double kappa, const double x[3], const double k[3],
                                            double dx[3], double dk[3], double& dt) {
  if constexpr (CANON) ham_rhs_canon<KIND>(a, kappa, x, k, dx, dk, dt);
  else ham_rhs<KIND>(a, kappa, x, k, dx, dk, dt);
}

// classical RK4 with step h in tau on (x, k); dt = optical path of the step
// (CANON: the canonically normalized Hamiltonian)
template <int KIND, bool CANON = false>
__device__ __forceinline__ void rk4_ham_step(double a, double kappa, const double x[3], const double k[3],
                                             double h, double xn[3], double kn[3], double& dt) {
  double d1x[3], d1k[3], d2x[3], d2k[3], d3x[3], d3k[3], d4x[3], d4k[3], X[3], K[3];
  double t1, t2, t3, t4;
  const double hh = 0.5 * h;
  ham_rhs_any<KIND, CANON>(a, kappa, x, k, d1x, d1k, t1);
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(hh, d1x[i], x[i]); K[i] = fma(hh, d1k[i], k[i]); }
  ham_rhs_any<KIND, CANON>(a, kappa, X, K, d2x, d2k, t2);
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(hh, d2x[i], x[i]); K[i] = fma(hh, d2k[i], k[i]); }
  ham_rhs_any<KIND, CANON>(a, kappa, X, K, d3x, d3k, t3);
#pragma unroll
  for (int i = 0; i < 3; ++i) { X[i] = fma(h, d3x[i], x[i]); K[i] = fma(h, d3k[i], k[i]); }
  ham_rhs_any<KIND, CANON>(a, kappa, X, K, d4x, d4k, t4);
  const double h6 = h * (1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    xn[i] = fma(h6, d1x[i] + 2.0 * (d2x[i] + d3x[i]) + d4x[i], x[i]);
    kn[i] = fma(h6, d1k[i] + 2.0 * (d2k[i] + d3k[i]) + d4k[i], k[i]);
  }
  dt = h6 * (t1 + 2.0 * (t2 + t3) + t4);
}

// k = M v (to_k) or v = M^-1 k at x, M diagonal in (r_hat, theta_hat, z_hat)
template <int KIND>
__device__ __forceinline__ void ham_convert(double a, double kappa, const double x[3], double u[3],
                                            bool to_k) {
  const double w = rsq64(fma(x[0], x[0], x[1] * x[1]));
  double mr, mt, mz;
  metric_diag(KIND, kappa, a, w, mr, mt, mz);
  const double fr = to_k ? mr : 1.0 / mr, ft = to_k ? mt : 1.0 / mt, fz = to_k ? mz : 1.0 / mz;
  const double ur = fma(x[0], u[0], x[1] * u[1]) * w * fr;
  const double ut = fma(x[0], u[1], -x[1] * u[0]) * w * ft;
  u[0] = fma(ur, x[0], -ut * x[1]) * w;
  u[1] = fma(ur, x[1], ut * x[0]) * w;
  u[2] *= fz;
}

// ---------------------------------------------------------------------------
// Eq. (12): intensity transmission at a plane interface (Sect. 3), from the
// tangential fields alone. Local basis (t1, t2, n), n pointing out of the
// crystal, t1 along the tangential wave vector, so every wave vector is
// (k1, 0, q) with complex q for evanescent waves. Fields: H = k x E; the
// normal power flux is Re(E1 H2* - E2 H1*) / 2. In vacuum k.E = 0 gives the
// tangential H from the tangential E (admittance, with k2 = 0):
//   H1 = -q E2,  H2 = (k1^2 + q^2) E1 / q.
// Continuity of tangential E and H, with the vacuum wave eliminated through
// its admittance, leaves a 2 x 2 complex system for the two crystal waves.
// Crystal waves: ordinary E = k x c; extraordinary D = (k.k) c - (c.k) k,
// E = eps^-1 D, eps^-1 = I / eo + (1 / ee - 1 / eo) c c^T; where k is along
// c both coincide and E = (0, 1, 0), k x (0, 1, 0) are taken.
// ---------------------------------------------------------------------------
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cx(double r, double i = 0.0) { return cplx{r, i}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cplx{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double d = 1.0 / fma(b.re, b.re, b.im * b.im);
  return cplx{fma(a.re, b.re, a.im * b.im) * d, fma(a.im, b.re, -a.re * b.im) * d};
}
__device__ __forceinline__ double cabs2(cplx a) { return fma(a.re, a.re, a.im * a.im); }
// Re(a b*)
__device__ __forceinline__ double cre_conj(cplx a, cplx b) { return fma(a.re, b.re, a.im * b.im); }

// normal component of a wave: dir = +1 carries power (or decays) towards
// +n, -1 towards -n; ordinary / vacuum: q^2 = eps - k1^2
__device__ __forceinline__ cplx q_iso_dev(double eps, double k1, int dir) {
  const double d = eps - k1 * k1;
  return d >= 0.0 ? cx(dir * sqrt(d)) : cx(0.0, dir * sqrt(-d));
}

// extraordinary: k^T eps k = eo ee with k = (k1, 0, q)
__device__ __forceinline__ cplx q_extra_dev(double eo, double ee, const double c[3], double k1, int dir) {
  const double de = ee - eo;
  const double a = eo + de * c[2] * c[2];
  const double b = de * c[2] * c[0] * k1;
  const double c0 = fma(eo + de * c[0] * c[0], k1 * k1, -eo * ee);
  const double disc = fma(b, b, -a * c0);
  const double ia = 1.0 / a;
  return disc >= 0.0 ? cx((-b + dir * sqrt(disc)) * ia) : cx(-b * ia, dir * sqrt(-disc) * ia);
}

// tangential (E1, E2, H1, H2) of a crystal wave k = (k1, 0, q)
__device__ __forceinline__ void crystal_tangential(double eo, double ee, const double c[3], bool ordinary,
                                                   double k1, cplx q, cplx f[4]) {
  // k x c
  const cplx kc0 = cx(0.0) - q * cx(c[1]);
  const cplx kc1 = q * cx(c[0]) - cx(k1 * c[2]);
  const cplx kc2 = cx(k1 * c[1]);
  const double deg = cabs2(kc0) + cabs2(kc1) + cabs2(kc2);
  const double kk = k1 * k1 + cabs2(q);
  cplx E0, E1, E2;
  if (deg <= 1e-24 * kk) {
    if (ordinary) {
      E0 = cx(0.0); E1 = cx(1.0); E2 = cx(0.0);
    } else {  // k x (0, 1, 0)
      E0 = cx(0.0) - q; E1 = cx(0.0); E2 = cx(k1);
    }
  } else if (ordinary) {
    E0 = kc0; E1 = kc1; E2 = kc2;
  } else {
    const cplx kdk = cx(k1 * k1) + q * q;
    const cplx cdk = cx(c[0] * k1) + cx(c[2]) * q;
    const cplx D0 = kdk * cx(c[0]) - cdk * cx(k1);
    const cplx D1 = kdk * cx(c[1]);
    const cplx D2 = kdk * cx(c[2]) - cdk * q;
    const cplx cD = cx(c[0]) * D0 + cx(c[1]) * D1 + cx(c[2]) * D2;
    const double io = 1.0 / eo, g = 1.0 / ee - io;
    E0 = io * D0 + (g * c[0]) * cD;
    E1 = io * D1 + (g * c[1]) * cD;
    E2 = io * D2 + (g * c[2]) * cD;
  }
  // H = k x E with k = (k1, 0, q)
  f[0] = E0;
  f[1] = E1;
  f[2] = cx(0.0) - q * E1;       // H1 = k2 E2 - q E1 with k2 = 0... = -q E1
  f[3] = q * E0 - cx(k1) * E2;   // H2 = q E0 - k1 E2
}

__device__ __forceinline__ double flux_t(const cplx f[4]) {
  return 0.5 * (cre_conj(f[0], f[3]) - cre_conj(f[1], f[2]));
}

// local basis at an interface: n outward, t1 along the tangential part of k
__device__ __forceinline__ void interface_basis(const double n[3], const double k[3], double t1[3], double t2[3],
                                                double &k1) {
  const double kn = k[0] * n[0] + k[1] * n[1] + k[2] * n[2];
  double kt[3] = {k[0] - kn * n[0], k[1] - kn * n[1], k[2] - kn * n[2]};
  k1 = sqrt(kt[0] * kt[0] + kt[1] * kt[1] + kt[2] * kt[2]);
  if (k1 > 1e-12) {
    const double ik = 1.0 / k1;
    t1[0] = kt[0] * ik; t1[1] = kt[1] * ik; t1[2] = kt[2] * ik;
  } else {
    // any tangent: n x (the axis least aligned with n)
    const double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
    const double e[3] = {ax <= ay && ax <= az ? 1.0 : 0.0, (ay < ax && ay <= az) ? 1.0 : 0.0,
                         (az < ax && az < ay) ? 1.0 : 0.0};
    double u[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2], n[0] * e[1] - n[1] * e[0]};
    const double iu = 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    t1[0] = u[0] * iu; t1[1] = u[1] * iu; t1[2] = u[2] * iu;
    k1 = 0.0;
  }
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

// Solve a x + b y = r (two complex 2-vectors per column) by Cramer's rule.
__device__ __forceinline__ void solve2(const cplx a[2], const cplx b[2], const cplx r[2], cplx &x, cplx &y) {
  const cplx det = a[0] * b[1] - a[1] * b[0];
  x = cdiv(r[0] * b[1] - r[1] * b[0], det);
  y = cdiv(a[0] * r[1] - a[1] * r[0], det);
}

// Unpolarized transmission from vacuum (unit direction d, n outward) into
// the ordinary (To) and the extraordinary (Te) crystal wave.
__device__ __forceinline__ void fresnel_in2_dev(double eo, double ee, const double cax[3], const double n[3],
                                                const double d[3], double &To, double &Te) {
  double t1[3], t2[3], k1;
  interface_basis(n, d, t1, t2, k1);
  const double c[3] = {cax[0] * t1[0] + cax[1] * t1[1] + cax[2] * t1[2],
                       cax[0] * t2[0] + cax[1] * t2[1] + cax[2] * t2[2],
                       cax[0] * n[0] + cax[1] * n[1] + cax[2] * n[2]};
  const double qi = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];  // < 0
  const cplx qr = q_iso_dev(1.0, k1, +1);
  const cplx qo = q_iso_dev(eo, k1, -1), qe = q_extra_dev(eo, ee, c, k1, -1);
  cplx fo[4], fe[4];
  crystal_tangential(eo, ee, c, true, k1, qo, fo);
  crystal_tangential(eo, ee, c, false, k1, qe, fe);
  // reflected admittance Y (k2 = 0): H1 = -q E2, H2 = (k1^2 + q^2) / q E1
  const cplx y22 = cdiv(cx(k1 * k1) + qr * qr, qr);
  // columns h - Y e of the two crystal waves
  const cplx A[2] = {fo[2] - (cx(0.0) - qr * fo[1]), fo[3] - y22 * fo[0]};
  const cplx B[2] = {fe[2] - (cx(0.0) - qr * fe[1]), fe[3] - y22 * fe[0]};
  To = 0.0;
  Te = 0.0;
  for (int pol = 0; pol < 2; ++pol) {
    // s: E = (0, 1, 0); p: E = k x (0, 1, 0) = (-qi, 0, k1)
    cplx fi[4];
    if (pol == 0) {
      fi[0] = cx(0.0); fi[1] = cx(1.0);
      fi[2] = cx(-qi); fi[3] = cx(0.0);  // H = k x E: H1 = -qi E1, H2 = qi E0 - k1 E2
    } else {
      fi[0] = cx(-qi); fi[1] = cx(0.0);
      fi[2] = cx(0.0); fi[3] = cx(-qi * qi - k1 * k1);
    }
    // H_i - Y E_i
    const cplx r[2] = {fi[2] - (cx(0.0) - qr * fi[1]), fi[3] - y22 * fi[0]};
    cplx ao, ae;
    solve2(A, B, r, ao, ae);
    const double si = fabs(flux_t(fi));
    To += cabs2(ao) * fabs(flux_t(fo)) / si;
    Te += cabs2(ae) * fabs(flux_t(fe)) / si;
  }
  To *= 0.5;
  Te *= 0.5;
}

// Unpolarized transmission from vacuum into the crystal wave of `extra`
// (0 ordinary, 1 extraordinary): fresnel_in2_dev for one wave (the same
// arithmetic), so that callers that need one carry one.
__device__ __forceinline__ double fresnel_in_dev(double eo, double ee, const double cax[3], const double n[3],
                                                 const double d[3], int extra) {
  double t1[3], t2[3], k1;
  interface_basis(n, d, t1, t2, k1);
  const double c[3] = {cax[0] * t1[0] + cax[1] * t1[1] + cax[2] * t1[2],
                       cax[0] * t2[0] + cax[1] * t2[1] + cax[2] * t2[2],
                       cax[0] * n[0] + cax[1] * n[1] + cax[2] * n[2]};
  const double qi = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
  const cplx qr = q_iso_dev(1.0, k1, +1);
  const cplx qo = q_iso_dev(eo, k1, -1), qe = q_extra_dev(eo, ee, c, k1, -1);
  cplx fo[4], fe[4];
  crystal_tangential(eo, ee, c, true, k1, qo, fo);
  crystal_tangential(eo, ee, c, false, k1, qe, fe);
  const cplx y22 = cdiv(cx(k1 * k1) + qr * qr, qr);
  const cplx A[2] = {fo[2] - (cx(0.0) - qr * fo[1]), fo[3] - y22 * fo[0]};
  const cplx B[2] = {fe[2] - (cx(0.0) - qr * fe[1]), fe[3] - y22 * fe[0]};
  double T = 0.0;
  for (int pol = 0; pol < 2; ++pol) {
    cplx fi[4];
    if (pol == 0) {
      fi[0] = cx(0.0); fi[1] = cx(1.0);
      fi[2] = cx(-qi); fi[3] = cx(0.0);
    } else {
      fi[0] = cx(-qi); fi[1] = cx(0.0);
      fi[2] = cx(0.0); fi[3] = cx(-qi * qi - k1 * k1);
    }
    const cplx r[2] = {fi[2] - (cx(0.0) - qr * fi[1]), fi[3] - y22 * fi[0]};
    cplx ao, ae;
    solve2(A, B, r, ao, ae);
    const double si = fabs(flux_t(fi));
    T += (extra ? cabs2(ae) * fabs(flux_t(fe)) : cabs2(ao) * fabs(flux_t(fo))) / si;
  }
  return 0.5 * T;
}

// Transmission from vacuum into the ordinary (Go) and extraordinary (Ge)
// crystal wave for the incident field along the unit vector e (transverse
// to d), and the unpolarized ones (Uo, Ue, as fresnel_in2_dev). With s
// along t2 (normal to the plane of incidence) and p = d x s, e = alpha s +
// beta p, and by linearity each crystal amplitude is alpha a_s + beta a_p.
__device__ __forceinline__ void fresnel_in_pol_dev(double eo, double ee, const double cax[3], const double n[3],
                                                   const double d[3], const double e[3], double &Go, double &Ge,
                                                   double &Uo, double &Ue) {
  double t1[3], t2[3], k1;
  interface_basis(n, d, t1, t2, k1);
  const double c[3] = {cax[0] * t1[0] + cax[1] * t1[1] + cax[2] * t1[2],
                       cax[0] * t2[0] + cax[1] * t2[1] + cax[2] * t2[2],
                       cax[0] * n[0] + cax[1] * n[1] + cax[2] * n[2]};
  const double qi = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];  // < 0
  const cplx qr = q_iso_dev(1.0, k1, +1);
  const cplx qo = q_iso_dev(eo, k1, -1), qe = q_extra_dev(eo, ee, c, k1, -1);
  cplx fo[4], fe[4];
  crystal_tangential(eo, ee, c, true, k1, qo, fo);
  crystal_tangential(eo, ee, c, false, k1, qe, fe);
  const cplx y22 = cdiv(cx(k1 * k1) + qr * qr, qr);
  const cplx A[2] = {fo[2] - (cx(0.0) - qr * fo[1]), fo[3] - y22 * fo[0]};
  const cplx B[2] = {fe[2] - (cx(0.0) - qr * fe[1]), fe[3] - y22 * fe[0]};
  // s and p as in fresnel_in2_dev, one incident flux |qi| / 2 for both
  const cplx rs[2] = {cx(-qi) - (cx(0.0) - qr * cx(1.0)), cx(0.0)};
  const cplx rp[2] = {cx(0.0), cx(-qi * qi - k1 * k1) - y22 * cx(-qi)};
  cplx aos, aes, aop, aep;
  solve2(A, B, rs, aos, aes);
  solve2(A, B, rp, aop, aep);
  const double si = 0.5 * fabs(qi);
  const double fo_ = fabs(flux_t(fo)) / si, fe_ = fabs(flux_t(fe)) / si;
  Uo = 0.5 * (cabs2(aos) + cabs2(aop)) * fo_;
  Ue = 0.5 * (cabs2(aes) + cabs2(aep)) * fe_;
  const double al = e[0] * t2[0] + e[1] * t2[1] + e[2] * t2[2];
  const double be = -qi * (e[0] * t1[0] + e[1] * t1[1] + e[2] * t1[2]) + k1 * (e[0] * n[0] + e[1] * n[1] + e[2] * n[2]);
  Go = cabs2(al * aos + be * aop) * fo_;
  Ge = cabs2(al * aes + be * aep) * fe_;
}

// A crystal wave of `extra` with wave vector k (power towards +n) meets the
// interface: transmitted fraction T and the fractions Ro, Re reflected into
// the ordinary and the extraordinary wave (Sect. 3: two reflections in the
// crystal, one refraction into vacuum).
__device__ __forceinline__ void fresnel_out2_dev(double eo, double ee, const double cax[3], const double n[3],
                                                 const double k[3], int extra, double &T, double &Ro, double &Re) {
  double t1[3], t2[3], k1;
  interface_basis(n, k, t1, t2, k1);
  const double c[3] = {cax[0] * t1[0] + cax[1] * t1[1] + cax[2] * t1[2],
                       cax[0] * t2[0] + cax[1] * t2[1] + cax[2] * t2[2],
                       cax[0] * n[0] + cax[1] * n[1] + cax[2] * n[2]};
  const double qm = k[0] * n[0] + k[1] * n[1] + k[2] * n[2];
  const cplx qv = q_iso_dev(1.0, k1, +1);
  const cplx qo = q_iso_dev(eo, k1, -1), qe = q_extra_dev(eo, ee, c, k1, -1);
  cplx fm[4], fo[4], fe[4];
  crystal_tangential(eo, ee, c, !extra, k1, cx(qm), fm);
  crystal_tangential(eo, ee, c, true, k1, qo, fo);
  crystal_tangential(eo, ee, c, false, k1, qe, fe);
  const cplx y22 = cdiv(cx(k1 * k1) + qv * qv, qv);
  // (h - Y e) of the reflected waves; right side Y e_m - h_m
  const cplx A[2] = {fo[2] - (cx(0.0) - qv * fo[1]), fo[3] - y22 * fo[0]};
  const cplx B[2] = {fe[2] - (cx(0.0) - qv * fe[1]), fe[3] - y22 * fe[0]};
  const cplx r[2] = {(cx(0.0) - qv * fm[1]) - fm[2], y22 * fm[0] - fm[3]};
  cplx bo, be;
  solve2(A, B, r, bo, be);
  const double si = fabs(flux_t(fm));
  // transmitted tangential E = e_m + bo e_o + be e_e, H from the admittance
  cplx ft[4];
  ft[0] = fm[0] + bo * fo[0] + be * fe[0];
  ft[1] = fm[1] + bo * fo[1] + be * fe[1];
  ft[2] = cx(0.0) - qv * ft[1];
  ft[3] = y22 * ft[0];
  T = fabs(flux_t(ft)) / si;
  Ro = cabs2(bo) * fabs(flux_t(fo)) / si;
  Re = cabs2(be) * fabs(flux_t(fe)) / si;
}

// as fresnel_out2_dev, R the fraction reflected into the same wave type
__device__ __forceinline__ void fresnel_out_dev(double eo, double ee, const double cax[3], const double n[3],
                                                const double k[3], int extra, double &T, double &R) {
  double Ro, Re;
  fresnel_out2_dev(eo, ee, cax, n, k, extra, T, Ro, Re);
  R = extra ? Re : Ro;
}

// ---------------------------------------------------------------------------
// kind dispatch helpers (wave-uniform in practice: slots are grouped by kind)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void accel_k(int kind, double a, const double x[3],
                                        const double v[3], double A[3]) {
  switch (kind) {
    case K_RE: accel<K_RE>(a, x[0], x[1], v[0], v[1], v[2], A[0], A[1], A[2]); break;
    case K_AO: accel<K_AO>(a, x[0], x[1], v[0], v[1], v[2], A[0], A[1], A[2]); break;
    case K_AE: accel<K_AE>(a, x[0], x[1], v[0], v[1], v[2], A[0], A[1], A[2]); break;
    default: A[0] = 0.0; A[1] = 0.0; A[2] = 0.0; break;
  }
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inside_open(const CloakP& c, const double x[3]) {
  double r2 = fma(x[0], x[0], x[1] * x[1]);
  return r2 > c.a2 && r2 < c.b2 && x[2] > c.z0 && x[2] < c.z1;
}

// Boundary functions used inside the integrator, negative inside and equal
// to the distance to first order: (r^2 - b^2) / (2 b), (a^2 - r^2) / (2 a),
// z - z1, z0 - z. |g| <= tol places the state within tol (1 + O(tol/b)) of
// the boundary; no square root is needed, and dg/dh along a velocity v is
// (x v_x + y v_y) / b (resp. -/a) or +-v_z.
__device__ __forceinline__ double gsq(const CloakP& c, int id, const double x[3]) {
  double r2 = fma(x[0], x[0], x[1] * x[1]);
  switch (id) {
    case B_SIDE: return (r2 - c.b2) * (0.5 / c.b);
    case B_INNER: return (c.a2 - r2) * (0.5 / c.a);
    case B_TOP: return x[2] - c.z1;
    default: return c.z0 - x[2];
  }
}

__device__ __forceinline__ double gsq_slope(const CloakP& c, int id, const double x[3], const double v[3]) {
  double rv = fma(x[0], v[0], x[1] * v[1]);
  switch (id) {
    case B_SIDE: return rv * c.inv_b;
    case B_INNER: return -rv * c.inv_a;
    case B_TOP: return v[2];
    default: return -v[2];
  }
}

// first entry of o + s d (s > 0) into r <= b, z0 <= z <= z1; surf B_SIDE /
// B_TOP / B_BOTTOM. Stable quadratic roots.
__device__ __forceinline__ bool vacuum_entry(const CloakP& c, const double o[3], const double d[3],
                                             double& s_out, int& surf) {
  bool found = false;
  double best = __builtin_inf();
  double A = fma(d[0], d[0], d[1] * d[1]);
  double B = fma(o[0], d[0], o[1] * d[1]);
  double C = fma(o[0], o[0], fma(o[1], o[1], -c.b2));
  if (A > 0.0 && C > 0.0) {
    double disc = fma(B, B, -A * C);
    if (disc >= 0.0) {
      double sq = sqrt(disc);
      double qq = -(B + copysign(sq, B));
      double s1 = qq / A, s2 = C / qq;
      double s = fmin(s1, s2);
      double z = fma(s, d[2], o[2]);
      if (s > 0.0 && z >= c.z0 && z <= c.z1) { best = s; surf = B_SIDE; found = true; }
    }
  }
  if (d[2] < 0.0 && o[2] > c.z1 && c.z1 < __builtin_inf()) {
    double s = (c.z1 - o[2]) / d[2];
    double x = fma(s, d[0], o[0]), y = fma(s, d[1], o[1]);
    if (s > 0.0 && fma(x, x, y * y) <= c.b2 && s < best) { best = s; surf = B_TOP; found = true; }
  }
  if (d[2] > 0.0 && o[2] < c.z0 && c.z0 > -__builtin_inf()) {
    double s = (c.z0 - o[2]) / d[2];
    double x = fma(s, d[0], o[0]), y = fma(s, d[1], o[1]);
    if (s > 0.0 && fma(x, x, y * y) <= c.b2 && s < best) { best = s; surf = B_BOTTOM; found = true; }
  }
  s_out = best;
  return found;
}

// uniaxial principal values and optic axis at x (Eq. (14) / Eq. (15), Eq. (1))
// `axis` is the branch kind's (kind >> 1), not c.axis: cloaks rendered together
// share one CloakP for their common geometry
__device__ __forceinline__ void material_axis(const CloakP &c, int axis, const double x[3], double &eo,
                                              double &ee, double cax[3]) {
  const double w = rsq64(fma(x[0], x[0], x[1] * x[1]));
  const double q = fma(-c.a, w, 1.0);
  const double ks = c.kappa * q * q;
  if (axis == 0) {  // radial: c = r_hat, eps_e = eps_r
    eo = c.kappa; ee = ks;
    cax[0] = x[0] * w; cax[1] = x[1] * w; cax[2] = 0.0;
  } else {            // azimuthal: c = theta_hat, eps_e = eps_theta
    eo = ks; ee = c.kappa;
    cax[0] = -x[1] * w; cax[1] = x[0] * w; cax[2] = 0.0;
  }
}

// outward normal of boundary `id` at x (the inner boundary's normal points
// into the metal, i.e. along -r_hat seen from the material ... we return r_hat;
// reflection only needs the line)
__device__ __forceinline__ void boundary_normal(int id, const double x[3], double n[3]) {
  if (id == B_TOP) { n[0] = 0.0; n[1] = 0.0; n[2] = 1.0; return; }
  if (id == B_BOTTOM) { n[0] = 0.0; n[1] = 0.0; n[2] = -1.0; return; }
  double w = rsq64(fma(x[0], x[0], x[1] * x[1]));
  n[0] = x[0] * w; n[1] = x[1] * w; n[2] = 0.0;
}

__device__ __forceinline__ void reflect3(double v[3], const double n[3]) {
  double d = 2.0 * (v[0] * n[0] + v[1] * n[1] + v[2] * n[2]);
  v[0] = fma(-d, n[0], v[0]);
  v[1] = fma(-d, n[1], v[1]);
  v[2] = fma(-d, n[2], v[2]);
}

// local frame (r_hat, t_hat, z_hat) at x; w = 1/r
__device__ __forceinline__ void local_frame(const double x[3], double rh[2], double th[2], double& w) {
  double r2 = fma(x[0], x[0], x[1] * x[1]);
  w = rsq64_1(r2);
  rh[0] = x[0] * w; rh[1] = x[1] * w;
  th[0] = -rh[1]; th[1] = rh[0];
}

// Eq. (12) at an exit, evaluated after the integration (one ray per lane):
// the crystal wave that left through boundary rid at x is rebuilt from the
// outgoing vacuum direction d. Its tangential k equals d's (Eq. (11)); its
// normal component is the outward root of the branch's dispersion
// k^T M^-1 k = 1, with M diagonal in (r, theta, z) and the normal one of
// those axes. T transmitted, Ro / Re reflected into the ordinary /
// extraordinary wave; exit_transmission returns T alone.
__device__ __forceinline__ void exit_fresnel(const CloakP &c, int kind, int rid, const double x[3],
                                             const double d[3], double &T, double &Ro, double &Re) {
  double rh[2], th[2], w;
  local_frame(x, rh, th, w);
  double mr, mt, mz;
  metric_diag(kind, c.kappa, c.a, w, mr, mt, mz);
  const double dr = d[0] * rh[0] + d[1] * rh[1], kt = d[0] * th[0] + d[1] * th[1];
  double kr, kz;
  if (rid == B_SIDE) {
    kz = d[2];
    kr = sqrt(fmax(mr * (1.0 - kt * kt / mt - kz * kz / mz), 0.0));
  } else {
    kr = dr;
    const double q = sqrt(fmax(mz * (1.0 - kr * kr / mr - kt * kt / mt), 0.0));
    kz = rid == B_TOP ? q : -q;
  }
  const double k[3] = {kr * rh[0] + kt * th[0], kr * rh[1] + kt * th[1], kz};
  double eo, ee, cax[3], nrm[3];
  material_axis(c, kind >> 1, x, eo, ee, cax);
  boundary_normal(rid, x, nrm);
  fresnel_out2_dev(eo, ee, cax, nrm, k, kind & 1, T, Ro, Re);
}

__device__ __forceinline__ double exit_transmission(const CloakP &c, int kind, int rid, const double x[3],
                                                    const double d[3]) {
  double T, Ro, Re;
  exit_fresnel(c, kind, rid, x, d, T, Ro, Re);
  return T;
}

// Entry refraction (Sect. 3) at a point of boundary `surf` with outward
// normal along r_hat (side) or +/- z (caps). kin: unit vacuum direction.
// Returns false if the transmitted wave is evanescent. v: ray velocity.
__device__ __forceinline__ bool refract_in(const CloakP& c, int kind, int surf, const double x[3],
                                           const double kin[3], double v[3]) {
  double rh[2], th[2], w;
  local_frame(x, rh, th, w);
  double mr, mt, mz;
  metric_diag(kind, c.kappa, c.a, w, mr, mt, mz);
  double kr = kin[0] * rh[0] + kin[1] * rh[1];
  double kt = kin[0] * th[0] + kin[1] * th[1];
  double kz = kin[2];
  double q2;
  if (surf == B_SIDE) {
    q2 = mr * (1.0 - kt * kt / mt - kz * kz / mz);
    if (!(q2 >= 0.0)) return false;
    kr = -sqrt(q2);  // into the material: -r_hat
  } else {
    q2 = mz * (1.0 - kr * kr / mr - kt * kt / mt);
    if (!(q2 >= 0.0)) return false;
    kz = surf == B_TOP ? -sqrt(q2) : sqrt(q2);
  }
  double vr = kr / mr, vt = kt / mt;
  v[0] = vr * rh[0] + vt * th[0];
  v[1] = vr * rh[1] + vt * th[1];
  v[2] = kz / mz;
  return true;
}

// Exit refraction into vacuum at boundary `id` (Sect. 3): k = M v, tangential
// part kept, normal part sqrt(1 - |k_t|^2) outward. Returns false on total
// internal reflection. Also returns |v^T M v - 1| in hres.
__device__ __forceinline__ bool refract_out(const CloakP& c, int kind, int id, const double x[3],
                                            const double v[3], double d[3], double& hres) {
  double rh[2], th[2], w;
  local_frame(x, rh, th, w);
  double mr, mt, mz;
  metric_diag(kind, c.kappa, c.a, w, mr, mt, mz);
  double vr = v[0] * rh[0] + v[1] * rh[1];
  double vt = v[0] * th[0] + v[1] * th[1];
  double vz = v[2];
  hres = fabs(fma(mr * vr, vr, fma(mt * vt, vt, mz * vz * vz)) - 1.0);
  double kr = mr * vr, kt = mt * vt, kz = mz * vz;
  if (id == B_SIDE) {
    double t2 = fma(kt, kt, kz * kz);
    if (t2 > 1.0) return false;
    kr = sqrt(1.0 - t2);
  } else {
    double t2 = fma(kr, kr, kt * kt);
    if (t2 > 1.0) return false;
    kz = id == B_TOP ? sqrt(1.0 - t2) : -sqrt(1.0 - t2);
  }
  d[0] = kr * rh[0] + kt * th[0];
  d[1] = kr * rh[1] + kt * th[1];
  d[2] = kz;
  return true;
}

// same-mode specular reflection inside the material at boundary `id`: M is
// diagonal in (r, theta, z), so the reflected wave flips the normal component
__device__ __forceinline__ void reflect_inside(int id, const double x[3], double v[3]) {
  double n[3];
  boundary_normal(id, x, n);
  reflect3(v, n);
}

__device__ __forceinline__ double hamiltonian_res(const CloakP& c, int kind, const double x[3],
                                                  const double v[3]) {
  double rh[2], th[2], w;
  local_frame(x, rh, th, w);
  double mr, mt, mz;
  metric_diag(kind, c.kappa, c.a, w, mr, mt, mz);
  double vr = v[0] * rh[0] + v[1] * rh[1];
  double vt = v[0] * th[0] + v[1] * th[1];
  return fabs(fma(mr * vr, vr, fma(mt * vt, vt, mz * v[2] * v[2])) - 1.0);
}

// larger root of |p + s d|_xy = R (outgoing crossing), 0 if none
__device__ __forceinline__ double leave_radius(const double p[3], const double d[3], double R) {
  double A = fma(d[0], d[0], d[1] * d[1]);
  if (!(A > 0.0)) return 0.0;
  double B = fma(p[0], d[0], p[1] * d[1]);
  double C = fma(p[0], p[0], fma(p[1], p[1], -R * R));
  double disc = fma(B, B, -A * C);
  if (disc < 0.0) return 0.0;
  double sq = sqrt(disc);
  double s = (B <= 0.0) ? (sq - B) / A : -C / (B + sq);
  return s > 0.0 ? s : 0.0;
}

// ---------------------------------------------------------------------------
// camera and room
// ---------------------------------------------------------------------------
struct CamP {
  double eye[3], F[3], R[3], U[3];
  double tan_half, aspect;
  double inv_w, inv_h;  // 1/w, 1/h when w, h are powers of two (exact), else 0
  int w, h, spp, m;
  unsigned long long seed;
};

// SplitMix64 (Steele, Lea & Flood 2014): n-th output of the generator seeded
// with `seed`
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed,
                                                         unsigned long long n) {
  unsigned long long z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void camera_ray(const CamP& cam, int cam_index, long long pix, int smp,
                                           double d[3]) {
  // pix < w h <= 2^30: 32-bit index arithmetic
  const unsigned int p32 = (unsigned int)pix, row = p32 / (unsigned int)cam.w, col = p32 - row * (unsigned int)cam.w;
  double ox = 0.5, oy = 0.5;
  if (cam.spp > 1) {
    unsigned long long key = ((unsigned long long)cam_index << 40) ^
                             ((unsigned long long)pix << 8) ^ (unsigned long long)smp;
    double x1 = (double)(splitmix64(cam.seed, 2 * key + 1) >> 11) * 0x1.0p-53;
    double x2 = (double)(splitmix64(cam.seed, 2 * key + 2) >> 11) * 0x1.0p-53;
    ox = ((double)(smp % cam.m) + x1) / cam.m;
    oy = ((double)(smp / cam.m) + x2) / cam.m;
  }
  // a power-of-two size divides exactly as a multiplication by its inverse
  const double fx = cam.inv_w > 0.0 ? ((double)col + ox) * cam.inv_w : ((double)col + ox) / cam.w;
  const double fy = cam.inv_h > 0.0 ? ((double)row + oy) * cam.inv_h : ((double)row + oy) / cam.h;
  double u = (fx * 2.0 - 1.0) * cam.tan_half * cam.aspect;
  double v = (1.0 - fy * 2.0) * cam.tan_half;
  double dx = cam.F[0] + u * cam.R[0] + v * cam.U[0];
  double dy = cam.F[1] + u * cam.R[1] + v * cam.U[1];
  double dz = cam.F[2] + u * cam.R[2] + v * cam.U[2];
  double w = rsq64(fma(dx, dx, fma(dy, dy, dz * dz)));
  d[0] = dx * w; d[1] = dy * w; d[2] = dz * w;
}

struct RoomP {
  double lo[3], hi[3], tile, inv_tile;
  int tile_pow2, pad;  // tile is a power of two: floor(u / tile) == floor(u * inv_tile) exactly
};

// face*2 + parity of the room point hit by o + s d (s >= 0) from inside
__device__ __forceinline__ int room_code(const RoomP& rm, const double o[3], const double d[3],
                                         double& s_hit) {
  // nearest wall: compare the distances (plane - o)/d as fractions with
  // positive denominators (no division), then divide once for the winner
  double bn = 1.0, bd = 0.0;  // best = bn / bd, +inf to start
  int face = -1;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (d[ax] != 0.0) {
      const double plane = d[ax] > 0.0 ? rm.hi[ax] : rm.lo[ax];
      const double num = d[ax] > 0.0 ? plane - o[ax] : o[ax] - plane;
      const double den = fabs(d[ax]);
      if (num * bd < bn * den) { bn = num; bd = den; face = 2 * ax + (d[ax] > 0.0 ? 1 : 0); }
    }
  }
  double best = face >= 0 ? bn / bd : 0.0;
  if (face < 0) { s_hit = 0.0; return 12; }
  if (best < 0.0) best = 0.0;
  s_hit = best;
  int ax = face >> 1;
  int ua = ax == 0 ? 1 : 0;
  int va = ax == 2 ? 1 : 2;
  double pu = fma(best, d[ua], o[ua]);
  double pv = fma(best, d[va], o[va]);
  const double fu = rm.tile_pow2 ? floor(pu * rm.inv_tile) : floor(pu / rm.tile);
  const double fv = rm.tile_pow2 ? floor(pv * rm.inv_tile) : floor(pv / rm.tile);
  long long par = ((long long)fu + (long long)fv) & 1;
  return face * 2 + (int)par;
}

// Distance, within its face, from the room point o + s d (face `face` of
// room_code) to the nearest tile edge or face boundary, and the cosine
// |d . n| of the ray with the face normal. A small error in o or d moves the
// point by (error across the ray) / cosine along the face.
__device__ __forceinline__ double tile_edge_distance(const RoomP& rm, const double o[3], const double d[3],
                                                     double s, int face, double& cosn) {
  const int ax = face >> 1;
  const int ua = ax == 0 ? 1 : 0;
  const int va = ax == 2 ? 1 : 2;
  double dist = __builtin_inf();
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int a = k == 0 ? ua : va;
    const double pc = fma(s, d[a], o[a]);
    const double f = pc / rm.tile - floor(pc / rm.tile);
    dist = fmin(dist, fmin(f, 1.0 - f) * rm.tile);
    dist = fmin(dist, fmin(fabs(pc - rm.lo[a]), fabs(rm.hi[a] - pc)));
  }
  cosn = fabs(d[ax]);
  return dist;
}

}  // namespace rtk
