/*
 * cloak_oracle.h -- plain FP64 CPU reference for ray tracing through the
 * uniaxial-dielectric cylindrical cloaks of Halimeh & Wegener,
 * "Photorealistic ray tracing of free-space invisibility cloaks made of
 * uniaxial dielectrics".
 *
 * TEST INFRASTRUCTURE. This library is the oracle that the GPU library is
 * checked against. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it. It shares no code, header or table with the
 * GPU library, and the GPU library never links or calls it.
 *
 * All pointers are host pointers owned by the caller. Lengths are in the
 * cloak's units, c0 = omega = 1, so the ODE time equals the optical path.
 */
#ifndef CLOAK_ORACLE_H
#define CLOAK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_AXIS_RADIAL = 0, ORC_AXIS_AZIMUTHAL = 1 };
enum { ORC_ORDINARY = 0, ORC_EXTRAORDINARY = 1 };
/* ORC_RK4_HAM: classical RK4 with a fixed step in the ray parameter tau of
   the Hamiltonian H(x, k) = k^T A k - f (A = eps, f = eps_o eps_e for the
   extraordinary wave; A = I, f = eps_o for the ordinary one), the form the
   paper compares its Eq. (8) tracer against (Sect. 4). ORC_RK4_HAMC: the same
   with the canonical normalization H / f = k^T M^-1 k - 1 (the same rays,
   tau proportional to the optical path). */
enum { ORC_RK4 = 0, ORC_DP45 = 1, ORC_RK4_HAM = 2, ORC_RK4_HAMC = 3 };
enum {
    ORC_EXITED = 0, ORC_MISSED = 1, ORC_ABSORBED = 2, ORC_MAXSTEPS = 3,
    ORC_DIVERGED = 4, ORC_TIR = 5, ORC_INVALID = 6, ORC_REFLECTED = 7
};

typedef struct {
    double a, b;          /* inner and outer radius, Sect. 4 (Eq. 13) */
    double z0, z1;        /* axial extent; -inf/+inf for an infinite cylinder */
    int32_t axis;         /* ORC_AXIS_*: Eq. (14) or Eq. (15) */
    int32_t inner_mirror; /* 1: r < a is a perfect metal mirror (Sect. 4) */
} orc_cloak;

typedef struct {
    int32_t scheme;       /* ORC_RK4, ORC_DP45, ORC_RK4_HAM or ORC_RK4_HAMC */
    int32_t max_bounces;  /* internal reflections before status TIR */
    double h;             /* RK4 step in t, RK4_HAM step in tau, DP45 initial step */
    double rtol, atol, hmax;
    double r_out;         /* report radius for orc_trace */
    int64_t max_steps;    /* step attempts per ray */
} orc_opts;

typedef struct {
    double eye[3], look[3], up[3], fov_deg;
    int32_t w, h, spp;    /* spp must be a perfect square */
    uint64_t seed;
} orc_camera;

typedef struct {
    double lo[3], hi[3], tile;
    float rgb[6][2][3];   /* face (x-,x+,y-,y+,z-,z+) x tile parity */
} orc_room;

/* Trace n vacuum rays (SoA 6 x n: ox,oy,oz,dx,dy,dz) through the cloak and
   report each outgoing ray where it crosses r = r_out. Outputs: SoA 6 x n
   (point, unit direction), optical path, status, |H-1| at the last interface
   (NaN when the ray never entered), step attempts, and the Eq. (12) weight
   of the reported ray (unpolarized entry transmission of the branch times
   the same-mode reflectance of each internal reflection times the exit
   transmission; 1 for a miss or a reflection off the metal end disk, 0 when
   the ray does not exit). Any output
   pointer but out6 may be NULL. OpenMP over rays. */
void orc_trace(const orc_cloak *c, const orc_opts *o, int32_t branch, int64_t n,
               const double *in6, double *out6, double *opl, int32_t *status,
               double *hres, int64_t *nsteps, double *trans);

/* Render selected samples: ids[i] = pixel * spp + sample, pixel = row * w + col.
   code = face * 2 + parity (0..11), 12 = black (absorbed, TIR, step limit,
   diverged). rec (7 x n SoA, may be NULL): origin and direction of the last
   vacuum ray, and the optical path from the eye to the room. c may be NULL
   (empty room). */
void orc_render_samples(const orc_cloak *c, const orc_opts *o, const orc_room *room,
                        const orc_camera *cam, int32_t cam_index, int32_t branch,
                        int64_t n, const int64_t *ids, uint8_t *code,
                        double *rec, int32_t *status, double *wimg);

/* Eq. (12): intensity transmission of unpolarized light (the mean over two
   orthogonal incident polarizations) from vacuum into the crystal, T[0]
   ordinary and T[1] extraordinary, and the reflected vacuum fraction R.
   nhat: normal pointing out of the crystal; kin: unit vacuum direction
   (kin . nhat < 0). Returns nonzero if the continuity system is singular. */
int32_t orc_fresnel_in(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                       const double kin[3], double T[2], double *R);

/* Eq. (12) at the entry for one linear polarization: the incident vacuum
   field along e_in (its part transverse to kin is used, normalized); T[0],
   T[1] the fluxes into the ordinary and extraordinary waves and R the
   reflected flux, over the incident flux. The mean over any two orthogonal
   e_in is orc_fresnel_in. Returns nonzero if e_in has no transverse part or
   the continuity system is singular. */
int32_t orc_fresnel_in_pol(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                           const double kin[3], const double e_in[3], double T[2], double *R);

/* Eq. (12) at the exit: an ordinary or extraordinary wave with wave vector
   k_in (power towards +nhat) meets the crystal/vacuum interface; T is the
   transmitted fraction (0 under total internal reflection), R[0] and R[1]
   the fractions reflected into the ordinary and extraordinary waves. */
int32_t orc_fresnel_out(double eps_o, double eps_e, const double chat[3], const double nhat[3],
                        const double k_in[3], int32_t branch, double *T, double R[2]);

/* Polarizer goggles (Sect. 4, Figs. 1d,e and 2d,e): e = the transmission
   axis of goggle 0 (in-plane: the camera's horizontal axis projected on the
   plane normal to the unit ray direction d) or 1 (axial: d x that
   projection). Returns nonzero if the projection vanishes. */
int32_t orc_goggle_axis(const orc_camera *cam, const double d[3], int32_t goggle, double e[3]);

/* Per camera sample (ids as orc_render_samples), the share of its light that
   reaches the camera through goggle `goggle` by way of branch `branch`: 1/4
   for a ray that stays in vacuum, 1/2 x the trace weight with the goggle's
   field at the entry for a ray through the crystal, 0 otherwise. */
void orc_render_goggle(const orc_cloak *c, const orc_opts *o, const orc_camera *cam, int32_t cam_index,
                       int32_t branch, int32_t goggle, int64_t n, const int64_t *ids, double *wg);

/* First-order reflections of vacuum rays (in6 as orc_trace) through branch
   `branch`, unpolarized light: w[j * n + i] the flux fraction of
   contribution j (0: the entry's reflected vacuum ray, 1 / 2: the ordinary
   / extraordinary wave reflected at the exit, followed to its own exit; 0
   if absent) and ray[(j * 6 + q) * n + i] that contribution's vacuum ray
   at the interface it leaves (point, then unit direction). */
void orc_trace_reflections(const orc_cloak *c, const orc_opts *o, int32_t branch, int64_t n, const double *in6,
                           double *w, double *ray);

/* First-order reflections (Sect. 4; Sect. 3 for the two reflected waves in
   the crystal): per camera sample (ids as orc_render_samples) and branch,
   three contributions j (0: the vacuum ray reflected at the first crystal
   interface, 1 / 2: the ordinary / extraordinary wave the branch's ray
   reflects into at its exit, followed to its own exit without further
   partial reflections), their image weights w[j * n + i] and room codes
   code[j * n + i] (12: none). goggle -1: unpolarized image (the entry's
   reflected fraction split evenly over the two branches); 0, 1: that
   goggle's image. */
void orc_render_reflections(const orc_cloak *c, const orc_opts *o, const orc_room *room, const orc_camera *cam,
                            int32_t cam_index, int32_t branch, int32_t goggle, int64_t n, const int64_t *ids,
                            double *w, uint8_t *code);

/* Pieces exposed for the pin tests. *//* Pieces exposed for the pin tests. */
void orc_eps_cyl(const orc_cloak *c, double r, double out3[3]);
void orc_metric(const orc_cloak *c, const double x[3], double M[9]);
void orc_metric_det_form(const orc_cloak *c, const double x[3], double M[9]);
void orc_rhs(const orc_cloak *c, int32_t branch, const double y[6], double dy[6]);
void orc_rhs_eq8_isotropic(const orc_cloak *c, const double y[6], double dy[6]);
int32_t orc_refract_in(double eps_o, double eps_e, const double chat[3],
                       const double nhat[3], const double kin[3], int32_t branch,
                       double k_out[3], double v_out[3]);
int32_t orc_refract_out(double eps_o, double eps_e, const double chat[3],
                        const double nhat[3], const double v_in[3], int32_t branch,
                        double d_out[3]);
void orc_camera_ray(const orc_camera *cam, int32_t cam_index, int64_t id,
                    double o[3], double d[3]);
int32_t orc_room_code(const orc_room *room, const double o[3], const double d[3],
                      double *s_hit);
uint64_t orc_splitmix64(uint64_t seed, uint64_t n);
double orc_test_oscillator(int32_t scheme, double h, double rtol, double T,
                           double y_out[6], int64_t *nsteps);
int32_t orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
