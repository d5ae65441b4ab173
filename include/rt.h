/*
 * rt.h -- C ABI of the MI355X (gfx950) ray tracer for the uniaxial-dielectric
 * cylindrical invisibility cloaks of Halimeh & Wegener, "Photorealistic ray
 * tracing of free-space invisibility cloaks made of uniaxial dielectrics".
 *
 * Conventions (every entry point):
 *  - Array arguments are DEVICE pointers (HIP global memory) owned by the
 *    caller; the library never frees or retains them past the call.
 *  - `stream` is a hipStream_t (NULL = the null stream). Calls validate their
 *    arguments synchronously, then enqueue work asynchronously on `stream`
 *    and return. Results are valid once the stream has been synchronized.
 *  - Return value: RT_OK or an RT_E_* code; rt_last_error() gives a
 *    thread-local message for the last failed call. No C++ exception crosses
 *    the ABI. Argument errors are reported before anything is enqueued.
 *  - Per-ray outcomes are never call failures: they are reported in the
 *    per-ray status arrays (RT_RAY_*).
 *  - Units: lengths in the cloak's units, c0 = omega = 1, so the ODE time of
 *    Eq. (2)/(8) is the optical path length and |k| is the phase index.
 *  - Handles (rt_cloak) are immutable after creation and may be used from
 *    several streams at once; calls that run concurrently must not share
 *    output buffers.
 *  - The library allocates a device workspace on first use and grows it when
 *    a larger call needs it (hipMalloc, synchronous); it is released by
 *    rt_release_workspace() or at process exit. Calls that use it on
 *    different streams are ordered on the device: each waits for the
 *    previous use (an event), so their work does not overlap, except that
 *    rt_render and rt_render_multi keep up to four workspaces, one per
 *    stream they are called on (a fifth stream takes the one used longest
 *    ago): renders issued on several streams run side by side, at one
 *    workspace's memory per stream. A call waits on the host for its
 *    workspace's previous use before it copies its camera records. Renders are processed in
 *    chunks of camera samples (2^26 unless max_chunk says otherwise, at most
 *    2^28), with a workspace of ~0.5 KB per sample of a chunk (~31 GB for a
 *    4096 x 4096 x 4 spp view).
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RT_OK = 0, RT_E_INVALID = 1, RT_E_NOMEM = 2, RT_E_DEVICE = 3, RT_E_UNSUPPORTED = 4 };

/* Optic-axis field of the cloak: Eq. (14) (c along r) or Eq. (15) (c along theta). */
enum { RT_AXIS_RADIAL = 0, RT_AXIS_AZIMUTHAL = 1 };

/* Ray branch inside the cloak (Sect. 2): ordinary (Eq. (2)) or extraordinary (Eq. (8)). */
enum { RT_POL_ORDINARY = 0, RT_POL_EXTRAORDINARY = 1 };

enum { RT_SCHEME_RK4 = 0, RT_SCHEME_DP45 = 1, RT_SCHEME_RK4_HAM = 2, RT_SCHEME_RK4_HAMC = 3 };
enum { RT_PREC_FP64 = 0, RT_PREC_MIXED = 1 };

/* Per-ray outcome. */
enum {
    RT_RAY_EXITED = 0,    /* crossed the cloak and left it through an interface */
    RT_RAY_MISSED = 1,    /* never touched the cloak */
    RT_RAY_ABSORBED = 2,  /* reached the inner radius where no mirror reflects it */
    RT_RAY_MAXSTEPS = 3,  /* step budget exhausted inside the cloak */
    RT_RAY_DIVERGED = 4,  /* non-finite state, step-size collapse, or |v^T M v - 1| > 1e-3
                             at an outer interface (no longer a ray of the medium) */
    RT_RAY_TIR = 5,       /* more internal reflections than max_bounces */
    RT_RAY_INVALID = 6,   /* non-finite input, zero direction or origin inside the cloak */
    RT_RAY_REFLECTED = 7  /* reflected at the entry (evanescent transmission, metal end disk) */
};

typedef struct rt_cloak_s *rt_cloak;
typedef struct rt_plan_s *rt_plan;
typedef struct rt_model_s *rt_model;

/* Cloak geometry and material (Sect. 4, Eqs. (13)-(15)). The material fills
   r1 <= r <= r2, z0 <= z <= z1 (z0 = -INFINITY, z1 = +INFINITY: infinitely
   long cylinder). inner_mirror = 1: r < r1 is the perfect metal cylinder the
   cloak hides (Sect. 4), including its end disks; 0: r < r1 absorbs. */
typedef struct {
    double r1, r2;
    double z0, z1;
    int32_t axis;
    int32_t inner_mirror;
} rt_cloak_desc;

/* Integration options. scheme: RT_SCHEME_RK4 (fixed step h, the paper's
   fourth-order Runge-Kutta, Sect. 4) or RT_SCHEME_DP45 (Dormand-Prince 5(4),
   initial step h, tolerances rtol/atol, maximum step hmax), both on the ray
   equation Eq. (8)/(2) in (x, v). RT_SCHEME_RK4_HAM: the Hamiltonian form the
   paper compares against (Sect. 4): state (x, k), H = k^T A k - f with A = eps
   and f = eps_o eps_e (extraordinary) or A = I and f = eps_o (ordinary),
   classical RK4 with the fixed step h in the ray parameter tau
   (dx/dtau = 2 A k, dt/dtau = 2 f). RT_SCHEME_RK4_HAMC: the same with the
   canonical normalization H / f = k^T M^-1 k - 1 (the same rays; the ray
   parameter advances with the optical path, dt/dtau = 2, and the right-hand
   side is singular at r1 as Eq. (8)'s is). Interfaces, events and
   outputs are those of the other schemes (k is converted to v = M^-1 k at
   every interface). precision: RT_PREC_FP64 (all arithmetic in FP64).
   RT_PREC_MIXED (the derivative evaluated in FP32 away from r1) is rejected
   with RT_E_UNSUPPORTED: its rounding, amplified near the singular inner
   radius, moves exits by more than the 1e-6 bar, and on this GPU FP32 and
   FP64 vector arithmetic issue at the same rate. fp64_band is unused.
   r_out: report radius of rt_trace_batch (>= r2). max_steps: step attempts per
   ray. max_bounces: internal reflections (inner mirror, total internal
   reflection) per ray, 0..64. block / refill_period: integrator launch shape
   (threads per block, steps between refills of finished lanes; 0 = library
   default). max_chunk: renders only, camera samples per integrator launch,
   at most 2^28 (0 = 2^26; results do not depend on it). A launch lasts at
   least as long as its longest ray (paths that pass close to r1 take tens of
   thousands of attempts), so views rendered together in one launch overlap
   one view's longest rays with the others' bulk. */
typedef struct {
    int32_t scheme;
    int32_t precision;
    double h, rtol, atol, hmax;
    double fp64_band;
    double r_out;
    int64_t max_steps;
    int32_t max_bounces;
    int32_t block;
    int32_t refill_period;
    int32_t max_chunk;
} rt_trace_opts;

/* Pinhole camera: eye, look-at point, up vector, vertical full field of view
   (degrees), image w x h (row 0 at the top, square pixels), spp samples per
   pixel (a perfect square; 1 = pixel centre, m*m = stratified m x m grid
   jittered by SplitMix64 outputs keyed by (camera index, pixel, sample)). */
typedef struct {
    double eye[3], look[3], up[3];
    double fov_deg;
    int32_t w, h, spp, reserved;
    uint64_t seed;
} rt_camera;

/* Backdrop: axis-aligned room [lo, hi] seen from inside, checkerboard tiles
   of side `tile`, colour rgb[face][parity] with faces x-, x+, y-, y+, z-, z+
   and parity (floor(u/tile) + floor(v/tile)) mod 2 of the in-face coordinates. */
typedef struct {
    double lo[3], hi[3];
    double tile;
    float rgb[6][2][3];
} rt_room;

/* Optional outputs of rt_render, each laid out per image (camera-major,
   then branch); NULL fields are not written. Per sample (ns = w*h*spp
   samples per image): rec: SoA 7 x ns doubles (origin and direction of the
   last vacuum ray, optical path from the eye to the room); status: RT_RAY_*;
   code: face*2 + parity of the room point seen, 12 = black; nsteps:
   integrator step attempts. Per pixel (w*h floats per image): tof: time of
   flight, the mean over the pixel's samples that reach the room of their
   optical path from the eye (c0 = 1, so optical path = time; the ray ODE's
   time inside the cloak, App. A), NaN if none does. With the empty room's
   image it gives the time-of-flight difference the cloak makes (Sect. 4).
   unpol: the unpolarized image (Eq. (12), Fig. 1c), one per (cloak,
   camera) rather than per branch (n_cloaks x n_cams x h x w x 3 floats, or
   n_cams x h x w x 3 without a cloak): per sample, the sum over the two
   branches of the share of its unpolarized light the branch carries to the
   room times the colour it sees there, averaged over the pixel's samples.
   A sample that stays in vacuum (a miss, the metal end disk) gives each
   branch 1/2; one that crosses the crystal gives its branch the weight
   rt_trace_batch reports as trans; light reflected at the crystal surface
   is not imaged. Needs pol_mask = 3 and RT_PREC_FP64, else RT_E_UNSUPPORTED
   (and always in rt_render_surrogate).
   goggle_inplane, goggle_axial: the images through a linear polarizer in
   front of the camera (Sect. 4, Figs. 1d,e and 2d,e), laid out as unpol.
   The in-plane goggle transmits the field along the camera's horizontal
   axis (F x up), which at elevation 0 lies in the cylinder's cross-section,
   the plane the cloaks are designed for: the paper's cylinder lies
   horizontally, so this is its "vertical" goggle (Fig. 1d, 2d), and the
   axial goggle its "horizontal" one (Fig. 1e, 2e). For a sample of unit
   direction d the axes are the horizontal axis projected transverse to d
   and d x that projection. Room light is unpolarized: a sample that stays
   in vacuum gives each goggle half its light (1/4 per branch); for one
   through the crystal, by reciprocity, the goggle's share is half its trace
   weight with the entry taking the goggle's field instead of unpolarized
   light (entry transmission of that field into the branch x internal
   reflectances x exit transmission). The two goggle images add up to the
   unpolarized one. Same requirements as unpol.
   reflections: nonzero adds first-order reflections (Sect. 4: reflections
   of the first order are kept, higher orders dropped) to unpol and the
   goggle images: the vacuum ray reflected where the sample first meets the
   crystal (fraction 1 - T_o - T_e of its light, half per branch), and at
   each branch's exit the waves reflected into the ordinary and the
   extraordinary mode (Sect. 3: two reflections in the crystal, one
   refraction), each followed through the cloak to its own exit, where it
   refracts out with its transmission; their own partial reflections are
   not followed. The branch images and the per-sample outputs are those of
   the primary rays alone. Needs unpol or a goggle image (RT_E_INVALID
   otherwise); renders in chunks of at most 2^22 samples and needs a second
   work table (about 1 KB per sample of a chunk); not taken by render plans
   or rt_render_surrogate (RT_E_UNSUPPORTED). */
typedef struct {
    double *rec;
    int32_t *status;
    uint8_t *code;
    int32_t *nsteps;
    float *tof;
    float *unpol;
    float *goggle_inplane;
    float *goggle_axial;
    int32_t reflections;
} rt_render_aux;

/* Build a cloak handle (host-side constants; no device memory).
   Errors: RT_E_INVALID unless 0 < r1 < r2, z0 < z1, axis in {0, 1}. */
int rt_build_cloak(const rt_cloak_desc *desc, rt_cloak *out);

/* Free a handle from rt_build_cloak. NULL is accepted. */
int rt_free_cloak(rt_cloak cloak);

/* Trace n vacuum rays through the cloak (Sects. 2-4): vacuum leg to the
   cloak, double refraction into branch `pol` (Sect. 3, Eqs. (6), (9)-(11)),
   integration of Eq. (2) (ordinary) or Eq. (8) (extraordinary), reflection at
   the inner metal cylinder (Sect. 4), exit refraction into vacuum (Sect. 3),
   and the vacuum leg to the cylinder r = r_out.
     in6:    SoA 6 x n doubles: origin x,y,z then direction x,y,z (any length > 0)
     out6:   SoA 6 x n doubles: point where the outgoing ray crosses r = r_out
             (the last state for rays that did not leave), unit direction
     opl:    n doubles, optical path from the origin to out6's point
     status: n int32, RT_RAY_*
     hres:   n doubles or NULL, |v^T M v - 1| at the last interface (NaN if the
             ray never entered)
     nsteps: n int32 or NULL, integrator step attempts
     trans:  n doubles or NULL, the ray's intensity weight from Eq. (12): the
             unpolarized transmission into branch `pol` at entry, times the
             same-branch reflectance at every internal reflection at the outer
             surface or an end cap, times the transmission into vacuum at exit.
             Plane-wave transmittances at a locally flat interface, from
             continuity of tangential E and H (Sect. 3); the cross-polarized
             reflected wave is dropped. 1 for a miss or a reflection off the
             metal end disk (the metal reflects every polarization), 0 for a
             ray that did not leave or that the crystal surface reflected.
             Needs RT_PREC_FP64.
   n = 0 is a no-op. Errors: RT_E_INVALID (NULL handle/options/required
   pointer, n < 0, r_out < r2, bad options), RT_E_UNSUPPORTED (trans with
   RT_PREC_MIXED), RT_E_NOMEM (workspace), RT_E_DEVICE (launch failure). */
int rt_trace_batch(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n,
                   const double *in6, double *out6, double *opl, int32_t *status,
                   double *hres, int32_t *nsteps, double *trans, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops, harnesses that forbid hipMalloc): rt_trace_batch
   without any allocation. Same arguments, semantics, outputs and errors as
   rt_trace_batch, for at most RT_NOALLOC_MAX_RAYS rays per call (more:
   RT_E_INVALID). The work table lives in a fixed device array of the
   library (~29.6 MB, held on each device the library runs on until the
   process ends) instead of the growing workspace; the call itself makes no
   hipMalloc, hipFree or other allocation and records no timing events. The
   array is shared by every call on a device and keeps the last call's
   contents (each call clears what it needs), so calls that overlap on one
   device (concurrent streams or threads) race and must be serialized by
   the caller. */
#define RT_NOALLOC_MAX_RAYS 65536
int rt_trace_batch_noalloc(rt_cloak cloak, const rt_trace_opts *opts, int32_t pol, int64_t n,
                           const double *in6, double *out6, double *opl, int32_t *status,
                           double *hres, int32_t *nsteps, double *trans, void *stream);

/* Render n_cams views of the room with the cloak (NULL = empty room) for each
   branch in pol_mask (bit 0 ordinary, bit 1 extraordinary), tracing each
   branch separately (Sect. 4): camera rays, cloak transit as in
   rt_trace_batch, room shading.
     rgb: float32 [n_cams][npol][h][w][3], mean colour over the samples of each
          pixel (npol = popcount(pol_mask), ordinary first); black for absorbed,
          totally reflected, diverged or step-limited samples
     aux: NULL or optional per-sample outputs (see rt_render_aux)
   All cameras must share w, h and spp. Errors as rt_trace_batch. */
int rt_render(rt_cloak cloak, const rt_trace_opts *opts, const rt_room *room,
              const rt_camera *cams, int32_t n_cams, int32_t pol_mask, float *rgb,
              const rt_render_aux *aux, void *stream);

/* Timing of the integrator kernel, for benchmarks. While enabled, every
   launch of the transit integrator is bracketed by HIP events recorded on the
   caller's stream. rt_profile_read waits for the recorded events, returns the
   summed duration (ms) and the number of launches since the last read, and
   forgets them. */
int rt_profile_enable(int32_t on);
int rt_profile_read(double *transit_ms, int64_t *launches);

/* Render the same views for several cloaks in one pass (Fig. 1 vs Fig. 2 of
   the paper: the radial and the azimuthal cloak seen identically), so that
   one integrator launch carries the rays of every (cloak, branch) pair.
   cloaks: n_cloaks (0..2) handles sharing r1, r2, z0, z1 and inner_mirror
   (they may differ in the optic axis); n_cloaks = 0 renders the empty room.
   rgb: float32 [max(n_cloaks,1)][n_cams][npol][h][w][3]; aux arrays follow
   the same [cloak][camera][branch] image order. Otherwise as rt_render;
   RT_E_INVALID if the cloaks' geometries differ. */
int rt_render_multi(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                    const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                    float *rgb, const rt_render_aux *aux, void *stream);

/* Render plan: one batch of views (the arguments of rt_render_multi, fixed
   at creation) recorded once into a HIP graph -- work-table reset, camera-ray
   generation and entry refraction, the hardest-first ordering, the
   persistent integrator, shading and the per-pixel resolve -- and replayed by
   rt_render_plan_launch. The plan owns its device workspace and a copy of the
   cameras; `rgb` and `aux` must stay valid while the plan exists, and every
   launch overwrites them. Launches of one plan must not overlap (each launch
   reuses the plan's workspace). The launch shape is taken from opts, else from
   an earlier rt_autotune_render of the same batch shape, else the defaults.
   Errors: as rt_render_multi, RT_E_DEVICE if capture or instantiation fails. */
int rt_render_plan_create(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                          const rt_room *room, const rt_camera *cams, int32_t n_cams,
                          int32_t pol_mask, float *rgb, const rt_render_aux *aux, rt_plan *out);
int rt_render_plan_launch(rt_plan plan, void *stream);
int rt_render_plan_destroy(rt_plan plan);

/* Autotuner of the integrator's launch shape for a batch: times every block
   size in {64, 128, 256} x refill period in {1, 2, 4, 8, 12, 16} on the batch itself
   (one warm-up and two timed renders each, into `rgb`, which is overwritten),
   writes opts with the fastest shape into `tuned` and its time per render
   into `best_ms` (may be NULL), and remembers the choice for later calls of
   the same batch shape that leave block and refill_period at 0. The shape
   does not change any result (per-ray work is independent of scheduling).
   Synchronous. */
int rt_autotune_render(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                       const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                       float *rgb, rt_trace_opts *tuned, double *best_ms);

/* Descriptor a handle was built from. */
int rt_cloak_get_desc(rt_cloak cloak, rt_cloak_desc *out);

/* ---------------------------------------------------------------------------
   Transit in entry/exit parameters. A ray enters the cloak through its side
   r = r2 at azimuth phi and height z, travelling with horizontal angle alpha
   to the inward normal (positive towards +theta) and elevation beta; it
   leaves (after the transit of rt_trace_batch: Sects. 2-4) on the outgoing
   ray, described at its crossing of r = r2 by azimuth phi', height z',
   horizontal angle alpha' to the outward normal and elevation beta', and T,
   the optical path from the entry point to that crossing (Eqs. (2)/(8) time,
   App. of units: c0 = omega = 1). For a side-to-side transit the wave
   numbers along the surface are conserved (Sect. 3 at both interfaces, and
   p_theta, p_z of the cylindrical metric in between), so alpha' = alpha and
   beta' = beta.
     x6:  float32 SoA 6 x ld (rows 0..n-1 used): phi, z, alpha, beta, the
          branch bit (0 ordinary, 1 extraordinary) and the optic-axis bit
          (0 radial Eq. (14), 1 azimuthal Eq. (15)); |alpha|, |beta| < pi/2
     y5:  float32 SoA 5 x ld: phi' in [0, 2 pi), z', alpha', beta', T
   --------------------------------------------------------------------------- */

/* Exact transit of every ray (or of the rays with mask[i] != 0; the others'
   outputs are left untouched) by the integrator of rt_trace_batch, all
   (axis, branch) pairs in one persistent launch.
   cloaks: 1 or 2 handles with different optic axes sharing r1, r2, z0, z1,
   inner_mirror; a ray whose axis bit has no handle is RT_RAY_INVALID.
   status: n int32 (RT_RAY_*); y5 is NaN for rays that did not leave.
   hres:   n floats or NULL, |v^T M v - 1| at the exit interface (NaN if the
           ray never entered): the integrator's drift from the ray
           Hamiltonian, which grows where it cannot resolve the path (entries
           with p_theta -> 0 pass next to the singular r = r1).
   nsteps: n int32 or NULL. r_out in opts is ignored. Errors as
   rt_trace_batch; n <= 2^28. */
int rt_transit_exact(const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts, int64_t n,
                     int64_t ld, const float *x6, const uint8_t *mask, float *y5, int32_t *status,
                     float *hres, int32_t *nsteps, void *stream);

/* ---------------------------------------------------------------------------
   Learned surrogate of the transit (not part of the paper): an MLP
   6 -> 256 -> 256 -> 256 -> 256 -> 5 with SiLU, layers 2-4 on BF16 matrix
   cores with FP32 accumulation, layers 1 and 5 in FP32. It predicts the
   residuals (t0..t4) of a transit against the closed-form transit of the
   infinite cylinder (dtheta_0, dz_0, T_0), which exists for all four
   (axis, branch) pairs of Eqs. (14)/(15):
     t0 = dtheta - dtheta_0, t1 = (z' - z) - dz_0, t2 = alpha' - alpha,
     t3 = beta' - beta,      t4 = T - T_0,
   where dtheta is the signed azimuth the ray sweeps (sign of alpha). That
   is the side job (RT_SUR_SIDE). A model set to the cap job (RT_SUR_CAP,
   rt_surrogate_set_job) learns instead the side entries of a cloak of
   finite height whose path meets an end cap, for which no closed form is
   built here: with h the entry's distance to the cap it heads for (sign of
   beta) and u = h / |dz_0| (< 1 exactly when the infinite-cylinder path
   rises past that cap), inputs (k_theta, |k_z|, u, alpha, branch, axis)
   and targets the state where the ray leaves the cap plane: the cap
   point's swept azimuth and radius, the radial component of the vacuum
   direction, the optical path to the cap point and the vertical component
   (d_theta = r2 k_theta / r_c follows from the conserved angular momentum),
   as residuals against a chord model of the path (the straight chord with
   the path's turning radius, traversed to rise fraction u, its radial wave
   number from the dispersion relation; exact for the azimuthal cloak's
   extraordinary branch):
     t0 = dtheta_c - frac dtheta_0, t1 = r_c - r_c^chord,
     t2 = d_r - d_r^chord, t3 = T_c - u T_0, t4 = |d_z| - |d_z|^chord;
   the exit on r = r2 is that state plus its straight vacuum leg.
   A model belongs to the device current at its creation; calls on one model
   must not overlap (they share its activation buffers). Arrays are device
   pointers unless stated; n <= 2^24, ld >= n.
   --------------------------------------------------------------------------- */
typedef struct {
    float lr, beta1, beta2, eps, weight_decay;  /* AdamW */
    float huber;  /* loss per element: 0 = squared error; delta > 0 = Huber (quadratic to delta) */
} rt_train_opts;

#define RT_SUR_SIDE 0  /* side-to-side transits, residuals against the closed forms */
#define RT_SUR_CAP 1   /* side entries whose path meets an end cap */

/* Gate of rt_surrogate_infer: a prediction is replaced by the exact transit
   when the entry lies in the near-singular band (p_min) or its cell of the
   trust map is untrusted, and
   side job: when the predicted exit violates the conservation of the
   tangential wave numbers (max(|k_theta' - k_theta|, |k_z' - k_z|)) by more
   than hres_max or the predicted exit height is within cap_margin of an
   end cap;
   cap job: when the entry heads for no cap (u >= 1), the predicted cap
   point lies within cap_margin of the cap's rims r1, r2, the vacuum
   direction has |d_z| < 0.05 (next to total reflection) or a horizontal
   speed below 0.05, or the two estimates of |d_z| (t4, and the
   normalization of (d_r, d_theta)) differ by more than 0.01. */
typedef struct {
    double tol;         /* calibration: largest exit error a trusted cell may show */
    double hres_max;    /* conservation residual limit */
    double cap_margin;  /* exit-height margin from the caps */
    int32_t min_count;  /* calibration rays a cell needs to be trusted */
    int32_t dilate;     /* also distrust cells within this many cells (same axis and branch) of an untrusted one */
    double unresolved;  /* calibration: exits whose exact transit drifted by |H - 1| > this are no reference */
    double p_min;       /* near-singular band: entries whose conserved wave number (k_theta for the
                           azimuthal cloak's extraordinary branch, |(k_theta, k_z)| for the radial
                           extraordinary and azimuthal ordinary branches) is below p_min pass within
                           ~p_min of r = r1, where the integrator itself does not resolve the path;
                           they are traced exactly (0 = no band) */
} rt_gate_opts;

/* New model with weights and biases uniform in +-1/sqrt(fan_in) (seeded),
   identity scaling and no trusted cells. */
int rt_surrogate_create(uint64_t seed, rt_model *out);
int rt_surrogate_free(rt_model model);
int rt_surrogate_nparams(int64_t *count);  /* 200,453 */
/* FP32 parameters in host memory: W1 [6][256], b1, W2 [256][256], b2, W3,
   b3, W4, b4, W5 [256][5], b5, each weight (fan_in, fan_out) row-major.
   set_params also resets the optimizer state. Synchronous. */
int rt_surrogate_get_params(rt_model model, float *host);
int rt_surrogate_set_params(rt_model model, const float *host);
/* Standardization (host, 22 floats): in_off[6], in_scale[6] (input k enters
   as (x_k - in_off_k) in_scale_k), out_mean[5], out_std[5] (the network's
   output o is (t_o - out_mean_o) / out_std_o). Synchronous. */
int rt_surrogate_get_scaling(rt_model model, float *scaling22);
int rt_surrogate_set_scaling(rt_model model, const float *scaling22);
/* Set the standardization from the weighted moments of x6 and t5 (rows
   with w = 0 ignored, w NULL = all ones); out_std is floored at 1e-3.
   Synchronous. */
int rt_surrogate_fit_scaling(rt_model model, int64_t n, int64_t ld, const float *x6, const float *t5,
                             const float *w, void *stream);
/* Training targets of transits: t5 (SoA 5 x ld) from the entries x6 and the
   exact exits y5/status of rt_transit_exact; w[i] = 1 for a finished
   side-to-side transit, 0 otherwise (its t5 entries are 0). */
int rt_surrogate_encode(const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld, const float *x6,
                        const float *y5, const int32_t *status, float *t5, float *w, void *stream);
/* Targets of either job (job RT_SUR_SIDE is rt_surrogate_encode). Cap job:
   w[i] = 1 for an entry inside the material's height range that leaves
   through the cap it heads for (u < 1), 0 otherwise; the cloaks must have
   finite height (RT_E_INVALID). */
int rt_surrogate_encode_job(int32_t job, const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld,
                            const float *x6, const float *y5, const int32_t *status, float *t5, float *w,
                            void *stream);
/* Set a model's job (RT_SUR_SIDE or RT_SUR_CAP); the cap job takes the
   geometry (r1, r2, z0, z1, finite height) of `cloak` (ignored for the side
   job, may be NULL), and calibration and inference then need cloaks of that
   geometry (RT_E_INVALID otherwise). Clears the trust map. New models have
   the side job. */
int rt_surrogate_set_job(rt_model model, int32_t job, rt_cloak cloak);
int rt_surrogate_get_job(rt_model model, int32_t *job);
/* Chain two models: rt_surrogate_infer and rt_render_surrogate with `first`
   offer the rows that first's gate rejects to `next` (its own gate and
   trust map), and the exact integrator traces what both reject. A chain
   holds two models; next = NULL unchains. Neither owns the other:
   rt_surrogate_free of either unchains them. Both must be calibrated before
   inference. The chain's exit tolerance (the tile-edge gate) is the larger
   of the two calibrations' tol. */
int rt_surrogate_chain(rt_model first, rt_model next);
/* Loss L = (1/n) sum_i w_i sum_o rho(y_io - (t_io - out_mean_o)/out_std_o)
   of one batch (w NULL = all ones) and its gradient, rho(d) = d^2, or for
   huber = delta > 0 the Huber function (d^2 up to |d| = delta, then
   2 delta |d| - delta^2). grads: NPARAM floats (device, same layout as
   get_params) or NULL; loss: 1 float (device) or NULL. */
int rt_surrogate_grad(rt_model model, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w,
                      float huber, float *grads, float *loss, void *stream);
/* One AdamW step on a batch: the gradient of rt_surrogate_grad, then, per
   parameter p with gradient g, FP32 first and second moments
   m <- beta1 m + (1 - beta1) g, v <- beta2 v + (1 - beta2) g^2, decoupled
   weight decay p <- p - lr weight_decay p on the weights (not the biases),
   and p <- p - lr (m / c1) / (sqrt(v / c2) + eps) with the bias corrections
   c1 = 1 - beta1^t, c2 = 1 - beta2^t of step t; the BF16 copies of W2..W4
   follow. */
int rt_surrogate_train(rt_model model, int64_t n, int64_t ld, const float *x6, const float *t5, const float *w,
                       const rt_train_opts *opts, float *loss, void *stream);
/* One AdamW step (as in rt_surrogate_train) with a gradient the caller
   supplies: grads, NPARAM floats (device, the layout of get_params).
   Errors: RT_E_INVALID for NULL grads or bad options. */
int rt_surrogate_step(rt_model model, const float *grads, const rt_train_opts *opts, void *stream);
/* Optimizer state in host memory: the AdamW first and second moments
   (NPARAM floats each, the layout of get_params; either pointer may be NULL
   in get_state) and the number of steps taken, which sets the bias
   corrections 1 - beta^step of the next step. set_state needs finite m and
   finite v >= 0, step >= 0. Synchronous. */
int rt_surrogate_get_state(rt_model model, float *m_host, float *v_host, int64_t *step);
int rt_surrogate_set_state(rt_model model, const float *m_host, const float *v_host, int64_t step);
/* Network prediction of the targets, de-standardized: t5 SoA 5 x ld. */
int rt_surrogate_forward(rt_model model, int64_t n, int64_t ld, const float *x6, float *t5, void *stream);
/* Build the trust map: predicts the calibration rays x6, measures each
   one's exit error max(|x - x_exact| / r2, angle(d, d_exact)) against the
   exact exits, and trusts a cell when it holds >= min_count rays, all of
   them finished transits with error <= tol, and no cell within `dilate`
   cells of it (in alpha and beta, and u for the cap job) fails that test
   (discontinuities of the transit run along thin curves that a cell's
   calibration rays can miss). The cap job counts only the rays its gate
   would predict (heading for a cap, a usable cap exit; see rt_gate_opts).
   hres_exact (n floats from rt_transit_exact, or NULL): exits with
   hres_exact > gate->unresolved (> 0) are left out, neither counted nor
   failing, since the integrator did not resolve them; with hres_exact and
   cloaks of infinite height, so are totally reflected exits (a side entry
   of the infinite cylinder conserves its tangential wave numbers and always
   transmits at its exit; the status only arises from the integrator's
   drift at grazing entries). Stores `gate` in the model.
   trusted_fraction (host, may be NULL): share of trusted cells.
   Synchronous. */
int rt_surrogate_calibrate(rt_model model, const rt_cloak *cloaks, int32_t n_cloaks, int64_t n, int64_t ld,
                           const float *x6, const float *y5_exact, const int32_t *status_exact,
                           const float *hres_exact, const rt_gate_opts *gate, double *trusted_fraction,
                           void *stream);
/* Trust map (host, 4 x cells_alpha x cells_beta x cells_u bytes,
   (axis*2+branch) major): side job uniform cells over (alpha, beta) in
   (-pi/2, pi/2)^2 (cells_u = 1), cap job over alpha in (-pi/2, pi/2),
   |beta| in [0, pi/2) and u in [0, 1). host and the counts may be NULL. */
int rt_surrogate_get_map(rt_model model, uint8_t *host, int32_t *cells_alpha, int32_t *cells_beta,
                         int32_t *cells_u);
/* Surrogate transit with exact fallback: y5/status as rt_transit_exact.
   fallback[i] (n bytes) = 1 where the gate rejected the prediction and the
   exact integrator traced the ray, 0 where y5 is the network's. Needs a
   calibrated model. */
int rt_surrogate_infer(rt_model model, const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                       int64_t n, int64_t ld, const float *x6, float *y5, uint8_t *fallback, int32_t *status,
                       void *stream);
/* Render as rt_render_multi, with the side-to-side transits taken from the
   surrogate where its gate accepts them (not part of the paper): a camera
   sample that refracts into the cloak through its side r = r2 with
   difficulty >= min_difficulty is offered to the network, whose accepted
   prediction gives the exit ray on r = r2 and, after its vacuum leg, the
   sample's colour; rejected side entries, easier side entries and the
   entries through the end caps are traced by the integrator, in one launch
   per chunk. The difficulty is the integrator's ordering key: -log2 of the
   conserved wave number p (p_theta / r2 for the azimuthal cloak's
   extraordinary branch, |(p_theta / r2, p_z)| otherwise), as the bucket
   floor(-log2 p) + 1 clamped to [0, 15], and 0 for the radial cloak's
   ordinary branch; paths with small p pass close to r = r1, where the steps
   shrink, so the bucket tracks the integration cost, while the network
   costs the same for every ray. min_difficulty = 0 offers every side entry.
   The exit error of an accepted ray is what the model's calibration bounds
   (tol of rt_surrogate_calibrate, in r2 units and radians); it moves the
   room point along its face by at most tol (r2 + L) / cos(theta) for a
   vacuum leg of length L meeting the face at angle theta to its normal. An
   accepted prediction whose room point lies within twice that distance of
   a tile edge or face boundary is traced by the integrator instead (tile-
   edge gate), so every sample takes the plain render's colour wherever the
   calibration bound holds.
     model:  a calibrated model on the current device
     min_difficulty: in [0, 16] (16 offers nothing)
     counts: host int64[2] or NULL: side entries offered to the network and
             entries whose prediction was accepted (summed over the chunks;
             needs one more synchronization per chunk)
   Synchronizes the stream once per chunk of samples (the network's launch
   is sized by the number of side entries). Candidate rows take 61 bytes per
   (sample, cloak, branch) of a chunk on top of rt_render_multi's workspace.
   Errors: as rt_render_multi; RT_E_INVALID for a NULL model, n_cloaks < 1,
   min_difficulty outside [0, 16] or an uncalibrated model. */
int rt_render_surrogate(rt_model model, const rt_cloak *cloaks, int32_t n_cloaks, const rt_trace_opts *opts,
                        const rt_room *room, const rt_camera *cams, int32_t n_cams, int32_t pol_mask,
                        int32_t min_difficulty, float *rgb, const rt_render_aux *aux, int64_t *counts,
                        void *stream);

/* Model file: parameters, scaling, gate, trust map, job and geometry. */
int rt_surrogate_save(rt_model model, const char *path);
int rt_surrogate_load(const char *path, rt_model *out);

/* Release the library's device workspace (synchronizes the device first). */
int rt_release_workspace(void);

/* Message of the last failed call on this thread ("" if none). */
const char *rt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RT_H */
