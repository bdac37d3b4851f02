/*
 * kerrtrace.h -- C ABI of the MI355X (gfx950) Kerr backward ray tracer.
 *
 * One null geodesic per image pixel is integrated backward from the observer
 * (Velasquez-Cadavid et al., "OSIRIS", Sect. 2.2) with Hamilton's equations
 * in Boyer-Lindquist Kerr coordinates (eq:edm, eq:ligH, eq:Kerr) while the
 * constraint H = 0 is tracked (Sect. 3.1).  Each ray ends on the horizon, on
 * a thin equatorial disk or on escape (Sect. 4.1, Sect. 5).
 *
 * Conventions
 *   - Geometrized units; M is a parameter (the paper sets M = 1, Sect. 1);
 *     M = 0 (with a = 0) is flat space, the reference image of Sect. 4.2.
 *   - The observer sits at (r_obs, theta_0 = incl, phi_0 = 0).  Pixel (i, j)
 *     has image-plane centre x = -fov_x + (i + 1/2) 2 fov_x / nx,
 *     y = -fov_y + (j + 1/2) 2 fov_y / ny (image plane of Sect. 2.3) and
 *     row-major index j*nx + i.
 *   - Initial momenta follow the second eq:momentums (Sect. 2.3) with p_r < 0
 *     (ingoing), E = -p_t, L = p_phi.
 *   - Every array is a DEVICE pointer into memory the caller owns.  The
 *     library allocates nothing and frees nothing.  Work is enqueued on
 *     hip_stream (a hipStream_t; NULL means the null stream) and the call
 *     returns without waiting; outputs are valid once the stream has been
 *     synchronised.  Structs are read during the call only.
 *   - Calls on one GPU that share a workspace must not overlap.
 *
 * Errors: every int-returning call returns KT_OK or a negative code and
 * leaves a message for kt_last_error().  Per-ray problems are never errors:
 * they become fate codes.
 */
#ifndef KERRTRACE_H
#define KERRTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KT_VERSION_NUMBER 203

/* return codes */
#define KT_OK 0
#define KT_EINVAL (-1)   /* an argument is out of range, non-finite or NULL */
#define KT_EDEVICE (-2)  /* a HIP call or kernel launch failed */
#define KT_ENOMEM (-3)   /* the workspace is smaller than kt_workspace_bytes() */

/* per-ray fate codes (uint8 per pixel) */
#define KT_FATE_ESCAPED 0   /* r > r_escape (celestial sphere r_cs, Sect. 4.1) */
#define KT_FATE_CAPTURED 1  /* r < r_H + capture_buffer (Sect. 4.1) */
#define KT_FATE_DISK 2      /* hit the disk between r_in and r_out (Sect. 5) */
#define KT_FATE_MAXSTEPS 3  /* step budget exhausted */
#define KT_FATE_STEPFAIL 4  /* step size underflow or non-finite state */
#define KT_FATE_INVALID 5   /* x^2 + y^2 >= r_obs^2: no real p_r */

/* integrators */
#define KT_RK4_S 0  /* classic RK4, fixed step h_fixed in s, d(lambda)/ds = Delta/r */
#define KT_DP45 1   /* Dormand-Prince 5(4), adaptive, FSAL (Sect. 3.1) */
#define KT_RKF45 2  /* Runge-Kutta-Fehlberg 4(5), adaptive, 4th order propagated (Sect. 3.1) */
#define KT_CK45 3   /* Cash-Karp 5(4), adaptive, 5th order propagated (Sect. 3.1) */
#define KT_BS 4     /* Bulirsch-Stoer: modified midpoint with 2, 4, .., 10 substeps,
                       Aitken-Neville (polynomial) extrapolation (order 10), adaptive (Sect. 3.1) */
#define KT_BS_RAT 5 /* Bulirsch-Stoer as KT_BS with rational-function extrapolation
                       (the Stoer-Bulirsch recursion, Sect. 3.1) */

/* arithmetic of the RHS */
#define KT_FP64 0
#define KT_MIXED 1  /* FP32 mass-dependent RHS part for r >= r_switch, FP64 re-run
                       of every ray whose max |H|_rel exceeds h_budget */

/* Observer and image plane (Sect. 2.3). */
typedef struct kt_camera {
    double r_obs;   /* observer radius, > r_H + capture_buffer */
    double incl;    /* theta_0 in (0, pi), radians */
    double fov_x;   /* half-width of the image plane, > 0 */
    double fov_y;   /* half-height, > 0 */
    int32_t nx, ny; /* resolution, >= 1 each, nx*ny < 2^31 */
} kt_camera;

/* The spacetime.  KT_METRIC_KERR: Kerr (eq:Kerr), mass M >= 0, spin |a| <= M.
   KT_METRIC_Q: the q-metric of the appendix (eq:q-metric, taken with
   signature (-,+,+,+)), a static axisymmetric vacuum with parameter M (its
   mass is M (1 + q)) and quadrupole parameter q > -1, a = 0; rays are
   captured at r < 2M + capture_buffer.  The q-metric runs single images
   (not kt_render_batch) with the adaptive FP64 schemes, without a disk
   (its redshift model is Kerr's), and is not differentiated by kt_adjoint. */
#define KT_METRIC_KERR 0
#define KT_METRIC_Q 1
typedef struct kt_spacetime {
    double M, a;
    int32_t metric;
    double q;
} kt_spacetime;

/* Thin equatorial disk (Sect. 5). Emissivity (M/r)^emis_index.  Circular
   orbits rotate with the prograde Keplerian Omega = sqrt(M)/(r^1.5 + a sqrt(M))
   (rotation = KT_ROT_KEPLER) or with constant specific angular momentum
   l0 = -u_phi/u_t, Omega = -(g_tphi + l0 g_tt)/(g_phiphi + l0 g_tphi)
   (rotation = KT_ROT_L0).  Where the orbit is not timelike, g is NaN and the
   intensity 0. */
#define KT_ROT_KEPLER 0
#define KT_ROT_L0 1
/* emissivity models */
#define KT_EMIS_POWER 0     /* I_em = (M/r)^emis_index */
#define KT_EMIS_TAPERED 1   /* I_em = (M/r)^2 (1 - sqrt(r_in/r)), times 3s^2 - 2s^3 with
                               s = (r_out - r)/(2M) on [r_out - 2M, r_out]: continuous in
                               r_in and r_out, so the image is differentiable in r_in */
typedef struct kt_disk {
    int32_t enabled;
    double r_in, r_out, emis_index;
    int32_t rotation;       /* KT_ROT_KEPLER or KT_ROT_L0 */
    double l0;              /* specific angular momentum for KT_ROT_L0 */
    int32_t emissivity;     /* KT_EMIS_POWER or KT_EMIS_TAPERED */
} kt_disk;

/* Light sources.  A point source at (r_src, pi - incl, pi), behind the hole:
   deflection diagnostics for Einstein rings (Sect. 4.3).  The coloured
   celestial sphere r = r_escape of Sect. 4.1: with sky set, the crossing of
   the sphere is located exactly (theta_f, phi_f are its coordinates) and
   classified into KT_SKY_* codes: four quadrants and a graticule of lines
   every grid_deg degrees (0: none) of half-width line_deg. */
typedef struct kt_source {
    int32_t enabled;
    double r_src;
    int32_t sky;
    double grid_deg, line_deg;
} kt_source;

/* celestial-sphere codes (uint8 per pixel) */
#define KT_SKY_NONE 0    /* did not reach the sphere (captured, disk, failed) */
#define KT_SKY_GREEN 1   /* 0 <= theta < pi/2, 0 <= phi < pi */
#define KT_SKY_RED 2     /* 0 <= theta < pi/2, pi <= phi < 2 pi */
#define KT_SKY_BLUE 3    /* pi/2 <= theta <= pi, 0 <= phi < pi */
#define KT_SKY_YELLOW 4  /* pi/2 <= theta <= pi, pi <= phi < 2 pi */
#define KT_SKY_LINE 5    /* on a graticule line */

typedef struct kt_integrator {
    int32_t method;         /* KT_RK4_S, KT_DP45, KT_RKF45, KT_CK45, KT_BS or KT_BS_RAT */
    int32_t precision;      /* KT_FP64 or KT_MIXED */
    double h_fixed;         /* RK4_S step in s, > 0 */
    double rtol, atol;      /* tolerances of the adaptive methods, > 0 */
    double h_init;          /* first trial step in lambda of the adaptive methods, > 0 */
    double capture_buffer;  /* delta_r of Sect. 4.1, >= 0 */
    double r_escape;        /* r_cs; 0 selects 1.1 r_obs */
    double h_budget;        /* MIXED: re-run in FP64 when max |H|_rel > h_budget */
    double r_switch;        /* MIXED: FP32 RHS part only where r >= r_switch */
    int64_t max_steps;      /* accepted-step budget per ray, >= 1 */
    int32_t checkpoint_every; /* kt_adjoint: a checkpoint every this many accepted
                                 steps, a power of two in [1, 1024]; 0 selects 64.
                                 1 stores every step (no recomputation in the
                                 backward sweep; the largest workspace).
                                 Renders ignore it (but reject other values) */
    int32_t split_above;    /* kt_adjoint with the forward step counts: a ray whose
                               forward render took more than this many accepted
                               steps has its backward sweep split into 64-step
                               segments swept on separate lanes; 0 picks the
                               threshold from the work list, -1 never splits
                               (and leaves the split buffers out of the
                               workspace).  Renders ignore it (but reject values
                               below -1) */
} kt_integrator;

/* Launch shape.  Pass NULL for the defaults: persistent, block 256,
   blocks_per_cu 0, batch 4, KT_ORDER_RING.  In a persistent launch each
   wave's first fetch from the ticket takes 64 ids (one per lane); batch
   applies to the fetches after it.
   The trace kernels exist in two builds with bit-identical outputs: one for
   2 waves per SIMD and one for 3 (fewer registers, a few more instructions
   per step).  A persistent launch runs the 3-wave build when its shape asks
   for 3 or more waves per SIMD (blocks_per_cu * block >= 768), or, with
   blocks_per_cu 0, when the render has at least 4 rays per lane of a
   3-wave grid (about 790k rays on 256 CUs); then blocks_per_cu 0 means the
   3-wave build's occupancy.  Other launches run the 2-wave build. */
typedef struct kt_launch {
    int32_t persistent;     /* 1: persistent waves refill lanes from a global ticket;
                               0: one ray per lane, no refill */
    int32_t block;          /* threads per workgroup: 64, 128 or 256 */
    int32_t blocks_per_cu;  /* persistent grid = CUs * blocks_per_cu; 0 = occupancy */
    int32_t batch;          /* ray ids taken per ticket fetch after a wave's first, 1..4096 */
    int32_t order;          /* KT_ORDER_RING (0) or KT_ORDER_ROWS: the order rays go out in */
} kt_launch;

/* Dispatch order.  Outputs are identical under both; only the time differs.
   KT_ORDER_RING sends rays out by their image-plane distance from the
   photon ring (nearest first: they take the most steps), sorted on the
   device at the start of each render; KT_ORDER_ROWS sends pixel ids in
   row-major order. */
#define KT_ORDER_RING 0
#define KT_ORDER_ROWS 1

/* Launch statistics (device memory, written at the end of a render). */
typedef struct kt_stats {
    uint64_t rays;           /* nx * ny */
    uint64_t evals;          /* all RHS evaluations, both passes */
    uint64_t evals_fp32;     /* evaluations whose mass term ran in FP32 */
    uint64_t fallback_rays;  /* MIXED: rays re-run in FP64 */
    uint64_t fate_count[8];  /* histogram of final fates */
    double trace_ms;         /* milliseconds the trace launches took: between two readings
                                of the GPU's constant-rate wall clock, enqueued on the
                                render's stream just before the first trace kernel and
                                just after the last (both passes of a MIXED render and
                                the list compaction between them); 0 if the device
                                reports no rate.  Taken on the device, so no host
                                synchronisation; the readings are only enqueued when
                                stats is set */
} kt_stats;

/* Per-pixel outputs: device arrays of nx*ny entries, row-major j*nx + i.
   Any pointer except fate may be NULL (that output is skipped).
   Values that do not apply to a ray are NaN (r_hit, g, psi, deflection) or
   0 (intensity, ring). */
typedef struct kt_outputs {
    uint8_t *fate;
    double *r_hit;       /* disk hit radius */
    double *g;           /* redshift nu_obs/nu_em at the disk (eq:redshift) */
    double *intensity;   /* g^3 I_em, I_em = (M/r_hit)^emis_index */
    double *max_abs_h;   /* max |H| over accepted states (Error of Sect. 3.1) */
    double *max_rel_h;   /* max |2 Sigma H| / D, D = sum of |terms| of 2 Sigma H */
    double *psi;         /* source: angle between ray and source direction at r_src */
    double *deflection;  /* source: swept angle from the observer to r_src */
    double *theta_f, *phi_f;  /* final (or disk-crossing) angles */
    uint8_t *n_cross;    /* equatorial crossings outside the disk before the end */
    uint8_t *used_fp64;  /* MIXED: 1 when the ray was re-run in FP64 */
    uint8_t *ring;       /* source: an odd multiple of pi lies between this pixel's
                            deflection and its +i or +j neighbour's */
    int32_t *n_steps;    /* accepted steps */
    int32_t *n_evals;    /* RHS evaluations */
    uint8_t *sky;        /* KT_SKY_* code (KT_SKY_NONE where the source's sky is off);
                            needs theta_f and phi_f */
    kt_stats *stats;     /* may be NULL */
} kt_outputs;

/* Render one image.  disk and source may be NULL (disabled).  workspace is a
   device buffer of at least kt_workspace_bytes(camera, integ) bytes, aligned
   to 256 bytes; its contents on entry do not matter.
   Returns KT_OK, KT_EINVAL, KT_ENOMEM or KT_EDEVICE. */
int kt_render(const kt_camera *camera, const kt_spacetime *spacetime, const kt_disk *disk,
              const kt_source *source, const kt_integrator *integ, const kt_outputs *out,
              void *workspace, size_t workspace_bytes, void *hip_stream);

/* kt_render with an explicit launch shape (NULL = defaults).  With KT_FP64
   the per-ray arithmetic does not depend on the launch shape: outputs are
   bit-identical for every valid shape.  With KT_MIXED the FP32 part runs
   only while every stepping lane of a wave is beyond r_switch, so which
   rays use it depends on how rays share waves; every result still meets
   h_budget or comes from the FP64 re-run. */
int kt_render_ex(const kt_camera *camera, const kt_spacetime *spacetime, const kt_disk *disk,
                 const kt_source *source, const kt_integrator *integ, const kt_outputs *out,
                 void *workspace, size_t workspace_bytes, void *hip_stream,
                 const kt_launch *launch);

/* Workspace size in bytes for this camera and integrator (0 on bad input). */
size_t kt_workspace_bytes(const kt_camera *camera, const kt_integrator *integ);

/* For callers that cannot allocate device memory -- code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation:
   kt_render_ex with the library's own scratch array of
   KT_NOALLOC_SCRATCH_BYTES in place of the workspace argument.  It calls no
   allocating routine.  The array is a file-scope device array: each GPU the
   library runs on holds one copy until the process ends.  The caller still
   owns and passes every output.
   Limit: renders whose kt_workspace_bytes() exceeds KT_NOALLOC_SCRATCH_BYTES
   (about 4.7M FP64 rays, 3.5M with KT_MIXED; a 2048^2 FP64 image fits)
   return KT_ENOMEM with a message, before any device work.
   Every call on one GPU shares that GPU's array and leaves its contents
   behind (the render clears what must start at zero with its own kernels):
   calls that overlap on one GPU -- from two host threads, or on two streams
   without ordering between them -- race.  Other arguments, results and
   errors as for kt_render_ex. */
#define KT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int kt_render_noalloc(const kt_camera *camera, const kt_spacetime *spacetime, const kt_disk *disk,
                      const kt_source *source, const kt_integrator *integ, const kt_outputs *out,
                      void *hip_stream, const kt_launch *launch);

/* One image of a batch: its own camera, spacetime, disk and source.  Disk
   and source are disabled with enabled = 0. */
typedef struct kt_image {
    kt_camera camera;
    kt_spacetime spacetime;
    kt_disk disk;
    kt_source source;
} kt_image;

#define KT_MAX_IMAGES 4096

/* Render n_images images of any sizes, spins, inclinations and distances in
   one persistent launch (the rays of all images share one ticket, so short
   and long images balance each other out).  The images' outputs are
   concatenated in table order: image k occupies entries
   [first_k, first_k + nx_k*ny_k) of every output array, first_k being the
   sum of nx*ny over the images before it; the total must be < 2^31.
   n_images lies in [1, KT_MAX_IMAGES].  integ is shared by all images
   (r_escape = 0 selects 1.1 r_obs per image).  Requesting ring needs every
   image's source enabled.  workspace: at least
   kt_workspace_bytes_batch(n_images, images, integ) bytes, 256-byte aligned.
   With KT_FP64 each image's outputs are bit-identical to a kt_render_ex of
   that image alone with the same integrator; launch may be NULL (defaults).
   The table is read during the call only.
   Returns KT_OK, KT_EINVAL (naming the offending image), KT_ENOMEM or
   KT_EDEVICE. */
int kt_render_batch(int32_t n_images, const kt_image *images, const kt_integrator *integ,
                    const kt_outputs *out, void *workspace, size_t workspace_bytes,
                    void *hip_stream, const kt_launch *launch);

/* Workspace size in bytes for kt_render_batch (0 on bad input, including a
   total of 2^31 rays or more). */
size_t kt_workspace_bytes_batch(int32_t n_images, const kt_image *images,
                                const kt_integrator *integ);

#define KT_AUTOTUNE_DEFAULT_COUNT 30

/* Launch-shape autotuner.  Renders the batch (the probe workload: pass a
   representative subset of a large batch to keep this short) once untimed
   and then `repeats` times with every candidate shape, timing each with HIP
   events on hip_stream, and writes the fastest candidate to *best.  Waves
   per SIMD are chosen through blocks_per_cu (blocks_per_cu * block / 256
   waves per SIMD).  candidates == NULL with n_candidates == 0 selects the
   built-in set of KT_AUTOTUNE_DEFAULT_COUNT shapes: persistent, block
   {128, 256} x 1, 2 or 3 waves per SIMD x ticket batch {4, 8, 16, 32, 64}.
   times_ms (may be NULL) receives the mean milliseconds per render of each
   candidate, in order.  Synchronises hip_stream; the outputs hold the last
   render's results.  repeats lies in [1, 100].  Other arguments as for
   kt_render_batch (n_images = 1 tunes a single image).
   Returns KT_OK, KT_EINVAL, KT_ENOMEM or KT_EDEVICE. */
int kt_autotune_batch(int32_t n_images, const kt_image *images, const kt_integrator *integ,
                      const kt_outputs *out, void *workspace, size_t workspace_bytes,
                      void *hip_stream, const kt_launch *candidates, int32_t n_candidates,
                      int32_t repeats, kt_launch *best, float *times_ms);

/* Gradient of a disk image with respect to the spin a, the inclination and
   the disk's inner radius r_in: the discrete adjoint of the rendered
   intensity (Sect. 5 observables, eq:redshift) through the Dormand-Prince
   integration with its accepted step sizes frozen.  For each pixel with
   fate KT_FATE_DISK and cot_intensity != 0 it writes
   cot_intensity * dI/d(a, incl, r_in) to grad_a, grad_incl, grad_r_in
   (device, nx*ny doubles each, any may be NULL; 0 elsewhere).
   grad_sum (device, 3 doubles, may be NULL) receives the sums of the three
   maps over the image: with cot_intensity = dLoss/dI that is the loss's
   gradient in (a, incl, r_in).  The sums are taken in a fixed order (a
   block-then-grid tree over pixel ids), so they are bit-identical from run
   to run whatever lanes ran the rays.
   Inputs: the same camera, spacetime, disk and integrator as the forward
   kt_render (method KT_DP45, KT_FP64, disk enabled), and that render's fate
   array, its r_hit array (optional, for a bit-identity check) and its
   n_steps array (optional: the differentiated rays are run longest first
   and neighbouring lanes get rays of similar length, and long rays can be
   split, below).  Each ray is re-integrated with the forward's own
   arithmetic, checkpointed every integ->checkpoint_every accepted steps (64
   when 0), and swept backward segment by segment, each segment recomputed
   from its checkpoint; with checkpoint_every 1 every accepted step is
   stored and the sweep reads them instead (same gradients bit for bit).
   Split sweeps (n_steps given, integ->split_above >= 0): a ray whose
   forward took more than split_above accepted steps (0: 0.85 times the mean
   number of steps per lane of the work list, at least 128; the longest rays
   first, whole step-count bins of 4 steps at a time, as many as fit 8192
   records and a store of 32 steps per lane of the grid; rays of more than
   2046 steps are not split) stores every step, and the transposed Jacobian
   of each 64-step segment is
   swept on four lanes at once, one per basis cotangent of (r, theta, p_r,
   p_theta) (that of phi stays zero: the field does not depend on phi); the
   segments' maps are then applied in order to the ray's cotangent.  This
   cuts the sequential length of the longest rays, which otherwise set the
   adjoint's run time.  Split rays' gradients equal the sequential sweep's
   up to rounding (the same products, associated differently); they do not
   depend on checkpoint_every.
   stats (device, 4 uint64, may be NULL): rays differentiated, rays that
   failed, rays beyond the checkpoint capacity (max(256, 2048 /
   checkpoint_every) checkpoints, i.e. at least 2048 accepted steps and
   256 * checkpoint_every from 8 on), rays whose re-integration did not
   reproduce r_hit; the last three get zero gradient and drop out of
   grad_sum, so a caller that needs the whole gradient checks them.
   workspace: kt_adjoint_workspace_bytes() bytes, 256-byte aligned.
   Returns KT_OK, KT_EINVAL, KT_ENOMEM or KT_EDEVICE. */
int kt_adjoint(const kt_camera *camera, const kt_spacetime *spacetime, const kt_disk *disk,
               const kt_integrator *integ, const uint8_t *fate, const double *r_hit,
               const int32_t *n_steps, const double *cot_intensity, double *grad_a,
               double *grad_incl, double *grad_r_in, double *grad_sum, uint64_t *stats,
               void *workspace, size_t workspace_bytes, void *hip_stream);

/* Workspace size of kt_adjoint for this camera and integrator (0 on bad input). */
size_t kt_adjoint_workspace_bytes(const kt_camera *camera, const kt_integrator *integ);

/* Initial state of every pixel (Sect. 2.3), for checking the camera alone:
   state is a device array of 7*nx*ny doubles laid out SoA as
   [r | theta | phi | p_r | p_theta | E | L], each block nx*ny long;
   invalid (device, nx*ny bytes) is 1 where x^2 + y^2 >= r_obs^2. */
int kt_init_rays(const kt_camera *camera, const kt_spacetime *spacetime, double *state,
                 uint8_t *invalid, void *hip_stream);

/* Message of the last failed call on this host thread ("" if none). */
const char *kt_last_error(void);

/* KT_VERSION_NUMBER of the built library. */
int kt_version(void);

#ifdef __cplusplus
}
#endif
#endif
