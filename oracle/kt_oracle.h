/*
 * kt_oracle.h -- plain FP64 CPU oracle for backward ray tracing of null
 * geodesics in Kerr spacetime (Boyer-Lindquist coordinates, Hamiltonian form).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or helper with the GPU
 * path and includes nothing from it.
 *
 * Conventions (Velasquez-Cadavid et al., "OSIRIS", EPJC):
 *   signature (-,+,+,+), geometrized units (Sect. 1, last paragraph);
 *   coordinates {t, r, theta, phi}; momenta p_mu covariant;
 *   E = -p_t and L = p_phi are constants of motion (Sect. 2.1).
 *
 * Every function is re-entrant; the image drivers are OpenMP-parallel over
 * pixels with schedule(dynamic, 64).
 */
#ifndef KT_ORACLE_H
#define KT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* fate codes */
#define KO_ESCAPED 0
#define KO_CAPTURED 1
#define KO_DISK 2
#define KO_MAXSTEPS 3
#define KO_STEPFAIL 4
#define KO_INVALID 5

/* spacetimes */
#define KO_KERR 0
#define KO_QMETRIC 1 /* the appendix's q-metric; M is its m, the mass is m (1 + q) */

/* integrators */
#define KO_RK4_S 0 /* classic RK4, fixed step in s with d(lambda)/ds = Delta/r */
#define KO_DP45 1  /* Dormand-Prince 5(4), adaptive, FSAL */
#define KO_RKF45 2 /* Runge-Kutta-Fehlberg 4(5), adaptive, 4th order propagated */
#define KO_CK45 3  /* Cash-Karp 5(4), adaptive, 5th order propagated */
#define KO_BS 4    /* Bulirsch-Stoer: modified midpoint n = 2,4,..,10, polynomial extrapolation (order 10) */
#define KO_BS_RAT 5 /* Bulirsch-Stoer with rational-function extrapolation (Bulirsch & Stoer 1966) */

typedef struct {
    /* spacetime: Kerr (M, a) or the q-metric (M, q) */
    double M, a;
    int32_t metric;
    double q;
    /* camera: observer at (r_obs, theta0 = incl, phi0 = 0); image plane
       [-fov_x, fov_x] x [-fov_y, fov_y] sampled at nx x ny pixel centres */
    double r_obs, incl, fov_x, fov_y;
    int32_t nx, ny;
    /* integrator */
    int32_t method;
    double h_fixed;      /* RK4_S step in s */
    double rtol, atol;   /* tolerances of the adaptive methods */
    double h_init;       /* first trial step in lambda of the adaptive methods */
    double cap_buffer;   /* delta_r: captured when r < r_+ + cap_buffer */
    double r_escape;     /* escaped when r > r_escape */
    int64_t max_steps;   /* accepted-step cap */
    /* thin equatorial disk; rotation 0: prograde Keplerian, 1: constant
       specific angular momentum l0 (Sect. 5) */
    int32_t disk_on;
    double r_in, r_out, emis_q;
    int32_t rotation;
    double l0;
    /* emissivity: 0 (M/r)^emis_q; 1 (M/r)^2 (1 - sqrt(r_in/r)) tapered to 0
       over [r_out - 2M, r_out] by the smoothstep 3s^2 - 2s^3 */
    int32_t emis_model;
    /* point source for the deflection diagnostics */
    int32_t src_on;
    double r_src;
    /* celestial sphere at r_escape (Sect. 4.1): when sky_on, the crossing
       of r = r_escape is located and classified into the four coloured
       quadrants and the graticule of lines every grid_deg degrees with
       half-width line_deg */
    int32_t sky_on;
    double grid_deg, line_deg;
} ko_setup;

/* sky codes */
#define KO_SKY_NONE 0   /* the ray did not reach the celestial sphere */
#define KO_SKY_GREEN 1  /* 0 <= theta < pi/2, 0 <= phi < pi */
#define KO_SKY_RED 2    /* 0 <= theta < pi/2, pi <= phi < 2 pi */
#define KO_SKY_BLUE 3   /* pi/2 <= theta <= pi, 0 <= phi < pi */
#define KO_SKY_YELLOW 4 /* pi/2 <= theta <= pi, pi <= phi < 2 pi */
#define KO_SKY_LINE 5   /* on a graticule line */

/* Per-ray results.  Arrays hold one entry per traced ray; any pointer may be
   NULL except fate. */
typedef struct {
    uint8_t *fate;
    double *r_hit, *g, *intensity;
    double *max_abs_h, *max_rel_h;
    double *psi, *deflection;
    double *theta_f, *phi_f;
    uint8_t *n_cross;
    int32_t *n_steps, *n_evals;
    uint8_t *sky;
} ko_out;

/* Covariant Kerr metric at (r, theta): g = {g_tt, g_tph, g_rr, g_thth, g_phph}. */
void ko_metric_cov(double M, double a, double r, double th, double g[5]);

/* Contravariant metric and its r- and theta-derivatives, same ordering. */
void ko_metric_inv(double M, double a, double r, double th, double gi[5],
                   double dgi_dr[5], double dgi_dth[5]);

/* H = 1/2 g^{mu nu} p_mu p_nu with p_t = -E, p_phi = L.
   state = {r, theta, phi, p_r, p_theta}. */
double ko_hamiltonian(double M, double a, const double state[5], double E, double L);

/* Scale-free constraint residual |2 Sigma H| / D, D = sum of the magnitudes
   of the terms of 2 Sigma H in Carter's separated form. */
double ko_hamiltonian_rel(double M, double a, const double state[5], double E, double L);

/* Hamilton's equations: out = d/dlambda {r, theta, phi, p_r, p_theta};
   out[5] = dt/dlambda. */
void ko_rhs(double M, double a, const double state[5], double E, double L, double out[6]);

/* Camera: initial state for image-plane point (x, y).
   out = {r, theta, phi, p_r, p_theta, E, L}.  Returns 0, or 1 when
   x^2 + y^2 >= r_obs^2 (no real p_r). */
int ko_camera_ray(double M, double a, double r_obs, double incl, double x, double y,
                  double out[7]);

/* Pixel-centre coordinates of pixel (i, j). */
void ko_pixel_xy(const ko_setup *s, int32_t i, int32_t j, double *x, double *y);

/* Trace rays through image-plane points (x[k], y[k]), k < n. */
void ko_trace_xy(const ko_setup *s, const double *x, const double *y, int64_t n,
                 const ko_out *o, int n_threads);

/* Trace the pixels pix[k] (row-major j*nx+i), k < n; pix == NULL means all
   nx*ny pixels in order.  Outputs are indexed by k. */
void ko_trace_pixels(const ko_setup *s, const int32_t *pix, int64_t n, const ko_out *o,
                     int n_threads);

/* Trace one ray and record every accepted state:
   traj[6*k + {0..5}] = {lambda (RK4_S: s), r, theta, phi, p_r, p_theta}.
   Returns the number of recorded states (<= max_points); the first is the
   initial state.  Fate etc. go to entry 0 of o. */
int64_t ko_trace_one(const ko_setup *s, double x, double y, double *traj, int64_t max_points,
                     const ko_out *o);

/* Ring-flag post-pass over a full nx x ny image of deflection angles: pixel
   p is flagged when, for its +i or +j neighbour q with both deflections
   finite, an odd multiple of pi lies between Psi_p and Psi_q. */
void ko_ring_flags(int32_t nx, int32_t ny, const double *deflection, uint8_t *ring);

/* Sky code of the direction (theta, phi), any representation (theta may lie
   outside [0, pi] after the ray crossed the polar axis). */
int ko_sky_code(double theta, double phi, double grid_deg, double line_deg);

/* Angular velocity Omega = u^phi / u^t of the disk's circular orbits at
   radius r in the equatorial plane for the given rotation model. */
double ko_disk_omega(double M, double a, double r, int32_t rotation, double l0);

/* Emitted intensity at radius r of the disk for the given model. */
double ko_emissivity(double M, double r, double r_in, double r_out, double emis_q, int32_t model);

/* The same for either spacetime (kind KO_KERR uses a, KO_QMETRIC uses q):
   covariant components, their r- and theta-derivatives, the contravariant
   components with derivatives, H, |H|_rel (for the q-metric |2H| over the
   sum of the magnitudes of its four terms), Hamilton's equations and the
   camera. */
void ko_metric_cov_k(int32_t kind, double M, double a, double q, double r, double th, double g[5]);
void ko_metric_derivs_k(int32_t kind, double M, double a, double q, double r, double th, double dr[5],
                        double dth[5]);
void ko_metric_inv_k(int32_t kind, double M, double a, double q, double r, double th, double gi[5],
                     double dgi_dr[5], double dgi_dth[5]);
double ko_hamiltonian_k(int32_t kind, double M, double a, double q, const double z[5], double E, double L);
double ko_hamiltonian_rel_k(int32_t kind, double M, double a, double q, const double z[5], double E,
                            double L);
void ko_rhs_k(int32_t kind, double M, double a, double q, const double z[5], double E, double L, double out[6]);
int ko_camera_ray_k(int32_t kind, double M, double a, double q, double r0, double incl, double x, double y,
                    double out[7]);

/* Outer horizon r_+ = M + sqrt(M^2 - a^2). */
double ko_horizon(double M, double a);

/* Integrator self-test on y'' = -y, y(0) = 0, y'(0) = 1 over [0, T] with n
   fixed steps of the given method's underlying tableau (DP5 propagates the
   5th-order solution).  Returns the final (y, y') in out[2]. */
void ko_harmonic_fixed(int32_t method, double T, int64_t n, double out[2]);

/* n fixed steps of size T/n of any method on a test problem: problem 0 is
   y'' = -y as (y, y'), problem 1 is the scalar y' = y^2.  y0 and out hold 2
   resp. 1 values. */
void ko_fixed_steps(int32_t method, int32_t problem, double T, int64_t n, const double *y0,
                    double *out);

/* One step of size h of any method on a test problem (as above): the
   propagated solution and the embedded error estimate.  Returns the number
   of evaluations the step took beyond f(y0). */
int ko_one_step(int32_t method, int32_t problem, double h, const double *y0, double *yn, double *e);

/* The Butcher tableau of KO_RKF45 or KO_CK45: A row-major 6x6, the weights
   of the propagated and of the embedded solution. */
void ko_tableau(int32_t method, double A[36], double b_prop[6], double b_emb[6]);

/* Extrapolation of Bulirsch-Stoer chain ends to zero substep: f[k] is the
   modified-midpoint value with n_k = 2 (k + 1) substeps, k = 0..K-1 (1 <= K
   <= 8); writes the tableau's last row T[K-1][0..K-1] (its last entry is
   the extrapolated value).  rational = 0: Aitken-Neville polynomials in
   (1/n)^2; 1: Stoer-Bulirsch rational functions in (1/n)^2. */
void ko_bs_extrapolate(int32_t rational, int32_t K, const double *f, double *row);

#ifdef __cplusplus
}
#endif
#endif
