/* oracle_driver.c -- test-only: drives the oracle's entry points over every
   kind of workload it serves, for a build with AddressSanitizer and
   UndefinedBehaviorSanitizer (any report fails the run).  It prints one
   line of checksums so a run can also be compared with an uninstrumented
   build. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "kt_oracle.h"

static double checksum = 0.0;

static void add(double v)
{
    if (isfinite(v)) checksum += v;
}

static void image(ko_setup s, int32_t nx, int32_t ny)
{
    s.nx = nx;
    s.ny = ny;
    const int64_t n = (int64_t)nx * ny;
    ko_out o;
    memset(&o, 0, sizeof o);
    o.fate = malloc(n);
    o.r_hit = malloc(n * sizeof(double));
    o.g = malloc(n * sizeof(double));
    o.intensity = malloc(n * sizeof(double));
    o.max_abs_h = malloc(n * sizeof(double));
    o.max_rel_h = malloc(n * sizeof(double));
    o.psi = malloc(n * sizeof(double));
    o.deflection = malloc(n * sizeof(double));
    o.theta_f = malloc(n * sizeof(double));
    o.phi_f = malloc(n * sizeof(double));
    o.n_cross = malloc(n);
    o.n_steps = malloc(n * sizeof(int32_t));
    o.n_evals = malloc(n * sizeof(int32_t));
    o.sky = malloc(n);
    ko_trace_pixels(&s, NULL, n, &o, 2);
    uint8_t *ring = malloc(n);
    ko_ring_flags(nx, ny, o.deflection, ring);
    for (int64_t k = 0; k < n; ++k) {
        add(o.fate[k] + o.n_cross[k] + o.sky[k] + ring[k] + o.n_steps[k] + 1e-3 * o.n_evals[k]);
        add(o.r_hit[k]);
        add(o.g[k]);
        add(o.intensity[k]);
        add(o.deflection[k]);
        add(o.theta_f[k]);
    }
    /* a pixel list with repeats and the last pixel, and the minimal output set */
    int32_t pix[3] = {0, (int32_t)(n - 1), 0};
    ko_out m;
    memset(&m, 0, sizeof m);
    m.fate = malloc(3);
    ko_trace_pixels(&s, pix, 3, &m, 1);
    add(m.fate[1]);
    double traj[6 * 64];
    double x, y;
    ko_pixel_xy(&s, nx / 2, ny / 2, &x, &y);
    add((double)ko_trace_one(&s, x, y, traj, 64, &m));
    free(m.fate);
    free(ring);
    free(o.fate), free(o.r_hit), free(o.g), free(o.intensity), free(o.max_abs_h), free(o.max_rel_h);
    free(o.psi), free(o.deflection), free(o.theta_f), free(o.phi_f), free(o.n_cross), free(o.n_steps);
    free(o.n_evals), free(o.sky);
}

int main(void)
{
    ko_setup base;
    memset(&base, 0, sizeof base);
    base.M = 1.0;
    base.a = 0.9;
    base.r_obs = 1000.0;
    base.incl = 1.0471975511965976;
    base.fov_x = base.fov_y = 12.0;
    base.method = KO_DP45;
    base.h_fixed = 1.0 / 128;
    base.rtol = base.atol = 1e-10;
    base.h_init = 1.0;
    base.cap_buffer = 0.01;
    base.r_escape = 1100.0;
    base.max_steps = 1000000;
    base.r_src = 1000.0;
    base.r_in = 2.32;
    base.r_out = 30.0;
    base.emis_q = 2.0;
    base.grid_deg = 6.0;
    base.line_deg = 0.25;

    ko_setup s = base;
    s.src_on = 1;
    for (int m = KO_DP45; m <= KO_BS_RAT; ++m) {  /* every adaptive scheme, ring and source */
        s.method = m;
        image(s, 7, 5);
    }
    s = base;
    s.method = KO_RK4_S;
    s.a = 0.0;
    image(s, 6, 6);
    s = base;  /* Keplerian and constant-l0 disks, both emissivities */
    s.disk_on = 1;
    s.fov_x = s.fov_y = 35.0;
    image(s, 9, 4);
    s.rotation = 1;
    s.l0 = 2.8;
    s.emis_model = 1;
    image(s, 4, 9);
    s = base;  /* lensing: Kerr, flat space, the q-metric */
    s.sky_on = 1;
    s.r_obs = 100.0;
    s.r_escape = 110.0;
    s.fov_x = s.fov_y = 20.0;
    s.incl = 1.5707963267948966;
    image(s, 5, 5);
    s.M = 0.0;
    s.a = 0.0;
    image(s, 3, 4);
    s.M = 1.0;
    s.metric = KO_QMETRIC;
    s.q = 0.5;
    image(s, 4, 4);
    s = base;  /* invalid pixels (x^2 + y^2 >= r_obs^2), 1x1 image, a step budget */
    s.r_obs = 20.0;
    s.r_escape = 30.0;
    s.r_src = 25.0;
    s.fov_x = s.fov_y = 25.0;
    image(s, 4, 4);
    image(s, 1, 1);
    s.max_steps = 3;
    image(s, 3, 2);

    double z[5] = {7.0, 1.1, 0.2, -0.4, 0.3}, out[6], g[5], gi[5], dr[5], dth[5];
    ko_metric_cov(1.0, 0.7, 7.0, 1.1, g);
    ko_metric_inv(1.0, 0.7, 7.0, 1.1, gi, dr, dth);
    ko_rhs(1.0, 0.7, z, 1.0, 2.0, out);
    for (int i = 0; i < 5; ++i) add(g[i] + gi[i] + dr[i] + dth[i] + out[i]);
    add(ko_hamiltonian(1.0, 0.7, z, 1.0, 2.0) + ko_hamiltonian_rel(1.0, 0.7, z, 1.0, 2.0));
    add(ko_hamiltonian_rel_k(KO_QMETRIC, 1.0, 0.0, 0.4, z, 1.0, 2.0));
    double st[7];
    add((double)ko_camera_ray(1.0, 0.5, 50.0, 1.0, 60.0, 0.0, st));
    add((double)ko_sky_code(1.0, 7.0, 6.0, 0.25) + ko_disk_omega(1.0, 0.5, 8.0, 1, 2.8));
    add(ko_emissivity(1.0, 8.0, 6.0, 30.0, 2.0, 1) + ko_horizon(1.0, 0.3));
    double y0[2] = {0.0, 1.0}, yn[2], e[2], A[36], bp[6], be[6], fv[8], row[8];
    for (int m = 0; m <= KO_BS_RAT; ++m) {
        ko_fixed_steps(m, 0, 1.0, 3, y0, yn);
        add(yn[0] + ko_one_step(m, 1, 0.1, y0, yn, e));
    }
    ko_harmonic_fixed(KO_DP45, 1.0, 4, yn);
    ko_tableau(KO_RKF45, A, bp, be);
    add(A[7] + bp[0] + be[5] + yn[0]);
    for (int k = 0; k < 8; ++k) fv[k] = 1.0 / (1.0 + k);
    for (int K = 1; K <= 8; ++K) {
        ko_bs_extrapolate(0, K, fv, row);
        add(row[K - 1]);
        ko_bs_extrapolate(1, K, fv, row);
        add(row[K - 1]);
    }
    printf("checksum %.17g\n", checksum);
    return 0;
}
