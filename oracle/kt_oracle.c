/*
 * kt_oracle.c -- plain FP64 CPU oracle for backward ray tracing of null
 * geodesics around a Kerr black hole.
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU library and is never part of
 * the product path.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * What it computes, and where the method is defined (Velasquez-Cadavid et
 * al., "OSIRIS: A New Code for Ray Tracing Around Compact Objects"):
 *   - the Kerr line element in Boyer-Lindquist coordinates, eq:Kerr, with
 *     Sigma, Delta and the outer horizon r_H (Sect. 4.3);
 *   - the contravariant metric as the matrix inverse of eq:Kerr, and its
 *     coordinate derivatives through d(g^-1) = -g^-1 (dg) g^-1;
 *   - the Hamiltonian H = 1/2 g^{mu nu} p_mu p_nu (eq:ligH) and Hamilton's
 *     equations written out in Sect. 2.1 (the t, r, theta, phi rates and the
 *     p_r, p_theta forces; p_t and p_phi are conserved);
 *   - backward ray tracing from the observer (Sect. 2.2) with initial momenta
 *     from the image plane through the observer tetrad, eq:matrix and the
 *     second eq:momentums (Sect. 2.3), with p_r taken ingoing;
 *   - the Dormand-Prince 5(4) embedded pair (cited in Sect. 3.1; FSAL, six
 *     evaluations per step) and classic RK4;
 *   - the schemes Sect. 3.1 compares it with: Runge-Kutta-Fehlberg 4(5),
 *     Cash-Karp 5(4) and Bulirsch-Stoer extrapolation;
 *   - the constraint monitor Error = |H_num| (Sect. 3.1);
 *   - termination at r < r_H + delta_r (captured) and r > r_cs (escaped),
 *     Sect. 4.1, and on a thin equatorial disk (Sect. 5);
 *   - the redshift g = nu_obs/nu_em of eq:redshift for circular emitters
 *     (Keplerian, or with the constant specific angular momentum l0 of
 *     Sect. 5), and I_obs = g^3 I_em;
 *   - the coloured celestial sphere of Sect. 4.1: four quadrants and a
 *     graticule, hit where the ray crosses r = r_cs;
 *   - the q-metric of the appendix (eq:q-metric, written with signature
 *     (-,+,+,+)) as a second static axisymmetric spacetime for null rays.
 * Readings where the paper is silent or garbled (sign of p_r, the printed
 * redshift being -1/g, step control, event location, tolerances) are listed
 * in the design notes; the constants used here are the same readings.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA
 * contraction, no fast-math).
 */
#include "kt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Spacetime: eq:Kerr and its derivatives.                                   */
/* ------------------------------------------------------------------------ */

void ko_metric_cov(double M, double a, double r, double th, double g[5])
{
    double s = sin(th), c = cos(th);
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * M * r + a * a;
    g[0] = -(1.0 - 2.0 * M * r / Sig);                           /* g_tt   */
    g[1] = -2.0 * M * r * a * s * s / Sig;                       /* g_tphi (half the dt dphi coefficient) */
    g[2] = Sig / Del;                                            /* g_rr   */
    g[3] = Sig;                                                  /* g_thth */
    g[4] = s * s * (r * r + a * a + 2.0 * M * r * a * a * s * s / Sig); /* g_phph */
}

/* Partial derivatives of the covariant components with respect to r and
   theta, differentiated term by term from eq:Kerr. */
static void metric_cov_derivs(double M, double a, double r, double th, double dr[5],
                              double dth[5])
{
    double s = sin(th), c = cos(th);
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * M * r + a * a;
    double Sig_r = 2.0 * r;
    double Sig_th = -2.0 * a * a * s * c;
    double Del_r = 2.0 * r - 2.0 * M;
    double Sig2 = Sig * Sig;

    /* g_tt = -1 + 2 M r / Sigma */
    dr[0] = 2.0 * M * (Sig - r * Sig_r) / Sig2;
    dth[0] = -2.0 * M * r * Sig_th / Sig2;
    /* g_tphi = -2 M a r sin^2 / Sigma */
    dr[1] = -2.0 * M * a * s * s * (Sig - r * Sig_r) / Sig2;
    dth[1] = -2.0 * M * a * r * (2.0 * s * c * Sig - s * s * Sig_th) / Sig2;
    /* g_rr = Sigma / Delta */
    dr[2] = (Sig_r * Del - Sig * Del_r) / (Del * Del);
    dth[2] = Sig_th / Del;
    /* g_thth = Sigma */
    dr[3] = Sig_r;
    dth[3] = Sig_th;
    /* g_phph = sin^2 (r^2 + a^2) + 2 M r a^2 sin^4 / Sigma */
    dr[4] = 2.0 * r * s * s + 2.0 * M * a * a * s * s * s * s * (Sig - r * Sig_r) / Sig2;
    dth[4] = 2.0 * s * c * (r * r + a * a)
           + 2.0 * M * r * a * a * (4.0 * s * s * s * c * Sig - s * s * s * s * Sig_th) / Sig2;
}

/* The q-metric (eq:q-metric) with f = 1 - 2M/r, D = 1 + M^2 sin^2/(r^2 - 2Mr),
   P = q (2 + q):  g_tt = -f^(1+q), g_rr = f^-(1+q) D^-P, g_thth = r^2 f^-q D^-P,
   g_phph = r^2 sin^2 f^-q; and its r- and theta-derivatives (may be NULL). */
static void qmetric_cov(double M, double q, double r, double th, double g[5], double dr[5], double dth[5])
{
    double s = sin(th), c = cos(th);
    double f = 1.0 - 2.0 * M / r;
    double rf = r * r - 2.0 * M * r;
    double D = 1.0 + M * M * s * s / rf;
    double P = q * (2.0 + q);
    double fq = pow(f, q), DmP = pow(D, -P);
    g[0] = -f * fq;
    g[1] = 0.0;
    g[2] = DmP / (f * fq);
    g[3] = r * r * DmP / fq;
    g[4] = r * r * s * s / fq;
    if (dr) {
        double lf_r = 2.0 * M / (r * r) / f;                       /* d ln f / dr */
        double lD_r = -M * M * s * s * (2.0 * r - 2.0 * M) / (rf * rf) / D;
        double lD_th = 2.0 * M * M * s * c / rf / D;
        dr[0] = g[0] * (1.0 + q) * lf_r;
        dth[0] = 0.0;
        dr[1] = dth[1] = 0.0;
        dr[2] = g[2] * (-(1.0 + q) * lf_r - P * lD_r);
        dth[2] = g[2] * (-P * lD_th);
        dr[3] = g[3] * (2.0 / r - q * lf_r - P * lD_r);
        dth[3] = g[3] * (-P * lD_th);
        dr[4] = g[4] * (2.0 / r - q * lf_r);
        dth[4] = 2.0 * r * r * s * c / fq;
    }
}

void ko_metric_cov_k(int32_t kind, double M, double a, double q, double r, double th, double g[5])
{
    if (kind == KO_QMETRIC)
        qmetric_cov(M, q, r, th, g, NULL, NULL);
    else
        ko_metric_cov(M, a, r, th, g);
}

void ko_metric_derivs_k(int32_t kind, double M, double a, double q, double r, double th, double dr[5],
                        double dth[5])
{
    if (kind == KO_QMETRIC) {
        double g[5];
        qmetric_cov(M, q, r, th, g, dr, dth);
    } else {
        metric_cov_derivs(M, a, r, th, dr, dth);
    }
}

void ko_metric_inv_k(int32_t kind, double M, double a, double q, double r, double th, double gi[5],
                     double dgi_dr[5], double dgi_dth[5])
{
    double g[5], dr[5], dth[5];
    ko_metric_cov_k(kind, M, a, q, r, th, g);
    ko_metric_derivs_k(kind, M, a, q, r, th, dr, dth);

    /* The metric is block diagonal: a (t, phi) 2x2 block plus g_rr, g_thth. */
    double det = g[0] * g[4] - g[1] * g[1];
    double p = g[4] / det;  /* g^tt   */
    double u = -g[1] / det; /* g^tphi */
    double w = g[0] / det;  /* g^phph */
    gi[0] = p;
    gi[1] = u;
    gi[2] = 1.0 / g[2];
    gi[3] = 1.0 / g[3];
    gi[4] = w;

    /* d(G^-1) = -G^-1 dG G^-1 on the 2x2 block; -dg/g^2 on the diagonal. */
    const double *d[2] = {dr, dth};
    double *o[2] = {dgi_dr, dgi_dth};
    for (int k = 0; k < 2; ++k) {
        double dA = d[k][0], dB = d[k][1], dC = d[k][4];
        o[k][0] = -(p * p * dA + 2.0 * p * u * dB + u * u * dC);
        o[k][1] = -(p * u * dA + (u * u + p * w) * dB + u * w * dC);
        o[k][4] = -(u * u * dA + 2.0 * u * w * dB + w * w * dC);
        o[k][2] = -d[k][2] / (g[2] * g[2]);
        o[k][3] = -d[k][3] / (g[3] * g[3]);
    }
}

void ko_metric_inv(double M, double a, double r, double th, double gi[5], double dgi_dr[5],
                   double dgi_dth[5])
{
    ko_metric_inv_k(KO_KERR, M, a, 0.0, r, th, gi, dgi_dr, dgi_dth);
}

double ko_horizon(double M, double a) { return M + sqrt(M * M - a * a); }

/* ------------------------------------------------------------------------ */
/* Hamiltonian (eq:ligH) and Hamilton's equations (eq:edm, Sect. 2.1).        */
/* ------------------------------------------------------------------------ */

double ko_hamiltonian_k(int32_t kind, double M, double a, double q, const double z[5], double E, double L)
{
    double gi[5], dr[5], dth[5];
    ko_metric_inv_k(kind, M, a, q, z[0], z[1], gi, dr, dth);
    double pt = -E, pph = L, pr = z[3], pth = z[4];
    return 0.5 * (gi[0] * pt * pt + 2.0 * gi[1] * pt * pph + gi[2] * pr * pr
                  + gi[3] * pth * pth + gi[4] * pph * pph);
}

double ko_hamiltonian(double M, double a, const double z[5], double E, double L)
{
    return ko_hamiltonian_k(KO_KERR, M, a, 0.0, z, E, L);
}

/* For the q-metric (diagonal): |2H| over the sum of the magnitudes of the
   four terms g^{mu mu} p_mu^2. */
double ko_hamiltonian_rel_k(int32_t kind, double M, double a, double q, const double z[5], double E,
                            double L)
{
    if (kind != KO_QMETRIC) return ko_hamiltonian_rel(M, a, z, E, L);
    double gi[5], dr[5], dth[5];
    ko_metric_inv_k(kind, M, a, q, z[0], z[1], gi, dr, dth);
    double t[4] = {gi[0] * E * E, gi[2] * z[3] * z[3], gi[3] * z[4] * z[4], gi[4] * L * L};
    return fabs(t[0] + t[1] + t[2] + t[3]) / (fabs(t[0]) + t[1] + t[2] + t[3]);
}

double ko_hamiltonian_rel(double M, double a, const double z[5], double E, double L)
{
    double r = z[0], th = z[1], pr = z[3], pth = z[4];
    double s = sin(th), c = cos(th);
    double Sig = r * r + a * a * c * c;
    double Del = r * r - 2.0 * M * r + a * a;
    double T = L / s - a * E * s;
    double W = (r * r + a * a) * E - a * L;
    double D = Del * pr * pr + pth * pth + T * T + W * W / Del;
    double H = ko_hamiltonian(M, a, z, E, L);
    return fabs(2.0 * Sig * H) / D;
}

void ko_rhs_k(int32_t kind, double M, double a, double q, const double z[5], double E, double L, double out[6])
{
    double gi[5], dr[5], dth[5];
    ko_metric_inv_k(kind, M, a, q, z[0], z[1], gi, dr, dth);
    double pt = -E, pph = L, pr = z[3], pth = z[4];
    out[0] = gi[2] * pr;                 /* r dot      = g^rr p_r               */
    out[1] = gi[3] * pth;                /* theta dot  = g^thth p_theta         */
    out[2] = gi[1] * pt + gi[4] * pph;   /* phi dot    = g^tphi p_t + g^phph p_phi */
    out[3] = (-pt * pt * dr[0] - 2.0 * pt * pph * dr[1] - pr * pr * dr[2]
              - pth * pth * dr[3] - pph * pph * dr[4]) / 2.0;
    out[4] = (-pt * pt * dth[0] - pr * pr * dth[2] - pth * pth * dth[3]
              - pph * (2.0 * pt * dth[1] + pph * dth[4])) / 2.0;
    out[5] = gi[0] * pt + gi[1] * pph;   /* t dot */
}

void ko_rhs(double M, double a, const double z[5], double E, double L, double out[6])
{
    ko_rhs_k(KO_KERR, M, a, 0.0, z, E, L, out);
}

/* ------------------------------------------------------------------------ */
/* Camera: eq:matrix, eq:pimf and the second eq:momentums (Sect. 2.3).       */
/* ------------------------------------------------------------------------ */

int ko_camera_ray_k(int32_t kind, double M, double a, double q, double r0, double incl, double x, double y,
                    double out[7])
{
    double g[5];
    ko_metric_cov_k(kind, M, a, q, r0, incl, g);
    double At = sqrt(g[4] / (g[1] * g[1] - g[0] * g[4]));
    /* observer-frame components with P^t = 1 (eq:pimf): */
    double Pth = y / r0;
    double Pph = -x / r0;
    double E = 1.0 / At + x * g[1] / (r0 * sqrt(g[4]));
    double L = -x * sqrt(g[4]) / r0;
    double pth = y * sqrt(g[3]) / r0;
    double rad = 1.0 - Pth * Pth - Pph * Pph;
    out[0] = r0;
    out[1] = incl;
    out[2] = 0.0;
    out[3] = rad > 0.0 ? -sqrt(g[2] * rad) : 0.0; /* ingoing */
    out[4] = pth;
    out[5] = E;
    out[6] = L;
    return rad > 0.0 ? 0 : 1;
}

int ko_camera_ray(double M, double a, double r0, double incl, double x, double y, double out[7])
{
    return ko_camera_ray_k(KO_KERR, M, a, 0.0, r0, incl, x, y, out);
}

void ko_pixel_xy(const ko_setup *s, int32_t i, int32_t j, double *x, double *y)
{
    *x = -s->fov_x + (i + 0.5) * (2.0 * s->fov_x / s->nx);
    *y = -s->fov_y + (j + 0.5) * (2.0 * s->fov_y / s->ny);
}

/* ------------------------------------------------------------------------ */
/* Integrators.                                                              */
/* ------------------------------------------------------------------------ */

#define NMAX 5
#define BS_K 5 /* Bulirsch-Stoer columns: order 2 BS_K */

typedef void (*field_fn)(const double *y, double *dy, const void *ctx);

/* Dormand & Prince (1980) RK5(4)7M tableau. */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
/* 5th-order weights (equal to the last row of A: first same as last) and
   embedded 4th-order weights. */
static const double DP_B5[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_B4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* One DP5(4) step of size h from y with k1 = f(y) given.  Writes the
   5th-order solution y5, k7 = f(y5) (the next step's k1) and the error
   vector e = y5 - y4.  Six new evaluations. */
static void dp45_step(field_fn f, const void *ctx, int n, const double *y, const double *k1,
                      double h, double *y5, double *k7, double *e)
{
    double k[7][NMAX];
    double ys[NMAX];
    memcpy(k[0], k1, sizeof(double) * n);
    for (int st = 1; st < 7; ++st) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < st; ++j) acc += DP_A[st][j] * k[j][i];
            ys[i] = y[i] + h * acc;
        }
        f(ys, k[st], ctx);
    }
    /* the seventh stage was evaluated at y + h sum_j b5_j k_j = y5 */
    for (int i = 0; i < n; ++i) {
        y5[i] = ys[i];
        k7[i] = k[6][i];
        double acc = 0.0;
        for (int j = 0; j < 7; ++j) acc += (DP_B5[j] - DP_B4[j]) * k[j][i];
        e[i] = h * acc;
    }
}

/* Six-stage embedded pairs without FSAL: stage rows A, the weights of the
   propagated solution and of the embedded one.  The error estimate is the
   difference of the two solutions. */
typedef struct {
    double A[6][5];
    double b_prop[6], b_emb[6];
} erk6_tableau;

/* Fehlberg (1969), RK4(5): the 4th-order solution is propagated and the
   5th-order one estimates its error. */
static const erk6_tableau RKF45 = {
    {{0, 0, 0, 0, 0},
     {1.0 / 4, 0, 0, 0, 0},
     {3.0 / 32, 9.0 / 32, 0, 0, 0},
     {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0},
     {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0},
     {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}},
    {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0},
    {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55},
};

/* Cash & Karp (1990), RK5(4): the 5th-order solution is propagated (local
   extrapolation) and the embedded 4th-order one estimates the error. */
static const erk6_tableau CK45 = {
    {{0, 0, 0, 0, 0},
     {1.0 / 5, 0, 0, 0, 0},
     {3.0 / 40, 9.0 / 40, 0, 0, 0},
     {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
     {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
     {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}},
    {37.0 / 378, 0, 250.0 / 621, 125.0 / 594, 0, 512.0 / 1771},
    {2825.0 / 27648, 0, 18575.0 / 48384, 13525.0 / 55296, 277.0 / 14336, 1.0 / 4},
};

/* One step of a six-stage pair from y with k1 = f(y) given: the propagated
   solution yn, kn = f(yn) (the next step's k1) and e = yn - y_embedded.
   Six new evaluations. */
static void erk6_step(const erk6_tableau *t, field_fn f, const void *ctx, int n, const double *y,
                      const double *k1, double h, double *yn, double *kn, double *e)
{
    double k[6][NMAX];
    double ys[NMAX];
    memcpy(k[0], k1, sizeof(double) * n);
    for (int st = 1; st < 6; ++st) {
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < st; ++j) acc += t->A[st][j] * k[j][i];
            ys[i] = y[i] + h * acc;
        }
        f(ys, k[st], ctx);
    }
    for (int i = 0; i < n; ++i) {
        double acc = 0.0, diff = 0.0;
        for (int j = 0; j < 6; ++j) {
            acc += t->b_prop[j] * k[j][i];
            diff += (t->b_prop[j] - t->b_emb[j]) * k[j][i];
        }
        yn[i] = y[i] + h * acc;
        e[i] = h * diff;
    }
    f(yn, kn, ctx);
}

/* Extrapolation of chain ends to zero substep size.  Row k of the tableau
   holds T[k][0] = f[k], the chain end with n_k = 2 (k + 1) substeps, and its
   extrapolations T[k][j] (j = 1..k), each from T[k][j-1] and the row above.
   With x_k = (1/n_k)^2 (the modified midpoint rule's error expansion is even
   in the substep for even n_k), evaluated at x = 0:
     polynomial (Aitken-Neville):
       T[k][j] = T[k][j-1] + (T[k][j-1] - T[k-1][j-1]) / ((n_k/n_{k-j})^2 - 1);
     rational (Stoer and Bulirsch's recursion for rational interpolation,
     with T[k-1][-1] = 0):
       d = T[k][j-1] - T[k-1][j-1],
       T[k][j] = T[k][j-1] + d / ((n_k/n_{k-j})^2 (1 - d / (T[k][j-1] - T[k-1][j-2])) - 1).
   Where a denominator of the rational form vanishes the entry is taken as
   T[k][j-1] (no correction). */
void ko_bs_extrapolate(int32_t rational, int32_t K, const double *f, double *row)
{
    double T[8][8];
    for (int k = 0; k < K; ++k) {
        const double nk = 2 * (k + 1);
        T[k][0] = f[k];
        for (int j = 1; j <= k; ++j) {
            const double nkj = 2 * (k - j + 1);
            const double ratio = (nk * nk) / (nkj * nkj);
            const double d = T[k][j - 1] - T[k - 1][j - 1];
            if (!rational) {
                T[k][j] = T[k][j - 1] + d / (ratio - 1.0);
            } else {
                const double below = j >= 2 ? T[k - 1][j - 2] : 0.0;
                const double din = T[k][j - 1] - below;
                double upd = 0.0;
                if (din != 0.0) {
                    const double den = ratio * (1.0 - d / din) - 1.0;
                    if (den != 0.0) upd = d / den;
                }
                T[k][j] = T[k][j - 1] + upd;
            }
        }
    }
    for (int j = 0; j < K; ++j) row[j] = T[K - 1][j];
}

/* Bulirsch-Stoer step: Gragg's modified midpoint rule over [0, h] with
   n_k = 2k substeps (k = 1..BS_K), each chain started from y, then the chain
   ends extrapolated to zero substep size (ko_bs_extrapolate: polynomial, or
   rational with `rational` set), component by component.  The step returns
   the last diagonal entry T[K][K] (order 2K) and e = T[K][K] - T[K][K-1].
   Evaluations: n_k - 1 per chain (k1 = f(y) starts every chain) plus f at
   the result for the next step: BS_K^2 + 1. */
static void bs_step(int rational, field_fn f, const void *ctx, int n, const double *y, const double *k1,
                    double h, double *yn, double *kn, double *e)
{
    double ends[NMAX][BS_K];
    for (int k = 0; k < BS_K; ++k) {
        const int ns = 2 * (k + 1);
        const double hs = h / ns;
        double zp[NMAX], zc[NMAX], fz[NMAX];
        for (int i = 0; i < n; ++i) {
            zp[i] = y[i];
            zc[i] = y[i] + hs * k1[i];
        }
        for (int m = 1; m < ns; ++m) {
            f(zc, fz, ctx);
            for (int i = 0; i < n; ++i) {
                const double znext = zp[i] + 2.0 * hs * fz[i];
                zp[i] = zc[i];
                zc[i] = znext;
            }
        }
        for (int i = 0; i < n; ++i) ends[i][k] = zc[i];
    }
    for (int i = 0; i < n; ++i) {
        double row[BS_K];
        ko_bs_extrapolate(rational, BS_K, ends[i], row);
        yn[i] = row[BS_K - 1];
        e[i] = row[BS_K - 1] - row[BS_K - 2];
    }
    f(yn, kn, ctx);
}

/* Classic RK4 step of size h from y with k1 = f(y) given.  Writes y_new and
   f(y_new).  Four new evaluations. */
static void rk4_step(field_fn f, const void *ctx, int n, const double *y, const double *k1,
                     double h, double *yn, double *kn)
{
    double k2[NMAX], k3[NMAX], k4[NMAX], ys[NMAX];
    for (int i = 0; i < n; ++i) ys[i] = y[i] + 0.5 * h * k1[i];
    f(ys, k2, ctx);
    for (int i = 0; i < n; ++i) ys[i] = y[i] + 0.5 * h * k2[i];
    f(ys, k3, ctx);
    for (int i = 0; i < n; ++i) ys[i] = y[i] + h * k3[i];
    f(ys, k4, ctx);
    for (int i = 0; i < n; ++i) yn[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    f(yn, kn, ctx);
}

/* One step of any method; returns the number of new evaluations.  RK4
   gives a zero error vector. */
static int step_any(int32_t method, field_fn f, const void *ctx, int n, const double *y,
                    const double *k1, double h, double *yn, double *kn, double *e)
{
    switch (method) {
    case KO_DP45:
        dp45_step(f, ctx, n, y, k1, h, yn, kn, e);
        return 6;
    case KO_RKF45:
        erk6_step(&RKF45, f, ctx, n, y, k1, h, yn, kn, e);
        return 6;
    case KO_CK45:
        erk6_step(&CK45, f, ctx, n, y, k1, h, yn, kn, e);
        return 6;
    case KO_BS:
    case KO_BS_RAT:
        bs_step(method == KO_BS_RAT, f, ctx, n, y, k1, h, yn, kn, e);
        return BS_K * BS_K + 1;
    default:
        rk4_step(f, ctx, n, y, k1, h, yn, kn);
        for (int i = 0; i < n; ++i) e[i] = 0.0;
        return 4;
    }
}

/* Exponent of the step-size controller: 1 / (order of the error estimate + 1). */
static double controller_exponent(int32_t method)
{
    return (method == KO_BS || method == KO_BS_RAT) ? 1.0 / (2 * BS_K - 1) : 1.0 / 5;
}

static void harmonic_field(const double *y, double *dy, const void *ctx)
{
    (void)ctx;
    dy[0] = y[1];
    dy[1] = -y[0];
}

static void riccati_field(const double *y, double *dy, const void *ctx)
{
    (void)ctx;
    dy[0] = y[0] * y[0];
}

void ko_harmonic_fixed(int32_t method, double T, int64_t n, double out[2])
{
    double y0[2] = {0.0, 1.0};
    ko_fixed_steps(method, 0, T, n, y0, out);
}

void ko_fixed_steps(int32_t method, int32_t problem, double T, int64_t n, const double *y0,
                    double *out)
{
    field_fn f = problem == 0 ? harmonic_field : riccati_field;
    const int dim = problem == 0 ? 2 : 1;
    double y[2], k[2], yn[2], kn[2], e[2];
    memcpy(y, y0, sizeof(double) * dim);
    const double h = T / (double)n;
    f(y, k, NULL);
    for (int64_t s = 0; s < n; ++s) {
        step_any(method, f, NULL, dim, y, k, h, yn, kn, e);
        memcpy(y, yn, sizeof(double) * dim);
        memcpy(k, kn, sizeof(double) * dim);
    }
    memcpy(out, y, sizeof(double) * dim);
}

int ko_one_step(int32_t method, int32_t problem, double h, const double *y0, double *yn, double *e)
{
    field_fn f = problem == 0 ? harmonic_field : riccati_field;
    const int dim = problem == 0 ? 2 : 1;
    double k[2], kn[2];
    f(y0, k, NULL);
    return step_any(method, f, NULL, dim, y0, k, h, yn, kn, e);
}

void ko_tableau(int32_t method, double A[36], double b_prop[6], double b_emb[6])
{
    const erk6_tableau *t = method == KO_RKF45 ? &RKF45 : &CK45;
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) A[6 * i + j] = j < 5 ? t->A[i][j] : 0.0;
        b_prop[i] = t->b_prop[i];
        b_emb[i] = t->b_emb[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Ray tracing.                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double M, a, E, L, q;
    int kind;
    int s_time; /* 1: field scaled by d(lambda)/ds = Delta / r */
} ray_ctx;

static void ray_field(const double *z, double *dz, const void *vctx)
{
    const ray_ctx *c = (const ray_ctx *)vctx;
    double out[6];
    ko_rhs_k(c->kind, c->M, c->a, c->q, z, c->E, c->L, out);
    double w = 1.0;
    if (c->s_time) {
        double r = z[0];
        w = (r * r - 2.0 * c->M * r + c->a * c->a) / r;
    }
    for (int i = 0; i < 5; ++i) dz[i] = w * out[i];
}

typedef struct {
    const ko_setup *s;
    ray_ctx ctx;
    int64_t evals;
} tracer;

/* One step of the configured method; returns the number of evaluations. */
static int take_step(tracer *t, const double *z, const double *k1, double h, double *zn,
                     double *kn, double *e)
{
    return step_any(t->s->method, ray_field, &t->ctx, 5, z, k1, h, zn, kn, e);
}

/* Locate the root of z(h')[comp] - target for h' in (0, h] with the Illinois
   variant of regula falsi.  Every trial is a fresh step of size h' from the
   step's start state z (same stepper).  fa = g(0), fb = g(h) bracket the
   root.  Stops when |g| <= tol or after 64 trials; zc is the last trial. */
static void locate_event(tracer *t, const double *z, const double *k1, double h, int comp,
                         double target, double fa, double fb, double tol, double *zc)
{
    double a = 0.0, b = h;
    double kc[5], ec[5];
    for (int it = 0; it < 64; ++it) {
        double c = b - fb * (b - a) / (fb - fa);
        t->evals += take_step(t, z, k1, c, zc, kc, ec);
        double fc = zc[comp] - target;
        if (fabs(fc) <= tol) return;
        if (fc * fb < 0.0) {
            a = b;
            fa = fb;
        } else {
            fa *= 0.5;
        }
        b = c;
        fb = fc;
    }
}

static void unit_dir(double th, double ph, double n[3])
{
    n[0] = sin(th) * cos(ph);
    n[1] = sin(th) * sin(ph);
    n[2] = cos(th);
}

/* Great-circle angle between the directions of two positions. */
static double arc_between(double th1, double ph1, double th2, double ph2)
{
    double u[3], v[3];
    unit_dir(th1, ph1, u);
    unit_dir(th2, ph2, v);
    double cx = u[1] * v[2] - u[2] * v[1];
    double cy = u[2] * v[0] - u[0] * v[2];
    double cz = u[0] * v[1] - u[1] * v[0];
    double cr = sqrt(cx * cx + cy * cy + cz * cz);
    double dt = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    return atan2(cr, dt);
}

int ko_sky_code(double theta, double phi, double grid_deg, double line_deg)
{
    /* canonical angles from the unit vector of the direction */
    double n[3];
    unit_dir(theta, phi, n);
    double th = acos(fmax(-1.0, fmin(1.0, n[2])));
    double ph = atan2(n[1], n[0]);
    if (ph < 0.0) ph += 2.0 * PI;
    if (ph >= 2.0 * PI) ph -= 2.0 * PI;
    if (grid_deg > 0.0) {
        double tdeg = th * 180.0 / PI, pdeg = ph * 180.0 / PI;
        double dt = fabs(tdeg - grid_deg * round(tdeg / grid_deg));
        double dp = fabs(pdeg - grid_deg * round(pdeg / grid_deg));
        if (dt <= line_deg || dp <= line_deg) return KO_SKY_LINE;
    }
    if (th < PI / 2) return ph < PI ? KO_SKY_GREEN : KO_SKY_RED;
    return ph < PI ? KO_SKY_BLUE : KO_SKY_YELLOW;
}

double ko_emissivity(double M, double r, double r_in, double r_out, double emis_q, int32_t model)
{
    if (model == 1) {
        double e = (M / r) * (M / r) * (1.0 - sqrt(r_in / r));
        double s = (r_out - r) / (2.0 * M);
        if (s < 1.0) e *= s * s * (3.0 - 2.0 * s);
        return e;
    }
    return pow(M / r, emis_q);
}

double ko_disk_omega(double M, double a, double r, int32_t rotation, double l0)
{
    if (rotation == 1) {
        /* constant specific angular momentum l0 = -u_phi / u_t */
        double g[5];
        ko_metric_cov(M, a, r, PI / 2, g);
        return -(g[1] + l0 * g[0]) / (g[4] + l0 * g[1]);
    }
    return sqrt(M) / (pow(r, 1.5) + a * sqrt(M));
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Trace one ray from image-plane point (x, y).  Writes entry k of o and, if
   traj != NULL, up to maxp accepted states. */
static int64_t trace_ray(const ko_setup *s, double x, double y, const ko_out *o, int64_t k,
                         double *traj, int64_t maxp)
{
    const double NaN = nan("");
    int fate = KO_MAXSTEPS;
    double r_hit = NaN, gred = NaN, inten = 0.0, psi = NaN, defl = NaN;
    int ncross = 0;
    int sky = KO_SKY_NONE;
    int64_t nsteps = 0, npts = 0;
    double maxabs = NaN, maxrel = NaN;

    double init[7];
    int invalid = ko_camera_ray_k(s->metric, s->M, s->a, s->q, s->r_obs, s->incl, x, y, init);
    double z[5] = {init[0], init[1], init[2], init[3], init[4]};
    double thf = z[1], phf = z[2];

    tracer t;
    t.s = s;
    t.ctx.M = s->M;
    t.ctx.a = s->a;
    t.ctx.E = init[5];
    t.ctx.L = init[6];
    t.ctx.kind = s->metric;
    t.ctx.q = s->q;
    t.ctx.s_time = (s->method == KO_RK4_S);
    t.evals = 0;

    if (invalid) {
        fate = KO_INVALID;
        goto done;
    }

    {
        const double E = init[5], L = init[6];
        const double r_cap = (s->metric == KO_QMETRIC ? 2.0 * s->M : ko_horizon(s->M, s->a)) + s->cap_buffer;
        const int dp = (s->method != KO_RK4_S); /* adaptive */
        const double expo = controller_exponent(s->method);
        double k1[5], zn[5], kn[5], e[5];
        double lam = 0.0;
        double h = dp ? s->h_init : s->h_fixed;
        int rejected = 0;
        double Psi = 0.0;
        int src_done = 0;

        ray_field(z, k1, &t.ctx);
        t.evals = 1;
        maxabs = fabs(ko_hamiltonian_k(s->metric, s->M, s->a, s->q, z, E, L));
        maxrel = ko_hamiltonian_rel_k(s->metric, s->M, s->a, s->q, z, E, L);
        if (traj && npts < maxp) {
            double *p = traj + 6 * npts++;
            p[0] = 0.0;
            memcpy(p + 1, z, sizeof z);
        }

        for (;;) {
            if (nsteps >= s->max_steps || t.evals >= 16 * s->max_steps) {
                fate = KO_MAXSTEPS;
                break;
            }
            t.evals += take_step(&t, z, k1, h, zn, kn, e);
            if (!all_finite(zn, 5)) {
                fate = KO_STEPFAIL;
                break;
            }
            double h_next = h;
            if (dp) {
                /* RMS of the error relative to sc_i = atol + rtol max(|y_i|, |y5_i|) */
                double acc = 0.0;
                for (int i = 0; i < 5; ++i) {
                    double sc = s->atol + s->rtol * fmax(fabs(z[i]), fabs(zn[i]));
                    acc += (e[i] / sc) * (e[i] / sc);
                }
                double err = sqrt(acc / 5.0);
                if (isnan(err)) {
                    fate = KO_STEPFAIL;
                    break;
                }
                if (err > 1.0) {
                    h *= fmax(0.2, 0.9 * pow(err, -expo));
                    rejected = 1;
                    if (h < 1e-12 * fmax(1.0, fabs(lam))) {
                        fate = KO_STEPFAIL;
                        break;
                    }
                    continue;
                }
                double fac = err < 1e-10 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -expo)));
                if (rejected) fac = fmin(fac, 1.0);
                rejected = 0;
                h_next = h * fac;
            }

            /* accepted step z -> zn */
            ++nsteps;
            double ha = fabs(ko_hamiltonian_k(s->metric, s->M, s->a, s->q, zn, E, L));
            double hr = ko_hamiltonian_rel_k(s->metric, s->M, s->a, s->q, zn, E, L);
            if (ha > maxabs) maxabs = ha;
            if (hr > maxrel) maxrel = hr;
            if (traj && npts < maxp) {
                double *p = traj + 6 * npts++;
                p[0] = lam + h;
                memcpy(p + 1, zn, sizeof zn);
            }

            /* thin disk in the equatorial plane */
            if (s->disk_on) {
                double ga = z[1] - PI / 2, gb = zn[1] - PI / 2;
                if (ga * gb < 0.0 || gb == 0.0) {
                    double zc[5];
                    if (gb == 0.0)
                        memcpy(zc, zn, sizeof zc);
                    else
                        locate_event(&t, z, k1, h, 1, PI / 2, ga, gb, 1e-14, zc);
                    double rc = zc[0];
                    if (rc >= s->r_in && rc <= s->r_out) {
                        double gm[5];
                        ko_metric_cov(s->M, s->a, rc, PI / 2, gm);
                        double Om = ko_disk_omega(s->M, s->a, rc, s->rotation, s->l0);
                        double norm = -gm[0] - 2.0 * Om * gm[1] - Om * Om * gm[4];
                        if (norm > 0.0) {
                            double ut = 1.0 / sqrt(norm);
                            gred = 1.0 / (ut * (E - Om * L));
                            inten = gred * gred * gred *
                                    ko_emissivity(s->M, rc, s->r_in, s->r_out, s->emis_q, s->emis_model);
                        } /* else: no timelike circular orbit there; g stays NaN */
                        r_hit = rc;
                        fate = KO_DISK;
                        thf = zc[1];
                        phf = zc[2];
                        goto done;
                    }
                    if (ncross < 255) ++ncross;
                }
            }
            if (zn[0] < r_cap) {
                fate = KO_CAPTURED;
                thf = zn[1];
                phf = zn[2];
                break;
            }
            if (s->src_on && !src_done) {
                if (z[0] < s->r_src && zn[0] >= s->r_src) {
                    double zc[5];
                    locate_event(&t, z, k1, h, 0, s->r_src, z[0] - s->r_src, zn[0] - s->r_src,
                                 1e-12 * s->r_src, zc);
                    defl = Psi + arc_between(z[1], z[2], zc[1], zc[2]);
                    psi = arc_between(zc[1], zc[2], PI - s->incl, PI);
                    src_done = 1;
                } else {
                    Psi += arc_between(z[1], z[2], zn[1], zn[2]);
                }
            }
            if (zn[0] > s->r_escape) {
                fate = KO_ESCAPED;
                thf = zn[1];
                phf = zn[2];
                if (s->sky_on) {
                    /* the point where the ray meets the celestial sphere */
                    double zc[5];
                    locate_event(&t, z, k1, h, 0, s->r_escape, z[0] - s->r_escape,
                                 zn[0] - s->r_escape, 1e-12 * s->r_escape, zc);
                    thf = zc[1];
                    phf = zc[2];
                    sky = ko_sky_code(thf, phf, s->grid_deg, s->line_deg);
                }
                break;
            }
            memcpy(z, zn, sizeof z);
            memcpy(k1, kn, sizeof k1);
            lam += h;
            h = h_next;
            thf = z[1];
            phf = z[2];
        }
    }

done:
    o->fate[k] = (uint8_t)fate;
    if (o->r_hit) o->r_hit[k] = r_hit;
    if (o->g) o->g[k] = gred;
    if (o->intensity) o->intensity[k] = inten;
    if (o->max_abs_h) o->max_abs_h[k] = maxabs;
    if (o->max_rel_h) o->max_rel_h[k] = maxrel;
    if (o->psi) o->psi[k] = psi;
    if (o->deflection) o->deflection[k] = defl;
    if (o->theta_f) o->theta_f[k] = thf;
    if (o->phi_f) o->phi_f[k] = phf;
    if (o->n_cross) o->n_cross[k] = (uint8_t)ncross;
    if (o->n_steps) o->n_steps[k] = (int32_t)nsteps;
    if (o->n_evals) o->n_evals[k] = (int32_t)t.evals;
    if (o->sky) o->sky[k] = (uint8_t)sky;
    return npts;
}

void ko_trace_xy(const ko_setup *s, const double *x, const double *y, int64_t n, const ko_out *o,
                 int n_threads)
{
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads)
#endif
    for (int64_t k = 0; k < n; ++k) trace_ray(s, x[k], y[k], o, k, NULL, 0);
}

void ko_trace_pixels(const ko_setup *s, const int32_t *pix, int64_t n, const ko_out *o,
                     int n_threads)
{
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads)
#endif
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = pix ? pix[k] : k;
        double x, y;
        ko_pixel_xy(s, (int32_t)(p % s->nx), (int32_t)(p / s->nx), &x, &y);
        trace_ray(s, x, y, o, k, NULL, 0);
    }
}

int64_t ko_trace_one(const ko_setup *s, double x, double y, double *traj, int64_t max_points,
                     const ko_out *o)
{
    return trace_ray(s, x, y, o, 0, traj, max_points);
}

/* Number of odd multiples of pi that are <= v. */
static double odd_pi_count(double v) { return floor((v + PI) / (2.0 * PI)); }

void ko_ring_flags(int32_t nx, int32_t ny, const double *defl, uint8_t *ring)
{
    for (int32_t j = 0; j < ny; ++j)
        for (int32_t i = 0; i < nx; ++i) {
            int64_t p = (int64_t)j * nx + i;
            uint8_t flag = 0;
            if (isfinite(defl[p])) {
                if (i + 1 < nx && isfinite(defl[p + 1])
                    && odd_pi_count(defl[p]) != odd_pi_count(defl[p + 1]))
                    flag = 1;
                if (j + 1 < ny && isfinite(defl[p + nx])
                    && odd_pi_count(defl[p]) != odd_pi_count(defl[p + nx]))
                    flag = 1;
            }
            ring[p] = flag;
        }
}
