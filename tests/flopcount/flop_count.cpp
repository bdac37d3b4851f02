// flop_count.cpp -- test-only: algorithmic FLOP of the ray tracer's hot
// path, counted mechanically with the counting scalar of flop.h.
//
//   flop_count units            the per-unit counts of the plain reference
//                               (hotpath_ref.h) as JSON
//   flop_count oracle nx ny fov a incl r_obs src pix...
//                               the oracle itself (its matrix-inverse form,
//                               ../../oracle/kt_oracle.c compiled with the
//                               counting scalar for double) tracing the given
//                               pixels with DP45 at rtol 1e-12: total FLOP,
//                               evaluations and accepted steps as JSON
//   flop_count rhs a E L r th pr pth
//   flop_count qrhs q E L r th pr pth
//                               the reference's Kerr (M = 1, spin a) or
//                               q-metric (M = 1) RHS and diagnostics in plain
//                               double, for checking it against the oracle
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "hotpath_ref.h"
#include "flop.h"

// The oracle with every double a Flop.
#define double Flop
#include "../../oracle/kt_oracle.c"
#undef double

static long long count_of(void (*fn)()) {
    g_flops = FlopCounter();
    fn();
    return g_flops.total();
}

static RayConsts<Flop> kconst() {
    RayConsts<Flop> k;
    k.M = 1.0;
    k.a = 0.9;
    k.a2 = 0.81;
    k.E = 1.0;
    k.L = 2.5;
    k.aE = 0.9;
    k.aL = 2.25;
    return k;
}

static Flop g_z[5] = {30.0, 1.1, 0.3, -0.8, 0.4};

static void unit_rhs() {
    Flop f[5], H, rel;
    carter_rhs(kconst(), g_z, f, false, &H, &rel);
}
static void unit_rhs_diag() {
    Flop f[5], H, rel;
    carter_rhs(kconst(), g_z, f, true, &H, &rel);
}
static void unit_qrhs() {
    Flop f[5], H, rel;
    q_rhs(Flop(1.0), Flop(0.5), Flop(1.5), Flop(1.25), Flop(1.0), Flop(2.5), g_z, f, false, &H, &rel);
}
static void unit_qrhs_diag() {
    Flop f[5], H, rel;
    q_rhs(Flop(1.0), Flop(0.5), Flop(1.5), Flop(1.25), Flop(1.0), Flop(2.5), g_z, f, true, &H, &rel);
}
static void unit_stages() {
    Flop k[7][5], ys[5];
    for (int j = 0; j < 7; ++j)
        for (int c = 0; c < 5; ++c) k[j][c] = 0.1 * (j + 1) + c;
    for (int i = 1; i < 7; ++i) dp_stage(i, g_z, k, Flop(0.5), ys);
}
static void unit_error() {
    Flop k[7][5], e[5];
    for (int j = 0; j < 7; ++j)
        for (int c = 0; c < 5; ++c) k[j][c] = 0.1 * (j + 1) + c;
    dp_error(k, Flop(0.5), e);
}
static void unit_control() {
    Flop yn[5] = {30.1, 1.11, 0.31, -0.79, 0.41}, e[5] = {1e-12, 2e-13, 3e-13, 1e-13, 2e-13};
    bool acc;
    dp_control(g_z, yn, e, Flop(1e-12), Flop(1e-12), Flop(0.5), &acc);
}
static void unit_arc() {
    Flop n1[3] = {0.6, 0.0, 0.8}, n2[3];
    (void)swept_arc(n1, Flop(0.59), Flop(0.807), Flop(0.01), n2);
}

int main(int argc, char** argv) {
    if (argc >= 2 && !strcmp(argv[1], "units")) {
        const long long rhs = count_of(unit_rhs), rhs_diag = count_of(unit_rhs_diag);
        const long long qrhs = count_of(unit_qrhs), qrhs_diag = count_of(unit_qrhs_diag);
        std::printf("{\"rhs\": %lld, \"diag\": %lld, \"stages\": %lld, \"error\": %lld, \"control\": %lld, "
                    "\"arc\": %lld, \"q_rhs\": %lld, \"q_diag\": %lld}\n",
                    rhs, rhs_diag - rhs, count_of(unit_stages), count_of(unit_error), count_of(unit_control),
                    count_of(unit_arc), qrhs, qrhs_diag - qrhs);
        return 0;
    }
    if (argc >= 9 && !strcmp(argv[1], "rhs")) {
        RayConsts<double> k;
        k.M = 1.0;
        k.a = atof(argv[2]);
        k.a2 = k.a * k.a;
        k.E = atof(argv[3]);
        k.L = atof(argv[4]);
        k.aE = k.a * k.E;
        k.aL = k.a * k.L;
        const double z[5] = {atof(argv[5]), atof(argv[6]), 0.0, atof(argv[7]), atof(argv[8])};
        double f[5], H, rel;
        carter_rhs(k, z, f, true, &H, &rel);
        std::printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", f[0], f[1], f[2], f[3], f[4], H, rel);
        return 0;
    }
    if (argc >= 9 && !strcmp(argv[1], "qrhs")) {
        const double q = atof(argv[2]), E = atof(argv[3]), L = atof(argv[4]);
        const double z[5] = {atof(argv[5]), atof(argv[6]), 0.0, atof(argv[7]), atof(argv[8])};
        double f[5], H, rel;
        q_rhs(1.0, q, 1.0 + q, q * (2.0 + q), E, L, z, f, true, &H, &rel);
        std::printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", f[0], f[1], f[2], f[3], f[4], H, rel);
        return 0;
    }
    if (argc >= 10 && !strcmp(argv[1], "oracle")) {
        ko_setup s;
        memset(&s, 0, sizeof s);
        s.nx = atoi(argv[2]);
        s.ny = atoi(argv[3]);
        s.fov_x = s.fov_y = atof(argv[4]);
        s.M = 1.0;
        s.a = atof(argv[5]);
        s.metric = KO_KERR;
        s.incl = atof(argv[6]);
        s.r_obs = atof(argv[7]);
        s.method = KO_DP45;
        s.rtol = s.atol = 1e-12;
        s.h_init = 1.0;
        s.h_fixed = 1.0 / 128;
        s.cap_buffer = 0.01;
        s.r_escape = 1.1 * s.r_obs.v;
        s.max_steps = 1000000;
        s.src_on = atoi(argv[8]);
        s.r_src = s.r_obs;
        s.r_in = 6.0;
        s.r_out = 30.0;
        s.emis_q = 2.0;
        const int n = argc - 9;
        int32_t* pix = (int32_t*)calloc(n, sizeof(int32_t));
        for (int i = 0; i < n; ++i) pix[i] = atoi(argv[9 + i]);
        uint8_t* fate = (uint8_t*)calloc(n, 1);
        int32_t* nst = (int32_t*)calloc(n, sizeof(int32_t));
        int32_t* nev = (int32_t*)calloc(n, sizeof(int32_t));
        ko_out o;
        memset(&o, 0, sizeof o);
        o.fate = fate;
        o.n_steps = nst;
        o.n_evals = nev;
        g_flops = FlopCounter();
        ko_trace_pixels(&s, pix, n, &o, 1);
        long long evals = 0, steps = 0;
        for (int i = 0; i < n; ++i) {
            evals += nev[i];
            steps += nst[i];
        }
        std::printf("{\"flop\": %lld, \"evals\": %lld, \"steps\": %lld, \"add\": %lld, \"mul\": %lld, "
                    "\"div\": %lld, \"sqrt\": %lld, \"fn\": %lld}\n",
                    g_flops.total(), evals, steps, g_flops.add, g_flops.mul, g_flops.div, g_flops.sqrt, g_flops.fn);
        return 0;
    }
    std::fprintf(stderr, "usage: flop_count units | rhs a E L r th pr pth | oracle nx ny fov a incl r_obs src pix...\n");
    return 2;
}
