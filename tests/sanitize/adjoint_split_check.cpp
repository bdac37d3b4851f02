// adjoint_split_check.cpp -- test-only: the algebra of split backward sweeps
// on the host, with the adjoint's own step VJP (kt_adjoint_math.h).
//
// Along a 300-step frozen Dormand-Prince trajectory of the field (steps of
// varying size, falling from r = 12M to 2.1M around an a = 0.7 hole, whose
// horizon is at 1.71M), the cotangent
// of the start state is computed twice:
//   sequential: the step VJPs applied one after the other from the end;
//   split: each 64-step segment swept from the four basis cotangents of
//     (r, theta, p_r, p_theta) with zero parameter cotangents, then the
//     segments' columns applied to the seeded cotangent, last segment first.
// The phi cotangent must stay exactly zero in every basis sweep (the field
// does not depend on phi), and the two results must agree to rounding.  The
// same combination taken first segment first must not agree (the check
// can tell the order).
#include <cmath>
#include <cstdio>

#include "kt_adjoint_math.h"

using namespace kt;
using namespace kt::adj;

static void step_map(double M, double a, double E, double L, const double y[5], double h, double out[5]) {
    double K[6][5], Y[5];
    for (int j = 0; j < 6; ++j) {
        for (int i = 0; i < 5; ++i) {
            double acc = 0.0;
            for (int l = 0; l < j; ++l) acc += dp_a(j, l) * K[l][i];
            Y[i] = y[i] + h * acc;
        }
        double s, c;
        field(M, a, E, L, Y, K[j], &s, &c);
    }
    for (int i = 0; i < 5; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += dp_b(j) * K[j][i];
        out[i] = y[i] + h * acc;
    }
}

int main() {
    const double M = 1.0, a = 0.7, E = 1.0, L = 2.9;
    constexpr int N = 300, SEG = 64, NSEG = (N + SEG - 1) / SEG;
    static double Y[N][5], H[N];
    double y[5] = {12.0, 1.2, 0.0, -0.9, 0.5};  // falls to r = 2.1
    for (int j = 0; j < N; ++j) {
        H[j] = 0.05 + 0.02 * std::sin(0.37 * j);
        for (int i = 0; i < 5; ++i) Y[j][i] = y[i];
        step_map(M, a, E, L, y, H[j], y);
    }
    const double seed[5] = {0.8, -1.3, 0.0, 0.4, 2.1};

    // sequential sweep
    double zb[5];
    for (int i = 0; i < 5; ++i) zb[i] = seed[i];
    ParBar pb{0.0, 0.0, 0.0};
    for (int j = N - 1; j >= 0; --j) dp_step_vjp(M, a, E, L, Y[j], H[j], zb, &pb);

    // split: segment columns
    static double A[NSEG][4][4], P[NSEG][4][3];
    const int idx[4] = {0, 1, 3, 4};
    int phi_nonzero = 0;
    for (int s = 0; s < NSEG; ++s) {
        const int first = s * SEG, last = first + SEG < N ? first + SEG : N;
        for (int b = 0; b < 4; ++b) {
            double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            v[idx[b]] = 1.0;
            ParBar q{0.0, 0.0, 0.0};
            for (int j = last - 1; j >= first; --j) dp_step_vjp(M, a, E, L, Y[j], H[j], v, &q);
            if (v[2] != 0.0) ++phi_nonzero;
            for (int i = 0; i < 4; ++i) A[s][b][i] = v[idx[i]];
            P[s][b][0] = q.E;
            P[s][b][1] = q.L;
            P[s][b][2] = q.a;
        }
    }
    auto combine = [&](bool last_first, double out[4], double par[3]) {
        double v[4] = {seed[0], seed[1], seed[3], seed[4]};
        par[0] = par[1] = par[2] = 0.0;
        for (int k = 0; k < NSEG; ++k) {
            const int s = last_first ? NSEG - 1 - k : k;
            double nv[4] = {0.0, 0.0, 0.0, 0.0};
            for (int b = 0; b < 4; ++b) {
                for (int i = 0; i < 4; ++i) nv[i] = std::fma(v[b], A[s][b][i], nv[i]);
                for (int i = 0; i < 3; ++i) par[i] = std::fma(v[b], P[s][b][i], par[i]);
            }
            for (int i = 0; i < 4; ++i) v[i] = nv[i];
        }
        for (int i = 0; i < 4; ++i) out[i] = v[i];
    };
    double v[4], par[3], vw[4], parw[3];
    combine(true, v, par);
    combine(false, vw, parw);
    const double seq[7] = {zb[0], zb[1], zb[3], zb[4], pb.E, pb.L, pb.a};
    const double spl[7] = {v[0], v[1], v[2], v[3], par[0], par[1], par[2]};
    const double wrong[7] = {vw[0], vw[1], vw[2], vw[3], parw[0], parw[1], parw[2]};
    double scale = 0.0, err = 0.0, err_wrong = 0.0;
    for (int i = 0; i < 7; ++i) scale = std::fmax(scale, std::fabs(seq[i]));
    for (int i = 0; i < 7; ++i) {
        err = std::fmax(err, std::fabs(spl[i] - seq[i]) / scale);
        err_wrong = std::fmax(err_wrong, std::fabs(wrong[i] - seq[i]) / scale);
    }
    std::printf("r_end %.6f scale %.6e phi_cotangent_sequential %.3e\n", y[0], scale, zb[2]);
    std::printf("phi_nonzero %d split_err %.3e wrong_order_err %.3e\n", phi_nonzero, err, err_wrong);
    return 0;
}
