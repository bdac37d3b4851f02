// adjoint_vjp_check.cpp -- test-only: the adjoint's step vector-Jacobian
// product (kt_adjoint_math.h) compiled for the host, against
//   (1) central differences of the frozen-step Dormand-Prince map built from
//       the same header's field(), and
//   (2) a variant that recomputes sin/cos of theta in the reverse loop
//       instead of keeping them from the forward pass (the form that gave
//       wrong gradients on the GPU): the two must agree bit for bit.
// Built with AddressSanitizer/UndefinedBehaviorSanitizer, MemorySanitizer,
// and with automatic variables initialised to a pattern and to zero; every
// build must print the same checksum line (an uninitialised read would show
// as a sanitizer report or as builds that disagree).
#include <cmath>
#include <cstdio>
#include <cstring>

#include "kt_adjoint_math.h"

using namespace kt;
using namespace kt::adj;

// The variant: stage sin/cos recomputed in the reverse loop.
static void dp_step_vjp_recompute(double M, double a, double E, double L, const double y[5], double h,
                                  double ybar[5], ParBar* pb) {
    double Y[6][5], K[5][5];
    for (int j = 0; j < 6; ++j) {
        for (int i = 0; i < 5; ++i) {
            double acc = 0.0;
            for (int l = 0; l < j; ++l) acc += dp_a(j, l) * K[l][i];
            Y[j][i] = y[i] + h * acc;
        }
        if (j < 5) {
            double s, c;
            field(M, a, E, L, Y[j], K[j], &s, &c);
        }
    }
    double kb[6][5];
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 5; ++i) kb[j][i] = h * dp_b(j) * ybar[i];
    for (int j = 5; j >= 0; --j) {
        double s, c;
        sincos_theta(Y[j][1], &s, &c);
        double Yb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        field_vjp(M, a, E, L, Y[j], s, c, kb[j], Yb, pb);
        for (int i = 0; i < 5; ++i) ybar[i] += Yb[i];
        for (int l = 0; l < j; ++l)
            for (int i = 0; i < 5; ++i) kb[l][i] += h * dp_a(j, l) * Yb[i];
    }
}

// The frozen-step map y -> y + h sum_j b_j k_j.
static void dp_step_map(double M, double a, double E, double L, const double y[5], double h, double out[5]) {
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

static unsigned long long g_state = 88172645463325252ull;
static double uniform(double lo, double hi) {
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return lo + (hi - lo) * (static_cast<double>(g_state >> 11) * (1.0 / 9007199254740992.0));
}

int main() {
    double checksum = 0.0, worst_fd = 0.0;
    int mismatches = 0;
    for (int t = 0; t < 200; ++t) {
        const double M = 1.0, a = uniform(-0.95, 0.95), E = uniform(0.8, 1.2), L = uniform(-4.0, 4.0);
        const double y[5] = {uniform(3.0, 60.0), uniform(0.3, 2.8), uniform(-1.0, 1.0), uniform(-1.0, 1.0),
                             uniform(-3.0, 3.0)};
        const double h = uniform(0.01, 0.5) * y[0] * 0.05;
        double v[5];
        for (double& x : v) x = uniform(-1.0, 1.0);
        double yb1[5], yb2[5];
        std::memcpy(yb1, v, sizeof v);
        std::memcpy(yb2, v, sizeof v);
        ParBar p1{0.0, 0.0, 0.0}, p2{0.0, 0.0, 0.0};
        dp_step_vjp(M, a, E, L, y, h, yb1, &p1);
        dp_step_vjp_recompute(M, a, E, L, y, h, yb2, &p2);
        if (std::memcmp(yb1, yb2, sizeof yb1) || p1.E != p2.E || p1.L != p2.L || p1.a != p2.a) ++mismatches;
        // central differences of v . map(y) in each state component
        for (int k = 0; k < 5; ++k) {
            double yp[5], ym[5], fp[5], fm[5];
            std::memcpy(yp, y, sizeof yp);
            std::memcpy(ym, y, sizeof ym);
            const double eps = 1e-6 * (std::fabs(y[k]) + 1.0);
            yp[k] += eps;
            ym[k] -= eps;
            dp_step_map(M, a, E, L, yp, h, fp);
            dp_step_map(M, a, E, L, ym, h, fm);
            double fd = 0.0;
            for (int i = 0; i < 5; ++i) fd += v[i] * (fp[i] - fm[i]) / (2.0 * eps);
            const double rel = std::fabs(fd - yb1[k]) / (std::fabs(fd) + 1e-3);
            if (rel > worst_fd) worst_fd = rel;
        }
        for (int i = 0; i < 5; ++i) checksum += yb1[i];
        checksum += p1.E + p1.L + p1.a;
    }
    std::printf("checksum %.17g mismatches %d worst_fd %.3e\n", checksum, mismatches, worst_fd);
    return (mismatches == 0 && worst_fd < 1e-6) ? 0 : 1;
}
