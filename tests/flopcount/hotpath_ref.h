// hotpath_ref.h -- test-only: the per-unit arithmetic of the hot path written
// plainly, templated on the scalar so that a counting scalar (flop.h) counts
// it.  Kerr's right-hand side is in Carter's separated form: the same
// function as Hamilton's equations with the matrix inverse of eq:Kerr,
// without the components and derivatives that cancel.  The q-metric's is
// written from its four diagonal contravariant components.  Names follow
// the paper's notation.
//
//   2 Sigma H = K = Delta p_r^2 + p_th^2 + T^2 - W^2 / Delta,
//   T = L / sin(theta) - a E sin(theta),  W = (r^2 + a^2) E - a L,
//   Sigma = r^2 + a^2 cos^2(theta),  Delta = r^2 - 2 M r + a^2.
#pragma once

template <class S>
struct RayConsts {
    S M, a, a2, E, L, aE, aL;  // per image (M, a, a^2) and per ray (E, L, aE, aL)
};

// Hamilton's equations: f = (dH/dp_r, dH/dp_th, dH/dL, -dH/dr, -dH/dtheta).
// With diag, also H and |H|_rel = |K| / (sum of the magnitudes of K's terms).
template <class S>
void carter_rhs(const RayConsts<S>& k, const S z[5], S f[5], bool diag, S* H, S* rel) {
    const S r = z[0], th = z[1], pr = z[3], pth = z[4];
    const S s = sin(th), c = cos(th);
    const S r2 = r * r;
    const S Sig = r2 + k.a2 * c * c;
    const S Del = r2 - 2.0 * k.M * r + k.a2;
    const S W = (r2 + k.a2) * k.E - k.aL;
    const S T = k.L / s - k.aE * s;
    const S pr2 = pr * pr, pth2 = pth * pth, T2 = T * T;
    const S WD = W / Del;
    const S W2D = W * WD;
    const S DP = Del * pr2;
    const S K = DP + pth2 + T2 - W2D;
    const S H2 = K / Sig;  // 2H
    f[0] = Del * pr / Sig;
    f[1] = pth / Sig;
    f[2] = (T / s + k.a * WD) / Sig;
    // (1/2) dK/dr = (r - M)(p_r^2 + (W/Delta)^2) - 2 r E W/Delta
    const S hKr = (r - k.M) * (pr2 + WD * WD) - 2.0 * r * k.E * WD;
    f[3] = (r * H2 - hKr) / Sig;
    // -dH/dtheta = cos(theta) [T (L/sin^2 + aE) - a^2 sin(theta) 2H] / Sigma
    f[4] = c * (T * (k.L / (s * s) + k.aE) - k.a2 * s * H2) / Sig;
    if (diag) {
        *H = 0.5 * H2;
        *rel = fabs(K) / (DP + pth2 + T2 + W2D);
    }
}

// Dormand & Prince (1980) RK5(4)7M, nonzero tableau entries only.
namespace dpref {
constexpr double A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
constexpr double B4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                          1.0 / 40};
}  // namespace dpref

// Stage state i (1..6, the 7th is the 5th-order solution) from the stage
// derivatives k[0..i-1]: y + h sum_j a_ij k_j.
template <class S>
void dp_stage(int i, const S y[5], const S k[7][5], S h, S out[5]) {
    for (int c = 0; c < 5; ++c) {
        S acc = 0.0;
        bool first = true;
        for (int j = 0; j < i; ++j) {
            if (dpref::A[i][j] == 0.0) continue;
            acc = first ? dpref::A[i][j] * k[j][c] : acc + dpref::A[i][j] * k[j][c];
            first = false;
        }
        out[c] = y[c] + h * acc;
    }
}

// Error estimate y5 - y4 = h sum_j (b5_j - b4_j) k_j.
template <class S>
void dp_error(const S k[7][5], S h, S e[5]) {
    for (int c = 0; c < 5; ++c) {
        S acc = 0.0;
        bool first = true;
        for (int j = 0; j < 7; ++j) {
            const double w = (j < 6 ? dpref::A[6][j] : 0.0) - dpref::B4[j];
            if (w == 0.0) continue;
            acc = first ? w * k[j][c] : acc + w * k[j][c];
            first = false;
        }
        e[c] = h * acc;
    }
}

// RMS error norm with sc_i = atol + rtol max(|y_i|, |y5_i|), and the new
// step size h 0.9 err^(-1/5) clamped to [0.2, 5] (5 for a negligible error).
template <class S>
S dp_control(const S y[5], const S yn[5], const S e[5], S rtol, S atol, S h, bool* accept) {
    S acc = 0.0;
    for (int c = 0; c < 5; ++c) {
        const S sc = atol + rtol * fmax(fabs(y[c]), fabs(yn[c]));
        const S q = e[c] / sc;
        acc = c == 0 ? q * q : acc + q * q;
    }
    const S err = sqrt(acc / 5.0);
    *accept = err <= 1.0;
    const S fac = err < 1e-10 ? S(5.0) : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    return h * fac;
}

// Great-circle angle between successive accepted positions (theta1, phi1)
// -> (theta2, phi2), given the unit vector n1 of the first: atan2(|n1 x n2|,
// n1.n2); writes n2 for the next step.  sin/cos of theta2 come from the
// FSAL evaluation at that state and are passed in.
template <class S>
S swept_arc(const S n1[3], S s2, S c2, S ph2, S n2[3]) {
    const S sp = sin(ph2), cp = cos(ph2);
    n2[0] = s2 * cp;
    n2[1] = s2 * sp;
    n2[2] = c2;
    const S cx = n1[1] * n2[2] - n1[2] * n2[1];
    const S cy = n1[2] * n2[0] - n1[0] * n2[2];
    const S cz = n1[0] * n2[1] - n1[1] * n2[0];
    return atan2(sqrt(cx * cx + cy * cy + cz * cz), n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
}

// The q-metric of the appendix (signature (-,+,+,+)): f = 1 - 2M/r,
// D = 1 + M^2 sin^2 / (r^2 f), P = q (2 + q);
//   -g^tt = G = f^-(1+q),  g^rr = A = f^(1+q) D^P,  g^thth = B = f^q D^P / r^2,
//   g^phph = C = f^q / (r^2 sin^2),
// H = (-E^2 G + p_r^2 A + p_th^2 B + L^2 C) / 2; each term's derivative is the
// term times the log-derivative of its component.  q1 = 1 + q and P are
// per-image constants.
template <class S>
void q_rhs(S M, S q, S q1, S P, S E, S L, const S z[5], S f[5], bool diag, S* H, S* rel) {
    const S r = z[0], th = z[1], pr = z[3], pth = z[4];
    const S s = sin(th), c = cos(th);
    const S r2 = r * r;
    const S rf = r2 - 2.0 * M * r;  // r^2 f
    const S fr = rf / r2;
    const S Dm1 = M * M * s * s / rf;
    const S D = 1.0 + Dm1;
    const S fq = pow(fr, q), DP = pow(D, P);
    const S A = fr * fq * DP, B = fq * DP / r2, C = fq / (r2 * s * s), G = 1.0 / (fr * fq);
    const S tG = E * E * G, tA = pr * pr * A, tB = pth * pth * B, tC = L * L * C;
    const S lf_r = 2.0 * M / rf;                            // d ln f / dr
    const S lD_r = -Dm1 * (2.0 * r - 2.0 * M) / (rf * D);   // d ln D / dr
    const S lD_th = 2.0 * Dm1 * c / (s * D);                // d ln D / dtheta
    const S two_r = 2.0 / r;
    const S Hr2 = tG * (q1 * lf_r) + tA * (q1 * lf_r + P * lD_r) + tB * (q * lf_r + P * lD_r - two_r)
                + tC * (q * lf_r - two_r);                  // 2 dH/dr
    const S Hth2 = (tA + tB) * (P * lD_th) - tC * (2.0 * c / s);  // 2 dH/dtheta
    f[0] = A * pr;
    f[1] = B * pth;
    f[2] = C * L;
    f[3] = -0.5 * Hr2;
    f[4] = -0.5 * Hth2;
    if (diag) {
        const S K = tA + tB + tC - tG;
        *H = 0.5 * K;
        *rel = fabs(K) / (tG + tA + tB + tC);
    }
}
