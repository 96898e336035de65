// Compile-time GLL tables for the kernels (degree P is a template parameter).
//
// Same definitions as gll_host.cpp (Sec. 3.3 of arXiv 2112.04167 places the
// nodes at the Gauss-Lobatto-Legendre points): interior nodes are the roots
// of L_P' (Newton on the Legendre recurrence), w_j = 2/(P(P+1) L_P(x_j)^2),
// D_ij = L_P(x_i)/(L_P(x_j)(x_i - x_j)), D_00 = -P(P+1)/4, D_PP = P(P+1)/4,
// and K1 = D^T diag(w) D.  Evaluated by the compiler, so every coefficient
// with a compile-time index becomes an immediate operand of the kernel code.
#pragma once

namespace dg {

namespace cx {

constexpr double abs(double x) { return x < 0 ? -x : x; }

// cos(x) for x in [0, pi] by its Taylor series around pi/2 (used only for
// Newton's starting points)
constexpr double cos0(double x)
{
    const double pi = 3.14159265358979323846;
    const double t = x - pi / 2;  // cos(x) = -sin(t)
    double term = t, s = 0.0;
    for (int k = 1; k < 40; k += 2) {
        s += term;
        term *= -t * t / ((k + 1.0) * (k + 2.0));
    }
    return -s;
}

struct Leg {
    double l, dl, d2l;
};

constexpr Leg legendre(int P, double x)
{
    double lm1 = 1.0, lc = x;
    for (int k = 2; k <= P; ++k) {
        const double ln = ((2.0 * k - 1.0) * x * lc - (k - 1.0) * lm1) / k;
        lm1 = lc;
        lc = ln;
    }
    Leg r{lc, 0.0, 0.0};
    if (x != 1.0 && x != -1.0) {
        r.dl = P * (lm1 - x * lc) / (1.0 - x * x);
        r.d2l = (2.0 * x * r.dl - P * (P + 1.0) * lc) / (1.0 - x * x);
    }
    return r;
}

}  // namespace cx

template <int P>
struct GllC {
    static constexpr int n = P + 1;
    double xi[n];
    double w[n];
    double D[n * n];
    double K1[n * n];
    // K0 = K1 - (e_P D_P^T + D_P e_P^T)/2 + (e_0 D_0^T + D_0 e_0^T)/2: the 1D
    // stiffness of a line plus the self-coupling of the consistency terms of
    // two interior faces (without penalty), in units of J g^2 w w nu
    double K0[n * n];

    constexpr GllC() : xi(), w(), D(), K1(), K0()
    {
        const double pi = 3.14159265358979323846;
        double x0[n] = {};
        x0[0] = -1.0;
        x0[P] = 1.0;
        for (int j = 1; j < P; ++j) {
            double x = -cx::cos0(pi * j / P);
            for (int it = 0; it < 100; ++it) {
                const cx::Leg L = cx::legendre(P, x);
                const double dx = L.dl / L.d2l;
                x -= dx;
                if (cx::abs(dx) < 1e-16) break;
            }
            x0[j] = x;
        }
        for (int j = 0; j < n; ++j) xi[j] = 0.5 * (x0[j] - x0[P - j]);
        double L[n] = {};
        for (int j = 0; j < n; ++j) {
            L[j] = cx::legendre(P, xi[j]).l;
            w[j] = 2.0 / (P * (P + 1.0) * L[j] * L[j]);
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                D[i * n + j] = (i != j) ? L[i] / (L[j] * (xi[i] - xi[j])) : 0.0;
        D[0] = -P * (P + 1.0) / 4.0;
        D[P * n + P] = P * (P + 1.0) / 4.0;
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double s = 0.0;
                for (int q = 0; q < n; ++q) s += D[q * n + a] * w[q] * D[q * n + b];
                K1[a * n + b] = s;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double k = K1[a * n + b];
                if (a == P) k -= 0.5 * D[P * n + b];
                if (b == P) k -= 0.5 * D[P * n + a];
                if (a == 0) k += 0.5 * D[b];
                if (b == 0) k += 0.5 * D[a];
                K0[a * n + b] = k;
            }
    }
};

template <int P>
inline constexpr GllC<P> kGll{};

}  // namespace dg
