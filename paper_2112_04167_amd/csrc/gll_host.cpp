// GLL nodes, weights and differentiation matrix (host, FP64).
//
// Sec. 3.3 of arXiv 2112.04167 uses tensor-product Lagrange polynomials on
// Gauss-Lobatto-Legendre points.  Definitions used here:
//   nodes   -1, +1 and the roots of L_P' (Newton iteration on the Legendre
//           three-term recurrence, started from the Chebyshev-Lobatto points);
//   weights 2 / (P (P+1) L_P(x_j)^2);
//   D_ij    L_P(x_i) / (L_P(x_j) (x_i - x_j)) for i != j,
//           D_00 = -P(P+1)/4, D_PP = P(P+1)/4, zero otherwise on the diagonal.
#include <cmath>

#include "dg_internal.h"

namespace dg {

namespace {

// L_P(x), L_P'(x), L_P''(x) at an interior point |x| < 1
void legendre3(int P, double x, double &l, double &dl, double &d2l)
{
    double lm1 = 1.0, lc = x;
    if (P == 0) {
        l = 1.0;
        dl = d2l = 0.0;
        return;
    }
    for (int k = 2; k <= P; ++k) {
        double ln = ((2.0 * k - 1.0) * x * lc - (k - 1.0) * lm1) / k;
        lm1 = lc;
        lc = ln;
    }
    l = lc;
    dl = P * (lm1 - x * lc) / (1.0 - x * x);
    d2l = (2.0 * x * dl - P * (P + 1.0) * l) / (1.0 - x * x);
}

double legendre_value(int P, double x)
{
    if (P == 0) return 1.0;
    double lm1 = 1.0, lc = x;
    for (int k = 2; k <= P; ++k) {
        double ln = ((2.0 * k - 1.0) * x * lc - (k - 1.0) * lm1) / k;
        lm1 = lc;
        lc = ln;
    }
    return lc;
}

}  // namespace

GllTables make_gll(int P)
{
    GllTables t;
    t.P = P;
    const int n = P + 1;
    t.xi.assign(n, 0.0);
    t.w.assign(n, 0.0);
    t.D.assign(n * n, 0.0);
    t.K1.assign(n * n, 0.0);
    t.xi[0] = -1.0;
    t.xi[P] = 1.0;
    for (int j = 1; j < P; ++j) {
        double x = -std::cos(M_PI * j / P);
        for (int it = 0; it < 100; ++it) {
            double l, dl, d2l;
            legendre3(P, x, l, dl, d2l);
            double dx = dl / d2l;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        t.xi[j] = x;
    }
    // symmetrise the node set
    {
        std::vector<double> x0 = t.xi;
        for (int j = 0; j < n; ++j) t.xi[j] = 0.5 * (x0[j] - x0[P - j]);
    }
    std::vector<double> L(n);
    for (int j = 0; j < n; ++j) {
        L[j] = legendre_value(P, t.xi[j]);
        t.w[j] = 2.0 / (P * (P + 1.0) * L[j] * L[j]);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) t.D[i * n + j] = L[i] / (L[j] * (t.xi[i] - t.xi[j]));
    t.D[0] = -P * (P + 1.0) / 4.0;
    t.D[P * n + P] = P * (P + 1.0) / 4.0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += t.D[q * n + a] * t.w[q] * t.D[q * n + b];
            t.K1[a * n + b] = s;
        }
    return t;
}

}  // namespace dg
