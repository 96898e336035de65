// Convective term of the momentum equation, F_c = -div(v v) (Sec. 3.1 of
// arXiv 2112.04167), by DG-SEM with consistent integration and local
// Lax-Friedrichs fluxes (Sec. 3.3), gfx950.
//
// Weak form per component i, with phi a velocity basis function (degree P,
// GLL nodes) and n the outward normal of element K:
//
//   (M F_c,i)_phi = sum_K int_K sum_k v_k v_i d_k phi - sum_K int_dK H_i phi,
//   H_i = ((v-.n) v-_i + (v+.n) v+_i) / 2 + alpha (v-_i - v+_i) / 2,
//   alpha = 2 max(|v-.n|, |v+.n|)   (spectral radius of d((u.n)u)/du),
//
// v- the element's trace, v+ the neighbour's (periodic axes wrap) or the
// wall state v_b (zero when not given).  Every integral uses Q = floor(3P/2)+1
// Gauss-Legendre points per direction, which integrates the polynomial part
// (degree 3P per direction) exactly; M is the diagonal GLL mass.
//
// One work-group of 256 threads per element.  The element's velocity is
// interpolated to the Q^3 Gauss points (three 1D passes, the three
// components together, in LDS).  Per output component i the nine (i, k)
// flux passes back to the nodes are factored into three: the z pass forms
// the three products v_i v_k on the fly, the y pass combines the k = 1, 2
// branches that share B_x, the x pass the remaining two.  Then both faces of
// each axis at once, each element computing the fluxes of its own faces (no
// atomics: the neighbour computes the same flux with the opposite sign).
// In every pass a thread owns whole 1D lines (see the line contractions
// below).  LDS at P = 7: 78 KB (two work-groups per CU); at P = 8: 121 KB.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "convection.h"
#include "device_common.h"
#include "dg_internal.h"
#include "gll_constexpr.h"

namespace dg {

namespace {


__host__ __device__ constexpr int conv_q(int P) { return 3 * P / 2 + 1; }

// Compile-time tables of degree P: the GLL basis l_a and its derivative at
// the Q Gauss-Legendre points, the Gauss weights and the GLL weights (the
// mass).  The Gauss points are the roots of L_Q, by Newton's method on the
// Legendre recurrence from the starting points -cos(pi (j + 3/4) / (Q + 1/2)),
// then symmetrised; the weights are 2 / ((1 - x^2) L_Q'(x)^2).
//
// Both point sets are symmetric about 0, so B[Q-1-q][n-1-a] = B[q][a] and
// dB[Q-1-q][n-1-a] = -dB[q][a], and every contraction splits into an even
// and an odd half (Solomonoff's even-odd decomposition): with e, o the sums
// and differences of mirrored inputs, half the multiply-adds and half the
// distinct coefficients.  The half tables (h = floor, the middle row or
// column of an odd size taken alone, so that the vanishing half of it is
// never formed):
//   nodes -> Gauss points, y = B x:       FE, FO [q < ceil(Q/2)][a < n/2], FM[q] = B[q][mid];
//   Gauss points -> nodes, y = B^T x:     TE [a < ceil(n/2)][q < Q/2], TO [a < n/2][q < Q/2], TM[a] = B[Q/2][a];
//   Gauss points -> nodes, y = dB^T x:    DE [a < ceil(n/2)][q < Q/2] (on o), DO [a < n/2][q < Q/2] (on e),
//                                         DM[a] = dB[Q/2][a].
// Every index is a compile-time constant where the kernel uses them, so the
// compiler emits the coefficients as immediates.
template <int P>
struct ConvTab {
    static constexpr int n = P + 1, Q = conv_q(P);
    static constexpr int hn = n / 2, hq = Q / 2, NN = (n + 1) / 2, NQ = (Q + 1) / 2;
    double B[Q][n];   // B[q][a] = l_a(x_q)
    double dB[Q][n];  // its derivative on [-1, 1]
    double wg[Q];     // Gauss weights
    double w[n];      // GLL weights
    double FE[NQ][hn > 0 ? hn : 1], FO[NQ][hn > 0 ? hn : 1], FM[NQ];
    double TE[NN][hq > 0 ? hq : 1], TO[NN][hq > 0 ? hq : 1], TM[NN];
    double DE[NN][hq > 0 ? hq : 1], DO[NN][hq > 0 ? hq : 1], DM[NN];

    constexpr ConvTab()
        : B(), dB(), wg(), w(), FE(), FO(), FM(), TE(), TO(), TM(), DE(), DO(), DM()
    {
        const double pi = 3.14159265358979323846;
        double x0[Q] = {};
        for (int j = 0; j < Q; ++j) {
            double x = -cx::cos0(pi * (j + 0.75) / (Q + 0.5));
            for (int it = 0; it < 100; ++it) {
                const cx::Leg L = cx::legendre(Q, x);
                const double dx = L.l / L.dl;
                x -= dx;
                if (cx::abs(dx) < 1e-16) break;
            }
            x0[j] = x;
        }
        double xg[Q] = {};
        for (int j = 0; j < Q; ++j) xg[j] = 0.5 * (x0[j] - x0[Q - 1 - j]);
        for (int j = 0; j < Q; ++j) {
            const double dl = cx::legendre(Q, xg[j]).dl;
            wg[j] = 2.0 / ((1.0 - xg[j] * xg[j]) * dl * dl);
        }
        const GllC<P> &g = kGll<P>;
        for (int a = 0; a < n; ++a) w[a] = g.w[a];
        for (int q = 0; q < Q; ++q)
            for (int a = 0; a < n; ++a) {
                double l = 1.0, dl = 0.0;
                for (int k = 0; k < n; ++k) {
                    if (k == a) continue;
                    const double r = 1.0 / (g.xi[a] - g.xi[k]);
                    dl = dl * (xg[q] - g.xi[k]) * r + l * r;
                    l *= (xg[q] - g.xi[k]) * r;
                }
                B[q][a] = l;
                dB[q][a] = dl;
            }
        for (int q = 0; q < NQ; ++q) {
            for (int a = 0; a < hn; ++a) {
                FE[q][a] = 0.5 * (B[q][a] + B[q][n - 1 - a]);
                FO[q][a] = 0.5 * (B[q][a] - B[q][n - 1 - a]);
            }
            FM[q] = (n % 2) ? B[q][hn] : 0.0;
        }
        for (int a = 0; a < NN; ++a) {
            for (int q = 0; q < hq; ++q) {
                TE[a][q] = 0.5 * (B[q][a] + B[Q - 1 - q][a]);
                TO[a][q] = 0.5 * (B[q][a] - B[Q - 1 - q][a]);
                DE[a][q] = 0.5 * (dB[q][a] - dB[Q - 1 - q][a]);
                DO[a][q] = 0.5 * (dB[q][a] + dB[Q - 1 - q][a]);
            }
            TM[a] = (Q % 2) ? B[hq][a] : 0.0;
            DM[a] = (Q % 2) ? dB[hq][a] : 0.0;
        }
    }
};

template <int P>
__constant__ ConvTab<P> c_conv = ConvTab<P>();

struct ConvArgs {
    const double *v[3];
    const double *vb[3];   // wall state (null: zero)
    double *out[3];
    const double *h[3];
    int n[3], bc[3];
    double scale;
    int accumulate;        // out += scale F_c instead of out = scale F_c
};

template <int P>
struct ConvLds {
    static constexpr int n = P + 1, Q = conv_q(P);
    // region A: the first interpolation pass Y1[3][n^2 Q], then the velocity
    // at the Gauss points U[3][Q^3]
    static constexpr int A = 3 * Q * Q * Q;
    // region S, after A: the second interpolation pass Y2[3][n Q^2], then the
    // transposed passes Z[3][n Q^2], Yb[2][n^2 Q]
    static constexpr int S = 3 * n * Q * Q + 2 * n * n * Q;
    // the face passes, all three axes at once: tg[3][12][Q^2] with, after
    // it, tq[3][12][n Q] and later hw[3][6][Q^2]; then hq[3][6][Q n] and
    // FB[3][6][n^2] from the start
    static constexpr int F = 36 * Q * Q + (36 * n * Q > 18 * Q * Q ? 36 * n * Q : 18 * Q * Q);
    static constexpr int ARENA = A + S > F ? A + S : F;
};

__device__ __forceinline__ int nb_index(int k, int nk, int bc, bool high)
{
    int kn = high ? k + 1 : k - 1;
    if (kn < 0 || kn >= nk) {
        if (bc != DG_BC_PERIODIC) return -1;
        kn = (kn + nk) % nk;
    }
    return kn;
}

// node (s, t) of the face layer `layer` normal to axis d, s on the lower
// tangential axis
template <int n>
__device__ __forceinline__ int layer_node(int d, int layer, int s, int t)
{
    return d == 0 ? (t * n + s) * n + layer : d == 1 ? (t * n + layer) * n + s : (layer * n + t) * n + s;
}

// Line contractions with the 1D tables.  Each thread owns whole lines and
// every loop over a table is unrolled, so the table entries have
// compile-time indices and are read with scalar loads from the kernel
// arguments; only the data lines go through LDS (or come from global
// memory).  Work split across threads by a compile-time range (C0, CN) is
// chosen per group of whole waves, so that both halves keep compile-time
// indices without divergence.

// even and odd halves of a line of Q values at the Gauss points
template <int P>
struct EoQ {
    static constexpr int Q = conv_q(P), hq = Q / 2;
    double e[hq > 0 ? hq : 1], o[hq > 0 ? hq : 1], m;
};

template <int P>
__device__ __forceinline__ void split_q(const double (&x)[conv_q(P)], EoQ<P> &s)
{
    constexpr int Q = conv_q(P), hq = Q / 2;
#pragma unroll
    for (int q = 0; q < hq; ++q) {
        s.e[q] = x[q] + x[Q - 1 - q];
        s.o[q] = x[q] - x[Q - 1 - q];
    }
    s.m = (Q % 2) ? x[hq] : 0.0;
}

// the even (E) and odd (O) parts of node pair (a, n-1-a) of B^T x, added to E, O
template <int P>
__device__ __forceinline__ void pair_bt(const ConvTab<P> &T, int a, const EoQ<P> &s, double &E, double &O)
{
    constexpr int n = P + 1, Q = conv_q(P), hq = Q / 2, hn = n / 2;
#pragma unroll
    for (int q = 0; q < hq; ++q) E = fma(T.TE[a][q], s.e[q], E);
    if (Q % 2) E = fma(T.TM[a], s.m, E);
    if (a < hn)
#pragma unroll
        for (int q = 0; q < hq; ++q) O = fma(T.TO[a][q], s.o[q], O);
}

// the same for dB^T x
template <int P>
__device__ __forceinline__ void pair_dbt(const ConvTab<P> &T, int a, const EoQ<P> &s, double &E, double &O)
{
    constexpr int n = P + 1, Q = conv_q(P), hq = Q / 2, hn = n / 2;
#pragma unroll
    for (int q = 0; q < hq; ++q) E = fma(T.DE[a][q], s.o[q], E);
    if (a < hn) {
#pragma unroll
        for (int q = 0; q < hq; ++q) O = fma(T.DO[a][q], s.e[q], O);
        if (Q % 2) O = fma(T.DM[a], s.m, O);
    }
}

// y[q] = sum_a B[q][a] x[a]: nodes to Gauss points
template <int P, int n = P + 1, int Q = conv_q(P)>
__device__ __forceinline__ void to_gauss(const ConvTab<P> &T, const double (&x)[n], double (&y)[Q])
{
    constexpr int hn = n / 2, hq = Q / 2, NQ = (Q + 1) / 2;
    double e[hn > 0 ? hn : 1], o[hn > 0 ? hn : 1];
#pragma unroll
    for (int a = 0; a < hn; ++a) {
        e[a] = x[a] + x[n - 1 - a];
        o[a] = x[a] - x[n - 1 - a];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double E = 0.0;
#pragma unroll
        for (int a = 0; a < hn; ++a) E = fma(T.FE[q][a], e[a], E);
        if (n % 2) E = fma(T.FM[q], x[hn], E);
        if (q < hq) {
            double O = 0.0;
#pragma unroll
            for (int a = 0; a < hn; ++a) O = fma(T.FO[q][a], o[a], O);
            y[q] = E + O;
            y[Q - 1 - q] = E - O;
        } else {
            y[q] = E;  // the middle point of an odd Q
        }
    }
}

// y[a] = sum_q B[q][a] x[q]: Gauss points back to nodes (B^T)
template <int P, int n = P + 1, int Q = conv_q(P)>
__device__ __forceinline__ void to_nodes(const ConvTab<P> &T, const double (&x)[Q], double (&y)[n])
{
    constexpr int hn = n / 2, NN = (n + 1) / 2;
    EoQ<P> s;
    split_q<P>(x, s);
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        double E = 0.0, O = 0.0;
        pair_bt<P>(T, a, s, E, O);
        if (a < hn) {
            y[a] = E + O;
            y[n - 1 - a] = E - O;
        } else {
            y[a] = E;  // the middle node of an odd n
        }
    }
}

// store node pair a of a line: y[a] = E + O, y[n-1-a] = E - O (the middle
// node of an odd line: E), each times f, at stride st from y0
template <int P>
__device__ __forceinline__ void store_pair(double *y0, int st, int a, double E, double O, double f)
{
    constexpr int n = P + 1, hn = n / 2;
    if (a < hn) {
        y0[a * st] = (E + O) * f;
        y0[(n - 1 - a) * st] = (E - O) * f;
    } else {
        y0[a * st] = E * f;
    }
}

// z pass of the volume term for output component i, Gauss column qxy, node
// pairs c in [C0, C0 + CN): Z_k[c][qxy] = f_k sum_qz T_k[qz][c] wg_qz U_i U_k
// with T_0 = T_1 = B, T_2 = dB
template <int P, int C0, int CN>
__device__ __forceinline__ void vol_z(const ConvTab<P> &T, const double *U, int i, int qxy, double f0,
                                      double f1, double f2, double *Z)
{
    constexpr int n = P + 1, Q = conv_q(P);
    constexpr int Q2 = Q * Q, Q3 = Q2 * Q, nQ2 = n * Q2;
    if constexpr (CN > 0) {
        double p0[Q], p1[Q], p2[Q];
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
            const int q = qz * Q2 + qxy;
            const double u0 = U[q], u1 = U[Q3 + q], u2 = U[2 * Q3 + q];
            const double ui = (i == 0 ? u0 : i == 1 ? u1 : u2) * T.wg[qz];
            p0[qz] = ui * u0;
            p1[qz] = ui * u1;
            p2[qz] = ui * u2;
        }
        EoQ<P> s0, s1, s2;
        split_q<P>(p0, s0);
        split_q<P>(p1, s1);
        split_q<P>(p2, s2);
#pragma unroll
        for (int c = C0; c < C0 + CN; ++c) {
            double E0 = 0.0, O0 = 0.0, E1 = 0.0, O1 = 0.0, E2 = 0.0, O2 = 0.0;
            pair_bt<P>(T, c, s0, E0, O0);
            pair_bt<P>(T, c, s1, E1, O1);
            pair_dbt<P>(T, c, s2, E2, O2);
            store_pair<P>(Z + qxy, Q2, c, E0, O0, f0);
            store_pair<P>(Z + nQ2 + qxy, Q2, c, E1, O1, f1);
            store_pair<P>(Z + 2 * nQ2 + qxy, Q2, c, E2, O2, f2);
        }
    }
}

// y pass, line (c, qx), node pairs b in [B0, B0 + BN):
// Yx = B_y^T Z_0, Ys = dB_y^T Z_1 + B_y^T Z_2
template <int P, int B0, int BN>
__device__ __forceinline__ void vol_y(const ConvTab<P> &T, const double *Z, int c, int qx, double *Yb)
{
    constexpr int n = P + 1, Q = conv_q(P);
    constexpr int nQ2 = n * Q * Q, n2Q = n * n * Q;
    if constexpr (BN > 0) {
        double z0[Q], z1[Q], z2[Q];
#pragma unroll
        for (int qy = 0; qy < Q; ++qy) {
            const int zi = (c * Q + qy) * Q + qx;
            z0[qy] = Z[zi];
            z1[qy] = Z[nQ2 + zi];
            z2[qy] = Z[2 * nQ2 + zi];
        }
        EoQ<P> s0, s1, s2;
        split_q<P>(z0, s0);
        split_q<P>(z1, s1);
        split_q<P>(z2, s2);
#pragma unroll
        for (int b = B0; b < B0 + BN; ++b) {
            double Ex = 0.0, Ox = 0.0, Es = 0.0, Os = 0.0;
            pair_bt<P>(T, b, s0, Ex, Ox);
            pair_dbt<P>(T, b, s1, Es, Os);
            pair_bt<P>(T, b, s2, Es, Os);
            store_pair<P>(Yb + c * n * Q + qx, Q, b, Ex, Ox, 1.0);
            store_pair<P>(Yb + n2Q + c * n * Q + qx, Q, b, Es, Os, 1.0);
        }
    }
}

// x pass, line (c, b) = cb, node pairs a in [A0, A0 + AN): acc = dB_x^T Yx + B_x^T Ys
template <int P, int A0, int AN>
__device__ __forceinline__ void vol_x(const ConvTab<P> &T, const double *Yb, int cb, double *acc)
{
    constexpr int n = P + 1, Q = conv_q(P);
    constexpr int n2Q = n * n * Q;
    if constexpr (AN > 0) {
        double yx[Q], ys[Q];
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
            yx[qx] = Yb[cb * Q + qx];
            ys[qx] = Yb[n2Q + cb * Q + qx];
        }
        EoQ<P> sx, ss;
        split_q<P>(yx, sx);
        split_q<P>(ys, ss);
#pragma unroll
        for (int a = A0; a < A0 + AN; ++a) {
            double E = 0.0, O = 0.0;
            pair_dbt<P>(T, a, sx, E, O);
            pair_bt<P>(T, a, ss, E, O);
            store_pair<P>(acc + cb * n, 1, a, E, O, 1.0);
        }
    }
}

template <int P>
__global__ void __launch_bounds__(256) k_convection(ConvArgs A)
{
    using L = ConvLds<P>;
    constexpr int n = L::n, Q = L::Q, n2 = n * n, n3 = n2 * n, Q2 = Q * Q;
    constexpr int nQ2 = n * Q2, n2Q = n2 * Q;
    constexpr int NT = 256;                    // threads per work-group (the launch's block size)
    constexpr int H = (n + 1) / 2;             // the lines c and c + H of the y interpolation pass
    constexpr int NN = (n + 1) / 2, PH = (NN + 1) / 2;  // node pairs, split [0, PH), [PH, NN)
    constexpr int WZ = (Q2 + 63) / 64 * 64;    // thread slots per half of a pass, whole waves
    constexpr int WY = (n * Q + 63) / 64 * 64;
    constexpr int WX = (n2 + 63) / 64 * 64;
    __shared__ double arena[L::ARENA];
    double *bufA = arena, *bufS = arena + L::A;
    __shared__ double acc[3][n3];
    // the weights used with lane-dependent indices
    __shared__ double twg[Q], tw[n];
    const int tid = threadIdx.x;
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const double J = hh[0] * hh[1] * hh[2] * 0.125;
    const size_t base = (size_t)el * n3;
    const ConvTab<P> &T = c_conv<P>;
    if (tid < Q) twg[tid] = T.wg[tid];
    if (tid < n) tw[tid] = T.w[tid];

    // ---- velocity at the Gauss points, U_k = (B (x) B (x) B) v_k, the three
    //      components together: x lines from global memory into Y1 (region
    //      A), y lines into Y2 (region S), z lines into U (region A again)
    double *Y1 = bufA, *Y2 = bufS, *U = bufA;
    for (int r = tid; r < 3 * n2; r += NT) {  // Y1[k][c][b][qx]
        const int k = r / n2, cb = r - k * n2;
        const double *src = (k == 0 ? A.v[0] : k == 1 ? A.v[1] : A.v[2]) + base + (size_t)cb * n;
        double x[n], y[Q];
#pragma unroll
        for (int a = 0; a < n; ++a) x[a] = src[a];
        to_gauss<P>(T, x, y);
#pragma unroll
        for (int q = 0; q < Q; ++q) Y1[r * Q + q] = y[q];
    }
    __syncthreads();
    for (int r = tid; r < 3 * H * Q; r += NT) {  // Y2[k][c][qy][qx], lines c and c + H
        const int qx = r % Q, kh = r / Q, k = kh / H, c0 = kh - k * H;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = c0 + h * H;
            if (c < n) {
                const int kc = k * n + c;
                double x[n], y[Q];
#pragma unroll
                for (int b = 0; b < n; ++b) x[b] = Y1[(kc * n + b) * Q + qx];
                to_gauss<P>(T, x, y);
#pragma unroll
                for (int q = 0; q < Q; ++q) Y2[(kc * Q + q) * Q + qx] = y[q];
            }
        }
    }
    __syncthreads();
    constexpr int HQ = (Q2 + 1) / 2;
    for (int r = tid; r < 3 * HQ; r += NT) {  // U[k][qz][qy][qx], columns p and p + HQ
        const int k = r / HQ, p = r - k * HQ;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int qxy = p + h * HQ;
            if (qxy < Q2) {
                double x[n], y[Q];
#pragma unroll
                for (int c = 0; c < n; ++c) x[c] = Y2[(k * n + c) * Q2 + qxy];
                to_gauss<P>(T, x, y);
#pragma unroll
                for (int q = 0; q < Q; ++q) U[(k * Q + q) * Q2 + qxy] = y[q];
            }
        }
    }
    __syncthreads();

    // ---- volume: acc_i = sum_k T_k^T (W J v_i v_k) with T_k = (2/h_k) dB along
    //      k and B along the others, factored as
    //      B_x^T [B_y^T dB_z^T F_i2 + dB_y^T B_z^T F_i1] + dB_x^T B_y^T B_z^T F_i0.
    //      Z (region S) and Yb (region S, after Z) do not overlap, so the x
    //      pass of component i and the z pass of i + 1 need no barrier
    //      between them.
    double *Z = bufS, *Yb = bufS + 3 * nQ2;
    const double g0 = 2.0 / hh[0], g1 = 2.0 / hh[1], g2 = 2.0 / hh[2];
    for (int i = 0; i < 3; ++i) {
        for (int r = tid; r < 2 * WZ; r += NT) {
            const int hf = r / WZ, qxy = r - hf * WZ;
            if (qxy < Q2) {
                const double f = twg[qxy % Q] * twg[qxy / Q] * J;
                if (hf == 0)
                    vol_z<P, 0, PH>(T, U, i, qxy, f * g0, f * g1, f * g2, Z);
                else
                    vol_z<P, PH, NN - PH>(T, U, i, qxy, f * g0, f * g1, f * g2, Z);
            }
        }
        __syncthreads();
        for (int r = tid; r < 2 * WY; r += NT) {
            const int hf = r / WY, cq = r - hf * WY;
            if (cq < n * Q) {
                if (hf == 0)
                    vol_y<P, 0, PH>(T, Z, cq / Q, cq % Q, Yb);
                else
                    vol_y<P, PH, NN - PH>(T, Z, cq / Q, cq % Q, Yb);
            }
        }
        __syncthreads();
        for (int r = tid; r < 2 * WX; r += NT) {
            const int hf = r / WX, cb = r - hf * WX;
            if (cb < n2) {
                if (hf == 0)
                    vol_x<P, 0, PH>(T, Yb, cb, acc[i]);
                else
                    vol_x<P, PH, NN - PH>(T, Yb, cb, acc[i]);
            }
        }
    }

    // ---- faces: acc_i -= int_F H_i phi, the six faces at once.  Slots:
    //      side * 6 + (own v_0..2, exterior v_0..2) per axis d, side 0 the
    //      low face and 1 the high one.  The two face layers of each axis
    //      receive their contributions in FB, added to acc in the output
    //      pass (the layers of different axes share edge nodes).
    constexpr int FS = 36 * Q2;                  // tg [3][12][Q][Q], then hq [3][6][Q][n] and FB
    double *tg = arena;                          // (qt, qs)
    double *tq = arena + FS;                     // [3][12][n][Q]: (t, qs)
    double *hw = arena + FS;                     // [3][6][Q][Q], after tq
    double *hq = arena;                          // [3][6][Q][n], after tg: (qt, s)
    double *FB = arena + 18 * Q * n;             // [3][6][n][n]: (t, s)
    __syncthreads();  // tq overwrites the volume's Yb
    for (int r = tid; r < 36 * n; r += NT) {  // the face lines along s, to the Gauss points
        const int d = r / (12 * n), slot = (r / n) % 12, t = r % n;
        const bool high = slot >= 6;
        const int comp = slot % 6, c3 = comp % 3;
        const double *src = nullptr;
        int lay = high ? n - 1 : 0;
        if (comp < 3) {
            src = (c3 == 0 ? A.v[0] : c3 == 1 ? A.v[1] : A.v[2]) + base;
        } else {
            const int kn = nb_index(e3[d], A.n[d], A.bc[d], high);
            if (kn >= 0) {
                int en[3] = {ex, ey, ez};
                en[d] = kn;
                src = (c3 == 0 ? A.v[0] : c3 == 1 ? A.v[1] : A.v[2]) +
                      ((size_t)(en[2] * A.n[1] + en[1]) * A.n[0] + en[0]) * n3;
                lay = high ? 0 : n - 1;
            } else {
                const double *wb = c3 == 0 ? A.vb[0] : c3 == 1 ? A.vb[1] : A.vb[2];
                src = wb ? wb + base : nullptr;
            }
        }
        double x[n], y[Q];
#pragma unroll
        for (int s = 0; s < n; ++s) x[s] = src ? src[layer_node<n>(d, lay, s, t)] : 0.0;
        to_gauss<P>(T, x, y);
#pragma unroll
        for (int q = 0; q < Q; ++q) tq[r * Q + q] = y[q];
    }
    __syncthreads();
    for (int r = tid; r < 36 * Q; r += NT) {  // along t: line (d, slot, qs)
        const int ds = r / Q, qs = r % Q;
        double x[n], y[Q];
#pragma unroll
        for (int t = 0; t < n; ++t) x[t] = tq[(ds * n + t) * Q + qs];
        to_gauss<P>(T, x, y);
#pragma unroll
        for (int q = 0; q < Q; ++q) tg[(ds * Q + q) * Q + qs] = y[q];
    }
    __syncthreads();
    for (int r = tid; r < 6 * Q2; r += NT) {  // the fluxes, weighted: point (d, side, q)
        const int ds = r / Q2, q = r % Q2, qs = q % Q, qt = q / Q;
        const int d = ds / 2, side = ds % 2;
        const double om0 = (d == 0 ? hh[1] * hh[2] : d == 1 ? hh[0] * hh[2] : hh[0] * hh[1]) * 0.25;
        const double sgn = side ? 1.0 : -1.0;
        const double *own = tg + (d * 12 + side * 6) * Q2, *ext = own + 3 * Q2;
        const double vm = sgn * own[d * Q2 + q], vp = sgn * ext[d * Q2 + q];
        const double alpha = 2.0 * fmax(fabs(vm), fabs(vp));
        const double om = om0 * twg[qs] * twg[qt];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double um = own[i * Q2 + q], up = ext[i * Q2 + q];
            hw[(ds * 3 + i) * Q2 + q] = -om * (0.5 * (vm * um + vp * up) + 0.5 * alpha * (um - up));
        }
    }
    __syncthreads();
    for (int r = tid; r < 18 * Q; r += NT) {  // back along s: line (d, side*3+i, qt)
        const int slot = r / Q, qt = r % Q;
        double x[Q], y[n];
#pragma unroll
        for (int q = 0; q < Q; ++q) x[q] = hw[(slot * Q + qt) * Q + q];
        to_nodes<P>(T, x, y);
#pragma unroll
        for (int s = 0; s < n; ++s) hq[(slot * Q + qt) * n + s] = y[s];
    }
    __syncthreads();
    for (int r = tid; r < 18 * n; r += NT) {  // back along t onto the face layers: line (d, side*3+i, s)
        const int slot = r / n, s = r % n;
        double x[Q], y[n];
#pragma unroll
        for (int q = 0; q < Q; ++q) x[q] = hq[(slot * Q + q) * n + s];
        to_nodes<P>(T, x, y);
#pragma unroll
        for (int t = 0; t < n; ++t) FB[(slot * n + t) * n + s] = y[t];
    }
    __syncthreads();
    for (int r = tid; r < n3; r += NT) {
        const int a = r % n, b = (r / n) % n, c = r / n2;
        const double f = A.scale / (J * tw[a] * tw[b] * tw[c]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double sum = acc[i][r];
            if (a == 0 || a == n - 1) sum += FB[((0 * 6 + (a ? 3 : 0) + i) * n + c) * n + b];
            if (b == 0 || b == n - 1) sum += FB[((1 * 6 + (b ? 3 : 0) + i) * n + c) * n + a];
            if (c == 0 || c == n - 1) sum += FB[((2 * 6 + (c ? 3 : 0) + i) * n + b) * n + a];
            const double val = f * sum;
            A.out[i][base + r] = A.accumulate ? A.out[i][base + r] + val : val;
        }
    }
}

}  // namespace

int launch_convection(const MeshDev &m, const double *const v[3], const double *const vb[3], double scale,
                      bool accumulate, double *const out[3], hipStream_t s)
{
    ConvArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.v[d] = v[d];
        a.vb[d] = vb ? vb[d] : nullptr;
        a.out[d] = out[d];
        a.n[d] = m.n[d];
        a.bc[d] = m.bc[d];
    }
    a.h[0] = m.h64;
    a.h[1] = m.h64 + m.n[0];
    a.h[2] = m.h64 + m.n[0] + m.n[1];
    a.scale = scale;
    a.accumulate = accumulate ? 1 : 0;
    const dim3 grid((unsigned)m.nel), block(256);
    switch (m.P) {
        case 3: hipLaunchKernelGGL(k_convection<3>, grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_convection<4>, grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL(k_convection<5>, grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL(k_convection<6>, grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL(k_convection<7>, grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL(k_convection<8>, grid, block, 0, s, a); break;
        default: set_error("convection needs a degree 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
