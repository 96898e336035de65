// The matrix-free SIP-DG apply on one group of elements (device code shared
// by the stand-alone apply kernel and the persistent batched solver).
//
// Operator (arXiv 2112.04167, Sec. 3.3: DG-SEM on tensor-product GLL
// hexahedra with the interior penalty method; Alg. 3: the Helmholtz problem
// of the diffusion substep and the Poisson problem of the projection
// substep):  y = (lambda M + K_nu) x, all integrals by the GLL rule.
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "device_common.h"
#include "gll_constexpr.h"
#include "kernels.h"

namespace dg {

template <int P, typename T>
__device__ __forceinline__ T Dm(int k) { return (T)kGll<P>.D[k]; }
template <int P, typename T>
__device__ __forceinline__ T K1m(int k) { return (T)kGll<P>.K1[k]; }
template <int P, typename T>
__device__ __forceinline__ T Wm(int k) { return (T)kGll<P>.w[k]; }

// ------------------------------------------------- even-odd contractions --
//
// D is anti-persymmetric (D_{P-i,P-j} = -D_ij) and K0 is persymmetric
// (K0_{P-i,P-j} = K0_ij), so y = A u costs half the multiply-adds when u is
// split into e_j = u_j + u_{P-j} and o_j = u_j - u_{P-j} (the even-odd
// decomposition of Solomonoff, 1992):
//   y_i = E_i + O_i,  y_{P-i} = S (E_i - O_i),   i < (P+1)/2,
//   E_i = sum_j (A_ij + A_{i,P-j})/2 e_j (+ A_im u_m),  O_i = sum_j (A_ij - A_{i,P-j})/2 o_j,
// S = +1 (persymmetric) or -1 (anti-persymmetric); m = P/2 is the middle node
// of an odd-sized line.
//
// The coefficients live in __constant__ memory (one table per degree and
// precision, initialised at compile time from the GLL tables): with
// compile-time indices the kernels fetch them with wide scalar loads
// instead of materialising every FP64 immediate with scalar moves.
template <int P, typename T>
struct EoMat {
    static constexpr int n = P + 1, h = n / 2;
    T E[h * h], O[h * h];
    T colm[h > 0 ? h : 1], rowm[h > 0 ? h : 1], mm;
};

template <int P, typename T>
struct EoTab {
    static constexpr int n = P + 1, h = n / 2;
    EoMat<P, T> K0, D, Dt;
    T DPE[h + 1], DPO[h];  // (D_Pi +- D_{P,P-i})/2, middle entry D_Pm
    T DP[n], D0[n];        // rows P and 0 of D
    T w[n];
};

template <int P, typename T>
constexpr EoMat<P, T> make_eo_mat(const double *A)
{
    constexpr int n = P + 1, h = n / 2, m = P / 2;
    EoMat<P, T> r{};
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < h; ++j) {
            r.E[i * h + j] = (T)(0.5 * (A[i * n + j] + A[i * n + P - j]));
            r.O[i * h + j] = (T)(0.5 * (A[i * n + j] - A[i * n + P - j]));
        }
    for (int i = 0; i < h; ++i) {
        r.colm[i] = (T)A[i * n + m];
        r.rowm[i] = (T)A[m * n + i];
    }
    r.mm = (T)A[m * n + m];
    return r;
}

template <int P, typename T>
constexpr EoTab<P, T> make_eo_tab()
{
    constexpr int n = P + 1, h = n / 2;
    EoTab<P, T> t{};
    double Dt[n * n] = {};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Dt[i * n + j] = kGll<P>.D[j * n + i];
    t.K0 = make_eo_mat<P, T>(kGll<P>.K0);
    t.D = make_eo_mat<P, T>(kGll<P>.D);
    t.Dt = make_eo_mat<P, T>(Dt);
    for (int i = 0; i < h; ++i) {
        t.DPE[i] = (T)(0.5 * (kGll<P>.D[P * n + i] + kGll<P>.D[P * n + P - i]));
        t.DPO[i] = (T)(0.5 * (kGll<P>.D[P * n + i] - kGll<P>.D[P * n + P - i]));
    }
    t.DPE[h] = (T)kGll<P>.D[P * n + h < n * n ? P * n + h : 0];
    for (int j = 0; j < n; ++j) {
        t.DP[j] = (T)kGll<P>.D[P * n + j];
        t.D0[j] = (T)kGll<P>.D[j];
        t.w[j] = (T)kGll<P>.w[j];
    }
    return t;
}

template <int P, typename T>
__constant__ EoTab<P, T> c_eo = make_eo_tab<P, T>();

// The same table through a pointer the compiler cannot see through.  A
// persistent loop that takes the table from here at each use re-reads the
// entries with scalar loads close to where they are needed, instead of
// hoisting every entry out of the loop and spilling the scalar registers that
// hold them (each spilled value then costs a VALU readlane per use).
template <int P, typename T>
__device__ __forceinline__ const EoTab<P, T> &eo_fresh()
{
    auto p = (const __attribute__((address_space(4))) EoTab<P, T> *)&c_eo<P, T>;
    asm volatile("" : "+s"(p));
    return *(const EoTab<P, T> *)p;
}

// E, O halves of y = A u for the even-odd table M
template <int P, typename T, int S>
__device__ __forceinline__ void eo_apply(const EoMat<P, T> &M, const T (&u)[P + 1],
                                         T (&E)[(P + 2) / 2], T (&O)[(P + 2) / 2])
{
    constexpr int n = P + 1, h = n / 2, m = P / 2;
    constexpr bool odd = (n % 2) == 1;
    T e[h], o[h];
#pragma unroll
    for (int j = 0; j < h; ++j) {
        e[j] = u[j] + u[P - j];
        o[j] = u[j] - u[P - j];
    }
#pragma unroll
    for (int i = 0; i < h; ++i) {
        T se = 0, so = 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            se = fma(M.E[i * h + j], e[j], se);
            so = fma(M.O[i * h + j], o[j], so);
        }
        if constexpr (odd) se = fma(M.colm[i], u[m], se);
        E[i] = se;
        O[i] = so;
    }
    if constexpr (odd) {
        T s = 0;
        if constexpr (S > 0) {
#pragma unroll
            for (int j = 0; j < h; ++j) s = fma(M.rowm[j], e[j], s);
            s = fma(M.mm, u[m], s);
        } else {
#pragma unroll
            for (int j = 0; j < h; ++j) s = fma(M.rowm[j], o[j], s);
        }
        E[h] = s;
        O[h] = 0;
    }
}

template <int P, typename T, int S>
__device__ __forceinline__ void eo_combine(const T (&E)[(P + 2) / 2], const T (&O)[(P + 2) / 2],
                                           T (&y)[P + 1])
{
    constexpr int n = P + 1, h = n / 2;
#pragma unroll
    for (int i = 0; i < h; ++i) {
        y[i] = E[i] + O[i];
        y[P - i] = S > 0 ? E[i] - O[i] : O[i] - E[i];
    }
    if constexpr (n % 2 == 1) y[h] = E[h];
}

// ------------------------------------------------------ the 1D operator --
//
// One line u[0..P] of an element along an axis (extent h, g = 2/h), with
// rho = h / h_N for each face neighbour.  In units of vs = J g^2 wt nu
// (constant nu; wt = product of the two tangential GLL weights) the line's
// rows of A are
//
//   y = K0 u + a D_P. + b D_0. ,  y_0 += s_lo,  y_P += s_hi
//
// with, for the high end (neighbour R: trace uR, raw derivative sum
// sR = D_0.xR, rho = h/h_R, pen = sigma h / (2 nu)):
//   interior   s_hi = pen (u_P - uR) - rho sR / 2,  a =  uR / 2
//   Dirichlet  s_hi = pen u_P - (D_P.u) / 2,        a = -u_P / 2
//   natural    s_hi = (D_P.u) / 2,                   a =  u_P / 2
// and for the low end (neighbour L: uL, sL = D_P.xL):
//   interior   s_lo = pen (u_0 - uL) + rho sL / 2,  b = -uL / 2
//   Dirichlet  s_lo = pen u_0 + (D_0.u) / 2,        b =  u_0 / 2
//   natural    s_lo = -(D_0.u) / 2,                  b = -u_0 / 2
// (K0 already holds the self-coupling of two interior faces; the Dirichlet
// and natural ends are rank-2 corrections of it.)  These are the face
// integrals of the SIP form with sigma = nu (P+1)^2 / min(h, h_N) written
// per line.
template <int P, typename T>
__device__ __forceinline__ void line_const(const T (&u)[P + 1], int klo, int khi, T rhoL, T rhoR,
                                           T uL, T sL, T uR, T sR, T (&y)[P + 1],
                                           const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1, hh = (P + 2) / 2;
    T E[hh], O[hh];
    eo_apply<P, T, 1>(tb.K0, u, E, O);
    const T halfpen = (T)(0.5 * n * n);
    T a, b, slo, shi;
    if (khi == 1) {
        const T pen = halfpen * dmax((T)1, rhoR);
        shi = pen * (u[P] - uR) - (T)0.5 * rhoR * sR;
        a = (T)0.5 * uR;
    } else {
        T dPu = 0;
#pragma unroll
        for (int j = 0; j < n; ++j) dPu = fma(tb.DP[j], u[j], dPu);
        if (khi == 2) {
            shi = halfpen * u[P] - (T)0.5 * dPu;
            a = (T)-0.5 * u[P];
        } else {
            shi = (T)0.5 * dPu;
            a = (T)0.5 * u[P];
        }
    }
    if (klo == 1) {
        const T pen = halfpen * dmax((T)1, rhoL);
        slo = pen * (u[0] - uL) + (T)0.5 * rhoL * sL;
        b = (T)-0.5 * uL;
    } else {
        T d0u = 0;
#pragma unroll
        for (int j = 0; j < n; ++j) d0u = fma(tb.D0[j], u[j], d0u);
        if (klo == 2) {
            slo = halfpen * u[0] + (T)0.5 * d0u;
            b = (T)0.5 * u[0];
        } else {
            slo = (T)-0.5 * d0u;
            b = (T)-0.5 * u[0];
        }
    }
    // a D_P. + b D_0. in even-odd form: D_0j = -D_{P,P-j}
    const T amb = a - b, apb = a + b;
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
        E[i] = fma(amb, tb.DPE[i], E[i]);
        O[i] = fma(apb, tb.DPO[i], O[i]);
    }
    if constexpr (n % 2 == 1) E[n / 2] = fma(amb, tb.DPE[n / 2], E[n / 2]);
    eo_combine<P, T, 1>(E, O, y);
    y[0] += slo;
    y[P] += shi;
}

// Nodal nu: y = D^T diag(w nu) D u + face terms, in units of J g^2 wt.  The
// line-wide part of the consistency term (c D_f.) enters as c added to the
// scaled derivative t_f before the transposed contraction.
//   high end: interior  y_P += pen (u_P - uR) - nu_P t'_P / 2 - nu_R rho sR / 2,
//                       t_P += -nu_P (u_P - uR) / 2
//             Dirichlet y_P += pen u_P - nu_P t'_P,  t_P += -nu_P u_P
//   low end:  interior  y_0 += nu_L rho sL / 2 + nu_0 t'_0 / 2 - pen (uL - u_0),
//                       t_0 += -nu_0 (uL - u_0) / 2
//             Dirichlet y_0 += nu_0 t'_0 + pen u_0,  t_0 += nu_0 u_0
// with t' = D u, pen = (h/2) sigma, sigma = max(nu, nu_N)(P+1)^2/min(h, h_N),
// rho = h / h_N.
template <int P, typename T>
__device__ __forceinline__ void line_nodal(const T (&u)[P + 1], const T (&nl)[P + 1], int klo,
                                           int khi, T rhoL, T rhoR, T uL, T sL, T nuL, T uR, T sR,
                                           T nuR, T (&y)[P + 1],
                                           const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1, hh = (P + 2) / 2;
    T E[hh], O[hh], t[n];
    eo_apply<P, T, -1>(tb.D, u, E, O);
    eo_combine<P, T, -1>(E, O, t);
    const T halfpen = (T)(0.5 * n * n);
    T slo = 0, shi = 0;
    const T tP = t[P], t0 = t[0];
#pragma unroll
    for (int q = 0; q < n; ++q) t[q] *= tb.w[q] * nl[q];
    if (khi == 1) {
        const T pen = halfpen * dmax(nl[P], nuR) * dmax((T)1, rhoR);
        shi = pen * (u[P] - uR) - (T)0.5 * (nl[P] * tP + nuR * rhoR * sR);
        t[P] = fma((T)-0.5 * nl[P], u[P] - uR, t[P]);
    } else if (khi == 2) {
        shi = halfpen * nl[P] * u[P] - nl[P] * tP;
        t[P] = fma(-nl[P], u[P], t[P]);
    }
    if (klo == 1) {
        const T pen = halfpen * dmax(nl[0], nuL) * dmax((T)1, rhoL);
        slo = (T)0.5 * (nuL * rhoL * sL + nl[0] * t0) - pen * (uL - u[0]);
        t[0] = fma((T)-0.5 * nl[0], uL - u[0], t[0]);
    } else if (klo == 2) {
        slo = nl[0] * t0 + halfpen * nl[0] * u[0];
        t[0] = fma(nl[0], u[0], t[0]);
    }
    eo_apply<P, T, -1>(tb.Dt, t, E, O);
    eo_combine<P, T, -1>(E, O, y);
    y[0] += slo;
    y[P] += shi;
}

// neighbour line: trace at `layer` and the raw derivative sum D_layer . v
template <int P, typename T>
__device__ __forceinline__ void nb_line(const T *__restrict__ base, int stride, int layer,
                                        T &uN, T &sN, const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1;
    T v[n];
#pragma unroll
    for (int k = 0; k < n; ++k) v[k] = base[k * stride];
    T s = 0;
#pragma unroll
    for (int k = 0; k < n; ++k) s = fma(layer == 0 ? tb.D0[k] : tb.DP[k], v[k], s);
    uN = v[layer];
    sN = s;
}

// --------------------------------------------------------- apply kernel --

// Neighbour lines loaded per sweep rather than all up front: fewer registers
// and more resident waves.  Measured on gfx950 this wins 2-25 % for every
// degree and precision except FP32 at P = 3 and FP64 at P = 7 (within a few
// per cent either way there; the up-front loads are kept).
template <int P, typename T>
constexpr bool apply_lazy()
{
    return !(P == 3 && sizeof(T) == 4) && !(P == 7 && sizeof(T) == 8);
}

// Epilogue modes of the apply kernel
enum { EPI_STORE = 0, EPI_CG = 1, EPI_RESID = 2 };

template <typename T>
struct ApplyArgs {
    const T *x;
    T *y;
    const T *nu;
    T nu_c;
    T lambda;
    Geo<T> geo;
    int nel;
    int ngroups;
    const int *order;  // visiting order of the element groups (may be null)
    // EPI_CG: partial dot x.y and sum(y) (finished by a separate kernel).
    // EPI_RESID: y = b - A x, partial sums of (y/M)^2 and y, (y/M) and 1/M^2 sums
    const T *b;
    double *partial;
    CgScalars *sc;
};

// Neighbour data of one line at its two ends: trace and raw derivative sum
// of the face neighbour (and its nu at the shared node); zero where the end
// is not an interior / periodic face.
template <typename T>
struct LineNb {
    T uL, sL, uR, sR, nuL, nuR;
};

// Load the neighbour lines of the line starting at node offset `off` (stride
// `ls` inside the element) along an axis with element stride `estr`.  The
// loads are unconditional (a boundary end reads the element's own line and
// discards it) so that all of them can be in flight at once.
template <int P, typename T, bool NUF>
__device__ __forceinline__ void load_nb(const ApplyArgs<T> &A, int el, int k, int nk, int bc,
                                        int estr, int off, int ls, LineNb<T> &f,
                                        const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1, N3 = n * n * n;
    int kL, kR;
    const int klo = face_kind(k, nk, bc, false, kL);
    const int khi = face_kind(k, nk, bc, true, kR);
    const size_t bL = (size_t)(el + (kL - k) * estr) * N3 + off;
    const size_t bR = (size_t)(el + (kR - k) * estr) * N3 + off;
    T vL[n], vR[n];
#pragma unroll
    for (int q = 0; q < n; ++q) {
        vL[q] = A.x[bL + q * ls];
        vR[q] = A.x[bR + q * ls];
    }
    T nuL = A.nu_c, nuR = A.nu_c;
    if constexpr (NUF) {
        nuL = A.nu[bL + P * ls];
        nuR = A.nu[bR];
    }
    T sL = 0, sR = 0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
        sL = fma(tb.DP[q], vL[q], sL);
        sR = fma(tb.D0[q], vR[q], sR);
    }
    f.uL = klo == 1 ? vL[P] : (T)0;
    f.sL = klo == 1 ? sL : (T)0;
    f.uR = khi == 1 ? vR[0] : (T)0;
    f.sR = khi == 1 ? sR : (T)0;
    f.nuL = nuL;
    f.nuR = nuR;
}

// x-neighbour lines of a work-group of consecutive elements.  A face whose
// neighbour is the adjacent element of the same group (same row) is read from
// LDS in phase B (in_lo / in_hi).  Of the other ends, at most one is read here
// (the low one if it lies outside the group, else the high one), in flight
// with the other neighbour lines; a second outside end (a group starting at
// the last element of a row, or nx = 1) is flagged in far_hi and read in
// phase B.  Inside a group only its two end elements need a line from global
// memory, which saves most of this access's L1 traffic (its lanes touch one
// cache line each).  Threads with no outside end issue no load (at P = 7 a
// wave is one element, so whole waves skip it), and a line's nodes are
// contiguous, so its loads merge into 16-byte ones.
template <int P, typename T, bool NUF>
__device__ __forceinline__ void load_nb_x(const ApplyArgs<T> &A, int el, int ex, int nx, int el_loc,
                                          int EB, int off, bool &in_lo, bool &in_hi, bool &far_hi,
                                          LineNb<T> &f, const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1, N3 = n * n * n;
    int kL, kR;
    const int klo = face_kind(ex, nx, A.geo.bc[0], false, kL);
    const int khi = face_kind(ex, nx, A.geo.bc[0], true, kR);
    in_lo = klo == 1 && ex > 0 && el_loc > 0;
    in_hi = khi == 1 && ex < nx - 1 && el_loc + 1 < EB;
    const bool g_lo = klo == 1 && !in_lo, g_hi = khi == 1 && !in_hi;
    far_hi = g_lo && g_hi;
    T v[n];
#pragma unroll
    for (int q = 0; q < n; ++q) v[q] = 0;
    T nuN = A.nu_c;
    if (g_lo || g_hi) {
        const size_t b = (size_t)(el + ((g_lo ? kL : kR) - ex)) * N3 + off;
#pragma unroll
        for (int q = 0; q < n; ++q) v[q] = A.x[b + q];
        if constexpr (NUF) nuN = A.nu[b + (g_lo ? P : 0)];
    }
    T sP = 0, s0 = 0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
        sP = fma(tb.DP[q], v[q], sP);
        s0 = fma(tb.D0[q], v[q], s0);
    }
    f.uL = g_lo ? v[P] : (T)0;
    f.sL = g_lo ? sP : (T)0;
    f.uR = (g_hi && !g_lo) ? v[0] : (T)0;
    f.sR = (g_hi && !g_lo) ? s0 : (T)0;
    f.nuL = g_lo ? nuN : A.nu_c;
    f.nuR = (g_hi && !g_lo) ? nuN : A.nu_c;
}

// Phase B part of load_nb_x: the ends read from the neighbour slots' LDS
// copies (xsl: this element's x-line (b=i, c=j) start, padded layout), and a
// second outside end from global memory.
template <int P, typename T, bool NUF>
__device__ __forceinline__ void finish_nb_x(const ApplyArgs<T> &A, int el, int ex, int nx,
                                            const T *xsl, const T *nsl, int E3, int off,
                                            bool in_lo, bool in_hi, bool far_hi, LineNb<T> &f,
                                            const EoTab<P, T> &tb = c_eo<P, T>)
{
    constexpr int n = P + 1, N3 = n * n * n;
    if (in_lo) {
        T v[n];
#pragma unroll
        for (int a = 0; a < n; ++a) v[a] = xsl[a - E3];
        T s = 0;
#pragma unroll
        for (int a = 0; a < n; ++a) s = fma(tb.DP[a], v[a], s);
        f.uL = v[P];
        f.sL = s;
        if constexpr (NUF) f.nuL = nsl[P - E3];
    }
    if (in_hi) {
        T v[n];
#pragma unroll
        for (int a = 0; a < n; ++a) v[a] = xsl[a + E3];
        T s = 0;
#pragma unroll
        for (int a = 0; a < n; ++a) s = fma(tb.D0[a], v[a], s);
        f.uR = v[0];
        f.sR = s;
        if constexpr (NUF) f.nuR = nsl[E3];
    }
    if (far_hi) {
        int kR;
        face_kind(ex, nx, A.geo.bc[0], true, kR);
        const size_t b = (size_t)(el + (kR - ex)) * N3 + off;
        nb_line<P, T>(A.x + b, 1, 0, f.uR, f.sR, tb);
        if constexpr (NUF) f.nuR = A.nu[b];
    }
}

// Per-element geometry shared through LDS: extents, reciprocals and the
// ratios rho = h / h_N of every face neighbour.
template <typename T>
struct ElGeo {
    T h[3], ih[3], rhoL[3], rhoR[3];
};

// The rows of one line along axis d in natural units: y = vs * (line
// operator), vs = J g^2 wt (nu).
template <int P, typename T, bool NUF>
__device__ __forceinline__ void line_apply(const ApplyArgs<T> &A, const T (&u)[P + 1],
                                           const T (&nl)[P + 1], int d, int k, int nk,
                                           const ElGeo<T> &G, T wt, const LineNb<T> &f, T &vs,
                                           T (&y)[P + 1], const EoTab<P, T> &tb = c_eo<P, T>)
{
    int kL, kR;
    const int bc = A.geo.bc[d];
    const int klo = face_kind(k, nk, bc, false, kL);
    const int khi = face_kind(k, nk, bc, true, kR);
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    vs = (T)0.5 * wt * G.h[t1] * G.h[t2] * G.ih[d];
    if constexpr (NUF) {
        line_nodal<P, T>(u, nl, klo, khi, G.rhoL[d], G.rhoR[d], f.uL, f.sL, f.nuL, f.uR, f.sR,
                         f.nuR, y, tb);
    } else {
        vs *= A.nu_c;
        line_const<P, T>(u, klo, khi, G.rhoL[d], G.rhoR[d], f.uL, f.sL, f.uR, f.sR, y, tb);
    }
}

// Whole-element 16-byte chunks: possible when all lines of an element lie in
// one wave (64 a multiple of (P+1)^2: P = 3, 7) and a line splits into
// 16-byte chunks.  The own element is then loaded, and y stored, as chunks
// that consecutive lanes take in order (half the memory instructions of one
// node per lane), transposed through the element's LDS slot by the wave
// itself.  FP64 only: in FP32 the transposes measured 1-2 % slower than the
// per-line loads and stores they replace.
template <int P, typename T>
constexpr bool chunk_ok()
{
    return sizeof(T) == 8 && (64 % ((P + 1) * (P + 1)) == 0) && ((P + 1) % 2 == 0);
}

// LDS layout of an element: node (a,b,c) at a + b*SB + c*SC with an odd row
// stride, so that the x-, y- and z-line access patterns of a wave fall on
// distinct banks.
template <int P>
struct Lds {
    static constexpr int n = P + 1;
    static constexpr int SB = (n % 2 == 0) ? n + 1 : n;
    static constexpr int SC = n * SB;
    static constexpr int E3 = n * SC;
};

// The apply on one group of EB elements (all threads of the work-group take
// part; the caller provides the LDS buffers xs, ys [EB*E3], nus [EB*E3 if
// NUF] and geo [EB]).  red receives this thread's share of the epilogue
// sums (EPI_CG: x.y, sum y; EPI_RESID: sum (r/M)^2, sum r, sum r/M^2,
// sum 1/M^2).  EBX: elements per group (default: the kernels' group size;
// a smaller EBX lets a caller run the apply in less LDS, the group index
// then counting groups of EBX elements).  LAZY: load each direction's
// neighbour lines just before its sweep instead of all up front (fewer
// registers, less latency overlap).
template <int P, typename T, bool NUF, int EPI, int EBX = Shape<P>::EB, bool LAZY = false,
          bool FRESH = false, bool CHUNK = false>
__device__ __forceinline__ void apply_group(const ApplyArgs<T> &A, int grp, T *xs, T *ys, T *nus,
                                            ElGeo<T> *geo, double (&red)[4])
{
    // the coefficient table, re-derived at each use inside a persistent loop
    auto TB = []() -> const EoTab<P, T> & {
        if constexpr (FRESH)
            return eo_fresh<P, T>();
        else
            return c_eo<P, T>;
    };
    using S = Shape<P>;
    constexpr int n = S::n, NL = S::NL, N3 = S::N3, EB = EBX, NT = EBX * NL;
    static_assert(EBX >= 1 && EBX <= S::EB, "group size");
    static_assert(!CHUNK || (chunk_ok<P, T>() && EPI != EPI_RESID), "chunked layout");
    constexpr int V = 16 / (int)sizeof(T);  // nodes per 16-byte chunk
    using VT = T __attribute__((ext_vector_type(16 / sizeof(T))));
    // the GLL weights, for the tangential weight product of each thread
    __shared__ T s_w[S::n];
    constexpr int SB = Lds<P>::SB, SC = Lds<P>::SC, E3 = Lds<P>::E3;
    red[0] = red[1] = red[2] = red[3] = 0.0;
    const int tid = threadIdx.x;
    const int el_loc = tid / NL;
    const int l = tid - el_loc * NL;
    const int i = l % n, j = l / n;
    const int el = grp * EB + el_loc;
    const bool active = (tid < NT) && (el < A.nel);
    const int nx = A.geo.n[0], ny = A.geo.n[1], nz = A.geo.n[2];
    int ex = 0, ey = 0, ez = 0;
    if (active) {
        ex = el % nx;
        const int r = el / nx;
        ey = r % ny;
        ez = r / ny;
    }
    const T *__restrict__ xe = A.x + (size_t)el * N3;
    T *xsl = xs + el_loc * E3;
    T *ysl = ys + el_loc * E3;
    T *nsl = nus + (NUF ? el_loc * E3 : 0);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < n; ++k) s_w[k] = (T)kGll<P>.w[k];
    }

    // phase A: own z-line (a=i, b=j) into registers and LDS; all neighbour
    // lines this thread will need (x-line (b=i,c=j), y-line (a=i,c=j),
    // z-line (a=i,b=j)) are requested up front so their latency overlaps
    T uz[n], nz_l[n];
    LineNb<T> fx, fy, fz;
    // group-internal x-neighbours are read from LDS in phase B (measured
    // faster in FP64 at every degree, and in FP32 once the other ends stopped
    // issuing loads of their own)
    bool x_in_lo = false, x_in_hi = false, x_far_hi = false;
    if (active) {
        if constexpr (!CHUNK) {
#pragma unroll
            for (int c = 0; c < n; ++c) uz[c] = xe[c * NL + l];
        }
        if constexpr (!LAZY) {
            load_nb_x<P, T, NUF>(A, el, ex, nx, el_loc, EB, j * NL + i * n, x_in_lo, x_in_hi,
                                 x_far_hi, fx, TB());
            load_nb<P, T, NUF>(A, el, ey, ny, A.geo.bc[1], nx, j * NL + i, n, fy, TB());
            load_nb<P, T, NUF>(A, el, ez, nz, A.geo.bc[2], nx * ny, l, NL, fz, TB());
        }
        // the element's geometry (every thread loads it, one writes it).
        // When a wave holds exactly one element (P = 7) its indices are made
        // wave-uniform, so the loads become scalar loads instead of vector
        // loads that each cost the address path a full wave instruction.
        int ke[3] = {ex, ey, ez};
        if constexpr (NL == 64) {
#pragma unroll
            for (int d = 0; d < 3; ++d) ke[d] = __builtin_amdgcn_readfirstlane(ke[d]);
        }
        ElGeo<T> g;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int kL, kR;
            face_kind(ke[d], A.geo.n[d], A.geo.bc[d], false, kL);
            face_kind(ke[d], A.geo.n[d], A.geo.bc[d], true, kR);
            g.h[d] = A.geo.h[d][ke[d]];
            g.ih[d] = A.geo.ih[d][ke[d]];
            g.rhoL[d] = g.h[d] * A.geo.ih[d][kL];
            g.rhoR[d] = g.h[d] * A.geo.ih[d][kR];
        }
        if (l == 0) geo[el_loc] = g;
        if constexpr (CHUNK) {
            // chunk r of this thread: nodes f..f+V-1 of the element, one row
#pragma unroll
            for (int r = 0; r < n / V; ++r) {
                const int f = V * (l + NL * r);
                const int o = f % n + ((f / n) % n) * SB + (f / NL) * SC;
                const VT v = *reinterpret_cast<const VT *>(xe + f);
#pragma unroll
                for (int k = 0; k < V; ++k) xsl[o + k] = v[k];
                if constexpr (NUF) {
                    const VT w = *reinterpret_cast<const VT *>(A.nu + (size_t)el * N3 + f);
#pragma unroll
                    for (int k = 0; k < V; ++k) nsl[o + k] = w[k];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < n; ++c) {
                xsl[i + j * SB + c * SC] = uz[c];
                if constexpr (NUF) {
                    nz_l[c] = A.nu[(size_t)el * N3 + c * NL + l];
                    nsl[i + j * SB + c * SC] = nz_l[c];
                } else {
                    nz_l[c] = 0;
                }
            }
        }
    }
    __syncthreads();
    const T wt = s_w[i] * s_w[j];  // product of the two tangential GLL weights

    // phase B: x-lines (b=i, c=j)
    if (active) {
        if constexpr (LAZY)
            load_nb_x<P, T, NUF>(A, el, ex, nx, el_loc, EB, j * NL + i * n, x_in_lo, x_in_hi,
                                 x_far_hi, fx, TB());
        finish_nb_x<P, T, NUF>(A, el, ex, nx, xsl + i * SB + j * SC, nsl + i * SB + j * SC, E3,
                               j * NL + i * n, x_in_lo, x_in_hi, x_far_hi, fx, TB());
        T u[n], nl[n], out[n];
#pragma unroll
        for (int a = 0; a < n; ++a) {
            u[a] = xsl[a + i * SB + j * SC];
            nl[a] = NUF ? nsl[a + i * SB + j * SC] : (T)0;
        }
        T vs;
        line_apply<P, T, NUF>(A, u, nl, 0, ex, nx, geo[el_loc], wt, fx, vs, out, TB());
#pragma unroll
        for (int a = 0; a < n; ++a) ysl[a + i * SB + j * SC] = vs * out[a];
    }
    __syncthreads();

    // phase C: y-lines (a=i, c=j)
    if (active) {
        if constexpr (LAZY)
            load_nb<P, T, NUF>(A, el, ey, ny, A.geo.bc[1], nx, j * NL + i, n, fy, TB());
        T u[n], nl[n], out[n];
#pragma unroll
        for (int b = 0; b < n; ++b) {
            u[b] = xsl[i + b * SB + j * SC];
            nl[b] = NUF ? nsl[i + b * SB + j * SC] : (T)0;
        }
        T vs;
        line_apply<P, T, NUF>(A, u, nl, 1, ey, ny, geo[el_loc], wt, fy, vs, out, TB());
#pragma unroll
        for (int b = 0; b < n; ++b) ysl[i + b * SB + j * SC] = fma(vs, out[b], ysl[i + b * SB + j * SC]);
    }
    __syncthreads();

    // phase D: z-lines (a=i, b=j), mass term, epilogue
    if (active) {
        if constexpr (LAZY)
            load_nb<P, T, NUF>(A, el, ez, nz, A.geo.bc[2], nx * ny, l, NL, fz, TB());
        if constexpr (CHUNK) {
#pragma unroll
            for (int c = 0; c < n; ++c) {
                uz[c] = xsl[i + j * SB + c * SC];
                nz_l[c] = NUF ? nsl[i + j * SB + c * SC] : (T)0;
            }
        }
        T out[n];
        T vs;
        const ElGeo<T> &G = geo[el_loc];
        line_apply<P, T, NUF>(A, uz, nz_l, 2, ez, nz, G, wt, fz, vs, out, TB());
        const T Jw = G.h[0] * G.h[1] * G.h[2] * (T)0.125 * wt;
        const double iJw = EPI == EPI_RESID ? 1.0 / (double)Jw : 0.0;
        T *__restrict__ ye = A.y + (size_t)el * N3;
        if constexpr (CHUNK) {
            // y of this thread's z-line into its own accumulator slots, then
            // out as chunks; the element's lines are all in this wave, so a
            // wavefront-scope fence (no work-group barrier) orders the
            // exchange
#pragma unroll
            for (int c = 0; c < n; ++c) {
                const T m = Jw * Wm<P, T>(c);
                T v = fma(vs, out[c], ysl[i + j * SB + c * SC]);
                v = fma(A.lambda * m, uz[c], v);
                ysl[i + j * SB + c * SC] = v;
                if constexpr (EPI == EPI_CG) {
                    red[0] += (double)uz[c] * (double)v;
                    red[1] += (double)v;
                }
            }
            // the chunks below read lines other lanes of this wave wrote:
            // order those LDS writes before the reads at wavefront scope
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int r = 0; r < n / V; ++r) {
                const int f = V * (l + NL * r);
                const int o = f % n + ((f / n) % n) * SB + (f / NL) * SC;
                VT v;
#pragma unroll
                for (int k = 0; k < V; ++k) v[k] = ysl[o + k];
                __builtin_nontemporal_store(v, reinterpret_cast<VT *>(ye + f));
            }
        } else {
#pragma unroll
            for (int c = 0; c < n; ++c) {
                const T m = Jw * Wm<P, T>(c);
                T v = fma(vs, out[c], ysl[i + j * SB + c * SC]);
                v = fma(A.lambda * m, uz[c], v);
                if constexpr (EPI == EPI_STORE) {
                    __builtin_nontemporal_store(v, &ye[c * NL + l]);
                } else if constexpr (EPI == EPI_CG) {
                    __builtin_nontemporal_store(v, &ye[c * NL + l]);
                    red[0] += (double)uz[c] * (double)v;
                    red[1] += (double)v;
                } else {  // EPI_RESID: y = b - A x
                    const T bv = A.b[(size_t)el * N3 + c * NL + l];
                    const T r = bv - v;
                    ye[c * NL + l] = r;
                    const double im = iJw * (1.0 / kGll<P>.w[c]);  // 1 / M
                    const double rm = (double)r * im;
                    red[0] += rm * rm;
                    red[1] += (double)r;
                    red[2] += rm * im;
                    red[3] += im * im;
                }
            }
        }
    }
}


}  // namespace dg
