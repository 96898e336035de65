// HIP kernels (gfx950) of the SIP-DG Helmholtz / Poisson solve.
//
// Operator (arXiv 2112.04167, Sec. 3.3: DG-SEM on tensor-product GLL
// hexahedra with the interior penalty method; Alg. 3: the Helmholtz problem
// of the diffusion substep and the Poisson problem of the projection
// substep):  y = (lambda M + K_nu) x, all integrals by the GLL rule.
//
// On a Cartesian product grid the operator splits into three sweeps of 1D
// operators along the x-, y- and z-lines of the mesh.  A line of one element
// couples only to the same line of the two face neighbours along that axis,
// through two numbers per neighbour: its trace at the shared face and its
// normal derivative there (a dot product over the neighbour's line).
//
// Work decomposition (one work-group = EB elements, one thread = one line of
// (P+1) nodes per direction):
//   phase A  thread (a,b) loads its z-line of x into registers and into LDS
//   phase B  thread (b,c) reads its x-line from LDS, reads the x-neighbours'
//            lines from global memory (L2), applies the 1D operator and
//            writes the result into the LDS accumulator
//   phase C  the same for the y-lines (accumulate)
//   phase D  thread (a,b) applies the z-line operator and the mass term in
//            registers, adds the LDS accumulator and stores y (coalesced)
// Every output value is produced by one thread in a fixed order, so results
// are bitwise reproducible.  Work-group ids are remapped so that each of the
// 8 XCDs sweeps a contiguous range of elements (its L2 then holds most
// neighbour lines).
//
// CG kernels use the same element/line mapping so that the GLL mass and the
// Jacobi diagonal are available per node without index divisions; dot
// products are FP64 and reduced deterministically (per-group partials, the
// last group to finish sums them in a fixed order).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "dg_internal.h"
#include "kernels.h"
#include "device_common.h"
#include "gll_constexpr.h"

namespace dg {

// coefficients of the compile-time GLL tables, in the kernel's precision
template <int P, typename T>
__device__ __forceinline__ T Dm(int k) { return (T)kGll<P>.D[k]; }
template <int P, typename T>
__device__ __forceinline__ T K1m(int k) { return (T)kGll<P>.K1[k]; }
template <int P, typename T>
__device__ __forceinline__ T Wm(int k) { return (T)kGll<P>.w[k]; }

// ------------------------------------------------------ the 1D operator --
//
// One line u[0..P] of an element along axis d (local coordinate xi in
// [-1,1], extent h, g = 2/h).  vs = volume scale J g^2 w_t1 w_t2 (times nu
// when constant), om = face weight w_t1 w_t2 h_t1 h_t2 / 4.  Low / high
// ends: kind (0 natural, 1 neighbour, 2 Dirichlet), neighbour trace uN,
// neighbour normal derivative dN (already scaled by its 2/h), neighbour
// extent hN and neighbour nu at the shared face node.
template <int P, typename T, bool NUF>
__device__ __forceinline__ void line_op(const T (&u)[P + 1], const T (&nl)[P + 1], T nu_c, T vs,
                                        T om, T g, T h, int klo, T uL, T dL, T hL, T nuL, int khi,
                                        T uR, T dR, T hR, T nuR, T (&out)[P + 1])
{
    constexpr int n = P + 1;
    const T pen = (T)(n * n);
    if constexpr (NUF) {
        T t[n];
#pragma unroll
        for (int q = 0; q < n; ++q) {
            T s = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) s = fma(Dm<P, T>(q * n + j), u[j], s);
            t[q] = s * (Wm<P, T>(q) * nl[q]);
        }
#pragma unroll
        for (int a = 0; a < n; ++a) {
            T s = 0;
#pragma unroll
            for (int q = 0; q < n; ++q) s = fma(Dm<P, T>(q * n + a), t[q], s);
            out[a] = vs * s;
        }
    } else {
#pragma unroll
        for (int a = 0; a < n; ++a) {
            T s = 0;
#pragma unroll
            for (int j = 0; j < n; ++j) s = fma(K1m<P, T>(a * n + j), u[j], s);
            out[a] = vs * s;
        }
    }
    if (klo == 0 && khi == 0) return;
    T d0 = 0, dP = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        d0 = fma(Dm<P, T>(j), u[j], d0);
        dP = fma(Dm<P, T>(P * n + j), u[j], dP);
    }
    d0 *= g;
    dP *= g;
    const T nu0 = NUF ? nl[0] : nu_c;
    const T nuP = NUF ? nl[P] : nu_c;
    T ch = 0, cl = 0;
    if (khi == 1) {
        const T jump = u[P] - uR;
        const T avg = (T)0.5 * (nuP * dP + nuR * dR);
        const T sig = dmax(nuP, nuR) * pen / dmin(h, hR);
        out[P] += om * (sig * jump - avg);
        ch = (T)(-0.5) * om * nuP * g * jump;
    } else if (khi == 2) {
        const T sig = nuP * pen / h;
        out[P] += om * (sig * u[P] - nuP * dP);
        ch = -om * nuP * g * u[P];
    }
    if (klo == 1) {
        const T jump = uL - u[0];
        const T avg = (T)0.5 * (nuL * dL + nu0 * d0);
        const T sig = dmax(nu0, nuL) * pen / dmin(h, hL);
        out[0] += om * (avg - sig * jump);
        cl = (T)(-0.5) * om * nu0 * g * jump;
    } else if (klo == 2) {
        const T sig = nu0 * pen / h;
        out[0] += om * (nu0 * d0 + sig * u[0]);
        cl = om * nu0 * g * u[0];
    }
#pragma unroll
    for (int j = 0; j < n; ++j) out[j] = fma(ch, Dm<P, T>(P * n + j), fma(cl, Dm<P, T>(j), out[j]));
}

// neighbour line: trace at `layer` and the raw derivative sum there
template <int P, typename T>
__device__ __forceinline__ void nb_line(const T *__restrict__ base, int stride, int layer,
                                        T &uN, T &sN)
{
    constexpr int n = P + 1;
    T v[n];
#pragma unroll
    for (int k = 0; k < n; ++k) v[k] = base[k * stride];
    T s = 0;
#pragma unroll
    for (int k = 0; k < n; ++k) s = fma(Dm<P, T>(layer * n + k), v[k], s);
    uN = v[layer];
    sN = s;
}

// --------------------------------------------------------- apply kernel --

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
    // EPI_CG: partial dot x.y and sum(y); last group computes alpha.
    // EPI_RESID: y = b - A x, partial sums of (y/M)^2 and y, (y/M) and 1/M^2 sums
    const T *b;
    double *partial;
    unsigned *counter;
    CgScalars *sc;
};

template <int P, typename T, bool NUF, int EPI>
__global__ void __launch_bounds__(Shape<P>::NTP) k_apply(ApplyArgs<T> A)
{
    using S = Shape<P>;
    constexpr int n = S::n, NL = S::NL, N3 = S::N3, EB = S::EB, NT = S::NT;
    __shared__ T xs[EB * N3];
    __shared__ T ys[EB * N3];
    __shared__ T nus[NUF ? EB * N3 : 1];
    __shared__ double red_sh[16 * 4];

    if constexpr (EPI == EPI_CG) {
        if (A.sc->done) return;
    }

    const int grp = xcd_remap(blockIdx.x, A.ngroups);
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
    const T hx = active ? A.geo.h[0][ex] : (T)1, hy = active ? A.geo.h[1][ey] : (T)1,
            hz = active ? A.geo.h[2][ez] : (T)1;
    const T *__restrict__ xe = A.x + (size_t)el * N3;
    T *xsl = xs + el_loc * N3;
    T *ysl = ys + el_loc * N3;
    T *nsl = nus + (NUF ? el_loc * N3 : 0);

    // phase A: z-line (a=i, b=j) into registers and LDS
    T uz[n], nz_l[n];
    if (active) {
#pragma unroll
        for (int c = 0; c < n; ++c) {
            uz[c] = xe[c * NL + l];
            xsl[c * NL + l] = uz[c];
            if constexpr (NUF) {
                nz_l[c] = A.nu[(size_t)el * N3 + c * NL + l];
                nsl[c * NL + l] = nz_l[c];
            } else {
                nz_l[c] = 0;
            }
        }
    }
    __syncthreads();

    // phase B: x-lines (b=i, c=j)
    if (active) {
        T u[n], nl[n], out[n];
#pragma unroll
        for (int a = 0; a < n; ++a) {
            u[a] = xsl[j * NL + i * n + a];
            nl[a] = NUF ? nsl[j * NL + i * n + a] : (T)0;
        }
        int kL, kR;
        const int klo = face_kind(ex, nx, A.geo.bc[0], false, kL);
        const int khi = face_kind(ex, nx, A.geo.bc[0], true, kR);
        T uL = 0, dL = 0, hL = hx, nuL = A.nu_c, uR = 0, dR = 0, hR = hx, nuR = A.nu_c;
        if (klo == 1) {
            const int eN = el + (kL - ex);
            const T *bN = A.x + (size_t)eN * N3 + j * NL + i * n;
            nb_line<P, T>(bN, 1, P, uL, dL);
            hL = A.geo.h[0][kL];
            dL *= (T)2 / hL;
            if constexpr (NUF) nuL = A.nu[(size_t)eN * N3 + j * NL + i * n + P];
        }
        if (khi == 1) {
            const int eN = el + (kR - ex);
            const T *bN = A.x + (size_t)eN * N3 + j * NL + i * n;
            nb_line<P, T>(bN, 1, 0, uR, dR);
            hR = A.geo.h[0][kR];
            dR *= (T)2 / hR;
            if constexpr (NUF) nuR = A.nu[(size_t)eN * N3 + j * NL + i * n + 0];
        }
        const T wt = Wm<P, T>(i) * Wm<P, T>(j);
        const T vs = wt * hy * hz / ((T)2 * hx) * (NUF ? (T)1 : A.nu_c);
        const T om = wt * hy * hz * (T)0.25;
        line_op<P, T, NUF>(u, nl, A.nu_c, vs, om, (T)2 / hx, hx, klo, uL, dL, hL, nuL, khi, uR, dR,
                           hR, nuR, out);
#pragma unroll
        for (int a = 0; a < n; ++a) ysl[j * NL + i * n + a] = out[a];
    }
    __syncthreads();

    // phase C: y-lines (a=i, c=j)
    if (active) {
        T u[n], nl[n], out[n];
#pragma unroll
        for (int b = 0; b < n; ++b) {
            u[b] = xsl[j * NL + b * n + i];
            nl[b] = NUF ? nsl[j * NL + b * n + i] : (T)0;
        }
        int kL, kR;
        const int klo = face_kind(ey, ny, A.geo.bc[1], false, kL);
        const int khi = face_kind(ey, ny, A.geo.bc[1], true, kR);
        T uL = 0, dL = 0, hL = hy, nuL = A.nu_c, uR = 0, dR = 0, hR = hy, nuR = A.nu_c;
        if (klo == 1) {
            const int eN = el + (kL - ey) * nx;
            const T *bN = A.x + (size_t)eN * N3 + j * NL + i;
            nb_line<P, T>(bN, n, P, uL, dL);
            hL = A.geo.h[1][kL];
            dL *= (T)2 / hL;
            if constexpr (NUF) nuL = A.nu[(size_t)eN * N3 + j * NL + P * n + i];
        }
        if (khi == 1) {
            const int eN = el + (kR - ey) * nx;
            const T *bN = A.x + (size_t)eN * N3 + j * NL + i;
            nb_line<P, T>(bN, n, 0, uR, dR);
            hR = A.geo.h[1][kR];
            dR *= (T)2 / hR;
            if constexpr (NUF) nuR = A.nu[(size_t)eN * N3 + j * NL + i];
        }
        const T wt = Wm<P, T>(i) * Wm<P, T>(j);
        const T vs = wt * hx * hz / ((T)2 * hy) * (NUF ? (T)1 : A.nu_c);
        const T om = wt * hx * hz * (T)0.25;
        line_op<P, T, NUF>(u, nl, A.nu_c, vs, om, (T)2 / hy, hy, klo, uL, dL, hL, nuL, khi, uR, dR,
                           hR, nuR, out);
#pragma unroll
        for (int b = 0; b < n; ++b) ysl[j * NL + b * n + i] += out[b];
    }
    __syncthreads();

    // phase D: z-lines (a=i, b=j), mass term, epilogue
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    if (active) {
        T out[n];
        int kL, kR;
        const int klo = face_kind(ez, nz, A.geo.bc[2], false, kL);
        const int khi = face_kind(ez, nz, A.geo.bc[2], true, kR);
        T uL = 0, dL = 0, hL = hz, nuL = A.nu_c, uR = 0, dR = 0, hR = hz, nuR = A.nu_c;
        const int nxy = nx * ny;
        if (klo == 1) {
            const int eN = el + (kL - ez) * nxy;
            const T *bN = A.x + (size_t)eN * N3 + l;
            nb_line<P, T>(bN, NL, P, uL, dL);
            hL = A.geo.h[2][kL];
            dL *= (T)2 / hL;
            if constexpr (NUF) nuL = A.nu[(size_t)eN * N3 + P * NL + l];
        }
        if (khi == 1) {
            const int eN = el + (kR - ez) * nxy;
            const T *bN = A.x + (size_t)eN * N3 + l;
            nb_line<P, T>(bN, NL, 0, uR, dR);
            hR = A.geo.h[2][kR];
            dR *= (T)2 / hR;
            if constexpr (NUF) nuR = A.nu[(size_t)eN * N3 + l];
        }
        const T wt = Wm<P, T>(i) * Wm<P, T>(j);
        const T vs = wt * hx * hy / ((T)2 * hz) * (NUF ? (T)1 : A.nu_c);
        const T om = wt * hx * hy * (T)0.25;
        line_op<P, T, NUF>(uz, nz_l, A.nu_c, vs, om, (T)2 / hz, hz, klo, uL, dL, hL, nuL, khi, uR,
                           dR, hR, nuR, out);
        const T Jw = hx * hy * hz * (T)0.125 * wt;
        T *__restrict__ ye = A.y + (size_t)el * N3;
#pragma unroll
        for (int c = 0; c < n; ++c) {
            const T m = Jw * Wm<P, T>(c);
            T v = ysl[c * NL + l] + out[c];
            v = fma(A.lambda * m, uz[c], v);
            if constexpr (EPI == EPI_STORE) {
                ye[c * NL + l] = v;
            } else if constexpr (EPI == EPI_CG) {
                ye[c * NL + l] = v;
                red[0] += (double)uz[c] * (double)v;
                red[1] += (double)v;
            } else {  // EPI_RESID: y = b - A x
                const T bv = A.b[(size_t)el * N3 + c * NL + l];
                const T r = bv - v;
                ye[c * NL + l] = r;
                const double rm = (double)r / (double)m;
                red[0] += rm * rm;
                red[1] += (double)r;
                red[2] += rm / (double)m;
                red[3] += 1.0 / ((double)m * (double)m);
            }
        }
    }
    if constexpr (EPI == EPI_CG) {
        double tot[2], red2[2] = {red[0], red[1]};
        if (publish_and_reduce<2>(red2, A.partial, A.counter, gridDim.x, tot, red_sh)) {
            if (threadIdx.x == 0) cg_after_apply(A.sc, tot[0], tot[1]);
        }
    } else if constexpr (EPI == EPI_RESID) {
        double tot[4];
        if (publish_and_reduce<4>(red, A.partial, A.counter, gridDim.x, tot, red_sh)) {
            if (threadIdx.x == 0) resid_finish(A.sc, tot);
        }
    }
}

// ---------------------------------------------------------- diag kernel --

template <int P, typename T, bool NUF>
__global__ void __launch_bounds__(Shape<P>::NTP) k_diag(ApplyArgs<T> A)
{
    using S = Shape<P>;
    constexpr int n = S::n, NL = S::NL, N3 = S::N3, EB = S::EB, NT = S::NT;
    const int grp = blockIdx.x;
    const int tid = threadIdx.x;
    const int el_loc = tid / NL;
    const int l = tid - el_loc * NL;
    const int el = grp * EB + el_loc;
    if (tid >= NT || el >= A.nel) return;
    const int nx = A.geo.n[0], ny = A.geo.n[1];
    const int ex = el % nx, ey = (el / nx) % ny, ez = el / (nx * ny);
    const int ee[3] = {ex, ey, ez};
    const T h[3] = {A.geo.h[0][ex], A.geo.h[1][ey], A.geo.h[2][ez]};
    const T J = h[0] * h[1] * h[2] * (T)0.125;
    const int strides[3] = {1, n, NL};
    const int estr[3] = {1, nx, nx * ny};
    const T pen = (T)(n * n);
    for (int c = 0; c < n; ++c) {
        const int loc = c * NL + l;
        const int a3[3] = {l % n, l / n, c};
        const T W = Wm<P, T>(a3[0]) * Wm<P, T>(a3[1]) * Wm<P, T>(a3[2]);
        const size_t gi = (size_t)el * N3 + loc;
        const T nuo = NUF ? A.nu[gi] : A.nu_c;
        T s = A.lambda * J * W;
        for (int d = 0; d < 3; ++d) {
            const int ad = a3[d];
            const T g = (T)2 / h[d];
            T acc = 0;
            for (int q = 0; q < n; ++q) {
                const T nq = NUF ? A.nu[(long long)gi + (long long)(q - ad) * strides[d]] : A.nu_c;
                const T Dq = Dm<P, T>(q * n + ad);
                acc = fma(Wm<P, T>(q) * nq, Dq * Dq, acc);
            }
            s = fma(J * g * g * (W / Wm<P, T>(ad)), acc, s);
            if (ad != 0 && ad != P) continue;
            const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
            const T om = Wm<P, T>(a3[t1]) * Wm<P, T>(a3[t2]) * h[t1] * h[t2] * (T)0.25;
            const bool high = (ad == P);
            int knb;
            const int kind = face_kind(ee[d], A.geo.n[d], A.geo.bc[d], high, knb);
            const T Dff = Dm<P, T>(ad * n + ad);
            const T sgn = high ? (T)-1 : (T)1;
            if (kind == 1) {
                const int eN = el + (knb - ee[d]) * estr[d];
                const int layerN = high ? 0 : P;
                const long long gN = (long long)eN * N3 + loc + (long long)(layerN - ad) * strides[d];
                const T nun = NUF ? A.nu[gN] : A.nu_c;
                const T sig = dmax(nuo, nun) * pen / dmin(h[d], A.geo.h[d][knb]);
                s += om * (sig + sgn * nuo * g * Dff);
                if (eN == el) {  // single periodic element: self-neighbour
                    if (high) s -= om * nun * g * Dm<P, T>(0 * n + P);
                    else s += om * nun * g * Dm<P, T>(P * n + 0);
                }
            } else if (kind == 2) {
                const T sig = nuo * pen / h[d];
                s += om * (sig + (T)2 * sgn * nuo * g * Dff);
            }
        }
        A.y[gi] = s;
    }
}

// ---------------------------------------------------------- launchers --

template <typename T>
static Geo<T> make_geo(const MeshDev &m, const int bc[3])
{
    Geo<T> g{};
    const T *h = std::is_same<T, double>::value ? (const T *)m.h64 : (const T *)m.h32;
    g.h[0] = h;
    g.h[1] = h + m.n[0];
    g.h[2] = h + m.n[0] + m.n[1];
    for (int d = 0; d < 3; ++d) {
        g.n[d] = m.n[d];
        g.bc[d] = bc[d];
    }
    return g;
}

int apply_groups(int P, int64_t nel)
{
    const int NL = (P + 1) * (P + 1);
    const int EB = 256 / NL > 0 ? 256 / NL : 1;
    return (int)((nel + EB - 1) / EB);
}

int apply_threads(int P)
{
    const int NL = (P + 1) * (P + 1);
    const int EB = 256 / NL > 0 ? 256 / NL : 1;
    return ((EB * NL + 63) / 64) * 64;
}

template <typename T>
static ApplyArgs<T> make_args(const MeshDev &m, const int bc[3], double lambda, const T *nu,
                              double nu_c, const T *x, T *y)
{
    ApplyArgs<T> a{};
    a.x = x;
    a.y = y;
    a.nu = nu;
    a.nu_c = (T)nu_c;
    a.lambda = (T)lambda;
    a.geo = make_geo<T>(m, bc);
    a.nel = (int)m.nel;
    a.ngroups = apply_groups(m.P, m.nel);
    return a;
}

template <int P, typename T, int EPI>
static void launch_apply_P(const ApplyArgs<T> &a, bool nuf, hipStream_t s)
{
    dim3 grid(a.ngroups), block(Shape<P>::NTP);
    if (nuf)
        hipLaunchKernelGGL((k_apply<P, T, true, EPI>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_apply<P, T, false, EPI>), grid, block, 0, s, a);
}

template <typename T, int EPI>
static int dispatch_apply(int P, const ApplyArgs<T> &a, bool nuf, hipStream_t s)
{
    switch (P) {
        case 3: launch_apply_P<3, T, EPI>(a, nuf, s); break;
        case 4: launch_apply_P<4, T, EPI>(a, nuf, s); break;
        case 5: launch_apply_P<5, T, EPI>(a, nuf, s); break;
        case 6: launch_apply_P<6, T, EPI>(a, nuf, s); break;
        case 7: launch_apply_P<7, T, EPI>(a, nuf, s); break;
        case 8: launch_apply_P<8, T, EPI>(a, nuf, s); break;
        default: set_error("polynomial degree outside 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

template <typename T>
int launch_apply(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                 const T *x, T *y, hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, x, y);
    return dispatch_apply<T, EPI_STORE>(m.P, a, nu != nullptr, s);
}

template <typename T>
int launch_apply_cg(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                    const T *p, T *q, double *partial, unsigned *counter, CgScalars *sc,
                    hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, p, q);
    a.partial = partial;
    a.counter = counter;
    a.sc = sc;
    return dispatch_apply<T, EPI_CG>(m.P, a, nu != nullptr, s);
}

template <typename T>
int launch_resid(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                 const T *x, const T *b, T *r, double *partial, unsigned *counter, CgScalars *sc,
                 hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, x, r);
    a.b = b;
    a.partial = partial;
    a.counter = counter;
    a.sc = sc;
    return dispatch_apply<T, EPI_RESID>(m.P, a, nu != nullptr, s);
}

template <int P, typename T>
static void launch_diag_P(const ApplyArgs<T> &a, bool nuf, hipStream_t s)
{
    dim3 grid(a.ngroups), block(Shape<P>::NTP);
    if (nuf)
        hipLaunchKernelGGL((k_diag<P, T, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_diag<P, T, false>), grid, block, 0, s, a);
}

template <typename T>
int launch_diag(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c, T *d,
                hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, nullptr, d);
    switch (m.P) {
        case 3: launch_diag_P<3, T>(a, nu != nullptr, s); break;
        case 4: launch_diag_P<4, T>(a, nu != nullptr, s); break;
        case 5: launch_diag_P<5, T>(a, nu != nullptr, s); break;
        case 6: launch_diag_P<6, T>(a, nu != nullptr, s); break;
        case 7: launch_diag_P<7, T>(a, nu != nullptr, s); break;
        case 8: launch_diag_P<8, T>(a, nu != nullptr, s); break;
        default: set_error("polynomial degree outside 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

#define DG_INST(T)                                                                               \
    template int launch_apply<T>(const MeshDev &, const int[3], double, const T *, double,      \
                                 const T *, T *, hipStream_t);                                   \
    template int launch_apply_cg<T>(const MeshDev &, const int[3], double, const T *, double,   \
                                    const T *, T *, double *, unsigned *, CgScalars *,           \
                                    hipStream_t);                                                \
    template int launch_resid<T>(const MeshDev &, const int[3], double, const T *, double,      \
                                 const T *, const T *, T *, double *, unsigned *, CgScalars *,   \
                                 hipStream_t);                                                   \
    template int launch_diag<T>(const MeshDev &, const int[3], double, const T *, double, T *,  \
                                hipStream_t);
DG_INST(double)
DG_INST(float)

}  // namespace dg
