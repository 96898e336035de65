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
// products are FP64 and reduced deterministically (per-group partials,
// summed in a fixed order by a one-work-group kernel launched after them).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdio>
#include <vector>

#include "dg_internal.h"
#include "kernels.h"
#include "device_common.h"
#include "gll_constexpr.h"
#include "apply_core.h"

namespace dg {

template <int P, typename T, bool NUF, int EPI, bool CH>
__global__ void __launch_bounds__(Shape<P>::NTP) k_apply(ApplyArgs<T> A)
{
    using S = Shape<P>;
    constexpr int EB = S::EB, E3 = Lds<P>::E3;
    __shared__ T xs[EB * E3];
    __shared__ T ys[EB * E3];
    __shared__ T nus[NUF ? EB * E3 : 1];
    __shared__ ElGeo<T> geo[EB];
    __shared__ double red_sh[16 * 4];

    if constexpr (EPI == EPI_CG) {
        if (A.sc->done) return;
    }
    const int slot = xcd_remap(blockIdx.x, A.ngroups);
    const int grp = A.order ? A.order[slot] : slot;
    double red[4];
    apply_group<P, T, NUF, EPI, Shape<P>::EB, apply_lazy<P, T>(), false, CH>(A, grp, xs, ys, nus,
                                                                            geo, red);
    if constexpr (EPI == EPI_CG) {
        double red2[2] = {red[0], red[1]};
        publish_partials<2>(red2, A.partial, gridDim.x, red_sh);
    } else if constexpr (EPI == EPI_RESID) {
        publish_partials<4>(red, A.partial, gridDim.x, red_sh);
    }
}

// ---------------------------------------------------------- diag kernel --

template <int P, typename T, bool NUF, bool INV>
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
        A.y[gi] = INV ? (T)1 / s : s;
    }
}

// ---------------------------------------------------------- launchers --

template <typename T>
static Geo<T> make_geo(const MeshDev &m, const int bc[3])
{
    Geo<T> g{};
    const T *h = std::is_same<T, double>::value ? (const T *)m.h64 : (const T *)m.h32;
    const T *ih = std::is_same<T, double>::value ? (const T *)m.ih64 : (const T *)m.ih32;
    g.h[0] = h;
    g.h[1] = h + m.n[0];
    g.h[2] = h + m.n[0] + m.n[1];
    g.ih[0] = ih;
    g.ih[1] = ih + m.n[0];
    g.ih[2] = ih + m.n[0] + m.n[1];
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

std::vector<int> apply_order(const int n[3], int P)
{
    const int NL = (P + 1) * (P + 1);
    const int EB = 256 / NL > 0 ? 256 / NL : 1;
    const long long nel = (long long)n[0] * n[1] * n[2];
    const int G = (int)((nel + EB - 1) / EB);
    // patch grid px * py = 8 with the smallest patch perimeter
    int px = 1, py = 1;
    double best = 1e300;
    for (int a = 1; a <= 8; a *= 2) {
        const int b = 8 / a;
        if (a > n[0] || b > n[1]) continue;
        const double per = (double)n[0] / a + (double)n[1] / b;
        if (per < best) {
            best = per;
            px = a;
            py = b;
        }
    }
    std::vector<long long> key(G);
    std::vector<int> ord(G);
    for (int g = 0; g < G; ++g) {
        const long long e0 = (long long)g * EB;
        const int ex = (int)(e0 % n[0]);
        const int ey = (int)((e0 / n[0]) % n[1]);
        const int ez = (int)(e0 / ((long long)n[0] * n[1]));
        const int patch = (int)((long long)ex * px / n[0]) + px * (int)((long long)ey * py / n[1]);
        key[g] = (((long long)patch * n[2] + ez) * n[1] + ey) * n[0] + ex;
        ord[g] = g;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
    return ord;
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
    a.order = m.order;
    return a;
}

// The own element is loaded and y stored in 16-byte chunks where the degree
// allows it (chunk_ok), the vectors are 16-byte aligned, and the epilogue
// stores y as computed (not the residual form).
template <int P, typename T, int EPI>
static bool use_chunks(const ApplyArgs<T> &a)
{
    if constexpr (!chunk_ok<P, T>() || EPI == EPI_RESID) {
        return false;
    } else {
        auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
        return al(a.x) && al(a.y) && (a.nu == nullptr || al(a.nu));
    }
}

template <int P, typename T, int EPI>
static void launch_apply_P(const ApplyArgs<T> &a, bool nuf, hipStream_t s)
{
    dim3 grid(a.ngroups), block(Shape<P>::NTP);
    if constexpr (chunk_ok<P, T>() && EPI != EPI_RESID) {
        if (use_chunks<P, T, EPI>(a)) {
            if (nuf)
                hipLaunchKernelGGL((k_apply<P, T, true, EPI, true>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((k_apply<P, T, false, EPI, true>), grid, block, 0, s, a);
            return;
        }
    }
    if (nuf)
        hipLaunchKernelGGL((k_apply<P, T, true, EPI, false>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_apply<P, T, false, EPI, false>), grid, block, 0, s, a);
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
                    const T *p, T *q, double *partial, CgScalars *sc,
                    hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, p, q);
    a.partial = partial;
    a.sc = sc;
    if (int rc = dispatch_apply<T, EPI_CG>(m.P, a, nu != nullptr, s)) return rc;
    return launch_finish_apply(partial, a.ngroups, sc, s);
}

template <typename T>
int launch_resid(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                 const T *x, const T *b, T *r, double *partial, CgScalars *sc,
                 hipStream_t s)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, x, r);
    a.b = b;
    a.partial = partial;
    a.sc = sc;
    if (int rc = dispatch_apply<T, EPI_RESID>(m.P, a, nu != nullptr, s)) return rc;
    return launch_finish_resid(partial, a.ngroups, sc, s);
}

template <int P, typename T>
static void launch_diag_P(const ApplyArgs<T> &a, bool nuf, bool inv, hipStream_t s)
{
    dim3 grid(a.ngroups), block(Shape<P>::NTP);
    if (nuf && inv)
        hipLaunchKernelGGL((k_diag<P, T, true, true>), grid, block, 0, s, a);
    else if (nuf)
        hipLaunchKernelGGL((k_diag<P, T, true, false>), grid, block, 0, s, a);
    else if (inv)
        hipLaunchKernelGGL((k_diag<P, T, false, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_diag<P, T, false, false>), grid, block, 0, s, a);
}

template <typename T>
int launch_diag(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c, T *d,
                hipStream_t s, bool inverse)
{
    ApplyArgs<T> a = make_args<T>(m, bc, lambda, nu, nu_c, nullptr, d);
    const bool nf = nu != nullptr;
    switch (m.P) {
        case 3: launch_diag_P<3, T>(a, nf, inverse, s); break;
        case 4: launch_diag_P<4, T>(a, nf, inverse, s); break;
        case 5: launch_diag_P<5, T>(a, nf, inverse, s); break;
        case 6: launch_diag_P<6, T>(a, nf, inverse, s); break;
        case 7: launch_diag_P<7, T>(a, nf, inverse, s); break;
        case 8: launch_diag_P<8, T>(a, nf, inverse, s); break;
        default: set_error("polynomial degree outside 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

#define DG_INST(T)                                                                               \
    template int launch_apply<T>(const MeshDev &, const int[3], double, const T *, double,      \
                                 const T *, T *, hipStream_t);                                   \
    template int launch_apply_cg<T>(const MeshDev &, const int[3], double, const T *, double,   \
                                    const T *, T *, double *, CgScalars *,                       \
                                    hipStream_t);                                                \
    template int launch_resid<T>(const MeshDev &, const int[3], double, const T *, double,      \
                                 const T *, const T *, T *, double *, CgScalars *,               \
                                 hipStream_t);                                                   \
    template int launch_diag<T>(const MeshDev &, const int[3], double, const T *, double, T *,  \
                                hipStream_t, bool);
DG_INST(double)
DG_INST(float)

}  // namespace dg
