// CG vector kernels of the SIP-DG solve (gfx950).
//
// Jacobi-preconditioned CG on A = lambda M + K_nu (arXiv 2112.04167: Krylov
// solves of the implicit pressure and diffusion problems, Sec. 3.3; stopping
// on the relative RMS residual at the collocation points, Sec. 4, i.e. on
// ||M^-1 r|| / ||M^-1 b||).  One CG step is three kernels:
//
//   apply   q = A p, with p.q and sum(q) reduced    -> alpha = rho / p.q
//   update  x += alpha p, r -= alpha q, reductions  -> rho', beta, residual
//   pupdate (singular: r -= mean r)  p = r/d + beta p
//
// All scalars live in device memory (CgScalars).  Each reducing kernel writes
// per-work-group partial sums; a one-work-group kernel launched after it sums
// them in a fixed order and updates the scalars, so no host round trip is
// needed per iteration.
// A solve that has finished (converged, iteration cap, breakdown) sets
// `done` and every later CG kernel returns at once, which lets the host
// enqueue iterations in chunks and read the state back rarely.
//
// Threads use the element/line mapping of the apply kernel: thread (el, l)
// owns line l = a + (P+1) b of element el and walks c = 0..P, so the GLL
// mass J w_a w_b w_c is formed in registers.  Dot products are FP64 for FP32
// vectors too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dg_internal.h"
#include "kernels.h"
#include "device_common.h"
#include "gll_constexpr.h"

namespace dg {

namespace {

// The diagonal is computed on the fly in the FP64 kernels only: in the FP32
// inner solve of the mixed mode it measured no faster than the stored one
// (the update kernel lost what the p-update gained), so the FP32 kernels
// keep the plain load.
template <typename T>
constexpr bool kDiagFly = sizeof(T) == 8;

// per-thread line context
template <int P, typename T>
struct LineCtx {
    bool active;
    size_t base;  // index of node (a,b,0)
    T Jw;         // J w_a w_b
    double iJw;   // 1 / (J w_a w_b)
    // on-the-fly diagonal (A.dtab): diag(a,b,c) = w_c dQ + dR Tz[c]
    T dQ, dR;
    const T *tz;
};

// 1/w_c (a compile-time constant)
template <int P>
__device__ __forceinline__ double inv_w(int c) { return 1.0 / kGll<P>.w[c]; }

template <int P, typename T>
__device__ __forceinline__ LineCtx<P, T> line_ctx(const CgVecArgs<T> &A)
{
    using S = Shape<P>;
    LineCtx<P, T> c;
    const int tid = threadIdx.x;
    const int el_loc = tid / S::NL;
    const int l = tid - el_loc * S::NL;
    const int el = blockIdx.x * S::EB + el_loc;
    c.active = (tid < S::NT) && (el < A.nel);
    c.base = (size_t)el * S::N3 + l;
    c.Jw = 0;
    c.iJw = 0.0;
    if (c.active) {
        const int nx = A.n[0], ny = A.n[1];
        const int ex = el % nx, r = el / nx, ey = r % ny, ez = r / ny;
        c.Jw = A.hx[ex] * A.hy[ey] * A.hz[ez] * (T)0.125 * (T)kGll<P>.w[l % S::n] *
               (T)kGll<P>.w[l / S::n];
        c.iJw = 1.0 / (double)c.Jw;
        if (kDiagFly<T> && A.dtab) {
            // the constant-nu operator on a Cartesian grid is a sum of 1D
            // operators along the axes, each scaled by the tangential GLL
            // mass, so its diagonal at node (a,b,c) is
            //   lambda J W + hy hz w_b w_c Tx[ex][a] + hx hz w_a w_c Ty[ey][b]
            //              + hx hy w_a w_b Tz[ez][c]
            // with Tx etc. the 1D diagonals (volume and face terms)
            const int a = l % S::n, b = l / S::n;
            const T hx = A.hx[ex], hy = A.hy[ey], hz = A.hz[ez];
            const T wa = (T)kGll<P>.w[a], wb = (T)kGll<P>.w[b];
            const T *tx = A.dtab + (size_t)ex * S::n;
            const T *ty = A.dtab + (size_t)(A.n[0] + ey) * S::n;
            c.tz = A.dtab + (size_t)(A.n[0] + A.n[1] + ez) * S::n;
            c.dQ = (T)A.lam * c.Jw + hy * hz * wb * tx[a] + hx * hz * wa * ty[b];
            c.dR = hx * hy * wa * wb;
        }
    }
    return c;
}

// 1/diag of node k of this thread's line: computed (A.dtab) or stored (A.d)
template <int P, typename T>
__device__ __forceinline__ T inv_diag(const CgVecArgs<T> &A, const LineCtx<P, T> &c, int k, size_t gi)
{
    if constexpr (kDiagFly<T>)
        if (A.dtab) return (T)1 / fma(c.dR, c.tz[k], (T)kGll<P>.w[k] * c.dQ);
    return A.d[gi];
}

// set-up, stage 1: b = M f (or b = f if weak), sum b and sum b^2
template <int P, typename T, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_setup1(CgVecArgs<T> A)
{
    using S = Shape<P>;
    __shared__ double sh[16 * 2];
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    double red[2] = {0.0, 0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            const T m = c.Jw * (T)kGll<P>.w[k];
            const T b = A.weak ? A.src[gi] : m * A.src[gi];
            A.bvec[gi] = b;
            red[0] += (double)b;
            red[1] += (double)b * (double)b;
        }
    }
    publish_partials<2>(red, A.partial, gridDim.x, sh);
}

// set-up, stage 2: project b (singular), r = b, x = 0 (unless keep_x: the
// caller's initial guess stays, and the solver recomputes r = b - A x and
// restarts from it), z = r/d, p = z and the initial norms.  d == nullptr:
// outer refinement loop (no z, p).
template <int P, typename T, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_setup2(CgVecArgs<T> A)
{
    using S = Shape<P>;
    __shared__ double sh[16 * 4];
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    const double mb = A.sc->mean_b;
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            T b = A.bvec[gi];
            if (SING) {
                b = (T)((double)b - mb);
                A.bvec[gi] = b;
            }
            A.r[gi] = b;
            if (!A.keep_x) A.x[gi] = (T)0;
            const double im = c.iJw * inv_w<P>(k);
            const double rm = (double)b * im;
            red[1] += rm * rm;
            red[3] += im * im;
            if (A.d || A.dtab) {  // 1/diag(A), stored or computed
                const T di = inv_diag<P, T>(A, c, k, gi);
                const T z = b * di;
                A.p[gi] = z;
                red[0] += (double)b * (double)z;
                red[2] += (double)di;
            }
        }
    }
    publish_partials<4>(red, A.partial, gridDim.x, sh);
}

// x += alpha p, r -= alpha q; reductions for rho' and the residual
template <int P, typename T, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_update(CgVecArgs<T> A)
{
    using S = Shape<P>;
    constexpr int NC = SING ? 5 : 2;
    __shared__ double sh[16 * NC];
    if (A.sc->done) return;
    const T alpha = (T)A.sc->alpha;
    const double mr = SING ? A.sc->mean_r : 0.0;  // singular: r is stored before projection
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    double red[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) red[k] = 0.0;
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            const T p = A.p[gi];
            A.x[gi] = fma(alpha, p, A.x[gi]);
            T r0 = A.r[gi];
            if (SING) r0 = (T)((double)r0 - mr);
            const T r = fma(-alpha, A.q[gi], r0);
            A.r[gi] = r;
            const double rd = (double)r * (double)inv_diag<P, T>(A, c, k, gi);
            const double im = c.iJw * inv_w<P>(k);
            const double rm = (double)r * im;
            if (SING) {
                red[0] += (double)r;
                red[1] += (double)r * rd;
                red[2] += rd;
                red[3] += rm * rm;
                red[4] += rm * im;
            } else {
                red[0] += (double)r * rd;
                red[1] += rm * rm;
            }
        }
    }
    publish_partials<NC>(red, A.partial, gridDim.x, sh);
}

// p = r/d + beta p; singular: with r - mean r, the projection of r, which is
// not stored back: the next update subtracts the same mean (sc->mean_r stays
// until then) when it reads r, so r in memory minus mean_r is the residual
template <int P, typename T, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_pupdate(CgVecArgs<T> A)
{
    using S = Shape<P>;
    if (A.sc->done) return;
    const T beta = (T)A.sc->beta;
    const double mr = A.sc->mean_r;
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    if (!c.active) return;
#pragma unroll
    for (int k = 0; k < S::n; ++k) {
        const size_t gi = c.base + (size_t)k * S::NL;
        T r = A.r[gi];
        if (SING) r = (T)((double)r - mr);
        A.p[gi] = fma(beta, A.p[gi], r * inv_diag<P, T>(A, c, k, gi));
    }
}

// ---- FP32 update and p-update on chunks of V nodes (V = 4 where 4 divides
// P+1: P = 3, 7; V = 2 where only 2 does: P = 5)
//
// The kernels above give each lane one node per access (4 bytes in FP32), so
// a wave's load covers 256 bytes.  Here thread t < (P+1)^2 of an element
// takes the chunk of V consecutive nodes a0..a0+V-1 of row b in plane c0
// (V t = a0 + (P+1) b + (P+1)^2 c0) and the chunks V planes further on, so
// that consecutive lanes read consecutive 4V-byte chunks: one access of a
// wave covers 256 V bytes, with 1/V of the memory instructions.  Same grid,
// partial-sum slots and arithmetic per node as k_update / k_pupdate.

template <int P>
constexpr int kChunkV = (P + 1) % 4 == 0 ? 4 : ((P + 1) % 2 == 0 ? 2 : 1);
template <int P>
constexpr bool kQuad = kChunkV<P> > 1;

// 1/w_i of the GLL weights, for runtime indices
template <int P>
struct InvW {
    double v[P + 1];
};
template <int P>
constexpr InvW<P> make_invw()
{
    InvW<P> t{};
    for (int i = 0; i <= P; ++i) t.v[i] = 1.0 / kGll<P>.w[i];
    return t;
}
template <int P>
__constant__ InvW<P> c_invw = make_invw<P>();

template <int P>
struct QuadCtx {
    bool active;
    size_t base;  // first node of the first chunk; chunk r starts at base + r Q
    int a0, c0;
    double iJb;   // 1 / (J w_b)
    static constexpr int V = kChunkV<P>;        // nodes per chunk
    static constexpr int Q = V * Shape<P>::NL;  // nodes between a thread's chunks (V planes)
    static constexpr int NR = (P + 1) / V;      // chunks per thread
    using VF = float __attribute__((ext_vector_type(kChunkV<P>)));
};

template <int P>
__device__ __forceinline__ QuadCtx<P> quad_ctx(const CgVecArgs<float> &A)
{
    using S = Shape<P>;
    constexpr int n = S::n;
    QuadCtx<P> q;
    const int tid = threadIdx.x;
    const int el_loc = tid / S::NL;
    const int t = tid - el_loc * S::NL;
    const int el = blockIdx.x * S::EB + el_loc;
    const int f = QuadCtx<P>::V * t;
    q.active = (tid < S::NT) && (el < A.nel);
    q.a0 = f % n;
    q.c0 = f / (n * n);
    q.base = (size_t)el * S::N3 + f;
    q.iJb = 0.0;
    if (q.active) {
        const int nx = A.n[0], ny = A.n[1];
        const int ex = el % nx, r = el / nx, ey = r % ny, ez = r / ny;
        const float J = A.hx[ex] * A.hy[ey] * A.hz[ez] * 0.125f;
        q.iJb = c_invw<P>.v[(f / n) % n] / (double)J;
    }
    return q;
}

template <typename VF>
__device__ __forceinline__ VF ldv(const float *p) { return *reinterpret_cast<const VF *>(p); }
template <typename VF>
__device__ __forceinline__ void stv(float *p, VF v) { *reinterpret_cast<VF *>(p) = v; }

template <int P, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_update_q(CgVecArgs<float> A)
{
    using Q = QuadCtx<P>;
    using VF = typename Q::VF;
    constexpr int NC = SING ? 5 : 2, NR = Q::NR, V = Q::V;
    __shared__ double sh[16 * NC];
    if (A.sc->done) return;
    const float alpha = (float)A.sc->alpha;
    const double mr = SING ? A.sc->mean_r : 0.0;  // singular: r is stored before projection
    const Q c = quad_ctx<P>(A);
    double red[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) red[k] = 0.0;
    if (c.active) {
        VF pv[NR], xv[NR], rv[NR], qv[NR], dv[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const size_t i = c.base + (size_t)r * Q::Q;
            pv[r] = ldv<VF>(A.p + i);
            xv[r] = ldv<VF>(A.x + i);
            rv[r] = ldv<VF>(A.r + i);
            qv[r] = ldv<VF>(A.q + i);
            dv[r] = ldv<VF>(A.d + i);
        }
        VF xo[NR], ro[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                xo[r][k] = fmaf(alpha, pv[r][k], xv[r][k]);
                float r0 = rv[r][k];
                if (SING) r0 = (float)((double)r0 - mr);
                ro[r][k] = fmaf(-alpha, qv[r][k], r0);
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) stv<VF>(A.x + c.base + (size_t)r * Q::Q, xo[r]);
#pragma unroll
        for (int r = 0; r < NR; ++r) stv<VF>(A.r + c.base + (size_t)r * Q::Q, ro[r]);
        double iwa[V];
#pragma unroll
        for (int k = 0; k < V; ++k) iwa[k] = c_invw<P>.v[c.a0 + k];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double iJbc = c.iJb * c_invw<P>.v[c.c0 + V * r];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const float rk = ro[r][k];
                const double rd = (double)rk * (double)dv[r][k];
                const double im = iJbc * iwa[k];
                const double rm = (double)rk * im;
                if (SING) {
                    red[0] += (double)rk;
                    red[1] += (double)rk * rd;
                    red[2] += rd;
                    red[3] += rm * rm;
                    red[4] += rm * im;
                } else {
                    red[0] += (double)rk * rd;
                    red[1] += rm * rm;
                }
            }
        }
    }
    publish_partials<NC>(red, A.partial, gridDim.x, sh);
}

template <int P, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_pupdate_q(CgVecArgs<float> A)
{
    using Q = QuadCtx<P>;
    using VF = typename Q::VF;
    constexpr int NR = Q::NR, V = Q::V;
    if (A.sc->done) return;
    const float beta = (float)A.sc->beta;
    const double mr = A.sc->mean_r;
    const Q c = quad_ctx<P>(A);
    if (!c.active) return;
    VF rv[NR], pv[NR], dv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const size_t i = c.base + (size_t)r * Q::Q;
        rv[r] = ldv<VF>(A.r + i);
        pv[r] = ldv<VF>(A.p + i);
        dv[r] = ldv<VF>(A.d + i);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        VF o;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            float rk = rv[r][k];
            if (SING) rk = (float)((double)rk - mr);
            o[k] = fmaf(beta, pv[r][k], rk * dv[r][k]);
        }
        stv<VF>(A.p + c.base + (size_t)r * Q::Q, o);
    }
}

// chunked kernels apply: FP32, 2 | P+1, a stored 1/diag, 16-byte aligned
// vectors
template <typename T>
bool use_quad(int P, const CgVecArgs<T> &a, bool update)
{
    if constexpr (sizeof(T) != 4) {
        return false;
    } else {
        if ((P + 1) % 2 != 0 || !a.d) return false;
        auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
        bool ok = al(a.r) && al(a.p) && al(a.d);
        if (update) ok = ok && al(a.x) && al(a.q);
        return ok;
    }
}

// singular: shift = sum(M x) / sum(M)
template <int P, typename T>
__global__ void __launch_bounds__(Shape<P>::NTP) k_mean_x(CgVecArgs<T> A)
{
    using S = Shape<P>;
    __shared__ double sh[16 * 2];
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    double red[2] = {0.0, 0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            const double m = (double)(c.Jw * (T)kGll<P>.w[k]);
            red[0] += m * (double)A.x[gi];
            red[1] += m;
        }
    }
    publish_partials<2>(red, A.partial, gridDim.x, sh);
}

template <int P, typename T>
__global__ void __launch_bounds__(Shape<P>::NTP) k_shift_x(CgVecArgs<T> A)
{
    using S = Shape<P>;
    const LineCtx<P, T> c = line_ctx<P, T>(A);
    if (!c.active) return;
    const double s = A.sc->shift;
#pragma unroll
    for (int k = 0; k < S::n; ++k) {
        const size_t gi = c.base + (size_t)k * S::NL;
        A.x[gi] = (T)((double)A.x[gi] - s);
    }
}

// mixed precision: scale = RMS of the projected FP64 residual
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_ir_scale(CgVecArgs<float> A)
{
    using S = Shape<P>;
    __shared__ double sh[16];
    const LineCtx<P, float> c = line_ctx<P, float>(A);
    const double mr = A.sc->mean_r;
    double red[1] = {0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const double v = A.src64[c.base + (size_t)k * S::NL] - mr;
            red[0] += v * v;
        }
    }
    publish_partials<1>(red, A.partial, gridDim.x, sh);
}

// r32 = (r64 - mean_r) / scale_new (the first inner right-hand side)
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_ir_to_inner(CgVecArgs<float> A)
{
    using S = Shape<P>;
    const LineCtx<P, float> c = line_ctx<P, float>(A);
    const double mr = A.sc->mean_r, sn = A.sc->scale_new, inv = 1.0 / sn;
    if (blockIdx.x == 0 && threadIdx.x == 0) A.sc->scale = sn;  // no work-group reads scale here
    if (!c.active) return;
#pragma unroll
    for (int k = 0; k < S::n; ++k) {
        const size_t gi = c.base + (size_t)k * S::NL;
        A.r[gi] = (float)((A.src64[gi] - mr) * inv);
    }
}

// residual replacement: r32 = (r64 - mean_r) / scale_new, x32 = 0; sums for
// rho' = r.z (z = r/diag), ||M^-1 r||^2, sum r, sum z
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_ir_replace(CgVecArgs<float> A)
{
    using S = Shape<P>;
    __shared__ double sh[16 * 4];
    const LineCtx<P, float> c = line_ctx<P, float>(A);
    const double mr = A.sc->mean_r, inv = 1.0 / A.sc->scale_new;
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            const float r = (float)((A.src64[gi] - mr) * inv);
            A.r[gi] = r;
            A.x[gi] = 0.0f;
            const double z = (double)r * (double)inv_diag<P, float>(A, c, k, gi);
            const double rm = (double)r * (c.iJw * inv_w<P>(k));
            red[0] += (double)r * z;
            red[1] += rm * rm;
            red[2] += (double)r;
            red[3] += z;
        }
    }
    publish_partials<4>(red, A.partial, gridDim.x, sh);
}

// FP64 CG restarted from a given residual (the start from the caller's
// initial guess, and the continuation of a mixed solve whose FP32 recurrence
// stalls): r = r - mean_r (singular), p = r/diag; sums for rho = r.p,
// ||M^-1 r||^2, sum 1/diag, sum 1/M^2.  x keeps its value.
template <int P, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_restart64(CgVecArgs<double> A)
{
    using S = Shape<P>;
    __shared__ double sh[16 * 4];
    const LineCtx<P, double> c = line_ctx<P, double>(A);
    const double mr = A.sc->mean_r;
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    if (A.sc->bnorm2 == 0.0) {  // b = 0: the solution is x = 0 whatever the start
        if (c.active)
#pragma unroll
            for (int k = 0; k < S::n; ++k) A.x[c.base + (size_t)k * S::NL] = 0.0;
    } else if (c.active) {
        double rv[S::n], dv[S::n];
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            rv[k] = A.r[c.base + (size_t)k * S::NL];
            dv[k] = inv_diag<P, double>(A, c, k, c.base + (size_t)k * S::NL);
        }
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            const double r = SING ? rv[k] - mr : rv[k];
            if (SING) A.r[gi] = r;
            const double z = r * dv[k];
            A.p[gi] = z;
            const double im = c.iJw * inv_w<P>(k);
            const double rm = r * im;
            red[0] += r * z;
            red[1] += rm * rm;
            red[2] += dv[k];
            red[3] += im * im;
        }
    }
    publish_partials<4>(red, A.partial, gridDim.x, sh);
}

// Sums of NC partial-sum arrays partial[c * nblk + 0..nblk) taken by the
// calling work-group, this thread's share in t[c].  The loads of all
// components are issued together (summing one component after another would
// wait for one L2 round trip per component); two accumulators per component,
// combined in a fixed order, so the result does not depend on timing.
template <int NC>
__device__ __forceinline__ void sum_partials(const double *partial, int nblk, double (&t)[NC])
{
    double a[NC], b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) a[c] = b[c] = 0.0;
    const int B = blockDim.x;
    int k = threadIdx.x;
    for (; k + B < nblk; k += 2 * B) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            a[c] += partial[(size_t)c * nblk + k];
            b[c] += partial[(size_t)c * nblk + k + B];
        }
    }
    if (k < nblk) {
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] += partial[(size_t)c * nblk + k];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) t[c] = a[c] + b[c];
}

// ---- CG preconditioned by the fast-diagonalisation inverse (FP64) --------
//
// z = F r is formed by the transform kernels (fdm.hip) between the update
// and the r.z reduction, so one step is: apply (q = A p, alpha), update
// (x, r, residual norm, stopping test), F, r.z partials, p-update (beta from
// the partials, no finishing kernel).

// x += alpha p, r -= alpha q; sums of (r/M)^2 (singular: also r and r/M^2,
// for the norm of the projected residual)
template <int P, bool SING>
__global__ void __launch_bounds__(Shape<P>::NTP) k_update_fdm(CgVecArgs<double> A)
{
    using S = Shape<P>;
    constexpr int NC = SING ? 3 : 1;
    __shared__ double sh[16 * NC];
    if (A.sc->done) return;
    const double alpha = A.sc->alpha;
    const double mr = SING ? A.sc->mean_r : 0.0;
    const LineCtx<P, double> c = line_ctx<P, double>(A);
    double red[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) red[k] = 0.0;
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            A.x[gi] = fma(alpha, A.p[gi], A.x[gi]);
            const double r = fma(-alpha, A.q[gi], A.r[gi] - mr);
            A.r[gi] = r;
            const double im = c.iJw * inv_w<P>(k);
            const double rm = r * im;
            if (SING) {
                red[0] += r;
                red[1] += rm * rm;
                red[2] += rm * im;
            } else {
                red[0] += rm * rm;
            }
        }
    }
    publish_partials<NC>(red, A.partial, gridDim.x, sh);
}

// sum (r - mean_r) z
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_rz(CgVecArgs<double> A)
{
    using S = Shape<P>;
    __shared__ double sh[16];
    if (A.sc->done) return;
    const double mr = A.sc->mean_r;
    const LineCtx<P, double> c = line_ctx<P, double>(A);
    double red[1] = {0.0};
    if (c.active) {
#pragma unroll
        for (int k = 0; k < S::n; ++k) {
            const size_t gi = c.base + (size_t)k * S::NL;
            red[0] += (A.r[gi] - mr) * A.z[gi];
        }
    }
    publish_partials<1>(red, A.partial, gridDim.x, sh);
}

// p = z + beta p with beta = rho'/rho: every work-group sums k_rz's partials
// (same grid, so gridDim.x of them) in the same fixed order, so all hold the
// same rho'; work-group 0 leaves it in rho_next, and rho itself changes only
// in the next apply's finish
template <int P, bool START>
__global__ void __launch_bounds__(Shape<P>::NTP) k_pupdate_fdm(CgVecArgs<double> A)
{
    using S = Shape<P>;
    __shared__ double sh[16];
    if (A.sc->done) return;
    double rz[1];
    sum_partials<1>(A.partial, (int)gridDim.x, rz);
    block_sum<1>(rz, sh);
    if (threadIdx.x == 0) sh[0] = rz[0];
    __syncthreads();
    const double rho_new = sh[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.sc->rho_next = rho_new;
        A.sc->rho_pending = 1;
    }
    const double beta = START ? 0.0 : rho_new / A.sc->rho;
    const LineCtx<P, double> c = line_ctx<P, double>(A);
    if (!c.active) return;
#pragma unroll
    for (int k = 0; k < S::n; ++k) {
        const size_t gi = c.base + (size_t)k * S::NL;
        A.p[gi] = START ? A.z[gi] : fma(beta, A.p[gi], A.z[gi]);
    }
}

// start from r = b - A x: x = 0 if b = 0
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_fdm_zero_x(CgVecArgs<double> A)
{
    using S = Shape<P>;
    if (A.sc->bnorm2 != 0.0) return;
    const LineCtx<P, double> c = line_ctx<P, double>(A);
    if (!c.active) return;
#pragma unroll
    for (int k = 0; k < S::n; ++k) A.x[c.base + (size_t)k * S::NL] = 0.0;
}

__global__ void k_fdm_start_scalars(CgScalars *sc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double res2 = sc->true_res2;
    sc->res2 = res2;
    sc->iter = 0;
    sc->status = DG_OK;
    sc->done = 0;
    sc->rho = 0.0;
    if (!isfinite(res2)) {
        sc->status = DG_ERR_NONFINITE;
        sc->done = 1;
    } else if (sc->bnorm2 == 0.0 || res2 == 0.0 || (sc->fixed_iters <= 0 && res2 <= sc->tol2)) {
        sc->done = 1;
    }
}

__global__ void __launch_bounds__(1024) k_finish_restart64(const double *partial, int nblk, CgScalars *sc)
{
    __shared__ double sh[16 * 4];
    double t[4];
    sum_partials<4>(partial, nblk, t);
    block_sum<4>(t, sh);
    if (threadIdx.x != 0) return;
    sc->rho = t[0];
    sc->res2 = t[1];
    sc->sum_invd = t[2];
    sc->sum_invM2 = t[3];
    sc->mean_r = 0.0;
    sc->iter = 0;
    sc->status = DG_OK;
    sc->done = 0;
    if (!isfinite(t[0]) || !isfinite(t[1])) {
        sc->status = DG_ERR_NONFINITE;
        sc->done = 1;
    } else if (sc->bnorm2 == 0.0 || t[1] == 0.0 || (sc->fixed_iters <= 0 && t[1] <= sc->tol2)) {
        sc->done = 1;
    }
}

__global__ void __launch_bounds__(1024) k_finish_replace(const double *partial, int nblk, CgScalars *in,
                                                        CgScalars *out, double delta2, int restart,
                                                        int maxit)
{
    __shared__ double sh[16 * 4];
    double t[4];
    sum_partials<4>(partial, nblk, t);
    block_sum<4>(t, sh);
    if (threadIdx.x != 0) return;
    double rz = t[0], mr = 0.0;
    if (in->singular) {
        mr = t[2] / (double)in->ndof;
        rz = t[0] - 2.0 * mr * t[3] + mr * mr * in->sum_invd;
    }
    // the recurrence residual being replaced belongs to the step that set
    // done; its predecessor's r.z is rho_prev
    const double sn = out->scale_new;
    in->beta = restart ? 0.0 : (rz / in->rho_prev) * (sn / out->scale);
    in->rho = rz;
    in->mean_r = mr;
    in->res2 = t[1];
    const double floor2 = out->tol2 / (sn * sn);
    in->tol2 = delta2 * t[1] > floor2 ? delta2 * t[1] : floor2;
    in->status = DG_OK;
    in->done = 0;
    in->maxit = maxit;
    if (!isfinite(rz) || !isfinite(t[1])) {
        in->status = DG_ERR_NONFINITE;
        in->done = 1;
    }
    out->scale = sn;
}

// x64 += scale * x32
template <int P>
__global__ void __launch_bounds__(Shape<P>::NTP) k_ir_accumulate(CgVecArgs<float> A)
{
    using S = Shape<P>;
    const LineCtx<P, float> c = line_ctx<P, float>(A);
    if (!c.active) return;
    const double s = A.sc->scale;
#pragma unroll
    for (int k = 0; k < S::n; ++k) {
        const size_t gi = c.base + (size_t)k * S::NL;
        A.dst64[gi] = fma(s, (double)A.x[gi], A.dst64[gi]);
    }
}

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// ------------------------------------------------------- finish kernels --
//
// One work-group sums the partials of the preceding kernel (fixed order) and
// updates the solve's scalars.  Partials are written with plain stores and
// read here after the kernel boundary, so no device-wide fences or atomics
// are needed on the hot path.
template <int NC, int OP>
__global__ void __launch_bounds__(1024) k_finish(const double *partial, int nblk, CgScalars *sc)
{
    __shared__ double sh[16 * NC];
    if ((OP == FIN_APPLY || OP == FIN_UPDATE || OP == FIN_UPDATE_FDM) && sc->done) return;
    double tot[NC];
    sum_partials<NC>(partial, nblk, tot);
    block_sum<NC>(tot, sh);
    if (threadIdx.x != 0) return;
    if constexpr (OP == FIN_APPLY) {
        cg_after_apply(sc, tot[0], tot[1]);
    } else if constexpr (OP == FIN_RESID) {
        resid_finish(sc, *reinterpret_cast<const double(*)[4]>(tot));
    } else if constexpr (OP == FIN_SETUP1) {
        sc->mean_b = sc->singular ? tot[0] / (double)sc->ndof : 0.0;
        if (!isfinite(tot[1])) {
            sc->status = DG_ERR_NONFINITE;
            sc->done = 1;
        }
    } else if constexpr (OP == FIN_SETUP2) {
        sc->rho = tot[0];
        sc->bnorm2 = tot[1];
        sc->res2 = tot[1];
        sc->true_res2 = tot[1];
        sc->sum_invd = tot[2];
        sc->sum_invM2 = tot[3];
        sc->tol2 = sc->tol2 * tot[1];  // host stored tol^2
        sc->iter = 0;
        sc->mean_r = 0.0;
        if (!isfinite(tot[1]) || !isfinite(tot[0])) {
            sc->status = DG_ERR_NONFINITE;
            sc->done = 1;
        } else if (tot[1] == 0.0 || (sc->fixed_iters <= 0 && tot[1] <= sc->tol2)) {
            sc->done = 1;
        }
    } else if constexpr (OP == FIN_UPDATE) {
        double rz, res2;
        if (NC == 5) {  // singular: r was projected to mean zero
            const double mr = tot[0] / (double)sc->ndof;
            rz = tot[1] - 2.0 * mr * tot[2] + mr * mr * sc->sum_invd;
            res2 = tot[3] - 2.0 * mr * tot[NC - 1] + mr * mr * sc->sum_invM2;
            sc->mean_r = mr;
        } else {
            rz = tot[0];
            res2 = tot[1];
            sc->mean_r = 0.0;
        }
        if (res2 < 0.0) res2 = 0.0;
        sc->beta = rz / sc->rho;
        sc->rho_prev = sc->rho;
        sc->rho = rz;
        sc->res2 = res2;
        sc->iter += 1;
        if (!isfinite(rz) || !isfinite(res2)) {
            sc->status = DG_ERR_NONFINITE;
            sc->done = 1;
        } else if (sc->fixed_iters > 0) {
            if (sc->iter >= sc->fixed_iters) sc->done = 1;
        } else if (res2 <= sc->tol2) {
            sc->done = 1;
        } else if (sc->iter >= sc->maxit) {
            sc->status = DG_NOT_CONVERGED;
            sc->done = 1;
        }
    } else if constexpr (OP == FIN_UPDATE_FDM) {
        double res2;
        if (NC == 3) {  // singular: norm of r - mean r
            const double mr = tot[0] / (double)sc->ndof;
            res2 = tot[1] - 2.0 * mr * tot[NC - 1] + mr * mr * sc->sum_invM2;
            sc->mean_r = mr;
        } else {
            res2 = tot[0];
            sc->mean_r = 0.0;
        }
        if (res2 < 0.0) res2 = 0.0;
        sc->res2 = res2;
        sc->iter += 1;
        if (!isfinite(res2)) {
            sc->status = DG_ERR_NONFINITE;
            sc->done = 1;
        } else if (sc->fixed_iters > 0) {
            if (sc->iter >= sc->fixed_iters) sc->done = 1;
        } else if (res2 <= sc->tol2) {
            sc->done = 1;
        } else if (sc->iter >= sc->maxit) {
            sc->status = DG_NOT_CONVERGED;
            sc->done = 1;
        }
    } else if constexpr (OP == FIN_MEANX) {
        sc->shift = tot[0] / tot[1];
    } else if constexpr (OP == FIN_IRSCALE) {
        // a power of two, so that changing the scaling is exact
        const double rms = sqrt(tot[0] / (double)sc->ndof);
        sc->scale_new = (rms > 0.0 && isfinite(rms)) ? exp2(rint(log2(rms))) : 1.0;
    }
}

}  // namespace

// ------------------------------------------------------------ launchers --

template <typename F>
static int with_P(int P, F &&f)
{
    switch (P) {
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        default: set_error("polynomial degree outside 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

template <typename F>
static void with_bool(bool b, F &&f)
{
    if (b) f(std::true_type{});
    else f(std::false_type{});
}

static void fill_h(const MeshDev &m, CgVecArgs<double> &a)
{
    a.hx = m.h64;
    a.hy = m.h64 + m.n[0];
    a.hz = m.h64 + m.n[0] + m.n[1];
}
static void fill_h(const MeshDev &m, CgVecArgs<float> &a)
{
    a.hx = m.h32;
    a.hy = m.h32 + m.n[0];
    a.hz = m.h32 + m.n[0] + m.n[1];
}

template <typename T>
static void prep(const MeshDev &m, CgVecArgs<T> &a)
{
    fill_h(m, a);
    for (int d = 0; d < 3; ++d) a.n[d] = m.n[d];
    a.nel = (int)m.nel;
    a.ngroups = apply_groups(m.P, m.nel);
}

#define DG_GRID(PC) dim3(apply_groups(decltype(PC)::value, m.nel)), dim3(Shape<decltype(PC)::value>::NTP)

template <typename T>
int cg_setup(const MeshDev &m, CgVecArgs<T> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        with_bool(a.singular, [&](auto SC) {
            constexpr bool SG = decltype(SC)::value;
            const int nb = apply_groups(P, m.nel);
            hipLaunchKernelGGL((k_setup1<P, T, SG>), DG_GRID(PC), 0, s, a);
            hipLaunchKernelGGL((k_finish<2, FIN_SETUP1>), dim3(1), dim3(1024), 0, s, a.partial, nb, a.sc);
            hipLaunchKernelGGL((k_setup2<P, T, SG>), DG_GRID(PC), 0, s, a);
            hipLaunchKernelGGL((k_finish<4, FIN_SETUP2>), dim3(1), dim3(1024), 0, s, a.partial, nb, a.sc);
        });
    });
}

template <typename T>
int cg_update(const MeshDev &m, CgVecArgs<T> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        with_bool(a.singular, [&](auto SC) {
            constexpr bool SG = decltype(SC)::value;
            const int nb = apply_groups(P, m.nel);
            if constexpr (std::is_same<T, float>::value && kQuad<P>) {
                if (use_quad<T>(P, a, true))
                    hipLaunchKernelGGL((k_update_q<P, SG>), DG_GRID(PC), 0, s, a);
                else
                    hipLaunchKernelGGL((k_update<P, T, SG>), DG_GRID(PC), 0, s, a);
            } else {
                hipLaunchKernelGGL((k_update<P, T, SG>), DG_GRID(PC), 0, s, a);
            }
            hipLaunchKernelGGL((k_finish<SG ? 5 : 2, FIN_UPDATE>), dim3(1), dim3(1024), 0, s,
                               a.partial, nb, a.sc);
        });
    });
}

template <typename T>
int cg_pupdate(const MeshDev &m, CgVecArgs<T> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        with_bool(a.singular, [&](auto SC) {
            constexpr bool SG = decltype(SC)::value;
            if constexpr (std::is_same<T, float>::value && kQuad<P>) {
                if (use_quad<T>(P, a, false))
                    hipLaunchKernelGGL((k_pupdate_q<P, SG>), DG_GRID(PC), 0, s, a);
                else
                    hipLaunchKernelGGL((k_pupdate<P, T, SG>), DG_GRID(PC), 0, s, a);
            } else {
                hipLaunchKernelGGL((k_pupdate<P, T, SG>), DG_GRID(PC), 0, s, a);
            }
        });
    });
}

template <typename T>
int cg_finish(const MeshDev &m, CgVecArgs<T> a, hipStream_t s)
{
    prep(m, a);
    if (!a.singular) return DG_OK;
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_mean_x<P, T>), DG_GRID(PC), 0, s, a);
        hipLaunchKernelGGL((k_finish<2, FIN_MEANX>), dim3(1), dim3(1024), 0, s, a.partial,
                           apply_groups(P, m.nel), a.sc);
        hipLaunchKernelGGL((k_shift_x<P, T>), DG_GRID(PC), 0, s, a);
    });
}

int ir_scale(const MeshDev &m, CgVecArgs<float> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_ir_scale<P>), DG_GRID(PC), 0, s, a);
        hipLaunchKernelGGL((k_finish<1, FIN_IRSCALE>), dim3(1), dim3(1024), 0, s, a.partial,
                           apply_groups(P, m.nel), a.sc);
    });
}

int ir_to_inner(const MeshDev &m, CgVecArgs<float> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_ir_to_inner<P>), DG_GRID(PC), 0, s, a);
    });
}

int ir_replace(const MeshDev &m, CgVecArgs<float> a, CgScalars *inner, double delta2, bool restart,
               int maxit, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_ir_replace<P>), DG_GRID(PC), 0, s, a);
        hipLaunchKernelGGL(k_finish_replace, dim3(1), dim3(1024), 0, s, a.partial, apply_groups(P, m.nel),
                           inner, a.sc, delta2, restart ? 1 : 0, maxit);
    });
}

int cg_restart64(const MeshDev &m, CgVecArgs<double> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        with_bool(a.singular, [&](auto SC) {
            constexpr bool SG = decltype(SC)::value;
            hipLaunchKernelGGL((k_restart64<P, SG>), DG_GRID(PC), 0, s, a);
        });
        hipLaunchKernelGGL(k_finish_restart64, dim3(1), dim3(1024), 0, s, a.partial,
                           apply_groups(P, m.nel), a.sc);
    });
}

int ir_accumulate(const MeshDev &m, CgVecArgs<float> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_ir_accumulate<P>), DG_GRID(PC), 0, s, a);
    });
}

int convert_f64_to_f32(const double *a, float *b, size_t n, hipStream_t s)
{
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)std::max<size_t>(blocks, 1)), dim3(256), 0, s,
                       a, b, n);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

int launch_finish_apply(double *partial, int nblk, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL((k_finish<2, FIN_APPLY>), dim3(1), dim3(1024), 0, s, partial, nblk, sc);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

int launch_finish_resid(double *partial, int nblk, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL((k_finish<4, FIN_RESID>), dim3(1), dim3(1024), 0, s, partial, nblk, sc);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

int cg_fdm_start(const MeshDev &m, CgVecArgs<double> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_fdm_zero_x<P>), DG_GRID(PC), 0, s, a);
        hipLaunchKernelGGL(k_fdm_start_scalars, dim3(1), dim3(64), 0, s, a.sc);
    });
}

int cg_update_fdm(const MeshDev &m, CgVecArgs<double> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        const int nb = apply_groups(P, m.nel);
        with_bool(a.singular, [&](auto SC) {
            constexpr bool SG = decltype(SC)::value;
            hipLaunchKernelGGL((k_update_fdm<P, SG>), DG_GRID(PC), 0, s, a);
            hipLaunchKernelGGL((k_finish<SG ? 3 : 1, FIN_UPDATE_FDM>), dim3(1), dim3(1024), 0, s,
                               a.partial, nb, a.sc);
        });
    });
}

int cg_rz(const MeshDev &m, CgVecArgs<double> a, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL((k_rz<P>), DG_GRID(PC), 0, s, a);
    });
}

int cg_pupdate_fdm(const MeshDev &m, CgVecArgs<double> a, bool start, hipStream_t s)
{
    prep(m, a);
    return with_P(m.P, [&](auto PC) {
        constexpr int P = decltype(PC)::value;
        with_bool(start, [&](auto SC) {
            hipLaunchKernelGGL((k_pupdate_fdm<P, decltype(SC)::value>), DG_GRID(PC), 0, s, a);
        });
    });
}

template int cg_setup<double>(const MeshDev &, CgVecArgs<double>, hipStream_t);
template int cg_setup<float>(const MeshDev &, CgVecArgs<float>, hipStream_t);
template int cg_update<double>(const MeshDev &, CgVecArgs<double>, hipStream_t);
template int cg_update<float>(const MeshDev &, CgVecArgs<float>, hipStream_t);
template int cg_pupdate<double>(const MeshDev &, CgVecArgs<double>, hipStream_t);
template int cg_pupdate<float>(const MeshDev &, CgVecArgs<float>, hipStream_t);
template int cg_finish<double>(const MeshDev &, CgVecArgs<double>, hipStream_t);
template int cg_finish<float>(const MeshDev &, CgVecArgs<float>, hipStream_t);

}  // namespace dg
