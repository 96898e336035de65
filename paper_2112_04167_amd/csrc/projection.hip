// Projection substep of Alg. 3 (arXiv 2112.04167) with the pressure at
// degree P-1 and the velocity at degree P (Sec. 3.3): the DG divergence of a
// velocity field, the DG gradient of a pressure field, and the velocity
// update v'' = v' - grad psi (gfx950).
//
// Both operators use the (P+1)-point GLL rule of the velocity, which is
// exact for the products involved (degree 2P-1 per direction):
//
//   D(v; v_b)_q = - sum_K int_K v . grad q + sum_F(interior) int_F {v}.n [q]
//                 + sum_F(boundary) int_F (v_b . n_out) q,
//   (G psi, w)  = sum_K int_K grad psi . w - sum_F(interior) int_F [psi] n.{w},
//
// q ranging over the pressure basis (tensor-product Lagrange polynomials of
// degree P-1 on its own GLL nodes) and w over the velocity basis; G is minus
// the adjoint of D without boundary data under the GLL masses.  With
// collocation at the velocity nodes, G psi at a node is the derivative of the
// pressure interpolant there, minus, on each interior face through the node,
// the jump of psi across the face divided by (w_face h) -- the face integral
// of the lifted jump over the node's mass.
//
// One work-group per element: the element's data is staged in LDS and the
// 1D factors (interpolation Vq and derivative dVq of the pressure basis at
// the velocity nodes) are applied one direction at a time, to the three
// components at once.  The face terms read the neighbour's face layer from
// global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"
#include "dg_internal.h"
#include "projection.h"

namespace dg {

namespace {

constexpr int kN = kMaxN;  // velocity nodes per direction, at most 9

// The scalar space is the pressure (degree Q = P - 1) or, for the
// variable-viscosity terms, the velocity space itself (Q = P).
struct ProjTables {
    double Vq[kN][kN];   // scalar basis value at velocity node:  Vq[a][i] = l_i(xi_a)
    double dVq[kN][kN];  // its derivative on [-1, 1]
    double w[kN];        // velocity GLL weights
};

struct ProjArgs {
    ProjTables t;
    const double *v[3];   // velocity (div) / update input (grad)
    const double *vb[3];  // boundary data (div; null: v_b = 0)
    const double *psi;    // pressure (grad)
    double *out;          // weak divergence (div), or its nodal form (nodal)
    double *g[3];         // gradient or updated velocity (grad)
    const double *h[3];   // element extents per axis
    int n[3], bc[3];
    double scale;         // div: factor on the weak vector; grad: factor on G psi
    int update;           // grad: g = v + scale G psi instead of scale G psi
    const double *fac;    // grad: nodal factor on scale G psi; nodal div: on the nodal result (null: 1)
    int nodal;            // div, equal order: out = fac scale M^-1 D(v; v_b), M the GLL mass
};

// neighbour of element index k along an axis: -1 on a non-periodic boundary
__host__ __device__ __forceinline__ int neighbour(int k, int nk, int bc, bool high)
{
    int kn = high ? k + 1 : k - 1;
    if (kn < 0 || kn >= nk) {
        if (bc != DG_BC_PERIODIC) return -1;
        kn = (kn + nk) % nk;
    }
    return kn;
}

// element-major offset of element (ex, ey, ez)
__host__ __device__ __forceinline__ size_t elem_base(const ProjArgs &A, int ex, int ey, int ez, int nodes)
{
    return ((size_t)(ez * A.n[1] + ey) * A.n[0] + ex) * nodes;
}

// index of node (a, b, c) [x fastest] and of the node at position (s, t) of
// the face layer `layer` normal to axis d (s: the lower tangential axis)
template <int n>
__host__ __device__ __forceinline__ int node3(int a, int b, int c) { return (c * n + b) * n + a; }
template <int n>
__host__ __device__ __forceinline__ int face_node(int d, int layer, int s, int t)
{
    return d == 0 ? node3<n>(layer, s, t) : d == 1 ? node3<n>(s, layer, t) : node3<n>(s, t, layer);
}

// ------------------------------------------- divergence and gradient --
// All three components of an element are contracted at once, one line per
// thread and pass, so that an element takes four (gradient) or five
// (divergence) barriers whatever its faces.  Component d's derivative axis
// is contracted last (divergence) or first (gradient), and its two face
// terms ride along as two extra layers on that axis: the tangential
// contractions act on them exactly as on the volume layers, and the last
// (first) pass adds them to the face layer of the output.  Buffers are in
// LDS; the phases are plain functions of the thread index, so that they can
// be run for every thread in turn on the host.

// the tangential axes of axis d, ascending
__host__ __device__ __forceinline__ int tan1(int d) { return d == 0 ? 1 : 0; }
__host__ __device__ __forceinline__ int tan2(int d) { return d == 2 ? 1 : 2; }
// entry d of a three-vector, d not known at compile time
__host__ __device__ __forceinline__ double sel3(int d, const double (&v)[3])
{
    return d == 0 ? v[0] : d == 1 ? v[1] : v[2];
}
// stride of an axis in a layout with axis 0 fastest and extents e0, e1
__host__ __device__ __forceinline__ int stride_of(int axis, int e0, int e1)
{
    return axis == 0 ? 1 : axis == 1 ? e0 : e0 * e1;
}
// extents of a per-component buffer: E along axis d, et1 and et2 along its
// tangential axes; the stride of `axis` in it
__host__ __device__ __forceinline__ int comp_stride(int axis, int d, int E, int et1, int et2)
{
    const int u1 = tan1(d);
    const int e0 = d == 0 ? E : (u1 == 0 ? et1 : et2);
    const int e1 = d == 1 ? E : (u1 == 1 ? et1 : et2);
    return stride_of(axis, e0, e1);
}

template <int P, int Q>
struct DivShape {
    static constexpr int n = P + 1, m = Q + 1, E = n + 2, n3 = n * n * n, m3 = m * m * m;
    static constexpr int X = E * n * n;  // scaled velocity plus face layers, per component
    static constexpr int Y = E * n * m;  // after the first tangential contraction
    static constexpr int Z = E * m * m;  // after the second
    static constexpr int BUF_A = 3 * X;  // X, later Z
    static constexpr int BUF_B = 3 * Y;  // Y, later the three components' results (m^3 each)
    // threads per work-group: one per line of the largest pass (3 (P+1)
    // (P+3) lines, 297 at P = 8), so that every pass is a single step
    static constexpr int NT = 3 * n * E <= 256 ? 256 : 320;
    static_assert(Z <= X && m3 <= Y, "buffer reuse");
};

// the velocity GLL weights in LDS (read with lane-dependent indices); the
// passes read the 1D factors from the kernel arguments, at indices known at
// compile time and the same on every lane
template <int P>
__host__ __device__ __forceinline__ void proj_weights(const ProjArgs &A, int tid, int nt, double *tw)
{
    for (int i = tid; i < P + 1; i += nt) tw[i] = A.t.w[i];
}

// X_d: the velocity component d times the GLL mass (layers 0..n-1 along d),
// then the face terms +- omega0 w_s w_t f of the low and high faces normal
// to d (layers n, n+1), f = {v_d}, v_b,d or 0 (no term)
template <int P, int Q>
__host__ __device__ __forceinline__ void div_load(const ProjArgs &A, int el, int tid, int nt, const double *tw,
                                                  double *bufA)
{
    using S = DivShape<P, Q>;
    constexpr int n = S::n, E = S::E, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const double J = hh[0] * hh[1] * hh[2] * 0.125;
    const size_t vb0 = elem_base(A, ex, ey, ez, n3);
    for (int r = tid; r < 3 * n3; r += nt) {
        const int d = r / n3, i = r - d * n3;
        const int a = i % n, b = (i / n) % n, c = i / (n * n);
        const int k = comp_stride(0, d, E, n, n) * a + comp_stride(1, d, E, n, n) * b +
                      comp_stride(2, d, E, n, n) * c;
        bufA[d * S::X + k] = tw[a] * tw[b] * tw[c] * J * A.v[d][vb0 + i];
    }
    for (int r = tid; r < 6 * n * n; r += nt) {
        const int face = r / (n * n), st = r - face * n * n, s = st % n, t = st / n;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        const int own = face_node<n>(d, high ? n - 1 : 0, s, t);
        double f = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            const size_t nb0 = elem_base(A, en[0], en[1], en[2], n3);
            f = 0.5 * (A.v[d][vb0 + own] + A.v[d][nb0 + face_node<n>(d, high ? 0 : n - 1, s, t)]);
        } else if (A.vb[d]) {
            f = A.vb[d][vb0 + own];
        }
        const int u1 = tan1(d), u2 = tan2(d);
        const double omega0 = (u1 == 0 ? hh[0] : hh[1]) * (u2 == 1 ? hh[1] : hh[2]) * 0.25;
        const int k = comp_stride(d, d, E, n, n) * (n + (high ? 1 : 0)) + comp_stride(u1, d, E, n, n) * s +
                      comp_stride(u2, d, E, n, n) * t;
        bufA[d * S::X + k] = (high ? omega0 : -omega0) * tw[s] * tw[t] * f;
    }
}

// pass 1: Vq along the first tangential axis (n -> m), X_d -> Y_d
template <int P, int Q>
__host__ __device__ __forceinline__ void div_pass1(const ProjTables &tab, int tid, const double *bufA,
                                                   double *bufB)
{
    using S = DivShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = n * E;
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, q = r - d * T, k2 = q % n, kd = q / n;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *x = bufA + d * S::X + comp_stride(u2, d, E, n, n) * k2 + comp_stride(d, d, E, n, n) * kd;
        const int sx = comp_stride(u1, d, E, n, n);
        double *y = bufB + d * S::Y + comp_stride(u2, d, E, m, n) * k2 + comp_stride(d, d, E, m, n) * kd;
        const int sy = comp_stride(u1, d, E, m, n);
        double xv[n];
#pragma unroll
        for (int k = 0; k < n; ++k) xv[k] = x[k * sx];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) s += tab.Vq[k][i] * xv[k];
            y[i * sy] = s;
        }
    }
}

// pass 2: Vq along the second tangential axis (n -> m), Y_d -> Z_d
template <int P, int Q>
__host__ __device__ __forceinline__ void div_pass2(const ProjTables &tab, int tid, const double *bufB,
                                                   double *bufA)
{
    using S = DivShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = m * E;
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, q = r - d * T, i1 = q % m, kd = q / m;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *y = bufB + d * S::Y + comp_stride(u1, d, E, m, n) * i1 + comp_stride(d, d, E, m, n) * kd;
        const int sy = comp_stride(u2, d, E, m, n);
        double *z = bufA + d * S::Z + comp_stride(u1, d, E, m, m) * i1 + comp_stride(d, d, E, m, m) * kd;
        const int sz = comp_stride(u2, d, E, m, m);
        double yv[n];
#pragma unroll
        for (int k = 0; k < n; ++k) yv[k] = y[k * sy];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) s += tab.Vq[k][i] * yv[k];
            z[i * sz] = s;
        }
    }
}

// pass 3: minus (2/h_d) dVq along d on the volume layers, plus the face
// layers on the first and last pressure layers; Z_d -> R_d (pressure layout)
template <int P, int Q>
__host__ __device__ __forceinline__ void div_pass3(const ProjArgs &A, const ProjTables &tab, int el, int tid,
                                                   const double *bufA,
                                                   double *bufB)
{
    using S = DivShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = m * m;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, q = r - d * T, i1 = q % m, i2 = q / m;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *z = bufA + d * S::Z + comp_stride(u1, d, E, m, m) * i1 + comp_stride(u2, d, E, m, m) * i2;
        const int sz = comp_stride(d, d, E, m, m);
        double *out = bufB + d * S::m3 + stride_of(u1, m, m) * i1 + stride_of(u2, m, m) * i2;
        const int so = stride_of(d, m, m);
        const double gd = 2.0 / sel3(d, hh);
        double zv[E];
#pragma unroll
        for (int k = 0; k < E; ++k) zv[k] = z[k * sz];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) s += tab.dVq[k][i] * zv[k];
            double o = -gd * s;
            if (i == 0) o += zv[n];
            if (i == m - 1) o += zv[n + 1];
            out[i * so] = o;
        }
    }
}

template <int P, int Q>
__host__ __device__ __forceinline__ void div_store(const ProjArgs &A, int el, int tid, int nt, const double *bufB)
{
    using S = DivShape<P, Q>;
    constexpr int m3 = S::m3;
    const size_t pb = (size_t)el * m3;
    for (int i = tid; i < m3; i += nt) A.out[pb + i] = A.scale * (bufB[i] + bufB[m3 + i] + bufB[2 * m3 + i]);
}

template <int P, int Q>
__global__ void __launch_bounds__((DivShape<P, Q>::NT)) k_divergence(ProjArgs A)
{
    using S = DivShape<P, Q>;
    __shared__ double tw[S::n];
    __shared__ double bufA[S::BUF_A], bufB[S::BUF_B];
    const int el = blockIdx.x, tid = threadIdx.x, nt = S::NT;
    proj_weights<P>(A, tid, nt, tw);
    __syncthreads();
    div_load<P, Q>(A, el, tid, nt, tw, bufA);
    __syncthreads();
    div_pass1<P, Q>(A.t, tid, bufA, bufB);
    __syncthreads();
    div_pass2<P, Q>(A.t, tid, bufB, bufA);
    __syncthreads();
    div_pass3<P, Q>(A, A.t, el, tid, bufA, bufB);
    __syncthreads();
    div_store<P, Q>(A, el, tid, nt, bufB);
}

template <int P, int Q>
struct GradShape {
    static constexpr int n = P + 1, m = Q + 1, E = n + 2, n3 = n * n * n, m3 = m * m * m;
    static constexpr int W1 = E * m * m;  // (2/h_d) dVq along d, plus the two face jumps
    static constexpr int W2 = E * n * m;  // after the first tangential interpolation
    static constexpr int W3 = E * n * n;  // after the second
    static constexpr int BUF_A = 3 * W3;  // W1, later W3
    static constexpr int BUF_B = 3 * W2;
    // threads per work-group: 256; at P = 8 the largest pass has 297 lines
    // and takes two steps (measured faster than 320 threads)
    static constexpr int NT = 256;
    static_assert(W1 <= W3, "buffer reuse");
};

// the element's pressure and its neighbours' traces on the six faces,
// [face][it][is] (is along the lower tangential axis)
template <int P, int Q>
__host__ __device__ __forceinline__ void grad_load(const ProjArgs &A, int el, int tid, int nt, double *q,
                                                   double *qn)
{
    constexpr int m = Q + 1, m3 = m * m * m;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const size_t pbase = elem_base(A, ex, ey, ez, m3);
    for (int i = tid; i < m3; i += nt) q[i] = A.psi[pbase + i];
    for (int r = tid; r < 6 * m * m; r += nt) {
        const int face = r / (m * m), i = r - face * m * m, is = i % m, it = i / m;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        double oth = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            oth = A.psi[elem_base(A, en[0], en[1], en[2], m3) + face_node<m>(d, high ? 0 : m - 1, is, it)];
        }
        qn[r] = oth;
    }
}

// pass 1: (2/h_d) dVq along d (m -> n) on the pressure lines along d, and on
// layers n, n+1 the jumps psi_L - psi_R across the low and high faces (0
// without a neighbour); pressure -> W1_d
template <int P, int Q>
__host__ __device__ __forceinline__ void grad_pass1(const ProjArgs &A, const ProjTables &tab, int el, int tid,
                                                    const double *q,
                                                    const double *qn, double *bufA)
{
    using S = GradShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = m * m;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, t = r - d * T, i1 = t % m, i2 = t / m;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *ql = q + stride_of(u1, m, m) * i1 + stride_of(u2, m, m) * i2;
        const int sq = stride_of(d, m, m);
        double *w = bufA + d * S::W1 + comp_stride(u1, d, E, m, m) * i1 + comp_stride(u2, d, E, m, m) * i2;
        const int sw = comp_stride(d, d, E, m, m);
        const double gd = 2.0 / sel3(d, hh);
        double qv[m];
#pragma unroll
        for (int i = 0; i < m; ++i) qv[i] = ql[i * sq];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < m; ++i) s += tab.dVq[k][i] * qv[i];
            w[k * sw] = gd * s;
        }
        const bool lo = neighbour(e3[d], A.n[d], A.bc[d], false) >= 0;
        const bool hi = neighbour(e3[d], A.n[d], A.bc[d], true) >= 0;
        w[n * sw] = lo ? qn[(2 * d) * T + t] - qv[0] : 0.0;
        w[(n + 1) * sw] = hi ? qv[m - 1] - qn[(2 * d + 1) * T + t] : 0.0;
    }
}

// pass 2: Vq along the first tangential axis (m -> n), W1_d -> W2_d
template <int P, int Q>
__host__ __device__ __forceinline__ void grad_pass2(const ProjTables &tab, int tid, const double *bufA,
                                                    double *bufB)
{
    using S = GradShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = m * E;
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, t = r - d * T, i2 = t % m, kd = t / m;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *w = bufA + d * S::W1 + comp_stride(u2, d, E, m, m) * i2 + comp_stride(d, d, E, m, m) * kd;
        const int sw = comp_stride(u1, d, E, m, m);
        double *o = bufB + d * S::W2 + comp_stride(u2, d, E, n, m) * i2 + comp_stride(d, d, E, n, m) * kd;
        const int so = comp_stride(u1, d, E, n, m);
        double wv[m];
#pragma unroll
        for (int i = 0; i < m; ++i) wv[i] = w[i * sw];
#pragma unroll
        for (int a = 0; a < n; ++a) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < m; ++i) s += tab.Vq[a][i] * wv[i];
            o[a * so] = s;
        }
    }
}

// pass 3: Vq along the second tangential axis (m -> n), W2_d -> W3_d
template <int P, int Q>
__host__ __device__ __forceinline__ void grad_pass3(const ProjTables &tab, int tid, const double *bufB,
                                                    double *bufA)
{
    using S = GradShape<P, Q>;
    constexpr int n = S::n, m = S::m, E = S::E, T = n * E;
    for (int r = tid; r < 3 * T; r += S::NT) {
        const int d = r / T, t = r - d * T, a1 = t % n, kd = t / n;
        const int u1 = tan1(d), u2 = tan2(d);
        const double *w = bufB + d * S::W2 + comp_stride(u1, d, E, n, m) * a1 + comp_stride(d, d, E, n, m) * kd;
        const int sw = comp_stride(u2, d, E, n, m);
        double *o = bufA + d * S::W3 + comp_stride(u1, d, E, n, n) * a1 + comp_stride(d, d, E, n, n) * kd;
        const int so = comp_stride(u2, d, E, n, n);
        double wv[m];
#pragma unroll
        for (int i = 0; i < m; ++i) wv[i] = w[i * sw];
#pragma unroll
        for (int a = 0; a < n; ++a) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < m; ++i) s += tab.Vq[a][i] * wv[i];
            o[a * so] = s;
        }
    }
}

// g_d = W3_d on the volume layers, minus the interpolated jump over
// (w_face h_d) on the first and last layers along d; then the factor, the
// scale and the update
template <int P, int Q>
__host__ __device__ __forceinline__ void grad_store(const ProjArgs &A, int el, int tid, int nt, const double *tw,
                                                    const double *bufA)
{
    using S = GradShape<P, Q>;
    constexpr int n = S::n, E = S::E, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const size_t vbase = elem_base(A, ex, ey, ez, n3);
    for (int r = tid; r < 3 * n3; r += nt) {
        const int d = r / n3, i = r - d * n3;
        const int co[3] = {i % n, (i / n) % n, i / (n * n)};
        const int u1 = tan1(d), u2 = tan2(d);
        const int cd = d == 0 ? co[0] : d == 1 ? co[1] : co[2];
        const int c1 = u1 == 0 ? co[0] : co[1], c2 = u2 == 1 ? co[1] : co[2];
        const double *w = bufA + d * S::W3 + comp_stride(u1, d, E, n, n) * c1 + comp_stride(u2, d, E, n, n) * c2;
        const int sw = comp_stride(d, d, E, n, n);
        double g = w[cd * sw];
        if (cd == 0) g -= (1.0 / (tw[0] * sel3(d, hh))) * w[n * sw];
        if (cd == n - 1) g -= (1.0 / (tw[n - 1] * sel3(d, hh))) * w[(n + 1) * sw];
        const double gv = A.fac ? A.scale * g * A.fac[vbase + i] : A.scale * g;
        A.g[d][vbase + i] = A.update ? A.v[d][vbase + i] + gv : gv;
    }
}

template <int P, int Q>
__global__ void __launch_bounds__((GradShape<P, Q>::NT)) k_gradient(ProjArgs A)
{
    using S = GradShape<P, Q>;
    __shared__ double tw[S::n];
    __shared__ double q[S::m3], qn[6 * S::m * S::m];
    __shared__ double bufA[S::BUF_A], bufB[S::BUF_B];
    const int el = blockIdx.x, tid = threadIdx.x, nt = S::NT;
    proj_weights<P>(A, tid, nt, tw);
    grad_load<P, Q>(A, el, tid, nt, q, qn);
    __syncthreads();
    grad_pass1<P, Q>(A, A.t, el, tid, q, qn, bufA);
    __syncthreads();
    grad_pass2<P, Q>(A.t, tid, bufA, bufB);
    __syncthreads();
    grad_pass3<P, Q>(A.t, tid, bufB, bufA);
    __syncthreads();
    grad_store<P, Q>(A, el, tid, nt, tw, bufA);
}

// ------------------------------------------------ equal-order variants --
// With the scalar space equal to the velocity space (Q = P) the
// interpolation factor Vq is the identity (exact zeros and ones from the
// product formula), so only the derivative pass along each axis remains:
// one 1D contraction per component, along the component's own axis, and
// the face terms act on the face nodes directly.  One thread takes one line
// of one component (3 (P+1)^2 lines, at most 243), with the derivative
// matrix from the kernel arguments at compile-time indices (the GLL weights
// of the divergence from LDS); a last pass sums (divergence) or scales and
// stores (gradient) node by node.
template <int P>
struct EqShape {
    static constexpr int n = P + 1, n2 = n * n, n3 = n2 * n;
    static constexpr int NT = 256;
    static_assert(3 * n2 <= NT, "one line per thread");
};

// the element's three velocity components (raw) and the face values f of
// the six faces (axis d, side; [t][s]): the mean of the two traces, the
// wall data, or 0 (no term)
template <int P>
__host__ __device__ __forceinline__ void eqdiv_load(const ProjArgs &A, int el, int tid, double *tv, double *fv,
                                                    double *tw)
{
    using S = EqShape<P>;
    constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const size_t vb0 = elem_base(A, ex, ey, ez, n3);
    for (int i = tid; i < n; i += S::NT) tw[i] = A.t.w[i];
    for (int r = tid; r < 3 * n3; r += S::NT) {
        const int d = r / n3, i = r - d * n3;
        tv[r] = A.v[d][vb0 + i];
    }
    for (int r = tid; r < 6 * n2; r += S::NT) {
        const int face = r / n2, st = r - face * n2, s = st % n, t = st / n;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int layer = high ? n - 1 : 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        double f = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            const size_t nb0 = elem_base(A, en[0], en[1], en[2], n3);
            f = 0.5 * (A.v[d][vb0 + face_node<n>(d, layer, s, t)] +
                       A.v[d][nb0 + face_node<n>(d, high ? 0 : n - 1, s, t)]);
        } else if (A.vb[d]) {
            f = A.vb[d][vb0 + face_node<n>(d, layer, s, t)];
        }
        fv[r] = f;
    }
}

// the line of component d at tangential position (s, t): minus (2/h_d) dV^T
// of the GLL-weighted values, plus the face terms on its end nodes; written
// back in place (every line is read whole before any is written, within
// its own thread, and lines are disjoint)
template <int P>
__host__ __device__ __forceinline__ void eqdiv_lines(const ProjArgs &A, const ProjTables &tab, int el, int tid,
                                                     double *tv, const double *fv, const double *tw)
{
    using S = EqShape<P>;
    constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const double J = hh[0] * hh[1] * hh[2] * 0.125;
    const int r = tid;
    if (r < 3 * n2) {
        const int d = r / n2, st = r - d * n2, s = st % n, t = st / n;
        const int u1 = tan1(d), u2 = tan2(d);
        double *x = tv + d * n3 + stride_of(u1, n, n) * s + stride_of(u2, n, n) * t;
        const int sd = stride_of(d, n, n);
        const double wst = tw[s] * tw[t];
        double xv[n];
#pragma unroll
        for (int k = 0; k < n; ++k) xv[k] = tw[k] * x[k * sd];
        const double c = wst * J, gd = 2.0 / sel3(d, hh);
        const double omega0 = (u1 == 0 ? hh[0] : hh[1]) * (u2 == 1 ? hh[1] : hh[2]) * 0.25;
        const double flo = fv[(2 * d) * n2 + st], fhi = fv[(2 * d + 1) * n2 + st];
        // rows of dV^T in the outer loop: each row is contiguous in the
        // kernel arguments, so its scalar loads stay few and short-lived
        double sum[n];
#pragma unroll
        for (int i = 0; i < n; ++i) sum[i] = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k)
#pragma unroll
            for (int i = 0; i < n; ++i) sum[i] += tab.dVq[k][i] * xv[k];
#pragma unroll
        for (int i = 0; i < n; ++i) {
            double o = -(gd * c) * sum[i];
            if (i == 0) o -= omega0 * wst * flo;
            if (i == n - 1) o += omega0 * wst * fhi;
            x[i * sd] = o;
        }
    }
}

// out = scale x (weak), or with A.nodal scale x (fac or 1) / M, x the sum of
// the three components' parts
template <int P>
__host__ __device__ __forceinline__ void eqdiv_store(const ProjArgs &A, int el, int tid, const double *tv,
                                                     const double *tw)
{
    using S = EqShape<P>;
    constexpr int n = S::n, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const double J = A.h[0][ex] * A.h[1][ey] * A.h[2][ez] * 0.125;
    const size_t vb0 = (size_t)el * n3;
    for (int i = tid; i < n3; i += S::NT) {
        const double x = tv[i] + tv[n3 + i] + tv[2 * n3 + i];
        if (A.nodal) {
            const int a = i % n, b = (i / n) % n, c = i / (n * n);
            const double v = A.scale * x / (J * tw[a] * tw[b] * tw[c]);
            A.out[vb0 + i] = A.fac ? v * A.fac[vb0 + i] : v;
        } else {
            A.out[vb0 + i] = A.scale * x;
        }
    }
}

template <int P>
__global__ void __launch_bounds__(EqShape<P>::NT) k_divergence_eq(ProjArgs A)
{
    using S = EqShape<P>;
    __shared__ double tv[3 * S::n3], fv[6 * S::n2], tw[S::n];
    const int el = blockIdx.x, tid = threadIdx.x;
    eqdiv_load<P>(A, el, tid, tv, fv, tw);
    __syncthreads();
    eqdiv_lines<P>(A, A.t, el, tid, tv, fv, tw);
    __syncthreads();
    eqdiv_store<P>(A, el, tid, tv, tw);
}

// the element's scalar and the neighbours' traces on the six faces (axis d,
// side; [t][s])
template <int P>
__host__ __device__ __forceinline__ void eqgrad_load(const ProjArgs &A, int el, int tid, double *q, double *qn)
{
    using S = EqShape<P>;
    constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const size_t base = elem_base(A, ex, ey, ez, n3);
    for (int r = tid; r < n3; r += S::NT) q[r] = A.psi[base + r];
    for (int r = tid; r < 6 * n2; r += S::NT) {
        const int face = r / n2, st = r - face * n2, s = st % n, t = st / n;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        double oth = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            oth = A.psi[elem_base(A, en[0], en[1], en[2], n3) + face_node<n>(d, high ? 0 : n - 1, s, t)];
        }
        qn[r] = oth;
    }
}

// the line along d at tangential position (s, t): (2/h_d) dV of the scalar,
// minus the jump over (w_face h_d) on the end nodes whose face has a
// neighbour; into the component's slot of R
template <int P>
__host__ __device__ __forceinline__ void eqgrad_lines(const ProjArgs &A, const ProjTables &tab, int el, int tid,
                                                      const double *q, const double *qn, double *R)
{
    using S = EqShape<P>;
    constexpr int n = S::n, n2 = S::n2, n3 = S::n3;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const int r = tid;
    if (r < 3 * n2) {
        const int d = r / n2, st = r - d * n2, s = st % n, t = st / n;
        const int u1 = tan1(d), u2 = tan2(d);
        const int off = stride_of(u1, n, n) * s + stride_of(u2, n, n) * t, sd = stride_of(d, n, n);
        double xv[n];
#pragma unroll
        for (int k = 0; k < n; ++k) xv[k] = q[off + k * sd];
        const double hd = sel3(d, hh), gd = 2.0 / hd;
        const bool lo = neighbour(e3[d], A.n[d], A.bc[d], false) >= 0;
        const bool hi = neighbour(e3[d], A.n[d], A.bc[d], true) >= 0;
        double *o = R + d * n3 + off;
#pragma unroll
        for (int i = 0; i < n; ++i) {
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) sum += tab.dVq[i][k] * xv[k];
            double g = gd * sum;
            if (i == 0 && lo) g -= (1.0 / (tab.w[0] * hd)) * (qn[(2 * d) * n2 + st] - xv[0]);
            if (i == n - 1 && hi) g -= (1.0 / (tab.w[n - 1] * hd)) * (xv[n - 1] - qn[(2 * d + 1) * n2 + st]);
            o[i * sd] = g;
        }
    }
}

template <int P>
__host__ __device__ __forceinline__ void eqgrad_store(const ProjArgs &A, int el, int tid, const double *R)
{
    using S = EqShape<P>;
    constexpr int n3 = S::n3;
    const size_t base = (size_t)el * n3;
    for (int r = tid; r < 3 * n3; r += S::NT) {
        const int d = r / n3, i = r - d * n3;
        const double gv = A.fac ? A.scale * R[r] * A.fac[base + i] : A.scale * R[r];
        A.g[d][base + i] = A.update ? A.v[d][base + i] + gv : gv;
    }
}

template <int P>
__global__ void __launch_bounds__(EqShape<P>::NT) k_gradient_eq(ProjArgs A)
{
    using S = EqShape<P>;
    __shared__ double q[S::n3], qn[6 * S::n2], R[3 * S::n3];
    const int el = blockIdx.x, tid = threadIdx.x;
    eqgrad_load<P>(A, el, tid, q, qn);
    __syncthreads();
    eqgrad_lines<P>(A, A.t, el, tid, q, qn, R);
    __syncthreads();
    eqgrad_store<P>(A, el, tid, R);
}

ProjTables make_tables(int P, int Q)
{
    ProjTables t{};
    const GllTables &gv = gll_cached(P);
    const GllTables &gp = gll_cached(Q);
    const int n = P + 1, m = Q + 1;
    for (int a = 0; a < n; ++a) {
        t.w[a] = gv.w[a];
        const double x = gv.xi[a];
        for (int i = 0; i < m; ++i) {
            // Lagrange basis l_i of the pressure nodes and its derivative at x
            double l = 1.0, dl = 0.0;
            for (int k = 0; k < m; ++k) {
                if (k == i) continue;
                const double r = 1.0 / (gp.xi[i] - gp.xi[k]);
                dl = dl * (x - gp.xi[k]) * r + l * r;
                l *= (x - gp.xi[k]) * r;
            }
            t.Vq[a][i] = l;
            t.dVq[a][i] = dl;
        }
    }
    return t;
}

// the (velocity degree, scalar degree) pairs: (P, P - 1) for P = 4..8 and
// (P, P) for P = 3..8
template <typename F>
int with_pair(int P, int Q, F &&f)
{
    using std::integral_constant;
    if (Q == P - 1) {
        switch (P) {
            case 4: f(integral_constant<int, 4>{}, integral_constant<int, 3>{}); break;
            case 5: f(integral_constant<int, 5>{}, integral_constant<int, 4>{}); break;
            case 6: f(integral_constant<int, 6>{}, integral_constant<int, 5>{}); break;
            case 7: f(integral_constant<int, 7>{}, integral_constant<int, 6>{}); break;
            case 8: f(integral_constant<int, 8>{}, integral_constant<int, 7>{}); break;
            default: set_error("the projection needs a velocity degree 4..8 (pressure 3..7)"); return DG_ERR_ARG;
        }
    } else {
        switch (P) {
            case 3: f(integral_constant<int, 3>{}, integral_constant<int, 3>{}); break;
            case 4: f(integral_constant<int, 4>{}, integral_constant<int, 4>{}); break;
            case 5: f(integral_constant<int, 5>{}, integral_constant<int, 5>{}); break;
            case 6: f(integral_constant<int, 6>{}, integral_constant<int, 6>{}); break;
            case 7: f(integral_constant<int, 7>{}, integral_constant<int, 7>{}); break;
            case 8: f(integral_constant<int, 8>{}, integral_constant<int, 8>{}); break;
            default: set_error("degree outside 3..8"); return DG_ERR_ARG;
        }
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

int check_pair(const MeshDev &mv, const MeshDev &mp)
{
    if (mp.P != mv.P - 1 && mp.P != mv.P) {
        set_error("the scalar mesh must have degree P-1 (pressure) or P of the velocity mesh");
        return DG_ERR_ARG;
    }
    for (int d = 0; d < 3; ++d)
        if (mp.n[d] != mv.n[d] || mp.v[d] != mv.v[d] || mp.bc[d] != mv.bc[d]) {
            set_error("the pressure and velocity meshes must share elements, vertices and BCs");
            return DG_ERR_ARG;
        }
    return DG_OK;
}

ProjArgs base_args(const MeshDev &mv, const MeshDev &mp)
{
    ProjArgs a{};
    a.t = make_tables(mv.P, mp.P);
    for (int d = 0; d < 3; ++d) {
        a.n[d] = mv.n[d];
        a.bc[d] = mv.bc[d];
    }
    a.h[0] = mv.h64;
    a.h[1] = mv.h64 + mv.n[0];
    a.h[2] = mv.h64 + mv.n[0] + mv.n[1];
    return a;
}

}  // namespace

int launch_divergence(const MeshDev &mv, const MeshDev &mp, const double *const v[3],
                      const double *const vb[3], double scale, double *out, hipStream_t s)
{
    if (int rc = check_pair(mv, mp)) return rc;
    ProjArgs a = base_args(mv, mp);
    for (int d = 0; d < 3; ++d) {
        a.v[d] = v[d];
        a.vb[d] = vb ? vb[d] : nullptr;
    }
    a.out = out;
    a.scale = scale;
    return with_pair(mv.P, mp.P, [&](auto PC, auto QC) {
        constexpr int Pv = decltype(PC)::value, Qv = decltype(QC)::value;
        if constexpr (Pv == Qv)
            hipLaunchKernelGGL((k_divergence_eq<Pv>), dim3((unsigned)mv.nel), dim3(EqShape<Pv>::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_divergence<Pv, Qv>), dim3((unsigned)mv.nel), dim3(DivShape<Pv, Qv>::NT), 0, s, a);
    });
}

int launch_divergence_nodal(const MeshDev &m, const double *const v[3], const double *const vb[3], double scale,
                            const double *fac, double *out, hipStream_t s)
{
    ProjArgs a = base_args(m, m);
    for (int d = 0; d < 3; ++d) {
        a.v[d] = v[d];
        a.vb[d] = vb ? vb[d] : nullptr;
    }
    a.out = out;
    a.scale = scale;
    a.fac = fac;
    a.nodal = 1;
    return with_pair(m.P, m.P, [&](auto PC, auto) {
        constexpr int Pv = decltype(PC)::value;
        hipLaunchKernelGGL((k_divergence_eq<Pv>), dim3((unsigned)m.nel), dim3(EqShape<Pv>::NT), 0, s, a);
    });
}

int launch_gradient(const MeshDev &mv, const MeshDev &mp, const double *psi, const double *const v[3],
                    double scale, double *const g[3], hipStream_t s, const double *fac)
{
    if (int rc = check_pair(mv, mp)) return rc;
    ProjArgs a = base_args(mv, mp);
    a.psi = psi;
    a.fac = fac;
    a.update = v ? 1 : 0;
    a.scale = scale;
    for (int d = 0; d < 3; ++d) {
        a.v[d] = v ? v[d] : nullptr;
        a.g[d] = g[d];
    }
    return with_pair(mv.P, mp.P, [&](auto PC, auto QC) {
        constexpr int Pv = decltype(PC)::value, Qv = decltype(QC)::value;
        if constexpr (Pv == Qv)
            hipLaunchKernelGGL((k_gradient_eq<Pv>), dim3((unsigned)mv.nel), dim3(EqShape<Pv>::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_gradient<Pv, Qv>), dim3((unsigned)mv.nel), dim3(GradShape<Pv, Qv>::NT), 0, s, a);
    });
}

// ----------------------------------------------------- nodal kernels --
namespace {

struct NodalArgs {
    const double *h[3];
    double w[kN];
    int n[3], P;
    size_t N;
};

NodalArgs nodal_args(const MeshDev &m)
{
    NodalArgs a{};
    const GllTables &g = gll_cached(m.P);
    for (int i = 0; i <= m.P; ++i) a.w[i] = g.w[i];
    a.h[0] = m.h64;
    a.h[1] = m.h64 + m.n[0];
    a.h[2] = m.h64 + m.n[0] + m.n[1];
    for (int d = 0; d < 3; ++d) a.n[d] = m.n[d];
    a.P = m.P;
    a.N = (size_t)m.ndof;
    return a;
}

// One work-group per element for the GLL-mass kernels: the node's position
// in the element and the element's extents come from 32-bit block and thread
// indices (no 64-bit division per node), and the weights from LDS (read
// from the kernel arguments with lane-dependent indices they would be
// vector loads).  The mass of node (a, b, c) is J w_a w_b w_c, J the
// element's h_x h_y h_z / 8.
template <int P>
__device__ __forceinline__ void element_mass_setup(const NodalArgs &A, double (&tw)[P + 1], double &J,
                                                   size_t &base)
{
    constexpr int n = P + 1;
    if (threadIdx.x < n) tw[threadIdx.x] = A.w[threadIdx.x];
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    J = A.h[0][ex] * A.h[1][ey] * A.h[2][ez] * 0.125;
    base = (size_t)el * (n * n * n);
    __syncthreads();
}

// out = s * x * (f or 1) / M   (weak vector -> scaled nodal field)
template <int P>
__global__ void __launch_bounds__(256) k_weak_to_nodal(NodalArgs A, const double *x, const double *f, double s,
                                                       double *out)
{
    constexpr int n = P + 1, n3 = n * n * n;
    __shared__ double tw[n];
    double J;
    size_t base;
    element_mass_setup<P>(A, tw, J, base);
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
        const int a = r % n, b = (r / n) % n, c = r / (n * n);
        const double v = s * x[base + r] / (J * tw[a] * tw[b] * tw[c]);
        out[base + r] = f ? v * f[base + r] : v;
    }
}

__global__ void k_viscosity(const double *vx, const double *vy, const double *vz, size_t N, double nu0,
                            double nu1, double ivref2, double *nu)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const double x = vx[i], y = vy[i], z = vz[i];
        nu[i] = nu0 + nu1 * (x * x + y * y + z * z) * ivref2;
    }
}

// out = (out or 0) + s M x  (nodal field -> weak vector, M the GLL mass)
template <int P>
__global__ void __launch_bounds__(256) k_mass(NodalArgs A, const double *x, double s, int accumulate, double *out)
{
    constexpr int n = P + 1, n3 = n * n * n;
    __shared__ double tw[n];
    double J;
    size_t base;
    element_mass_setup<P>(A, tw, J, base);
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
        const int a = r % n, b = (r / n) % n, c = r / (n * n);
        const double v = s * x[base + r] * (J * tw[a] * tw[b] * tw[c]);
        out[base + r] = accumulate ? out[base + r] + v : v;
    }
}

// Nitsche load of Dirichlet data g on the faces of one side of axis d:
// b += scale [ int_F sigma g phi - int_F nu d_n(phi) g ], sigma = nu (P+1)^2 / h
// (the SIP form's Dirichlet face), GLL rule on the face.  One thread per face
// node: the penalty term lands on the node itself, the consistency term on
// the node's normal line (d_n phi_k = +-(2/h) l_k'(+-1)), so the threads of
// one launch touch disjoint nodes.
struct DirArgs {
    const double *h[3];
    double w[kN], D0[kN], DP[kN];  // GLL weights, l_k'(-1), l_k'(+1)
    int n[3], d, high;
    const double *nu;
    double nu_c;
    const double *g;
    double scale;
    double *b;
};

template <int P>
__global__ void k_dirichlet_load(DirArgs A)
{
    constexpr int n = P + 1, n3 = n * n * n;
    const int d = A.d, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const size_t total = (size_t)A.n[t1] * A.n[t2] * n * n;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int st = (int)(idx % (n * n));
        const size_t q = idx / (n * n);
        const int s = st % n, t = st / n;
        int e[3];
        e[d] = A.high ? A.n[d] - 1 : 0;
        e[t1] = (int)(q % A.n[t1]);
        e[t2] = (int)(q / A.n[t1]);
        const size_t base = ((size_t)(e[2] * A.n[1] + e[1]) * A.n[0] + e[0]) * n3;
        const int layer = A.high ? n - 1 : 0;
        const int f = face_node<n>(d, layer, s, t);
        const double h = A.h[d][e[d]];
        const double omega = A.w[s] * A.w[t] * A.h[t1][e[t1]] * A.h[t2][e[t2]] * 0.25;
        const double nuf = A.nu ? A.nu[base + f] : A.nu_c;
        const double gf = A.g[base + f];
        A.b[base + f] += A.scale * omega * (nuf * n * n / h) * gf;
        const double sgn = A.high ? 2.0 / h : -2.0 / h;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            const double dn = sgn * (A.high ? A.DP[k] : A.D0[k]);
            A.b[base + face_node<n>(d, k, s, t)] -= A.scale * omega * nuf * dn * gf;
        }
    }
}

constexpr int kMaxComb = 32;
struct CombArgs {
    const double *x0;
    const double *x[kMaxComb];
    double c[kMaxComb];
    int k;
    size_t N;
    double *y;
};

__global__ void k_lincomb(CombArgs A)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.N; i += (size_t)gridDim.x * blockDim.x) {
        double s = A.x0 ? A.x0[i] : 0.0;
        for (int j = 0; j < A.k; ++j) s = fma(A.c[j], A.x[j][i], s);
        A.y[i] = s;
    }
}

// the same two values per thread with 16-byte accesses (N even, every
// vector 16-byte aligned); the same arithmetic per value
__global__ void k_lincomb2(CombArgs A)
{
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const size_t N2 = A.N / 2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2; i += (size_t)gridDim.x * blockDim.x) {
        dv2 s = A.x0 ? ((const dv2 *)A.x0)[i] : dv2{0.0, 0.0};
        for (int j = 0; j < A.k; ++j) {
            const dv2 xj = ((const dv2 *)A.x[j])[i];
            s.x = fma(A.c[j], xj.x, s.x);
            s.y = fma(A.c[j], xj.y, s.y);
        }
        ((dv2 *)A.y)[i] = s;
    }
}

// launch a kernel templated on the degree (3..8)
template <template <int> class K, typename... Args>
int launch_by_degree(int P, dim3 grid, hipStream_t st, Args... args)
{
    switch (P) {
        case 3: hipLaunchKernelGGL(K<3>::fn, grid, dim3(256), 0, st, args...); break;
        case 4: hipLaunchKernelGGL(K<4>::fn, grid, dim3(256), 0, st, args...); break;
        case 5: hipLaunchKernelGGL(K<5>::fn, grid, dim3(256), 0, st, args...); break;
        case 6: hipLaunchKernelGGL(K<6>::fn, grid, dim3(256), 0, st, args...); break;
        case 7: hipLaunchKernelGGL(K<7>::fn, grid, dim3(256), 0, st, args...); break;
        case 8: hipLaunchKernelGGL(K<8>::fn, grid, dim3(256), 0, st, args...); break;
        default: set_error("degree outside 3..8"); return DG_ERR_ARG;
    }
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}
template <int P>
struct WeakToNodalK {
    static constexpr auto fn = k_weak_to_nodal<P>;
};
template <int P>
struct MassK {
    static constexpr auto fn = k_mass<P>;
};

dim3 flat_grid(size_t N) { return dim3((unsigned)std::max<size_t>(1, std::min<size_t>((N + 255) / 256, 8192))); }

}  // namespace

int launch_weak_to_nodal(const MeshDev &m, const double *x, const double *f, double s, double *out,
                         hipStream_t st)
{
    if (m.nel == 0) return DG_OK;
    return launch_by_degree<WeakToNodalK>(m.P, dim3((unsigned)m.nel), st, nodal_args(m), x, f, s, out);
}

int launch_viscosity(const MeshDev &m, const double *const v[3], double nu0, double nu1, double vref,
                     double *nu, hipStream_t st)
{
    const size_t N = (size_t)m.ndof;
    hipLaunchKernelGGL(k_viscosity, flat_grid(N), dim3(256), 0, st, v[0], v[1], v[2], N, nu0, nu1,
                       1.0 / (vref * vref), nu);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

int launch_mass(const MeshDev &m, const double *x, double s, bool accumulate, double *out, hipStream_t st)
{
    if (m.nel == 0) return DG_OK;
    return launch_by_degree<MassK>(m.P, dim3((unsigned)m.nel), st, nodal_args(m), x, s, accumulate ? 1 : 0, out);
}

int launch_dirichlet_load(const MeshDev &m, const int bc[3], const double *nu, double nu_c, const double *g,
                          double scale, double *b, hipStream_t st)
{
    DirArgs a{};
    const GllTables &gt = gll_cached(m.P);
    const int n = m.P + 1;
    for (int k = 0; k < n; ++k) {
        a.w[k] = gt.w[k];
        a.D0[k] = gt.D[0 * n + k];
        a.DP[k] = gt.D[(n - 1) * n + k];
    }
    a.h[0] = m.h64;
    a.h[1] = m.h64 + m.n[0];
    a.h[2] = m.h64 + m.n[0] + m.n[1];
    for (int d = 0; d < 3; ++d) a.n[d] = m.n[d];
    a.nu = nu;
    a.nu_c = nu_c;
    a.g = g;
    a.scale = scale;
    a.b = b;
    for (int d = 0; d < 3; ++d) {
        if (bc[d] != DG_BC_DIRICHLET) continue;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const size_t total = (size_t)m.n[t1] * m.n[t2] * n * n;
        const dim3 grid((unsigned)std::max<size_t>(1, std::min<size_t>((total + 255) / 256, 8192)));
        for (int hi = 0; hi < 2; ++hi) {  // one side per launch: their normal lines may share nodes
            a.d = d;
            a.high = hi;
            switch (m.P) {
                case 3: hipLaunchKernelGGL(k_dirichlet_load<3>, grid, dim3(256), 0, st, a); break;
                case 4: hipLaunchKernelGGL(k_dirichlet_load<4>, grid, dim3(256), 0, st, a); break;
                case 5: hipLaunchKernelGGL(k_dirichlet_load<5>, grid, dim3(256), 0, st, a); break;
                case 6: hipLaunchKernelGGL(k_dirichlet_load<6>, grid, dim3(256), 0, st, a); break;
                case 7: hipLaunchKernelGGL(k_dirichlet_load<7>, grid, dim3(256), 0, st, a); break;
                case 8: hipLaunchKernelGGL(k_dirichlet_load<8>, grid, dim3(256), 0, st, a); break;
                default: set_error("degree outside 3..8"); return DG_ERR_ARG;
            }
            DG_HIP_CHECK(hipGetLastError());
        }
    }
    return DG_OK;
}

int launch_lincomb(size_t N, const double *x0, int k, const double *c, const double *const *xs, double *y,
                   hipStream_t st)
{
    if (k < 0 || k > kMaxComb) {
        set_error("at most 32 terms in a linear combination");
        return DG_ERR_ARG;
    }
    CombArgs a{};
    a.x0 = x0;
    a.k = k;
    a.N = N;
    a.y = y;
    bool vec = N % 2 == 0 && ((uintptr_t)y % 16) == 0 && ((uintptr_t)x0 % 16) == 0;
    for (int j = 0; j < k; ++j) {
        a.c[j] = c[j];
        a.x[j] = xs[j];
        vec = vec && ((uintptr_t)xs[j] % 16) == 0;
    }
    if (vec)
        hipLaunchKernelGGL(k_lincomb2, flat_grid(N / 2), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_lincomb, flat_grid(N), dim3(256), 0, st, a);
    DG_HIP_CHECK(hipGetLastError());
    return DG_OK;
}

}  // namespace dg
