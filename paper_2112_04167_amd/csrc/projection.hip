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
// the velocity nodes) are applied one direction at a time.  The face terms
// read the neighbour's face layer from global memory.
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
    double *out;          // weak divergence (div)
    double *g[3];         // gradient or updated velocity (grad)
    const double *h[3];   // element extents per axis
    int n[3], bc[3];
    double scale;         // div: factor on the weak vector; grad: factor on G psi
    int update;           // grad: g = v + scale G psi instead of scale G psi
    const double *fac;    // grad: nodal factor on scale G psi (null: 1)
};

// neighbour of element index k along an axis: -1 on a non-periodic boundary
__device__ __forceinline__ int neighbour(int k, int nk, int bc, bool high)
{
    int kn = high ? k + 1 : k - 1;
    if (kn < 0 || kn >= nk) {
        if (bc != DG_BC_PERIODIC) return -1;
        kn = (kn + nk) % nk;
    }
    return kn;
}

// element-major offset of element (ex, ey, ez)
__device__ __forceinline__ size_t elem_base(const ProjArgs &A, int ex, int ey, int ez, int nodes)
{
    return ((size_t)(ez * A.n[1] + ey) * A.n[0] + ex) * nodes;
}

// index of node (a, b, c) [x fastest] and of the node at position (s, t) of
// the face layer `layer` normal to axis d (s: the lower tangential axis)
template <int n>
__device__ __forceinline__ int node3(int a, int b, int c) { return (c * n + b) * n + a; }
template <int n>
__device__ __forceinline__ int face_node(int d, int layer, int s, int t)
{
    return d == 0 ? node3<n>(layer, s, t) : d == 1 ? node3<n>(s, layer, t) : node3<n>(s, t, layer);
}

// ---------------------------------------------------------- divergence --
template <int P, int Q>
__global__ void __launch_bounds__(256) k_divergence(ProjArgs A)
{
    constexpr int n = P + 1, m = Q + 1, n3 = n * n * n, m3 = m * m * m;
    // the 1D tables in LDS: their lane-dependent rows would otherwise be
    // vector loads from the kernel arguments, one per multiply-add
    __shared__ double tV[n * m], tdV[n * m], tw[n];
    for (int i = threadIdx.x; i < n * m; i += blockDim.x) {
        tV[i] = A.t.Vq[i / m][i % m];
        tdV[i] = A.t.dVq[i / m][i % m];
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = A.t.w[i];
    __syncthreads();
    __shared__ double tv[n3];       // scaled velocity component
    __shared__ double s1[n * n * m];
    __shared__ double s2[n * m * m];
    __shared__ double acc[m3];
    __shared__ double fs[n * n], fq[n * m];
    // the face values f = {v_d} or v_b,d of the six faces (axis d, side),
    // [t][s], staged at the start so that their global loads are in flight
    // with the first component's
    __shared__ double fv[6][n * n];
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hx = A.h[0][ex], hy = A.h[1][ey], hz = A.h[2][ez];
    const double hh[3] = {hx, hy, hz};
    const double J = hx * hy * hz * 0.125;
    const size_t vb0 = elem_base(A, ex, ey, ez, n3);
    for (int i = threadIdx.x; i < m3; i += blockDim.x) acc[i] = 0.0;
    for (int r = threadIdx.x; r < 6 * n * n; r += blockDim.x) {
        const int face = r / (n * n), i = r - face * n * n, sn = i % n, tn = i / n;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        const int own = face_node<n>(d, high ? n - 1 : 0, sn, tn);
        double f = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            const size_t nb0 = elem_base(A, en[0], en[1], en[2], n3);
            f = 0.5 * (A.v[d][vb0 + own] + A.v[d][nb0 + face_node<n>(d, high ? 0 : n - 1, sn, tn)]);
        } else if (A.vb[d]) {
            f = A.vb[d][vb0 + own];
        }
        fv[face][i] = f;
    }
    // volume: acc -= (A2 (x) A1 (x) A0)^T (W J v_d), A_d = (2/h_d) dVq, others Vq
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {
            const int a = i % n, b = (i / n) % n, c = i / (n * n);
            tv[i] = tw[a] * tw[b] * tw[c] * J * A.v[d][vb0 + i];
        }
        __syncthreads();
        const double gd = 2.0 / hh[d];
        // over a (x): s1[c][b][ix]
        for (int i = threadIdx.x; i < n * n * m; i += blockDim.x) {
            const int ix = i % m, cb = i / m;
            double s = 0.0;
            for (int a = 0; a < n; ++a) s += (d == 0 ? gd * tdV[(a) * m + (ix)] : tV[(a) * m + (ix)]) * tv[cb * n + a];
            s1[i] = s;
        }
        __syncthreads();
        // over b (y): s2[c][iy][ix]
        for (int i = threadIdx.x; i < n * m * m; i += blockDim.x) {
            const int ix = i % m, iy = (i / m) % m, c = i / (m * m);
            double s = 0.0;
            for (int b = 0; b < n; ++b)
                s += (d == 1 ? gd * tdV[(b) * m + (iy)] : tV[(b) * m + (iy)]) * s1[(c * n + b) * m + ix];
            s2[i] = s;
        }
        __syncthreads();
        // over c (z)
        for (int i = threadIdx.x; i < m3; i += blockDim.x) {
            const int ix = i % m, iy = (i / m) % m, iz = i / (m * m);
            double s = 0.0;
            for (int c = 0; c < n; ++c)
                s += (d == 2 ? gd * tdV[(c) * m + (iz)] : tV[(c) * m + (iz)]) * s2[(c * m + iy) * m + ix];
            acc[i] -= s;
        }
    }
    // faces: +- sum over the face nodes of omega f q, f = {v_d} or v_b,d
    for (int d = 0; d < 3; ++d) {
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        for (int hi = 0; hi < 2; ++hi) {
            const bool high = hi == 1;
            const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
            if (kn < 0 && !A.vb[d]) continue;  // boundary with v_b = 0: no term
            const double omega0 = hh[t1] * hh[t2] * 0.25, sgn = high ? 1.0 : -1.0;
            __syncthreads();
            for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
                const int s = i % n, t = i / n;
                fs[i] = sgn * omega0 * tw[s] * tw[t] * fv[2 * d + hi][i];  // [t][s]
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n * m; i += blockDim.x) {  // over s: fq[t][is]
                const int is = i % m, t = i / m;
                double sum = 0.0;
                for (int s = 0; s < n; ++s) sum += tV[(s) * m + (is)] * fs[t * n + s];
                fq[i] = sum;
            }
            __syncthreads();
            const int ip = high ? m - 1 : 0;
            for (int i = threadIdx.x; i < m * m; i += blockDim.x) {  // over t
                const int is = i % m, it = i / m;
                double sum = 0.0;
                for (int t = 0; t < n; ++t) sum += tV[(t) * m + (it)] * fq[t * m + is];
                const int q = d == 0 ? (it * m + is) * m + ip : d == 1 ? (it * m + ip) * m + is
                                                                        : (ip * m + it) * m + is;
                acc[q] += sum;
            }
        }
    }
    __syncthreads();
    const size_t pb = (size_t)el * m3;
    for (int i = threadIdx.x; i < m3; i += blockDim.x) A.out[pb + i] = A.scale * acc[i];
}

// ------------------------------------------------------------ gradient --
template <int P, int Q>
__global__ void __launch_bounds__(256) k_gradient(ProjArgs A)
{
    constexpr int n = P + 1, m = Q + 1, n3 = n * n * n, m3 = m * m * m;
    // the 1D tables in LDS: their lane-dependent rows would otherwise be
    // vector loads from the kernel arguments, one per multiply-add
    __shared__ double tV[n * m], tdV[n * m], tw[n];
    for (int i = threadIdx.x; i < n * m; i += blockDim.x) {
        tV[i] = A.t.Vq[i / m][i % m];
        tdV[i] = A.t.dVq[i / m][i % m];
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = A.t.w[i];
    __syncthreads();
    __shared__ double q[m3];
    __shared__ double s1[m * m * n];
    __shared__ double s2[m * n * n];
    __shared__ double g[n3];
    __shared__ double jf[m * m], jt[n * m], jump[n * n];
    // the neighbours' pressure traces on the six faces (axis d, side),
    // [it][is], staged with psi so that every global load is in flight
    // before the first barrier
    __shared__ double qn[6][m * m];
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const size_t vbase = elem_base(A, ex, ey, ez, n3), pbase = elem_base(A, ex, ey, ez, m3);
    auto at = [&](int d, int layer, int s, int t) {
        return d == 0 ? (t * m + s) * m + layer : d == 1 ? (t * m + layer) * m + s : (layer * m + t) * m + s;
    };
    for (int i = threadIdx.x; i < m3; i += blockDim.x) q[i] = A.psi[pbase + i];
    for (int r = threadIdx.x; r < 6 * m * m; r += blockDim.x) {
        const int face = r / (m * m), i = r - face * m * m, is = i % m, it = i / m;
        const int d = face >> 1;
        const bool high = (face & 1) != 0;
        const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
        double oth = 0.0;
        if (kn >= 0) {
            int en[3] = {ex, ey, ez};
            en[d] = kn;
            oth = A.psi[elem_base(A, en[0], en[1], en[2], m3) + at(d, high ? 0 : m - 1, is, it)];
        }
        qn[face][i] = oth;
    }
    for (int d = 0; d < 3; ++d) {
        const double gd = 2.0 / hh[d];
        __syncthreads();
        for (int i = threadIdx.x; i < m * m * n; i += blockDim.x) {  // over ix: s1[iz][iy][a]
            const int a = i % n, r = i / n;
            double s = 0.0;
            for (int ix = 0; ix < m; ++ix) s += (d == 0 ? gd * tdV[(a) * m + (ix)] : tV[(a) * m + (ix)]) * q[r * m + ix];
            s1[i] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m * n * n; i += blockDim.x) {  // over iy: s2[iz][b][a]
            const int a = i % n, b = (i / n) % n, iz = i / (n * n);
            double s = 0.0;
            for (int iy = 0; iy < m; ++iy)
                s += (d == 1 ? gd * tdV[(b) * m + (iy)] : tV[(b) * m + (iy)]) * s1[(iz * m + iy) * n + a];
            s2[i] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {  // over iz: g[c][b][a]
            const int a = i % n, b = (i / n) % n, c = i / (n * n);
            double s = 0.0;
            for (int iz = 0; iz < m; ++iz)
                s += (d == 2 ? gd * tdV[(c) * m + (iz)] : tV[(c) * m + (iz)]) * s2[(iz * n + b) * n + a];
            g[i] = s;
        }
        // interior faces: g_d -= [psi] / (w_face h_d) on the face's nodes
        for (int hi = 0; hi < 2; ++hi) {
            const bool high = hi == 1;
            const int kn = neighbour(e3[d], A.n[d], A.bc[d], high);
            if (kn < 0) continue;
            // L = the element on the low side of the face, R the high side
            const int pl = m - 1, pr = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
                const int is = i % m, it = i / m;
                const double own = q[at(d, high ? pl : pr, is, it)];
                const double oth = qn[2 * d + hi][i];
                jf[i] = high ? own - oth : oth - own;  // psi_L - psi_R on pressure face nodes
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n * m; i += blockDim.x) {  // over is: jt[it][s]
                const int s = i % n, it = i / n;
                double sum = 0.0;
                for (int is = 0; is < m; ++is) sum += tV[(s) * m + (is)] * jf[it * m + is];
                jt[i] = sum;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n * n; i += blockDim.x) {  // over it: jump[t][s]
                const int s = i % n, t = i / n;
                double sum = 0.0;
                for (int it = 0; it < m; ++it) sum += tV[(t) * m + (it)] * jt[it * n + s];
                jump[i] = sum;
            }
            __syncthreads();
            const int layer = high ? n - 1 : 0;
            const double f = 1.0 / (tw[layer] * hh[d]);
            for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
                const int s = i % n, t = i / n;
                g[face_node<n>(d, layer, s, t)] -= f * jump[i];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n3; i += blockDim.x) {
            const double gv = A.fac ? A.scale * g[i] * A.fac[vbase + i] : A.scale * g[i];
            A.g[d][vbase + i] = A.update ? A.v[d][vbase + i] + gv : gv;
        }
    }
}

// ------------------------------------------------ equal-order variants --
// With the scalar space equal to the velocity space (Q = P) the
// interpolation factor Vq is the identity (exact zeros and ones from the
// product formula), so only the derivative pass along each axis remains:
// one 1D contraction per direction and node instead of three passes, and the
// face terms act on the face nodes directly.  Same sums in the same order as
// the general kernels above, so the results are bitwise theirs.
template <int P>
__global__ void __launch_bounds__(256) k_divergence_eq(ProjArgs A)
{
    constexpr int n = P + 1, n2 = n * n, n3 = n2 * n;
    __shared__ double tdV[n * n], tw[n];  // the 1D tables in LDS (see k_divergence)
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) tdV[i] = A.t.dVq[i / n][i % n];
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = A.t.w[i];
    __syncthreads();
    __shared__ double tv[3][n3];
    // the face values f of the six faces (axis d, side), [t][s]: the mean of
    // the two traces, the wall data, or 0 (no term), staged with the volume
    // data so that all global loads are in flight before the first barrier
    __shared__ double fv[6][n2];
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const double J = hh[0] * hh[1] * hh[2] * 0.125;
    const size_t vb0 = elem_base(A, ex, ey, ez, n3);
    for (int r = threadIdx.x; r < 3 * n3; r += blockDim.x) {
        const int d = r / n3, i = r - d * n3;
        const int a = i % n, b = (i / n) % n, c = i / (n * n);
        tv[d][i] = tw[a] * tw[b] * tw[c] * J * A.v[d][vb0 + i];
    }
    for (int r = threadIdx.x; r < 6 * n2; r += blockDim.x) {
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
            f = 0.5 * (A.v[d][vb0 + face_node<n>(d, layer, s, t)] + A.v[d][nb0 + face_node<n>(d, high ? 0 : n - 1, s, t)]);
        } else if (A.vb[d]) {
            f = A.vb[d][vb0 + face_node<n>(d, layer, s, t)];
        }
        fv[face][st] = f;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
        const int a = r % n, b = (r / n) % n, c = r / (n * n);
        const int co[3] = {a, b, c};
        double acc = 0.0;
        {
            const double gd = 2.0 / hh[0];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) sum += gd * tdV[(k) * n + (a)] * tv[0][(c * n + b) * n + k];
            acc -= sum;
        }
        {
            const double gd = 2.0 / hh[1];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) sum += gd * tdV[(k) * n + (b)] * tv[1][(c * n + k) * n + a];
            acc -= sum;
        }
        {
            const double gd = 2.0 / hh[2];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) sum += gd * tdV[(k) * n + (c)] * tv[2][(k * n + b) * n + a];
            acc -= sum;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const int s = co[t1], t = co[t2];
#pragma unroll
            for (int hi = 0; hi < 2; ++hi) {
                const bool high = hi == 1;
                if (co[d] != (high ? n - 1 : 0)) continue;
                const double omega0 = hh[t1] * hh[t2] * 0.25, sgn = high ? 1.0 : -1.0;
                acc += sgn * omega0 * tw[s] * tw[t] * fv[2 * d + hi][t * n + s];
            }
        }
        A.out[vb0 + r] = A.scale * acc;
    }
}

template <int P>
__global__ void __launch_bounds__(256) k_gradient_eq(ProjArgs A)
{
    constexpr int n = P + 1, n2 = n * n, n3 = n2 * n;
    // the 1D tables in LDS (see k_divergence); tdVt = tdV transposed, for the
    // x derivative, whose lanes run along the table's row index (strided
    // rows would put consecutive lanes on the same LDS banks)
    __shared__ double tdV[n * n], tdVt[n * n], tw[n];
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
        tdV[i] = A.t.dVq[i / n][i % n];
        tdVt[i] = A.t.dVq[i % n][i / n];
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = A.t.w[i];
    __syncthreads();
    // psi of the element, the neighbours' traces on the six faces (axis d,
    // side; [t][s]) and the nodal factor, all staged before the first
    // barrier so that their global loads are in flight together
    __shared__ double q[n3], qn[6][n2], fq[n3];
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const size_t base = elem_base(A, ex, ey, ez, n3);
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
        q[r] = A.psi[base + r];
        if (A.fac) fq[r] = A.fac[base + r];
    }
    for (int r = threadIdx.x; r < 6 * n2; r += blockDim.x) {
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
        qn[face][st] = oth;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n3; r += blockDim.x) {
        const int a = r % n, b = (r / n) % n, c = r / (n * n);
        const int co[3] = {a, b, c};
        for (int d = 0; d < 3; ++d) {
            const double gd = 2.0 / hh[d];
            double g = 0.0;
            if (d == 0) {
#pragma unroll
                for (int k = 0; k < n; ++k) g += gd * tdVt[(k) * n + (a)] * q[(c * n + b) * n + k];
            } else if (d == 1) {
#pragma unroll
                for (int k = 0; k < n; ++k) g += gd * tdV[(b) * n + (k)] * q[(c * n + k) * n + a];
            } else {
#pragma unroll
                for (int k = 0; k < n; ++k) g += gd * tdV[(c) * n + (k)] * q[(k * n + b) * n + a];
            }
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            for (int hi = 0; hi < 2; ++hi) {
                const bool high = hi == 1;
                const int layer = high ? n - 1 : 0;
                if (co[d] != layer) continue;
                if (neighbour(e3[d], A.n[d], A.bc[d], high) < 0) continue;
                const double oth = qn[2 * d + hi][co[t2] * n + co[t1]];
                const double own = q[r];
                const double jump = high ? own - oth : oth - own;
                const double f = 1.0 / (tw[layer] * hh[d]);
                g -= f * jump;
            }
            const double gv = A.fac ? A.scale * g * fq[r] : A.scale * g;
            A.g[d][base + r] = A.update ? A.v[d][base + r] + gv : gv;
        }
    }
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
            hipLaunchKernelGGL((k_divergence_eq<Pv>), dim3((unsigned)mv.nel), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_divergence<Pv, Qv>), dim3((unsigned)mv.nel), dim3(256), 0, s, a);
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
            hipLaunchKernelGGL((k_gradient_eq<Pv>), dim3((unsigned)mv.nel), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_gradient<Pv, Qv>), dim3((unsigned)mv.nel), dim3(256), 0, s, a);
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
