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
// interpolated to the Q^3 Gauss points (three 1D passes per component, in
// LDS).  Per output component i the nine (i, k) flux passes back to the
// nodes are factored into three: the z pass forms the three products
// v_i v_k on the fly, the y pass combines the k = 1, 2 branches that share
// B_x, the x pass the remaining two.  Then both faces of each axis at once,
// each element computing the fluxes of its own faces (no atomics: the
// neighbour computes the same flux with the opposite sign).  LDS at P = 7:
// 79 KB (two work-groups per CU); at P = 8: 124 KB.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "convection.h"
#include "device_common.h"
#include "dg_internal.h"

namespace dg {

namespace {

constexpr int kN = kMaxN;         // velocity nodes per direction, at most 9
constexpr int kMaxQ = 3 * 8 / 2 + 1;  // Gauss points per direction, at most 13

struct ConvTables {
    double B[kMaxQ][kN];   // B[q][a] = l_a(x_q): GLL basis at the Gauss points
    double dB[kMaxQ][kN];  // its derivative on [-1, 1]
    double wg[kMaxQ];      // Gauss weights
    double w[kN];          // GLL weights (the mass)
};

struct ConvArgs {
    ConvTables t;
    const double *v[3];
    const double *vb[3];   // wall state (null: zero)
    double *out[3];
    const double *h[3];
    int n[3], bc[3];
    double scale;
    int accumulate;        // out += scale F_c instead of out = scale F_c
};

__host__ __device__ constexpr int conv_q(int P) { return 3 * P / 2 + 1; }

template <int P>
struct ConvLds {
    static constexpr int n = P + 1, Q = conv_q(P);
    // region A: the velocity at the Gauss points U[3][Q^3], later the face
    // points' traces tg[12][Q^2] and weighted fluxes hw[6][Q^2]
    static constexpr int vol = 3 * Q * Q * Q, fa = 18 * Q * Q;
    static constexpr int A = vol > fa ? vol : fa;
    // region S: interpolation scratch (n^3 + n^2 Q + n Q^2), then the
    // transposed passes Z[3][n Q^2], Yb[2][n^2 Q], then the face-node
    // buffers tr[12][n^2], tq[12][n Q], hq[6][Q n]
    static constexpr int s_in = n * n * n + n * n * Q + n * Q * Q;
    static constexpr int s_bk = 3 * n * Q * Q + 2 * n * n * Q;
    static constexpr int s_fc = 12 * n * n + 12 * n * Q + 6 * Q * n;
    static constexpr int S = s_in > s_bk ? (s_in > s_fc ? s_in : s_fc) : (s_bk > s_fc ? s_bk : s_fc);
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

template <int P>
__global__ void __launch_bounds__(256) k_convection(ConvArgs A)
{
    using L = ConvLds<P>;
    constexpr int n = L::n, Q = L::Q, n3 = n * n * n, Q2 = Q * Q, Q3 = Q * Q * Q;
    constexpr int nQ2 = n * Q2, n2Q = n * n * Q;
    __shared__ double bufA[L::A];
    __shared__ double bufS[L::S];
    __shared__ double acc[3][n3];
    // the 1D tables in LDS, compacted to Q x n: their lane-dependent rows
    // would otherwise be vector loads from the kernel arguments
    __shared__ double tB[Q * n], tdB[Q * n], twg[Q], tw[n];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int el = blockIdx.x;
    const int ex = el % A.n[0], ey = (el / A.n[0]) % A.n[1], ez = el / (A.n[0] * A.n[1]);
    const int e3[3] = {ex, ey, ez};
    const double hh[3] = {A.h[0][ex], A.h[1][ey], A.h[2][ez]};
    const double J = hh[0] * hh[1] * hh[2] * 0.125;
    const size_t base = (size_t)el * n3;
    double *U = bufA;
    for (int i = threadIdx.x; i < Q * n; i += blockDim.x) {
        tB[i] = A.t.B[i / n][i % n];
        tdB[i] = A.t.dB[i / n][i % n];
    }
    for (int i = threadIdx.x; i < Q; i += blockDim.x) twg[i] = A.t.wg[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = A.t.w[i];
    __syncthreads();

    // ---- velocity at the Gauss points: U_k = (B (x) B (x) B) v_k
    {
        double *X = bufS, *Y1 = bufS + n3, *Y2 = bufS + n3 + n2Q;
        for (int k = 0; k < 3; ++k) {
            for (int i = tid; i < n3; i += nth) X[i] = A.v[k][base + i];
            __syncthreads();
            for (int i = tid; i < n2Q; i += nth) {  // x: Y1[c][b][qx]
                const int qx = i % Q, cb = i / Q;
                double sum = 0.0;
#pragma unroll
                for (int a = 0; a < n; ++a) sum = fma(tB[(qx) * n + (a)], X[cb * n + a], sum);
                Y1[i] = sum;
            }
            __syncthreads();
            for (int i = tid; i < nQ2; i += nth) {  // y: Y2[c][qy][qx]
                const int qx = i % Q, qy = (i / Q) % Q, c = i / Q2;
                double sum = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) sum = fma(tB[(qy) * n + (b)], Y1[(c * n + b) * Q + qx], sum);
                Y2[i] = sum;
            }
            __syncthreads();
            for (int i = tid; i < Q3; i += nth) {  // z: U_k[qz][qy][qx]
                const int qxy = i % Q2, qz = i / Q2;
                double sum = 0.0;
#pragma unroll
                for (int c = 0; c < n; ++c) sum = fma(tB[(qz) * n + (c)], Y2[c * Q2 + qxy], sum);
                U[k * Q3 + i] = sum;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < 3 * n3; i += nth) (&acc[0][0])[i] = 0.0;

    // ---- volume: acc_i = sum_k T_k^T (W J v_i v_k) with T_k = (2/h_k) dB along
    //      k and B along the others, factored as
    //      B_x^T [B_y^T dB_z^T F_i2 + dB_y^T B_z^T F_i1] + dB_x^T B_y^T B_z^T F_i0
    double *Z = bufS, *Yb = bufS + 3 * nQ2;
    const double g0 = 2.0 / hh[0], g1 = 2.0 / hh[1], g2 = 2.0 / hh[2];
    for (int i = 0; i < 3; ++i) {
        __syncthreads();
        for (int r = tid; r < nQ2; r += nth) {  // z: Z_k[c][qy][qx]
            const int qx = r % Q, qy = (r / Q) % Q, c = r / Q2;
            const int qxy = qy * Q + qx;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                const int q = qz * Q2 + qxy;
                const double ui = U[i * Q3 + q] * twg[qz];
                s0 = fma(tB[(qz) * n + (c)], ui * U[q], s0);
                s1 = fma(tB[(qz) * n + (c)], ui * U[Q3 + q], s1);
                s2 = fma(tdB[(qz) * n + (c)], ui * U[2 * Q3 + q], s2);
            }
            const double f = twg[qx] * twg[qy] * J;
            Z[r] = s0 * f * g0;
            Z[nQ2 + r] = s1 * f * g1;
            Z[2 * nQ2 + r] = s2 * f * g2;
        }
        __syncthreads();
        for (int r = tid; r < n2Q; r += nth) {  // y: Yb_x = B_y^T Z_0, Yb_s = dB_y^T Z_1 + B_y^T Z_2
            const int qx = r % Q, b = (r / Q) % n, c = r / (n * Q);
            double sx = 0.0, ss = 0.0;
#pragma unroll
            for (int qy = 0; qy < Q; ++qy) {
                const int zi = (c * Q + qy) * Q + qx;
                sx = fma(tB[(qy) * n + (b)], Z[zi], sx);
                ss = fma(tdB[(qy) * n + (b)], Z[nQ2 + zi], ss);
                ss = fma(tB[(qy) * n + (b)], Z[2 * nQ2 + zi], ss);
            }
            Yb[r] = sx;
            Yb[n2Q + r] = ss;
        }
        __syncthreads();
        for (int r = tid; r < n3; r += nth) {  // x: acc_i[c][b][a]
            const int a = r % n, cb = r / n;
            double sum = 0.0;
#pragma unroll
            for (int qx = 0; qx < Q; ++qx) {
                sum = fma(tdB[(qx) * n + (a)], Yb[cb * Q + qx], sum);
                sum = fma(tB[(qx) * n + (a)], Yb[n2Q + cb * Q + qx], sum);
            }
            acc[i][r] += sum;
        }
    }

    // ---- faces: acc_i -= int_F H_i phi, both faces of an axis at once
    double *tr = bufS;                 // [12][n*n]: side*6 + (own v_0..2, exterior v_0..2), [t][s]
    double *tq = tr + 12 * n * n;      // [12][n*Q]: [t][qs]
    double *hq = tq + 12 * n * Q;      // [6][Q*n]: side*3 + i, [qt][s]
    double *tg = bufA;                 // [12][Q*Q]: [qt][qs]
    double *hw = bufA + 12 * Q2;       // [6][Q*Q]
    for (int d = 0; d < 3; ++d) {
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const double om0 = hh[t1] * hh[t2] * 0.25;
        __syncthreads();  // the previous phase's readers of these buffers are done
        for (int r = tid; r < 12 * n * n; r += nth) {
            const int slot = r / (n * n), st = r % (n * n), s = st % n, t = st / n;
            const bool high = slot >= 6;
            const int comp = slot % 6;
            const int layer = high ? n - 1 : 0;
            double val;
            if (comp < 3) {
                val = A.v[comp][base + layer_node<n>(d, layer, s, t)];
            } else {
                const int kn = nb_index(e3[d], A.n[d], A.bc[d], high);
                if (kn >= 0) {
                    int en[3] = {ex, ey, ez};
                    en[d] = kn;
                    const size_t nbase = ((size_t)(en[2] * A.n[1] + en[1]) * A.n[0] + en[0]) * n3;
                    val = A.v[comp - 3][nbase + layer_node<n>(d, high ? 0 : n - 1, s, t)];
                } else {
                    const double *wb = A.vb[comp - 3];
                    val = wb ? wb[base + layer_node<n>(d, layer, s, t)] : 0.0;
                }
            }
            tr[r] = val;
        }
        __syncthreads();
        for (int r = tid; r < 12 * n * Q; r += nth) {  // along s
            const int slot = r / (n * Q), q = r % Q, t = (r / Q) % n;
            double sum = 0.0;
#pragma unroll
            for (int s = 0; s < n; ++s) sum = fma(tB[(q) * n + (s)], tr[slot * n * n + t * n + s], sum);
            tq[r] = sum;
        }
        __syncthreads();
        for (int r = tid; r < 12 * Q2; r += nth) {  // along t
            const int slot = r / Q2, qs = r % Q, qt = (r / Q) % Q;
            double sum = 0.0;
#pragma unroll
            for (int t = 0; t < n; ++t) sum = fma(tB[(qt) * n + (t)], tq[slot * n * Q + t * Q + qs], sum);
            tg[r] = sum;
        }
        __syncthreads();
        for (int r = tid; r < 2 * Q2; r += nth) {
            const int side = r / Q2, q = r % Q2, qs = q % Q, qt = q / Q;
            const double sgn = side ? 1.0 : -1.0;
            const double *own = tg + side * 6 * Q2, *ext = own + 3 * Q2;
            const double vm = sgn * own[d * Q2 + q], vp = sgn * ext[d * Q2 + q];
            const double alpha = 2.0 * fmax(fabs(vm), fabs(vp));
            const double om = om0 * twg[qs] * twg[qt];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double um = own[i * Q2 + q], up = ext[i * Q2 + q];
                hw[(side * 3 + i) * Q2 + q] = -om * (0.5 * (vm * um + vp * up) + 0.5 * alpha * (um - up));
            }
        }
        __syncthreads();
        for (int r = tid; r < 6 * Q * n; r += nth) {  // back along s: hq[side*3+i][qt][s]
            const int slot = r / (Q * n), s = r % n, qt = (r / n) % Q;
            double sum = 0.0;
#pragma unroll
            for (int qs = 0; qs < Q; ++qs) sum = fma(tB[(qs) * n + (s)], hw[slot * Q2 + qt * Q + qs], sum);
            hq[r] = sum;
        }
        __syncthreads();
        for (int r = tid; r < 6 * n * n; r += nth) {  // back along t onto the two face layers
            const int slot = r / (n * n), s = r % n, t = (r / n) % n;
            const int side = slot / 3, i = slot % 3;
            double sum = 0.0;
#pragma unroll
            for (int qt = 0; qt < Q; ++qt) sum = fma(tB[(qt) * n + (t)], hq[slot * Q * n + qt * n + s], sum);
            acc[i][layer_node<n>(d, side ? n - 1 : 0, s, t)] += sum;
        }
    }
    __syncthreads();
    for (int r = tid; r < n3; r += nth) {
        const int a = r % n, b = (r / n) % n, c = r / (n * n);
        const double f = A.scale / (J * tw[a] * tw[b] * tw[c]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double val = f * acc[i][r];
            A.out[i][base + r] = A.accumulate ? A.out[i][base + r] + val : val;
        }
    }
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_Q
// (three-term recurrence for P_Q and its derivative), started from the
// Chebyshev-like guesses cos(pi (j + 3/4) / (Q + 1/2)).
void gauss_legendre(int Q, double *x, double *w)
{
    for (int j = 0; j < Q; ++j) {
        double z = std::cos(M_PI * (j + 0.75) / (Q + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= Q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (Q == 1) p0 = 1.0;
            dp = Q * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= Q; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = Q * (z * p1 - p0) / (z * z - 1.0);
        x[Q - 1 - j] = z;
        w[Q - 1 - j] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

ConvTables make_conv_tables(int P)
{
    ConvTables t{};
    const GllTables &g = gll_cached(P);
    const int n = P + 1, Q = conv_q(P);
    double xg[kMaxQ];
    gauss_legendre(Q, xg, t.wg);
    for (int a = 0; a < n; ++a) t.w[a] = g.w[a];
    for (int q = 0; q < Q; ++q) {
        const double x = xg[q];
        for (int a = 0; a < n; ++a) {
            double l = 1.0, dl = 0.0;
            for (int k = 0; k < n; ++k) {
                if (k == a) continue;
                const double r = 1.0 / (g.xi[a] - g.xi[k]);
                dl = dl * (x - g.xi[k]) * r + l * r;
                l *= (x - g.xi[k]) * r;
            }
            t.B[q][a] = l;
            t.dB[q][a] = dl;
        }
    }
    return t;
}

}  // namespace

int launch_convection(const MeshDev &m, const double *const v[3], const double *const vb[3], double scale,
                      bool accumulate, double *const out[3], hipStream_t s)
{
    ConvArgs a{};
    a.t = make_conv_tables(m.P);
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
