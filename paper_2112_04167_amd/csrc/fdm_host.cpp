// Host side of the fast-diagonalisation preconditioner: the 1D SIP-DG
// operator of one mesh axis and its generalised eigendecomposition.
//
// On a Cartesian product mesh with a constant nu, every volume and face term
// of the SIP form (Sec. 3.3 of arXiv 2112.04167: DG-SEM on tensor-product
// GLL hexahedra with interior penalty, all integrals by GLL quadrature)
// factorises into a 1D term along one axis times the GLL masses of the other
// two, so in global tensor ordering
//
//     A = lambda Mz (x) My (x) Mx + nu (Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx),
//
// K_d being the 1D SIP matrix of axis d for nu = 1 (the penalty is linear in
// nu).  With K_d S_d = M_d S_d Lam_d and S_d^T M_d S_d = I (Lynch, Rice &
// Thomas 1964),
//
//     A^-1 = (Sz (x) Sy (x) Sx) (lambda + nu (Lam_x (+) Lam_y (+) Lam_z))^-1 (Sz (x) Sy (x) Sx)^T.
//
// The symmetric eigenproblem of C = M^-1/2 K M^-1/2 is solved by Householder
// reduction to tridiagonal form followed by implicit symmetric QR steps with
// Wilkinson shifts (Golub & Van Loan, Matrix Computations, Sec. 8.3).
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>

#include "dg_internal.h"
#include "fdm.h"

namespace dg {

namespace {

// Dense 1D SIP matrix (nu = 1) and the diagonal GLL mass of one axis.
// Global 1D index g = e (P+1) + a.  Interior (and periodic) faces:
//   jump [u] = u_L(P) - u_R(0), average {du/dn} = (g_L D_P. u_L + g_R D_0. u_R)/2,
//   sigma = (P+1)^2 / min(h_L, h_R), contribution -[u]{dv/dn} - {du/dn}[v] + sigma [u][v];
// Dirichlet faces use the interior trace, the outward normal and
// sigma = (P+1)^2 / h; Neumann faces add nothing.
void sip_1d(const std::vector<double> &v, int P, int bc, const GllTables &t, std::vector<double> &K,
            std::vector<double> &M)
{
    const int ne = (int)v.size() - 1, n = P + 1, L = ne * n;
    K.assign((size_t)L * L, 0.0);
    M.assign(L, 0.0);
    const double pen = (double)n * n;
    auto h = [&](int e) { return v[e + 1] - v[e]; };
    for (int e = 0; e < ne; ++e) {
        const double he = h(e), g2h = 2.0 / he;  // (h/2) (2/h)^2
        for (int a = 0; a < n; ++a) {
            M[e * n + a] = 0.5 * he * t.w[a];
            for (int b = 0; b < n; ++b) K[(size_t)(e * n + a) * L + e * n + b] += g2h * t.K1[a * n + b];
        }
    }
    // rank-2 face term on the index list idx (duplicates accumulate)
    std::vector<int> idx;
    std::vector<double> jmp, avg;
    auto add_face = [&](double sigma) {
        const size_t m = idx.size();
        for (size_t i = 0; i < m; ++i)
            for (size_t j = 0; j < m; ++j)
                K[(size_t)idx[i] * L + idx[j]] +=
                    -jmp[i] * avg[j] - avg[i] * jmp[j] + sigma * jmp[i] * jmp[j];
    };
    for (int e = 0; e < ne; ++e) {
        const bool last = (e + 1 == ne);
        if (!last || bc == DG_BC_PERIODIC) {
            const int r = last ? 0 : e + 1;
            idx.clear();
            jmp.clear();
            avg.clear();
            for (int a = 0; a < n; ++a) {
                idx.push_back(e * n + a);
                jmp.push_back(a == P ? 1.0 : 0.0);
                avg.push_back(0.5 * (2.0 / h(e)) * t.D[P * n + a]);
            }
            for (int a = 0; a < n; ++a) {
                idx.push_back(r * n + a);
                jmp.push_back(a == 0 ? -1.0 : 0.0);
                avg.push_back(0.5 * (2.0 / h(r)) * t.D[0 * n + a]);
            }
            add_face(pen / std::min(h(e), h(r)));
        } else if (bc == DG_BC_DIRICHLET) {
            idx.clear();
            jmp.clear();
            avg.clear();
            for (int a = 0; a < n; ++a) {
                idx.push_back(e * n + a);
                jmp.push_back(a == P ? 1.0 : 0.0);
                avg.push_back((2.0 / h(e)) * t.D[P * n + a]);
            }
            add_face(pen / h(e));
        }
    }
    if (bc == DG_BC_DIRICHLET) {  // low end of the first element, outward normal -1
        idx.clear();
        jmp.clear();
        avg.clear();
        for (int a = 0; a < n; ++a) {
            idx.push_back(a);
            jmp.push_back(a == 0 ? 1.0 : 0.0);
            avg.push_back(-(2.0 / h(0)) * t.D[0 * n + a]);
        }
        add_face(pen / h(0));
    }
}

// Householder reduction of the symmetric n x n matrix A (row-major) to
// tridiagonal form: A = Q T Q^T.  On return d, e hold the diagonal and the
// sub-diagonal of T and Q (row-major) the accumulated reflections.
void householder_tridiag(int n, std::vector<double> &A, std::vector<double> &d, std::vector<double> &e,
                         std::vector<double> &Q)
{
    std::vector<std::vector<double>> vs(n);
    std::vector<double> betas(n, 0.0), p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of x = A[k+1.., k]
        double sig = 0.0;
        for (int i = 1; i < m; ++i) sig += A[(size_t)(k + 1 + i) * n + k] * A[(size_t)(k + 1 + i) * n + k];
        const double x0 = A[(size_t)(k + 1) * n + k];
        std::vector<double> v(m);
        v[0] = 1.0;
        for (int i = 1; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
        double beta = 0.0, alpha = x0;
        if (sig != 0.0) {
            const double mu = std::sqrt(x0 * x0 + sig);
            // v0 = x0 - mu, computed without cancellation
            const double v0 = x0 <= 0.0 ? x0 - mu : -sig / (x0 + mu);
            beta = 2.0 * v0 * v0 / (sig + v0 * v0);
            for (int i = 1; i < m; ++i) v[i] /= v0;
            alpha = mu;
        }
        // A[k+1.., k+1..] <- H A H,  H = I - beta v v^T
        if (beta != 0.0) {
            const size_t o = (size_t)(k + 1);
            for (int i = 0; i < m; ++i) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += A[(o + i) * n + o + j] * v[j];
                p[i] = beta * s;
            }
            double pv = 0.0;
            for (int i = 0; i < m; ++i) pv += p[i] * v[i];
            const double c = 0.5 * beta * pv;
            for (int i = 0; i < m; ++i) w[i] = p[i] - c * v[i];
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) A[(o + i) * n + o + j] -= v[i] * w[j] + w[i] * v[j];
        }
        A[(size_t)(k + 1) * n + k] = A[(size_t)k * n + k + 1] = alpha;
        for (int i = 1; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = A[(size_t)k * n + k + 1 + i] = 0.0;
        vs[k] = std::move(v);
        betas[k] = beta;
    }
    d.assign(n, 0.0);
    e.assign(n > 1 ? n - 1 : 0, 0.0);
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
    // Q = H_0 H_1 ... H_{n-3}, accumulated from the last reflection
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (betas[k] == 0.0) continue;
        const int m = n - k - 1;
        const size_t o = (size_t)(k + 1);
        const std::vector<double> &v = vs[k];
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += v[i] * Q[(o + i) * n + o + j];
            s *= betas[k];
            for (int i = 0; i < m; ++i) Q[(o + i) * n + o + j] -= s * v[i];
        }
    }
}

// Implicit symmetric QR steps with Wilkinson shifts on the tridiagonal
// (d, e); the rotations are applied to the columns of Z (row-major n x n).
bool tridiag_qr(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Z)
{
    const double eps = 2.220446049250313e-16;
    int m = n - 1;
    long long guard = 0;
    while (m > 0) {
        if (std::fabs(e[m - 1]) <= eps * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
            e[m - 1] = 0.0;
            --m;
            continue;
        }
        int p = m - 1;
        while (p > 0 && std::fabs(e[p - 1]) > eps * (std::fabs(d[p - 1]) + std::fabs(d[p]))) --p;
        if (++guard > 60LL * n) return false;
        // Wilkinson shift from the trailing 2x2 block
        const double del = 0.5 * (d[m - 1] - d[m]);
        const double em = e[m - 1];
        const double den = del + (del >= 0.0 ? 1.0 : -1.0) * std::hypot(del, em);
        const double mu = d[m] - em * em / den;
        double x = d[p] - mu, z = e[p];
        for (int k = p; k < m; ++k) {
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, s = r > 0.0 ? -z / r : 0.0;
            if (k > p) e[k - 1] = c * x - s * z;  // the bulge below e[k-1] is removed
            const double a = d[k], b = e[k], g = d[k + 1];
            d[k] = a * c * c - 2.0 * b * c * s + g * s * s;
            d[k + 1] = a * s * s + 2.0 * b * c * s + g * c * c;
            e[k] = (a - g) * c * s + b * (c * c - s * s);
            double bulge = 0.0;
            if (k + 1 < m) {
                bulge = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
            }
            for (int i = 0; i < n; ++i) {
                double *zr = &Z[(size_t)i * n];
                const double zk = zr[k], zk1 = zr[k + 1];
                zr[k] = c * zk - s * zk1;
                zr[k + 1] = s * zk + c * zk1;
            }
            x = e[k];
            z = bulge;
        }
    }
    return true;
}

}  // namespace

bool sym_eig(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &V)
{
    std::vector<double> d, e, Q;
    householder_tridiag(n, A, d, e, Q);
    if (!tridiag_qr(n, d, e, Q)) return false;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
    lam.assign(n, 0.0);
    V.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        lam[j] = d[ord[j]];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Q[(size_t)i * n + ord[j]];
    }
    return true;
}

int fdm_axis_compute(const std::vector<double> &v, int P, int bc, FdmAxis &out)
{
    const GllTables &t = gll_cached(P);
    std::vector<double> K, M;
    sip_1d(v, P, bc, t, K, M);
    const int L = (int)M.size();
    std::vector<double> is(L);
    for (int i = 0; i < L; ++i) is[i] = 1.0 / std::sqrt(M[i]);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) K[(size_t)i * L + j] *= is[i] * is[j];
    // symmetrise the rounding of the scaling
    for (int i = 0; i < L; ++i)
        for (int j = i + 1; j < L; ++j) {
            const double s = 0.5 * (K[(size_t)i * L + j] + K[(size_t)j * L + i]);
            K[(size_t)i * L + j] = K[(size_t)j * L + i] = s;
        }
    std::vector<double> lam, Q;
    if (!sym_eig(L, K, lam, Q)) {
        set_error("fast diagonalisation: the 1D eigenproblem did not converge");
        return DG_ERR_DEVICE;
    }
    out.L = L;
    out.lam = lam;
    out.S.assign((size_t)L * L, 0.0);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) out.S[(size_t)i * L + j] = Q[(size_t)i * L + j] * is[i];
    return DG_OK;
}

std::shared_ptr<const FdmAxis> fdm_axis_cached(const std::vector<double> &v, int P, int bc, int *rc)
{
    // the eigendecompositions depend only on the vertices, the degree and
    // the BC of the axis; a bounded cache keeps them for repeated meshes
    static std::mutex mu;
    static std::map<std::tuple<std::vector<double>, int, int>, std::shared_ptr<FdmAxis>> cache;
    const auto key = std::make_tuple(v, P, bc);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *rc = DG_OK;
            return it->second;
        }
    }
    auto ax = std::make_shared<FdmAxis>();
    *rc = fdm_axis_compute(v, P, bc, *ax);
    if (*rc) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() >= 512) cache.clear();  // holders keep their shared_ptr
    cache.emplace(key, ax);
    return ax;
}

}  // namespace dg
