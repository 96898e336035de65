// C-ABI entry points: meshes, the matrix-free apply, and the Jacobi-PCG /
// mixed-precision refinement drivers (host side).
//
// The drivers enqueue whole CG iterations (apply, update, p-update) in
// chunks; the device keeps every scalar and flags completion itself, so the
// host reads the solver state back once per chunk only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "batched.h"
#include "dg_internal.h"
#include "fdm.h"
#include "kernels.h"
#include "projection.h"
#include "trace.h"

namespace dg {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

const GllTables &gll_cached(int P)
{
    static std::mutex mu;
    static std::map<int, std::unique_ptr<GllTables>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(P);
    if (it == cache.end()) it = cache.emplace(P, std::make_unique<GllTables>(make_gll(P))).first;
    return *it->second;
}

}  // namespace dg

using namespace dg;

// Workspace of one mesh: FP64 CG vectors, FP32 inner vectors, reduction
// scratch and the device scalar blocks.
struct Workspace {
    size_t bytes = 0;
    void *base = nullptr;
    int64_t ndof = 0;
    int precision = -1;
    double *r64 = nullptr, *p64 = nullptr, *q64 = nullptr, *d64 = nullptr, *b64 = nullptr;
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr,
          *b32 = nullptr, *nu32 = nullptr;
    double *partial = nullptr;
    double *dtab64 = nullptr;     // per-axis 1D diagonal terms (constant nu)
    std::vector<double> htab64;   // host copy (alive until the next solve's upload)
    int tab_bc[3] = {-1, -1, -1}; // boundary conditions and nu the device tables hold
    double tab_nu = 0.0;
    double *fdm = nullptr;        // fast-diagonalisation tables (fdm_table_bytes)
    std::vector<double> fdm_img;  // host image (alive until the next upload)
    int fdm_bc[3] = {-1, -1, -1}; // boundary conditions the device tables hold
    CgScalars *sc = nullptr;      // [0] outer / FP64, [1] inner FP32
    CgScalars *host_sc = nullptr; // pinned
    bool external = false;        // memory lent by the caller (never freed here)
    bool host_external = false;
};

// Workspace of the batched solver: per system two FP64 and seven
// inner-precision vectors, plus reduction slots and the device state.
struct BatchWorkspace {
    size_t bytes = 0;
    void *base = nullptr;
    void *host_state = nullptr;  // pinned copy of the device state
};

struct dg_mesh {
    MeshDev dev;
    hipStream_t stream = nullptr;
    Workspace ws;
    BatchWorkspace bws;
    void *geo_block = nullptr;  // device: extents, reciprocals, visiting order
    bool geo_external = false;
    double *aux = nullptr;      // device: the projection's pressure load (ndof doubles)
    double *step_buf = nullptr; // device: the IMEX step's stage fields (grow-only)
    size_t step_doubles = 0;
    // concurrent solves: the workspaces of the second and third solve
    // (created on first use; their streams are shared by all meshes, see
    // concurrent_streams), and the event those streams start from
    Workspace alt_ws[kMaxConcurrent - 1];
    hipEvent_t alt_event = nullptr;
};

namespace {

size_t partial_doubles(const MeshDev &m) { return (size_t)apply_groups(m.P, m.nel) * 6 + 64; }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t diag_table_len(const MeshDev &m) { return (size_t)(m.n[0] + m.n[1] + m.n[2]) * (m.P + 1); }

size_t footprint(const MeshDev &m, int precision)
{
    const size_t N = (size_t)m.ndof;
    size_t b = 0;
    b += 5 * align256(N * sizeof(double));  // r, p, q, d, b (FP64)
    if (precision == DG_MIXED) b += 7 * align256(N * sizeof(float));
    b += align256(partial_doubles(m) * sizeof(double));
    b += align256(diag_table_len(m) * sizeof(double));
    b += align256(fdm_table_bytes(m.n, m.P));
    b += align256(2 * sizeof(CgScalars));
    return b;
}

int ensure_workspace(dg_mesh *m, Workspace &w, int precision)
{
    const size_t need = footprint(m->dev, precision);
    if (w.base && w.bytes >= need && w.ndof == m->dev.ndof &&
        (precision != DG_MIXED || w.precision == DG_MIXED))
        return DG_OK;
    if (w.external) {
        if (w.bytes < need) {
            set_error("lent workspace too small for this solve");
            return DG_ERR_ARG;
        }
    } else {
        if (w.base) {
            DG_HIP_CHECK(hipStreamSynchronize(m->stream));
            DG_HIP_CHECK(hipFree(w.base));
            w.base = nullptr;
        }
        hipError_t e = hipMalloc(&w.base, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("workspace allocation of " + std::to_string(need) + " bytes failed");
            w.base = nullptr;
            return DG_ERR_OOM;
        }
    }
    if (!w.host_sc) DG_HIP_CHECK(hipHostMalloc((void **)&w.host_sc, 2 * sizeof(CgScalars), 0));
    if (!w.external) w.bytes = need;
    w.ndof = m->dev.ndof;
    w.precision = precision;
    char *p = (char *)w.base;
    const size_t N = (size_t)m->dev.ndof;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return (void *)r;
    };
    w.r64 = (double *)take(N * 8);
    w.p64 = (double *)take(N * 8);
    w.q64 = (double *)take(N * 8);
    w.d64 = (double *)take(N * 8);
    w.b64 = (double *)take(N * 8);
    if (precision == DG_MIXED) {
        w.x32 = (float *)take(N * 4);
        w.r32 = (float *)take(N * 4);
        w.p32 = (float *)take(N * 4);
        w.q32 = (float *)take(N * 4);
        w.d32 = (float *)take(N * 4);
        w.b32 = (float *)take(N * 4);
        w.nu32 = (float *)take(N * 4);
    } else {
        w.x32 = w.r32 = w.p32 = w.q32 = w.d32 = w.b32 = w.nu32 = nullptr;
    }
    w.partial = (double *)take(partial_doubles(m->dev) * 8);
    w.dtab64 = (double *)take(diag_table_len(m->dev) * sizeof(double));
    w.tab_bc[0] = w.tab_bc[1] = w.tab_bc[2] = -1;
    w.fdm = (double *)take(fdm_table_bytes(m->dev.n, m->dev.P));
    w.fdm_bc[0] = w.fdm_bc[1] = w.fdm_bc[2] = -1;

    w.sc = (CgScalars *)take(2 * sizeof(CgScalars));
    return DG_OK;
}

CgScalars init_scalars(const MeshDev &m, double tol, int maxit, int fixed_iters, bool singular)
{
    CgScalars s;
    std::memset(&s, 0, sizeof(s));
    s.tol2 = tol * tol;
    s.maxit = maxit;
    s.fixed_iters = fixed_iters;
    s.singular = singular ? 1 : 0;
    s.ndof = m.ndof;
    s.status = DG_OK;
    return s;
}

bool has_dirichlet(const int bc[3])
{
    return bc[0] == DG_BC_DIRICHLET || bc[1] == DG_BC_DIRICHLET || bc[2] == DG_BC_DIRICHLET;
}

template <typename T>
CgVecArgs<T> vec_args(const Workspace &w, bool singular, CgScalars *sc)
{
    CgVecArgs<T> a{};
    a.partial = w.partial;
    a.sc = sc;
    a.singular = singular;
    return a;
}

double now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Iterations to enqueue before the next look at the device state.  The
// chunks double (from `first`, up to `cap`) while no convergence rate is
// known; once two residual norms are known, the reduction per iteration
// between them predicts the iterations still needed to reach tol2, and the
// next chunk is 1.25 times that plus one (never more than the doubling
// schedule would give).  Iterations enqueued past convergence return at once
// but still cost a launch each; too short a chunk costs a host round trip, so
// the prediction errs long.  The iteration-0 norm is the device's last true
// residual when `from_true` (the solve started with r = b - A x).
struct ChunkPlan {
    int chunk, cap;
    bool from_true;
    double res2 = -1.0;
    int iter = 0;
    ChunkPlan(int first, int cap_, bool from_true_) : chunk(first), cap(cap_), from_true(from_true_) {}
    void next(const CgScalars &h)
    {
        const int doubled = std::min(chunk * 2, cap);
        int pred = doubled;
        double r0 = res2;
        int i0 = iter;
        if (r0 < 0.0 && from_true) {
            r0 = h.true_res2;
            i0 = 0;
        }
        if (h.fixed_iters > 0) {
            pred = std::max(1, h.fixed_iters - h.iter);
        } else if (r0 > 0.0 && h.res2 > 0.0 && h.res2 < r0 && h.iter > i0 && h.tol2 > 0.0 && h.tol2 < h.res2) {
            const double per = std::log(h.res2 / r0) / (h.iter - i0);  // < 0
            const double need = std::log(h.tol2 / h.res2) / per;      // > 0
            if (std::isfinite(need) && need < 1e6) pred = (int)std::ceil(1.25 * need) + 1;
        }
        res2 = h.res2;
        iter = h.iter;
        chunk = std::max(1, std::min(pred, doubled));
    }
};

// Run CG iterations until the device flags completion.  T: vector type.
// from_true: the device's true residual holds the starting residual norm.
template <typename T>
int cg_iterate(dg_mesh *m, const int bc[3], double lambda, const T *nu, double nu_c,
               CgVecArgs<T> a, CgScalars *dev_sc, CgScalars *host_sc, int cap_hint, bool from_true = false)
{
    const MeshDev &md = m->dev;
    hipStream_t s = m->stream;
    ChunkPlan plan(4, 64, from_true);
    int launched = 0;
    for (;;) {
        const int chunk = plan.chunk;
        for (int k = 0; k < chunk; ++k) {
            int rc = launch_apply_cg<T>(md, bc, lambda, nu, nu_c, a.p, const_cast<T *>(a.q),
                                        a.partial, dev_sc, s);
            if (rc) return rc;
            if ((rc = cg_update<T>(md, a, s))) return rc;
            if ((rc = cg_pupdate<T>(md, a, s))) return rc;
        }
        launched += chunk;
        DG_HIP_CHECK(hipMemcpyAsync(host_sc, dev_sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        DG_HIP_CHECK(hipStreamSynchronize(s));
        if (host_sc->done) break;
        if (launched > cap_hint + 64) {
            set_error("CG did not flag completion");
            return DG_ERR_DEVICE;
        }
        plan.next(*host_sc);
    }
    return DG_OK;
}

int check_mesh(dg_mesh *m)
{
    if (!m) {
        set_error("null mesh");
        return DG_ERR_ARG;
    }
    return DG_OK;
}

// The 1D diagonal terms of the constant-nu operator (arXiv 2112.04167,
// Sec. 3.3: SIP on a Cartesian product grid, GLL quadrature).  The operator
// is lambda M plus, per axis d, the 1D SIP operator along d scaled by the
// tangential GLL mass, so its diagonal at node (a,b,c) of element
// (ex,ey,ez) is lambda J W + hy hz w_b w_c T_x[ex][a] + ... with
//   T_d[k][a] = nu K1_aa / (2 h_k) + (face terms at a = 0, P) / 4,
// the face terms being those of the interior-penalty form with
// sigma = nu (P+1)^2 / min(h_k, h_N) (interior, periodic) or nu (P+1)^2 / h_k
// (Dirichlet).  The same terms as the stored diagonal, in another order.
void diag_tables(const MeshDev &md, const int bc[3], double nu, std::vector<double> &t)
{
    const GllTables &g = gll_cached(md.P);
    const int P = md.P, n = P + 1;
    const double pen = (double)n * n;
    t.assign(diag_table_len(md), 0.0);
    size_t off = 0;
    for (int d = 0; d < 3; ++d) {
        const int nk = md.n[d];
        auto h = [&](int k) { return md.v[d][k + 1] - md.v[d][k]; };
        for (int k = 0; k < nk; ++k) {
            const double hk = h(k), gk = 2.0 / hk;
            for (int a = 0; a < n; ++a) {
                double T = nu * g.K1[a * n + a] / (2.0 * hk);
                if (a == 0 || a == P) {
                    const bool high = (a == P);
                    int kn = k, kind;
                    if (!high && k > 0) {
                        kn = k - 1;
                        kind = 1;
                    } else if (high && k < nk - 1) {
                        kn = k + 1;
                        kind = 1;
                    } else if (bc[d] == DG_BC_PERIODIC) {
                        kn = high ? 0 : nk - 1;
                        kind = 1;
                    } else {
                        kind = bc[d] == DG_BC_DIRICHLET ? 2 : 0;
                    }
                    const double Daa = g.D[a * n + a], sgn = high ? -1.0 : 1.0;
                    double f = 0.0;
                    if (kind == 1) {
                        f = nu * pen / std::min(hk, h(kn)) + sgn * nu * gk * Daa;
                        if (kn == k)  // a single periodic element is its own neighbour
                            f += high ? -nu * gk * g.D[0 * n + P] : nu * gk * g.D[P * n + 0];
                    } else if (kind == 2) {
                        f = nu * pen / hk + 2.0 * sgn * nu * gk * Daa;
                    }
                    T += 0.25 * f;
                }
                t[off + (size_t)k * n + a] = T;
            }
        }
        off += (size_t)nk * n;
    }
}

// upload the tables of this solve on the solve's stream (unless the device
// already holds those of the same boundary conditions and nu)
int upload_diag_tables(dg_mesh *m, Workspace &w, const int bc[3], double nu)
{
    if (w.tab_bc[0] == bc[0] && w.tab_bc[1] == bc[1] && w.tab_bc[2] == bc[2] && w.tab_nu == nu)
        return DG_OK;
    diag_tables(m->dev, bc, nu, w.htab64);
    DG_HIP_CHECK(hipMemcpyAsync(w.dtab64, w.htab64.data(), w.htab64.size() * sizeof(double),
                                hipMemcpyHostToDevice, m->stream));
    for (int d = 0; d < 3; ++d) w.tab_bc[d] = bc[d];
    w.tab_nu = nu;
    return DG_OK;
}

// FP64 Jacobi-PCG, on the workspace w (the mesh's own, or memory lent to it)
int solve_fp64(dg_mesh *m, Workspace &w, const int bc[3], double lambda, const double *nu,
               double nu_c, const double *rhs, double *x, const dg_solve_opts &o,
               dg_solve_info &info)
{
    int rc = ensure_workspace(m, w, DG_FP64);
    if (rc) return rc;
    const MeshDev &md = m->dev;
    hipStream_t s = m->stream;
    const bool singular = (lambda == 0.0) && !has_dirichlet(bc);
    CgScalars init = init_scalars(md, o.tol, o.maxit, o.fixed_iters, singular);
    *w.host_sc = init;
    DG_HIP_CHECK(hipMemcpyAsync(w.sc, w.host_sc, sizeof(CgScalars), hipMemcpyHostToDevice, s));
    CgVecArgs<double> a = vec_args<double>(w, singular, w.sc);
    if (nu) {
        if ((rc = launch_diag<double>(md, bc, lambda, nu, nu_c, w.d64, s, true))) return rc;
        a.d = w.d64;
    } else {  // constant nu: the diagonal is computed where it is used
        if ((rc = upload_diag_tables(m, w, bc, nu_c))) return rc;
        a.dtab = w.dtab64;
        a.lam = lambda;
    }
    a.x = x;
    a.r = w.r64;
    a.p = w.p64;
    a.q = w.q64;
    a.src = rhs;
    a.bvec = w.b64;
    a.weak = o.rhs_is_weak;
    a.keep_x = 1;
    if ((rc = cg_setup<double>(md, a, s))) return rc;
    // start from the caller's x: r = b - A x (projected), then restart CG from r
    // (the restart sets x = 0 and finishes at once if b = 0)
    if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.r64, w.partial, w.sc,
                                   s)))
        return rc;
    if ((rc = cg_restart64(md, a, s))) return rc;
    const int cap = o.fixed_iters > 0 ? o.fixed_iters : o.maxit;
    if ((rc = cg_iterate<double>(m, bc, lambda, nu, nu_c, a, w.sc, w.host_sc, cap, true))) return rc;
    if ((rc = cg_finish<double>(md, a, s))) return rc;
    // true residual from x
    if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.q64, w.partial,
                                   w.sc, s)))
        return rc;
    DG_HIP_CHECK(hipMemcpyAsync(w.host_sc, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    const CgScalars &h = *w.host_sc;
    info.iters = h.iter;
    info.outer_iters = 0;
    info.status = h.status;
    info.rel_res = h.bnorm2 > 0 ? std::sqrt(h.res2 / h.bnorm2) : 0.0;
    info.true_rel_res = h.bnorm2 > 0 ? std::sqrt(h.true_res2 / h.bnorm2) : 0.0;
    return h.status;
}

// the fast-diagonalisation tables of the mesh for these BCs, uploaded on the
// mesh's stream unless the workspace already holds them
int ensure_fdm_tables(dg_mesh *m, Workspace &w, const int bc[3], FdmDev &f)
{
    if (fdm_table_bytes(m->dev.n, m->dev.P) == 0) {
        set_error("fast diagonalisation needs at most 512 nodes per mesh line (n_d (P+1) <= 512)");
        return DG_ERR_ARG;
    }
    if (!(w.fdm_bc[0] == bc[0] && w.fdm_bc[1] == bc[1] && w.fdm_bc[2] == bc[2])) {
        if (int rc = fdm_build_tables(m->dev, bc, w.fdm_img)) return rc;
        DG_HIP_CHECK(hipMemcpyAsync(w.fdm, w.fdm_img.data(), w.fdm_img.size() * sizeof(double),
                                    hipMemcpyHostToDevice, m->stream));
        for (int d = 0; d < 3; ++d) w.fdm_bc[d] = bc[d];
    }
    fdm_bind(m->dev.n, m->dev.P, w.fdm, f);
    return DG_OK;
}

// CG preconditioned by the fast-diagonalisation inverse of the constant-nu
// operator (FP64).  For a constant nu that inverse is exact, and CG stops
// after one or two steps (rounding); for a nodal nu the preconditioner uses
// nu_ref = sqrt(min nu * max nu), which bounds the preconditioned condition
// number by max nu / min nu.
//
// The solve is split into phases (prepare, start, chunks of iterations with a
// poll of the device state after each, end) so that one host thread can run
// several such solves at once on separate streams; each solve does the same
// arithmetic whether it runs alone or beside others.  A run is FP64 CG
// preconditioned by fast diagonalisation or, with `jacobi`, FP64 Jacobi-PCG
// (the arithmetic of solve_fp64).
struct FdmRun {
    Workspace *w = nullptr;
    hipStream_t s = nullptr;
    const int *bc = nullptr;
    bool jacobi = false;
    double lambda = 0.0, nu_c = 0.0, nu_ref = 0.0;
    const double *nu = nullptr, *rhs = nullptr;
    double *x = nullptr;
    bool singular = false, done = false;
    bool f32 = false;         // FP32 transforms (fdm_apply32)
    bool true_resid = true;   // recompute b - A x at the end (info.true_rel_res)
    bool ended = false;       // the closing work ran with the last chunk (see fdm_chunk)
    FdmDev f{};
    CgVecArgs<double> a{};
    int cap = 0, launched = 0;
    ChunkPlan plan{2, 16, true};
};

// nu_ref of the preconditioner (one host synchronisation for a nodal nu)
int fdm_nu_ref(dg_mesh *m, Workspace &w, const double *nu, double nu_c, double &nu_ref)
{
    nu_ref = nu_c;
    if (!nu) return DG_OK;
    double lo = 0.0, hi = 0.0;
    if (int rc = field_range(nu, (size_t)m->dev.ndof, w.partial, partial_doubles(m->dev), lo, hi, m->stream))
        return rc;
    if (!(lo > 0.0) || !std::isfinite(hi)) {
        set_error("the fast-diagonalisation preconditioner needs a positive, finite nu field");
        return lo != lo || hi != hi ? DG_ERR_NONFINITE : DG_ERR_ARG;
    }
    nu_ref = std::sqrt(lo * hi);
    return DG_OK;
}

// the workspace and its tables (uploads on the mesh's stream)
int fdm_prepare(dg_mesh *m, FdmRun &R)
{
    if (int rc = ensure_workspace(m, *R.w, DG_FP64)) return rc;
    if (R.jacobi) return R.nu ? DG_OK : upload_diag_tables(m, *R.w, R.bc, R.nu_c);
    return ensure_fdm_tables(m, *R.w, R.bc, R.f);
}

// z = the preconditioner applied to r (q as scratch: N doubles, or 2 N
// floats for the FP32 transforms)
int fdm_precond(const MeshDev &md, FdmRun &R)
{
    Workspace &w = *R.w;
    if (R.f32)
        return fdm_apply32(md, R.f, R.lambda, R.nu_ref, R.singular, w.r64, w.d64, (float *)w.q64, w.sc, R.s);
    return fdm_apply(md, R.f, R.lambda, R.nu_ref, R.singular, w.r64, w.d64, w.q64, w.sc, R.s);
}

// Jacobi-PCG start: b, the diagonal (nodal nu) or its tables, r = b - A x
// from the caller's x and the restart from r, as in solve_fp64
int jacobi_start(dg_mesh *m, FdmRun &R, const dg_solve_opts &o)
{
    const MeshDev &md = m->dev;
    Workspace &w = *R.w;
    hipStream_t s = R.s;
    int rc;
    R.singular = (R.lambda == 0.0) && !has_dirichlet(R.bc);
    *w.host_sc = init_scalars(md, o.tol, o.maxit, o.fixed_iters, R.singular);
    DG_HIP_CHECK(hipMemcpyAsync(w.sc, w.host_sc, sizeof(CgScalars), hipMemcpyHostToDevice, s));
    CgVecArgs<double> &a = R.a;
    a = vec_args<double>(w, R.singular, w.sc);
    if (R.nu) {
        if ((rc = launch_diag<double>(md, R.bc, R.lambda, R.nu, R.nu_c, w.d64, s, true))) return rc;
        a.d = w.d64;
    } else {
        a.dtab = w.dtab64;
        a.lam = R.lambda;
    }
    a.x = R.x;
    a.r = w.r64;
    a.p = w.p64;
    a.q = w.q64;
    a.src = R.rhs;
    a.bvec = w.b64;
    a.weak = o.rhs_is_weak;
    a.keep_x = 1;
    if ((rc = cg_setup<double>(md, a, s))) return rc;
    if ((rc = launch_resid<double>(md, R.bc, R.lambda, R.nu, R.nu_c, R.x, w.b64, w.r64, w.partial, w.sc, s)))
        return rc;
    if ((rc = cg_restart64(md, a, s))) return rc;
    R.cap = o.fixed_iters > 0 ? o.fixed_iters : o.maxit;
    R.plan = ChunkPlan(4, 64, true);
    R.launched = 0;
    R.done = false;
    R.ended = false;
    return DG_OK;
}

// b, r = b - A x from the caller's x, the first preconditioned direction
int fdm_start(dg_mesh *m, FdmRun &R, const dg_solve_opts &o)
{
    if (R.jacobi) return jacobi_start(m, R, o);
    const MeshDev &md = m->dev;
    Workspace &w = *R.w;
    hipStream_t s = R.s;
    int rc;
    R.singular = (R.lambda == 0.0) && !has_dirichlet(R.bc);
    *w.host_sc = init_scalars(md, o.tol, o.maxit, o.fixed_iters, R.singular);
    DG_HIP_CHECK(hipMemcpyAsync(w.sc, w.host_sc, sizeof(CgScalars), hipMemcpyHostToDevice, s));
    CgVecArgs<double> &a = R.a;
    a = vec_args<double>(w, R.singular, w.sc);
    a.x = R.x;
    a.r = w.r64;
    a.p = w.p64;
    a.q = w.q64;
    a.z = w.d64;  // the diagonal slot holds z (no Jacobi diagonal here)
    a.src = R.rhs;
    a.bvec = w.b64;
    a.weak = o.rhs_is_weak;
    a.keep_x = 1;
    if ((rc = cg_setup<double>(md, a, s))) return rc;  // b, norms (no diagonal: d, dtab null)
    // r = b - A x from the caller's x, its norm and the stopping test
    if ((rc = launch_resid<double>(md, R.bc, R.lambda, R.nu, R.nu_c, R.x, w.b64, w.r64, w.partial, w.sc, s)))
        return rc;
    if ((rc = cg_fdm_start(md, a, s))) return rc;
    if ((rc = fdm_precond(md, R))) return rc;
    if ((rc = cg_rz(md, a, s))) return rc;
    if ((rc = cg_pupdate_fdm(md, a, true, s))) return rc;
    R.cap = o.fixed_iters > 0 ? o.fixed_iters : o.maxit;
    R.plan = ChunkPlan(2, 16, true);
    R.launched = 0;
    R.done = false;
    R.ended = false;
    return DG_OK;
}

// one chunk of iterations (they do nothing once the device has flagged
// completion) and the copy of the device state back to the host
int fdm_chunk(dg_mesh *m, FdmRun &R)
{
    const MeshDev &md = m->dev;
    Workspace &w = *R.w;
    hipStream_t s = R.s;
    int rc;
    if (R.jacobi) {
        for (int k = 0; k < R.plan.chunk; ++k) {
            if ((rc = launch_apply_cg<double>(md, R.bc, R.lambda, R.nu, R.nu_c, R.a.p, w.q64, w.partial, w.sc, s)))
                return rc;
            if ((rc = cg_update<double>(md, R.a, s))) return rc;
            if ((rc = cg_pupdate<double>(md, R.a, s))) return rc;
        }
        R.launched += R.plan.chunk;
        if (!R.true_resid && (rc = cg_finish<double>(md, R.a, s))) return rc;
        DG_HIP_CHECK(hipMemcpyAsync(w.host_sc, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        return DG_OK;
    }
    for (int k = 0; k < R.plan.chunk; ++k) {
        if ((rc = launch_apply_cg<double>(md, R.bc, R.lambda, R.nu, R.nu_c, R.a.p, w.q64, w.partial, w.sc, s)))
            return rc;
        if ((rc = cg_update_fdm(md, R.a, s))) return rc;
        if ((rc = fdm_precond(md, R))) return rc;
        if ((rc = cg_rz(md, R.a, s))) return rc;
        if ((rc = cg_pupdate_fdm(md, R.a, false, s))) return rc;
    }
    R.launched += R.plan.chunk;
    // Without a final b - A x, the closing work (the singular mean shift of
    // x) is enqueued with every chunk, so that the chunk that converges also
    // ends the solve and its poll is the last host wait.  On a chunk that
    // does not converge the shift only moves x along the null space (r is
    // carried by its recurrence), and the last chunk's shift sets the mean.
    if (!R.true_resid && (rc = cg_finish<double>(md, R.a, s))) return rc;
    DG_HIP_CHECK(hipMemcpyAsync(w.host_sc, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    return DG_OK;
}

// wait for the chunk; R.done once the device has flagged completion
int fdm_poll(FdmRun &R)
{
    DG_HIP_CHECK(hipStreamSynchronize(R.s));
    if (R.w->host_sc->done) {
        R.done = true;
        R.ended = !R.true_resid;
        return DG_OK;
    }
    if (R.launched > R.cap + 64) {
        set_error("CG did not flag completion");
        return DG_ERR_DEVICE;
    }
    R.plan.next(*R.w->host_sc);
    return DG_OK;
}

// the singular mean shift, the true residual, and the result
int fdm_end(dg_mesh *m, FdmRun &R, dg_solve_info &info)
{
    const MeshDev &md = m->dev;
    Workspace &w = *R.w;
    hipStream_t s = R.s;
    int rc;
    if (R.ended) {  // finished with the last chunk, whose scalars are on the host
        const CgScalars &h = *w.host_sc;
        info.iters = h.iter;
        info.outer_iters = 0;
        info.status = h.status;
        info.rel_res = h.bnorm2 > 0 ? std::sqrt(h.res2 / h.bnorm2) : 0.0;
        info.true_rel_res = info.rel_res;
        return h.status;
    }
    if ((rc = cg_finish<double>(md, R.a, s))) return rc;
    if (R.true_resid &&
        (rc = launch_resid<double>(md, R.bc, R.lambda, R.nu, R.nu_c, R.x, w.b64, w.q64, w.partial, w.sc, s)))
        return rc;
    DG_HIP_CHECK(hipMemcpyAsync(w.host_sc, w.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    const CgScalars &h = *w.host_sc;
    info.iters = h.iter;
    info.outer_iters = 0;
    info.status = h.status;
    info.rel_res = h.bnorm2 > 0 ? std::sqrt(h.res2 / h.bnorm2) : 0.0;
    info.true_rel_res = R.true_resid ? (h.bnorm2 > 0 ? std::sqrt(h.true_res2 / h.bnorm2) : 0.0) : info.rel_res;
    return h.status;
}

// f32: the preconditioner's transforms in FP32 (CG itself stays FP64)
int solve_fdm(dg_mesh *m, Workspace &w, const int bc[3], double lambda, const double *nu,
              double nu_c, const double *rhs, double *x, const dg_solve_opts &o, dg_solve_info &info,
              bool f32 = false, bool true_resid = true)
{
    FdmRun R;
    R.f32 = f32;
    R.true_resid = true_resid;
    R.w = &w;
    R.s = m->stream;
    R.bc = bc;
    R.lambda = lambda;
    R.nu = nu;
    R.nu_c = nu_c;
    R.rhs = rhs;
    R.x = x;
    int rc;
    if ((rc = fdm_prepare(m, R))) return rc;
    if ((rc = fdm_nu_ref(m, w, nu, nu_c, R.nu_ref))) return rc;
    if ((rc = fdm_start(m, R, o))) return rc;
    while (!R.done) {
        if ((rc = fdm_chunk(m, R))) return rc;
        if ((rc = fdm_poll(R))) return rc;
    }
    return fdm_end(m, R, info);
}

// The streams of the second to last concurrent solve: one set per device
// for the whole process (non-blocking, default priority, created on first
// use and kept until the process ends), shared by every mesh, so that
// meshes do not each hold hardware queues of their own.  Concurrent solves
// of two meshes from two host threads then share these streams: their work
// is ordered on them, which is correct and only less concurrent.
int concurrent_streams(hipStream_t (&out)[kMaxConcurrent - 1], bool create)
{
    static std::mutex mu;
    static std::map<int, std::array<hipStream_t, kMaxConcurrent - 1>> pool;
    int dev = 0;
    DG_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = pool.find(dev);
    if (it == pool.end()) {
        if (!create) {
            for (auto &x : out) x = nullptr;
            return DG_OK;
        }
        std::array<hipStream_t, kMaxConcurrent - 1> a{};
        for (auto &x : a) DG_HIP_CHECK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        it = pool.emplace(dev, a).first;
    }
    for (int k = 0; k < kMaxConcurrent - 1; ++k) out[k] = it->second[k];
    return DG_OK;
}

// One system of a concurrent run: its operator (BCs, lambda, nu field or
// nu_c), right-hand side (weak: a weak load), solution, and preconditioner
// (jacobi: Jacobi-PCG in FP64, else fast diagonalisation, FP32 transforms
// when f32).
struct ConcSys {
    int bc[3];
    double lambda;
    const double *nu;
    double nu_c;
    const double *rhs;
    double *x;
    int weak;
    bool jacobi, f32;
};

// Up to kMaxConcurrent solves at once: the first on the mesh's stream with
// its workspace, the others on the shared extra streams with workspaces of
// the mesh's own (created on first use).
int conc_solve(dg_mesh *m, int nsys, const ConcSys *sys, const dg_solve_opts &o, dg_solve_info *info,
               bool true_resid)
{
    if (nsys < 1 || nsys > kMaxConcurrent) {
        set_error("concurrent solves: need 1 <= nsys <= 4");
        return DG_ERR_ARG;
    }
    TraceRange tr("solve: concurrent");
    FdmRun R[kMaxConcurrent];
    int rc;
    hipStream_t alt[kMaxConcurrent - 1] = {};
    if (nsys > 1 && (rc = concurrent_streams(alt, true))) return rc;
    for (int k = 0; k < nsys; ++k) {
        R[k].w = k == 0 ? &m->ws : &m->alt_ws[k - 1];
        R[k].s = k == 0 ? m->stream : alt[k - 1];
        R[k].bc = sys[k].bc;
        R[k].jacobi = sys[k].jacobi;
        R[k].lambda = sys[k].lambda;
        R[k].nu = sys[k].nu;
        R[k].nu_c = sys[k].nu_c;
        R[k].rhs = sys[k].rhs;
        R[k].x = sys[k].x;
        R[k].f32 = sys[k].f32;
        R[k].true_resid = true_resid;
        if ((rc = fdm_prepare(m, R[k]))) return rc;
    }
    // nu_ref of the fast-diagonalisation runs, once per nu field
    for (int k = 0; k < nsys; ++k) {
        if (R[k].jacobi) continue;
        int j = 0;
        while (j < k && (R[j].jacobi || R[j].nu != R[k].nu || R[j].nu_c != R[k].nu_c)) ++j;
        if (j < k)
            R[k].nu_ref = R[j].nu_ref;
        else if ((rc = fdm_nu_ref(m, m->ws, R[k].nu, R[k].nu_c, R[k].nu_ref)))
            return rc;
    }
    // the other streams start after the mesh's stream has done its work so
    // far (the right-hand sides, the tables)
    if (nsys > 1) {
        if (!m->alt_event) DG_HIP_CHECK(hipEventCreateWithFlags(&m->alt_event, hipEventDisableTiming));
        DG_HIP_CHECK(hipEventRecord(m->alt_event, m->stream));
        for (int k = 1; k < nsys; ++k) DG_HIP_CHECK(hipStreamWaitEvent(R[k].s, m->alt_event, 0));
    }
    for (int k = 0; k < nsys; ++k) {
        dg_solve_opts ok = o;
        ok.rhs_is_weak = sys[k].weak;
        if ((rc = fdm_start(m, R[k], ok))) return rc;
    }
    for (;;) {
        bool all = true;
        for (int k = 0; k < nsys; ++k)
            if (!R[k].done && (rc = fdm_chunk(m, R[k]))) return rc;
        for (int k = 0; k < nsys; ++k) {
            if (!R[k].done && (rc = fdm_poll(R[k]))) return rc;
            all = all && R[k].done;
        }
        if (all) break;
    }
    int worst = DG_OK;
    for (int k = 0; k < nsys; ++k) {
        dg_solve_info ik{};
        rc = fdm_end(m, R[k], ik);
        if (info) info[k] = ik;
        if (rc < 0 && (worst >= 0 || rc < worst)) worst = rc;
        else if (rc > 0 && worst == DG_OK) worst = rc;
    }
    return worst;
}

int fdm_concurrent(dg_mesh *m, int nsys, double lambda, const double *nu, double nu_c,
                   const double *const *rhs, double *const *x, const int *weak, const dg_solve_opts &o,
                   dg_solve_info *info, bool true_resid)
{
    if (nsys < 1 || nsys > kMaxConcurrent) {
        set_error("concurrent solves: need 1 <= nsys <= 4");
        return DG_ERR_ARG;
    }
    ConcSys sys[kMaxConcurrent];
    for (int k = 0; k < nsys; ++k) {
        for (int d = 0; d < 3; ++d) sys[k].bc[d] = m->dev.bc[d];
        sys[k].lambda = lambda;
        sys[k].nu = nu;
        sys[k].nu_c = nu_c;
        sys[k].rhs = rhs[k];
        sys[k].x = x[k];
        sys[k].weak = weak ? weak[k] : o.rhs_is_weak;
        sys[k].jacobi = false;
        sys[k].f32 = o.precision == DG_MIXED;
    }
    return conc_solve(m, nsys, sys, o, info, true_resid);
}

// FP64 refinement around FP32 Jacobi-PCG with residual replacement: the FP32
// recurrence runs until its residual has dropped by inner_tol (or claims
// convergence); then the FP32 correction is added to the FP64 solution, the
// FP64 residual is recomputed and tested, and the recurrence continues from
// it with the same search direction (rescaled) instead of restarting.
// When the FP32 recurrence is limited by its precision (kappa * eps_32 not
// small) -- a cycle falls far short of its target, or needs more than three
// times the iterations of the first cycle -- or the FP32 iteration cap is
// reached, the solve continues as FP64 PCG from the current solution.
int solve_mixed(dg_mesh *m, const int bc[3], double lambda, const double *nu, double nu_c,
                const double *rhs, double *x, const dg_solve_opts &o, dg_solve_info &info)
{
    Workspace &w = m->ws;
    int rc = ensure_workspace(m, w, DG_MIXED);
    if (rc) return rc;
    const MeshDev &md = m->dev;
    hipStream_t s = m->stream;
    const bool singular = (lambda == 0.0) && !has_dirichlet(bc);
    const size_t N = (size_t)md.ndof;
    CgScalars *osc = w.sc, *isc = w.sc + 1;
    CgScalars *hosc = w.host_sc, *hisc = w.host_sc + 1;

    // FP32 operator data
    const float *nu32 = nullptr;
    if (nu) {
        if ((rc = convert_f64_to_f32(nu, w.nu32, N, s))) return rc;
        nu32 = w.nu32;
    }
    // the Jacobi diagonal: stored for the FP32 inner solve (computing it there
    // measured no faster); for the FP64 continuation of a constant-nu solve it
    // is computed where it is used, as in solve_fp64
    if ((rc = launch_diag<float>(md, bc, lambda, nu32, nu_c, w.d32, s, true))) return rc;
    const float *d32 = w.d32;
    const double *tab64 = nullptr;
    if (!nu) {
        if ((rc = upload_diag_tables(m, w, bc, nu_c))) return rc;
        tab64 = w.dtab64;
    }

    // outer set-up: b (projected), r = b, x = 0, ||M^-1 b||
    *hosc = init_scalars(md, o.tol, o.maxit, 0, singular);
    DG_HIP_CHECK(hipMemcpyAsync(osc, hosc, sizeof(CgScalars), hipMemcpyHostToDevice, s));
    CgVecArgs<double> oa = vec_args<double>(w, singular, osc);
    oa.x = x;
    oa.r = w.r64;
    oa.p = nullptr;
    oa.q = nullptr;
    oa.d = nullptr;
    oa.src = rhs;
    oa.bvec = w.b64;
    oa.weak = o.rhs_is_weak;
    oa.keep_x = 1;
    if ((rc = cg_setup<double>(md, oa, s))) return rc;
    // start from the caller's x: r64 = b - A x (projected)
    if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.r64, w.partial, osc,
                                   s)))
        return rc;
    // first inner right-hand side r32 = r64 / scale, then the inner set-up
    CgVecArgs<float> ia = vec_args<float>(w, singular, osc);
    ia.src64 = w.r64;
    ia.r = w.b32;
    ia.x = w.x32;
    ia.d = d32;
    if ((rc = ir_scale(md, ia, s))) return rc;
    if ((rc = ir_to_inner(md, ia, s))) return rc;
    *hisc = init_scalars(md, o.inner_tol, o.inner_maxit, 0, singular);
    DG_HIP_CHECK(hipMemcpyAsync(isc, hisc, sizeof(CgScalars), hipMemcpyHostToDevice, s));
    CgVecArgs<float> ca = vec_args<float>(w, singular, isc);
    ca.x = w.x32;
    ca.r = w.r32;
    ca.p = w.p32;
    ca.q = w.q32;
    ca.d = d32;
    ca.src = w.b32;
    ca.bvec = w.b32;  // in place (already weak)
    ca.weak = 1;
    if ((rc = cg_setup<float>(md, ca, s))) return rc;
    DG_HIP_CHECK(hipMemcpyAsync(hosc, osc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    const double bnorm2 = hosc->bnorm2;
    const double tol2 = hosc->tol2;  // tol^2 ||M^-1 b||^2
    int status = hosc->status;
    if (status >= 0 && bnorm2 == 0.0) {  // b = 0: x = 0 whatever the initial guess
        DG_HIP_CHECK(hipMemsetAsync(x, 0, md.ndof * sizeof(double), s));
        DG_HIP_CHECK(hipStreamSynchronize(s));
        info.iters = 0;
        info.outer_iters = 0;
        info.status = DG_OK;
        info.rel_res = info.true_rel_res = 0.0;
        return DG_OK;
    }
    double res2 = hosc->true_res2;  // ||M^-1 (b - A x0)||^2
    int outer = 0;
    int inner_iters = 0, fp64_iters = 0;
    bool fp64_continue = false;
    double cycle_start = res2;  // ||M^-1 r||^2 at the start of the FP32 cycle
    int first_cycle = -1;         // FP32 iterations of the first cycle
    ia.r = w.r32;
    while (status == DG_OK && bnorm2 > 0.0 && res2 > tol2) {
        const int iters_before = inner_iters;
        if ((rc = cg_iterate<float>(m, bc, lambda, nu32, nu_c, ca, isc, hisc, o.inner_maxit))) return rc;
        inner_iters = hisc->iter;
        const int istat = hisc->status;
        if (istat < 0 && istat != DG_ERR_NOT_SPD) {
            status = istat;
            break;
        }
        if (first_cycle < 0) first_cycle = inner_iters - iters_before;
        // x64 += scale * x32 ; r64 = b - A64 x64 (projected), ||M^-1 r||
        CgVecArgs<float> acc = vec_args<float>(w, singular, osc);
        acc.x = w.x32;
        acc.dst64 = x;
        if ((rc = ir_accumulate(md, acc, s))) return rc;
        if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.r64, w.partial,
                                       osc, s)))
            return rc;
        DG_HIP_CHECK(hipMemcpyAsync(hosc, osc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        DG_HIP_CHECK(hipStreamSynchronize(s));
        res2 = hosc->true_res2;
        ++outer;
        if (!std::isfinite(res2)) {
            status = DG_ERR_NONFINITE;
            break;
        }
        if (res2 <= tol2) break;
        const double target = std::max(o.inner_tol * o.inner_tol * cycle_start, tol2);
        if (res2 > 25.0 * target || istat == DG_NOT_CONVERGED || inner_iters >= o.inner_maxit) {
            fp64_continue = true;
            break;
        }
        if (outer >= o.maxit) {
            status = DG_NOT_CONVERGED;
            break;
        }
        cycle_start = res2;
        // replace the recurrence residual; a breakdown restarts the direction
        if ((rc = ir_scale(md, ia, s))) return rc;
        const int cap = std::min<long long>(o.inner_maxit, (long long)inner_iters + std::max(3 * first_cycle, 50));
        if ((rc = ir_replace(md, ia, isc, o.inner_tol * o.inner_tol, istat == DG_ERR_NOT_SPD, cap, s)))
            return rc;
        if ((rc = cg_pupdate<float>(md, ca, s))) return rc;
    }
    if (fp64_continue && status == DG_OK) {
        // FP64 PCG from x, starting at the residual r64 just computed
        if (nu && (rc = launch_diag<double>(md, bc, lambda, nu, nu_c, w.d64, s, true))) return rc;
        CgVecArgs<double> fa = vec_args<double>(w, singular, osc);
        fa.dtab = tab64;
        fa.lam = lambda;
        fa.x = x;
        fa.r = w.r64;
        fa.p = w.p64;
        fa.q = w.q64;
        fa.d = nu ? w.d64 : nullptr;
        if ((rc = cg_restart64(md, fa, s))) return rc;
        if ((rc = cg_iterate<double>(m, bc, lambda, nu, nu_c, fa, osc, hosc, o.maxit))) return rc;
        fp64_iters = hosc->iter;
        status = hosc->status;
        if (!singular && status >= 0) {
            if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.r64, w.partial,
                                           osc, s)))
                return rc;
            DG_HIP_CHECK(hipMemcpyAsync(hosc, osc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            DG_HIP_CHECK(hipStreamSynchronize(s));
            res2 = hosc->true_res2;
        }
    }
    if (singular && status >= 0) {
        if ((rc = cg_finish<double>(md, oa, s))) return rc;
        if ((rc = launch_resid<double>(md, bc, lambda, nu, nu_c, x, w.b64, w.r64, w.partial,
                                       osc, s)))
            return rc;
        DG_HIP_CHECK(hipMemcpyAsync(hosc, osc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        DG_HIP_CHECK(hipStreamSynchronize(s));
        res2 = hosc->true_res2;
    }
    info.iters = inner_iters + fp64_iters;
    info.outer_iters = outer;
    info.status = status;
    info.rel_res = bnorm2 > 0 ? std::sqrt(res2 / bnorm2) : 0.0;
    info.true_rel_res = info.rel_res;
    return status;
}

// lent: workspace memory the caller provides (FP64 solves only); nullptr =
// the mesh's own workspace, allocated on demand
// true_resid = false: the fast-diagonalisation solve skips its final
// b - A x (info true_rel_res = rel_res)
int solve_common(dg_mesh *m, const int bc[3], double lambda, const double *nu, double nu_c,
                 const double *rhs, double *x, const dg_solve_opts *opts, dg_solve_info *info,
                 Workspace *lent = nullptr, bool true_resid = true)
{
    const double t0 = now();
    if (int rc = check_mesh(m)) return rc;
    dg_solve_opts o;
    dg_default_opts(&o);
    if (opts) o = *opts;
    if (!rhs || !x || (const void *)rhs == (const void *)x) {
        set_error("rhs and x must be distinct device arrays");
        return DG_ERR_ARG;
    }
    if (!(lambda >= 0.0) || !std::isfinite(lambda) || (!nu && !(nu_c > 0.0))) {
        set_error("lambda must be >= 0 and nu > 0");
        return DG_ERR_ARG;
    }
    if (!(o.tol > 0.0) || o.maxit < 0 || (o.precision != DG_FP64 && o.precision != DG_MIXED)) {
        set_error("bad solver options");
        return DG_ERR_ARG;
    }
    dg_solve_info inf{};
    int rc;
    if (o.precond != DG_PC_JACOBI && o.precond != DG_PC_FDM) {
        set_error("unknown preconditioner");
        return DG_ERR_ARG;
    }
    Workspace &wk = lent ? *lent : m->ws;
    if (lent && o.precision != DG_FP64) {
        set_error("the no-allocation solve is FP64 only");
        return DG_ERR_ARG;
    }
    TraceRange tr(o.precond == DG_PC_FDM
                      ? (o.precision == DG_MIXED ? "solve: FDM-PCG, FP32 transforms" : "solve: FDM-PCG FP64")
                      : (o.precision == DG_MIXED ? "solve: Jacobi-PCG mixed" : "solve: Jacobi-PCG FP64"));
    if (o.precond == DG_PC_FDM) {
        rc = solve_fdm(m, wk, bc, lambda, nu, nu_c, rhs, x, o, inf, o.precision == DG_MIXED, true_resid);
    } else if (lent) {
        rc = solve_fp64(m, *lent, bc, lambda, nu, nu_c, rhs, x, o, inf);
    } else if (o.precision == DG_MIXED) {
        if (!(o.inner_tol > 0.0 && o.inner_tol < 1.0) || o.inner_maxit <= 0) {
            set_error("bad inner solver options");
            return DG_ERR_ARG;
        }
        rc = solve_mixed(m, bc, lambda, nu, nu_c, rhs, x, o, inf);
    } else {
        rc = solve_fp64(m, m->ws, bc, lambda, nu, nu_c, rhs, x, o, inf);
    }
    inf.seconds = now() - t0;
    if (rc < 0 && g_last_error.empty()) set_error("solver error " + std::to_string(rc));
    if (rc == DG_ERR_NOT_SPD) set_error("CG breakdown: p^T A p <= 0");
    if (rc == DG_ERR_NONFINITE) set_error("non-finite value in the data or the iteration");
    if (info) *info = inf;
    return rc;
}

// Device block of the mesh geometry: hx|hy|hz, 1/h (FP64), the same in FP32,
// and the visiting order of the apply's element groups.
size_t geo_bytes(const int n[3], int P, int64_t nel)
{
    const size_t S = (size_t)n[0] + n[1] + n[2];
    return align256(S * 8) * 2 + align256(S * 4) * 2 + align256((size_t)apply_groups(P, nel) * 4);
}

int upload_geometry(dg_mesh *m, void *ext)
{
    MeshDev &d = m->dev;
    const size_t S = (size_t)d.n[0] + d.n[1] + d.n[2];
    const size_t bytes = geo_bytes(d.n, d.P, d.nel);
    std::vector<char> host(bytes, 0);
    char *hp = host.data();
    size_t off = 0;
    auto put = [&](const void *src, size_t nb) {
        std::memcpy(hp + off, src, nb);
        const size_t at = off;
        off += align256(nb);
        return at;
    };
    std::vector<double> h, ih;
    std::vector<float> hf, ihf;
    for (int k = 0; k < 3; ++k)
        for (int e = 0; e < d.n[k]; ++e) h.push_back(d.v[k][e + 1] - d.v[k][e]);
    for (double v : h) {
        ih.push_back(1.0 / v);
        hf.push_back((float)v);
        ihf.push_back(1.0f / (float)v);
    }
    const std::vector<int> ord = apply_order(d.n, d.P);
    const size_t o_h64 = put(h.data(), S * 8), o_ih64 = put(ih.data(), S * 8);
    const size_t o_h32 = put(hf.data(), S * 4), o_ih32 = put(ihf.data(), S * 4);
    const size_t o_ord = put(ord.data(), ord.size() * 4);
    if (ext) {
        m->geo_block = ext;
        m->geo_external = true;
    } else {
        DG_HIP_CHECK(hipMalloc(&m->geo_block, bytes));
    }
    char *base = (char *)m->geo_block;
    d.h64 = (double *)(base + o_h64);
    d.ih64 = (double *)(base + o_ih64);
    d.h32 = (float *)(base + o_h32);
    d.ih32 = (float *)(base + o_ih32);
    d.order = (int *)(base + o_ord);
    DG_HIP_CHECK(hipMemcpyAsync(m->geo_block, host.data(), bytes, hipMemcpyHostToDevice, m->stream));
    DG_HIP_CHECK(hipStreamSynchronize(m->stream));
    return DG_OK;
}

size_t batched_footprint(const MeshDev &m, int precision, int nsys)
{
    const size_t N = (size_t)m.ndof;
    const size_t ti = precision == DG_FP64 ? sizeof(double) : sizeof(float);
    size_t b = 0;
    b += (size_t)nsys * (2 * align256(N * sizeof(double)) + 8 * align256(N * ti));
    b += align256(batched_partial_doubles() * sizeof(double));
    b += align256(batched_sync_bytes()) + align256(batched_result_bytes());
    return b;
}

int solve_batched(dg_mesh *m, int nsys, const double *lambdas, const double *const *nu_fields,
                  const int *is_poisson, const double *const *rhs, double *const *x,
                  const dg_solve_opts &o, dg_solve_info *infos, int flags)
{
    TraceRange tr("solve: batched");
    const MeshDev &md = m->dev;
    hipStream_t s = m->stream;
    const bool f32 = o.precision == DG_MIXED;
    const size_t N = (size_t)md.ndof;
    const size_t ti = f32 ? sizeof(float) : sizeof(double);
    // room for this call's systems only; a later call with more systems (or
    // the other precision) grows it, as dg_solve_footprint(m, precision, nsys)
    // states
    const size_t need = batched_footprint(md, o.precision, nsys);
    BatchWorkspace &w = m->bws;
    if (!w.base || w.bytes < need) {
        if (w.base) {
            DG_HIP_CHECK(hipStreamSynchronize(s));
            DG_HIP_CHECK(hipFree(w.base));
            w.base = nullptr;
        }
        hipError_t e = hipMalloc(&w.base, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("batched workspace allocation of " + std::to_string(need) + " bytes failed");
            return DG_ERR_OOM;
        }
        w.bytes = need;
    }
    const size_t host_bytes = batched_result_bytes() + 256;
    if (!w.host_state) DG_HIP_CHECK(hipHostMalloc(&w.host_state, host_bytes, 0));
    char *p = (char *)w.base;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align256(bytes);
        return (void *)r;
    };
    BatchRequest rq{};
    rq.nsys = nsys;
    rq.tol = o.tol;
    // mixed: replace the FP32 recurrence residual once it has dropped by
    // inner_tol; FP64: only when it claims convergence
    rq.delta = f32 ? o.inner_tol : 0.0;
    rq.maxit = o.inner_maxit;
    rq.max_replace = std::max(1, std::min(o.maxit, 1000));
    rq.weak = o.rhs_is_weak;
    rq.handoff = (flags & DG_BATCH_HANDOFF) ? 1 : 0;
    rq.inner_fp32 = f32;
    {
        double vol = 1.0;
        for (int d = 0; d < 3; ++d) vol *= md.v[d][md.n[d]] - md.v[d][0];
        rq.mass_mean = vol / (double)md.ndof;
    }
    for (int k = 0; k < nsys; ++k) {
        BatchSysDesc &D = rq.sys[k];
        D.x64 = x[k];
        D.rhs = rhs[k];
        D.b64 = (double *)take(N * 8);
        D.r64 = (double *)take(N * 8);
        D.xi = take(N * ti);
        D.ri = take(N * ti);
        D.pi = take(N * ti);
        D.qi = take(N * ti);
        D.ui = take(N * ti);
        D.si = take(N * ti);
        D.di = take(N * ti);
        void *nui = take(N * ti);
        const bool pois = is_poisson && is_poisson[k];
        for (int d = 0; d < 3; ++d)
            D.bc[d] = (pois && md.bc[d] == DG_BC_DIRICHLET) ? DG_BC_NEUMANN : md.bc[d];
        D.lambda = pois ? 0.0 : lambdas[k];
        D.singular = (D.lambda == 0.0 && !has_dirichlet(D.bc)) ? 1 : 0;
        D.nu64 = (!pois && nu_fields && nu_fields[k]) ? nu_fields[k] : nullptr;
        D.nui = nullptr;
        int rc;
        if (f32) {
            if (D.nu64) {
                if ((rc = convert_f64_to_f32(D.nu64, (float *)nui, N, s))) return rc;
                D.nui = nui;
            }
            rc = launch_diag<float>(md, D.bc, D.lambda, (const float *)D.nui, 1.0, (float *)D.di, s, true);
        } else {
            D.nui = D.nu64;
            rc = launch_diag<double>(md, D.bc, D.lambda, D.nu64, 1.0, (double *)D.di, s, true);
        }
        if (rc) return rc;
    }
    rq.partial = (double *)take(batched_partial_doubles() * sizeof(double));
    rq.sync = take(batched_sync_bytes());
    rq.results = take(batched_result_bytes());
    int bpc = 0;
    int rc = batched_launch(md, rq, s, &bpc);
    if (rc) return rc;
    char *hs = (char *)w.host_state;
    DG_HIP_CHECK(hipMemcpyAsync(hs, rq.results, batched_result_bytes(), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipMemcpyAsync(hs + batched_result_bytes(), (char *)rq.sync + batched_sync_err_offset(),
                                sizeof(unsigned), hipMemcpyDeviceToHost, s));
    DG_HIP_CHECK(hipStreamSynchronize(s));
    if ((rc = batched_check_sync(hs + batched_result_bytes()))) return rc;
    int worst = DG_OK;
    for (int k = 0; k < nsys; ++k) {
        BatchSysResult r{};
        batched_read_results(hs, k, &r);
        dg_solve_info ci{};
        if (r.status == kBatchHandoff) {
            // the last unconverged system: continue from its current solution
            // with the single-system solver (same operator, options and rule)
            const BatchSysDesc &D = rq.sys[k];
            // (FP64 with the fast-diagonalisation preconditioner if asked for)
            const int rc2 =
                o.precond == DG_PC_FDM ? solve_fdm(m, m->ws, D.bc, D.lambda, D.nu64, 1.0, rhs[k], x[k], o, ci)
                : f32                 ? solve_mixed(m, D.bc, D.lambda, D.nu64, 1.0, rhs[k], x[k], o, ci)
                                      : solve_fp64(m, m->ws, D.bc, D.lambda, D.nu64, 1.0, rhs[k], x[k], o, ci);
            r.status = rc2 < 0 ? rc2 : ci.status;
        }
        if (infos) {
            infos[k].iters = r.iters + ci.iters;
            infos[k].outer_iters = r.replaced + ci.outer_iters;
            infos[k].status = r.status;
            if (ci.iters || ci.outer_iters) {
                infos[k].rel_res = ci.rel_res;
                infos[k].true_rel_res = ci.true_rel_res;
            } else {
                infos[k].rel_res = r.bnorm2 > 0 ? std::sqrt(r.res64 / r.bnorm2) : 0.0;
                infos[k].true_rel_res = infos[k].rel_res;
            }
        }
        if (r.status < 0 && (worst >= 0 || r.status < worst)) worst = r.status;
        else if (r.status > 0 && worst == DG_OK) worst = r.status;
    }
    return worst;
}

}  // namespace

// ---------------------------------------------------- no-allocation solve --
// Workspace of helmholtz_solve_noalloc: a fixed device array instead of
// hipMalloc.  Each GPU the library runs on holds its own copy (it comes with
// the library's code object) until the process ends; every call on that GPU
// reuses it.  Host code must use its device address (scratch_address), never
// the symbol itself, which on the host is only a stand-in.
static constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kScratchDevices = 64;

// the device address of `scratch` on the current device, looked up once per
// device with that device current
static int scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[kScratchDevices] = {};
    int dev = -1;
    DG_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("device ordinal out of range for the scratch table");
        return DG_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(std::string("scratch address lookup failed: ") + hipGetErrorString(e));
            return DG_ERR_DEVICE;
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return DG_OK;
}

namespace dg {

int mesh_concurrent_streams(hipStream_t out[kMaxConcurrent - 1])
{
    hipStream_t a[kMaxConcurrent - 1] = {};
    if (int rc = concurrent_streams(a, true)) return rc;
    for (int k = 0; k < kMaxConcurrent - 1; ++k) out[k] = a[k];
    return DG_OK;
}

int solve_fdm_concurrent(dg_mesh *m, int nsys, double lambda, const double *nu, double nu_c,
                         const double *const *rhs, double *const *x, const int *weak,
                         const dg_solve_opts &o, dg_solve_info *info, bool true_resid)
{
    if (int rc = check_mesh(m)) return rc;
    return fdm_concurrent(m, nsys, lambda, nu, nu_c, rhs, x, weak, o, info, true_resid);
}

// The projection substep (dg_project).  step_mode (the IMEX step): the
// pressure solve skips its final b - A x, and the call returns without
// waiting for the device when both meshes share a stream (the step's next
// work is ordered after it there).
int project_impl(dg_mesh *mv, dg_mesh *mp, double *const vv[3], const double *const vbv[3], double *psi,
                 const dg_solve_opts *opts, dg_solve_info *info, bool step_mode)
{
    TraceRange tr("projection");
    double *vx = vv[0], *vy = vv[1], *vz = vv[2];
    const double t0 = now();
    if (int rc = check_mesh(mv)) return rc;
    if (int rc = check_mesh(mp)) return rc;
    if (!vx || !vy || !vz || !psi) {
        set_error("null velocity or pressure array");
        return DG_ERR_ARG;
    }
    // the pressure load -D(v'; v_b), a weak vector, in the pressure mesh's
    // own buffer, on the pressure mesh's stream after the velocity's work
    if (!mp->aux) {
        hipError_t e = hipMalloc((void **)&mp->aux, (size_t)mp->dev.ndof * sizeof(double));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            mp->aux = nullptr;
            set_error("projection load allocation failed");
            return DG_ERR_OOM;
        }
    }
    if (mv->stream != mp->stream) DG_HIP_CHECK(hipStreamSynchronize(mv->stream));
    const double *v[3] = {vx, vy, vz}, *vb[3] = {vbv[0], vbv[1], vbv[2]};
    int rc = launch_divergence(mv->dev, mp->dev, v, vb, -1.0, mp->aux, mp->stream);
    if (rc) return rc;
    dg_solve_opts o;
    dg_default_opts(&o);
    if (opts) o = *opts;
    o.rhs_is_weak = 1;
    dg_solve_info pinfo{};
    int pbc[3];
    for (int d = 0; d < 3; ++d)
        pbc[d] = mp->dev.bc[d] == DG_BC_DIRICHLET ? DG_BC_NEUMANN : mp->dev.bc[d];
    rc = solve_common(mp, pbc, 0.0, nullptr, 1.0, mp->aux, psi, &o, &pinfo, nullptr, !step_mode);
    if (rc < 0) {
        if (info) *info = pinfo;
        return rc;
    }
    double *g[3] = {vx, vy, vz};
    const int rc2 = launch_gradient(mv->dev, mp->dev, psi, v, -1.0, g, mp->stream);
    if (rc2) return rc2;
    if (!step_mode || mv->stream != mp->stream) DG_HIP_CHECK(hipStreamSynchronize(mp->stream));
    pinfo.seconds = now() - t0;
    if (info) *info = pinfo;
    return rc;
}

int mesh_create_impl(int nx, int ny, int nz, int P, const double *xv, const double *yv,
                     const double *zv, const int bc[3], void *hip_stream, void *geo_mem,
                     dg_mesh **out)
{
    g_last_error.clear();
    if (!out || !xv || !yv || !zv || !bc) {
        set_error("null argument");
        return DG_ERR_ARG;
    }
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1 || P < kMinPKernel || P > kMaxPKernel) {
        set_error("need n >= 1 per axis and 3 <= P <= 8");
        return DG_ERR_ARG;
    }
    const int64_t nel = (int64_t)nx * ny * nz;
    const int64_t ndof = nel * (P + 1) * (P + 1) * (P + 1);
    if (ndof >= (int64_t)1 << 31) {
        set_error("mesh too large (>= 2^31 nodes)");
        return DG_ERR_ARG;
    }
    const int nn[3] = {nx, ny, nz};
    const double *vv[3] = {xv, yv, zv};
    for (int d = 0; d < 3; ++d) {
        if (bc[d] != DG_BC_PERIODIC && bc[d] != DG_BC_DIRICHLET && bc[d] != DG_BC_NEUMANN) {
            set_error("bad boundary condition code");
            return DG_ERR_ARG;
        }
        for (int k = 0; k < nn[d]; ++k)
            if (!(vv[d][k + 1] > vv[d][k]) || !std::isfinite(vv[d][k + 1] - vv[d][k])) {
                set_error("vertices must be finite and strictly increasing");
                return DG_ERR_ARG;
            }
    }
    auto m = std::make_unique<dg_mesh>();
    MeshDev &d = m->dev;
    d.P = P;
    d.nel = nel;
    d.ndof = ndof;
    for (int k = 0; k < 3; ++k) {
        d.n[k] = nn[k];
        d.bc[k] = bc[k];
        d.v[k].assign(vv[k], vv[k] + nn[k] + 1);
    }
    m->stream = (hipStream_t)hip_stream;
    if (int rc = upload_geometry(m.get(), geo_mem)) return rc;
    (void)gll_cached(P);
    *out = m.release();
    return DG_OK;
}

size_t mesh_geo_bytes(const int n[3], int P)
{
    return geo_bytes(n, P, (int64_t)n[0] * n[1] * n[2]);
}

size_t solve_footprint_for(const int n[3], int P, int precision)
{
    MeshDev d;
    d.P = P;
    for (int k = 0; k < 3; ++k) d.n[k] = n[k];
    d.nel = (int64_t)n[0] * n[1] * n[2];
    d.ndof = d.nel * (P + 1) * (P + 1) * (P + 1);
    return footprint(d, precision);
}

void mesh_lend_workspace(dg_mesh *m, void *dev, size_t bytes, void *host_sc)
{
    m->ws.base = dev;
    m->ws.bytes = bytes;
    m->ws.external = true;
    m->ws.ndof = -1;
    m->ws.host_sc = (CgScalars *)host_sc;
    m->ws.host_external = true;
}

size_t solve_host_scalar_bytes() { return 2 * sizeof(CgScalars); }

int64_t mesh_ndof(const dg_mesh *m) { return m->dev.ndof; }

}  // namespace dg

// X[node] = 1D coordinate table of axis d at (element index, node index)
__global__ void k_expand_coords(const double *tab, int nx, int ny, int nz, int n, double *X,
                                double *Y, double *Z)
{
    const size_t n3 = (size_t)n * n * n;
    const size_t N = (size_t)nx * ny * nz * n3;
    const double *tx = tab, *ty = tab + (size_t)nx * n, *tz = ty + (size_t)ny * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t el = i / n3, loc = i - el * n3;
        const int a = (int)(loc % n), b = (int)((loc / n) % n), c = (int)(loc / ((size_t)n * n));
        const int ex = (int)(el % nx), ey = (int)((el / nx) % ny), ez = (int)(el / ((size_t)nx * ny));
        if (X) X[i] = tx[(size_t)ex * n + a];
        if (Y) Y[i] = ty[(size_t)ey * n + b];
        if (Z) Z[i] = tz[(size_t)ez * n + c];
    }
}

// ---------------------------------------------------------------- C-ABI --

namespace dg {

const MeshDev *mesh_device(dg_mesh *m) { return m ? &m->dev : nullptr; }
hipStream_t mesh_stream(dg_mesh *m) { return m->stream; }

double *mesh_step_buffer(dg_mesh *m, size_t doubles)
{
    if (m->step_buf && m->step_doubles >= doubles) return m->step_buf;
    if (m->step_buf) {
        // a caller's stream may still use the old buffer (dg_viscous_fd2
        // takes any stream): wait for the whole device before freeing it
        (void)hipDeviceSynchronize();
        (void)hipFree(m->step_buf);
        m->step_buf = nullptr;
        m->step_doubles = 0;
    }
    hipError_t e = hipMalloc((void **)&m->step_buf, doubles * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        m->step_buf = nullptr;
        set_error("step workspace allocation of " + std::to_string(doubles * sizeof(double)) + " bytes failed");
        return nullptr;
    }
    m->step_doubles = doubles;
    return m->step_buf;
}

}  // namespace dg

extern "C" {

const char *dg_last_error(void) { return g_last_error.c_str(); }

void dg_default_opts(dg_solve_opts *o)
{
    if (!o) return;
    o->tol = 1e-10;
    o->maxit = 100000;
    o->precision = DG_FP64;
    o->inner_tol = 1e-2;
    o->inner_maxit = 20000;
    o->rhs_is_weak = 0;
    o->fixed_iters = 0;
    o->precond = DG_PC_JACOBI;
}

int dg_mesh_create(int nx, int ny, int nz, int P, const double *xv, const double *yv,
                   const double *zv, const int bc[3], void *hip_stream, dg_mesh **out)
{
    return dg::mesh_create_impl(nx, ny, nz, P, xv, yv, zv, bc, hip_stream, nullptr, out);
}

int dg_mesh_destroy(dg_mesh *m)
{
    if (!m) return DG_OK;
    (void)hipStreamSynchronize(m->stream);
    if (m->ws.base && !m->ws.external) (void)hipFree(m->ws.base);
    if (m->ws.host_sc && !m->ws.host_external) (void)hipHostFree(m->ws.host_sc);
    if (m->bws.base) (void)hipFree(m->bws.base);
    if (m->bws.host_state) (void)hipHostFree(m->bws.host_state);
    if (m->geo_block && !m->geo_external) (void)hipFree(m->geo_block);
    if (m->aux) (void)hipFree(m->aux);
    if (m->step_buf) (void)hipFree(m->step_buf);
    hipStream_t alt[kMaxConcurrent - 1] = {};
    if (m->alt_ws[0].base && concurrent_streams(alt, false) == DG_OK)
        for (hipStream_t x : alt)
            if (x) (void)hipStreamSynchronize(x);
    for (int k = 0; k < kMaxConcurrent - 1; ++k) {
        if (m->alt_ws[k].base) (void)hipFree(m->alt_ws[k].base);
        if (m->alt_ws[k].host_sc) (void)hipHostFree(m->alt_ws[k].host_sc);
    }
    if (m->alt_event) (void)hipEventDestroy(m->alt_event);
    delete m;
    return DG_OK;
}

int64_t dg_mesh_ndof(const dg_mesh *m) { return m ? m->dev.ndof : -1; }

int dg_mesh_coordinates(dg_mesh *m, double *X, double *Y, double *Z, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    const MeshDev &d = m->dev;
    const int n = d.P + 1;
    const GllTables &t = gll_cached(d.P);
    std::vector<double> tab;
    for (int k = 0; k < 3; ++k)
        for (int e = 0; e < d.n[k]; ++e) {
            const double x0 = d.v[k][e], h = d.v[k][e + 1] - d.v[k][e];
            for (int a = 0; a < n; ++a) tab.push_back(x0 + h * 0.5 * (1.0 + t.xi[a]));
        }
    hipStream_t s = stream ? (hipStream_t)stream : m->stream;
    double *dt = nullptr;
    DG_HIP_CHECK(hipMalloc((void **)&dt, tab.size() * sizeof(double)));
    DG_HIP_CHECK(hipMemcpyAsync(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
    const size_t blocks = std::min<size_t>(((size_t)d.ndof + 255) / 256, 8192);
    hipLaunchKernelGGL(k_expand_coords, dim3((unsigned)blocks), dim3(256), 0, s, dt, d.n[0], d.n[1],
                       d.n[2], n, X, Y, Z);
    DG_HIP_CHECK(hipGetLastError());
    DG_HIP_CHECK(hipStreamSynchronize(s));
    DG_HIP_CHECK(hipFree(dt));
    return DG_OK;
}

size_t dg_solve_footprint(const dg_mesh *m, int precision, int nrhs)
{
    if (!m) return 0;
    if (nrhs <= 1) return footprint(m->dev, precision);
    return batched_footprint(m->dev, precision, nrhs);
}

int helmholtz_apply(dg_mesh *m, double lambda, const void *nu_field, double nu_const,
                    const void *x, void *y, int precision, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    if (!x || !y || x == y) {
        set_error("x and y must be distinct device arrays");
        return DG_ERR_ARG;
    }
    if (!nu_field && !(nu_const > 0.0)) {
        set_error("nu_const must be > 0 without a nu field");
        return DG_ERR_ARG;
    }
    hipStream_t s = stream ? (hipStream_t)stream : m->stream;
    if (precision == DG_FP64)
        return launch_apply<double>(m->dev, m->dev.bc, lambda, (const double *)nu_field, nu_const,
                                    (const double *)x, (double *)y, s);
    if (precision == DG_FP32)
        return launch_apply<float>(m->dev, m->dev.bc, lambda, (const float *)nu_field, nu_const,
                                   (const float *)x, (float *)y, s);
    set_error("precision must be DG_FP64 or DG_FP32");
    return DG_ERR_ARG;
}

int helmholtz_diag(dg_mesh *m, double lambda, const void *nu_field, double nu_const, void *dout,
                   int precision, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    if (!dout || (!nu_field && !(nu_const > 0.0))) {
        set_error("bad arguments");
        return DG_ERR_ARG;
    }
    hipStream_t s = stream ? (hipStream_t)stream : m->stream;
    if (precision == DG_FP64)
        return launch_diag<double>(m->dev, m->dev.bc, lambda, (const double *)nu_field, nu_const,
                                   (double *)dout, s);
    if (precision == DG_FP32)
        return launch_diag<float>(m->dev, m->dev.bc, lambda, (const float *)nu_field, nu_const,
                                  (float *)dout, s);
    set_error("precision must be DG_FP64 or DG_FP32");
    return DG_ERR_ARG;
}

int helmholtz_solve(dg_mesh *m, double lambda, const double *nu_field, double nu_const,
                    const double *rhs, double *x, const dg_solve_opts *opts, dg_solve_info *info)
{
    if (int rc = check_mesh(m)) return rc;
    return solve_common(m, m->dev.bc, lambda, nu_field, nu_const, rhs, x, opts, info);
}

int helmholtz_solve_batched(dg_mesh *m, int nsys, const double *lambdas,
                            const double *const *nu_fields, const int *is_poisson,
                            const double *const *rhs, double *const *x, const dg_solve_opts *opts,
                            dg_solve_info *infos)
{
    return helmholtz_solve_batched_ex(m, nsys, lambdas, nu_fields, is_poisson, rhs, x, opts, infos,
                                      0);
}

int helmholtz_solve_batched_ex(dg_mesh *m, int nsys, const double *lambdas,
                               const double *const *nu_fields, const int *is_poisson,
                               const double *const *rhs, double *const *x,
                               const dg_solve_opts *opts, dg_solve_info *infos, int flags)
{
    const double t0 = now();
    if (int rc = check_mesh(m)) return rc;
    if (nsys < 1 || nsys > kMaxBatch || !rhs || !x) {
        set_error("need 1 <= nsys <= 8 and rhs, x arrays");
        return DG_ERR_ARG;
    }
    dg_solve_opts o;
    dg_default_opts(&o);
    o.precision = DG_MIXED;
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.maxit < 1 || o.inner_maxit < 1 || !(o.inner_tol > 0.0 && o.inner_tol < 1.0) ||
        (o.precision != DG_FP64 && o.precision != DG_MIXED)) {
        set_error("bad solver options");
        return DG_ERR_ARG;
    }
    for (int k = 0; k < nsys; ++k) {
        const bool pois = is_poisson && is_poisson[k];
        if (!rhs[k] || !x[k] || (const void *)rhs[k] == (const void *)x[k]) {
            set_error("rhs and x must be distinct device arrays");
            return DG_ERR_ARG;
        }
        if (!pois && (!lambdas || !(lambdas[k] >= 0.0) || !std::isfinite(lambdas[k]))) {
            set_error("lambda must be >= 0");
            return DG_ERR_ARG;
        }
        for (int j = 0; j < k; ++j)
            if (x[j] == x[k]) {
                set_error("every system needs its own x");
                return DG_ERR_ARG;
            }
    }
    if (flags & ~(DG_BATCH_HANDOFF | DG_BATCH_CONCURRENT)) {
        set_error("unknown batched-solve flags");
        return DG_ERR_ARG;
    }
    if (o.precond != DG_PC_JACOBI && o.precond != DG_PC_FDM) {
        set_error("unknown preconditioner");
        return DG_ERR_ARG;
    }
    int rc;
    if (flags & DG_BATCH_CONCURRENT) {
        // ordinary single-system solves at once on separate streams: the
        // Poisson systems with the FP64 fast-diagonalisation inverse (exact
        // for their constant coefficient), the Helmholtz systems with
        // opts.precond (Jacobi: FP64 only; fast diagonalisation: FP32
        // transforms with DG_MIXED); every x starts from zero
        if (nsys > kMaxConcurrent) {
            set_error("concurrent batched solve: at most 4 systems");
            return DG_ERR_ARG;
        }
        ConcSys sys[kMaxConcurrent];
        for (int k = 0; k < nsys; ++k) {
            const bool pois = is_poisson && is_poisson[k];
            for (int d = 0; d < 3; ++d)
                sys[k].bc[d] = pois && m->dev.bc[d] == DG_BC_DIRICHLET ? DG_BC_NEUMANN : m->dev.bc[d];
            sys[k].lambda = pois ? 0.0 : lambdas[k];
            sys[k].nu = pois || !nu_fields ? nullptr : nu_fields[k];
            sys[k].nu_c = 1.0;
            sys[k].rhs = rhs[k];
            sys[k].x = x[k];
            sys[k].weak = o.rhs_is_weak;
            sys[k].jacobi = !pois && o.precond == DG_PC_JACOBI;
            sys[k].f32 = !pois && o.precond == DG_PC_FDM && o.precision == DG_MIXED;
            if (sys[k].jacobi && o.precision != DG_FP64) {
                set_error("concurrent batched solve: the Jacobi-preconditioned systems run in FP64 only");
                return DG_ERR_ARG;
            }
        }
        for (int k = 0; k < nsys; ++k)
            if ((rc = launch_lincomb((size_t)m->dev.ndof, nullptr, 0, nullptr, nullptr, x[k], m->stream)))
                return rc;
        rc = conc_solve(m, nsys, sys, o, infos, true);
    } else {
        rc = solve_batched(m, nsys, lambdas, nu_fields, is_poisson, rhs, x, o, infos, flags);
    }
    if (infos)
        for (int k = 0; k < nsys; ++k) infos[k].seconds = now() - t0;
    return rc;
}

int helmholtz_solve_noalloc(dg_mesh *m, double lambda, const double *nu_field, double nu_const,
                            const double *rhs, double *x, const dg_solve_opts *opts,
                            dg_solve_info *info)
{
    if (int rc = check_mesh(m)) return rc;
    const size_t need = footprint(m->dev, DG_FP64);
    if (need > kScratchBytes) {
        set_error("helmholtz_solve_noalloc: this mesh needs " + std::to_string(need) +
                  " bytes of workspace; the scratch array holds " + std::to_string(kScratchBytes) +
                  " (about 3.3M nodes)");
        return DG_ERR_ARG;
    }
    void *base = nullptr;
    if (int rc = scratch_address(&base)) return rc;
    Workspace w;
    CgScalars host_sc[2];
    w.base = base;
    w.bytes = kScratchBytes;
    w.external = true;
    w.host_sc = host_sc;
    w.host_external = true;
    return solve_common(m, m->dev.bc, lambda, nu_field, nu_const, rhs, x, opts, info, &w);
}

int helmholtz_fdm_apply(dg_mesh *m, double lambda, double nu_const, int is_poisson, const double *b,
                        double *x, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    if (!b || !x || (const void *)b == (const void *)x) {
        set_error("b and x must be distinct device arrays");
        return DG_ERR_ARG;
    }
    int bc[3];
    for (int d = 0; d < 3; ++d)
        bc[d] = (is_poisson && m->dev.bc[d] == DG_BC_DIRICHLET) ? DG_BC_NEUMANN : m->dev.bc[d];
    if (is_poisson) {
        lambda = 0.0;
        nu_const = 1.0;
    }
    if (!(lambda >= 0.0) || !std::isfinite(lambda) || !(nu_const > 0.0) || !std::isfinite(nu_const)) {
        set_error("lambda must be >= 0 and nu_const > 0");
        return DG_ERR_ARG;
    }
    Workspace &w = m->ws;
    int rc = ensure_workspace(m, w, DG_FP64);
    if (rc) return rc;
    FdmDev f;
    if ((rc = ensure_fdm_tables(m, w, bc, f))) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : m->stream;
    if (s != m->stream) DG_HIP_CHECK(hipStreamSynchronize(m->stream));  // the table upload
    const bool singular = lambda == 0.0 && !has_dirichlet(bc);
    return fdm_apply(m->dev, f, lambda, nu_const, singular, b, x, w.q64, nullptr, s);
}

int dg_divergence(dg_mesh *mv, dg_mesh *mp, const double *vx, const double *vy, const double *vz,
                  const double *vbx, const double *vby, const double *vbz, double *b, void *stream)
{
    if (int rc = check_mesh(mv)) return rc;
    if (int rc = check_mesh(mp)) return rc;
    if (!vx || !vy || !vz || !b) {
        set_error("null velocity or output array");
        return DG_ERR_ARG;
    }
    const double *v[3] = {vx, vy, vz}, *vb[3] = {vbx, vby, vbz};
    hipStream_t s = stream ? (hipStream_t)stream : mv->stream;
    return launch_divergence(mv->dev, mp->dev, v, vb, 1.0, b, s);
}

int dg_gradient(dg_mesh *mv, dg_mesh *mp, const double *psi, double *gx, double *gy, double *gz,
                void *stream)
{
    if (int rc = check_mesh(mv)) return rc;
    if (int rc = check_mesh(mp)) return rc;
    if (!psi || !gx || !gy || !gz) {
        set_error("null pressure or output array");
        return DG_ERR_ARG;
    }
    double *g[3] = {gx, gy, gz};
    hipStream_t s = stream ? (hipStream_t)stream : mv->stream;
    return launch_gradient(mv->dev, mp->dev, psi, nullptr, 1.0, g, s);
}

int dg_project(dg_mesh *mv, dg_mesh *mp, double *vx, double *vy, double *vz, const double *vbx,
               const double *vby, const double *vbz, double *psi, const dg_solve_opts *opts,
               dg_solve_info *info)
{
    double *v[3] = {vx, vy, vz};
    const double *vb[3] = {vbx, vby, vbz};
    return project_impl(mv, mp, v, vb, psi, opts, info, false);
}

int dg_viscosity(dg_mesh *m, const double *vx, const double *vy, const double *vz, double nu0,
                 double nu1, double vref, double *nu, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    if (!vx || !vy || !vz || !nu || !(vref > 0.0) || !std::isfinite(nu0) || !std::isfinite(nu1)) {
        set_error("null array or bad viscosity coefficients (vref > 0)");
        return DG_ERR_ARG;
    }
    const double *v[3] = {vx, vy, vz};
    return launch_viscosity(m->dev, v, nu0, nu1, vref, nu, stream ? (hipStream_t)stream : m->stream);
}

int dg_viscous_terms(dg_mesh *m, const double *nu, const double *vx, const double *vy, const double *vz,
                     const double *vbx, const double *vby, const double *vbz, double *fd1x, double *fd1y,
                     double *fd1z, double *fd3x, double *fd3y, double *fd3z, void *stream)
{
    if (int rc = check_mesh(m)) return rc;
    if (!nu || !vx || !vy || !vz) {
        set_error("null viscosity or velocity array");
        return DG_ERR_ARG;
    }
    const MeshDev &md = m->dev;
    hipStream_t s = stream ? (hipStream_t)stream : m->stream;
    const double *v[3] = {vx, vy, vz}, *vb[3] = {vbx, vby, vbz};
    double *f1[3] = {fd1x, fd1y, fd1z}, *f3[3] = {fd3x, fd3y, fd3z};
    int rc;
    // F_d1 = div(nu grad v_d) = -M^-1 K_nu v_d (the SIP operator at lambda = 0)
    for (int d = 0; d < 3; ++d) {
        if (!f1[d]) continue;
        if ((rc = launch_apply<double>(md, md.bc, 0.0, nu, 0.0, v[d], f1[d], s))) return rc;
        if ((rc = launch_weak_to_nodal(md, f1[d], nullptr, -1.0, f1[d], s))) return rc;
    }
    // F_d3 = -grad(nu div v): w = nu M^-1 D(v; v_b) (equal order), F_d3 = -G w
    if (f3[0] || f3[1] || f3[2]) {
        if (!(f3[0] && f3[1] && f3[2])) {
            set_error("F_d3 needs all three output components");
            return DG_ERR_ARG;
        }
        if (!m->aux) {
            if (stream && s != m->stream) DG_HIP_CHECK(hipStreamSynchronize(s));
            hipError_t e = hipMalloc((void **)&m->aux, (size_t)md.ndof * sizeof(double));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                m->aux = nullptr;
                set_error("viscous-term scratch allocation failed");
                return DG_ERR_OOM;
            }
        }
        if ((rc = launch_divergence_nodal(md, v, vb, 1.0, nu, m->aux, s))) return rc;
        if ((rc = launch_gradient(md, md, m->aux, nullptr, -1.0, f3, s))) return rc;
    }
    return DG_OK;
}

int dg_lincomb(int64_t n, const double *x0, int k, const double *coef, const double *const *xs, double *y,
               void *stream)
{
    if (n < 0 || !y || k < 0 || (k > 0 && (!coef || !xs))) {
        set_error("bad linear-combination arguments");
        return DG_ERR_ARG;
    }
    for (int j = 0; j < k; ++j)
        if (!xs[j]) {
            set_error("null term in a linear combination");
            return DG_ERR_ARG;
        }
    return launch_lincomb((size_t)n, x0, k, coef, xs, y, (hipStream_t)stream);
}

int poisson_solve(dg_mesh *m, const double *rhs, double *x, const dg_solve_opts *opts,
                  dg_solve_info *info)
{
    if (int rc = check_mesh(m)) return rc;
    int bc[3];
    for (int d = 0; d < 3; ++d)
        bc[d] = m->dev.bc[d] == DG_BC_DIRICHLET ? DG_BC_NEUMANN : m->dev.bc[d];
    return solve_common(m, bc, 0.0, nullptr, 1.0, rhs, x, opts, info);
}

}  // extern "C"
