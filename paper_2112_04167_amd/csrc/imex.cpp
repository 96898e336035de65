// One IMEX Runge-Kutta step for incompressible flow with variable viscosity
// (Alg. 3 of arXiv 2112.04167) with the Butcher tableaux of its App. A.
//
// The stage loop runs on the host and drives the library's kernels: the
// convective term (convection.hip), the viscous terms F_d1, F_d2, F_d3 (SIP
// apply and the equal-order DG gradient / divergence of projection.hip),
// the projection substep (dg_project) and the Helmholtz solves
// (helmholtz_solve), with the linear combinations of the stage loads as one
// kernel each.  Per stage j the step keeps only the combinations it needs,
//     C_j = F_c + F_d2 + F_d3,   D1_j = F_d1,   D3_j = F_d3,
// from which
//     v'_i = v + dt [ sum_j a^E_ij (C_j + D1_j + D3_j) + sum_j a^I_ij F_s,j ],
//     g_i  = v''_i + dt sum_j [ (a^I_ij - a^E_ij) D1_j - a^E_ij D3_j ],
//     v    = v_s + dt sum_j [ (b^E_j - a^E_sj) C_j + (b^I_j - a^I_sj)(D1_j + F_s,j) ],
// and a stage's terms are evaluated only if one of these uses them.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "convection.h"
#include "dg_internal.h"
#include "dg_sipdg.h"
#include "projection.h"
#include "trace.h"

namespace dg {
namespace {

constexpr int S8 = DG_RK_MAX_STAGES;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Rows {
    int s;
    std::vector<double> c, bI, bE;
    std::vector<std::vector<double>> aI, aE;  // ragged lower-triangular rows
};

void fill(const Rows &r, dg_tableau *t)
{
    std::memset(t, 0, sizeof(*t));
    t->s = r.s;
    for (int i = 0; i < r.s; ++i) {
        t->c[i] = r.c[i];
        t->bI[i] = r.bI[i];
        t->bE[i] = r.bE[i];
        for (size_t j = 0; j < r.aI[i].size(); ++j) t->aI[i * S8 + j] = r.aI[i][j];
        for (size_t j = 0; j < r.aE[i].size(); ++j) t->aE[i * S8 + j] = r.aE[i][j];
    }
}

// App. A, left array of each pair the implicit part, right the explicit one
Rows tableau_rows(int method)
{
    Rows r{};
    switch (method) {
        case DG_RK_TR:
            r.s = 3;
            r.c = {0, 1, 1};
            r.aI = {{0}, {0, 1}, {0.5, 0, 0.5}};
            r.bI = {0.5, 0, 0.5};
            r.aE = {{0}, {1}, {0.5, 0.5}};
            r.bE = {0.5, 0.5, 0};
            break;
        case DG_RK_CB2:
            r.s = 3;
            r.c = {0, 0.4, 1};
            r.aI = {{0}, {0, 0.4}, {0, 5.0 / 6.0, 1.0 / 6.0}};
            r.bI = {0, 5.0 / 6.0, 1.0 / 6.0};
            r.aE = {{0}, {0.4}, {0, 1}};
            r.bE = {0, 5.0 / 6.0, 1.0 / 6.0};
            break;
        case DG_RK_CB3C: {
            const double c2 = 3375509829940.0 / 4525919076317.0, c3 = 272778623835.0 / 1039454778728.0;
            const double b2 = 673488652607.0 / 2334033219546.0, b3 = 493801219040.0 / 853653026979.0,
                         b4 = 184814777513.0 / 1389668723319.0;
            r.s = 4;
            r.c = {0, c2, c3, 1};
            r.aI = {{0}, {0, c2},
                    {0, -11712383888607531889907.0 / 32694570495602105556248.0, 566138307881.0 / 912153721139.0},
                    {0, b2, b3, b4}};
            r.bI = {0, b2, b3, b4};
            r.aE = {{0}, {c2}, {0, c3}, {0, b2, 1660544566939.0 / 2334033219546.0}};
            r.bE = {0, b2, b3, b4};
            break;
        }
        case DG_RK_CB3E:
            r.s = 4;
            r.c = {0, 1.0 / 3.0, 1, 1};
            r.aI = {{0}, {0, 1.0 / 3.0}, {0, 0.5, 0.5}, {0, 0.75, -0.25, 0.5}};
            r.bI = {0, 0.75, -0.25, 0.5};
            r.aE = {{0}, {1.0 / 3.0}, {0, 1}, {0, 0.75, 0.25}};
            r.bE = {0, 0.75, -0.25, 0.5};
            break;
        case DG_RK_CB4: {
            const double p1 = 232049084587.0 / 1377130630063.0, p2 = 322009889509.0 / 2243393849156.0,
                         p3 = -195109672787.0 / 1233165545817.0;
            const std::vector<double> b = {p1, p2, p3, -340582416761.0 / 705418832319.0,
                                           463396075661.0 / 409972144477.0, 323177943294.0 / 1626646580633.0};
            r.s = 6;
            r.c = {0, 0.25, 0.75, 0.375, 0.5, 1};
            r.aI = {{0},
                    {0.125, 0.125},
                    {216145252607.0 / 961230882893.0, 257479850128.0 / 1143310606989.0,
                     30481561667.0 / 101628412017.0},
                    {p1, -381180097479.0 / 1276440792700.0, -54660926949.0 / 461115766612.0,
                     344309628413.0 / 552073727558.0},
                    {p1, p2, -100836174740.0 / 861952129159.0, -250423827953.0 / 1283875864443.0, 0.5},
                    b};
            r.bI = b;
            r.aE = {{0},
                    {0.25},
                    {153985248130.0 / 1004999853329.0, 902825336800.0 / 1512825644809.0},
                    {p1, 99316866929.0 / 820744730663.0, 82888780751.0 / 969573940619.0},
                    {p1, p2, 57501241309.0 / 765040883867.0, 76345938311.0 / 676824576433.0},
                    {p1, p2, p3, -4099309936455.0 / 6310162971841.0, 1395992540491.0 / 933264948679.0}};
            r.bE = b;
            break;
        }
        case DG_RK_ARS3:
            r.s = 5;
            r.c = {0, 0.5, 2.0 / 3.0, 0.5, 1};
            r.aI = {{0}, {0, 0.5}, {0, 1.0 / 6.0, 0.5}, {0, -0.5, 0.5, 0.5}, {0, 1.5, -1.5, 0.5, 0.5}};
            r.bI = {0, 1.5, -1.5, 0.5, 0.5};
            r.aE = {{0}, {0.5}, {11.0 / 18.0, 1.0 / 18.0}, {5.0 / 6.0, -5.0 / 6.0, 0.5}, {0.25, 1.75, 0.75, -1.75}};
            r.bE = {0.25, 1.75, 0.75, -1.75, 0};
            break;
        default:
            r.s = 0;
    }
    return r;
}

int check_tableau(const dg_tableau *t)
{
    if (!t || t->s < 2 || t->s > S8) {
        set_error("tableau: 2 <= s <= 8 stages");
        return DG_ERR_ARG;
    }
    const int s = t->s;
    bool ok = t->c[0] == 0.0 && t->aI[0] == 0.0;
    for (int i = 0; i < s && ok; ++i) {
        ok = std::isfinite(t->c[i]) && std::isfinite(t->bI[i]) && std::isfinite(t->bE[i]) && t->aI[i * S8 + i] >= 0.0;
        for (int j = 0; j < s && ok; ++j) {
            const double ai = t->aI[i * S8 + j], ae = t->aE[i * S8 + j];
            ok = std::isfinite(ai) && std::isfinite(ae) && (j < i || ae == 0.0) && (j <= i || ai == 0.0);
        }
    }
    if (!ok) {
        set_error("tableau: needs c_1 = 0, a^I_11 = 0, a^E strictly and a^I lower triangular, a^I_ii >= 0");
        return DG_ERR_ARG;
    }
    return DG_OK;
}

// F_d2 = M^-1 D(nu (d_i v_0, d_i v_1, d_i v_2)) per component i: T[3k + i]
// = nu d_i v_k by the equal-order gradient with a nodal factor, then the
// equal-order divergence with the field's own trace as boundary data
int fd2_terms(const MeshDev &md, const double *nu, const double *const v[3], double *T, double *const out[3],
              hipStream_t s)
{
    const size_t N = (size_t)md.ndof;
    int rc;
    for (int k = 0; k < 3; ++k) {
        double *g[3] = {T + (3 * k) * N, T + (3 * k + 1) * N, T + (3 * k + 2) * N};
        if ((rc = launch_gradient(md, md, v[k], nullptr, 1.0, g, s, nu))) return rc;
    }
    for (int i = 0; i < 3; ++i) {
        const double *w[3] = {T + (size_t)i * N, T + (size_t)(3 + i) * N, T + (size_t)(6 + i) * N};
        if ((rc = launch_divergence_nodal(md, w, w, 1.0, nullptr, out[i], s))) return rc;
    }
    return DG_OK;
}

// F_d1 = -M^-1 (K_nu v - L_nu(v_b)) per component: the SIP operator at
// lambda = 0 with the wall data v_b (null: zero) as its Dirichlet data
int fd1_terms(const MeshDev &md, const double *nu, const double *const v[3], const double *const vb[3],
              double *const out[3], hipStream_t s)
{
    int rc;
    for (int d = 0; d < 3; ++d) {
        if ((rc = launch_apply<double>(md, md.bc, 0.0, nu, 0.0, v[d], out[d], s))) return rc;
        if (vb && vb[d] && (rc = launch_dirichlet_load(md, md.bc, nu, 0.0, vb[d], -1.0, out[d], s))) return rc;
        if ((rc = launch_weak_to_nodal(md, out[d], nullptr, -1.0, out[d], s))) return rc;
    }
    return DG_OK;
}

// F_d3 = -G(nu M^-1 D(v; v_b)), equal order; w: scratch for the nodal
// field nu M^-1 D(v; v_b)
int fd3_terms(const MeshDev &md, const double *nu, const double *const v[3], const double *const vb[3],
              double *w, double *const out[3], hipStream_t s)
{
    int rc;
    if ((rc = launch_divergence_nodal(md, v, vb, 1.0, nu, w, s))) return rc;
    return launch_gradient(md, md, w, nullptr, -1.0, out, s);
}

// the events a step orders its streams with (destroyed with the object)
struct StepEvents {
    hipEvent_t e[3] = {};
    int create()
    {
        for (hipEvent_t &x : e)
            if (hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) {
                x = nullptr;
                set_error("event creation failed");
                return DG_ERR_DEVICE;
            }
        return DG_OK;
    }
    ~StepEvents()
    {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" {

int dg_imex_tableau(int method, dg_tableau *out)
{
    if (!out) {
        set_error("null tableau");
        return DG_ERR_ARG;
    }
    const Rows r = tableau_rows(method);
    if (r.s == 0) {
        set_error("unknown IMEX-RK method");
        return DG_ERR_ARG;
    }
    fill(r, out);
    return DG_OK;
}

int dg_dirichlet_load(dg_mesh *m, const double *nu_field, double nu_const, const double *g, double scale,
                      double *b, void *stream)
{
    const MeshDev *md = mesh_device(m);
    if (!md || !g || !b || (const void *)g == (const void *)b) {
        set_error("null mesh, data or load array, or data aliasing the load");
        return DG_ERR_ARG;
    }
    if (!nu_field && !(nu_const > 0.0 && std::isfinite(nu_const))) {
        set_error("nu_const must be > 0 without a nodal viscosity");
        return DG_ERR_ARG;
    }
    return launch_dirichlet_load(*md, md->bc, nu_field, nu_const, g, scale, b,
                                 stream ? (hipStream_t)stream : mesh_stream(m));
}

int dg_convection(dg_mesh *m, const double *vx, const double *vy, const double *vz, const double *vbx,
                  const double *vby, const double *vbz, double scale, int accumulate, double *ox, double *oy,
                  double *oz, void *stream)
{
    const MeshDev *md = mesh_device(m);
    if (!md || !vx || !vy || !vz || !ox || !oy || !oz) {
        set_error("null mesh, velocity or output array");
        return DG_ERR_ARG;
    }
    const double *v[3] = {vx, vy, vz}, *vb[3] = {vbx, vby, vbz};
    double *o[3] = {ox, oy, oz};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if ((const void *)o[a] == (const void *)v[b]) {
                set_error("convection outputs must not alias the velocity");
                return DG_ERR_ARG;
            }
    return launch_convection(*md, v, vb, scale, accumulate != 0, o, stream ? (hipStream_t)stream : mesh_stream(m));
}

int dg_viscous_fd2(dg_mesh *m, const double *nu, const double *vx, const double *vy, const double *vz,
                   double *ox, double *oy, double *oz, void *stream)
{
    const MeshDev *md = mesh_device(m);
    if (!md || !nu || !vx || !vy || !vz || !ox || !oy || !oz) {
        set_error("null mesh, viscosity, velocity or output array");
        return DG_ERR_ARG;
    }
    const size_t N = (size_t)md->ndof;
    hipStream_t s = stream ? (hipStream_t)stream : mesh_stream(m);
    if (stream && s != mesh_stream(m)) DG_HIP_CHECK(hipStreamSynchronize(s));  // a buffer swap frees
    double *buf = mesh_step_buffer(m, 9 * N);
    if (!buf) return DG_ERR_OOM;
    const double *v[3] = {vx, vy, vz};
    double *o[3] = {ox, oy, oz};
    return fd2_terms(*md, nu, v, buf, o, s);
}

int dg_imex_step(dg_mesh *mv, dg_mesh *mp, const dg_tableau *tab, double dt, double nu0, double nu1,
                 double vref, double *vx, double *vy, double *vz, const double *const *forcing,
                 const double *const *wall, int final_projection, const dg_solve_opts *opts, dg_step_info *info)
{
    const double t0 = now_s();
    TraceRange tr("dg_imex_step");
    dg_step_info st{};
    const MeshDev *mdp = mesh_device(mv);
    if (!mdp || !mesh_device(mp) || !vx || !vy || !vz) {
        set_error("null mesh or velocity array");
        return DG_ERR_ARG;
    }
    if (int rc = check_tableau(tab)) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt) || !(vref > 0.0) || !std::isfinite(nu0) || !std::isfinite(nu1)) {
        set_error("dt > 0, vref > 0 and finite viscosity coefficients required");
        return DG_ERR_ARG;
    }
    const MeshDev &md = *mdp;
    if (md.P < 4 || mesh_device(mp)->P != md.P - 1) {
        set_error("the step needs a velocity degree 4..8 and a pressure mesh of degree P-1");
        return DG_ERR_ARG;
    }
    const int s = tab->s;
    auto aI = [&](int i, int j) { return tab->aI[i * S8 + j]; };
    auto aE = [&](int i, int j) { return tab->aE[i * S8 + j]; };
    // which terms of stage j the step uses
    std::vector<char> needC(s, 0), needD1(s, 0);
    for (int j = 0; j < s; ++j) {
        for (int i = j + 1; i < s; ++i) {
            if (aE(i, j) != 0.0) needC[j] = needD1[j] = 1;
            if (aI(i, j) != 0.0) needD1[j] = 1;
        }
        if (tab->bE[j] - aE(s - 1, j) != 0.0) needC[j] = 1;
        if (tab->bI[j] - aI(s - 1, j) != 0.0) needD1[j] = 1;
    }
    // workspace: stage velocity (3N), nu (N), F_d2 scratch and the three
    // Helmholtz loads (9N), the nodal scratch of F_d3 (N), per used
    // stage C, D1, D3 (9N), the pressure (Np)
    const size_t N = (size_t)md.ndof, Np = (size_t)mesh_device(mp)->ndof;
    std::vector<int> slot(s, -1);
    int nslots = 0;
    for (int j = 0; j < s; ++j)
        if (needC[j] || needD1[j]) slot[j] = nslots++;
    double *buf = mesh_step_buffer(mv, (14 + 9 * (size_t)nslots) * N + Np);
    if (!buf) return DG_ERR_OOM;
    double *Vi[3] = {buf, buf + N, buf + 2 * N};
    double *nu = buf + 3 * N, *T = buf + 4 * N, *w3 = buf + 13 * N;
    double *terms = buf + 14 * N, *psi = terms + 9 * (size_t)nslots * N;
    auto C = [&](int j, int d) { return terms + ((size_t)slot[j] * 9 + d) * N; };
    auto D1 = [&](int j, int d) { return terms + ((size_t)slot[j] * 9 + 3 + d) * N; };
    auto D3 = [&](int j, int d) { return terms + ((size_t)slot[j] * 9 + 6 + d) * N; };
    auto Fs = [&](int j, int d) -> const double * { return forcing ? forcing[3 * j + d] : nullptr; };
    // wall data of stage j (null: no-slip walls)
    bool has_dirichlet = false;
    for (int d = 0; d < 3; ++d) has_dirichlet = has_dirichlet || md.bc[d] == DG_BC_DIRICHLET;
    auto walls = [&](int j, const double *out[3]) -> const double *const * {
        for (int d = 0; d < 3; ++d) out[d] = wall ? wall[3 * j + d] : nullptr;
        return (wall && (out[0] || out[1] || out[2])) ? out : nullptr;
    };
    double *V0[3] = {vx, vy, vz};
    hipStream_t sv = mesh_stream(mv);
    dg_solve_opts o;
    dg_default_opts(&o);
    if (opts) o = *opts;
    o.rhs_is_weak = 0;
    if (!(o.tol > 0.0) || o.maxit < 0 || (o.precision != DG_FP64 && o.precision != DG_MIXED) ||
        (o.precond != DG_PC_JACOBI && o.precond != DG_PC_FDM)) {
        set_error("bad solver options");
        return DG_ERR_ARG;
    }
    // the pressure solves: with the fast-diagonalisation preconditioner always
    // its FP64 transforms, which are exact for the constant-coefficient
    // Poisson problem (one iteration); DG_MIXED then applies to the velocity
    // solves only (FP32 transforms for their variable-nu operator)
    dg_solve_opts op = o;
    if (op.precond == DG_PC_FDM) op.precision = DG_FP64;
    int rc;

    // A stage's three groups of terms are independent: F_d1 runs on the first
    // extra stream, F_d3 (with its own scratch) on the second, F_d2 and F_c
    // on the mesh's stream, which then waits for the other two.
    hipStream_t alt[kMaxConcurrent - 1] = {};
    if ((rc = mesh_concurrent_streams(alt))) return rc;
    StepEvents ev;
    if ((rc = ev.create())) return rc;
    auto stage_terms = [&](int j, const double *const v[3]) -> int {
        TraceRange tj("imex: stage terms");
        int r;
        const double *wb[3];
        const double *const *vb = walls(j, wb);
        DG_HIP_CHECK(hipEventRecord(ev.e[0], sv));
        DG_HIP_CHECK(hipStreamWaitEvent(alt[0], ev.e[0], 0));
        DG_HIP_CHECK(hipStreamWaitEvent(alt[1], ev.e[0], 0));
        if (needD1[j]) {
            double *out[3] = {D1(j, 0), D1(j, 1), D1(j, 2)};
            if ((r = fd1_terms(md, nu, v, vb, out, alt[0]))) return r;
        }
        double *c3[3] = {nullptr, nullptr, nullptr}, *d3[3] = {nullptr, nullptr, nullptr};
        if (needC[j]) {
            for (int d = 0; d < 3; ++d) {
                c3[d] = C(j, d);
                d3[d] = D3(j, d);
            }
            if ((r = fd3_terms(md, nu, v, vb, w3, d3, alt[1]))) return r;
            if ((r = fd2_terms(md, nu, v, T, c3, sv))) return r;
            if ((r = launch_convection(md, v, vb, 1.0, true, c3, sv))) return r;
        }
        DG_HIP_CHECK(hipEventRecord(ev.e[1], alt[0]));
        DG_HIP_CHECK(hipEventRecord(ev.e[2], alt[1]));
        DG_HIP_CHECK(hipStreamWaitEvent(sv, ev.e[1], 0));
        DG_HIP_CHECK(hipStreamWaitEvent(sv, ev.e[2], 0));
        if (needC[j])
            for (int d = 0; d < 3; ++d) {
                const double one = 1.0;
                const double *x = d3[d];
                if ((r = launch_lincomb(N, c3[d], 1, &one, &x, c3[d], sv))) return r;
            }
        return DG_OK;
    };
    // the projection with the wall data vb (null: v_b = 0), or with the
    // velocity's own trace (d_n psi = 0) for the final projection
    auto project = [&](double *const v[3], const double *const *vb, bool own_trace) -> int {
        if (int r = launch_lincomb(Np, nullptr, 0, nullptr, nullptr, psi, sv)) return r;  // psi = 0
        dg_solve_info pi{};
        const double *b3[3] = {nullptr, nullptr, nullptr};
        for (int d = 0; d < 3; ++d) b3[d] = own_trace ? v[d] : (vb ? vb[d] : nullptr);
        const int r = project_impl(mv, mp, v, b3, psi, &op, &pi, true);
        if (r < 0) return r;
        st.solves += 1;
        st.pressure_iters += pi.iters;
        if (r > st.status) st.status = r;
        return DG_OK;
    };

    // stage 1: v_1 = v, nu_1 = nu(v)
    if ((rc = launch_viscosity(md, V0, nu0, nu1, vref, nu, sv))) return rc;
    if ((rc = stage_terms(0, V0))) return rc;
    std::vector<double> coef;
    std::vector<const double *> xs;
    for (int i = 1; i < s; ++i) {
        // predictor v'_i
        for (int d = 0; d < 3; ++d) {
            coef.clear();
            xs.clear();
            for (int j = 0; j < i; ++j) {
                if (aE(i, j) == 0.0) continue;
                for (const double *x : {C(j, d), D1(j, d), D3(j, d)}) {
                    coef.push_back(dt * aE(i, j));
                    xs.push_back(x);
                }
            }
            for (int j = 0; j <= i; ++j)
                if (aI(i, j) != 0.0 && Fs(j, d)) {
                    coef.push_back(dt * aI(i, j));
                    xs.push_back(Fs(j, d));
                }
            if ((rc = launch_lincomb(N, V0[d], (int)coef.size(), coef.data(), xs.data(), Vi[d], sv))) return rc;
        }
        // projection, viscosity at the projected velocity
        const double *wb[3];
        const double *const *vbi = walls(i, wb);
        if ((rc = project(Vi, vbi, false))) return rc;
        if ((rc = launch_viscosity(md, Vi, nu0, nu1, vref, nu, sv))) return rc;
        // load and Helmholtz solve per component.  The three loads go to
        // the F_d2 scratch T (free until this stage's terms), and with the
        // fast-diagonalisation preconditioner the three solves, which share
        // their operator, run at once on separate streams.
        const double aii = aI(i, i);
        const double lam = aii > 0.0 ? 1.0 / (dt * aii) : 1.0;
        double *Gd[3] = {T, T + N, T + 2 * N};
        int weakd[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            coef.clear();
            xs.clear();
            coef.push_back(lam);
            xs.push_back(Vi[d]);
            for (int j = 0; j < i; ++j) {
                const double c1 = dt * (aI(i, j) - aE(i, j)), c3 = -dt * aE(i, j);
                if (c1 != 0.0) {
                    coef.push_back(lam * c1);
                    xs.push_back(D1(j, d));
                }
                if (c3 != 0.0) {
                    coef.push_back(lam * c3);
                    xs.push_back(D3(j, d));
                }
            }
            if (aii > 0.0) {
                if ((rc = launch_lincomb(N, nullptr, (int)coef.size(), coef.data(), xs.data(), Gd[d], sv)))
                    return rc;
                if (has_dirichlet && vbi && vbi[d]) {
                    // weak load M (lambda g) + L_nu(v_b): the wall data as Dirichlet data
                    if ((rc = launch_mass(md, Gd[d], 1.0, false, Gd[d], sv))) return rc;
                    if ((rc = launch_dirichlet_load(md, md.bc, nu, 0.0, vbi[d], 1.0, Gd[d], sv))) return rc;
                    weakd[d] = 1;
                }
            } else {  // no implicit term in this stage: v_i = g_i
                if ((rc = launch_lincomb(N, Vi[d], (int)coef.size() - 1, coef.data() + 1, xs.data() + 1, Vi[d], sv)))
                    return rc;
            }
        }
        if (aii > 0.0) {
            TraceRange ts("imex: velocity solves");
            dg_solve_info hi[3] = {};
            if (o.precond == DG_PC_FDM) {
                // (the step reports no true residuals: no final b - A x)
                rc = solve_fdm_concurrent(mv, 3, lam, nu, 0.0, Gd, Vi, weakd, o, hi, false);
                if (rc < 0) return rc;
                if (rc > st.status) st.status = rc;
            } else {
                for (int d = 0; d < 3; ++d) {
                    dg_solve_opts od = o;
                    od.rhs_is_weak = weakd[d];
                    rc = helmholtz_solve(mv, lam, nu, 0.0, Gd[d], Vi[d], &od, &hi[d]);
                    if (rc < 0) return rc;
                    if (rc > st.status) st.status = rc;
                }
            }
            for (int d = 0; d < 3; ++d) {
                st.solves += 1;
                st.velocity_iters += hi[d].iters;
                if (hi[d].status > st.status) st.status = hi[d].status;
            }
        }
        if ((rc = stage_terms(i, Vi))) return rc;
    }
    // assembly: v = v_s + dt sum_j [(bE_j - aE_sj) C_j + (bI_j - aI_sj)(D1_j + F_s,j)]
    for (int d = 0; d < 3; ++d) {
        coef.clear();
        xs.clear();
        for (int j = 0; j < s; ++j) {
            const double ce = dt * (tab->bE[j] - aE(s - 1, j)), ci = dt * (tab->bI[j] - aI(s - 1, j));
            if (ce != 0.0) {
                coef.push_back(ce);
                xs.push_back(C(j, d));
            }
            if (ci != 0.0) {
                coef.push_back(ci);
                xs.push_back(D1(j, d));
                if (Fs(j, d)) {
                    coef.push_back(ci);
                    xs.push_back(Fs(j, d));
                }
            }
        }
        if ((rc = launch_lincomb(N, Vi[d], (int)coef.size(), coef.data(), xs.data(), V0[d], sv))) return rc;
    }
    if (final_projection && (rc = project(V0, nullptr, true))) return rc;
    {
        TraceRange tw("imex: wait for the device");
        DG_HIP_CHECK(hipStreamSynchronize(sv));
    }
    st.seconds = now_s() - t0;
    if (info) *info = st;
    return st.status;
}

}  // extern "C"
