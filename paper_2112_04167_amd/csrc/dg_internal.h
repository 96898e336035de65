// Internal declarations of the SIP-DG library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dg_sipdg.h"

namespace dg {

constexpr int kMaxN = 9;  // P <= 8
constexpr int kMinPKernel = 3;
constexpr int kMaxPKernel = 8;

// thread-local error text behind dg_last_error()
void set_error(const std::string &msg);

#define DG_HIP_CHECK(expr)                                                        \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) {                                                   \
            ::dg::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));   \
            return DG_ERR_DEVICE;                                                 \
        }                                                                         \
    } while (0)

// 1D GLL tables of degree P (host, FP64), computed from their definitions.
struct GllTables {
    int P = 0;
    std::vector<double> xi, w, D;  // D row-major (i, j) = l_j'(xi_i)
    std::vector<double> K1;        // D^T diag(w) D (1D stiffness on [-1,1] without the 2/h factor)
};
GllTables make_gll(int P);
const GllTables &gll_cached(int P);  // one table per P for the process

// Geometry / BC description the kernels read (device pointers).
template <typename T>
struct Geo {
    const T *h[3];   // element extents per axis (device)
    const T *ih[3];  // their reciprocals
    int n[3];        // elements per axis
    int bc[3];       // DG_BC_* per axis (after any Poisson BC mapping)
};

struct MeshDev {
    int n[3];
    int P;
    int bc[3];
    int64_t nel, ndof;
    std::vector<double> v[3];  // host vertices
    double *h64 = nullptr;     // device: hx | hy | hz
    float *h32 = nullptr;
    double *ih64 = nullptr;    // device: 1/hx | 1/hy | 1/hz
    float *ih32 = nullptr;
    int *order = nullptr;      // device: apply work-group -> element group (see apply_order)
};

// Order in which the apply visits its element groups: position k of the
// sequence (after the XCD remap of the block id) -> element group.  The x-y
// plane is cut into 8 patches, one per XCD, and every patch is swept plane by
// plane in z, so that a group's z-neighbours were loaded shortly before and
// stay in the XCD's L2.
std::vector<int> apply_order(const int n[3], int P);

// Internal mesh / workspace entry points used by the request server.
int mesh_create_impl(int nx, int ny, int nz, int P, const double *xv, const double *yv,
                     const double *zv, const int bc[3], void *hip_stream, void *geo_mem,
                     dg_mesh **out);
size_t mesh_geo_bytes(const int n[3], int P);
size_t solve_footprint_for(const int n[3], int P, int precision);
void mesh_lend_workspace(dg_mesh *m, void *dev, size_t bytes, void *host_sc);
size_t solve_host_scalar_bytes();
int64_t mesh_ndof(const dg_mesh *m);

// --- kernel launchers (kernels.hip) ----------------------------------------
// y = A x; T = double or float; nu == nullptr -> constant nu_c.
template <typename T>
int launch_apply(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                 const T *x, T *y, hipStream_t s);
// d = diag(A), or 1/diag(A) when inverse (the Jacobi preconditioner)
template <typename T>
int launch_diag(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c, T *d,
                hipStream_t s, bool inverse = false);
int apply_groups(int P, int64_t nel);  // number of work-groups of the apply grid

// Mesh accessors for the step driver (solver.cpp): device description,
// stream, and a grow-only device buffer of at least `doubles` values owned by
// the mesh (freed with it; null and the error text set on failure).
const MeshDev *mesh_device(dg_mesh *m);
hipStream_t mesh_stream(dg_mesh *m);
double *mesh_step_buffer(dg_mesh *m, size_t doubles);

// Up to kMaxConcurrent FP64 CG solves preconditioned by fast diagonalisation,
// of one Helmholtz operator (lambda, nu field or nu_c, the mesh's BCs) with
// different right-hand sides rhs[k] (weak[k]: a weak load) and initial
// guesses / solutions x[k], run at once on separate streams from this
// thread (solver.cpp).  The first runs on the mesh's stream; the others
// start after the work enqueued there so far.  Returns when all have ended,
// with the worst status; info[k] per solve.  Options are not checked here.
// true_resid = false: no final b - A x (info true_rel_res = rel_res).
// The projection substep as dg_project does it; step_mode: no final b - A x
// in the pressure solve, and no wait for the device at the end when both
// meshes share a stream (solver.cpp).
int project_impl(dg_mesh *mv, dg_mesh *mp, double *const v[3], const double *const vb[3], double *psi,
                 const dg_solve_opts *opts, dg_solve_info *info, bool step_mode);
constexpr int kMaxConcurrent = 4;
// the two extra streams of the concurrent solves (one pair per device,
// shared by all meshes, created on first use; solver.cpp)
int mesh_concurrent_streams(hipStream_t out[kMaxConcurrent - 1]);
int solve_fdm_concurrent(dg_mesh *m, int nsys, double lambda, const double *nu, double nu_c,
                         const double *const *rhs, double *const *x, const int *weak,
                         const dg_solve_opts &o, dg_solve_info *info, bool true_resid = true);

}  // namespace dg
