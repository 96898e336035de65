/*
 * dg_sipdg.h -- C-ABI of the MI355X SIP-DG Helmholtz / Poisson library.
 *
 * The library solves the implicit sub-problems of the IMEX Runge-Kutta / SDC
 * projection schemes of arXiv 2112.04167 (Alg. 3 and Alg. 4):
 *
 *   Helmholtz (diffusion substep, one per velocity component):
 *       v - dt a_ii div(nu grad v) = g   ->   lambda u - div(nu grad u) = f,
 *       lambda = 1/(dt a_ii), f = lambda g, homogeneous Dirichlet data;
 *   Poisson (projection substep):
 *       lap(psi) = div(v')  with Neumann data  ->  lambda = 0, nu = 1.
 *
 * Discretisation (Sec. 3.3): hexahedral elements, tensor-product Lagrange
 * polynomials of degree P on GLL points, DG-SEM with the symmetric interior
 * penalty method.  All integrals use the (P+1)-point GLL rule, so the mass
 * matrix M is diagonal.  The discrete operator is A = lambda M + K_nu:
 *
 *   a(u,v) = sum_K int_K (nu grad u.grad v + lambda u v)
 *          + sum_F int_F (-{nu d_n u}[v] - {nu d_n v}[u] + sigma [u][v]),
 *   sigma  = max(nu_L, nu_R) (P+1)^2 / min(h_L, h_R)  at every face node,
 *
 * h being the element extent normal to the face; a Dirichlet face uses the
 * interior trace, the outward normal and sigma = nu (P+1)^2 / h; a Neumann
 * face adds nothing; periodic axes wrap around.
 *
 * Stopping rule (Sec. 4: relative RMS residual at the collocation points):
 *   || M^-1 (b - A x) ||_2 <= tol || M^-1 b ||_2   with b = M f.
 *
 * Meshes are Cartesian products of 1D vertex arrays (uniform or graded).
 *
 * ---------------------------------------------------------------- layout --
 * Every nodal array (x, y, rhs, nu_field) is element-major: node (a,b,c) of
 * element (ex,ey,ez) is at
 *     ((ez*ny + ey)*nx + ex)*(P+1)^3 + (c*(P+1) + b)*(P+1) + a,
 * its coordinates are x = xv[ex] + (xv[ex+1]-xv[ex]) (1 + xi_a)/2 (likewise
 * y, z), xi the GLL nodes on [-1,1].
 *
 * ------------------------------------------------------------- ownership --
 * The caller owns every device array passed in (rhs, x, y, nu_field); the
 * library never frees them.  The library owns the mesh handle, its geometry
 * and its solver workspace (allocated at the first solve, grown on demand,
 * freed by dg_mesh_destroy).  All work is enqueued on the mesh's HIP stream
 * (or the stream passed to helmholtz_apply); the *_solve calls return after
 * the result is known (they synchronise that stream).
 *
 * ---------------------------------------------------------------- errors --
 * Every call returns a status: 0 = DG_OK, > 0 a warning, < 0 an error, and
 * never throws across the ABI.  dg_last_error() returns a thread-local text
 * for the last error.  On an error the contents of output arrays are
 * unspecified; on DG_NOT_CONVERGED x holds the last iterate and info is set.
 * A mesh handle must not be used by two threads at once.
 */
#ifndef DG_SIPDG_H
#define DG_SIPDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DG_OK = 0,
    DG_NOT_CONVERGED = 1,
    DG_ERR_ARG = -1,
    DG_ERR_OOM = -2,
    DG_ERR_DEVICE = -3,
    DG_ERR_NOT_SPD = -4,     /* p^T A p <= 0 met in CG */
    DG_ERR_NONFINITE = -5,   /* NaN / Inf in the data or in a CG scalar */
    DG_ERR_BUDGET = -6       /* request larger than the server's HBM budget */
};

enum { DG_BC_PERIODIC = 0, DG_BC_DIRICHLET = 1, DG_BC_NEUMANN = 2 };  /* per axis */
enum { DG_FP64 = 0, DG_FP32 = 1, DG_MIXED = 1 };  /* apply: FP32 data; solve: FP32 inner + FP64 IR */
/* preconditioner of the CG solves:
   DG_PC_JACOBI  diag(A) (point Jacobi);
   DG_PC_FDM     the fast-diagonalisation inverse of the constant-nu operator
                 on the Cartesian mesh (see helmholtz_fdm_apply): exact for a
                 constant nu, so CG stops after one or two steps; with a nodal
                 nu field it uses nu_ref = sqrt(min nu max nu), and CG then
                 converges at a rate set by max nu / min nu.  Needs at most
                 512 nodes per mesh line (n_d (P+1) <= 512).  With precision
                 DG_FP64 the transforms are FP64; with DG_MIXED they are FP32
                 (FP32 matrices, MFMA arithmetic and intermediates, at twice
                 the FP64 matrix rate) while CG stays FP64 with the same
                 stopping test: the preconditioner is then no longer exact,
                 and a constant-nu solve takes a few iterations. */
enum { DG_PC_JACOBI = 0, DG_PC_FDM = 1 };

typedef struct dg_mesh dg_mesh;  /* opaque */

typedef struct {
    double tol;         /* relative collocation residual (default 1e-10) */
    int maxit;          /* CG iteration cap (FP64) / cap on FP64 residual replacements (mixed) */
    int precision;      /* DG_FP64 or DG_MIXED */
    double inner_tol;   /* mixed: the FP32 CG recurrence residual is replaced by the FP64
                           residual b - A x once it has dropped by this factor since the
                           last replacement (or claims convergence) */
    int inner_maxit;    /* mixed (and batched): cap on FP32 CG iterations in total */
    int rhs_is_weak;    /* 0: rhs is the nodal f (b = M f); 1: rhs is b itself */
    int fixed_iters;    /* > 0: run exactly this many CG iterations, no stopping test */
    int precond;        /* DG_PC_JACOBI (default) or DG_PC_FDM */
} dg_solve_opts;

typedef struct {
    int iters;            /* CG iterations (mixed: FP32 iterations, plus FP64 iterations if the
                             solve continued in FP64 because the FP32 cycles stalled) */
    int outer_iters;      /* mixed: FP64 residual evaluations (replacements); 0 in FP64 mode */
    int status;
    double rel_res;       /* recurrence residual at exit (FP64: CG recurrence) */
    double true_rel_res;  /* || M^-1 (b - A x) || / || M^-1 b || recomputed from x */
    double seconds;       /* host wall time of the call */
} dg_solve_info;

/* Default options: tol 1e-10, maxit 100000, FP64, inner_tol 1e-2,
   inner_maxit 20000, nodal rhs, no fixed iteration count, Jacobi. */
void dg_default_opts(dg_solve_opts *opts);

/* Create a Cartesian mesh of nx*ny*nz hexahedra of degree P (3 <= P <= 8;
   fewer than 2^31 nodes in all) from host vertex arrays xv[nx+1],
   yv[ny+1], zv[nz+1] (strictly increasing), with per-axis boundary
   conditions bc[3] (DG_BC_*).  The element extents and GLL tables are
   copied to the device.  hip_stream: the HIP stream the mesh's work goes to
   (NULL = default stream).  Returns DG_ERR_ARG on bad sizes or vertices. */
int dg_mesh_create(int nx, int ny, int nz, int P, const double *xv, const double *yv,
                   const double *zv, const int bc[3], void *hip_stream, dg_mesh **out);
int dg_mesh_destroy(dg_mesh *m);
int64_t dg_mesh_ndof(const dg_mesh *m);                      /* E (P+1)^3 */
/* Nodal coordinates (the GLL nodes mapped to every element) in the ABI
   layout: device double arrays X, Y, Z of dg_mesh_ndof values each (any of
   them may be NULL).  Asynchronous on `stream` (NULL = the mesh's stream). */
int dg_mesh_coordinates(dg_mesh *m, double *X, double *Y, double *Z, void *stream);
/* Bytes of device workspace a solve allocates (for admission control).
   nrhs = 1: helmholtz_solve / poisson_solve; nrhs > 1: helmholtz_solve_batched
   with nsys = nrhs systems.  A mesh keeps the largest workspace it has
   needed (per kind) until dg_mesh_destroy; a batched solve with
   DG_BATCH_HANDOFF may also allocate that of nrhs = 1 (the continuation). */
size_t dg_solve_footprint(const dg_mesh *m, int precision, int nrhs);

/* y = (lambda M + K_nu) x  -- the matrix-free, sum-factorised SIP-DG apply
   (the Helmholtz operator of Alg. 3's diffusion solve; lambda = 0 gives the
   Laplacian of the projection solve, with the mesh's own BCs).
   x, y: device arrays of dg_mesh_ndof values, double (DG_FP64) or float
   (DG_FP32), x != y.  nu_field: device nodal viscosity of the same type, or
   NULL for the constant nu_const (> 0).  stream: HIP stream (NULL = the
   mesh's stream).  Asynchronous: returns once the kernel is enqueued.
   Performance only: in FP64 at P = 3 and 7, 16-byte-aligned x, y and
   nu_field (as hipMalloc and torch return them) take a faster path of wide
   loads and stores; any other alignment is accepted and gives the same y. */
int helmholtz_apply(dg_mesh *m, double lambda, const void *nu_field, double nu_const,
                    const void *x, void *y, int precision, void *stream);

/* d = diag(lambda M + K_nu), same argument conventions as helmholtz_apply
   (the Jacobi preconditioner). */
int helmholtz_diag(dg_mesh *m, double lambda, const void *nu_field, double nu_const, void *d,
                   int precision, void *stream);

/* x = (lambda M + nu K)^-1 b for a constant nu, by fast diagonalisation
   (Lynch, Rice & Thomas 1964): on the Cartesian product mesh the operator is
   the Kronecker sum lambda Mz(x)My(x)Mx + nu (Mz(x)My(x)Kx + Mz(x)Ky(x)Mx +
   Kz(x)My(x)Mx) of the 1D SIP matrices K_d and GLL masses M_d of the axes
   (Sec. 3.3: every volume and face integral of the GLL-collocated form
   factorises), so with K_d S_d = M_d S_d Lam_d, S_d^T M_d S_d = I,
       x = (Sz(x)Sy(x)Sx) (lambda + nu (Lx (+) Ly (+) Lz))^-1 (Sz(x)Sy(x)Sx)^T b.
   The three 1D transforms each way run as FP64 matrix-core (MFMA)
   contractions along the mesh lines; the 1D eigenproblems are solved on the
   host at first use and cached.  b, x: device double arrays (ABI layout),
   b the weak load vector (b = M f), x != b.  is_poisson: lambda = 0, nu = 1
   and the mesh's Dirichlet axes become Neumann axes, as in poisson_solve.  If
   the operator is singular (lambda = 0, no Dirichlet axis) the constant mode
   is dropped: pass b with zero sum; x then has zero M-weighted mean.
   Uses the mesh's workspace (allocated on first use).  Asynchronous on
   `stream` (NULL = the mesh's stream).  DG_ERR_ARG if a mesh line has more
   than 512 nodes. */
int helmholtz_fdm_apply(dg_mesh *m, double lambda, double nu_const, int is_poisson,
                        const double *b, double *x, void *stream);

/* Solve (lambda M + K_nu) x = b by Jacobi-preconditioned CG (FP64), or by
   FP64 iterative refinement around FP32 Jacobi-PCG inner solves (DG_MIXED;
   FP64 residuals, updates and dot products).  lambda >= 0; nu_field: device
   double nodal viscosity or NULL for nu_const.  rhs: device double, the
   nodal f (b = M f) unless opts->rhs_is_weak.  x: device double, in: the
   initial guess (the solve starts from r = b - A x; pass zeros for none),
   out: the solution (if b = 0, x = 0 whatever the guess).  The stopping test
   stays relative to ||M^-1 b||.  If lambda = 0 and the mesh has no Dirichlet axis
   the problem is singular: b is projected to mean zero and x is returned
   with M-weighted mean zero.  opts may be NULL (defaults), info may be NULL. */
int helmholtz_solve(dg_mesh *m, double lambda, const double *nu_field, double nu_const,
                    const double *rhs, double *x, const dg_solve_opts *opts, dg_solve_info *info);

/* helmholtz_solve for callers that cannot allocate device memory: code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
   The same FP64 Jacobi-PCG (opts->precision must be DG_FP64, else
   DG_ERR_ARG), with every solver buffer (CG vectors, reduction slots, device
   scalars, diagonal tables) taken from a static device array of 128 MiB that
   the library holds on each GPU it runs on until the process ends; no
   hipMalloc, hipFree or other allocating call is made.  Meshes whose FP64
   solve workspace (dg_solve_footprint(m, DG_FP64, 1)) exceeds 128 MiB -- about
   3.3M nodes -- are refused with DG_ERR_ARG.  Every call on a GPU shares that
   GPU's array: calls that overlap on one GPU (two threads, or two streams
   before the first call has returned) race and give wrong results.  Nothing
   in the array needs clearing between calls (the solve initialises what it
   reads).  Arguments, results and statuses as in helmholtz_solve; the
   result is bitwise that of helmholtz_solve in FP64. */
int helmholtz_solve_noalloc(dg_mesh *m, double lambda, const double *nu_field, double nu_const,
                            const double *rhs, double *x, const dg_solve_opts *opts,
                            dg_solve_info *info);

/* The pressure Poisson problem of the projection substep (Alg. 3): lambda = 0,
   nu = 1, and every Dirichlet axis of the mesh becomes a natural Neumann
   axis (the pressure carries Neumann data).  The system is then singular
   (constants): rhs is projected, x is returned with M-weighted mean zero.
   rhs, x (in: initial guess, out: solution), opts and info as in
   helmholtz_solve. */
int poisson_solve(dg_mesh *m, const double *rhs, double *x, const dg_solve_opts *opts,
                  dg_solve_info *info);

/* ------------------------------------------------------ projection --
 * The projection substep of Alg. 3: with the predicted velocity v' (degree
 * P, three nodal components) and the boundary velocity v_b,
 *     solve  lap(psi) = div v',  d_n psi = n.(v' - v_b) on the boundary;
 *     v'' = v' - grad psi,
 * the pressure psi at degree P-1 (Sec. 3.3).  Discretisation (DG, all
 * integrals by the (P+1)-point GLL rule of the velocity, exact here):
 *   D(v; v_b)_q = - sum_K int_K v.grad q + sum_F(interior) int_F {v}.n [q]
 *                 + sum_F(boundary) int_F (v_b.n_out) q        (weak divergence),
 *   (G psi, w)  = sum_K int_K grad psi.w - sum_F(interior) int_F [psi] n.{w},
 * so G is minus the adjoint of D(.; 0) under the GLL masses; the pressure
 * problem is the SIP Poisson problem of degree P-1 with natural boundaries
 * (poisson_solve on the pressure mesh) with the load -D(v'; v_b): the
 * Neumann data n.(v' - v_b) is folded into it.
 * mv: velocity mesh, degree P = 4..8; mp: pressure mesh with the same
 * elements, vertices and BCs and degree P-1 (DG_ERR_ARG otherwise).  All
 * arrays are device doubles in the ABI layout of their mesh. */

/* b = D(v; v_b), a weak vector on the pressure basis.  vbx, vby, vbz: the
   boundary velocity components as nodal velocity fields (only their values
   on boundary faces are read), or NULL for v_b = 0.  Asynchronous on
   `stream` (NULL = the velocity mesh's stream). */
int dg_divergence(dg_mesh *mv, dg_mesh *mp, const double *vx, const double *vy, const double *vz,
                  const double *vbx, const double *vby, const double *vbz, double *b, void *stream);
/* (gx, gy, gz) = G psi at the velocity nodes (nodal values: the derivative of
   the pressure interpolant minus the lifted face jumps).  Asynchronous. */
int dg_gradient(dg_mesh *mv, dg_mesh *mp, const double *psi, double *gx, double *gy, double *gz,
                void *stream);
/* The substep: load -D(v'; v_b), poisson_solve on mp (opts as there, e.g.
   precond DG_PC_FDM; the load is weak), v <- v - G psi in place.  psi: in,
   the initial guess of the pressure solve (zeros, or the previous stage's
   psi); out, the pressure (M-weighted mean zero).  info: that of the
   pressure solve, seconds for the whole substep.  Allocates one pressure
   vector on mp at first use (freed with mp); synchronises mp's stream. */
int dg_project(dg_mesh *mv, dg_mesh *mp, double *vx, double *vy, double *vz, const double *vbx,
               const double *vby, const double *vbz, double *psi, const dg_solve_opts *opts,
               dg_solve_info *info);

/* ------------------------------------------- variable viscosity terms --
 * The variable-viscosity part of an implicit stage (Alg. 3): the viscosity
 * at the projected velocity, nu_i = nu(v''_i), and the explicit terms
 *     F_d1 = div(nu grad v),   F_d3 = -grad(nu div v)
 * that the stage's Helmholtz load takes from the earlier stages:
 *     g_i = v''_i + dt sum_{j<i} [ (a^I_ij - a^E_ij) F_d1,j - a^E_ij F_d3,j ].
 * Discretisation: F_d1 per component is the nodal field -M^-1 K_nu v with
 * K_nu the SIP operator of the Helmholtz solves at lambda = 0 (nodal nu, the
 * mesh's BCs: homogeneous Dirichlet data on Dirichlet axes); F_d3 = -G w,
 * w = nu M^-1 D(v; v_b), with D and G the divergence and gradient of the
 * projection substep taken on the velocity basis itself (equal order). */

/* nu = nu0 + nu1 (|v| / vref)^2 at every node (the viscosity model of the
   variable-viscosity test cases, Sec. 4).  vref > 0.  Asynchronous. */
int dg_viscosity(dg_mesh *m, const double *vx, const double *vy, const double *vz, double nu0,
                 double nu1, double vref, double *nu, void *stream);
/* F_d1 (fd1x, fd1y, fd1z) and F_d3 (fd3x, fd3y, fd3z) of the velocity v with
   the nodal viscosity nu; either triple may be all NULL to skip that term.
   vbx, vby, vbz: boundary velocity for the divergence in F_d3, or NULL
   (v_b = 0).  Allocates one scratch vector on m at the first F_d3 (freed
   with m).  Asynchronous on `stream` (NULL = the mesh's stream). */
int dg_viscous_terms(dg_mesh *m, const double *nu, const double *vx, const double *vy, const double *vz,
                     const double *vbx, const double *vby, const double *vbz, double *fd1x, double *fd1y,
                     double *fd1z, double *fd3x, double *fd3y, double *fd3z, void *stream);
/* y = x0 + sum_{j<k} coef[j] xs[j] over n device doubles (x0 may be NULL:
   zero; y may be x0); k <= 32; coef and xs are host arrays.  For the stage
   load g_i above.  Asynchronous on `stream` (NULL = the default stream). */
int dg_lincomb(int64_t n, const double *x0, int k, const double *coef, const double *const *xs, double *y,
               void *stream);

/* --------------------------------------------- the full IMEX-RK step --
 * Alg. 3 of arXiv 2112.04167 for incompressible flow with the viscosity
 * nu(v) = nu0 + nu1 (|v| / vref)^2, with the explicit terms
 *     F_c = -div(v v),  F_d2 = div(nu (grad v)^T),  F_d3 = -grad(nu div v),
 * the implicit F_d1 = div(nu grad v), and the forcing F_s = f.  Stage 1 is
 * v_1 = v, nu_1 = nu(v); stage i = 2..s:
 *   v'_i  = v + dt [ sum_{j<i} a^E_ij (F_c + F_d + F_d3)_j + sum_{j<=i} a^I_ij F_s,j ]
 *   v''_i = projection of v'_i (dg_project with v_b = 0, pressure at P-1)
 *   nu_i  = nu(v''_i)
 *   g_i   = v''_i + dt sum_{j<i} [ (a^I_ij - a^E_ij) F_d1,j - a^E_ij F_d3,j ]
 *   v_i   = solution of v_i - dt a^I_ii div(nu_i grad v_i) = g_i (walls: v = 0)
 * and the step ends with
 *   v <- v_s + dt sum_i [ (b^E_i - a^E_si)(F_c + F_d2 + F_d3)_i + (b^I_i - a^I_si)(F_d1 + F_s)_i ]
 * (terms with vanishing factors are not evaluated), then, if asked, a final
 * projection with d_n psi = 0.
 * Discretisation: F_c by DG-SEM with local Lax-Friedrichs fluxes, the
 * integrals by floor(3P/2)+1 Gauss points per direction ("consistent
 * integration", Sec. 3.3): for each element K with outward normal n,
 *   (M F_c,i)_phi = int_K sum_k v_k v_i d_k phi - int_dK H_i phi,
 *   H_i = ((v-.n) v-_i + (v+.n) v+_i)/2 + alpha (v-_i - v+_i)/2,
 *   alpha = 2 max(|v-.n|, |v+.n|),
 * v+ the neighbour's trace or, on a wall, v_b (zero when not given); M the
 * GLL mass.  F_d2,i = M^-1 D(nu (d_i v_0, d_i v_1, d_i v_2)) with the
 * equal-order D and G of dg_viscous_terms (d_i v_k the i-th component of
 * G v_k; the field's own trace as its boundary data).  Walls carry the
 * caller's v_b at the stage times (zero when not given), imposed in the
 * Helmholtz solves by the Nitsche load of dg_dirichlet_load. */

enum { DG_RK_TR = 0, DG_RK_CB2 = 1, DG_RK_CB3C = 2, DG_RK_CB3E = 3, DG_RK_CB4 = 4, DG_RK_ARS3 = 5 };
#define DG_RK_MAX_STAGES 8

/* An IMEX Runge-Kutta tableau: s stages (2 <= s <= 8), abscissae c[s]
   shared by both parts, implicit aI and explicit aE (row-major s x s in
   8 x 8 arrays: a[i][j] at [i * 8 + j]), weights bI, bE.  The step needs
   c[0] = 0, a first stage without implicit term (aI[0][0] = 0), aE strictly
   lower triangular and aI lower triangular with aI[i][i] >= 0. */
typedef struct {
    int s;
    double c[DG_RK_MAX_STAGES];
    double aI[DG_RK_MAX_STAGES * DG_RK_MAX_STAGES], bI[DG_RK_MAX_STAGES];
    double aE[DG_RK_MAX_STAGES * DG_RK_MAX_STAGES], bE[DG_RK_MAX_STAGES];
} dg_tableau;

/* The tableaux of App. A: RK-TR (3 stages, order 2), RK-CB2 (3, 2),
   RK-CB3c (4, 3), RK-CB3e (4, 3), RK-CB4 (6, 4) and RK-ARS3 (5, 3; Ascher,
   Ruuth & Spiteri's (4,4,3)).  DG_ERR_ARG for an unknown method. */
int dg_imex_tableau(int method, dg_tableau *out);

typedef struct {
    int status;          /* worst status of the step's solves (DG_OK or DG_NOT_CONVERGED) */
    int solves;          /* pressure + velocity solves run */
    int pressure_iters;  /* CG iterations over the projections */
    int velocity_iters;  /* CG iterations over the Helmholtz solves */
    double seconds;      /* host wall time of the step */
} dg_step_info;

/* b += scale L(g): inhomogeneous Dirichlet data g for the SIP Helmholtz
   problem (Alg. 3: the velocity solves take v_i = v_b on the walls).  With
   n the outward normal of each face F of the mesh's Dirichlet axes and
   sigma = nu (P+1)^2 / h as in the operator, L(g)_i = sum_F int_F
   (sigma g phi_i - nu d_n(phi_i) g), by the GLL rule: solving
   (lambda M + K_nu) x = M f + L(g) (helmholtz_solve with rhs_is_weak) gives
   the discrete solution with x = g on those faces.  g: nodal field (only its
   values on the Dirichlet faces are read); nu_field: nodal viscosity or
   NULL for nu_const (> 0); b: weak vector, g != b.  Asynchronous on
   `stream` (NULL = the mesh's stream). */
int dg_dirichlet_load(dg_mesh *m, const double *nu_field, double nu_const, const double *g, double scale,
                      double *b, void *stream);
/* (ox, oy, oz) = scale F_c(v), or += scale F_c(v) when accumulate, as nodal
   fields.  vbx, vby, vbz: the wall state (only boundary-face values read),
   or NULL (zero).  Degree 3..8.  Asynchronous on `stream` (NULL = the mesh's
   stream); the outputs must not alias v. */
int dg_convection(dg_mesh *m, const double *vx, const double *vy, const double *vz, const double *vbx,
                  const double *vby, const double *vbz, double scale, int accumulate, double *ox, double *oy,
                  double *oz, void *stream);
/* (ox, oy, oz) = F_d2(v) with the nodal viscosity nu.  Allocates nine scratch
   vectors on m at first use (the mesh's step workspace, freed with m).
   Asynchronous on `stream` (NULL = the mesh's stream); outputs must not
   alias v or nu. */
int dg_viscous_fd2(dg_mesh *m, const double *nu, const double *vx, const double *vy, const double *vz,
                   double *ox, double *oy, double *oz, void *stream);
/* One step of size dt > 0 in place on (vx, vy, vz) (device, velocity mesh
   mv of degree 4..8; mp its pressure mesh of degree P-1, as for dg_project).
   forcing: NULL (no forcing) or a host array of 3 s device pointers,
   forcing[3 j + d] the d-th component of f(t + c_j dt) (each may be NULL:
   zero).  wall: NULL (no-slip walls) or a host array of 3 s device pointers,
   wall[3 j + d] a nodal velocity field whose values on the faces of the
   Dirichlet axes are v_b(t + c_j dt) (each may be NULL: zero); stage j uses
   it as the Dirichlet data of its Helmholtz solves (dg_dirichlet_load),
   in F_d1, in the projection's Neumann data and F_d3's divergence, and as
   the exterior state of the convective flux.  final_projection: 1 to end
   with the projection with d_n psi = 0 (for variable viscosity).  opts: the
   options of every pressure and velocity solve (NULL: defaults; DG_PC_FDM
   recommended; the velocity solves start from v''_i).  With DG_PC_FDM the
   pressure solves always use the FP64 transforms (exact for the constant-
   coefficient Poisson problem), and precision DG_MIXED selects the FP32
   transforms for the velocity solves only.  With DG_PC_FDM the
   three velocity solves of a stage, which share their operator, run at once
   on the mesh's stream and two more streams (non-blocking, default
   priority; one pair per device, shared by all meshes, created at first use
   and kept until the process ends), each with its own FP64 solve workspace
   (created at first use and kept with the mesh).  Allocates
   the mesh's step workspace (about (9 s' + 14) N doubles, s' the stages
   whose terms the tableau uses) at first use; synchronous.  Returns the
   first error of a kernel or solve, else info->status. */
int dg_imex_step(dg_mesh *mv, dg_mesh *mp, const dg_tableau *tab, double dt, double nu0, double nu1,
                 double vref, double *vx, double *vy, double *vz, const double *const *forcing,
                 const double *const *wall, int final_projection, const dg_solve_opts *opts,
                 dg_step_info *info);

/* nsys systems on one mesh, solved together in one persistent, cooperative
   launch: the 3 velocity Helmholtz problems and the pressure Poisson problem
   of one implicit stage (Alg. 3).  Each system runs Jacobi-PCG with its own
   scalars, stopping test and retirement; with DG_MIXED the recurrence is
   FP32 with FP64 residual replacement (as in helmholtz_solve), with DG_FP64
   it is FP64 throughout.  lambdas[i], nu_fields[i] (device double nodal or
   NULL for nu = 1), is_poisson[i] (1: lambda ignored, Poisson as in
   poisson_solve), rhs[i], x[i] (device double, output only: the batched
   solve starts every system from zero).  infos[nsys] may be
   NULL.  nsys <= 8.  The launch shape (resident work-groups per CU) is
   autotuned per (device, P, precision, nsys, mesh size) on first use.
   Returns the worst status over the systems; DG_ERR_DEVICE if the device
   cannot run cooperative launches or a grid-barrier wait timed out. */
int helmholtz_solve_batched(dg_mesh *m, int nsys, const double *lambdas,
                            const double *const *nu_fields, const int *is_poisson,
                            const double *const *rhs, double *const *x,
                            const dg_solve_opts *opts, dg_solve_info *infos);

/* helmholtz_solve_batched with flags.  DG_BATCH_HANDOFF: once a single system
   is left unconverged (the others have retired), the persistent launch ends
   and that system is finished by the single-system solver (helmholtz_solve /
   poisson_solve with the same options), starting from its current solution.
   With one system left, ordinary kernel launches cost less per iteration
   than the launch's two grid barriers.  The system's info then counts the
   iterations and replacements of both parts.  DG_BATCH_CONCURRENT (nsys <=
   4): no persistent launch; the systems run as ordinary single-system
   solves at once, the first on the mesh's stream and the others on extra
   streams (one set per device shared by all meshes, non-blocking, default
   priority, kept until the process ends), each with an FP64 solve
   workspace of its own (kept with the mesh).  Poisson systems use the FP64
   fast-diagonalisation preconditioner (exact for their constant
   coefficient); the others use opts.precond: DG_PC_JACOBI runs FP64
   Jacobi-PCG (DG_ERR_ARG with DG_MIXED), DG_PC_FDM runs FDM-PCG with FP64
   or, for DG_MIXED, FP32 transforms.  Each system gets the result of the
   corresponding single-system solve started from zero, bit for bit.
   flags = 0 is helmholtz_solve_batched. */
enum { DG_BATCH_HANDOFF = 1, DG_BATCH_CONCURRENT = 2 };
int helmholtz_solve_batched_ex(dg_mesh *m, int nsys, const double *lambdas,
                               const double *const *nu_fields, const int *is_poisson,
                               const double *const *rhs, double *const *x,
                               const dg_solve_opts *opts, dg_solve_info *infos, int flags);

/* ------------------------------------------------------------- serving --
 * A request server for the implicit-stage solves: solves of different mesh
 * sizes, degrees and lambda arrive at any time.  A request is admitted when
 * its device footprint (mesh geometry, right-hand side, solution and solver
 * workspace, all carved from one device arena of hbm_budget_bytes) fits
 * next to the solves already running and a slot is free (strict arrival
 * order).  Admitted solves run concurrently, each on its own HIP stream
 * driven by its own host thread, so new work is admitted while older work
 * is still on the device (continuous batching).  All solve state stays on
 * the device; results stay there until fetched.
 *
 * Each request is a cube [0,1]^3 of n^3 elements, all axes periodic, nu = 1,
 * solved to the collocation-residual tolerance `tol` (Sec. 4). */
typedef struct {
    int n;              /* n^3 elements, 1 <= n */
    int P;              /* degree, 3..8 */
    int is_poisson;     /* 1: pressure Poisson problem (lambda = 0, singular) */
    double lambda;      /* Helmholtz lambda > 0 (ignored for Poisson) */
    const double *rhs;  /* host nodal f (n^3 (P+1)^3 values, copied at submit),
                           or NULL: f ~ U[-1,1] generated on the device from
                           rhs_seed with SplitMix64 (Steele, Lea & Flood 2014):
                           f_i = 2 (z_i >> 11) / 2^53 - 1, z_i the (i+1)-th
                           output of SplitMix64 started from rhs_seed */
    uint64_t rhs_seed;
    double tol;         /* relative collocation residual, e.g. 1e-10 */
    int precision;      /* DG_FP64 or DG_MIXED */
    int keep_result;    /* 1: keep x on the device until dg_server_fetch;
                           0: drop it at completion (only the info is kept).
                           Kept results occupy the arena: a queued request
                           that does not fit while no solve is running and no
                           fetch is in progress fails with DG_ERR_BUDGET
                           instead of waiting for a fetch */
    int precond;        /* DG_PC_JACOBI or DG_PC_FDM (FP64 precision only) */
} dg_request;

/* max_slots: solves allowed on the device at once (>= 1). */
int dg_server_create(size_t hbm_budget_bytes, int max_slots, void **srv);
/* Non-blocking.  Returns the request id; DG_ERR_BUDGET if the request can
   never fit the arena, DG_ERR_ARG on bad fields. */
int dg_server_submit(void *srv, const dg_request *req, int64_t *req_id);
/* DG_PENDING (2) while queued or running; otherwise the solve's status
   (DG_OK, DG_NOT_CONVERGED or an error) and *info. */
int dg_server_poll(void *srv, int64_t req_id, dg_solve_info *info);
/* Copy a finished, kept result (n^3 (P+1)^3 doubles) to host memory and
   release its device memory.  DG_PENDING if not finished yet. */
int dg_server_fetch(void *srv, int64_t req_id, double *x_host);
/* Block until every submitted request has finished (or failed: see
   keep_result; drain never waits on a fetch). */
int dg_server_drain(void *srv);
/* Statistics of finished requests; latency = completion - submission. */
typedef struct {
    int64_t completed;
    double p50, p99, mean, max;  /* latency, seconds */
    double makespan;             /* first submission -> last completion, s */
    double peak_bytes;           /* largest arena use */
    int peak_active;             /* largest number of solves on the device */
} dg_server_stats;
int dg_server_get_stats(void *srv, dg_server_stats *st);
/* Waits for running solves, then frees everything. */
int dg_server_destroy(void *srv);

enum { DG_PENDING = 2 };

const char *dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
