// Device-side CG state and kernel launchers (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

// Scalars of one CG solve, resident in device memory.  Written only by the
// one-work-group kernel that finishes a reduction (one thread), read by every
// later kernel.
struct CgScalars {
    double rho;        // r.z of the current iterate
    double rho_prev;   // r.z of the previous iterate (for a residual replacement)
    double alpha, beta;
    double pq, sumq;   // p.Ap and sum(Ap) of the current step
    double bnorm2;     // ||M^-1 b||^2
    double res2;       // ||M^-1 r||^2 (recurrence; singular: of the projected r)
    double tol2;       // tol^2 * bnorm2
    double mean_r;     // singular: mean of r removed in the p-update
    double mean_b;     // singular: mean of the load removed at set-up
    double sum_invd;   // singular: sum 1/d
    double sum_invM2;  // singular: sum 1/M^2
    double shift;      // singular: M-weighted mean of x removed at the end
    double true_res2;  // ||M^-1 (b - A x)||^2 of the last residual evaluation
    double scale;      // mixed: power-of-two scaling of the inner vectors (true = scale * stored)
    double scale_new;  // mixed: scaling chosen for the next residual replacement
    int iter, maxit, fixed_iters, done, status, singular;
    long long ndof;
    int rho_pending;   // fast-diagonalisation CG: a new r.z waits in rho_next
    int pad;
    double rho_next;   // r.z left by the p-update, made rho by the next apply's finish
};

// Device helpers called by the kernels that finish a reduction.
__device__ inline void cg_after_apply(CgScalars *sc, double pq, double sumq)
{
    if (sc->rho_pending) {  // the r.z of the p-update that precedes this apply
        sc->rho_pending = 0;
        sc->rho_prev = sc->rho;
        sc->rho = sc->rho_next;
        if (!isfinite(sc->rho)) {
            sc->status = DG_ERR_NONFINITE;
            sc->done = 1;
            return;
        }
    }
    sc->pq = pq;
    sc->sumq = sumq;
    if (!isfinite(pq)) {
        sc->status = DG_ERR_NONFINITE;
        sc->done = 1;
    } else if (pq <= 0.0) {
        sc->status = DG_ERR_NOT_SPD;
        sc->done = 1;
    } else {
        sc->alpha = sc->rho / pq;
    }
}

__device__ inline void resid_finish(CgScalars *sc, const double (&t)[4])
{
    // t = {sum (r/M)^2, sum r, sum r/M^2, sum 1/M^2}
    double res2 = t[0];
    if (sc->singular) {
        const double m = t[1] / (double)sc->ndof;
        res2 = t[0] - 2.0 * m * t[2] + m * m * t[3];
        sc->mean_r = m;
    } else {
        sc->mean_r = 0.0;
    }
    sc->true_res2 = res2 > 0.0 ? res2 : 0.0;
}

// reductions finished by a one-work-group kernel after the producer
enum { FIN_APPLY = 0, FIN_RESID, FIN_SETUP1, FIN_SETUP2, FIN_UPDATE, FIN_MEANX, FIN_IRSCALE,
       FIN_UPDATE_FDM };
int launch_finish_apply(double *partial, int nblk, CgScalars *sc, hipStream_t s);
int launch_finish_resid(double *partial, int nblk, CgScalars *sc, hipStream_t s);

template <typename T>
int launch_apply_cg(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                    const T *p, T *q, double *partial, CgScalars *sc,
                    hipStream_t s);
template <typename T>
int launch_resid(const MeshDev &m, const int bc[3], double lambda, const T *nu, double nu_c,
                 const T *x, const T *b, T *r, double *partial, CgScalars *sc,
                 hipStream_t s);
int apply_threads(int P);

// CG vector kernels (element/line mapped, FP64 reductions)
template <typename T>
struct CgVecArgs {
    T *x, *r, *p;
    const T *q, *d;
    const T *src;       // set-up: rhs (nodal f or weak b); convert: FP64 source
    T *bvec;            // set-up: the load vector b
    const double *src64;
    double *dst64;
    const T *hx, *hy, *hz;
    int n[3];
    int nel, ngroups;
    int weak;
    int keep_x;         // set-up: leave x (the caller's initial guess) as it is
    // Jacobi diagonal computed on the fly (constant nu) instead of read from d:
    // per-axis 1D terms [nx | ny | nz][P+1] (see diag_tables) and lambda
    const T *dtab;
    double lam;
    const T *z;         // FDM-PCG: the preconditioned residual
    bool singular;      // host-side: selects the singular (projected) kernels
    double *partial;
    CgScalars *sc;
};

const GllTables &gll_cached(int P);

template <typename T>
int cg_setup(const MeshDev &m, CgVecArgs<T> a, hipStream_t s);   // b, r, z, p, x = 0 (unless keep_x), norms
template <typename T>
int cg_update(const MeshDev &m, CgVecArgs<T> a, hipStream_t s);  // x, r and the new rho
template <typename T>
int cg_pupdate(const MeshDev &m, CgVecArgs<T> a, hipStream_t s); // p = z + beta p
template <typename T>
int cg_finish(const MeshDev &m, CgVecArgs<T> a, hipStream_t s);  // singular: x -= M-mean
// mixed precision (a.sc: the refinement scalars)
int convert_f64_to_f32(const double *a, float *b, size_t n, hipStream_t s);
int ir_scale(const MeshDev &m, CgVecArgs<float> a, hipStream_t s);      // sc->scale_new = 2^round(log2 RMS(src64 - mean_r))
int ir_to_inner(const MeshDev &m, CgVecArgs<float> a, hipStream_t s);   // r = (src64 - mean_r)/scale_new; scale = scale_new
int ir_accumulate(const MeshDev &m, CgVecArgs<float> a, hipStream_t s); // dst64 += scale * x
// residual replacement of the inner CG: r = (src64 - mean_r)/scale_new, x = 0,
// then (on inner) rho, beta = rho'/rho * scale_new/scale (0 if restart), the
// replacement threshold tol2 = max(delta2 ||M^-1 r||^2, outer tol2/scale_new^2),
// the inner iteration cap maxit (counted from the first inner set-up), done =
// 0; finally scale = scale_new.  Follow with cg_pupdate.
int ir_replace(const MeshDev &m, CgVecArgs<float> a, CgScalars *inner, double delta2, bool restart,
               int maxit, hipStream_t s);
// FP64 CG restarted from the residual in a.r (mean a.sc->mean_r removed if
// singular): p = r/diag, rho, residual norm; a.sc->tol2 is kept.
int cg_restart64(const MeshDev &m, CgVecArgs<double> a, hipStream_t s);

// CG preconditioned by the fast-diagonalisation inverse (FP64).  The
// residual in memory minus sc->mean_r is the (projected) residual; z = the
// preconditioned residual in a.z.
// start: after r = b - A x (launch_resid): x = 0 if b = 0, the residual norm
// and the stopping test, iteration count 0
int cg_fdm_start(const MeshDev &m, CgVecArgs<double> a, hipStream_t s);
// x += alpha p, r -= alpha q, ||M^-1 r|| and the stopping test
int cg_update_fdm(const MeshDev &m, CgVecArgs<double> a, hipStream_t s);
// per-work-group partial sums of rho' = (r - mean_r).z
int cg_rz(const MeshDev &m, CgVecArgs<double> a, hipStream_t s);
// p = z + beta p, beta = rho'/rho (start: p = z), every work-group summing
// the partials of cg_rz itself; rho' is left in rho_next for the next
// apply's finish (cg_after_apply), so no work-group reads a rho another one
// has changed
int cg_pupdate_fdm(const MeshDev &m, CgVecArgs<double> a, bool start, hipStream_t s);

}  // namespace dg
