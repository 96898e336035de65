// Projection substep kernels (internal): DG divergence of a degree-P
// velocity onto the degree-(P-1) pressure basis and DG gradient of the
// pressure onto the velocity nodes (see projection.hip for the definitions).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

// out = scale * D(v; v_b) (weak vector on the pressure basis); vb may be null
// (v_b = 0) and each vb[d] may be null (that component's boundary flux zero)
int launch_divergence(const MeshDev &mv, const MeshDev &mp, const double *const v[3],
                      const double *const vb[3], double scale, double *out, hipStream_t s);
// out = scale fac M^-1 D(v; v_b) at every node of m (equal order: the
// scalar space is the velocity space; fac a nodal factor, null: 1)
int launch_divergence_nodal(const MeshDev &m, const double *const v[3], const double *const vb[3], double scale,
                            const double *fac, double *out, hipStream_t s);
// g = scale fac G psi (fac a nodal factor of the velocity mesh, null: 1), or
// g = v + scale fac G psi when v is given (g may alias v).  mp: the pressure
// mesh (degree P-1) or, for the equal-order operators of the
// variable-viscosity terms, the velocity mesh itself
int launch_gradient(const MeshDev &mv, const MeshDev &mp, const double *psi, const double *const v[3],
                    double scale, double *const g[3], hipStream_t s, const double *fac = nullptr);
// out = s x (f or 1) / M at every node (M the GLL mass): a weak vector to a
// nodal field
int launch_weak_to_nodal(const MeshDev &m, const double *x, const double *f, double s, double *out,
                         hipStream_t st);
// out = (out or 0) + s M x at every node (a nodal field to a weak vector)
int launch_mass(const MeshDev &m, const double *x, double s, bool accumulate, double *out, hipStream_t st);
// b += scale L(g): the Nitsche load of the Dirichlet data g (nodal field,
// its values on the faces of the Dirichlet axes of bc are read) with the
// viscosity nu (nodal, or nu_c when null)
int launch_dirichlet_load(const MeshDev &m, const int bc[3], const double *nu, double nu_c, const double *g,
                          double scale, double *b, hipStream_t st);
// nu = nu0 + nu1 |v|^2 / vref^2 at every node
int launch_viscosity(const MeshDev &m, const double *const v[3], double nu0, double nu1, double vref,
                     double *nu, hipStream_t st);
// y = (x0 or 0) + sum_j c[j] xs[j], k <= 32 terms (y may alias x0)
int launch_lincomb(size_t N, const double *x0, int k, const double *c, const double *const *xs, double *y,
                   hipStream_t st);

}  // namespace dg
