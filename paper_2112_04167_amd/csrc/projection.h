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
// g = G psi, or g = v - G psi when v is given (g may alias v)
int launch_gradient(const MeshDev &mv, const MeshDev &mp, const double *psi, const double *const v[3],
                    double *const g[3], hipStream_t s);

}  // namespace dg
