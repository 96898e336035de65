// Convective term F_c = -div(v v) with local Lax-Friedrichs fluxes (internal;
// see convection.hip for the definition).
#pragma once
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {

// out_d = scale F_c,d (or out_d += scale F_c,d when accumulate) as nodal
// fields; vb: wall state per component (null: zero)
int launch_convection(const MeshDev &m, const double *const v[3], const double *const vb[3], double scale,
                      bool accumulate, double *const out[3], hipStream_t s);

}  // namespace dg
