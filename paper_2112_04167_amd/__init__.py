"""MI355X-native SIP-DG Helmholtz / Poisson solver (implicit-stage solve of
the IMEX Runge-Kutta / SDC projection schemes of arXiv 2112.04167).

The compute path is the HIP library built from csrc/ (see include/dg_sipdg.h);
this package only marshals arguments to it.
"""
from .binding import (DG_BC_DIRICHLET, DG_BC_NEUMANN, DG_BC_PERIODIC, DG_ERR_ARG,  # noqa: F401
                      DG_ERR_BUDGET, DG_ERR_DEVICE, DG_ERR_NONFINITE, DG_ERR_NOT_SPD, DG_ERR_OOM,
                      DG_FP32, DG_FP64, DG_MIXED, DG_NOT_CONVERGED, DG_OK, DG_PC_FDM, DG_PC_JACOBI,
                      DG_PENDING, DG_RK_ARS3, DG_RK_CB2, DG_RK_CB3C, DG_RK_CB3E, DG_RK_CB4, DG_RK_TR,
                      DGError, RK_METHODS, dg_convection, dg_dirichlet_load, dg_imex_step, dg_viscous_fd2, imex_tableau,
                      Mesh, Server, default_opts, dg_divergence, dg_gradient, dg_lincomb, dg_mesh_create,
                      dg_project, dg_viscosity, dg_viscous_terms,
                      exported_symbols,
                      helmholtz_apply, helmholtz_diag, helmholtz_fdm_apply, helmholtz_solve, helmholtz_solve_batched,
                      helmholtz_solve_noalloc,
                      last_error, lib, mesh_coordinates, mesh_from_spec, poisson_solve)
