"""Variable-viscosity terms of the implicit stage (oracle).

Test infrastructure only (see the package docstring).

Alg. 3 of arXiv 2112.04167 splits the viscous term of the momentum equation
as F_d = F_d1 + F_d2 + F_d3 with

    F_d1 = div(nu grad v),   F_d2 = div(nu (grad v)^T),   F_d3 = -grad(nu div v),

evaluates the viscosity at the projected velocity of each stage, nu_i =
nu(v''_i), and forms the load of the stage's Helmholtz problems from the
earlier stages' F_d1 and F_d3:

    g_i = v''_i + dt sum_{j<i} [ (a^I_ij - a^E_ij) F_d1,j - a^E_ij F_d3,j ].

The viscosity model of the variable-viscosity test cases (Sec. 4) is
nu(v) = nu_0 + nu_1 (|v| / v_ref)^2.

Discretisation (the reading written out in the build's design notes):
  * F_d1 per component: the nodal field -M^-1 (A_nu v - L_nu(v_b)) with
    A_nu the SIP operator of the Helmholtz solves at lambda = 0 and the
    nodal nu, L_nu the Nitsche load of the wall data v_b on the Dirichlet
    axes (zero when v_b is not given);
  * F_d3: w = nu M^-1 D(v; v_b) with D the weak DG divergence of the
    projection substep taken on the velocity basis itself (equal order),
    then F_d3 = -G w with G the matching DG gradient (minus the adjoint of
    D(.; 0) under the GLL mass).
"""
import numpy as np

from . import dense, naive, projection


def viscosity(v, nu0, nu1, vref):
    """nu = nu_0 + nu_1 (|v| / v_ref)^2 at every node."""
    s = sum(np.asarray(c, dtype=np.float64) ** 2 for c in v)
    return nu0 + nu1 * s / (vref * vref)


def fd1(spec, nu, v, vb=None):
    """div(nu grad v_d) for each component, as nodal fields: -M^-1 (K_nu v_d
    - L_nu(v_b,d)), the wall data v_b (None: zero) as the Dirichlet data of
    the SIP form (dense.dirichlet_load)."""
    M = dense.mass_diag(spec)
    op = naive.Operator(spec, 0.0, nu)
    out = []
    for d, c in enumerate(v):
        y = op.apply(np.asarray(c, dtype=np.float64))
        if vb is not None and vb[d] is not None:
            y = y - dense.dirichlet_load(spec, nu, vb[d])
        out.append(-y / M)
    return out


def fd3(spec, nu, v, vb=None):
    """-grad(nu div v) as three nodal fields (equal-order DG divergence and
    gradient)."""
    P = spec["P"]
    M = dense.mass_diag(spec)
    w = np.asarray(nu, dtype=np.float64) * projection.divergence(spec, v, vb, q_degree=P) / M
    g = projection.gradient(spec, w, q_degree=P)
    return [-c for c in g]


def stage_load(vpp, fd1s, fd3s, dt, aI, aE):
    """g_i = v''_i + dt sum_j [(aI_j - aE_j) F_d1,j - aE_j F_d3,j] per component."""
    out = []
    for d in range(3):
        g = np.array(vpp[d], dtype=np.float64)
        for j in range(len(fd1s)):
            g = g + dt * (aI[j] - aE[j]) * fd1s[j][d] - dt * aE[j] * fd3s[j][d]
        out.append(g)
    return out
