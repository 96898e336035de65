"""IMEX Runge-Kutta step for incompressible flow with variable viscosity
(oracle of Alg. 3 of arXiv 2112.04167, with the Butcher tableaux of its
App. A).

Test infrastructure only (see the package docstring).

One step from v at time t of size dt with an s-stage tableau (a^E, b^E)
explicit / (a^I, b^I) implicit sharing the abscissae c (c_1 = 0):

  stage 1:  v_1 = v, nu_1 = nu(v);
  stage i = 2..s:
    v'_i  = v + dt [ sum_{j<i} a^E_ij (F_c,j + F_d,j + F_d3,j) + sum_{j<=i} a^I_ij F_s,j ]
    psi   : lap(psi) = div v'_i,  d_n psi = n.(v'_i - v_b)      (projection)
    v''_i = v'_i - grad psi
    nu_i  = nu(v''_i)
    g_i   = v''_i + dt sum_{j<i} [ (a^I_ij - a^E_ij) F_d1,j - a^E_ij F_d3,j ]
    v_i   : v_i - dt a^I_ii div(nu_i grad v_i) = g_i,  v_i = v_b on walls
  update:   v <- v_s + dt sum_i [ (b^E_i - a^E_si)(F_c,i + F_d2,i + F_d3,i)
                                 + (b^I_i - a^I_si)(F_d1,i + F_s,i) ]
  optional final projection with d_n psi = 0,

where F_d = F_d1 + F_d2 + F_d3 and every term of stage j is evaluated at
(v_j, nu_j), the forcing F_s,j = f(t + c_j dt).  The wall velocity of stage
j, v_b(t + c_j dt) (zero when not given), is the Dirichlet data of the
stage's Helmholtz problems and of F_d1 (dense.dirichlet_load), the Neumann
data of its projection, the boundary data of F_d3's divergence and the
exterior state of the convective flux.

The tableaux are transcribed from App. A as exact fractions (the left array
of each pair is the implicit part).  Terms are evaluated at every stage
(no skipping of vanishing coefficients: that is the GPU path's business).
"""
from fractions import Fraction as Fr

import numpy as np

from . import convection, dense, naive, pcg, projection, viscous


def _tab(c, AI, bI, AE, bE):
    s = len(c)

    def full(rows):
        A = [[Fr(0)] * s for _ in range(s)]
        for i, r in enumerate(rows):
            for j, x in enumerate(r):
                A[i][j] = Fr(x)
        return A

    return dict(s=s, c=[Fr(x) for x in c], AI=full(AI), bI=[Fr(x) for x in bI],
                AE=full(AE), bE=[Fr(x) for x in bE])


_CB3c_c2 = Fr(3375509829940, 4525919076317)
_CB3c_c3 = Fr(272778623835, 1039454778728)
_CB3c_b = [0, Fr(673488652607, 2334033219546), Fr(493801219040, 853653026979),
           Fr(184814777513, 1389668723319)]
_CB4_b = [Fr(232049084587, 1377130630063), Fr(322009889509, 2243393849156),
          Fr(-195109672787, 1233165545817), Fr(-340582416761, 705418832319),
          Fr(463396075661, 409972144477), Fr(323177943294, 1626646580633)]

TABLEAUX = {
    "RK-TR": _tab([0, 1, 1],
                  [[0], [0, 1], [Fr(1, 2), 0, Fr(1, 2)]], [Fr(1, 2), 0, Fr(1, 2)],
                  [[0], [1, 0], [Fr(1, 2), Fr(1, 2), 0]], [Fr(1, 2), Fr(1, 2), 0]),
    "RK-CB2": _tab([0, Fr(2, 5), 1],
                   [[0], [0, Fr(2, 5)], [0, Fr(5, 6), Fr(1, 6)]], [0, Fr(5, 6), Fr(1, 6)],
                   [[0], [Fr(2, 5), 0], [0, 1, 0]], [0, Fr(5, 6), Fr(1, 6)]),
    "RK-CB3c": _tab([0, _CB3c_c2, _CB3c_c3, 1],
                    [[0], [0, _CB3c_c2],
                     [0, Fr(-11712383888607531889907, 32694570495602105556248), Fr(566138307881, 912153721139)],
                     _CB3c_b], _CB3c_b,
                    [[0], [_CB3c_c2], [0, _CB3c_c3],
                     [0, Fr(673488652607, 2334033219546), Fr(1660544566939, 2334033219546)]], _CB3c_b),
    "RK-CB3e": _tab([0, Fr(1, 3), 1, 1],
                    [[0], [0, Fr(1, 3)], [0, Fr(1, 2), Fr(1, 2)], [0, Fr(3, 4), Fr(-1, 4), Fr(1, 2)]],
                    [0, Fr(3, 4), Fr(-1, 4), Fr(1, 2)],
                    [[0], [Fr(1, 3)], [0, 1], [0, Fr(3, 4), Fr(1, 4)]],
                    [0, Fr(3, 4), Fr(-1, 4), Fr(1, 2)]),
    "RK-CB4": _tab([0, Fr(1, 4), Fr(3, 4), Fr(3, 8), Fr(1, 2), 1],
                   [[0], [Fr(1, 8), Fr(1, 8)],
                    [Fr(216145252607, 961230882893), Fr(257479850128, 1143310606989),
                     Fr(30481561667, 101628412017)],
                    [Fr(232049084587, 1377130630063), Fr(-381180097479, 1276440792700),
                     Fr(-54660926949, 461115766612), Fr(344309628413, 552073727558)],
                    [Fr(232049084587, 1377130630063), Fr(322009889509, 2243393849156),
                     Fr(-100836174740, 861952129159), Fr(-250423827953, 1283875864443), Fr(1, 2)],
                    _CB4_b], _CB4_b,
                   [[0], [Fr(1, 4)],
                    [Fr(153985248130, 1004999853329), Fr(902825336800, 1512825644809)],
                    [Fr(232049084587, 1377130630063), Fr(99316866929, 820744730663),
                     Fr(82888780751, 969573940619)],
                    [Fr(232049084587, 1377130630063), Fr(322009889509, 2243393849156),
                     Fr(57501241309, 765040883867), Fr(76345938311, 676824576433)],
                    [Fr(232049084587, 1377130630063), Fr(322009889509, 2243393849156),
                     Fr(-195109672787, 1233165545817), Fr(-4099309936455, 6310162971841),
                     Fr(1395992540491, 933264948679)]], _CB4_b),
    "RK-ARS3": _tab([0, Fr(1, 2), Fr(2, 3), Fr(1, 2), 1],
                    [[0], [0, Fr(1, 2)], [0, Fr(1, 6), Fr(1, 2)], [0, Fr(-1, 2), Fr(1, 2), Fr(1, 2)],
                     [0, Fr(3, 2), Fr(-3, 2), Fr(1, 2), Fr(1, 2)]],
                    [0, Fr(3, 2), Fr(-3, 2), Fr(1, 2), Fr(1, 2)],
                    [[0], [Fr(1, 2)], [Fr(11, 18), Fr(1, 18)], [Fr(5, 6), Fr(-5, 6), Fr(1, 2)],
                     [Fr(1, 4), Fr(7, 4), Fr(3, 4), Fr(-7, 4)]],
                    [Fr(1, 4), Fr(7, 4), Fr(3, 4), Fr(-7, 4), 0]),
}

# stages and order of each method (Table 1)
ORDER = {"RK-TR": 2, "RK-CB2": 2, "RK-CB3c": 3, "RK-CB3e": 3, "RK-CB4": 4, "RK-ARS3": 3}


def as_float(tab):
    """The tableau as float arrays: (c, AI, bI, AE, bE)."""
    f = lambda x: np.array(x, dtype=np.float64)
    return (f([float(x) for x in tab["c"]]), f([[float(x) for x in r] for r in tab["AI"]]),
            f([float(x) for x in tab["bI"]]), f([[float(x) for x in r] for r in tab["AE"]]),
            f([float(x) for x in tab["bE"]]))


def helmholtz_solve(spec, lam, nu, rhs_nodal, solver="pcg", tol=1e-14, g_wall=None):
    """u with lambda M u + K_nu u = M rhs + L_nu(g_wall): the wall data
    g_wall (None: zero) as Dirichlet data on the Dirichlet axes."""
    M = dense.mass_diag(spec)
    b = M * rhs_nodal
    if g_wall is not None:
        b = b + dense.dirichlet_load(spec, nu, g_wall)
    if solver == "dense":
        A = dense.assemble(spec, lam, nu)
        return dense.solve(spec, A, b, lam)
    op = naive.Operator(spec, lam, nu)
    x, info = pcg.pcg(op.apply, b, op.diag(), M, tol=tol)
    assert info["status"] == pcg.OK, info
    return x


def step(spec, v, t, dt, tab, nu0, nu1, vref, forcing=None, final_projection=False, solver="pcg", wall=None):
    """One IMEX-RK step (Alg. 3).  v: three nodal arrays (velocity, degree
    P); forcing, wall: t -> three nodal arrays (the forcing; the wall
    velocity v_b, read on the Dirichlet faces), or None (zero);
    nu = nu0 + nu1 |v|^2/vref^2.  Returns (v_new, info) with the per-stage
    quantities in info."""
    c, AI, bI, AE, bE = as_float(tab)
    s = len(c)
    v = [np.asarray(x, dtype=np.float64) for x in v]
    zero = [np.zeros_like(v[0]) for _ in range(3)]
    Fs = [forcing(t + c[j] * dt) if forcing is not None else zero for j in range(s)]
    Vb = [wall(t + c[j] * dt) if wall is not None else None for j in range(s)]
    Fc, Fd1, Fd2, Fd3 = [None] * s, [None] * s, [None] * s, [None] * s

    def terms(j, vj, nuj):
        Fc[j] = convection.convection(spec, vj, Vb[j])
        Fd1[j] = viscous.fd1(spec, nuj, vj, Vb[j])
        Fd2[j] = convection.fd2(spec, nuj, vj)
        Fd3[j] = viscous.fd3(spec, nuj, vj, Vb[j])

    stage_v = [v]
    terms(0, v, viscous.viscosity(v, nu0, nu1, vref))
    for i in range(1, s):
        vp = []
        for d in range(3):
            acc = np.zeros_like(v[0])
            for j in range(i):
                acc += AE[i, j] * (Fc[j][d] + (Fd1[j][d] + Fd2[j][d] + Fd3[j][d]) + Fd3[j][d])
            for j in range(i + 1):
                acc += AI[i, j] * Fs[j][d]
            vp.append(v[d] + dt * acc)
        vpp, _ = projection.project(spec, vp, Vb[i])
        nui = viscous.viscosity(vpp, nu0, nu1, vref)
        vi = []
        for d in range(3):
            g = vpp[d].copy()
            for j in range(i):
                g += dt * ((AI[i, j] - AE[i, j]) * Fd1[j][d] - AE[i, j] * Fd3[j][d])
            if AI[i, i] == 0.0:
                vi.append(g)
            else:
                lam = 1.0 / (dt * AI[i, i])
                vi.append(helmholtz_solve(spec, lam, nui, lam * g, solver,
                                          g_wall=None if Vb[i] is None else Vb[i][d]))
        stage_v.append(vi)
        terms(i, vi, nui)
    out = []
    for d in range(3):
        acc = np.zeros_like(v[0])
        for i in range(s):
            acc += (bE[i] - AE[s - 1, i]) * (Fc[i][d] + Fd2[i][d] + Fd3[i][d])
            acc += (bI[i] - AI[s - 1, i]) * (Fd1[i][d] + Fs[i][d])
        out.append(stage_v[-1][d] + dt * acc)
    if final_projection:
        out, _ = projection.project(spec, out, out)
    return out, dict(stage_v=stage_v)
