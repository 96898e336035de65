"""GPU parity of inhomogeneous Dirichlet data (the wall velocity v_b of
Alg. 3 in the velocity solves and in the whole step): the Nitsche load
against the oracle's face-by-face evaluation (<= 1e-13 relative: same sums),
a solve with wall data that reproduces a polynomial solution exactly
(<= 1e-11, the solve's own tolerance), the step keeping plane Couette flow,
and one step of the vortex array with time-dependent walls on every face
(the VVD case of Sec. 4.2) against the oracle's step (<= 1e-10)."""
import numpy as np
import pytest

import synth
from oracle import dense, imex
from tests.gpu_util import say, to_dev, torch_dev
from tests.helpers import make_spec, ndof, node_coords

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,P,bc,nodal", [((2, 2, 3), 3, (0, 0, 1), False), ((2, 3, 2), 5, (1, 0, 1), True),
                                          ((2, 2, 2), 8, (1, 1, 1), True), ((3, 1, 2), 6, (1, 2, 0), False)],
                         ids=["P3_walls_z", "P5_walls_xz_nodal", "P8_box_nodal", "P6_wall_x_neumann_y"])
def test_dirichlet_load_matches_oracle(n, P, bc, nodal):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec(n, P, bc, True)
    N = ndof(spec)
    rng = np.random.default_rng(P)
    g = rng.uniform(-1, 1, N)
    nu = 0.5 + rng.uniform(0, 1, N) if nodal else 0.7
    b0 = rng.uniform(-1, 1, N)
    m = dg.mesh_from_spec(spec)
    bd = to_dev(b0)
    dg.dg_dirichlet_load(m, to_dev(nu) if nodal else None, to_dev(g), bd, nu_const=0.7, scale=-1.5)
    torch.cuda.synchronize()
    want = b0 - 1.5 * dense.dirichlet_load(spec, nu, g)
    e = rel(bd.cpu().numpy() - b0, want - b0)
    say("dirichlet load", n, P, bc, e)
    assert e <= 1e-13
    m.destroy()


def test_solve_with_wall_data_reproduces_polynomial():
    # u = 1 + x y + z^2 - x/2 on a box with walls on every face, nodal nu
    # linear: the load M f + L(u) gives u itself as the discrete solution
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((2, 2, 3), 5, (1, 1, 1), True)
    X, Y, Z = node_coords(spec)
    u = 1 + X * Y + Z ** 2 - 0.5 * X
    nu = 1 + 0.5 * Z + 0.2 * X
    lam = 3.0
    f = lam * u - (0.2 * (Y - 0.5) + 0.5 * 2 * Z + nu * 2)
    M = dense.mass_diag(spec)
    m = dg.mesh_from_spec(spec)
    b = to_dev(M * f)
    dg.dg_dirichlet_load(m, to_dev(nu), to_dev(u), b)
    x = torch.zeros_like(b)
    info = dg.helmholtz_solve(m, lam, to_dev(nu), 0.0, b, x, dg.default_opts(tol=1e-13, rhs_is_weak=1))
    err = np.max(np.abs(x.cpu().numpy() - u))
    say("wall-data solve", info, err)
    assert info["status"] == 0 and err <= 1e-11
    m.destroy()


def test_step_keeps_couette_flow():
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((2, 2, 3), 5, (0, 0, 1), True)
    X, Y, Z = node_coords(spec)
    ps = dict(spec)
    ps["P"] = 4
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    v0 = [Z.copy(), 0 * Z, 0 * Z]
    vd = [to_dev(c) for c in v0]
    tab = dg.imex_tableau("RK-ARS3")
    wall = [[to_dev(Z), None, None] for _ in range(tab.s)]
    info = dg.dg_imex_step(mv, mp, tab, 0.05, 0.02, 0.0, 2.0, vd, wall=wall, final_projection=True,
                           opts=dg.default_opts(tol=1e-13, precond=dg.DG_PC_FDM))
    err = max(np.max(np.abs(vd[d].cpu().numpy() - v0[d])) for d in range(3))
    say("couette", info, err)
    assert info["status"] == 0 and err <= 1e-11
    mv.destroy()
    mp.destroy()


@pytest.mark.parametrize("method", ["RK-ARS3", "RK-CB3e"])
def test_step_vvd_matches_oracle(method):
    # the vortex array in [-1/2, 1/2]^3 with walls on every face carrying the
    # exact (time-dependent) velocity, the manufactured forcing, nu(v)
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((2, 2, 2), 4, (1, 1, 1), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    t, dt, nu0, nu1 = 0.1, 1.0 / 32, 0.01, 0.01
    ps = dict(spec)
    ps["P"] = 3
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    tab = dg.imex_tableau(method)
    v = synth.vvp_velocity(X, Y, Z, t)
    vd = [to_dev(c) for c in v]
    f = [[to_dev(c) for c in synth.vvp_forcing(X, Y, Z, t + tab.c[j] * dt, nu0, nu1)] for j in range(tab.s)]
    w = [[to_dev(c) for c in synth.vvp_velocity(X, Y, Z, t + tab.c[j] * dt)] for j in range(tab.s)]
    info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, vd, forcing=f, wall=w,
                           final_projection=True, opts=dg.default_opts(tol=1e-13, precond=dg.DG_PC_FDM))
    want, _ = imex.step(spec, v, t, dt, imex.TABLEAUX[method], nu0, nu1, synth.VVP_VMAX,
                        lambda tt: synth.vvp_forcing(X, Y, Z, tt, nu0, nu1), final_projection=True,
                        solver="dense", wall=lambda tt: synth.vvp_velocity(X, Y, Z, tt))
    say("vvd step", method, info)
    assert info["status"] == 0
    for d in range(3):
        e = rel(vd[d].cpu().numpy(), want[d])
        say("vvd step", method, d, e)
        assert e <= 1e-10
    ex = synth.vvp_velocity(X, Y, Z, t + dt)
    say("vvd error vs exact", max(rel(want[d], ex[d]) for d in range(3)))
    mv.destroy()
    mp.destroy()


def test_step_vvd_error_falls_with_resolution():
    # one RK-CB3e step (dt = 1/64) of the vortex array with walls on every
    # face carrying the exact velocity: the error against the exact solution
    # falls with the resolution as in the periodic case (a wall treatment
    # that is not consistent would leave an O(1) remainder)
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    errs = []
    for ne, P in ((2, 4), (2, 6), (3, 6)):
        spec = make_spec((ne,) * 3, P, (1, 1, 1), False, lo=-0.5, hi=0.5)
        X, Y, Z = node_coords(spec)
        M = dense.mass_diag(spec)
        t, dt, nu0, nu1 = 0.1, 1.0 / 64, 0.01, 0.01
        ps = dict(spec)
        ps["P"] = P - 1
        mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
        tab = dg.imex_tableau("RK-CB3e")
        vd = [to_dev(c) for c in synth.vvp_velocity(X, Y, Z, t)]
        f = [[to_dev(c) for c in synth.vvp_forcing(X, Y, Z, t + tab.c[j] * dt, nu0, nu1)] for j in range(tab.s)]
        w = [[to_dev(c) for c in synth.vvp_velocity(X, Y, Z, t + tab.c[j] * dt)] for j in range(tab.s)]
        info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, vd, forcing=f, wall=w,
                               final_projection=True, opts=dg.default_opts(precond=dg.DG_PC_FDM))
        assert info["status"] == 0
        ex = synth.vvp_velocity(X, Y, Z, t + dt)
        errs.append(max(np.sqrt(np.dot(M, (vd[d].cpu().numpy() - ex[d]) ** 2) / np.dot(M, ex[d] ** 2))
                        for d in range(3)))
        mv.destroy()
        mp.destroy()
    say("vvd spatial errors", errs)
    assert errs[0] / errs[1] >= 4 and errs[1] / errs[2] >= 4, errs


def test_step_full_size_couette():
    # the channel at the batched configuration's size (24^3 elements, P = 5,
    # walls in z): plane Couette flow kept by one RK-CB3e step
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = synth.mesh_spec("batched_channel")
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    X, Y, Z = dg.mesh_coordinates(mv)
    v = [Z.clone(), torch.zeros_like(Z), torch.zeros_like(Z)]
    tab = dg.imex_tableau("RK-CB3e")
    wall = [[Z, None, None] for _ in range(tab.s)]
    info = dg.dg_imex_step(mv, mp, tab, 1e-3, 0.02, 0.0, 2.0, v, wall=wall, final_projection=True,
                           opts=dg.default_opts(tol=1e-12, precond=dg.DG_PC_FDM))
    err = max(float((v[0] - Z).abs().max()), float(v[1].abs().max()), float(v[2].abs().max()))
    say("full-size couette", info, err)
    assert info["status"] == 0 and err <= 1e-10
    mv.destroy()
    mp.destroy()
