"""GPU parity of the IMEX-RK step (Alg. 3 with the tableaux of App. A) and
of its new terms against the oracle.

Bars: the convective term F_c (local Lax-Friedrichs fluxes, Gauss rule of
floor(3P/2)+1 points) and F_d2 element by element <= 1e-12 relative (the same
exactly integrated sums in FP64, summed in another order); one whole step
from the same state <= 1e-10 relative, the GPU's solves run to 1e-13 and the
oracle's velocity solves by dense Cholesky, its pressure solves by fast
diagonalisation (exact).  Temporal order of the GPU step: on the VVP case
(resolved mesh) and on a shear flow whose projection is exact, the order of
Table 1 within 0.3."""
import numpy as np
import pytest

import synth
from oracle import convection, imex
from tests.gpu_util import say, to_dev, torch_dev
from tests.helpers import make_spec, ndof, node_coords

pytestmark = pytest.mark.gpu

CASES = [((2, 2, 2), 3, (0, 0, 0), False, False),
         ((3, 2, 2), 4, (0, 0, 1), True, True),
         ((1, 3, 2), 5, (0, 1, 2), False, True),
         ((2, 1, 2), 6, (1, 0, 0), True, False),
         ((2, 2, 1), 7, (2, 1, 0), False, True),
         ((1, 2, 2), 8, (0, 0, 1), False, False)]
IDS = ["P3_periodic", "P4_channel_vb", "P5_n1x_vb", "P6_wall_x", "P7_mixed_vb", "P8_channel"]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_convection_matches_oracle(case):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    n, P, bc, st, with_vb = case
    spec = make_spec(n, P, bc, st)
    N = ndof(spec)
    rng = np.random.default_rng(50 + P)
    v = [rng.uniform(-1, 1, N) for _ in range(3)]
    vb = [rng.uniform(-1, 1, N) for _ in range(3)] if with_vb else None
    m = dg.mesh_from_spec(spec)
    out = [torch.full((N,), np.nan, dtype=torch.float64, device=dev) for _ in range(3)]
    dg.dg_convection(m, [to_dev(c) for c in v], out, vb=None if vb is None else [to_dev(c) for c in vb])
    torch.cuda.synchronize()
    want = convection.convection(spec, v, vb)
    for d in range(3):
        e = rel(out[d].cpu().numpy(), want[d])
        say("convection", case, d, e)
        assert e <= 1e-12
    # accumulate and scale: out += -2 F_c
    base = [c.clone() for c in out]
    dg.dg_convection(m, [to_dev(c) for c in v], out, vb=None if vb is None else [to_dev(c) for c in vb],
                     scale=-2.0, accumulate=True)
    torch.cuda.synchronize()
    for d in range(3):
        assert torch.allclose(out[d], -base[d], rtol=1e-13, atol=1e-13 * float(base[d].abs().max()))
    m.destroy()


@pytest.mark.parametrize("case", CASES[1:], ids=IDS[1:])
def test_fd2_matches_oracle(case):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    n, P, bc, st, _ = case
    spec = make_spec(n, P, bc, st)
    N = ndof(spec)
    rng = np.random.default_rng(60 + P)
    v = [rng.uniform(-1, 1, N) for _ in range(3)]
    nu = 0.01 + 0.02 * rng.uniform(0, 1, N)
    m = dg.mesh_from_spec(spec)
    out = [torch.full((N,), np.nan, dtype=torch.float64, device=dev) for _ in range(3)]
    dg.dg_viscous_fd2(m, to_dev(nu), [to_dev(c) for c in v], out)
    torch.cuda.synchronize()
    want = convection.fd2(spec, nu, v)
    for d in range(3):
        e = rel(out[d].cpu().numpy(), want[d])
        say("fd2", case, d, e)
        assert e <= 1e-12
    m.destroy()


def _gpu_step(spec, v, t, dt, method, nu0, nu1, forcing, final_projection, tol=1e-13, precision=0, precond=1):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    vd = [to_dev(c) for c in v]
    tab = dg.imex_tableau(method)
    f = None
    if forcing is not None:
        f = [[to_dev(c) for c in forcing(t + tab.c[j] * dt)] for j in range(tab.s)]
    info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, vd, forcing=f,
                           final_projection=final_projection,
                           opts=dg.default_opts(tol=tol, precond=precond, precision=precision))
    out = [c.cpu().numpy() for c in vd]
    mv.destroy()
    mp.destroy()
    return out, info


@pytest.mark.parametrize("method", ["RK-TR", "RK-CB2", "RK-CB3c", "RK-CB3e", "RK-CB4", "RK-ARS3"])
def test_step_vvp_matches_oracle(method):
    # one step of the VVP vortex array (periodic [-1/2,1/2]^3, nu(v) =
    # 0.01 + 0.01 (|v|/2)^2, the manufactured forcing) from the exact
    # velocity at t = 0.1, with the final projection
    spec = make_spec((2, 2, 2), 4, (0, 0, 0), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    t, dt, nu0, nu1 = 0.1, 1.0 / 32, 0.01, 0.01
    v = synth.vvp_velocity(X, Y, Z, t)
    f = lambda tt: synth.vvp_forcing(X, Y, Z, tt, nu0, nu1)
    got, info = _gpu_step(spec, v, t, dt, method, nu0, nu1, f, True)
    want, _ = imex.step(spec, v, t, dt, imex.TABLEAUX[method], nu0, nu1, synth.VVP_VMAX, f,
                        final_projection=True, solver="dense")
    say("step", method, info)
    assert info["status"] == 0
    for d in range(3):
        e = rel(got[d], want[d])
        say("step", method, d, e)
        assert e <= 1e-10


@pytest.mark.parametrize("method", ["RK-CB3e", "RK-ARS3"])
def test_step_vvp_fp32_preconditioner_matches_oracle(method):
    # the same step with every solve preconditioned by the FP32 transforms
    # (precision DG_MIXED): CG stays FP64 with the same stopping test, so the
    # step meets the same bar
    spec = make_spec((2, 2, 2), 4, (0, 0, 0), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    t, dt, nu0, nu1 = 0.1, 1.0 / 32, 0.01, 0.01
    v = synth.vvp_velocity(X, Y, Z, t)
    f = lambda tt: synth.vvp_forcing(X, Y, Z, tt, nu0, nu1)
    got, info = _gpu_step(spec, v, t, dt, method, nu0, nu1, f, True, precision=1)
    want, _ = imex.step(spec, v, t, dt, imex.TABLEAUX[method], nu0, nu1, synth.VVP_VMAX, f,
                        final_projection=True, solver="dense")
    say("step fp32 preconditioner", method, info)
    assert info["status"] == 0
    for d in range(3):
        e = rel(got[d], want[d])
        say("step fp32 preconditioner", method, d, e)
        assert e <= 1e-10


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_step_vvp_jacobi_matches_oracle(precision):
    # the step with Jacobi-PCG for every solve (velocity solves one after
    # another, FP64 or FP32 CG with FP64 residual replacement; the stage's
    # term groups still on three streams)
    spec = make_spec((2, 2, 2), 4, (0, 0, 0), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    t, dt, nu0, nu1 = 0.1, 1.0 / 32, 0.01, 0.01
    v = synth.vvp_velocity(X, Y, Z, t)
    f = lambda tt: synth.vvp_forcing(X, Y, Z, tt, nu0, nu1)
    got, info = _gpu_step(spec, v, t, dt, "RK-ARS3", nu0, nu1, f, True, tol=1e-12, precision=precision,
                          precond=0)
    want, _ = imex.step(spec, v, t, dt, imex.TABLEAUX["RK-ARS3"], nu0, nu1, synth.VVP_VMAX, f,
                        final_projection=True, solver="dense")
    say("step jacobi", precision, info)
    assert info["status"] == 0
    for d in range(3):
        e = rel(got[d], want[d])
        say("step jacobi", precision, d, e)
        assert e <= 1e-10


@pytest.mark.parametrize("method,fp", [("RK-CB3e", False), ("RK-ARS3", True)])
def test_step_channel_matches_oracle(method, fp):
    # walls in z (v_b = 0), graded z, no forcing, degree 5 / pressure 4
    spec = make_spec((2, 2, 3), 5, (0, 0, 1), True)
    X, Y, Z = node_coords(spec)
    s = np.sin(np.pi * Z)
    v = [s * np.sin(2 * np.pi * Y), s * np.cos(2 * np.pi * X), 0.3 * s * np.sin(2 * np.pi * (X + Y))]
    got, info = _gpu_step(spec, v, 0.0, 0.02, method, 0.01, 0.02, None, fp)
    want, _ = imex.step(spec, v, 0.0, 0.02, imex.TABLEAUX[method], 0.01, 0.02, synth.VVP_VMAX, None,
                        final_projection=fp, solver="dense")
    say("channel step", method, fp, info)
    assert info["status"] == 0
    for d in range(3):
        e = rel(got[d], want[d])
        say("channel step", method, d, e)
        assert e <= 1e-10


def test_step_argument_errors():
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = make_spec((2, 2, 2), 4, (0, 0, 0), False)
    ps = dict(spec)
    ps["P"] = 3
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    v = [torch.zeros(mv.ndof, dtype=torch.float64, device=dev) for _ in range(3)]
    bad = dg.imex_tableau("RK-CB3e")
    bad.aE[0 * 8 + 1] = 0.5        # explicit part not strictly lower triangular
    for tab, dt, mesh_p in ((bad, 0.01, mp), ("RK-CB3e", 0.0, mp), ("RK-CB3e", 0.01, mv)):
        info = dg.dg_imex_step(mv, mesh_p, tab, dt, 0.01, 0.01, 2.0, v, raise_on_error=False)
        assert info["rc"] == dg.DG_ERR_ARG
    mv.destroy()
    mp.destroy()


def _gpu_run(spec, method, T, dts, vel, frc, nu0=0.01, nu1=0.01):
    """Runs to time T with each step size; returns {dt: velocity} and the
    exact velocity at T (device tensors).  vel, frc: problem data
    generators of synth (xp = torch)."""
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    X, Y, Z = dg.mesh_coordinates(mv)
    tab = dg.imex_tableau(method)
    opts = dg.default_opts(tol=1e-13, precond=dg.DG_PC_FDM)
    res = {}
    for dt in dts:
        v = [c.contiguous() for c in vel(X, Y, Z, 0.0, xp=torch)]
        t = 0.0
        for _ in range(int(round(T / dt))):
            f = [[c.contiguous() for c in frc(X, Y, Z, t + tab.c[j] * dt, nu0, nu1, xp=torch)]
                 for j in range(tab.s)]
            info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, v, forcing=f,
                                   final_projection=True, opts=opts)
            assert info["status"] == 0
            t += dt
        res[dt] = v
    exact = vel(X, Y, Z, T, xp=torch)
    mv.destroy()
    mp.destroy()
    return res, exact


def _rms(torch, a):
    return float(torch.sqrt(sum((x * x).mean() for x in a) / 3))


@pytest.mark.parametrize("method", ["RK-CB2", "RK-CB3e", "RK-ARS3"])
def test_step_temporal_order_vvp(method):
    # the VVP vortex array (Sec. 4.2: nu0 = nu1 = 0.01, periodic) on 4^3
    # elements of degree 6 up to T = 1/8: differences to a dt = 2^-10 run of
    # the same discretisation fall at the method's order between dt = 2^-5
    # and 2^-7.  (Below about 1e-6 a first-order remainder of the splitting
    # takes over, whose size falls with the spatial resolution: the SIP
    # pressure operator is not exactly D M^-1 G.)
    torch, dev = torch_dev()
    spec = make_spec((4, 4, 4), 6, (0, 0, 0), False, lo=-0.5, hi=0.5)
    dts = [2.0 ** -5, 2.0 ** -6, 2.0 ** -7, 2.0 ** -10]
    res, exact = _gpu_run(spec, method, 0.125, dts, synth.vvp_velocity, synth.vvp_forcing)
    ref = res[dts[-1]]
    err = [_rms(torch, [res[dt][d] - ref[d] for d in range(3)]) for dt in dts[:-1]]
    eoc = [float(np.log2(err[i] / err[i + 1])) for i in range(2)]
    ex = _rms(torch, [ref[d] - exact[d] for d in range(3)])
    say("vvp order", method, err, eoc, "error vs exact at dt=2^-10", ex)
    p = 2 if method == "RK-CB2" else 3
    assert all(e >= p - 0.3 for e in eoc), (err, eoc)
    assert ex <= 1e-4


@pytest.mark.parametrize("method", ["RK-TR", "RK-CB2", "RK-CB3c", "RK-CB3e", "RK-CB4", "RK-ARS3"])
def test_step_temporal_order_shear(method):
    # the shear flow u(y, t) = sin(2 pi (y + t)) with nu(u): the projection
    # is exact here, so every tableau shows its order (Table 1)
    torch, dev = torch_dev()
    spec = make_spec((1, 3, 1), 5, (0, 0, 0), False)
    dts = [1 / 16, 1 / 32, 1 / 64, 1 / 512]
    res, exact = _gpu_run(spec, method, 0.125, dts, synth.shear_velocity, synth.shear_forcing)
    ref = res[dts[-1]]
    err = [_rms(torch, [res[dt][d] - ref[d] for d in range(3)]) for dt in dts[:-1]]
    eoc = [float(np.log2(err[i] / err[i + 1])) for i in range(2)]
    say("shear order", method, err, eoc)
    p = imex.ORDER[method]
    assert all(e >= p - 0.3 for e in eoc), (err, eoc)


@pytest.mark.parametrize("n,P,method,nsteps,fp", [((2, 2, 2), 5, "RK-CB3e", 2, True),
                                                  ((1, 1, 2), 8, "RK-ARS3", 1, True),
                                                  ((2, 1, 2), 6, "RK-CB4", 2, False)],
                         ids=["P5_two_steps", "P8_one_step", "P6_two_steps_no_final_projection"])
def test_steps_other_degrees_match_oracle(n, P, method, nsteps, fp):
    # consecutive steps of the VVP case at other degrees (pressure P - 1),
    # each against the oracle's step from the oracle's own previous state
    spec = make_spec(n, P, (0, 0, 0), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    t, dt, nu0, nu1 = 0.05, 1.0 / 64, 0.01, 0.01
    f = lambda tt: synth.vvp_forcing(X, Y, Z, tt, nu0, nu1)
    v_g = v_o = synth.vvp_velocity(X, Y, Z, t)
    for k in range(nsteps):
        v_g, info = _gpu_step(spec, v_g, t, dt, method, nu0, nu1, f, fp)
        v_o, _ = imex.step(spec, v_o, t, dt, imex.TABLEAUX[method], nu0, nu1, synth.VVP_VMAX, f,
                           final_projection=fp, solver="dense")
        t += dt
        assert info["status"] == 0
        for d in range(3):
            e = rel(v_g[d], v_o[d])
            say("steps", P, method, k, d, e)
            assert e <= 1e-10


def test_user_tableau_with_an_explicit_stage_matches_oracle():
    # a caller's own 3-stage tableau whose middle stage has no implicit term
    # (a^I_22 = 0: v_2 = g_2, no solve), through the dg_tableau struct
    import paper_2112_04167_amd as dg
    from fractions import Fraction as Fr
    c = [0, Fr(1, 2), 1]
    AI = [[0, 0, 0], [Fr(1, 2), 0, 0], [Fr(1, 4), Fr(1, 4), Fr(1, 2)]]
    AE = [[0, 0, 0], [Fr(1, 2), 0, 0], [Fr(1, 2), Fr(1, 2), 0]]
    bI, bE = [Fr(1, 4), Fr(1, 4), Fr(1, 2)], [Fr(1, 2), 0, Fr(1, 2)]
    otab = dict(s=3, c=c, AI=AI, bI=bI, AE=AE, bE=bE)
    t = dg.binding.dg_tableau()
    t.s = 3
    for i in range(3):
        t.c[i], t.bI[i], t.bE[i] = float(c[i]), float(bI[i]), float(bE[i])
        for j in range(3):
            t.aI[i * 8 + j], t.aE[i * 8 + j] = float(AI[i][j]), float(AE[i][j])
    torch, dev = torch_dev()
    spec = make_spec((2, 2, 2), 4, (0, 0, 0), False, lo=-0.5, hi=0.5)
    X, Y, Z = node_coords(spec)
    tt, dt, nu0, nu1 = 0.0, 1.0 / 64, 0.01, 0.01
    v = synth.vvp_velocity(X, Y, Z, tt)
    f = lambda s_: synth.vvp_forcing(X, Y, Z, s_, nu0, nu1)
    ps = dict(spec)
    ps["P"] = 3
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    vd = [to_dev(x) for x in v]
    fd = [[to_dev(x) for x in f(tt + float(c[j]) * dt)] for j in range(3)]
    info = dg.dg_imex_step(mv, mp, t, dt, nu0, nu1, synth.VVP_VMAX, vd, forcing=fd, final_projection=True,
                           opts=dg.default_opts(tol=1e-13, precond=dg.DG_PC_FDM))
    want, _ = imex.step(spec, v, tt, dt, otab, nu0, nu1, synth.VVP_VMAX, f, final_projection=True, solver="dense")
    say("user tableau", info)
    # two stage projections, three velocity solves (stage 3 only), the final projection
    assert info["status"] == 0 and info["solves"] == 6
    for d in range(3):
        assert rel(vd[d].cpu().numpy(), want[d]) <= 1e-10
    mv.destroy()
    mp.destroy()


@pytest.mark.parametrize("method", ["RK-ARS3", "RK-CB3e"])
def test_step_full_size_vvp(method):
    # the bench's step at its own size (16^3 elements, P = 7, dt = 2^-8,
    # FDM-preconditioned solves to 1e-10, the final projection): one step
    # from the exact vortex-array state stays within 1e-6 of the exact
    # solution (measured 2.0e-7 / 2.7e-7; the spatial and temporal errors
    # of this resolution), with the solver counts of a healthy step
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    spec = synth.mesh_spec("vvp_large")
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    X, Y, Z = dg.mesh_coordinates(mv)
    dt, nu0, nu1 = 2.0 ** -8, 0.01, 0.01
    tab = dg.imex_tableau(method)
    v = [c.contiguous() for c in synth.vvp_velocity(X, Y, Z, 0.0, xp=torch)]
    f = [[c.contiguous() for c in synth.vvp_forcing(X, Y, Z, tab.c[j] * dt, nu0, nu1, xp=torch)]
         for j in range(tab.s)]
    info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, v, forcing=f, final_projection=True,
                           opts=dg.default_opts(precond=dg.DG_PC_FDM))
    ve = synth.vvp_velocity(X, Y, Z, dt, xp=torch)
    err = max(float(torch.linalg.vector_norm(v[d] - ve[d]) / torch.linalg.vector_norm(ve[d])) for d in range(3))
    say("full-size step", method, info, err)
    assert info["status"] == 0 and err <= 1e-6
    assert info["pressure_iters"] <= 2 * (tab.s - 1) + 2 and info["velocity_iters"] <= 6 * 3 * (tab.s - 1)
    mv.destroy()
    mp.destroy()
