"""Benchmark of the SIP-DG Helmholtz implicit-stage solve on one MI355X.

Step = one matrix-free SIP-DG Helmholtz apply y = (lambda M + K) x on the
32^3-element, P=7 (16.8M nodes) tanh-stretched channel mesh (Dirichlet z,
periodic x,y), lambda = 1/(0.4358665 dt nu), dt = nu = 1e-3, FP64, inputs
resident in HBM, x/y rotated over 5 buffer pairs (1.3 GiB) so that the
256 MB last-level cache cannot serve a repeat.  value = GDOF/s of the apply.

Also reported on the same JSON line (each measured after the timed steps):
  roofline      algorithmic bytes of the apply kernel (16 B/node) over its
                HIP-event duration on its own stream, vs 8 TB/s
  cpu_baseline  the CPU oracle's naive apply on the same mesh (host cores)
  solve         FP64 Jacobi-PCG Helmholtz solve of the same mesh to 1e-10
                (collocation-residual rule), solves/s and DOF-iterations/s
  poisson       the pressure Poisson solve of the same mesh (lambda = 0)
  mixed         FP32-inner / FP64-refinement solves of the 4^3, P=7 case
  solve_mixed   the same Helmholtz solve, FP32 CG with FP64 residual
                replacement, to the same 1e-10 residual
  poisson_mixed the Poisson solve in the mixed mode
  mixed_small   FP64 vs mixed on the 4^3, P=7 case, lambda in {1e2,1e4,1e6}
  batched       the 24^3, P=5 stage (3 velocity + 1 pressure) in one
                persistent launch vs the same 4 systems solved one after the
                other by the plain FP64 solver (and by the mixed solver)
  serving       the request stream (Poisson arrivals), p50/p99 latency
  fdm           the fast-diagonalisation inverse of the same mesh (three FP64
                MFMA transforms each way along the mesh lines): time per
                application and FP64 matrix rate against the 78.6 TFLOP/s peak
  solve_fdm     the Helmholtz and Poisson solves of the same mesh with CG
  poisson_fdm   preconditioned by that inverse (same 1e-10 rule)
  (batched and serving also report the stage and the full 2000-request
  stream with the fast-diagonalisation preconditioner)
  stage         one implicit stage of Alg. 3 on the 24^3 channel mesh: the
                projection substep (pressure at P-1 = 4, FDM-PCG) followed by
                the three velocity Helmholtz solves (P = 5, nodal nu)
  stage_varnu   the same stage with the variable viscosity of Alg. 3:
                nu_i = nu(v''_i) = nu0 + nu1 (|v''|/v_ref)^2, the earlier
                stage's F_d1 = div(nu grad v) and F_d3 = -grad(nu div v), the
                load g_i, and the three solves with the new nodal nu

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
                       [--legs solve,poisson,...] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
APPLY_BYTES_PER_DOF_FP64 = 16.0   # read x once, write y once
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_p7_fp64_stretched32.md")
COUNTER_FILE = os.path.join(ROOT, "profiles", "apply_p7_fp64_stretched32_counters.md")
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profile_value(path, key):
    """A per-launch figure of the apply kernel from a committed rocprofv3
    counter summary, or None if the kernel source changed since the counters
    were taken."""
    from paper_2112_04167_amd.prof_summary import kernel_sha
    try:
        with open(path) as fh:
            kv = dict(l.strip().split(": ", 1) for l in fh if ": " in l and l.startswith("    "))
    except OSError:
        return None
    if kv.get("kernel_sha") != kernel_sha():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """Per-launch HBM traffic (bytes) of the apply kernel (FETCH_SIZE + WRITE_SIZE)."""
    return profile_value(TRAFFIC_FILE, "traffic_bytes_per_launch")


def measured_flops():
    """Per-launch FP64 FLOPs of the apply kernel (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes)."""
    return profile_value(COUNTER_FILE, "flops_per_launch")


def bench_apply(dg, torch, spec, lam, steps, warmup, npairs=5):
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mesh = dg.mesh_from_spec(spec, stream=stream)
    N = mesh.ndof
    gen = torch.Generator(device=dev)
    gen.manual_seed(21120)
    xs = [torch.rand(N, dtype=torch.float64, device=dev, generator=gen) * 2 - 1 for _ in range(npairs)]
    ys = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(npairs)]
    for k in range(warmup):
        dg.helmholtz_apply(mesh, lam, None, 1.0, xs[k % npairs], ys[k % npairs], stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e0, e1 = ev[k]
        e0.record(stream)
        dg.helmholtz_apply(mesh, lam, None, 1.0, xs[k % npairs], ys[k % npairs], stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    durs = np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])
    mesh.destroy()
    return N, t1 - t0, durs


def bench_solve(dg, torch, spec, lam, seed, reps, poisson=False, precond=0, ref=None):
    """Median wall time of a solve from x = 0; with ref (a solution of the
    same system) also the relative difference to it."""
    import synth
    dev = torch.device("cuda:0")
    mesh = dg.mesh_from_spec(spec)
    N = mesh.ndof
    f = torch.from_numpy(synth.uniform_field(N, seed)).to(dev)
    x = torch.zeros_like(f)
    o = dg.default_opts(precond=precond)
    times, infos = [], []
    if precond:   # untimed first solve: the host eigendecompositions (cached afterwards)
        (dg.poisson_solve(mesh, f, x, o) if poisson else dg.helmholtz_solve(mesh, lam, None, 1.0, f, x, o))
    for _ in range(reps):
        x.zero_()  # x is the initial guess: every timed solve starts from zero
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if poisson:
            info = dg.poisson_solve(mesh, f, x, o)
        else:
            info = dg.helmholtz_solve(mesh, lam, None, 1.0, f, x, o)
        t1 = time.perf_counter()
        times.append(t1 - t0)
        infos.append(info)
    mesh.destroy()
    t = float(np.median(times))
    it = infos[-1]["iters"]
    out = dict(seconds_median=t, solves_per_s=1.0 / t, iters=it, status=infos[-1]["status"],
               true_rel_res=infos[-1]["true_rel_res"], ndof=N)
    if not precond:
        # FP64 CG with a constant nu: apply 16, update 48, p-update 24 B/node
        # (the diagonal is computed, not read)
        out.update(gdof_iter_per_s=N * it / t / 1e9, bytes_per_dof_iter=88.0,
                   frac_of_solve_bound=(N * it * 88.0 / t) / (HBM_PEAK_GBS * 1e9))
    if ref is not None:
        out["rel_diff_vs_jacobi_fp64"] = float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))
    out["x"] = x
    return out


FP64_MATRIX_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix (MFMA)


def bench_fdm(dg, torch, spec, lam, reps=20):
    """The fast-diagonalisation inverse alone: HIP-event time per application
    on its stream; algorithmic flops 2 L N per transform, forward and
    backward along three axes: 4 N (Lx + Ly + Lz)."""
    import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mesh = dg.mesh_from_spec(spec, stream=stream)
    N = mesh.ndof
    b = torch.from_numpy(synth.uniform_field(N, 7)).to(dev)
    x = torch.empty_like(b)
    dg.helmholtz_fdm_apply(mesh, lam, 1.0, b, x, stream=stream)   # tables
    for _ in range(3):
        dg.helmholtz_fdm_apply(mesh, lam, 1.0, b, x, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        dg.helmholtz_fdm_apply(mesh, lam, 1.0, b, x, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    durs = np.array([a.elapsed_time(c) * 1e-3 for a, c in ev])
    P = spec["P"]
    Ls = [spec[k] * (P + 1) for k in ("nx", "ny", "nz")]
    flops = 4.0 * N * sum(Ls)
    mesh.destroy()
    t = float(np.median(durs))
    return {"bound": "mfma", "achieved": flops / t / 1e12, "peak": FP64_MATRIX_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flops / t / 1e12 / FP64_MATRIX_PEAK_TFLOPS,
            "flops_per_application": flops, "us_median": t * 1e6, "us_min": float(durs.min()) * 1e6,
            "kernels": "k_fdm_axis x5 (x, y, z fwd+scale+bwd, y, x)", "line_lengths": Ls}


def cpu_baseline(spec, lam, budget_s=12.0):
    from oracle import naive
    import synth
    op = naive.Operator(spec, lam, 1.0)
    x = synth.uniform_field(op.N, 7)
    op.apply(x)  # warm
    reps, t0 = 0, time.perf_counter()
    while True:
        op.apply(x)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    out = dict(value=op.N * reps / dt / 1e9, unit="GDOF/s", cores=naive.num_threads(),
               kind="oracle",
               sample="%d full applies of the 32^3 P=7 stretched mesh (%d nodes), %.1f s"
                      % (reps, op.N, dt))
    out["solves"] = cpu_solves()
    return out


def cpu_solves(sample_iters=5):
    """The oracle's Jacobi-PCG (all host cores) on the solve configurations:
    whole solves where they take seconds (4^3 P=4; the 4^3 P=7 mixed-case
    systems in FP64; the 24^3 P=5 channel velocity system with nodal nu),
    a fixed sample of iterations on the 32^3 P=7 systems (Helmholtz and
    Poisson), reported as a rate and the implied time of the GPU's
    iteration count."""
    from oracle import dense, naive, pcg
    import synth
    res = {}

    def run(name, spec, lam, nu, f, fixed=0, singular=False):
        op = naive.Operator(spec, lam, nu)
        M = dense.mass_diag(spec)
        d = op.diag()
        t0 = time.perf_counter()
        _, info = pcg.pcg(op.apply, M * f, d, M, tol=1e-10, fixed_iters=fixed, singular=singular)
        t = time.perf_counter() - t0
        res[name] = dict(nodes=op.N, iters=info["iters"], seconds=t, seconds_per_iter=t / max(1, info["iters"]),
                         whole_solve=fixed == 0)

    s1 = synth.mesh_spec("small_periodic")
    run("small_periodic_4x4x4_P4", s1, 1.0, 1.0, synth.uniform_field(s1["nx"] ** 3 * 125, 0))
    s3 = synth.mesh_spec("mixed_small")
    for lam in (1e2, 1e4, 1e6):
        run("mixed_small_P7_lambda_%g_fp64" % lam, s3, lam, 1.0,
            synth.uniform_field(s3["nx"] ** 3 * 512, synth.SEEDS["mixed"]))
    s4 = synth.mesh_spec("batched_channel")
    N4 = s4["nx"] ** 3 * 216
    # the channel viscosity nu(x) = 1e-3 (1 + 0.5 sin 2 pi x cos 2 pi y) at the
    # nodes (element-major layout; GLL nodes from the oracle)
    from oracle import gll
    xi = gll.nodes(s4["P"])
    n4 = s4["P"] + 1

    def c1(v):
        v = np.asarray(v)
        return v[:-1, None] + np.diff(v)[:, None] * (1.0 + xi[None, :]) / 2.0

    shp = (s4["nz"], s4["ny"], s4["nx"], n4, n4, n4)
    X = np.broadcast_to(c1(s4["xv"])[None, None, :, None, None, :], shp).reshape(-1)
    Y = np.broadcast_to(c1(s4["yv"])[None, :, None, None, :, None], shp).reshape(-1)
    nu4 = 1e-3 * (1.0 + 0.5 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y))
    run("channel_24_P5_velocity_nodal_nu", s4, synth.batched_lambda(), nu4,
        synth.uniform_field(N4, synth.SEEDS["batched_velocity"][0]))
    s2 = synth.mesh_spec("stretched_large")
    N2 = s2["nx"] ** 3 * 512
    run("stretched_32_P7_helmholtz_%d_iters" % sample_iters, s2, synth.large_helmholtz_lambda(), 1.0,
        synth.uniform_field(N2, synth.SEEDS["large_helmholtz"]), fixed=sample_iters)
    res["stretched_32_P7_helmholtz_%d_iters" % sample_iters]["implied_36_iter_solve_s"] = \
        36 * res["stretched_32_P7_helmholtz_%d_iters" % sample_iters]["seconds_per_iter"]
    ps = dict(s2)
    ps["bc"] = (0, 0, 2)
    run("stretched_32_P7_poisson_%d_iters" % sample_iters, ps, 0.0, 1.0,
        synth.uniform_field(N2, synth.SEEDS["large_poisson"]), fixed=sample_iters, singular=True)
    res["stretched_32_P7_poisson_%d_iters" % sample_iters]["implied_2738_iter_solve_s"] = \
        2738 * res["stretched_32_P7_poisson_%d_iters" % sample_iters]["seconds_per_iter"]
    return res


def bench_mixed_small(dg, torch, reps=20):
    """FP32-inner / FP64-refinement solves of the 4^3, P=7 periodic case."""
    import synth
    dev = torch.device("cuda:0")
    spec = synth.mesh_spec("mixed_small")
    mesh = dg.mesh_from_spec(spec)
    N = mesh.ndof
    f = torch.from_numpy(synth.uniform_field(N, synth.SEEDS["mixed"])).to(dev)
    x = torch.zeros_like(f)
    out = {}
    for lam in (1e2, 1e4, 1e6):
        row = {}
        sols = {}
        for name, prec in (("fp64", dg.DG_FP64), ("mixed", dg.DG_MIXED)):
            o = dg.default_opts(precision=prec)
            x.zero_()
            dg.helmholtz_solve(mesh, lam, None, 1.0, f, x, o)
            ts = []
            for _ in range(reps):
                x.zero_()  # x is the initial guess: every timed solve starts from zero
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = dg.helmholtz_solve(mesh, lam, None, 1.0, f, x, o)
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            row[name] = dict(ms=t * 1e3, iters=info["iters"], outer=info["outer_iters"],
                             true_rel_res=info["true_rel_res"])
            sols[name] = x.clone()
        # error of the mixed result against the FP64 one (which the GPU tests
        # hold to 1e-10 of the exact discrete solution)
        row["mixed"]["rel_err_vs_fp64"] = float(torch.linalg.vector_norm(sols["mixed"] - sols["fp64"]) /
                                                torch.linalg.vector_norm(sols["fp64"]))
        out["lambda=%g" % lam] = row
    mesh.destroy()
    return out


def bench_mixed_large(dg, torch, spec, lam, poisson=False):
    """The mixed-precision solve of the large mesh (same right-hand side and
    1e-10 residual rule as the FP64 leg of the same problem)."""
    import synth
    dev = torch.device("cuda:0")
    mesh = dg.mesh_from_spec(spec)
    seed = synth.SEEDS["large_poisson" if poisson else "large_helmholtz"]
    f = torch.from_numpy(synth.uniform_field(mesh.ndof, seed)).to(dev)
    x = torch.zeros_like(f)
    o = dg.default_opts(precision=dg.DG_MIXED)

    def solve():
        if poisson:
            return dg.poisson_solve(mesh, f, x, o)
        return dg.helmholtz_solve(mesh, lam, None, 1.0, f, x, o)

    solve()
    ts = []
    for _ in range(1 if poisson else 5):
        x.zero_()  # x is the initial guess: every timed solve starts from zero
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = solve()
        ts.append(time.perf_counter() - t0)
    # error against the FP64 solve of the same problem (untimed)
    x64 = torch.zeros_like(f)
    if poisson:
        dg.poisson_solve(mesh, f, x64)
    else:
        dg.helmholtz_solve(mesh, lam, None, 1.0, f, x64)
    err = float(torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64))
    mesh.destroy()
    t = float(np.median(ts))
    return dict(seconds_median=t, solves_per_s=1.0 / t, inner_iters=info["iters"],
                outer_iters=info["outer_iters"], true_rel_res=info["true_rel_res"],
                rel_err_vs_fp64=err)


def bench_batched(dg, torch):
    """The 24^3, P=5 stage: 3 velocity (nodal nu) + 1 pressure system in one
    persistent launch, against the same 4 systems solved one after another
    by the plain FP64 solver."""
    import synth
    dev = torch.device("cuda:0")
    spec = synth.mesh_spec("batched_channel")
    mesh = dg.mesh_from_spec(spec)
    N = mesh.ndof
    X, Y, _ = dg.mesh_coordinates(mesh)
    nu = 1e-3 * (1.0 + 0.5 * torch.sin(2 * np.pi * X) * torch.cos(2 * np.pi * Y))   # input field
    lam = synth.batched_lambda()
    fs = [torch.from_numpy(synth.uniform_field(N, s)).to(dev) for s in synth.SEEDS["batched_velocity"]]
    fs.append(torch.from_numpy(synth.uniform_field(N, synth.SEEDS["batched_pressure"])).to(dev))
    xs = [torch.zeros_like(fs[0]) for _ in range(4)]
    lams, nus, pois = [lam] * 3 + [0.0], [nu] * 3 + [None], [0, 0, 0, 1]
    o = dg.default_opts(precision=dg.DG_MIXED)
    dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o)   # autotune + warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, infos = dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o)
    tb = time.perf_counter() - t0
    x_pure = [x.clone() for x in xs]
    # the same launch, ended once only the Poisson system is left, which the
    # single-system mixed solver then finishes from its current solution
    dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o, handoff=True)   # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rch, infosh = dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o, handoff=True)
    th = time.perf_counter() - t0
    x_hand = [x.clone() for x in xs]
    o64 = dg.default_opts()
    ofdm = dg.default_opts(precond=dg.DG_PC_FDM)

    def sequential(o):
        for xk in xs:
            xk.zero_()  # x is the initial guess of the single solves: start from zero
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        seq = []
        for k in range(4):
            if pois[k]:
                seq.append(dg.poisson_solve(mesh, fs[k], xs[k], o))
            else:
                seq.append(dg.helmholtz_solve(mesh, lam, nu, 0.0, fs[k], xs[k], o))
        return time.perf_counter() - t0, seq

    ts, seq = sequential(o64)
    x_ref64 = [x.clone() for x in xs]

    def errs_to(xm, ref):
        return [float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(xm, ref)]

    def errs(xm):  # error of each mixed result against the FP64 solve of its system
        return errs_to(xm, xs)

    err_pure, err_hand = errs(x_pure), errs(x_hand)
    tm, seqm = sequential(o)
    x_mixed = [x.clone() for x in xs]
    sequential(ofdm)   # untimed: the host eigendecompositions of both BC sets
    tf, seqf = sequential(ofdm)
    err_fdm = errs_to([x.clone() for x in xs], x_ref64)
    # the 4 systems as ordinary solves at once on separate streams
    # (DG_BATCH_CONCURRENT: the Poisson system FDM-preconditioned, the
    # velocity systems Jacobi FP64), against the same solves one after another
    dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o64, concurrent=True)   # warm: workspaces
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rcc, infosc = dg.helmholtz_solve_batched(mesh, lams, nus, pois, fs, xs, o64, concurrent=True)
    tc = time.perf_counter() - t0
    x_conc = [x.clone() for x in xs]
    for xk in xs:
        xk.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(4):
        if pois[k]:
            dg.poisson_solve(mesh, fs[k], xs[k], ofdm)
        else:
            dg.helmholtz_solve(mesh, lam, nu, 0.0, fs[k], xs[k], o64)
    tcs = time.perf_counter() - t0
    conc_same = all(bool(torch.equal(a, b)) for a, b in zip(x_conc, xs))
    mesh.destroy()
    return dict(ndof_per_field=N, batched_seconds=tb, batched_solves_per_s=4.0 / tb,
                sequential_fp64_seconds=ts, sequential_fp64_solves_per_s=4.0 / ts,
                sequential_mixed_seconds=tm, sequential_mixed_solves_per_s=4.0 / tm,
                speedup=ts / tb, status=rc,
                handoff_seconds=th, handoff_solves_per_s=4.0 / th, handoff_speedup=ts / th,
                handoff_status=rch, handoff_iters=[i["iters"] for i in infosh],
                handoff_true_rel_res=[i["true_rel_res"] for i in infosh],
                inner_iters=[i["iters"] for i in infos], outer_iters=[i["outer_iters"] for i in infos],
                true_rel_res=[i["true_rel_res"] for i in infos],
                rel_err_vs_fp64=err_pure, handoff_rel_err_vs_fp64=err_hand,
                fp64_iters=[i["iters"] for i in seq],
                sequential_mixed_iters=[i["iters"] for i in seqm],
                sequential_mixed_true_rel_res=[i["true_rel_res"] for i in seqm],
                concurrent_seconds=tc, concurrent_solves_per_s=4.0 / tc, concurrent_status=rcc,
                concurrent_iters=[i["iters"] for i in infosc],
                concurrent_sequential_same_preconditioners_seconds=tcs,
                concurrent_speedup_vs_sequential=tcs / tc, concurrent_speedup_vs_persistent=tb / tc,
                concurrent_equals_sequential_bitwise=conc_same,
                # the 4 systems one after another, CG preconditioned by the
                # fast-diagonalisation inverse (FP64; nu_ref for the nodal nu)
                sequential_fdm_seconds=tf, sequential_fdm_solves_per_s=4.0 / tf,
                sequential_fdm_speedup_vs_fp64=ts / tf,
                sequential_fdm_iters=[i["iters"] for i in seqf],
                sequential_fdm_true_rel_res=[i["true_rel_res"] for i in seqf],
                sequential_fdm_rel_diff_vs_jacobi_fp64=err_fdm)


def bench_stage(dg, torch, reps=5):
    """One implicit stage of Alg. 3 on the 24^3 channel mesh: project the
    predicted velocity v' (pressure of degree P-1 = 4, natural boundaries,
    v_b = 0, FDM-PCG), then solve v - dt a_ii div(nu grad v) = v'' for the
    three components (degree 5, nodal nu, Dirichlet walls).  The Helmholtz
    problem is passed divided by lambda = 1/(dt a_ii): operator M + K_{nu /
    lambda}, load M v'' (the same solution, with no arithmetic outside the
    library in the timed region)."""
    import synth
    dev = torch.device("cuda:0")
    spec = synth.mesh_spec("batched_channel")
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    N = mv.ndof
    X, Y, _ = dg.mesh_coordinates(mv)
    lam = synth.batched_lambda()
    nu_s = (1e-3 * (1.0 + 0.5 * torch.sin(2 * np.pi * X) * torch.cos(2 * np.pi * Y)) / lam).contiguous()
    v0 = [torch.from_numpy(synth.uniform_field(N, s)).to(dev) for s in synth.SEEDS["batched_velocity"]]
    xs = [torch.zeros_like(v0[0]) for _ in range(3)]
    psi = torch.zeros(mp.ndof, dtype=torch.float64, device=dev)
    op = dg.default_opts(precond=dg.DG_PC_FDM)
    out = {"ndof_velocity": N, "ndof_pressure": mp.ndof}
    for name, ov in (("fp64", dg.default_opts()), ("mixed", dg.default_opts(precision=dg.DG_MIXED))):
        times, tproj = [], []
        for r in range(reps + 1):
            v = [c.clone() for c in v0]
            psi.zero_()
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ip = dg.dg_project(mv, mp, v, psi, opts=op)
            t1 = time.perf_counter()
            iv = [dg.helmholtz_solve(mv, 1.0, nu_s, 0.0, v[k], xs[k], ov) for k in range(3)]
            t2 = time.perf_counter()
            if r > 0:   # the first stage builds the pressure tables and tunes
                times.append(t2 - t0)
                tproj.append(t1 - t0)
        t = float(np.median(times))
        out[name] = dict(stage_ms=t * 1e3, projection_ms=float(np.median(tproj)) * 1e3,
                         pressure_iters=ip["iters"], pressure_true_rel_res=ip["true_rel_res"],
                         velocity_iters=[i["iters"] for i in iv],
                         velocity_true_rel_res=[i["true_rel_res"] for i in iv],
                         stages_per_s=1.0 / t)
    mv.destroy()
    mp.destroy()
    return out


def bench_stage_varnu(dg, torch, reps=5):
    """One variable-viscosity implicit stage (Alg. 3, stage i = 2 of an
    SDIRK-type scheme) on the 24^3 channel mesh: projection (pressure P-1 =
    4, FDM-PCG), nu_2 = nu(v''), F_d1 and F_d3 of the first stage's velocity
    u_1 with nu_1 = nu(u_1), load g = v'' + dt [(aI - aE) F_d1 - aE F_d3]
    (times lambda = 1/(dt gamma)), three Helmholtz solves with the nodal
    nu_2 (Jacobi-PCG, FP64 and mixed).  nu0 = nu1 = 1e-3, v_ref = 2,
    dt = 1e-3, gamma = 0.4358665, aI = 0.2820667, aE = gamma."""
    import synth
    dev = torch.device("cuda:0")
    spec = synth.mesh_spec("batched_channel")
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec), dg.mesh_from_spec(ps)
    N = mv.ndof
    dt, gamma, aI, aE = 1e-3, 0.4358665, 0.2820667, 0.4358665
    lam = 1.0 / (dt * gamma)
    v0 = [torch.from_numpy(synth.uniform_field(N, s)).to(dev) for s in synth.SEEDS["batched_velocity"]]
    u1 = [torch.from_numpy(synth.uniform_field(N, 100 + s)).to(dev) for s in synth.SEEDS["batched_velocity"]]
    nu1, nu2 = torch.empty_like(v0[0]), torch.empty_like(v0[0])
    F1 = [torch.empty_like(v0[0]) for _ in range(3)]
    F3 = [torch.empty_like(v0[0]) for _ in range(3)]
    g = [torch.empty_like(v0[0]) for _ in range(3)]
    xs = [torch.zeros_like(v0[0]) for _ in range(3)]
    psi = torch.zeros(mp.ndof, dtype=torch.float64, device=dev)
    op = dg.default_opts(precond=dg.DG_PC_FDM)
    out = {"ndof_velocity": N, "ndof_pressure": mp.ndof}
    for name, ov in (("fp64", dg.default_opts()), ("mixed", dg.default_opts(precision=dg.DG_MIXED))):
        times, tterms = [], []
        for r in range(reps + 1):
            v = [c.clone() for c in v0]
            psi.zero_()
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ip = dg.dg_project(mv, mp, v, psi, opts=op)
            dg.dg_viscosity(mv, v, 1e-3, 1e-3, 2.0, nu2)
            dg.dg_viscosity(mv, u1, 1e-3, 1e-3, 2.0, nu1)
            dg.dg_viscous_terms(mv, nu1, u1, fd1=F1, fd3=F3)
            for k in range(3):
                dg.dg_lincomb(g[k], None, [lam, lam * dt * (aI - aE), -lam * dt * aE], [v[k], F1[k], F3[k]])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            iv = [dg.helmholtz_solve(mv, lam, nu2, 0.0, g[k], xs[k], ov) for k in range(3)]
            t2 = time.perf_counter()
            if r > 0:
                times.append(t2 - t0)
                tterms.append(t1 - t0)
        t = float(np.median(times))
        out[name] = dict(stage_ms=t * 1e3, projection_and_terms_ms=float(np.median(tterms)) * 1e3,
                         pressure_iters=ip["iters"], velocity_iters=[i["iters"] for i in iv],
                         velocity_true_rel_res=[i["true_rel_res"] for i in iv], stages_per_s=1.0 / t)
    mv.destroy()
    mp.destroy()
    return out


def convection_flops(P):
    """Algorithmic FP64 flops of the convective term per element (2 per
    multiply-add of the sum-factorised contractions): interpolation of three
    components to the Q^3 Gauss points, the nine transposed (i, k) passes back
    to the nodes, and per face the interpolation of six traces and the
    projection of three fluxes, Q = floor(3P/2) + 1."""
    n, Q = P + 1, 3 * P // 2 + 1
    interp = 3 * (n * n * Q * n + n * Q * Q * n + Q ** 3 * n)
    vol = 9 * (n * Q * Q * Q + n * n * Q * Q + n ** 3 * Q)
    faces = 6 * (6 * (n * Q * n + Q * Q * n) + 3 * (Q * n * Q + n * n * Q))
    return 2.0 * (interp + vol + faces)


def bench_imex_step(dg, torch, reps=3):
    """One full IMEX-RK step (Alg. 3) of the VVP vortex array on 16^3
    elements of degree 7 (pressure degree 6): RK-ARS3 and RK-CB3e,
    nu(v) = 0.01 + 0.01 (|v|/2)^2, dt = 2^-8 from the exact velocity at
    t = 0, the manufactured forcing at the stage times (evaluated once,
    before timing), the final projection, every solve FDM-preconditioned
    to 1e-10 (FP64 transforms; the *_fdm32 entries: FP32 transforms, CG
    still FP64 with the same stopping test); RK-ARS3 again with walls on
    every face carrying the exact velocity (VVD).  Also the convective term
    alone (HIP events on its stream) against the FP64 vector peak."""
    import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    spec = synth.mesh_spec("vvp_large")
    ps = dict(spec)
    ps["P"] = spec["P"] - 1
    mv, mp = dg.mesh_from_spec(spec, stream=stream), dg.mesh_from_spec(ps, stream=stream)
    N = mv.ndof
    X, Y, Z = dg.mesh_coordinates(mv)
    nu0 = nu1 = 0.01
    dt = 2.0 ** -8
    v0 = [c.contiguous() for c in synth.vvp_velocity(X, Y, Z, 0.0, xp=torch)]
    out = {"ndof_velocity": N, "ndof_pressure": mp.ndof, "elements": mv.nx * mv.ny * mv.nz, "dt": dt}
    opts = dg.default_opts(precond=dg.DG_PC_FDM)
    opts32 = dg.default_opts(precond=dg.DG_PC_FDM, precision=dg.DG_MIXED)
    def periodic_steps(methods):
        for method in methods:
            tab = dg.imex_tableau(method.split("_")[0])
            f = [[c.contiguous() for c in synth.vvp_forcing(X, Y, Z, tab.c[j] * dt, nu0, nu1, xp=torch)]
                 for j in range(tab.s)]
            times, info, v = [], None, None
            for r in range(reps + 1):
                v = [c.clone() for c in v0]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = dg.dg_imex_step(mv, mp, tab, dt, nu0, nu1, synth.VVP_VMAX, v, forcing=f,
                                       final_projection=True, opts=opts32 if method.endswith("_fdm32") else opts)
                torch.cuda.synchronize()
                if r > 0:
                    times.append(time.perf_counter() - t0)
            ve = synth.vvp_velocity(X, Y, Z, dt, xp=torch)
            err = max(float(torch.linalg.vector_norm(v[d] - ve[d]) / torch.linalg.vector_norm(ve[d]))
                      for d in range(3))
            t = float(np.median(times))
            out[method] = dict(step_ms=t * 1e3, steps_per_s=1.0 / t, stages=tab.s, solves=info["solves"],
                               pressure_iters=info["pressure_iters"], velocity_iters=info["velocity_iters"],
                               rel_error_vs_exact_after_one_step=err)

    periodic_steps(("RK-ARS3", "RK-CB3e"))
    # the same step with walls on every face carrying the exact velocity
    # (the VVD case): RK-ARS3 on the same elements with Dirichlet axes
    sw = dict(spec)
    sw["bc"] = (1, 1, 1)
    pw = dict(sw)
    pw["P"] = sw["P"] - 1
    mvw, mpw = dg.mesh_from_spec(sw, stream=stream), dg.mesh_from_spec(pw, stream=stream)
    tab = dg.imex_tableau("RK-ARS3")
    f = [[c.contiguous() for c in synth.vvp_forcing(X, Y, Z, tab.c[j] * dt, nu0, nu1, xp=torch)]
         for j in range(tab.s)]
    wl = [[c.contiguous() for c in synth.vvp_velocity(X, Y, Z, tab.c[j] * dt, xp=torch)] for j in range(tab.s)]
    times = []
    for r in range(reps + 1):
        v = [c.clone() for c in v0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = dg.dg_imex_step(mvw, mpw, tab, dt, nu0, nu1, synth.VVP_VMAX, v, forcing=f, wall=wl,
                               final_projection=True, opts=opts)
        torch.cuda.synchronize()
        if r > 0:
            times.append(time.perf_counter() - t0)
    ve = synth.vvp_velocity(X, Y, Z, dt, xp=torch)
    err = max(float(torch.linalg.vector_norm(v[d] - ve[d]) / torch.linalg.vector_norm(ve[d])) for d in range(3))
    t = float(np.median(times))
    out["RK-ARS3_walls"] = dict(step_ms=t * 1e3, steps_per_s=1.0 / t, stages=tab.s, solves=info["solves"],
                                pressure_iters=info["pressure_iters"], velocity_iters=info["velocity_iters"],
                                rel_error_vs_exact_after_one_step=err)
    mvw.destroy()
    mpw.destroy()
    # RK-ARS3 on the vortex array at 32^3 elements of degree 7 (16.8M nodes
    # per component, the size of the apply's mesh)
    v32 = synth.vertices_uniform(32, -0.5, 0.5)
    sl = dict(nx=32, ny=32, nz=32, P=7, xv=v32, yv=v32.copy(), zv=v32.copy(), bc=(0, 0, 0))
    pl = dict(sl)
    pl["P"] = sl["P"] - 1
    mvl, mpl = dg.mesh_from_spec(sl, stream=stream), dg.mesh_from_spec(pl, stream=stream)
    XL, YL, ZL = dg.mesh_coordinates(mvl)
    tab = dg.imex_tableau("RK-ARS3")
    dtl = 2.0 ** -9
    fl = [[c.contiguous() for c in synth.vvp_forcing(XL, YL, ZL, tab.c[j] * dtl, nu0, nu1, xp=torch)]
          for j in range(tab.s)]
    vl0 = [c.contiguous() for c in synth.vvp_velocity(XL, YL, ZL, 0.0, xp=torch)]
    for name, ol in (("RK-ARS3_32cubed", opts), ("RK-ARS3_32cubed_fdm32", opts32)):
        times = []
        for r in range(3):
            v = [c.clone() for c in vl0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = dg.dg_imex_step(mvl, mpl, tab, dtl, nu0, nu1, synth.VVP_VMAX, v, forcing=fl,
                                   final_projection=True, opts=ol)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
        ve = synth.vvp_velocity(XL, YL, ZL, dtl, xp=torch)
        err = max(float(torch.linalg.vector_norm(v[d] - ve[d]) / torch.linalg.vector_norm(ve[d])) for d in range(3))
        t = float(np.median(times))
        out[name] = dict(ndof_velocity=mvl.ndof, dt=dtl, step_ms=t * 1e3, steps_per_s=1.0 / t,
                         solves=info["solves"], pressure_iters=info["pressure_iters"],
                         velocity_iters=info["velocity_iters"], rel_error_vs_exact_after_one_step=err)
    del fl, vl0, v, ve, XL, YL, ZL
    mvl.destroy()
    mpl.destroy()
    # the periodic steps with the FP32 transforms for the velocity solves
    periodic_steps(("RK-ARS3_fdm32", "RK-CB3e_fdm32"))
    # the convective term alone
    o = [torch.empty_like(v0[0]) for _ in range(3)]
    for _ in range(3):
        dg.dg_convection(mv, v0, o, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    for e0, e1 in ev:
        e0.record(stream)
        dg.dg_convection(mv, v0, o, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    durs = np.array([a.elapsed_time(c) * 1e-3 for a, c in ev])
    tc = float(np.median(durs))
    nel = spec["nx"] * spec["ny"] * spec["nz"]
    flops = convection_flops(spec["P"]) * nel
    # flops: the algorithmic count of the direct sum-factorised contractions;
    # the kernel's even-odd contractions execute about 0.55 of its
    # multiply-adds (plus the sums and differences of mirrored values)
    out["convection"] = {"bound": "alu", "achieved": flops / tc / 1e12, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": flops / tc / 1e12 / FP64_PEAK_TFLOPS,
                         "flops_counted": "algorithmic (direct sum factorisation)",
                         "flops_per_launch": flops, "us_median": tc * 1e6,
                         "gauss_points_per_direction": 3 * spec["P"] // 2 + 1}
    mv.destroy()
    mp.destroy()
    return out


def bench_serving(dg, nreq, slots, precision, budget=96 << 30, precond=0, rate=200.0):
    """Real-time replay of the request stream (Poisson arrivals, 200/s; a
    larger rate replays the same requests faster, to find the capacity)."""
    import synth
    stream = synth.serving_stream(rate=rate)[:nreq]
    srv = dg.Server(budget, slots)
    t0 = time.perf_counter()
    ids = []
    for r in stream:
        wait = r["t_arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        ids.append(srv.submit(r["n"], r["P"], r["lam"], None, is_poisson=r["poisson"],
                              rhs_seed=r["rhs_seed"], precision=precision, precond=precond))
    # wait for the backlog, reporting progress
    last = time.perf_counter()
    while srv.stats()["completed"] < len(ids) and time.perf_counter() - t0 < 3600.0:
        time.sleep(0.2)
        if time.perf_counter() - last > 30.0:
            last = time.perf_counter()
            log("  serving: %d / %d done after %.0f s" % (srv.stats()["completed"], len(ids),
                                                          last - t0))
    srv.drain()
    st = srv.stats()
    bad = []
    for r, i in zip(stream, ids):
        try:
            rc, info = srv.poll(i)
        except dg.DGError as e:
            rc, info = e.status, dict(iters=-1, outer_iters=-1, true_rel_res=-1.0)
        if rc != 0:
            bad.append(dict(id=r["id"], status=rc, n=r["n"], P=r["P"], poisson=r["poisson"],
                            lam=r["lam"], iters=info["iters"], outer=info["outer_iters"],
                            rel_res=info["true_rel_res"]))
    srv.destroy()
    ndof = sum(r["n"] ** 3 * (r["P"] + 1) ** 3 for r in stream)
    st.update(requests=nreq, slots=slots, precision="mixed" if precision else "fp64",
              precond="fdm" if precond else "jacobi",
              solves_per_s=nreq / st["makespan"], failed=len(bad), failures=bad[:20],
              offered_per_s=nreq / max(stream[-1]["t_arrival"], 1e-9), mean_ndof=ndof / nreq)
    # served rate over offered rate: below 1 the queue grew for the whole
    # replay and solves_per_s is the capacity; near 1 the server kept up
    st["served_over_offered"] = st["solves_per_s"] / st["offered_per_s"]
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="apply only (for profiling runs)")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs after the apply: solve, poisson, solve_mixed, "
                         "poisson_mixed, mixed_small, batched, serving (default all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=60,
                    help="prefix of the 2000-request stream replayed per serving mode")
    ap.add_argument("--serving-modes",
                    default="fifo_fp64,continuous_fp64,continuous_mixed,continuous_fdm,continuous_fdm_10x_rate",
                    help="serving modes to replay")
    ap.add_argument("--serving-fdm-requests", type=int, default=2000,
                    help="requests replayed in the fast-diagonalisation serving mode")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one GPU "
              "(the apply would shard by z-slabs of elements with a one-layer halo)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2112_04167_amd as dg
    import synth

    if args.calib_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 5 x 1 GiB read + 1 GiB write")
        del a, b
    spec = synth.mesh_spec("stretched_large")
    lam = synth.large_helmholtz_lambda()
    log("apply: %d steps, %d warmup" % (args.steps, args.warmup))
    N, elapsed, durs = bench_apply(dg, torch, spec, lam, args.steps, args.warmup)
    avg = float(durs.mean())
    value = N * args.steps / elapsed / 1e9
    achieved = APPLY_BYTES_PER_DOF_FP64 * N / avg / 1e9
    traffic = measured_traffic()
    out = {
        "metric": "GDOF/s Helmholtz apply; solves/s and p99 latency at 1e-10 rel. residual",
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform random x in [-1,1])",
        "config": {"workload": "SIP-DG Helmholtz apply, 32^3 hex elements, P=7 (16.8M nodes), "
                               "tanh z-stretching 1.5, Dirichlet z / periodic x,y, "
                               "lambda=2294280.47, nu=1",
                   "elements": [32, 32, 32], "P": 7, "ndof": N, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_apply<7,double,false,0,true>",
                     "kernel_avg_us": avg * 1e6, "kernel_min_us": float(durs.min()) * 1e6,
                     "algorithmic_bytes_per_launch": APPLY_BYTES_PER_DOF_FP64 * N},
    }
    flops = measured_flops()
    if flops is not None:
        # the FP64 rate of the same kernel against the chip's FP64 vector peak
        tf = flops / avg / 1e12
        out["flops"] = {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP64_PEAK_TFLOPS, "flops_per_launch": flops,
                        "counter": "SQ_INSTS_VALU_FLOPS_FP64 x 64"}
    legs = set(("fdm", "solve", "poisson", "solve_fdm", "poisson_fdm", "solve_mixed", "poisson_mixed",
                "mixed_small", "batched", "stage", "stage_varnu", "imex_step", "serving")
               if args.legs == "all" else args.legs.split(","))
    if not args.quick:
        if "fdm" in legs:
            log("fast-diagonalisation inverse")
            out["fdm"] = bench_fdm(dg, torch, spec, lam)
        xref = {}
        if "solve" in legs:
            log("FP64 Helmholtz solve")
            out["solve"] = bench_solve(dg, torch, spec, lam, synth.SEEDS["large_helmholtz"], reps=5)
            xref["solve"] = out["solve"].pop("x")
        if "poisson" in legs:
            log("Poisson solve")
            out["poisson"] = bench_solve(dg, torch, spec, 0.0, synth.SEEDS["large_poisson"], reps=1,
                                         poisson=True)
            xref["poisson"] = out["poisson"].pop("x")
        if "solve_fdm" in legs:
            log("Helmholtz solve, fast-diagonalisation preconditioner")
            out["solve_fdm"] = bench_solve(dg, torch, spec, lam, synth.SEEDS["large_helmholtz"], reps=10,
                                           precond=dg.DG_PC_FDM, ref=xref.get("solve"))
            out["solve_fdm"].pop("x")
            if "solve" in out:
                out["solve_fdm"]["speedup_vs_jacobi_fp64"] = (out["solve"]["seconds_median"] /
                                                              out["solve_fdm"]["seconds_median"])
        if "poisson_fdm" in legs:
            log("Poisson solve, fast-diagonalisation preconditioner")
            out["poisson_fdm"] = bench_solve(dg, torch, spec, 0.0, synth.SEEDS["large_poisson"], reps=10,
                                             poisson=True, precond=dg.DG_PC_FDM, ref=xref.get("poisson"))
            out["poisson_fdm"].pop("x")
            if "poisson" in out:
                out["poisson_fdm"]["speedup_vs_jacobi_fp64"] = (out["poisson"]["seconds_median"] /
                                                                out["poisson_fdm"]["seconds_median"])
        xref.clear()
        if "solve_mixed" in legs:
            log("mixed-precision Helmholtz solve (same mesh)")
            out["solve_mixed"] = bench_mixed_large(dg, torch, spec, lam)
        if "poisson_mixed" in legs:
            log("mixed-precision Poisson solve (same mesh)")
            out["poisson_mixed"] = bench_mixed_large(dg, torch, spec, 0.0, poisson=True)
        if "mixed_small" in legs:
            log("mixed-precision small solves")
            out["mixed_small"] = bench_mixed_small(dg, torch)
        if "batched" in legs:
            log("batched stage solve")
            out["batched"] = bench_batched(dg, torch)
        if "stage" in legs:
            log("implicit stage: projection + three velocity solves")
            out["stage"] = bench_stage(dg, torch)
        if "stage_varnu" in legs:
            log("variable-viscosity implicit stage")
            out["stage_varnu"] = bench_stage_varnu(dg, torch)
        if "imex_step" in legs:
            log("full IMEX-RK step (VVP vortex array)")
            out["imex_step"] = bench_imex_step(dg, torch)
        if args.serving_requests > 0 and "serving" in legs:
            out["serving"] = {}
            for name, slots, prec, pc, nreq in (
                    ("fifo_fp64", 1, dg.DG_FP64, 0, args.serving_requests),
                    ("continuous_fp64", 8, dg.DG_FP64, 0, args.serving_requests),
                    ("continuous_mixed", 8, dg.DG_MIXED, 0, args.serving_requests),
                    ("continuous_fdm", 8, dg.DG_FP64, dg.DG_PC_FDM, args.serving_fdm_requests),
                    ("continuous_fdm_10x_rate", 8, dg.DG_FP64, dg.DG_PC_FDM, args.serving_fdm_requests)):
                if name not in args.serving_modes.split(",") or nreq <= 0:
                    continue
                log("serving:", name, nreq, "requests")
                out["serving"][name] = bench_serving(dg, nreq, slots, prec, precond=pc,
                                                     rate=2000.0 if name.endswith("10x_rate") else 200.0)
        if not args.no_cpu:
            log("CPU oracle baseline")
            out["cpu_baseline"] = cpu_baseline(spec, lam)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
