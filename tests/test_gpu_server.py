"""GPU tests of the continuous-batching request server.

  * results match the oracle's exact discrete solution (fast diagonalisation;
    periodic cube, nu = 1) to <= 1e-10 relative, Helmholtz and singular
    Poisson requests alike; mixed-precision results are held to the
    refinement tolerance on the oracle-recomputed collocation residual
    (<= 1e-10, x 1.2 for the recomputation's rounding) and, in error, to the
    measured value with a margin, kappa stated (1.55e-10 at kappa = 3.5e3);
  * the device right-hand-side generator (SplitMix64) reproduces the host
    implementation of the same published generator bit for bit;
  * a request's result is the same alone and in a mix of concurrent
    requests (bitwise: the solve's arithmetic does not depend on the other
    work on the device);
  * admission respects the HBM budget, and over-budget requests are refused;
  * latency statistics are recorded."""
import numpy as np
import pytest

import synth
from oracle import dense, kron, naive, pcg
from tests.gpu_util import say, torch_dev
from tests.helpers import make_spec

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def exact(n, P, lam, f):
    spec = make_spec(n, P, (0, 0, 0))
    M = dense.mass_diag(spec)
    return kron.FDM(spec, lam).solve(M * f)


def kappa(n, P, lam):
    ev = kron.FDM(make_spec(n, P, (0, 0, 0)), lam).eigenvalues_generalized()
    return ev[-1] / ev[0]


def server(budget=8 << 30, slots=4):
    import paper_2112_04167_amd as dg
    torch_dev()
    return dg.Server(budget, slots)


def test_server_results_against_oracle():
    srv = server()
    reqs = [(3, 4, 10.0, False), (4, 3, 1e4, False), (2, 6, 0.0, True), (3, 5, 1.0, False),
            (2, 8, 0.0, True), (5, 3, 300.0, False)]
    ids, fs = [], []
    for k, (n, P, lam, pois) in enumerate(reqs):
        f = synth.uniform_field(n ** 3 * (P + 1) ** 3, 100 + k)
        fs.append(f)
        ids.append(srv.submit(n, P, lam, f, is_poisson=pois, keep_result=True))
    srv.drain()
    for k, (n, P, lam, pois) in enumerate(reqs):
        rc, info = srv.poll(ids[k])
        assert rc == 0, (k, info)
        x = srv.fetch(ids[k], n ** 3 * (P + 1) ** 3)
        e = rel(x, exact(n, P, lam, fs[k]))
        say("server req", k, info["iters"], "kappa", kappa(n, P, lam), "err vs x*", e)
        assert e <= 1e-10
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["p99"] >= st["p50"] > 0
    srv.destroy()


def test_server_device_rhs_generator():
    srv = server()
    n, P, lam, seed = 3, 4, 7.0, 987654321
    rid = srv.submit(n, P, lam, None, rhs_seed=seed, keep_result=True)
    srv.drain()
    rc, info = srv.poll(rid)
    assert rc == 0
    x = srv.fetch(rid, n ** 3 * (P + 1) ** 3)
    f = synth.splitmix64_uniform(n ** 3 * (P + 1) ** 3, seed)
    assert rel(x, exact(n, P, lam, f)) <= 1e-10
    srv.destroy()


@pytest.mark.parametrize("precision", [0, 1])
def test_server_same_alone_and_in_the_mix(precision):
    n, P, lam, seed = 6, 5, 50.0, 4242
    N = n ** 3 * (P + 1) ** 3
    srv = server(slots=1)
    rid = srv.submit(n, P, lam, None, rhs_seed=seed, keep_result=True, precision=precision)
    srv.drain()
    alone = srv.fetch(rid, N)
    srv.destroy()
    srv = server(slots=6)
    others = []
    stream = synth.serving_stream(nreq=16, nmax=12)
    for r in stream[:8]:
        others.append(srv.submit(r["n"], r["P"], r["lam"], None, is_poisson=r["poisson"],
                                 rhs_seed=r["rhs_seed"], precision=precision))
    rid = srv.submit(n, P, lam, None, rhs_seed=seed, keep_result=True, precision=precision)
    for r in stream[8:]:
        others.append(srv.submit(r["n"], r["P"], r["lam"], None, is_poisson=r["poisson"],
                                 rhs_seed=r["rhs_seed"], precision=precision))
    srv.drain()
    mixed = srv.fetch(rid, N)
    st = srv.stats()
    say("mix stats", st)
    assert st["peak_active"] > 1        # the work really overlapped
    assert np.array_equal(alone, mixed)
    for o in others:
        assert srv.poll(o)[0] == 0
    f = synth.splitmix64_uniform(N, seed)
    if precision == 0:
        assert rel(mixed, exact(n, P, lam, f)) <= 1e-10
    else:
        # mixed mode is held to its refinement tolerance: the collocation
        # residual recomputed by the oracle; the error follows through the
        # conditioning of the operator
        spec = make_spec(n, P, (0, 0, 0))
        M = dense.mass_diag(spec)
        op = naive.Operator(spec, lam, 1.0)
        assert pcg.true_rel_res(op.apply, mixed, M * f, M) <= 1.2e-10
        # kappa(M^-1 A) = 3.5e3: at the 1e-10 residual the mixed result is
        # measured 1.55e-10 from x* (its FP32 recurrence leaves more of the
        # residual in low modes than FP64 CG does); bound with a margin
        say("mixed in the mix: kappa", kappa(n, P, lam), "err vs x*", rel(mixed, exact(n, P, lam, f)))
        assert rel(mixed, exact(n, P, lam, f)) <= 2.5e-10
    srv.destroy()


def test_server_admission_budget():
    import paper_2112_04167_amd as dg
    # a budget that holds about two requests of this size at a time
    n, P = 8, 5
    N = n ** 3 * (P + 1) ** 3
    # FP64 request: rhs, x and the five CG work vectors, plus small tables
    per_req = 7 * N * 8 + (1 << 16)
    budget = int(2.5 * per_req)
    srv = server(budget=budget, slots=8)
    ids = [srv.submit(n, P, 20.0 + k, None, rhs_seed=k) for k in range(6)]
    srv.drain()
    st = srv.stats()
    say("budget stats", st, budget)
    assert st["completed"] == 6
    assert st["peak_bytes"] <= budget
    assert st["peak_active"] <= 2
    for i in ids:
        assert srv.poll(i)[0] == 0
    with pytest.raises(dg.DGError) as e:
        srv.submit(40, 8, 1.0, None, rhs_seed=1)
    assert e.value.status == dg.DG_ERR_BUDGET
    srv.destroy()


def test_server_held_results_do_not_stall_drain():
    # kept results fill the arena: a request that no longer fits while nothing
    # runs fails with DG_ERR_BUDGET instead of waiting for a fetch, so drain()
    # returns; after a fetch frees memory the same request is served again
    import paper_2112_04167_amd as dg
    n, P = 6, 5
    N = n ** 3 * (P + 1) ** 3
    xb = ((N * 8 + 255) // 256) * 256
    probe = dg.mesh_from_spec(make_spec(n, P, (0, 0, 0)))
    ws = probe.footprint(dg.DG_FP64)
    probe.destroy()
    # one request takes geometry + workspace + rhs + x (= ws + 2 xb + small);
    # every finished request keeps its x (xb): two results fit, a third does not
    budget = ws + int(3.5 * xb) + (1 << 16)
    srv = server(budget=budget, slots=1)
    ids = [srv.submit(n, P, 10.0 + k, None, rhs_seed=k, keep_result=True) for k in range(3)]
    srv.drain()
    def status(i):
        try:
            return srv.poll(i)[0]
        except dg.DGError as e:   # the binding raises on a failed request
            return e.status

    st = [status(i) for i in ids]
    say("held-result statuses", st, budget)
    assert st[0] == 0 and st[1] == 0 and st[2] == dg.DG_ERR_BUDGET
    x0 = srv.fetch(ids[0], N)
    assert np.all(np.isfinite(x0))
    with pytest.raises(dg.DGError):   # fetched once: no second copy
        srv.fetch(ids[0], N)
    rid = srv.submit(n, P, 12.0, None, rhs_seed=2, keep_result=True)
    srv.drain()
    assert srv.poll(rid)[0] == 0
    f = synth.splitmix64_uniform(N, 2)
    assert rel(srv.fetch(rid, N), exact(n, P, 12.0, f)) <= 1e-10
    srv.destroy()


def test_server_fdm_requests_against_oracle():
    # requests solved by CG with the fast-diagonalisation preconditioner
    # (FP64): Helmholtz and singular Poisson requests within 1e-10 of x*, in
    # one or two iterations; a mixed-precision FDM request is refused
    import paper_2112_04167_amd as dg
    srv = server(slots=4)
    reqs = [(3, 4, 10.0, False), (5, 3, 0.0, True), (4, 7, 1e4, False), (6, 8, 0.0, True), (2, 5, 1.0, False)]
    ids, fs = [], []
    for k, (n, P, lam, pois) in enumerate(reqs):
        f = synth.uniform_field(n ** 3 * (P + 1) ** 3, 200 + k)
        fs.append(f)
        ids.append(srv.submit(n, P, lam, f, is_poisson=pois, keep_result=True, precond=dg.DG_PC_FDM))
    srv.drain()
    for k, (n, P, lam, pois) in enumerate(reqs):
        rc, info = srv.poll(ids[k])
        assert rc == 0, (k, info)
        x = srv.fetch(ids[k], n ** 3 * (P + 1) ** 3)
        e = rel(x, exact(n, P, lam, fs[k]))
        say("server fdm req", k, info["iters"], "err vs x*", e)
        assert info["iters"] <= 2 and e <= 1e-10
    with pytest.raises(dg.DGError):
        srv.submit(3, 4, 1.0, None, precision=dg.DG_MIXED, precond=dg.DG_PC_FDM)
    srv.destroy()
