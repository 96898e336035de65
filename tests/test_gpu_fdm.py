"""GPU parity of the fast-diagonalisation inverse (helmholtz_fdm_apply, FP64
MFMA transforms along the mesh lines) and of CG preconditioned by it
(opts.precond = DG_PC_FDM, with FP64 or, for precision DG_MIXED, FP32
transforms) against the oracle.

Bars: the inverse against the oracle's own fast diagonalisation (numpy
eigendecompositions, independent of the library's host eigensolver)
<= 1e-11 relative, on shapes whose line lengths L = n_d (P+1) are and are not
multiples of the 16-row MFMA tiles; solves against the exact discrete
solution x* <= 1e-10 (with either precision of the transforms: CG is FP64
with the same stopping test); iteration-locked runs with a nodal nu against
the oracle's PCG with the same preconditioner <= 1e-11."""
import numpy as np
import pytest

import synth
from oracle import dense, kron, naive, pcg
from tests.gpu_util import say, to_dev, torch_dev
from tests.helpers import make_spec, ndof, manufactured_u, channel_nu

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gpu_fdm(spec, lam, nu, b, is_poisson=False):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    mesh = dg.mesh_from_spec(spec)
    bd = to_dev(b)
    xd = torch.full_like(bd, np.nan)   # every output value must be written
    dg.helmholtz_fdm_apply(mesh, lam, nu, bd, xd, is_poisson=is_poisson)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    mesh.destroy()
    return x


def gpu_solve(spec, lam, nu, f, poisson=False, x0=None, **opts):
    import paper_2112_04167_amd as dg
    torch, dev = torch_dev()
    mesh = dg.mesh_from_spec(spec)
    fd = to_dev(f)
    xd = torch.zeros_like(fd) if x0 is None else to_dev(np.asarray(x0, dtype=np.float64))
    o = dg.default_opts(precond=dg.DG_PC_FDM, **opts)
    if poisson:
        info = dg.poisson_solve(mesh, fd, xd, o, raise_on_error=False)
    else:
        nud = None if np.isscalar(nu) else to_dev(nu)
        info = dg.helmholtz_solve(mesh, lam, nud, nu if np.isscalar(nu) else 0.0, fd, xd, o,
                                  raise_on_error=False)
    x = xd.cpu().numpy()
    mesh.destroy()
    return x, info


# (elements, P, bc, tanh-z, lambda, nu): L = n_d (P+1) from 5 to 63, padded
# to 16-row tiles; P = 7 with 4 column tiles per bundle, P = 8 with 81
# columns in two chunks (4 tiles, then 1 of 17 columns)
CASES = [((4, 4, 4), 4, (0, 0, 0), False, 1.0, 1.0),
         ((5, 3, 7), 7, (0, 0, 1), True, 30.0, 1.0),
         ((3, 2, 5), 5, (1, 2, 0), True, 2.0, 0.3),
         ((2, 3, 1), 8, (0, 1, 2), False, 0.5, 2.0),
         ((6, 1, 2), 3, (2, 0, 1), False, 4.0, 1.0),
         ((7, 2, 3), 6, (1, 1, 1), True, 0.0, 1.0)]


@pytest.mark.parametrize("case", CASES, ids=["P4_periodic", "P7_stretched", "P5_mixed_bc", "P8_chunks",
                                             "P3_n1", "P6_dirichlet_lam0"])
def test_fdm_inverse_matches_oracle(case):
    n, P, bc, st, lam, nu = case
    spec = make_spec(n, P, bc, st)
    b = synth.uniform_field(ndof(spec), 50 + P)
    x = gpu_fdm(spec, lam, nu, b)
    xo = kron.FDM(spec, lam, nu).apply_inverse(b)
    say("fdm inverse", case, rel(x, xo))
    assert np.all(np.isfinite(x))
    assert rel(x, xo) <= 1e-11


def test_fdm_inverse_singular_poisson():
    # the Poisson BC mapping (Dirichlet -> Neumann) and the dropped constant
    # mode: b with zero sum gives the M-mean-zero solution of A x = b
    spec = make_spec((3, 3, 2), 6, (0, 1, 0), False)
    b = synth.uniform_field(ndof(spec), 61)
    b -= b.mean()
    x = gpu_fdm(spec, 0.0, 1.0, b, is_poisson=True)
    pspec = dict(spec)
    pspec["bc"] = (0, 2, 0)
    xs = kron.FDM(pspec, 0.0).solve(b)
    M = dense.mass_diag(pspec)
    say("fdm singular", rel(x, xs), np.dot(M, x))
    assert rel(x, xs) <= 1e-11
    assert abs(np.dot(M, x)) <= 1e-11 * np.linalg.norm(x) * np.sqrt(M.sum())


def test_fdm_inverse_full_size_stretched():
    # 32^3, P = 7 (L = 256 per axis, 16.8M nodes) with the tanh-z grading
    spec = synth.mesh_spec("stretched_large")
    lam = synth.large_helmholtz_lambda()
    b = synth.uniform_field(ndof(spec), 7)
    x = gpu_fdm(spec, lam, 1.0, b)
    xo = kron.FDM(spec, lam).apply_inverse(b)
    say("fdm full size", rel(x, xo))
    assert rel(x, xo) <= 1e-11


def test_fdm_pcg_small_periodic_manufactured():
    spec = synth.mesh_spec("small_periodic")
    lam = 1.0
    f = (lam + 12 * np.pi ** 2) * manufactured_u(spec) + synth.uniform_field(ndof(spec), 0)
    x, info = gpu_solve(spec, lam, 1.0, f)
    xs = kron.FDM(spec, lam).solve(dense.mass_diag(spec) * f)
    say("fdm pcg small", info, rel(x, xs))
    assert info["status"] == 0 and info["iters"] <= 2
    assert info["true_rel_res"] <= 1e-10 and rel(x, xs) <= 1e-10


@pytest.mark.parametrize("poisson", [False, True])
def test_fdm_pcg_stretched_large_full_size(poisson):
    # the 32^3, P = 7 stretched systems: Jacobi-PCG needs 36 (Helmholtz) and
    # 2738 (Poisson, kappa 5.9e6) iterations; the exact preconditioner one
    spec = synth.mesh_spec("stretched_large")
    if poisson:
        f = synth.uniform_field(ndof(spec), synth.SEEDS["large_poisson"])
        lam = 0.0
        pspec = dict(spec)
        pspec["bc"] = (0, 0, 2)
    else:
        f = synth.uniform_field(ndof(spec), synth.SEEDS["large_helmholtz"])
        lam = synth.large_helmholtz_lambda()
        pspec = spec
    x, info = gpu_solve(spec, lam, 1.0, f, poisson=poisson)
    M = dense.mass_diag(pspec)
    xs = kron.FDM(pspec, lam).solve(M * f)
    say("fdm pcg large poisson=%s" % poisson, info, "err vs x*", rel(x, xs))
    assert info["status"] == 0 and info["iters"] <= 3
    assert info["true_rel_res"] <= 1e-10 and rel(x, xs) <= 1e-10
    if poisson:
        assert abs(np.dot(M, x)) <= 1e-12 * np.linalg.norm(x) * np.sqrt(M.sum())


@pytest.mark.parametrize("k", [2, 5])
def test_fdm_pcg_nodal_nu_iteration_locked(k):
    # nodal nu: the preconditioner is the inverse for nu_ref = sqrt(min max);
    # k steps locked to the oracle's PCG with the same preconditioner
    spec = make_spec((3, 3, 2), 5, (0, 0, 1), False)
    nu = channel_nu(spec)
    lam = synth.batched_lambda()
    f = synth.uniform_field(ndof(spec), 41)
    x, info = gpu_solve(spec, lam, nu, f, fixed_iters=k)
    assert info["iters"] == k
    op = naive.Operator(spec, lam, nu)
    M = dense.mass_diag(spec)
    F = kron.FDM(spec, lam, np.sqrt(nu.min() * nu.max()))
    xo, _ = pcg.pcg(op.apply, M * f, op.diag(), M, fixed_iters=k, precond=F.apply_inverse)
    say("fdm locked", k, rel(x, xo))
    assert rel(x, xo) <= 1e-11


def test_fdm_pcg_channel_velocity_full_size():
    # the 24^3, P = 5 channel velocity system (nodal nu, max/min = 3)
    spec = synth.mesh_spec("batched_channel")
    nu = channel_nu(spec)
    lam = synth.batched_lambda()
    f = synth.uniform_field(ndof(spec), synth.SEEDS["batched_velocity"][0])
    x, info = gpu_solve(spec, lam, nu, f)
    op = naive.Operator(spec, lam, nu)
    M = dense.mass_diag(spec)
    xo, io = pcg.pcg(op.apply, M * f, op.diag(), M, tol=1e-10)
    say("fdm channel velocity", info, "jacobi oracle iters", io["iters"], rel(x, xo))
    assert info["status"] == 0 and info["iters"] <= 18
    assert pcg.true_rel_res(op.apply, x, M * f, M) <= 1.2e-10
    assert rel(x, xo) <= 1e-10


def test_fdm_pcg_initial_guess_and_errors():
    import paper_2112_04167_amd as dg
    spec = make_spec((3, 2, 3), 5, (0, 1, 0), True)
    lam = 3.0
    f = synth.uniform_field(ndof(spec), 91)
    xs = kron.FDM(spec, lam).solve(dense.mass_diag(spec) * f)
    xe, ie = gpu_solve(spec, lam, 1.0, f, x0=xs)
    assert ie["status"] == 0 and ie["iters"] == 0 and rel(xe, xs) <= 1e-12
    xf, iff = gpu_solve(spec, lam, 1.0, f, x0=10.0 * synth.uniform_field(ndof(spec), 93))
    assert iff["status"] == 0 and rel(xf, xs) <= 1e-10
    xm, im = gpu_solve(spec, lam, 1.0, f, precision=1)       # FP32 transforms
    assert im["status"] == 0 and rel(xm, xs) <= 1e-10
    long_line = make_spec((65, 1, 1), 7, (0, 0, 0), False)  # 520 nodes on an x line
    _, il = gpu_solve(long_line, lam, 1.0, synth.uniform_field(ndof(long_line), 1))
    assert il["rc"] == dg.DG_ERR_ARG


# the FP32 transforms: every CASES shape (line lengths from 5 to 63, all BC
# kinds, the P = 8 chunked bundles), plus the singular Poisson problem
@pytest.mark.parametrize("case", CASES, ids=["P4_periodic", "P7_stretched", "P5_mixed_bc", "P8_chunks",
                                             "P3_n1", "P6_dirichlet_lam0"])
def test_fdm32_pcg_matches_exact_solution(case):
    n, P, bc, st, lam, nu = case
    spec = make_spec(n, P, bc, st)
    f = synth.uniform_field(ndof(spec), 70 + P)
    x, info = gpu_solve(spec, lam, nu, f, precision=1)
    xs = kron.FDM(spec, lam, nu).solve(dense.mass_diag(spec) * f)
    say("fdm32 pcg", case, info, rel(x, xs))
    # FP32 transforms: no longer exact, but within a few iterations
    assert info["status"] == 0 and 2 <= info["iters"] <= 8
    assert info["true_rel_res"] <= 1e-10 and rel(x, xs) <= 1e-10


def test_fdm32_pcg_singular_poisson():
    spec = make_spec((3, 3, 2), 6, (0, 1, 0), False)
    f = synth.uniform_field(ndof(spec), 62)
    x, info = gpu_solve(spec, 0.0, 1.0, f, poisson=True, precision=1)
    pspec = dict(spec)
    pspec["bc"] = (0, 2, 0)
    M = dense.mass_diag(pspec)
    xs = kron.FDM(pspec, 0.0).solve(M * f)
    say("fdm32 singular", info, rel(x, xs))
    assert info["status"] == 0 and info["iters"] <= 8
    assert rel(x, xs) <= 1e-10
    assert abs(np.dot(M, x)) <= 1e-12 * np.linalg.norm(x) * np.sqrt(M.sum())


@pytest.mark.parametrize("poisson", [False, True])
def test_fdm32_pcg_stretched_large_full_size(poisson):
    # the 32^3, P = 7 systems (L = 256 per axis) with FP32 transforms
    spec = synth.mesh_spec("stretched_large")
    if poisson:
        f = synth.uniform_field(ndof(spec), synth.SEEDS["large_poisson"])
        lam = 0.0
        pspec = dict(spec)
        pspec["bc"] = (0, 0, 2)
    else:
        f = synth.uniform_field(ndof(spec), synth.SEEDS["large_helmholtz"])
        lam = synth.large_helmholtz_lambda()
        pspec = spec
    x, info = gpu_solve(spec, lam, 1.0, f, poisson=poisson, precision=1)
    M = dense.mass_diag(pspec)
    xs = kron.FDM(pspec, lam).solve(M * f)
    say("fdm32 pcg large poisson=%s" % poisson, info, "err vs x*", rel(x, xs))
    assert info["status"] == 0 and info["iters"] <= 8
    assert info["true_rel_res"] <= 1e-10 and rel(x, xs) <= 1e-10


def test_fdm32_pcg_channel_velocity_full_size():
    # nodal nu (max/min = 3): the FP32 transforms cost at most one more
    # iteration than the FP64 ones here
    spec = synth.mesh_spec("batched_channel")
    nu = channel_nu(spec)
    lam = synth.batched_lambda()
    f = synth.uniform_field(ndof(spec), synth.SEEDS["batched_velocity"][0])
    x64, i64 = gpu_solve(spec, lam, nu, f)
    x32, i32 = gpu_solve(spec, lam, nu, f, precision=1)
    op = naive.Operator(spec, lam, nu)
    M = dense.mass_diag(spec)
    say("fdm32 channel velocity", i64["iters"], i32["iters"], rel(x32, x64))
    assert i32["status"] == 0 and i32["iters"] <= i64["iters"] + 1
    assert pcg.true_rel_res(op.apply, x32, M * f, M) <= 1.2e-10
    assert rel(x32, x64) <= 2e-10


@pytest.mark.parametrize("ntc", [1, 2, 4])
def test_fdm_inverse_every_tile_shape(ntc, tmp_path):
    # every transform tile shape the autotuner may choose (1, 2 or 4 column
    # tiles per work-group), forced through the tuning cache in a fresh
    # process (the cache is read once per process), against the oracle
    import json
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, os.path.join(here, "fdm_forced_tiles.py"), str(tmp_path / "tune.txt"),
                        str(ntc)], capture_output=True, text=True, timeout=240)
    say("forced tiles", ntc, r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0
    lines = [json.loads(s) for s in r.stdout.splitlines() if s.startswith("{")]
    assert len(lines) == 4
    for c in lines:
        assert c["rel"] <= 1e-11, c
