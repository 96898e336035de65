"""Pins of the oracle's exact solvers and its PCG.

  * fast diagonalisation == dense Cholesky / bordered solve (tiny meshes);
  * manufactured u = sin(2 pi x) sin(2 pi y) sin(2 pi z) on the periodic cube:
    the exact discrete solution converges at order P+1 in the M-norm;
  * PCG with the collocation-residual stop of Sec. 4 reaches the exact
    discrete solution, runs exactly k iterations when asked, and reports the
    failure modes (not converged, non-finite data, loss of definiteness)."""
import numpy as np
import pytest

import synth
from oracle import dense, kron, naive, pcg
from tests.helpers import make_spec, ndof, manufactured_u


@pytest.mark.parametrize("n,P,bc,st,lam", [
    ((2, 2, 2), 3, (0, 0, 1), True, 2.0),
    ((2, 2, 2), 3, (0, 2, 0), False, 0.0),
    ((3, 3, 3), 2, (0, 0, 0), False, 0.0),
    ((2, 2, 2), 4, (1, 1, 1), False, 0.0),
    ((1, 2, 3), 3, (0, 1, 2), True, 1e3),
])
def test_fdm_matches_cholesky(n, P, bc, st, lam):
    s = make_spec(n, P, bc, st)
    b = np.random.default_rng(7).uniform(-1, 1, ndof(s))
    A = dense.assemble(s, lam, 1.0)
    xd = dense.solve(s, A, b, lam)
    xf = kron.FDM(s, lam).solve(b)
    assert np.linalg.norm(xd - xf) <= 1e-12 * np.linalg.norm(xd)
    bb = b - b.mean() if dense.singular(s, lam) else b
    assert np.linalg.norm(A @ xf - bb) <= 1e-11 * np.linalg.norm(bb)
    if dense.singular(s, lam):
        assert abs(np.dot(dense.mass_diag(s), xf)) <= 1e-13 * np.linalg.norm(xf)


@pytest.mark.parametrize("P", [3, 4])
def test_manufactured_convergence_order(P):
    errs = []
    lam = 1.0
    for n in (2, 4, 8):
        s = make_spec(n, P, (0, 0, 0))
        u = manufactured_u(s)
        f = (lam + 12 * np.pi ** 2) * u
        M = dense.mass_diag(s)
        x = kron.FDM(s, lam).solve(M * f)
        errs.append(np.sqrt(np.dot(M, (x - u) ** 2)))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc[-1] > P + 1 - 0.3, eoc


def test_manufactured_convergence_dirichlet_stretched():
    # homogeneous Dirichlet in z is exact for sin(2 pi z) on [0,1]; the tanh
    # grading needs n = 16 to reach the asymptotic rate
    P = 4
    errs = []
    for n in (4, 8, 16):
        s = make_spec(n, P, (0, 0, 1), zstretch=True)
        u = manufactured_u(s)
        lam = 10.0
        f = (lam + 12 * np.pi ** 2) * u
        M = dense.mass_diag(s)
        x = kron.FDM(s, lam).solve(M * f)
        errs.append(np.sqrt(np.dot(M, (x - u) ** 2)))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc[-1] > P + 1 - 0.5, eoc


def _setup(s, lam, nu=1.0, seed=0):
    op = naive.Operator(s, lam, nu)
    M = dense.mass_diag(s)
    f = synth.uniform_field(ndof(s), seed)
    return op, M, M * f


def test_pcg_reaches_exact_solution_small_periodic():
    s = synth.mesh_spec("small_periodic")
    op, M, b = _setup(s, 1.0)
    x, info = pcg.pcg(op.apply, b, op.diag(), M, tol=1e-10)
    assert info["status"] == pcg.OK
    assert 110 <= info["iters"] <= 150
    xs = kron.FDM(s, 1.0).solve(b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert pcg.true_rel_res(op.apply, x, b, M) <= 1e-10 * 1.5


def test_pcg_singular_poisson():
    s = make_spec((3, 3, 2), 3, (0, 2, 0), True)
    op, M, b = _setup(s, 0.0, seed=3)
    x, info = pcg.pcg(op.apply, b, op.diag(), M, tol=1e-11, singular=True)
    assert info["status"] == pcg.OK
    xs = kron.FDM(s, 0.0).solve(b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert abs(np.dot(M, x)) <= 1e-12 * np.linalg.norm(x)


def test_pcg_fixed_iterations_and_maxit():
    s = make_spec(2, 3, (0, 0, 0))
    op, M, b = _setup(s, 1.0)
    d = op.diag()
    _, info = pcg.pcg(op.apply, b, d, M, fixed_iters=7)
    assert info["iters"] == 7 and info["status"] == pcg.OK
    x, info = pcg.pcg(op.apply, b, d, M, tol=1e-12, maxit=3)
    assert info["status"] == pcg.NOT_CONVERGED and info["iters"] == 3
    assert np.all(np.isfinite(x))


def test_pcg_failure_modes():
    s = make_spec(2, 3, (0, 0, 0))
    op, M, b = _setup(s, 1.0)
    bad = b.copy()
    bad[5] = np.nan
    _, info = pcg.pcg(op.apply, bad, op.diag(), M)
    assert info["status"] == pcg.ERR_NONFINITE
    # a strongly negative lambda makes A indefinite: p^T A p <= 0 shows up
    opn, M, b = _setup(s, -1e4)
    d = np.abs(opn.diag())
    _, info = pcg.pcg(opn.apply, b, d, M)
    assert info["status"] == pcg.ERR_NOT_SPD


@pytest.mark.parametrize("lam", [1e2, 1e4, 1e6])
def test_iterative_refinement_reaches_exact_solution(lam):
    # FP64 refinement around FP32 PCG (kappa u_32 << 1 here: kappa = 2.5e3,
    # 26, 1.25 on the 4^3, P = 7 periodic mesh): the result is the exact
    # discrete solution to the FP64 bar, the recomputed residual meets the
    # rule, and each cycle gains at least inner_tol (1e-2; more when one CG
    # step overshoots it, as at kappa = 1.25), so three to six FP64 residuals
    # are needed for 1e-10
    spec = synth.mesh_spec("mixed_small")
    f = synth.uniform_field(ndof(spec), synth.SEEDS["mixed"])
    op = naive.Operator(spec, lam, 1.0)
    M = dense.mass_diag(spec)
    x, info = pcg.iterative_refinement(op.apply, M * f, op.diag(), M, tol=1e-10)
    assert info["status"] == pcg.OK
    assert 3 <= info["outer"] <= 7
    assert pcg.true_rel_res(op.apply, x, M * f, M) <= 1e-10
    xs = kron.FDM(spec, lam).solve(M * f)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_iterative_refinement_inner_solve_is_fp32():
    # one inner solve alone stops at FP32 accuracy: against the exact solution
    # it is off by ~1e-7 (the rounding of FP32 storage), not ~1e-15; and the
    # refinement with the same inner solve reaches 1e-10
    spec = make_spec((3, 3, 3), 4, (0, 0, 1), True)
    lam = 50.0
    f = synth.uniform_field(ndof(spec), 12)
    op = naive.Operator(spec, lam, 1.0)
    M = dense.mass_diag(spec)
    xs = kron.FDM(spec, lam).solve(M * f)
    x1, info1 = pcg.iterative_refinement(op.apply, M * f, op.diag(), M, tol=1e-10, inner_tol=1e-12,
                                         maxit=1)
    e1 = np.linalg.norm(x1 - xs) / np.linalg.norm(xs)
    assert info1["outer"] == 1 and 1e-9 < e1 < 1e-4
    x, info = pcg.iterative_refinement(op.apply, M * f, op.diag(), M, tol=1e-10, inner_tol=1e-3)
    assert info["status"] == pcg.OK and info["outer"] >= 2
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_iterative_refinement_singular_poisson():
    spec = make_spec((3, 2, 2), 3, (0, 2, 0), False)
    f = synth.uniform_field(ndof(spec), 13)
    op = naive.Operator(spec, 0.0, 1.0)
    M = dense.mass_diag(spec)
    x, info = pcg.iterative_refinement(op.apply, M * f, op.diag(), M, tol=1e-10, singular=True)
    assert info["status"] == pcg.OK
    xs = kron.FDM(spec, 0.0).solve(M * f)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert abs(np.dot(M, x)) <= 1e-13 * np.linalg.norm(x)


# ---- the fast-diagonalisation preconditioner (the exact inverse of the
# constant-nu operator on a Cartesian product mesh) ------------------------

@pytest.mark.parametrize("n,P,bc,st,lam,nu", [
    ((2, 3, 2), 3, (0, 0, 1), True, 2.0, 1.0),
    ((2, 2, 3), 4, (1, 2, 0), True, 0.0, 0.7),
    ((1, 2, 2), 3, (0, 1, 2), False, 5.0, 2.0),
    ((3, 2, 1), 2, (2, 2, 2), False, 0.0, 1.0),      # singular (all Neumann)
    ((2, 2, 2), 3, (0, 0, 0), False, 0.0, 1.3),      # singular (periodic)
])
def test_fdm_inverse_against_dense_operator(n, P, bc, st, lam, nu):
    # F (A x) = x with A from the element-by-element dense assembly, a
    # construction independent of the Kronecker factors F is built from; for a
    # singular operator F drops the constant mode: F (A x) = x minus its
    # M-weighted mean
    s = make_spec(n, P, bc, st)
    A = dense.assemble(s, lam, nu)
    x = np.random.default_rng(3).uniform(-1, 1, ndof(s))
    F = kron.FDM(s, lam, nu)
    y = F.apply_inverse(A @ x)
    want = x
    if dense.singular(s, lam):
        M = dense.mass_diag(s)
        want = x - np.dot(M, x) / M.sum()
    assert np.linalg.norm(y - want) <= 1e-11 * np.linalg.norm(want)


def test_fdm_preconditioned_cg_constant_nu():
    # with the exact inverse as preconditioner, CG takes one step (two at most
    # for rounding) and lands on the exact discrete solution
    s = make_spec((3, 2, 3), 4, (0, 0, 1), True)
    lam, nu = 7.0, 1.0
    f = synth.uniform_field(ndof(s), 31)
    M = dense.mass_diag(s)
    op = naive.Operator(s, lam, nu)
    F = kron.FDM(s, lam, nu)
    x, info = pcg.pcg(op.apply, M * f, op.diag(), M, tol=1e-10, precond=F.apply_inverse)
    assert info["status"] == pcg.OK and info["iters"] <= 2
    xs = dense.solve(s, dense.assemble(s, lam, nu), M * f, lam)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_fdm_preconditioned_cg_nodal_nu():
    # nodal nu with max/min = 3 (the channel viscosity): the preconditioner
    # with nu_ref = sqrt(min max) bounds the preconditioned condition number
    # by 3, so CG needs at most ln(2/tol)/ln((sqrt 3 + 1)/(sqrt 3 - 1)) ~ 18
    # steps for 1e-10
    from tests.helpers import channel_nu
    s = make_spec((2, 3, 2), 4, (0, 0, 1), False)
    nu = channel_nu(s, 1.0)
    lam = 20.0
    f = synth.uniform_field(ndof(s), 32)
    M = dense.mass_diag(s)
    op = naive.Operator(s, lam, nu)
    F = kron.FDM(s, lam, np.sqrt(nu.min() * nu.max()))
    x, info = pcg.pcg(op.apply, M * f, op.diag(), M, tol=1e-10, precond=F.apply_inverse)
    _, ij = pcg.pcg(op.apply, M * f, op.diag(), M, tol=1e-10)
    assert info["status"] == pcg.OK and info["iters"] <= 18 and info["iters"] < ij["iters"]
    xs = dense.solve(s, dense.assemble(s, lam, nu), M * f, lam)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
