"""Jacobi-preconditioned conjugate gradients and mixed-precision iterative
refinement, step by step (oracle).

Test infrastructure only (see the package docstring).

arXiv 2112.04167 solves the pressure and diffusion problems of Alg. 3 with
Krylov methods (Sec. 3.3) and stops at a relative tolerance on the RMS
residual evaluated at the collocation points (Sec. 4).  The residual at the
collocation points of  lambda u - div(nu grad u) = f  is the nodal residual
M^-1 (b - A x) (b = M f, M the diagonal GLL mass), so the test is

    || M^-1 (b - A x) ||_2  <=  tol * || M^-1 b ||_2        (x0 = 0).

The Krylov method here is textbook preconditioned CG (Hestenes & Stiefel)
with the Jacobi preconditioner diag(A).  For the singular Poisson problem
(lambda = 0, no Dirichlet face) the load and every residual are projected
to Euclidean mean zero and the result is shifted to M-weighted mean zero.
"""
import numpy as np

OK, NOT_CONVERGED, ERR_NOT_SPD, ERR_NONFINITE = 0, 1, -4, -5


def pcg(apply, b, d, Mdiag, tol=1e-10, maxit=10000, singular=False, x0=None, fixed_iters=0):
    """Returns (x, info) with info = dict(iters, rel_res, status, history).

    apply: x -> A x;  d = diag(A);  Mdiag = diagonal mass.
    fixed_iters > 0 runs exactly that many iterations (no stopping test)."""
    b = np.array(b, dtype=np.float64)
    if not np.all(np.isfinite(b)):
        return np.zeros_like(b), dict(iters=0, rel_res=np.nan, status=ERR_NONFINITE, history=[])
    if singular:
        b = b - b.mean()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x) if x0 is not None else b.copy()
    if singular:
        r = r - r.mean()
    bnorm = np.linalg.norm(b / Mdiag)
    z = r / d
    p = z.copy()
    rho = float(np.dot(r, z))
    k = 0
    status = OK
    hist = []
    res = np.linalg.norm(r / Mdiag)
    while True:
        hist.append(res / bnorm if bnorm > 0 else 0.0)
        if fixed_iters > 0:
            if k >= fixed_iters:
                break
        else:
            if res <= tol * bnorm:
                break
            if k >= maxit:
                status = NOT_CONVERGED
                break
        q = apply(p)
        gam = float(np.dot(p, q))
        if not np.isfinite(gam):
            status = ERR_NONFINITE
            break
        if gam <= 0.0:
            status = ERR_NOT_SPD
            break
        alpha = rho / gam
        x += alpha * p
        r -= alpha * q
        if singular:
            r -= r.mean()
        z = r / d
        rho_new = float(np.dot(r, z))
        p = z + (rho_new / rho) * p
        rho = rho_new
        k += 1
        res = np.linalg.norm(r / Mdiag)
    if singular:
        x -= np.dot(Mdiag, x) / Mdiag.sum()
    return x, dict(iters=k, rel_res=res / bnorm if bnorm > 0 else 0.0, status=status, history=hist)


def true_rel_res(apply, x, b, Mdiag, singular=False):
    """|| M^-1 (b - A x) || / || M^-1 b || recomputed from x (rule of Sec. 4)."""
    b = np.asarray(b, dtype=np.float64)
    if singular:
        b = b - b.mean()
    r = b - apply(x)
    if singular:
        r = r - r.mean()
    return float(np.linalg.norm(r / Mdiag) / np.linalg.norm(b / Mdiag))

