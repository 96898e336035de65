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

Mixed precision is not in the paper.  ``iterative_refinement`` is the plain
textbook scheme (Wilkinson's iterative refinement around an inexact inner
solve): the correction equation A d = r is solved by the same PCG with its
vectors and operator results rounded to FP32 (dot products and scalars in
FP64), the correction is added in FP64, and the FP64 residual b - A x is
recomputed from x for the outer test.
"""
import numpy as np

OK, NOT_CONVERGED, ERR_NOT_SPD, ERR_NONFINITE = 0, 1, -4, -5


def pcg(apply, b, d, Mdiag, tol=1e-10, maxit=10000, singular=False, x0=None, fixed_iters=0,
        precond=None):
    """Returns (x, info) with info = dict(iters, rel_res, status, history).

    apply: x -> A x;  d = diag(A) (the Jacobi preconditioner z = r/d);
    precond: r -> z replaces it when given;  Mdiag = diagonal mass.
    fixed_iters > 0 runs exactly that many iterations (no stopping test)."""
    prec = precond if precond is not None else (lambda v: v / d)
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
    z = prec(r)
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
        z = prec(r)
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



def _pcg32(apply, r64, d, Mdiag, inner_tol, maxit, singular):
    """One inner solve A d = r in FP32 storage: every vector (and every
    operator result) is rounded to float32 when it is stored; dot products
    and the scalars alpha, beta are FP64.  Stops once the recurrence
    residual ||M^-1 r|| has dropped by inner_tol.  Returns (d as FP64, iters,
    status)."""
    f32 = np.float32
    # scale the right-hand side by a power of two so FP32 keeps its range
    amax = float(np.max(np.abs(r64)))
    scale = 2.0 ** np.round(np.log2(amax)) if amax > 0 else 1.0
    r = (r64 / scale).astype(f32)
    if singular:
        r = (r.astype(np.float64) - r.astype(np.float64).mean()).astype(f32)
    d32 = d.astype(f32)
    M32 = Mdiag.astype(f32)
    x = np.zeros_like(r)
    z = (r / d32).astype(f32)
    p = z.copy()
    rho = float(np.dot(r.astype(np.float64), z.astype(np.float64)))
    start = np.linalg.norm((r / M32).astype(np.float64))
    res = start
    k = 0
    status = OK
    while res > inner_tol * start and k < maxit:
        q = apply(p.astype(np.float64)).astype(f32)
        gam = float(np.dot(p.astype(np.float64), q.astype(np.float64)))
        if not np.isfinite(gam):
            status = ERR_NONFINITE
            break
        if gam <= 0.0:
            status = ERR_NOT_SPD
            break
        alpha = rho / gam
        x = (x + f32(alpha) * p).astype(f32)
        r = (r - f32(alpha) * q).astype(f32)
        if singular:
            r = (r.astype(np.float64) - r.astype(np.float64).mean()).astype(f32)
        z = (r / d32).astype(f32)
        rho_new = float(np.dot(r.astype(np.float64), z.astype(np.float64)))
        p = (z + f32(rho_new / rho) * p).astype(f32)
        rho = rho_new
        k += 1
        res = np.linalg.norm((r / M32).astype(np.float64))
    if k >= maxit and res > inner_tol * start:
        status = NOT_CONVERGED
    return scale * x.astype(np.float64), k, status


def iterative_refinement(apply, b, d, Mdiag, tol=1e-10, inner_tol=1e-2, maxit=50,
                         inner_maxit=10000, singular=False):
    """FP64 iterative refinement around FP32 Jacobi-PCG, step by step:

        x = 0, r = b
        while ||M^-1 r|| > tol ||M^-1 b||:
            d = PCG32(A, r)   to inner_tol (relative, recurrence residual)
            x += d            (FP64)
            r = b - A x       (FP64, recomputed from x)

    Returns (x, info) with info = dict(outer, inner, rel_res, status)."""
    b = np.array(b, dtype=np.float64)
    if singular:
        b = b - b.mean()
    bnorm = np.linalg.norm(b / Mdiag)
    x = np.zeros_like(b)
    r = b.copy()
    res = np.linalg.norm(r / Mdiag)
    outer = inner = 0
    status = OK
    while bnorm > 0 and res > tol * bnorm:
        if outer >= maxit:
            status = NOT_CONVERGED
            break
        dx, k, st = _pcg32(apply, r, d, Mdiag, inner_tol, inner_maxit, singular)
        inner += k
        if st < 0:
            status = st
            break
        x += dx
        r = b - apply(x)
        if singular:
            r = r - r.mean()
        res = np.linalg.norm(r / Mdiag)
        outer += 1
        if not np.isfinite(res):
            status = ERR_NONFINITE
            break
    if singular:
        x -= np.dot(Mdiag, x) / Mdiag.sum()
    return x, dict(outer=outer, inner=inner, rel_res=res / bnorm if bnorm > 0 else 0.0,
                   status=status)
