"""CPU FP64 oracle for the SIP-DG Helmholtz/Poisson implicit-stage solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code,
tables or constants with the HIP library: it computes its own GLL tables,
its own operator and its own solvers, in plain FP64.

What it follows (arXiv 2112.04167):
  * Sec. 3.3 -- hexahedral elements, tensor-product Lagrange polynomials on
    GLL points, DG-SEM, interior penalty for the pressure and viscous
    diffusion problems;
  * Alg. 3 (and Alg. 4) -- the implicit sub-problems
        v - dt*a_ii*div(nu grad v) = g  with Dirichlet data   (Helmholtz)
        lap(psi) = div(v')              with Neumann data     (Poisson);
  * Sec. 4 -- the stopping rule: relative RMS residual at the collocation
    points.

Where the paper is silent (penalty constant, quadrature of the face and
volume integrals, average of nu in the consistency term, pressure BC and the
singular Poisson problem) the oracle takes the readings written out in the
docstrings of ``dense`` and ``naive.c``.

Modules:
  gll    -- GLL nodes, weights, differentiation matrix (closed forms).
  dense  -- dense assembly of A from basis-function evaluations (tiny meshes),
            dense Cholesky exact solve.
  kron   -- 1D SIP matrices, Kronecker-sum assembly, fast-diagonalization
            exact solver (Lynch, Rice & Thomas 1964).
  naive  -- ctypes wrapper of naive.c: naive matrix-free apply (triple loops).
  pcg    -- Jacobi-PCG, and FP64 iterative refinement around an FP32 inner
            Jacobi-PCG, both step by step.
  build  -- compiles naive.c with gcc.
"""
