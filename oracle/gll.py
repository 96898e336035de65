"""GLL nodes, weights and collocation differentiation matrix (oracle).

Test infrastructure only (see the package docstring).

Sec. 3.3 of arXiv 2112.04167 puts the solution on tensor-product Lagrange
polynomials based on Gauss-Lobatto-Legendre (GLL) points of degree P.  The
paper gives no formulas; the ones below are the textbook definitions:

  * nodes: xi_0 = -1, xi_P = +1, interior nodes = roots of L_P'(x);
  * weights: w_j = 2 / (P (P+1) L_P(xi_j)^2);
  * D_ij = l_j'(xi_i):  L_P(xi_i) / (L_P(xi_j) (xi_i - xi_j))  for i != j,
    D_00 = -P(P+1)/4,  D_PP = +P(P+1)/4,  D_ii = 0 otherwise.

Parity pins live in tests/test_oracle_gll.py (closed-form nodes for P=2..4,
quadrature exactness to degree 2P-1, D applied to monomials, the
summation-by-parts identity, and a brute-force Lagrange-derivative check).
"""
import numpy as np


def legendre(P, x):
    """L_P(x) and L_P'(x) by the three-term recurrence (Bonnet)."""
    x = np.asarray(x, dtype=np.float64)
    if P == 0:
        return np.ones_like(x), np.zeros_like(x)
    l0, l1 = np.ones_like(x), x.copy()
    for k in range(2, P + 1):
        l0, l1 = l1, ((2 * k - 1) * x * l1 - (k - 1) * l0) / k
    # derivative from the standard identity (1-x^2) L_P' = P (L_{P-1} - x L_P),
    # valid away from +-1; the endpoints use L_P'(+-1) = (+-1)^(P+1) P(P+1)/2.
    with np.errstate(divide="ignore", invalid="ignore"):
        dl = P * (l0 - x * l1) / (1.0 - x * x)
    end = np.abs(np.abs(x) - 1.0) == 0.0
    if np.any(end):
        dl = np.where(end, np.sign(x) ** (P + 1) * P * (P + 1) / 2.0, dl)
    return l1, dl


def _legendre_d2(P, x):
    """L_P''(x) from Legendre's equation (1-x^2) y'' - 2x y' + P(P+1) y = 0."""
    l, dl = legendre(P, x)
    return (2.0 * x * dl - P * (P + 1) * l) / (1.0 - x * x)


def nodes(P):
    """GLL nodes of degree P (P+1 points, ascending)."""
    if P < 1:
        raise ValueError("P >= 1 required")
    n = P + 1
    # start from Chebyshev-Gauss-Lobatto points, then Newton on L_P'(x) = 0
    x = -np.cos(np.pi * np.arange(n) / P)
    xi = x[1:-1].copy()
    for _ in range(100):
        _, dl = legendre(P, xi)
        step = dl / _legendre_d2(P, xi)
        xi -= step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    out = np.empty(n)
    out[0], out[-1] = -1.0, 1.0
    out[1:-1] = np.sort(xi)
    # enforce exact antisymmetry of the node set
    out = 0.5 * (out - out[::-1])
    return out


def weights(P):
    """GLL quadrature weights w_j = 2 / (P(P+1) L_P(xi_j)^2)."""
    xi = nodes(P)
    l, _ = legendre(P, xi)
    return 2.0 / (P * (P + 1) * l * l)


def diff_matrix(P):
    """Collocation differentiation matrix D_ij = l_j'(xi_i)."""
    xi = nodes(P)
    l, _ = legendre(P, xi)
    n = P + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = l[i] / (l[j] * (xi[i] - xi[j]))
    D[0, 0] = -P * (P + 1) / 4.0
    D[P, P] = P * (P + 1) / 4.0
    return D


def tables(P):
    """(xi, w, D) for degree P."""
    return nodes(P), weights(P), diff_matrix(P)
