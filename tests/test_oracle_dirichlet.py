"""Pins of the oracle's inhomogeneous Dirichlet load (the lifting of the wall
data v_b into the velocity solves of Alg. 3): the SIP problem with the load
`M f + L(g)` reproduces polynomial solutions exactly, the load reads only
the boundary values of g, and a smooth solution with nonzero wall data
converges at order P+1."""
import numpy as np
import pytest

from oracle import dense, kron
from tests.helpers import make_spec, node_coords


@pytest.mark.parametrize("bc,P", [((0, 0, 1), 4), ((1, 1, 1), 5), ((1, 0, 1), 3)])
def test_polynomial_solution_reproduced(bc, P):
    # u of degree <= 2 per direction (periodic in x, y where those are
    # periodic), nodal nu linear: the discrete solution is u itself
    spec = make_spec((2, 2, 3), P, bc, True)
    X, Y, Z = node_coords(spec)
    if bc == (0, 0, 1):
        u, ux, uy, uz, lap = 1 + 2 * Z - Z ** 2, 0 * X, 0 * X, 2 - 2 * Z, -2 + 0 * X
        nu, nux, nuy, nuz = 1 + 0.5 * Z, 0.0, 0.0, 0.5
    elif bc == (1, 1, 1):
        u, ux, uy, uz, lap = 1 + X * Y + Z ** 2 - 0.5 * X, Y - 0.5, X, 2 * Z, 2 + 0 * X
        nu, nux, nuy, nuz = 1 + 0.5 * Z + 0.2 * X, 0.2, 0.0, 0.5
    else:
        u, ux, uy, uz, lap = X * Z + 0.3 * X ** 2, Z + 0.6 * X, 0 * X, X, 0.6 + 0 * X
        nu, nux, nuy, nuz = 0.8 + 0.3 * X, 0.3, 0.0, 0.0
    lam = 3.0
    f = lam * u - (nux * ux + nuy * uy + nuz * uz + nu * lap)
    A = dense.assemble(spec, lam, nu)
    b = dense.mass_diag(spec) * f + dense.dirichlet_load(spec, nu, u)
    x = np.linalg.solve(A, b)
    assert np.max(np.abs(x - u)) <= 1e-12


def test_load_reads_only_boundary_values():
    spec = make_spec((2, 2, 2), 4, (1, 0, 1), False)
    X, Y, Z = node_coords(spec)
    g = np.sin(3 * X) + Z
    on = np.isclose(X, 0) | np.isclose(X, 1) | np.isclose(Z, 0) | np.isclose(Z, 1)
    g2 = g + np.where(on, 0.0, 5.0)
    L1, L2 = dense.dirichlet_load(spec, 0.7, g), dense.dirichlet_load(spec, 0.7, g2)
    assert np.array_equal(L1, L2)
    assert np.max(np.abs(L1)) > 0
    assert np.max(np.abs(dense.dirichlet_load(make_spec((2, 2, 2), 4, (0, 0, 0), False), 0.7, g))) == 0.0


def test_smooth_solution_with_wall_data_converges_at_order_P_plus_1():
    # u = cos(2 pi x) sin(2 pi y) exp(z) with u != 0 on the z walls (periodic
    # x, y, Dirichlet z), constant nu: errors at n = 2, 4, 8 elements per
    # axis fall like h^(P+1)
    P, lam, nu = 3, 2.0, 1.0
    errs = []
    for n in (2, 4, 8):
        spec = make_spec((n, n, n), P, (0, 0, 1), False)
        X, Y, Z = node_coords(spec)
        u = np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.exp(Z)
        f = lam * u - nu * (1.0 - 8 * np.pi ** 2) * u
        M = dense.mass_diag(spec)
        x = kron.FDM(spec, lam, nu).solve(M * f + dense.dirichlet_load(spec, nu, u))
        errs.append(np.sqrt(np.dot(M, (x - u) ** 2)))
    eoc = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert eoc[-1] >= P + 1 - 0.3, (errs, eoc)
