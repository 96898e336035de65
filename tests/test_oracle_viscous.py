"""Pins of the oracle's variable-viscosity stage terms: the viscosity law
(closed form), F_d1 = div(nu grad v) and F_d3 = -grad(nu div v) against
their analytic values on smooth periodic fields (convergence with h), and
the adjointness of the equal-order divergence and gradient that F_d3 is
built from."""
import numpy as np
import pytest

from oracle import dense, projection, viscous
from tests.helpers import make_spec, node_coords

TP = 2 * np.pi


def test_viscosity_law_closed_form():
    rng = np.random.default_rng(4)
    v = [rng.uniform(-2, 2, 50) for _ in range(3)]
    nu = viscous.viscosity(v, 0.01, 0.02, 2.0)
    want = 0.01 + 0.02 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / 4.0
    assert np.max(np.abs(nu - want)) <= 1e-17 + 1e-15 * np.max(want)


@pytest.mark.parametrize("n,P,bc,st", [((2, 2, 2), 4, (0, 0, 0), False), ((2, 3, 2), 5, (0, 1, 2), True)])
def test_equal_order_gradient_is_minus_adjoint_of_divergence(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    N = dense.mass_diag(s).size
    rng = np.random.default_rng(9)
    w = rng.uniform(-1, 1, N)
    u = [rng.uniform(-1, 1, N) for _ in range(3)]
    M = dense.mass_diag(s)
    G = projection.gradient(s, w, q_degree=P)
    lhs = sum(np.dot(M * G[d], u[d]) for d in range(3))
    rhs = -np.dot(w, projection.divergence(s, u, None, q_degree=P))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def _eoc(errs):
    return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))


@pytest.mark.parametrize("P", [4, 5])
def test_fd1_converges_to_div_nu_grad_v(P):
    errs = []
    for n in (2, 4, 8):
        s = make_spec(n, P, (0, 0, 0))
        X, Y, Z = node_coords(s)
        nu = 1.0 + 0.5 * np.sin(TP * X) * np.cos(TP * Y)
        u = np.sin(TP * X) * np.sin(TP * Y) * np.sin(TP * Z)
        ux = TP * np.cos(TP * X) * np.sin(TP * Y) * np.sin(TP * Z)
        uy = TP * np.sin(TP * X) * np.cos(TP * Y) * np.sin(TP * Z)
        nux = 0.5 * TP * np.cos(TP * X) * np.cos(TP * Y)
        nuy = -0.5 * TP * np.sin(TP * X) * np.sin(TP * Y)
        exact = -3 * TP * TP * nu * u + nux * ux + nuy * uy
        f = viscous.fd1(s, nu, [u, u, u])
        M = dense.mass_diag(s)
        errs.append(np.sqrt(np.dot(M, (f[0] - exact) ** 2)))
    assert _eoc(errs)[-1] > P - 1.5, (errs, _eoc(errs))


@pytest.mark.parametrize("P", [4, 5])
def test_fd3_converges_to_minus_grad_nu_div_v(P):
    # v = grad phi, phi = sin sin sin / (2 pi): div v = -12 pi^2 phi, and with a
    # constant nu, -grad(nu div v) = 12 pi^2 nu grad phi
    nu0 = 0.7
    errs = []
    for n in (2, 4, 8):
        s = make_spec(n, P, (0, 0, 0))
        X, Y, Z = node_coords(s)
        g = [np.cos(TP * X) * np.sin(TP * Y) * np.sin(TP * Z),
             np.sin(TP * X) * np.cos(TP * Y) * np.sin(TP * Z),
             np.sin(TP * X) * np.sin(TP * Y) * np.cos(TP * Z)]
        f = viscous.fd3(s, nu0 * np.ones_like(X), g)
        M = dense.mass_diag(s)
        exact = [3 * TP * TP * nu0 * c for c in g]
        errs.append(np.sqrt(sum(np.dot(M, (f[d] - exact[d]) ** 2) for d in range(3))))
    assert _eoc(errs)[-1] > P - 1.5, (errs, _eoc(errs))


def test_fd3_vanishes_on_constant_field():
    s = make_spec((2, 3, 2), 4, (0, 1, 0), True)
    X, Y, Z = node_coords(s)
    v = [0 * X + 1.5, 0 * X - 0.5, 0 * X + 2.0]
    nu = 1.0 + X * Y
    f = viscous.fd3(s, nu, v, v)   # boundary data = the field itself
    assert max(np.max(np.abs(c)) for c in f) <= 1e-10


def test_stage_load_linear_combination():
    rng = np.random.default_rng(1)
    vpp = [rng.uniform(size=10) for _ in range(3)]
    f1 = [[rng.uniform(size=10) for _ in range(3)] for _ in range(2)]
    f3 = [[rng.uniform(size=10) for _ in range(3)] for _ in range(2)]
    g = viscous.stage_load(vpp, f1, f3, 0.1, [0.3, 0.5], [0.2, 0.7])
    want = vpp[1] + 0.1 * ((0.3 - 0.2) * f1[0][1] - 0.2 * f3[0][1] + (0.5 - 0.7) * f1[1][1] - 0.7 * f3[1][1])
    assert np.allclose(g[1], want, rtol=0, atol=1e-15)
