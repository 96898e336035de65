"""Pins of the oracle's DG divergence / gradient (velocity degree P, pressure
degree P-1) and of its projection substep (Alg. 3), each against something
the mathematics fixes:

  * adjointness (G psi, w)_{M_v} = -(psi, D(w; 0)): D and G are written out
    separately from their integral definitions, so a sign or index slip in
    either (face orientation, lifting weight, layer) breaks it;
  * exactness: for a velocity field of degree <= P-1 with v_b = v on the
    boundary, D(v; v) = M_p (div v) at the pressure nodes to rounding (the
    integrals are exact and a continuous field has no jumps); for a linear
    pressure G psi = grad psi exactly; constants have zero gradient;
  * convergence: the divergence of a smooth periodic field and the result of
    the projection of u + grad phi (u divergence-free) converge with h."""
import numpy as np
import pytest

from oracle import dense, gll, projection
from tests.helpers import make_spec, node_coords


def vnodes(spec):
    return node_coords(spec)


SHAPES = [((2, 2, 2), 4, (0, 0, 0), False),
          ((2, 3, 2), 3, (0, 1, 2), True),
          ((1, 2, 3), 5, (1, 0, 1), False),
          ((3, 1, 2), 4, (2, 2, 0), True)]


@pytest.mark.parametrize("n,P,bc,st", SHAPES)
def test_gradient_is_minus_adjoint_of_divergence(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    ps = projection.pressure_spec(s)
    rng = np.random.default_rng(5)
    Nv = dense.mass_diag(s).size
    Np = dense.mass_diag(ps).size
    psi = rng.uniform(-1, 1, Np)
    w = [rng.uniform(-1, 1, Nv) for _ in range(3)]
    Mv = dense.mass_diag(s)
    G = projection.gradient(s, psi)
    lhs = sum(np.dot(Mv * G[d], w[d]) for d in range(3))
    rhs = -np.dot(psi, projection.divergence(s, w, None))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


@pytest.mark.parametrize("n,P,bc,st", SHAPES)
def test_divergence_exact_for_polynomial_fields(n, P, bc, st):
    # v of degree <= P-1 per direction (non-periodic axes only carry
    # polynomials; on periodic axes the field must be periodic: constant)
    s = make_spec(n, P, bc, st)
    X, Y, Z = vnodes(s)
    deg = P - 1
    px = X ** deg if bc[0] != 0 else 0 * X
    py = Y ** (deg - 1) if bc[1] != 0 else 0 * Y
    pz = Z ** 2 if bc[2] != 0 else 0 * Z
    v = [px * 0.5 + 1.0 + (Y if bc[1] != 0 else 0), py - 2.0, pz + (X if bc[0] != 0 else 0)]
    div_exact = lambda Xp, Yp, Zp: ((0.5 * deg * Xp ** (deg - 1)) if bc[0] != 0 else 0 * Xp) + \
        (((deg - 1) * Yp ** (deg - 2)) if bc[1] != 0 else 0 * Yp) + ((2 * Zp) if bc[2] != 0 else 0 * Zp)
    ps = projection.pressure_spec(s)
    Xp, Yp, Zp = node_coords(ps)
    D = projection.divergence(s, v, v)
    want = dense.mass_diag(ps) * div_exact(Xp, Yp, Zp)
    assert np.linalg.norm(D - want) <= 1e-11 * max(1.0, np.linalg.norm(want))


@pytest.mark.parametrize("n,P,bc,st", SHAPES)
def test_gradient_exact_for_linear_pressure_and_zero_for_constants(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    ps = projection.pressure_spec(s)
    Xp, Yp, Zp = node_coords(ps)
    one = np.ones_like(Xp)
    G1 = projection.gradient(s, one)
    assert max(np.max(np.abs(g)) for g in G1) <= 1e-11
    if all(b != 0 for b in bc):   # a linear function is single-valued only without periodic axes
        G = projection.gradient(s, 2 * Xp + 3 * Yp - Zp)
        for d, c in enumerate((2.0, 3.0, -1.0)):
            assert np.max(np.abs(G[d] - c)) <= 1e-10


def _manufactured(spec):
    X, Y, Z = vnodes(spec)
    tp = 2 * np.pi
    u = [np.sin(tp * Y), np.sin(tp * Z), np.sin(tp * X)]                  # divergence-free
    phi = np.sin(tp * X) * np.sin(tp * Y) * np.sin(tp * Z) / tp
    gphi = [np.cos(tp * X) * np.sin(tp * Y) * np.sin(tp * Z),
            np.sin(tp * X) * np.cos(tp * Y) * np.sin(tp * Z),
            np.sin(tp * X) * np.sin(tp * Y) * np.cos(tp * Z)]
    return u, gphi


@pytest.mark.parametrize("P", [4, 5])
def test_divergence_converges_on_periodic_field(P):
    errs = []
    for n in (2, 4, 8):
        s = make_spec(n, P, (0, 0, 0))
        ps = projection.pressure_spec(s)
        u, gphi = _manufactured(s)
        v = [u[d] + gphi[d] for d in range(3)]
        Xp, Yp, Zp = node_coords(ps)
        tp = 2 * np.pi
        div = -3 * tp * np.sin(tp * Xp) * np.sin(tp * Yp) * np.sin(tp * Zp)   # lap phi
        Mp = dense.mass_diag(ps)
        d = projection.divergence(s, v) / Mp
        errs.append(np.sqrt(np.dot(Mp, (d - div) ** 2)))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc[-1] > P - 1.3, (errs, eoc)


def test_projection_removes_gradient_part():
    # v' = u + grad phi on the periodic cube: v'' -> u, and the error falls
    # with h at about order P
    P = 4
    errs = []
    for n in (2, 4, 8):
        s = make_spec(n, P, (0, 0, 0))
        u, gphi = _manufactured(s)
        v = [u[d] + gphi[d] for d in range(3)]
        vpp, psi = projection.project(s, v)
        M = dense.mass_diag(s)
        errs.append(np.sqrt(sum(np.dot(M, (vpp[d] - u[d]) ** 2) for d in range(3))))
        Mp = dense.mass_diag(projection.pressure_spec(s))
        assert abs(np.dot(Mp, psi)) <= 1e-12 * np.linalg.norm(psi)
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-3 and eoc[-1] > P - 1.3, (errs, eoc)
