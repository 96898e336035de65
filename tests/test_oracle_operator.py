"""Pins of the oracle's SIP-DG operator.

Three independent constructions (basis-function dense assembly, the naive
matrix-free loop of naive.c, the Kronecker sum of 1D SIP matrices) must agree;
A must be symmetric, positive definite when lambda > 0 or a Dirichlet face
exists, and have exactly the constants as null space otherwise; and it must
reproduce the boundary load of a linear field (consistency of the interior
penalty form) and the Laplace eigenvalues pi^2 / (2 pi)^2 of the 1D
Dirichlet / periodic problems."""
import numpy as np
import pytest

from oracle import dense, kron, naive
from tests.helpers import make_spec, ndof, node_coords

CASES = [
    ((2, 2, 2), 2, (0, 0, 0), False),
    ((2, 3, 2), 3, (0, 1, 2), True),
    ((1, 2, 3), 2, (0, 1, 1), True),
    ((3, 2, 2), 3, (1, 2, 0), True),
    ((2, 2, 1), 4, (1, 0, 0), False),
    ((1, 1, 1), 3, (0, 0, 0), False),
    ((3, 1, 1), 1, (2, 1, 0), False),
]


@pytest.mark.parametrize("n,P,bc,st", CASES)
def test_three_constructions_agree(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    lam, nu = 1.7, 1.3
    Ad = dense.assemble(s, lam, nu)
    Ak = kron.assemble(s, lam, nu)
    assert np.abs(Ad - Ak).max() <= 1e-13 * np.abs(Ad).max()
    op = naive.Operator(s, lam, nu)
    x = np.random.default_rng(0).uniform(-1, 1, ndof(s))
    y = op.apply(x)
    assert np.abs(Ad @ x - y).max() <= 1e-13 * np.abs(y).max()
    assert np.abs(np.diag(Ad) - op.diag()).max() <= 1e-13 * np.abs(np.diag(Ad)).max()


@pytest.mark.parametrize("n,P,bc,st", CASES)
def test_nodal_nu_dense_vs_naive(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    rng = np.random.default_rng(1)
    nu = rng.uniform(0.3, 2.0, ndof(s))
    Ad = dense.assemble(s, 0.9, nu)
    op = naive.Operator(s, 0.9, nu)
    x = rng.uniform(-1, 1, ndof(s))
    y = op.apply(x)
    assert np.abs(Ad @ x - y).max() <= 1e-13 * np.abs(y).max()
    assert np.abs(np.diag(Ad) - op.diag()).max() <= 1e-13 * np.abs(np.diag(Ad)).max()
    assert np.abs(Ad - Ad.T).max() <= 1e-14 * np.abs(Ad).max()
    assert np.linalg.eigvalsh(Ad).min() > 0.0


@pytest.mark.parametrize("n,P,bc,st", CASES)
def test_symmetric_and_definite(n, P, bc, st):
    s = make_spec(n, P, bc, st)
    for lam in (0.0, 2.5):
        A = dense.assemble(s, lam, 1.0)
        assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
        ev = np.linalg.eigvalsh(A)
        if lam > 0 or 1 in bc:
            assert ev[0] > 1e-8 * ev[-1]
        else:
            # exactly one zero mode (the constants), the rest positive
            assert abs(ev[0]) <= 1e-12 * ev[-1]
            assert ev[1] > 1e-8 * ev[-1]
            one = np.ones(A.shape[0])
            assert np.abs(A @ one).max() <= 1e-13 * np.abs(A).max()


def test_null_space_naive_large():
    s = make_spec((3, 4, 2), 5, (0, 2, 0), True)
    op = naive.Operator(s, 0.0, 1.0)
    y = op.apply(np.ones(ndof(s)))
    assert np.abs(y).max() <= 1e-12 * np.abs(op.diag()).max()


@pytest.mark.parametrize("P", [2, 3, 5])
def test_linear_field_consistency(P):
    # u = x on a Neumann x-axis: a(u, v) = int (-lap u) v + int_{x=1} v - int_{x=0} v
    # = boundary load only, exactly (GLL integrates every term exactly here)
    s = make_spec((3, 2, 2), P, (2, 0, 0), False)
    X, _, _ = node_coords(s)
    lam = 0.0
    y = naive.Operator(s, lam, 1.0).apply(X)
    n = P + 1
    from oracle import gll
    w = gll.weights(P)
    hy = hz = 0.5
    omega = np.outer(w, w) * hy * hz / 4.0     # (c, b)
    expect = np.zeros((2, 2, 3, n, n, n))     # ez ey ex c b a
    expect[:, :, 2, :, :, P] += omega
    expect[:, :, 0, :, :, 0] -= omega
    np.testing.assert_allclose(y, expect.reshape(-1), rtol=0, atol=1e-12)


def test_linear_field_consistency_nodal_nu():
    # with nu = 1 + x (linear): -div(nu grad x) = -1, flux nu at x=1 is 2, at x=0 is 1
    P = 4
    s = make_spec((2, 1, 1), P, (2, 0, 0), False)
    X, _, _ = node_coords(s)
    nu = 1.0 + X
    y = naive.Operator(s, 0.0, nu).apply(X)
    from oracle import dense as dn
    M = dn.mass_diag(s)
    n = P + 1
    from oracle import gll
    w = gll.weights(P)
    omega = np.outer(w, w) * 1.0 * 1.0 / 4.0
    expect = (-M).reshape(1, 1, 2, n, n, n).copy()
    expect[0, 0, 1, :, :, P] += 2.0 * omega
    expect[0, 0, 0, :, :, 0] -= 1.0 * omega
    np.testing.assert_allclose(y, expect.reshape(-1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("P", [3, 5, 8])
def test_1d_laplace_eigenvalues(P):
    # smallest Dirichlet eigenvalue of -u'' on (0,1) is pi^2; first nonzero
    # periodic one is (2 pi)^2 (double)
    import scipy.linalg
    import synth
    v = synth.vertices_uniform(8)
    K, M = kron.sip_1d(v, P, kron.DIRICHLET)
    ev = scipy.linalg.eigh(K, np.diag(M), eigvals_only=True)
    assert abs(ev[0] - np.pi ** 2) < 1e-4 * np.pi ** 2
    K, M = kron.sip_1d(v, P, kron.PERIODIC)
    ev = scipy.linalg.eigh(K, np.diag(M), eigvals_only=True)
    assert abs(ev[0]) < 1e-10
    assert abs(ev[1] - 4 * np.pi ** 2) < 1e-4 * 4 * np.pi ** 2
    assert abs(ev[2] - 4 * np.pi ** 2) < 1e-4 * 4 * np.pi ** 2


def test_penalty_is_coercive_but_not_by_much():
    # the 1D Dirichlet SIP operator is definite with sigma = (P+1)^2/h; a
    # penalty a few times smaller loses definiteness (so the constant matters)
    import scipy.linalg
    import synth
    v = synth.vertices_uniform(4)
    for P in (3, 5, 7):
        K, M = kron.sip_1d(v, P, kron.DIRICHLET)
        assert np.linalg.eigvalsh(K).min() > 0
        # rebuild with a quarter of the penalty: subtract 3/4 of the penalty part
        Kp, _ = kron.sip_1d(v, P, kron.DIRICHLET, nu=1.0)
        n = P + 1
        h = np.diff(v)
        pen = np.zeros_like(K)
        for e in range(len(h)):
            if e + 1 < len(h):
                i, j = e * n + P, (e + 1) * n
                sg = n * n / min(h[e], h[e + 1])
                pen[i, i] += sg; pen[j, j] += sg; pen[i, j] -= sg; pen[j, i] -= sg
        pen[0, 0] += n * n / h[0]
        pen[-1, -1] += n * n / h[-1]
        assert np.linalg.eigvalsh(Kp - 0.75 * pen).min() < 0
