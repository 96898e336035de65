"""Pins of the oracle's GLL tables against closed forms and mathematics."""
import math

import numpy as np
import pytest

from oracle import gll, dense


@pytest.mark.parametrize("P,xi,w", [
    (2, [-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
     [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_closed_form_nodes_weights(P, xi, w):
    # textbook closed forms of the low-order Gauss-Lobatto-Legendre rules
    np.testing.assert_allclose(gll.nodes(P), xi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gll.weights(P), w, rtol=0, atol=1e-15)


@pytest.mark.parametrize("P", range(1, 10))
def test_quadrature_exactness(P):
    xi, w = gll.nodes(P), gll.weights(P)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * P):          # exact up to degree 2P-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, k
    # and not exact at degree 2P (a Lobatto rule, not Gauss)
    assert abs(np.dot(w, xi ** (2 * P)) - 2.0 / (2 * P + 1)) > 1e-6


@pytest.mark.parametrize("P", range(1, 10))
def test_diff_matrix_on_polynomials(P):
    xi, D = gll.nodes(P), gll.diff_matrix(P)
    for k in range(0, P + 1):           # exact on polynomials of degree <= P
        exact = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(D @ xi ** k, exact, rtol=0, atol=1e-12 * max(1, k * P))


@pytest.mark.parametrize("P", range(1, 10))
def test_summation_by_parts(P):
    w, D = gll.weights(P), gll.diff_matrix(P)
    Q = np.diag(w) @ D
    B = np.zeros((P + 1, P + 1))
    B[0, 0], B[P, P] = -1.0, 1.0
    np.testing.assert_allclose(Q + Q.T, B, rtol=0, atol=1e-13)


@pytest.mark.parametrize("P", range(1, 9))
def test_diff_matrix_brute_force(P):
    # derivative of each Lagrange basis polynomial from the product formula
    xi = gll.nodes(P)
    _, dV = dense.lagrange_eval(xi, xi)
    np.testing.assert_allclose(gll.diff_matrix(P), dV, rtol=0, atol=1e-12)


def test_nodes_are_roots_of_legendre_derivative():
    for P in range(2, 12):
        xi = gll.nodes(P)
        # independent: numpy's Legendre series derivative
        c = np.zeros(P + 1)
        c[P] = 1.0
        dL = np.polynomial.legendre.legder(c)
        assert np.max(np.abs(np.polynomial.legendre.legval(xi[1:-1], dL))) < 1e-11 * P * P
