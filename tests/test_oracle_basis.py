"""Pins for the oracle's 1D basis: exact rationals, closed-form integrals, reproduction."""
import numpy as np
import pytest

from oracle.basis import (gauss_legendre, gll_nodes, lagrange_derivatives, lagrange_values,
                          mass_1d, prolongation_1d, stiffness_1d)


def test_gll_nodes_closed_forms():
    assert np.allclose(gll_nodes(1), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-16)
    s5 = 1.0 / np.sqrt(5.0)
    assert np.allclose(gll_nodes(3), [0.0, (1 - s5) / 2, (1 + s5) / 2, 1.0], atol=1e-15)
    s37 = np.sqrt(3.0 / 7.0)
    assert np.allclose(gll_nodes(4), [0.0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("k", range(1, 9))
def test_gll_nodes_are_roots_of_legendre_derivative(k):
    # interior GLL nodes are the roots of P_k' on [-1, 1]
    x = 2 * gll_nodes(k)[1:-1] - 1
    dP = np.polynomial.legendre.Legendre.basis(k).deriv()
    assert np.max(np.abs(dP(x)), initial=0.0) < 1e-11 * k * k
    assert np.all(np.diff(gll_nodes(k)) > 0)


def test_mass_stiffness_k1_k2_exact():
    assert np.allclose(mass_1d(1), [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-16)
    assert np.allclose(stiffness_1d(1), [[1, -1], [-1, 1]], atol=1e-15)
    assert np.allclose(30 * mass_1d(2), [[4, 2, -1], [2, 16, 2], [-1, 2, 4]], atol=1e-13)
    assert np.allclose(3 * stiffness_1d(2), [[7, -8, 1], [-8, 16, -8], [1, -8, 7]], atol=1e-13)


def test_prolongation_k2_exact():
    P0 = prolongation_1d(2, 0)
    assert np.allclose(P0, [[1, 0, 0], [3 / 8, 3 / 4, -1 / 8], [0, 1, 0]], atol=1e-15)
    P1 = prolongation_1d(2, 1)
    assert np.allclose(P1, [[0, 1, 0], [-1 / 8, 3 / 4, 3 / 8], [0, 0, 1]], atol=1e-15)


@pytest.mark.parametrize("k", range(1, 9))
def test_mass_stiffness_integrate_monomials(k):
    """u^T B v = int_0^1 x^a x^b and u^T D v = int a b x^(a+b-2) for a, b <= k."""
    xi = gll_nodes(k)
    B, D = mass_1d(k), stiffness_1d(k)
    for a in range(k + 1):
        for b in range(k + 1):
            u, v = xi ** a, xi ** b
            assert abs(u @ B @ v - 1.0 / (a + b + 1)) < 1e-13
            exact_d = 0.0 if a == 0 or b == 0 else a * b / (a + b - 1)
            assert abs(u @ D @ v - exact_d) < 2e-12 * (1 + exact_d)


@pytest.mark.parametrize("k", range(1, 9))
def test_partition_of_unity_and_symmetry(k):
    B, D = mass_1d(k), stiffness_1d(k)
    assert abs(B.sum() - 1.0) < 1e-14
    assert np.max(np.abs(D @ np.ones(k + 1))) < 1e-12
    assert np.allclose(B, B.T, atol=0) and np.allclose(D, D.T, atol=1e-15)
    # centro-symmetry (reversal of the node order) of the symmetric node set
    J = np.eye(k + 1)[::-1]
    assert np.allclose(J @ B @ J, B, atol=1e-15)
    assert np.allclose(J @ D @ J, D, atol=1e-12)


@pytest.mark.parametrize("k", range(1, 9))
@pytest.mark.parametrize("c", [0, 1])
def test_prolongation_reproduces_polynomials(k, c):
    xi = gll_nodes(k)
    P = prolongation_1d(k, c)
    for a in range(k + 1):
        assert np.max(np.abs(P @ xi ** a - ((xi + c) / 2) ** a)) < 1e-13


@pytest.mark.parametrize("k", [2, 5, 8])
def test_lagrange_derivative_matches_finite_difference(k):
    xi = gll_nodes(k)
    x = np.linspace(0.013, 0.987, 7)
    eps = 1e-6
    fd = (lagrange_values(xi, x + eps) - lagrange_values(xi, x - eps)) / (2 * eps)
    assert np.max(np.abs(fd - lagrange_derivatives(xi, x))) < 1e-6 * k ** 2
    assert np.allclose(lagrange_values(xi, xi), np.eye(k + 1), atol=1e-14)


def test_gauss_rule_exactness():
    x, w = gauss_legendre(5)
    for a in range(10):
        assert abs(w @ x ** a - 1.0 / (a + 1)) < 1e-15
