"""Pins of the oracle's reference element (Sec. 4.1) against library
routines and closed forms, independent of the oracle's own code."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy.special import eval_legendre

import oracle as O

NS = [1, 2, 3, 4, 5]


@pytest.mark.parametrize("n", NS)
def test_recursion_matches_scipy_legendre(n):
    x = np.linspace(-1, 1, 41)
    P = O.legendre_values(n, x)
    for k in range(n):
        np.testing.assert_allclose(P[k], eval_legendre(k, x), atol=1e-15)


@pytest.mark.parametrize("n", NS)
def test_gauss_legendre_exactness(n):
    # Gauss-Legendre with n points integrates x^k exactly for k <= 2n-1.
    e = O.ReferenceElement(n)
    assert np.all(np.diff(e.xi) > 0)
    for k in range(2 * n):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.sum(e.w * e.xi ** k) - exact) < 1e-15 * 4


@pytest.mark.parametrize("n", NS)
def test_orthogonality_and_completeness(n):
    e = O.ReferenceElement(n)
    # sum_j w_j p_k p_l = 2/(2k+1) delta_kl (Sec. 4.1)
    G = e.B.T @ np.diag(e.w) @ e.B
    np.testing.assert_allclose(G, np.diag(2.0 / (2 * np.arange(n) + 1)),
                               atol=1e-15)
    # discrete completeness relation (Sec. 4.1, eq. completeness): B F = I,
    # and F B = I
    np.testing.assert_allclose(e.B @ e.F, np.identity(n), atol=1e-14)
    np.testing.assert_allclose(e.F @ e.B, np.identity(n), atol=1e-14)


@pytest.mark.parametrize("n", NS)
def test_D_closed_form_against_quadrature(n):
    # D_ij = int_{-1}^{1} p_i p_j', computed with numpy's Legendre series
    e = O.ReferenceElement(n)
    for i in range(n):
        for j in range(n):
            pi = npleg.Legendre.basis(i)
            dpj = npleg.Legendre.basis(j).deriv()
            prod = (pi * dpj).integ()
            val = prod(1.0) - prod(-1.0)
            assert abs(e.D[i, j] - val) < 1e-13


@pytest.mark.parametrize("n", NS)
def test_integration_by_parts_identity(n):
    # (D + L) = (R - D)^T  (Sec. 4.1, eq. legendre_derivative)
    e = O.ReferenceElement(n)
    np.testing.assert_allclose(e.D + e.L, (e.R - e.D).T, atol=0)
    np.testing.assert_allclose(e.D + e.D.T, e.R - e.L, atol=0)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_transformation_reading(n):
    # The printed F = T B W does not type-check with B_kj = p_j(x_k); the
    # consistent statement is F = T B^T W (recorded reading).  h cancels.
    e = O.ReferenceElement(n)
    h = 0.37
    T = e.That / h
    W = np.diag(h * e.w / 2)
    np.testing.assert_allclose(e.F, T @ e.B.T @ W, atol=1e-14)
    assert np.max(np.abs(e.F - T @ e.B @ W)) > 1e-3
