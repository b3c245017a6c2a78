"""Pins of the oracle's derivative and Laplacian operators (Secs. 3, 4.2,
4.3, 6) against closed forms, finite-difference reductions and invariants."""
import math

import numpy as np
import pytest

import oracle as O

NS = [1, 2, 3, 4, 5]


@pytest.mark.parametrize("n", NS)
def test_centred_lspace_matches_printed_block_form(n):
    # Mbar^per = 1/2 (1^+ (x) RL + 1 (x) (D - D^T) - 1^- (x) LR)
    # (Sec. 4.2, eq. discrete_der and the printed periodic block matrix)
    g = O.Grid1D(n, 6, 0.0, 1.0)
    e = g.el
    M = g.lspace_operator(0.5).toarray()
    N = 6
    ref = np.zeros((N * n, N * n))
    for m in range(N):
        b = slice(m * n, (m + 1) * n)
        ref[b, b] = 0.5 * (e.D - e.D.T)
        ref[b, slice(((m + 1) % N) * n, ((m + 1) % N + 1) * n)] += 0.5 * e.RL
        ref[b, slice(((m - 1) % N) * n, ((m - 1) % N + 1) * n)] -= 0.5 * e.LR
    np.testing.assert_allclose(M, ref, atol=0)
    # skew-symmetric (Sec. 4.2, remark after eq. matrix_xspace)
    np.testing.assert_allclose(M, -M.T, atol=0)


@pytest.mark.parametrize("n", NS)
@pytest.mark.parametrize("kind", ["centred", "forward", "backward"])
def test_derivative_of_constant_is_zero(n, kind):
    g = O.Grid1D(n, 7, 0.0, 2.0)
    d = g.derivative(kind) @ np.ones(7 * n)
    assert np.max(np.abs(d)) < 1e-12


def _continuous_piecewise_poly(n, N, h, rng):
    """A periodic continuous function that is a polynomial of degree n-1 in
    every cell, with its exact derivative, at the GL nodes (n >= 2)."""
    xi, _ = np.polynomial.legendre.leggauss(n)
    v = rng.standard_normal(N)            # face values, periodic
    vals = np.zeros((N, n))
    ders = np.zeros((N, n))
    for m in range(N):
        vl, vr = v[m], v[(m + 1) % N]
        q = np.polynomial.Polynomial(rng.standard_normal(max(n - 2, 0)) if n > 2 else [0.0])
        bubble = np.polynomial.Polynomial([1.0, 0.0, -1.0]) * q   # zero at +-1
        p = np.polynomial.Polynomial([(vl + vr) / 2, (vr - vl) / 2]) + bubble
        vals[m] = p(xi)
        ders[m] = p.deriv()(xi) * 2.0 / h
    return vals.ravel(), ders.ravel()


@pytest.mark.parametrize("n", [2, 3, 4, 5])
@pytest.mark.parametrize("kind", ["centred", "forward", "backward"])
def test_derivative_exact_on_continuous_piecewise_polynomials(n, kind):
    # With a continuous f every flux equals the trace, so the weak derivative
    # (Sec. 3, eq. discrete_derivative) is the exact derivative.
    rng = np.random.default_rng(n)
    g = O.Grid1D(n, 9, -1.0, 2.0)
    f, df = _continuous_piecewise_poly(n, 9, g.h, rng)
    np.testing.assert_allclose(g.derivative(kind) @ f, df,
                               atol=1e-11 * np.max(np.abs(df)))


def test_p1_reductions_are_finite_differences():
    # P = 1: centred difference (Sec. 3 and Sec. 4.2 remarks), forward and
    # backward differences.
    g = O.Grid1D(1, 11, 0.0, 1.3)
    u = np.random.default_rng(0).standard_normal(11)
    h = g.h
    np.testing.assert_allclose(g.derivative("centred") @ u,
                               (np.roll(u, -1) - np.roll(u, 1)) / (2 * h), atol=1e-13)
    np.testing.assert_allclose(g.derivative("forward") @ u,
                               (np.roll(u, -1) - u) / h, atol=1e-13)
    np.testing.assert_allclose(g.derivative("backward") @ u,
                               (u - np.roll(u, 1)) / h, atol=1e-13)


@pytest.mark.parametrize("n", NS)
def test_centred_derivative_is_W_skew(n):
    # M = W D_x is skew-symmetric (Sec. 4.2, eq. matrix_xspace remark):
    # x^T W (D y) = -(D x)^T W y
    rng = np.random.default_rng(10 + n)
    g = O.Grid1D(n, 8, 0.0, 3.0)
    W = g.weights()
    D = g.derivative("centred")
    x, y = rng.standard_normal((2, 8 * n))
    a, b = x @ (W * (D @ y)), (D @ x) @ (W * y)
    assert abs(a + b) < 1e-13 * (abs(a) + 1)


@pytest.mark.parametrize("n", NS)
def test_one_sided_derivatives_are_W_adjoint(n):
    # W D_backward = -(W D_forward)^T, so -W Lap is symmetric
    g = O.Grid1D(n, 7, 0.0, 2.0)
    W = np.diag(g.weights())
    Df = g.derivative("forward").toarray()
    Db = g.derivative("backward").toarray()
    np.testing.assert_allclose(W @ Db, -(W @ Df).T, atol=1e-12 * np.abs(W @ Db).max())


@pytest.mark.parametrize("n", [1, 3, 5])
def test_centred_derivative_order(n):
    # odd n: order n on a smooth periodic function
    errs = []
    for N in (16, 32):
        g = O.Grid2D(n, N, N)
        X, Y = g.node_coords()
        e = O.dx(g, np.sin(2 * X + 1) * np.cos(Y)) - 2 * np.cos(2 * X + 1) * np.cos(Y)
        errs.append(math.sqrt(O.inner(g, e, e)))
    assert math.log2(errs[0] / errs[1]) > n - 0.3


def test_p1_laplacian_is_five_point():
    g = O.Grid2D(1, 12, 9, 0.0, 2 * math.pi, 0.0, 1.7)
    u = np.random.default_rng(1).standard_normal(g.shape)
    L = O.laplacian(g, u)[:, :, 0, 0]
    np.testing.assert_allclose(L, O.five_point_laplacian(u[:, :, 0, 0], g.hx, g.hy),
                               atol=1e-12 * np.abs(L).max())


@pytest.mark.parametrize("n", NS)
def test_laplacian_symmetric_nsd_nullspace(n):
    g = O.Grid2D(n, 4, 3, 0.0, 1.0, 0.0, 1.5)
    _, _, Lap = O.dense_operators(g)
    W = np.diag(O.to_image(g.weights()).ravel())
    K = -W @ Lap
    np.testing.assert_allclose(K, K.T, atol=1e-10 * np.abs(K).max())
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    scale = np.abs(ev).max()
    assert ev.min() > -1e-10 * scale
    assert np.sum(ev < 1e-9 * scale) == 1            # null space = constants
    np.testing.assert_allclose(Lap @ np.ones(K.shape[0]), 0, atol=1e-9 * scale)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_dense_kronecker_matches_matrix_free(n):
    g = O.Grid2D(n, 3, 4, 0.0, 1.0, 0.0, 2.0)
    u = np.random.default_rng(2).standard_normal(g.shape)
    Dx, Dy, Lap = O.dense_operators(g)
    U = O.to_image(u).ravel()
    shp = (g.Ny * n, g.Nx * n)
    np.testing.assert_allclose(O.from_image((Dx @ U).reshape(shp), n), O.dx(g, u), atol=1e-11)
    np.testing.assert_allclose(O.from_image((Dy @ U).reshape(shp), n), O.dy(g, u), atol=1e-11)
    np.testing.assert_allclose(O.from_image((Lap @ U).reshape(shp), n), O.laplacian(g, u),
                               atol=1e-9)
