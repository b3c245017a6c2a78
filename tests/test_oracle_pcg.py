"""Pins of the oracle's fast-diagonalisation preconditioner and PCG (beyond
the paper's plain CG of Sec. 6): the preconditioner against the sparse LDG
operator and the dense brute-force solve, against a closed-form eigenvalue at
P = 1, and PCG against plain CG (identity preconditioner) and the dense
solve."""
import math

import numpy as np
import pytest

import oracle as O


def _wnorm(g, u):
    return math.sqrt(O.inner(g, u, u))


@pytest.mark.parametrize("n,Nx,Ny,ly", [(1, 5, 4, 1.3), (2, 4, 6, 1.0), (3, 3, 5, 0.7),
                                        (4, 6, 3, 1.3), (5, 3, 4, 2.0)])
def test_fd_inverts_laplacian(n, Nx, Ny, ly):
    # -Lap(M r) = r - mean_W(r) and mean_W(M r) = 0, with the sparse
    # operator; M r equals the dense minimum-norm solve.
    g = O.Grid2D(n, Nx, Ny, 0.0, 1.0, 0.0, ly)
    r = np.random.default_rng(10 + n).standard_normal(g.shape)
    fd = O.FastDiagonalisation(g)
    z = fd.apply(r)
    b = r - O.wmean(g, r)
    back = -O.laplacian(g, z)
    assert _wnorm(g, back - b) <= 1e-11 * _wnorm(g, b)
    assert abs(O.wmean(g, z)) <= 1e-13 * np.abs(z).max()
    ref = O.dense_poisson_solve(g, r)
    assert _wnorm(g, z - ref) <= 1e-10 * _wnorm(g, ref)


def test_fd_p1_closed_form_eigenvalue():
    # At P = 1 the Laplacian is the 5-point stencil; sin(kx) sin(ly) is an
    # eigenvector with eigenvalue -(4/h^2)(sin^2(k h/2) + sin^2(l h/2)).
    N = 24
    g = O.Grid2D(1, N, N)
    X, Y = g.node_coords()
    for k, l in [(1, 1), (3, 2), (7, 11)]:
        mode = np.sin(k * X) * np.sin(l * Y)
        mu = 4.0 / g.hx ** 2 * (math.sin(k * g.hx / 2) ** 2 + math.sin(l * g.hx / 2) ** 2)
        z = O.FastDiagonalisation(g).apply(mode)
        np.testing.assert_allclose(z, mode / mu, atol=1e-13 * np.abs(mode / mu).max())


def test_fd_constant_maps_to_zero():
    g = O.Grid2D(3, 5, 4)
    z = O.FastDiagonalisation(g).apply(np.full(g.shape, 2.5))
    assert np.abs(z).max() <= 1e-12


@pytest.mark.parametrize("n,N", [(2, 6), (4, 5)])
def test_pcg_identity_equals_cg(n, N):
    # M = I reproduces plain CG exactly (same operations in the same order).
    g = O.Grid2D(n, N, N)
    w = np.random.default_rng(n).standard_normal(g.shape)
    guess = np.random.default_rng(99).standard_normal(g.shape) * 0.1
    a = O.cg_poisson(g, w, guess=guess, rtol=1e-12)
    b = O.pcg_poisson(g, w, guess=guess, rtol=1e-12, precond=None)
    assert a.iters == b.iters and a.converged and b.converged
    assert np.array_equal(a.x, b.x)


@pytest.mark.parametrize("n,Nx,Ny", [(1, 6, 5), (3, 4, 4), (5, 3, 5)])
def test_pcg_fd_converges_at_once(n, Nx, Ny):
    g = O.Grid2D(n, Nx, Ny, 0.0, 1.0, 0.0, 1.4)
    w = np.random.default_rng(3 * n).standard_normal(g.shape)
    fd = O.FastDiagonalisation(g)
    res = O.pcg_poisson(g, w, rtol=1e-12, precond=fd.apply)
    ref = O.dense_poisson_solve(g, w)
    assert res.converged and res.iters <= 2
    assert _wnorm(g, res.x - ref) <= 1e-10 * _wnorm(g, ref)


def test_pcg_fd_moderate_grid_vs_plain_cg():
    # 32 x 32 cells, n = 4: same solution as plain CG to its tolerance, in a
    # handful of iterations instead of hundreds.
    g = O.Grid2D(4, 32, 32)
    X, Y = g.node_coords()
    w = np.sin(3 * X) * np.cos(Y) + 0.3 * np.cos(5 * X + 2 * Y) ** 3
    plain = O.cg_poisson(g, w, rtol=1e-12)
    pcg = O.pcg_poisson(g, w, rtol=1e-12, precond=O.FastDiagonalisation(g).apply)
    assert pcg.converged and pcg.iters <= 3 < plain.iters
    assert _wnorm(g, pcg.x - plain.x) <= 1e-9 * _wnorm(g, plain.x)
