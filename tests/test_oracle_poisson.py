"""Pins of the oracle's CG Poisson solve (Sec. 6): dense brute force on tiny
grids, an exactly solvable eigen-mode at P = 1, and the convergence order
that Table 3 reports."""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n,Nx,Ny", [(1, 5, 4), (2, 4, 4), (3, 3, 5), (4, 4, 3), (5, 3, 3)])
def test_cg_matches_dense_solve(n, Nx, Ny):
    g = O.Grid2D(n, Nx, Ny, 0.0, 1.0, 0.0, 1.3)
    w = np.random.default_rng(n).standard_normal(g.shape)
    res = O.cg_poisson(g, w, rtol=1e-14, max_iter=10000)
    ref = O.dense_poisson_solve(g, w)
    assert res.converged
    err = math.sqrt(O.inner(g, res.x - ref, res.x - ref))
    assert err < 1e-9 * math.sqrt(O.inner(g, ref, ref))
    assert abs(O.wmean(g, res.x)) < 1e-14 * np.abs(ref).max()


def test_cg_zero_rhs_returns_zero():
    g = O.Grid2D(2, 4, 4)
    res = O.cg_poisson(g, np.full(g.shape, 3.0))       # constant: b = 0
    assert res.iters == 0 and np.all(res.x == 0)


def test_p1_eigenmode_one_iteration():
    # At P = 1 the Laplacian is the 5-point stencil; sin x sin y is an
    # eigenvector with eigenvalue -(8/h^2) sin^2(h/2) (hx = hy = h).
    N = 20
    g = O.Grid2D(1, N, N)
    X, Y = g.node_coords()
    w = np.sin(X) * np.sin(Y)
    lam = 8.0 / g.hx ** 2 * math.sin(g.hx / 2) ** 2
    res = O.cg_poisson(g, w, rtol=1e-12)
    assert res.iters == 1
    np.testing.assert_allclose(res.x, w / lam, atol=1e-14)


def _orders():
    out = {}
    with open(os.path.join(GOLDEN, "table3_orders.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            P, D, *o = line.split()
            out[(int(P), float(D))] = [float(v) for v in o]
    return out


@pytest.mark.parametrize("n", [2, 3, 4])
def test_poisson_order_matches_table3(n):
    # Table 3 reports order P for P >= 2; the Poisson solve shows it too.
    printed = _orders()[(n, 0.0)]
    errs = []
    for N in (16, 32):
        g = O.Grid2D(n, N, N)
        X, Y = g.node_coords()
        w = np.sin(2 * X) * np.sin(3 * Y)
        e = O.cg_poisson(g, w, rtol=1e-13).x - w / 13.0
        errs.append(math.sqrt(O.inner(g, e, e)))
    order = math.log2(errs[0] / errs[1])
    assert abs(order - np.mean(printed)) < 0.3


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_ldg_laplacian_is_symmetric_and_signed(n, bc):
    # W L symmetric; negative semi-definite with the constants as null space
    # (periodic) or negative definite (Dirichlet)
    g1 = O.Grid1D(n, 7, 0.0, 1.3, bc)
    L = g1.laplacian().toarray()
    W = np.diag(g1.weights())
    S = W @ L
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    scale = np.abs(ev).max()
    if bc == "periodic":
        assert ev[-1] <= 1e-12 * scale and abs(ev[-1]) <= 1e-12 * scale
        assert ev[-2] < -1e-8 * scale
        assert np.abs(L @ np.ones(L.shape[0])).max() <= 1e-12 * scale
    else:
        assert ev[-1] < -1e-8 * scale


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_ldg_laplacian_exact_on_polynomials_away_from_the_ends(n):
    # a global polynomial of degree <= n - 1 has no jumps on interior faces
    # and its LDG derivatives are exact there, so L q = q'' on every cell not
    # next to an end (Dirichlet) or the wrap (periodic)
    N = 8
    for bc in ("periodic", "dirichlet"):
        g1 = O.Grid1D(n, N, -0.4, 1.1, bc)
        x = g1.nodes()
        c = np.arange(1, n + 1) * 0.37
        q = np.polynomial.polynomial.polyval(x, c)
        d2 = np.polynomial.polynomial.polyval(x, np.polynomial.polynomial.polyder(c, 2))
        Lq = g1.laplacian() @ q
        inner_cells = slice(2 * n, (N - 2) * n)
        assert np.abs(Lq[inner_cells] - d2[inner_cells]).max() <= 1e-9 * max(1.0, np.abs(d2).max())
        J = g1.jumps() @ q
        interior = slice(1, N)                  # faces between two cells
        assert np.abs(J[interior]).max() <= 1e-12 * np.abs(q).max()
