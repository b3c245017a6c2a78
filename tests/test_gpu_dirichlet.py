"""The homogeneous Dirichlet closure of the bracket (zero numerical flux on
the boundary faces) on the GPU against the oracle, and Table 2's Dirichlet
row (Sec. 5.2).  Tolerance as for the periodic bracket: element-wise within
1e-12 of max |oracle|."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1311_7477_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1311_7477_amd import dg as _dg
    _dg.lib()
    return _dg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


BCS = [("dirichlet", "dirichlet"), ("dirichlet", "periodic"), ("periodic", "dirichlet")]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 5), (37, 23), (64, 40)])
@pytest.mark.parametrize("bcs", BCS)
@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_dirichlet_bracket_parity(dg, n, nx, ny, bcs, form):
    print(f"dirichlet bracket n={n} {nx}x{ny} {bcs} form={form}", flush=True)
    bx, by = bcs
    g = O.Grid2D(n, nx, ny, 0.0, 2.0, -1.0, 1.5, bx, by)
    rng = np.random.default_rng(n + 3 * nx + 7 * ny + form)
    f = rng.standard_normal(g.shape)
    h = rng.standard_normal(g.shape)
    code = {"periodic": dg.DG_BC_PERIODIC, "dirichlet": dg.DG_BC_DIRICHLET}
    grid = dg.Grid(n, nx, ny, 0.0, 2.0, -1.0, 1.5, code[bx], code[by])
    got = dg.bracket_form(grid, _dev(f), _dev(h), form).cpu().numpy()
    Jpp, Jpx, Jxp = O.bracket_forms(g, f, h)
    ref = [(Jpp + Jpx + Jxp) / 3, Jpp, Jpx, Jxp][form]
    # (a form can vanish identically, e.g. on a 1 x 1 periodic axis: then the
    # bar is 1e-12 of the inputs' O(1) scale)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1.0)


@pytest.mark.parametrize("rw", [8, 16])
def test_table2_dirichlet_row_on_gpu(dg, rw):
    g = O.Grid2D(3, 112, 112, 0.0, math.pi, 0.0, math.pi, "dirichlet", "dirichlet")
    f, h = I.conservation_pair(3, 112)
    grid = dg.Grid(3, 112, 112, 0.0, math.pi, 0.0, math.pi, dg.DG_BC_DIRICHLET,
                   dg.DG_BC_DIRICHLET)
    grid.set_tiles(8, rw)
    J = dg.poisson_bracket(grid, _dev(f), _dev(h)).cpu().numpy()
    got = [O.inner(g, np.ones_like(f), J), O.inner(g, f, J), O.inner(g, h, J)]
    for v, p in zip(got, (-0.19, 0.034, -0.79)):
        digits = 2 - int(math.floor(math.log10(abs(p)))) - 1
        assert round(v, digits) == p, (v, p)


def test_dirichlet_grid_rejects_solver_paths(dg):
    grid = dg.Grid(2, 8, 8, bc_y=dg.DG_BC_DIRICHLET)
    w = torch.zeros(grid.shape, dtype=torch.float64, device="cuda")
    ws = dg.Workspace(grid)
    for call in (lambda: dg.cg_solve_poisson(grid, w, torch.zeros_like(w), ws),
                 lambda: dg.rk_step(grid, w, dg.State(grid), ws, 1e-3, 0.0),
                 lambda: dg.laplace_apply(grid, w),
                 lambda: grid.tune(w),
                 lambda: dg.Batch(2).attach(grid, w, 1e-3, 0.0)):
        with pytest.raises(dg.DgError) as e:
            call()
        assert e.value.code == dg.DG_E_UNSUPPORTED
