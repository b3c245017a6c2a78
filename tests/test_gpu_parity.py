"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
* bracket, Laplacian: element-wise max error <= 1e-12 x max |oracle| on
  inputs without cancellation (white noise, spectral fields for the
  bracket); FP64 with a different but fixed summation order.
* CG: the GPU solution's residual, recomputed with the oracle's operator,
  meets 1.5 x rtol; the difference to the oracle's solution is bounded by
  the conditioning (kappa x rtol); iteration counts agree within 2.
* trajectories (smooth, 10 RK3 steps): <= 1e-12 relative with both solves
  at rtol 1e-14.
"""
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


GRIDS = [(1, 1), (2, 3), (3, 5), (7, 4), (37, 23), (64, 40)]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nx,ny", GRIDS)
def test_laplace_parity(dg, n, nx, ny):
    print(f"laplace n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny, 0.0, 2.0, -1.0, 1.5)
    u = I.white_noise(n, nx, ny, seed=nx * 7 + ny + n)
    grid = dg.Grid(n, nx, ny, 0.0, 2.0, -1.0, 1.5)
    got = dg.laplace_apply(grid, _dev(u)).cpu().numpy()
    ref = O.laplacian(g, u)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nx,ny", GRIDS)
@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_bracket_parity(dg, n, nx, ny, form):
    print(f"bracket n={n} nx={nx} ny={ny} form={form}", flush=True)
    g = O.Grid2D(n, nx, ny, 0.0, 2.0, -1.0, 1.5)
    rng = np.random.default_rng(n + 10 * nx + 100 * ny)
    f, h = rng.standard_normal((2,) + g.shape)
    grid = dg.Grid(n, nx, ny, 0.0, 2.0, -1.0, 1.5)
    got = dg.bracket_form(grid, _dev(f), _dev(h), form).cpu().numpy()
    forms = O.bracket_forms(g, f, h)
    ref = (forms[0] + forms[1] + forms[2]) / 3 if form == 0 else forms[form - 1]
    scale = max(np.max(np.abs(f)) * np.max(np.abs(h)) / min(g.hx, g.hy) ** 2, 1.0)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-3 * scale)


def test_bracket_table2_on_gpu(dg):
    # Table 2 periodic rows reproduced by the GPU bracket (Sec. 5.2)
    f, h = I.conservation_pair(3, 112)
    g = O.Grid2D(3, 112, 112, 0.0, math.pi, 0.0, math.pi)
    grid = dg.Grid(3, 112, 112, 0.0, math.pi, 0.0, math.pi)
    W = g.weights()
    one = np.ones_like(f)
    expect = {1: (0.0, 0.068, -0.038), 2: (0.0, -0.068, 0.0), 3: (0.0, 0.0, 0.038),
              0: (0.0, 0.0, 0.0)}
    for form, vals in expect.items():
        J = dg.bracket_form(grid, _dev(f), _dev(h), form).cpu().numpy()
        got = [float(np.sum(W * v * J)) for v in (one, f, h)]
        for a, b in zip(got, vals):
            if b == 0.0:
                assert abs(a) < 1e-13
            else:
                assert round(a, 3) == b


def test_full_size_laplace_and_bracket(dg):
    # the metric workload's shape: n = 4, 512 x 512
    n, N = 4, 512
    print("full-size bracket/laplace n=4 N=512", flush=True)
    g = O.Grid2D(n, N, N)
    w = I.random_spectrum(n, N, k0=10.0, seed=1)
    u = I.white_noise(n, N, N, seed=5)
    grid = dg.Grid(n, N, N)
    ref = O.laplacian(g, u)
    got = dg.laplace_apply(grid, _dev(u)).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # bracket of a smooth spectral pair
    f = w
    h = np.sin(w)
    ref = O.bracket(g, f, h)
    got = dg.poisson_bracket(grid, _dev(f), _dev(h)).cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def _solve(dg, n, nx, ny, w, rtol, guess=None, max_iter=100000, mixed=False):
    grid = dg.Grid(n, nx, ny)
    ws = dg.Workspace(grid, dg.DG_PREC_MIXED if mixed else dg.DG_PREC_FP64)
    psi = _dev(np.zeros_like(w) if guess is None else guess)
    opts = dg.cg_opts(rtol=rtol, max_iter=max_iter,
                      precision=dg.DG_PREC_MIXED if mixed else dg.DG_PREC_FP64)
    res = dg.cg_solve_poisson(grid, _dev(w), psi, ws, opts)
    return res, psi.cpu().numpy()


@pytest.mark.parametrize("n,nx,ny", [(1, 9, 7), (2, 16, 16), (3, 32, 32), (4, 13, 29),
                                     (5, 24, 24), (3, 1, 5), (2, 3, 3)])
def test_cg_parity(dg, n, nx, ny):
    print(f"cg n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny)
    w = I.white_noise(n, nx, ny, seed=n) + 3.0  # nonzero mean is removed
    rtol = 1e-12
    res, psi = _solve(dg, n, nx, ny, w, rtol)
    ref = O.cg_poisson(g, w, rtol=rtol)
    assert res.converged
    assert abs(res.iters - ref.iters) <= 2, (res.iters, ref.iters)
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    assert math.sqrt(O.inner(g, r, r)) <= 1.5 * rtol * math.sqrt(O.inner(g, b, b))
    e = psi - ref.x
    assert math.sqrt(O.inner(g, e, e)) <= 1e-8 * math.sqrt(O.inner(g, ref.x, ref.x))
    assert abs(O.wmean(g, psi)) < 1e-13 * np.max(np.abs(psi))


def test_cg_edge_cases(dg):
    n, N = 2, 8
    g = O.Grid2D(n, N, N)
    # constant right-hand side: b = 0 -> psi = 0, no iterations
    res, psi = _solve(dg, n, N, N, np.full(g.shape, 2.5), 1e-12,
                      guess=I.white_noise(n, N, N, 3))
    assert res.converged and res.iters == 0 and np.all(psi == 0)
    # max_iter forces non-convergence, reported not raised
    w = I.white_noise(n, N, N, 4)
    res, psi = _solve(dg, n, N, N, w, 1e-12, max_iter=3)
    assert not res.converged and res.iters == 3
    # exact guess converges at r0
    ref = O.cg_poisson(g, w, rtol=1e-14)
    res, psi = _solve(dg, n, N, N, w, 1e-10, guess=ref.x)
    assert res.converged and res.iters == 0


def test_cg_full_size_residual(dg):
    n, N = 4, 512
    print("cg full size n=4 N=512", flush=True)
    g = O.Grid2D(n, N, N)
    w = I.random_spectrum(n, N, k0=10.0, seed=1)
    rtol = 1e-10
    res, psi = _solve(dg, n, N, N, w, rtol)
    assert res.converged
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    assert math.sqrt(O.inner(g, r, r)) <= 1.5 * rtol * math.sqrt(O.inner(g, b, b))


def test_mixed_precision_solve(dg):
    n, N = 5, 32
    g = O.Grid2D(n, N, N)
    w, _ = I.double_shear_layer(n, N)
    rtol = 1e-10
    r64, p64 = _solve(dg, n, N, N, w, rtol)
    rmx, pmx = _solve(dg, n, N, N, w, rtol, mixed=True)
    assert r64.converged and rmx.converged and rmx.outer_iters >= 1
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, pmx)
    assert math.sqrt(O.inner(g, r, r)) <= 1.5 * rtol * math.sqrt(O.inner(g, b, b))
    e = pmx - p64
    assert math.sqrt(O.inner(g, e, e)) <= 1e-7 * math.sqrt(O.inner(g, p64, p64))


def _true_rel_residual(g, w, psi):
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    return math.sqrt(O.inner(g, r, r) / O.inner(g, b, b))


@pytest.mark.parametrize("N", [128, 256])
def test_mixed_precision_large_grid(dg, N):
    # n = 5 double shear layer.  An FP64 residual is attainable only to
    # ~ eps |Lap_h| |psi| (~1.4e-10 of ||b|| at 128^2, growing ~6x per
    # doubling of N), so rtol = 1e-10 lies below what any FP64 evaluation
    # can confirm here: the FP64 CG stops on its recursive residual, the
    # mixed CG on its FP64 one or at the attainable accuracy (converged =
    # 2).  Bars: both stop, the mixed iterations stay within 12x the FP64
    # ones, and the mixed solution's true residual (oracle operator) is
    # within 1.5 x rtol or within 64x the FP64 solution's own.
    n = 5
    print(f"mixed n=5 N={N}", flush=True)
    g = O.Grid2D(n, N, N)
    w, _ = I.double_shear_layer(n, N)
    rtol = 1e-10
    r64, p64 = _solve(dg, n, N, N, w, rtol)
    rmx, pmx = _solve(dg, n, N, N, w, rtol, mixed=True)
    assert r64.converged and rmx.converged, (r64, rmx)
    assert rmx.iters <= 12 * r64.iters, (rmx.iters, r64.iters)
    t64, tmx = _true_rel_residual(g, w, p64), _true_rel_residual(g, w, pmx)
    assert tmx <= max(1.5 * rtol, 64 * t64), (tmx, t64)
    assert abs(tmx - rmx.rel_residual) <= 0.5 * tmx + 1e-11
    e = pmx - p64
    assert math.sqrt(O.inner(g, e, e)) <= 1e-5 * math.sqrt(O.inner(g, p64, p64))


def test_rk3_config1_trajectory(dg):
    # 10 SSP-RK3 steps, n = 3, 32 x 32, D = 1e-3, dt = 1e-3 (Taylor-Green +
    # 1e-3 noise); both sides solve to rtol 1e-13 (1e-14 lies below the
    # attainable FP64 residual of this operator: the oracle's CG stalls there)
    n, N, D, dt, steps = 3, 32, 1e-3, 1e-3, 10
    print("rk3 config1", flush=True)
    g = O.Grid2D(n, N, N)
    w0 = I.taylor_green_noise(n, N, seed=0)
    grid = dg.Grid(n, N, N)
    ws = dg.Workspace(grid)
    st = dg.State(grid)
    w = _dev(w0)
    wr, t, hist = w0.copy(), 0.0, O.PsiHistory()
    opts = dg.cg_opts(rtol=1e-13)
    for k in range(steps):
        res = dg.rk_step(grid, w, st, ws, dt, D, opts)
        wr, its = O.rk3_step(g, wr, t, dt, D, hist, rtol=1e-13, max_iter=5000)
        t += dt
        assert res.converged
        assert all(abs(a - b) <= 2 for a, b in zip(res.cg_iters, its)), (res.cg_iters, its)
    got = w.cpu().numpy()
    e = got - wr
    assert math.sqrt(O.inner(g, e, e) / O.inner(g, wr, wr)) <= 1e-12
    assert abs(st.t - steps * dt) < 1e-15
    # invariants of the final state
    psi = st.psi().cpu().numpy()
    V, E, Om = dg.invariants(grid, w, _dev(psi), ws)
    Vr, Er, Omr = O.invariants(g, got, psi)
    assert abs(V - Vr) <= 1e-13 and abs(E - Er) <= 1e-13 * abs(Er) and abs(Om - Omr) <= 1e-13 * Omr


def test_inviscid_conservation_on_gpu(dg):
    # D = 0: V exact; Omega changes only through RK3 (tiny for small dt)
    n, N = 4, 32
    g = O.Grid2D(n, N, N)
    w0 = I.random_spectrum(n, N, k0=4.0, seed=2)
    grid = dg.Grid(n, N, N)
    ws = dg.Workspace(grid)
    st = dg.State(grid)
    w = _dev(w0)
    psi0 = torch.zeros_like(w)
    dg.cg_solve_poisson(grid, w, psi0, ws, dg.cg_opts(rtol=1e-13))
    V0, E0, Om0 = dg.invariants(grid, w, psi0, ws)
    for _ in range(5):
        dg.rk_step(grid, w, st, ws, 1e-3, 0.0, dg.cg_opts(rtol=1e-13))
    psi = torch.zeros_like(w)
    dg.cg_solve_poisson(grid, w, psi, ws, dg.cg_opts(rtol=1e-13))
    V, E, Om = dg.invariants(grid, w, psi, ws)
    assert abs(V) < 1e-12
    assert abs(Om - Om0) / Om0 < 1e-9
    assert abs(E - E0) / E0 < 1e-9


def test_bitwise_determinism(dg):
    n, N = 4, 64
    w0 = I.random_spectrum(n, N, k0=6.0, seed=9)
    outs = []
    for _ in range(2):
        grid = dg.Grid(n, N, N)
        ws = dg.Workspace(grid)
        st = dg.State(grid)
        w = _dev(w0)
        for _ in range(2):
            dg.rk_step(grid, w, st, ws, 1e-3, 1e-4, dg.cg_opts(rtol=1e-12))
        outs.append(w.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
