"""Parity of the fast-diagonalisation preconditioner and of the
preconditioned CG (through the C ABI) with the FP64 oracle.

Tolerances:
* z = (-Lap_h)^+ r: both sides are exact up to rounding, from different
  eigenbases (the device: the host-built Bloch basis in factored form, cell
  Fourier transforms and per-wave-number mixing; the oracle: numpy eigh of
  the dense 1D operators).  Eigenvalues
  carry absolute errors ~ eps x lambda_max, so the smallest modes -- which
  dominate z -- agree only to ~ eps x kappa relative, kappa =
  mu_max / mu_min of -Lap_h (dense eigh can lose a further LAPACK-dependent
  factor of ~10-30 on the smallest eigenvalues): element-wise max error of
  the W-mean-free parts <= 2e-14 x kappa x max |oracle| (the oracle's eigh
  leaves a roundoff-size constant in its result; the device's is checked to
  be zero-mean).  The sharp check is the residual: ||b + Lap_h z||_W <=
  1e-11 ||b||_W with the oracle's operator.
* PCG: the GPU solution's residual, recomputed with the oracle's operator,
  meets 1.5 x rtol (at the full 512^2 size rtol is 1e-10: the FP64 residual
  of a solution is attainable only to ~ eps lambda_max ||psi||, ~1e-11 of
  ||b|| there); its difference to the oracle's solution is bounded by the
  conditioning; an exact preconditioner converges in at most 2 iterations
  on both sides.
* Mixed-precision PCG (the preconditioner applied in FP32, the iteration in
  FP64): the same residual bound as the FP64 PCG, since every residual is
  FP64; the FP32 apply is exact to ~1e-6 relative, so each iteration gains
  about six digits and at most 4 iterations reach 1e-12.  At the full
  double-shear-layer size (n = 5, 1024^2) the recomputed residual meets
  1.5 x rtol or is within 2x of the FP64 PCG's (the attainable accuracy
  there is ~1e-9 of ||b||), and the solutions agree to 1e-8.
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


def _wn(g, u):
    return math.sqrt(O.inner(g, u, u))


CASES = [(1, 5, 4, 1.0, 1.3), (2, 6, 6, 2.0, 2.0), (3, 37, 23, 2.0, 1.5),
         (4, 64, 40, 6.283185307179586, 6.283185307179586), (5, 7, 4, 1.0, 3.0),
         (4, 1, 3, 1.0, 1.0), (2, 2, 2, 1.0, 1.0), (5, 64, 64, 6.283185307179586, 6.283185307179586),
         # beyond 512 cells on an axis with both counts even the cell
         # transforms are FFTs of half length: N/2 even and odd on either
         # axis, the other axis below and above 512, a 6-cell axis (three
         # complex values per row); an odd count keeps the folded products
         (2, 1024, 96, 6.283185307179586, 3.0), (1, 522, 530, 1.0, 1.2),
         (3, 516, 6, 1.5, 1.0), (1, 601, 520, 2.0, 2.5),
         # a 4-cell axis on the FFT path: its one wave pair carries the wave
         # numbers 0, 2 (column 0) and 1 (the partner slot); short axes whose
         # few pairs leave most of a tile's pair slots empty (8 cells: pairs
         # 0, 1 and the merged wave number 2; 6 cells: half length 3, odd)
         (2, 40, 4, 1.0, 1.0), (3, 48, 8, 2.0, 1.0), (2, 36, 6, 1.0, 1.5)]


@pytest.mark.parametrize("n,nx,ny,lx,ly", CASES)
def test_precond_apply_parity(dg, n, nx, ny, lx, ly):
    print(f"precond apply n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny, 0.0, lx, 0.0, ly)
    r = I.white_noise(n, nx, ny, seed=5 * n + nx) + 0.7     # the mean is dropped
    grid = dg.Grid(n, nx, ny, 0.0, lx, 0.0, ly)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    got = dg.precond_apply(grid, _dev(r), ws).cpu().numpy()
    fd = O.FastDiagonalisation(g)
    ref = fd.apply(r)
    inv = np.abs(fd.inv_mu[fd.inv_mu != 0])
    kappa = inv.max() / inv.min()
    # the constant mode is the null space: both results are compared with
    # their (roundoff-size) W-means removed
    d = (got - O.wmean(g, got)) - (ref - O.wmean(g, ref))
    assert np.max(np.abs(d)) <= 2e-14 * kappa * np.max(np.abs(ref))
    assert abs(O.wmean(g, got)) <= 1e-13 * np.max(np.abs(ref))
    b = r - O.wmean(g, r)
    assert _wn(g, b + O.laplacian(g, got)) <= 1e-11 * _wn(g, b)


@pytest.mark.parametrize("n,nx,ny,lx,ly", [c for c in CASES
                                            if c[1] % 2 == 0 and c[2] % 2 == 0
                                            and max(c[1], c[2]) > 32])
def test_precond_apply_products_option(dg, n, nx, ny, lx, ly):
    # grids that take the FFT path by default, with DG_WS_FD_PRODUCTS: the
    # folded matrix products, against the oracle at the same bar, and against
    # the FFT path (two exact inverses: within 2e-14 kappa)
    print(f"precond apply (products) n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny, 0.0, lx, 0.0, ly)
    r = I.white_noise(n, nx, ny, seed=5 * n + nx) + 0.7
    grid = dg.Grid(n, nx, ny, 0.0, lx, 0.0, ly)
    ws_p = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD | dg.DG_WS_FD_PRODUCTS)
    ws_f = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    got = dg.precond_apply(grid, _dev(r), ws_p).cpu().numpy()
    fft = dg.precond_apply(grid, _dev(r), ws_f).cpu().numpy()
    fd = O.FastDiagonalisation(g)
    ref = fd.apply(r)
    inv = np.abs(fd.inv_mu[fd.inv_mu != 0])
    kappa = inv.max() / inv.min()
    scale = np.max(np.abs(ref))
    d = (got - O.wmean(g, got)) - (ref - O.wmean(g, ref))
    assert np.max(np.abs(d)) <= 2e-14 * kappa * scale
    d = (got - O.wmean(g, got)) - (fft - O.wmean(g, fft))
    assert np.max(np.abs(d)) <= 2e-14 * kappa * scale
    b = r - O.wmean(g, r)
    assert _wn(g, b + O.laplacian(g, got)) <= 1e-11 * _wn(g, b)


def _pcg(dg, n, nx, ny, w, rtol, guess=None, precond=True, max_iter=100000, mixed=False):
    grid = dg.Grid(n, nx, ny)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    psi = _dev(np.zeros_like(w) if guess is None else guess)
    opts = dg.cg_opts(rtol=rtol, max_iter=max_iter,
                      precision=dg.DG_PREC_MIXED if mixed else dg.DG_PREC_FP64,
                      precond=dg.DG_PRECOND_FD if precond else dg.DG_PRECOND_NONE)
    res = dg.cg_solve_poisson(grid, _dev(w), psi, ws, opts)
    return res, psi.cpu().numpy()


# the last cases take the FFT path (N/2 odd on both axes; one short axis)
@pytest.mark.parametrize("n,nx,ny", [(1, 9, 7), (2, 16, 16), (3, 37, 23), (4, 13, 29),
                                     (5, 24, 24), (3, 1, 5), (1, 522, 530), (2, 1024, 96)])
def test_pcg_parity(dg, n, nx, ny):
    print(f"pcg n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny)
    w = I.white_noise(n, nx, ny, seed=n) + 3.0
    rtol = 1e-12
    res, psi = _pcg(dg, n, nx, ny, w, rtol)
    ref = O.pcg_poisson(g, w, rtol=rtol, precond=O.FastDiagonalisation(g).apply)
    assert res.converged and ref.converged
    assert res.iters <= 2 and ref.iters <= 2 and abs(res.iters - ref.iters) <= 1
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    assert _wn(g, r) <= 1.5 * rtol * _wn(g, b)
    assert _wn(g, psi - ref.x) <= 1e-9 * _wn(g, ref.x)
    assert abs(O.wmean(g, psi)) < 1e-13 * np.max(np.abs(psi))


@pytest.mark.parametrize("n,nx,ny", [(1, 9, 7), (2, 16, 16), (3, 37, 23), (4, 13, 29),
                                     (5, 24, 24), (3, 1, 5), (4, 64, 48), (1, 522, 530),
                                     (2, 1024, 96), (3, 48, 8), (2, 36, 6)])
def test_pcg_mixed_parity(dg, n, nx, ny):
    print(f"mixed pcg n={n} nx={nx} ny={ny}", flush=True)
    g = O.Grid2D(n, nx, ny)
    w = I.white_noise(n, nx, ny, seed=n + 11) + 3.0
    rtol = 1e-12
    res, psi = _pcg(dg, n, nx, ny, w, rtol, mixed=True)
    ref = O.pcg_poisson(g, w, rtol=rtol, precond=O.FastDiagonalisation(g).apply)
    assert res.converged and 1 <= res.iters <= 4
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    assert _wn(g, r) <= 1.5 * rtol * _wn(g, b)
    assert _wn(g, psi - ref.x) <= 1e-9 * _wn(g, ref.x)
    assert abs(O.wmean(g, psi)) < 1e-13 * np.max(np.abs(psi))


def test_pcg_edge_cases(dg):
    n, N = 3, 8
    g = O.Grid2D(n, N, N)
    res, psi = _pcg(dg, n, N, N, np.full(g.shape, -1.5), 1e-12,
                    guess=I.white_noise(n, N, N, 2))
    assert res.converged and res.iters == 0 and np.all(psi == 0)
    w = I.white_noise(n, N, N, 6)
    ref = O.dense_poisson_solve(g, w)
    res, psi = _pcg(dg, n, N, N, w, 1e-10, guess=ref)
    assert res.converged and res.iters == 0
    res, psi = _pcg(dg, n, N, N, w, 1e-12, max_iter=0)
    assert not res.converged and res.iters == 0


def test_pcg_full_size(dg):
    # the bench workload's shape: n = 4, 512 x 512, random-spectrum omega
    n, N = 4, 512
    print("pcg full size n=4 N=512", flush=True)
    g = O.Grid2D(n, N, N)
    w = I.random_spectrum(n, N, k0=10.0, seed=1)
    rtol = 1e-10
    res, psi = _pcg(dg, n, N, N, w, rtol)
    assert res.converged and res.iters <= 2
    b = w - O.wmean(g, w)
    r = b + O.laplacian(g, psi)
    assert _wn(g, r) <= 1.5 * rtol * _wn(g, b)
    plain, p0 = _pcg(dg, n, N, N, w, rtol, precond=False)
    assert plain.converged
    assert _wn(g, psi - p0) <= 1e-8 * _wn(g, p0)


def test_pcg_mixed_full_size_shear_layer(dg):
    # the double shear layer at n = 5, 1024 x 1024 (the mixed-precision workload)
    n, N = 5, 1024
    print("mixed pcg full size n=5 N=1024", flush=True)
    w, _ = I.double_shear_layer(n, N)
    rtol = 1e-10
    r64, p64 = _pcg(dg, n, N, N, w, rtol)
    rmx, pmx = _pcg(dg, n, N, N, w, rtol, mixed=True)
    print(f"iterations fp64 {r64.iters} mixed {rmx.iters}", flush=True)
    assert r64.converged and rmx.converged and rmx.iters <= 4
    g = O.Grid2D(n, N, N)
    b = w - O.wmean(g, w)
    bn = _wn(g, b)
    t64 = _wn(g, b + O.laplacian(g, p64))
    tmx = _wn(g, b + O.laplacian(g, pmx))
    assert tmx <= max(1.5 * rtol * bn, 2.0 * t64)
    assert _wn(g, pmx - p64) <= 1e-8 * _wn(g, p64)


def test_rk_step_preconditioned_matches_plain(dg):
    n, N, D = 4, 48, 1e-4
    w0, umax = I.random_spectrum(n, N, k0=4.0, seed=2, return_umax=True)
    dt = I.cfl_dt(n, N, umax)
    out = {}
    for pc in (dg.DG_PRECOND_NONE, dg.DG_PRECOND_FD):
        grid = dg.Grid(n, N, N)
        ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
        st = dg.State(grid)
        w = _dev(w0)
        its = []
        for _ in range(3):
            r = dg.rk_step(grid, w, st, ws, dt, D, dg.cg_opts(rtol=1e-13, precond=pc))
            assert r.converged
            its += r.cg_iters
        out[pc] = (w.cpu().numpy(), its)
    a, b = out[dg.DG_PRECOND_NONE][0], out[dg.DG_PRECOND_FD][0]
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(a))
    assert max(out[dg.DG_PRECOND_FD][1]) <= 2 < min(out[dg.DG_PRECOND_NONE][1])


def test_precond_errors(dg):
    grid = dg.Grid(2, 8, 8)
    plain = dg.Workspace(grid)
    w = torch.zeros(grid.shape, dtype=torch.float64, device="cuda")
    psi = torch.zeros_like(w)
    with pytest.raises(dg.DgError) as e:
        dg.cg_solve_poisson(grid, w, psi, plain, dg.cg_opts(precond=dg.DG_PRECOND_FD))
    assert e.value.code == dg.DG_E_WORKSPACE
    with pytest.raises(dg.DgError) as e:
        dg.precond_apply(grid, w, plain)
    assert e.value.code == dg.DG_E_WORKSPACE
    both = dg.Workspace(grid, dg.DG_PREC_MIXED | dg.DG_WS_FD)
    res = dg.cg_solve_poisson(grid, w, psi, both, dg.cg_opts(precision=dg.DG_PREC_MIXED,
                                                               precond=dg.DG_PRECOND_FD))
    assert res.converged and res.iters == 0 and float(psi.abs().max()) == 0.0
    with pytest.raises(dg.DgError) as e:
        dg.cg_solve_poisson(grid, w, psi, both, dg.cg_opts(precision=7,
                                                             precond=dg.DG_PRECOND_FD))
    assert e.value.code == dg.DG_E_INVAL
    with pytest.raises(dg.DgError) as e:
        dg.precond_apply(grid, w, both, out=w)
    assert e.value.code == dg.DG_E_ALIAS
    # a batch takes preconditioned steps only with the preconditioner chosen
    # before its members attach
    b = dg.Batch(2)
    b.attach(grid, w.clone(), 1e-3, 0.0)
    with pytest.raises(dg.DgError) as e:
        b.rk_step(dg.cg_opts(precond=dg.DG_PRECOND_FD))
    assert e.value.code == dg.DG_E_WORKSPACE
    with pytest.raises(dg.DgError) as e:
        b.use_precond()
    assert e.value.code == dg.DG_E_INVAL
    with pytest.raises(dg.DgError) as e:
        dg.Batch(1).use_precond(0x40)
    assert e.value.code == dg.DG_E_INVAL
    with pytest.raises(dg.DgError) as e:
        b.rk_step(dg.cg_opts(precision=dg.DG_PREC_MIXED))
    assert e.value.code == dg.DG_E_UNSUPPORTED


@pytest.mark.parametrize("D", [0.0, 1e-4])
def test_full_size_turbulence_invariants(dg, D):
    # The decaying-turbulence workload at its full size (n = 4, 512^2,
    # k0 = 10, seed 1, CFL 0.1) for 20 SSP-RK3 steps with the preconditioned
    # solve: the device invariants equal the oracle's sums of the same
    # fields; V stays at roundoff; with D = 0 E and Omega change only by the
    # time-stepping error (~1e-15 per step, relative), with D > 0 both
    # decrease at every step (dOmega/dt = D <omega, Lap_h omega>_W <= 0).
    n, N = 4, 512
    print(f"full-size invariants D={D}", flush=True)
    w0, umax = I.random_spectrum(n, N, k0=10.0, seed=1, return_umax=True)
    dt = I.cfl_dt(n, N, umax, cfl=0.1)
    g = O.Grid2D(n, N, N)
    grid = dg.Grid(n, N, N)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    opts = dg.cg_opts(rtol=1e-12, precond=dg.DG_PRECOND_FD)
    st, w = dg.State(grid), _dev(w0)

    def invariants():
        psi = torch.zeros_like(w)
        assert dg.cg_solve_poisson(grid, w, psi, ws, opts).converged
        return dg.invariants(grid, w, psi, ws), psi
    (V0, E0, Om0), psi = invariants()
    Vr, Er, Omr = O.invariants(g, w0, psi.cpu().numpy())
    assert abs(V0 - Vr) <= 1e-12 and abs(E0 - Er) <= 1e-12 * Er and abs(Om0 - Omr) <= 1e-12 * Omr
    hist = [(E0, Om0)]
    for _ in range(20):
        assert dg.rk_step(grid, w, st, ws, dt, D, opts).converged
        (V, E, Om), _ = invariants()
        hist.append((E, Om))
        assert abs(V) <= 1e-12 * math.sqrt(Om0)
    E, Om = hist[-1]
    if D == 0.0:
        assert abs(E - E0) <= 1e-11 * E0 and abs(Om - Om0) <= 1e-11 * Om0
    else:
        assert all(b[1] < a[1] and b[0] < a[0] for a, b in zip(hist, hist[1:]))
        # the enstrophy lost over 20 steps against its initial rate
        # D <omega, Lap_h omega>_W (the rate changes little over 20 dt)
        rate0 = D * O.inner(g, w0, O.laplacian(g, w0))
        assert 0.5 <= (Om - Om0) / (20 * dt * rate0) <= 2.0
