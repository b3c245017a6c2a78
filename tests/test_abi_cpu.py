"""CPU-side checks of the C ABI: the library loads and exports every symbol
the header declares; the host-built operator tables reproduce the oracle's
operators; argument validation fails cleanly without touching a GPU."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgark.h")
LIB = os.path.join(ROOT, "paper_1311_7477_amd", "libdgark.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="libdgark.so not built (run __graft_entry__.build())")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = _declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _tables(n, N=3, x1=1.0, y1=1.0, bc=0):
    from paper_1311_7477_amd import dg
    t = np.array(dg.Grid(n, N, N, 0.0, x1, 0.0, y1, bc_x=bc, bc_y=bc).tables())
    o = 0

    def take(m):
        nonlocal o
        v = t[o:o + m]
        o += m
        return v
    d = {}
    d["xi"], d["w"] = take(n), take(n)
    d["C0"] = take(n * n).reshape(n, n)
    d["cR"], d["sR"], d["cL"], d["sL"] = take(n), take(n), take(n), take(n)
    for ax in ("x", "y"):
        d["L0" + ax] = take(n * n).reshape(n, n)
        for k in ("eR", "lR", "eL", "lL"):
            d[k + ax] = take(n)
        d["L0B" + ax] = take(n * n).reshape(n, n)
        d["eRB" + ax] = take(n)
        d["lLB" + ax] = take(n)
    assert o == len(t)
    return d


def _assemble(n, N, A0, eR, tR, eL, tL):
    M = np.zeros((N * n, N * n))
    for m in range(N):
        b = slice(m * n, (m + 1) * n)
        M[b, b] += A0
        r = ((m + 1) % N) * n
        l_ = ((m - 1) % N) * n
        M[b, r:r + n] += np.outer(eR, tR)
        M[b, l_:l_ + n] += np.outer(eL, tL)
    return M


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_host_tables_reproduce_oracle_operators(n):
    # the C++ tables (built from the Legendre recursion and the block
    # algebra of the fluxes) against the oracle's sparse operators (built
    # from lspace_operator and the explicit jump operator); x and y with
    # different cell sizes, since the jump penalty makes the LDG blocks
    # depend on h
    N, lx, ly = 6, 1.7, 5.0
    d = _tables(n, N, lx, ly)
    for ax, length in (("x", lx), ("y", ly)):
        g = O.Grid1D(n, N, 0.0, length)
        np.testing.assert_allclose(d["xi"], g.el.xi, atol=1e-15)
        np.testing.assert_allclose(d["w"], g.el.w, atol=1e-15)
        Dc = _assemble(n, N, d["C0"], d["cR"], d["sR"], d["cL"], d["sL"]) / g.h
        ref = g.derivative("centred").toarray()
        np.testing.assert_allclose(Dc, ref, atol=1e-13 * np.abs(ref).max())
        Lp = _assemble(n, N, d["L0" + ax], d["eR" + ax], d["lR" + ax], d["eL" + ax],
                       d["lL" + ax]) / g.h ** 2
        ref = g.laplacian().toarray()
        np.testing.assert_allclose(Lp, ref, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("N", [1, 2, 6])
def test_host_tables_reproduce_oracle_dirichlet_laplacian(n, N):
    # homogeneous Dirichlet axis: interior blocks, the last cell without its
    # right coupling, the first cell with L0B / eRB and no left coupling, the
    # second one coupled to the first through lLB,
    # against the oracle's operator built from the boundary fluxes and the
    # jump operator with its two boundary faces
    lx, ly = 1.3, 2.9
    d = _tables(n, N, lx, ly, bc=1)
    for ax, length in (("x", lx), ("y", ly)):
        g = O.Grid1D(n, N, 0.0, length, "dirichlet")
        M = np.zeros((N * n, N * n))
        for m in range(N):
            b = slice(m * n, (m + 1) * n)
            first = m == 0
            M[b, b] += d["L0B" + ax] if first else d["L0" + ax]
            if m + 1 < N:
                eR = d["eRB" + ax] if first else d["eR" + ax]
                M[b, (m + 1) * n:(m + 2) * n] += np.outer(eR, d["lR" + ax])
            if m > 0:
                lL = d["lLB" + ax] if m == 1 else d["lL" + ax]
                M[b, (m - 1) * n:m * n] += np.outer(d["eL" + ax], lL)
        M /= g.h ** 2
        ref = g.laplacian().toarray()
        np.testing.assert_allclose(M, ref, atol=1e-13 * np.abs(ref).max())


def test_grid_create_validation():
    from paper_1311_7477_amd import dg
    for bad in [dict(n=0), dict(n=6), dict(nx=0), dict(ny=-1), dict(x1=-1.0),
                dict(y1=float("nan"))]:
        args = dict(n=2, nx=4, ny=4, x1=1.0, y1=1.0)
        args.update(bad)
        with pytest.raises(dg.DgError) as ei:
            dg.Grid(args["n"], args["nx"], args["ny"], 0.0, args["x1"], 0.0, args["y1"])
        assert ei.value.code == dg.DG_E_INVAL
    with pytest.raises(dg.DgError) as ei:
        dg.Grid(2, 4, 4, bc_x=7)
    assert ei.value.code == dg.DG_E_INVAL
    # a Dirichlet axis: no host-built Bloch basis (the periodic axis of the
    # same grid has one), cell tiles of 8 waves only; host-side rejections
    # need no GPU
    d = dg.Grid(2, 4, 4, bc_x=dg.DG_BC_DIRICHLET)
    with pytest.raises(dg.DgError) as ei:
        d.fd_basis(0)
    assert ei.value.code == dg.DG_E_UNSUPPORTED
    assert d.fd_basis(1)[0].shape == (8, 8)
    with pytest.raises(dg.DgError) as ei:
        d.set_tiles(16, 8)
    assert ei.value.code == dg.DG_E_INVAL
    d.set_tiles(8, 16)
    assert d.tiles() == (8, 16)


def test_workspace_bytes_and_field_size():
    from paper_1311_7477_amd import dg
    g = dg.Grid(4, 512, 512)
    assert g.elems == 512 * 512 * 16
    F = g.elems * 8
    # CG vectors x, r, p0, p1 (lane-interleaved, no padding when 64 | nx),
    # RK stage fields s1, s2, reduction scratch
    b64, bmx = g.workspace_bytes(dg.DG_PREC_FP64), g.workspace_bytes(dg.DG_PREC_MIXED)
    assert 6 * F <= b64 < 6 * F + 2 ** 20
    assert bmx == b64 + 3 * g.elems * 4          # FP32 r, p0, p1
    # fast-diagonalisation option: z, two node-plane fields, and per axis
    # (square grid: the y factors are the x factors) the cell Fourier basis
    # (N x N), the forward and inverse mixing blocks (K = N/2 + 1 blocks of
    # 2n x 2n) and the eigenvalues (n N), each in FP64 and FP32, plus the K
    # cos / sin column pairs
    def axis(N, n):
        K = N // 2 + 1
        return (N * N + 2 * K * (2 * n) ** 2 + N * n) * (8 + 4) + 2 * K * 4

    def field(n, Nx, Ny):
        # a work field holds the node planes or the packed spectra of the
        # FFTs along x or y, with room for N/2 + 1 complex values per row
        return 8 * n * n * max(Nx * Ny, Ny * 2 * (Nx // 2 + 1), Nx * 2 * (Ny // 2 + 1))
    # ... plus, for RK steps queued ahead, a copy of omega and three sets of
    # device CG scalars (18 doubles and 10 ints each)
    queued = F + 3 * (18 * 8 + 10 * 4)
    bfd = g.workspace_bytes(dg.DG_PREC_FP64 | dg.DG_WS_FD)
    assert bfd == b64 + F + 2 * field(4, 512, 512) + axis(512, 4) + queued
    # unequal axes keep both factor sets
    r = dg.Grid(2, 6, 5)
    extra = r.workspace_bytes(dg.DG_WS_FD) - r.workspace_bytes(dg.DG_PREC_FP64)
    L6 = 5 * 1 * 4 * 64
    assert extra == (L6 * 8 + 2 * field(2, 6, 5) + axis(6, 2) + axis(5, 2)
                     + r.elems * 8 + 3 * (18 * 8 + 10 * 4))
    # ragged nx: the interleaved vectors are padded to whole groups of 64 cells
    h = dg.Grid(3, 100, 7)
    L = 7 * 2 * 9 * 64
    assert h.workspace_bytes(dg.DG_PREC_FP64) >= 4 * L * 8 + 2 * h.elems * 8
    with pytest.raises(dg.DgError):
        g.workspace_bytes(7)
    # the product-path option changes no allocation and needs DG_WS_FD
    assert g.workspace_bytes(dg.DG_WS_FD | dg.DG_WS_FD_PRODUCTS) == bfd
    assert (g.workspace_bytes(dg.DG_PREC_MIXED | dg.DG_WS_FD | dg.DG_WS_FD_PRODUCTS)
            == g.workspace_bytes(dg.DG_PREC_MIXED | dg.DG_WS_FD))
    with pytest.raises(dg.DgError) as e:
        g.workspace_bytes(dg.DG_WS_FD_PRODUCTS)
    assert e.value.code == dg.DG_E_INVAL
    # a Dirichlet axis: two dense work images and per axis the dense
    # (n N)^2 eigenbasis and n N eigenvalues in FP64 and FP32
    def dense(N, n):
        m = N * n
        return (m * m + m) * (8 + 4)
    d = dg.Grid(3, 40, 24, bc_y=dg.DG_BC_DIRICHLET)
    Ld = 24 * 1 * 9 * 64
    extra = d.workspace_bytes(dg.DG_WS_FD) - d.workspace_bytes(dg.DG_PREC_FP64)
    assert extra == (Ld * 8 + 2 * 8 * 9 * 40 * 24 + dense(40, 3) + dense(24, 3)
                     + d.elems * 8 + 3 * (18 * 8 + 10 * 4))
    sq = dg.Grid(2, 16, 16, bc_x=dg.DG_BC_DIRICHLET, bc_y=dg.DG_BC_DIRICHLET)
    Ls = 16 * 1 * 4 * 64
    extra = sq.workspace_bytes(dg.DG_WS_FD) - sq.workspace_bytes(dg.DG_PREC_FP64)
    assert extra == (Ls * 8 + 2 * 8 * 4 * 16 * 16 + dense(16, 2)
                     + sq.elems * 8 + 3 * (18 * 8 + 10 * 4))


def test_null_arguments_are_rejected():
    from paper_1311_7477_amd import dg
    L = dg.lib()
    g = dg.Grid(2, 4, 4)
    assert L.dg_laplace_apply(g.handle, None, None, None) == dg.DG_E_INVAL
    assert L.dg_poisson_bracket(g.handle, None, None, None, None) == dg.DG_E_INVAL
    assert b"NULL" in L.dg_last_error()
    assert L.dg_cg_solve_poisson(g.handle, None, None, None, None, None, None) == dg.DG_E_INVAL
    x = ctypes.c_void_p(0x1000)
    # aliasing is detected before any launch
    assert L.dg_laplace_apply(g.handle, x, x, None) == dg.DG_E_ALIAS
    assert L.dg_poisson_bracket(g.handle, x, ctypes.c_void_p(0x100000), x, None) == dg.DG_E_ALIAS
    assert L.dg_bracket_form(g.handle, ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000),
                             ctypes.c_void_p(0x30000), 9, None) == dg.DG_E_INVAL
    assert L.dg_batch_use_precond(None, dg.DG_WS_FD) == dg.DG_E_INVAL


@pytest.mark.parametrize("n,N,length", [(1, 7, 1.0), (2, 6, 2.0), (3, 5, 6.283185307179586),
                                        (4, 8, 0.5), (5, 9, 3.0), (4, 1, 1.0), (2, 2, 1.0)])
def test_fd_basis_diagonalises_the_oracle_operator(n, N, length):
    # The host-built Bloch eigenbasis against the oracle's sparse 1D LDG
    # operator and Gauss weights: L V = V diag(lam), V^T W V = I, the
    # constant mode, and the spectrum of the oracle's dense eigh.
    from paper_1311_7477_amd import dg
    g = dg.Grid(n, N, 3, 0.0, length, 0.0, 1.0)
    V, lam, zero = g.fd_basis(0)
    g1 = O.Grid1D(n, N, 0.0, length)
    L = g1.laplacian().toarray()
    W = np.diag(g1.weights())
    scale = np.abs(lam).max()
    assert np.abs(L @ V - V * lam[None, :]).max() <= 1e-11 * scale * np.abs(V).max()
    assert np.abs(V.T @ W @ V - np.eye(N * n)).max() <= 1e-12
    assert abs(lam[zero]) <= 1e-11 * scale
    c = V[:, zero]
    assert np.ptp(c) <= 1e-12 * np.abs(c).max()
    ref = np.sort(np.linalg.eigvals(L).real)
    np.testing.assert_allclose(np.sort(lam), ref, atol=1e-10 * scale)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("N", [1, 2, 3, 7])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_axis_operator_is_the_oracle_operator(n, N, bc):
    # The host assembly of the 1D LDG second derivative (the operator the
    # preconditioner diagonalises, densely on a Dirichlet axis) against the
    # oracle's sparse 1D operator, built independently from the flux
    # definitions (Sec. 6 with the jump penalty and the boundary closure)
    from paper_1311_7477_amd import dg
    code = {"periodic": dg.DG_BC_PERIODIC, "dirichlet": dg.DG_BC_DIRICHLET}
    g = dg.Grid(n, N, N + 2, 0.0, 1.7, -1.0, 4.0, code[bc], code[bc])
    for axis, (Nc, a, b) in enumerate([(N, 0.0, 1.7), (N + 2, -1.0, 4.0)]):
        ref = O.Grid1D(n, Nc, a, b, bc).laplacian().toarray()
        got = g.axis_operator(axis)
        assert got.shape == ref.shape
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_tile_shapes_default_and_validation():
    from paper_1311_7477_amd import dg
    g = dg.Grid(3, 10, 12)
    assert g.tiles() == (8, 8)
    for cw, rw in [(4, 8), (16, 16), (8, 16)]:
        g.set_tiles(cw, rw)
        assert g.tiles() == (cw, rw)
    for cw, rw in [(2, 8), (8, 4), (32, 8), (8, 32), (0, 0)]:
        with pytest.raises(dg.DgError) as e:
            g.set_tiles(cw, rw)
        assert e.value.code == dg.DG_E_INVAL
    assert g.tiles() == (8, 16)
    # workspaces are sized for every tile shape: the same bytes whatever the shape
    b = g.workspace_bytes()
    g.set_tiles(4, 8)
    assert g.workspace_bytes() == b
