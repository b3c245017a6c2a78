"""dg_invariants_noalloc (the allocation-free variant of dg_invariants_dev)
against dg_invariants_dev, through the C ABI: the same kernel and the same
block count, so the three sums must agree bit for bit.  Two calls in a row,
the second on a smaller grid, so that the shared static scratch is reused
with fewer blocks."""
import numpy as np
import pytest

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


def _case(dg, n, nx, ny, seed):
    grid = dg.Grid(n, nx, ny)
    w = torch.from_numpy(I.white_noise(n, nx, ny, seed=seed)).to("cuda")
    psi = torch.from_numpy(I.white_noise(n, nx, ny, seed=seed + 1)).to("cuda")
    return grid, w, psi


def test_noalloc_invariants_match_workspace_variant(dg):
    print("noalloc invariants: n=4 300x260 then n=2 7x5", flush=True)
    outs = []
    for n, nx, ny, seed in ((4, 300, 260, 3), (2, 7, 5, 8)):
        grid, w, psi = _case(dg, n, nx, ny, seed)
        ws = dg.Workspace(grid)
        ref = dg.invariants_dev(grid, w, psi, ws)
        got = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        dg.invariants_noalloc(grid, w, psi, got)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), (a, b)
        # the host-returning variant agrees too
        assert np.array_equal(a, np.array(dg.invariants(grid, w, psi, ws)))
        outs.append(a)
    assert not np.array_equal(outs[0], outs[1])
    # repeated calls on one stream reuse the scratch: same values again
    grid, w, psi = _case(dg, 4, 300, 260, 3)
    again = torch.empty(3, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dg.invariants_noalloc(grid, w, psi, again)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy(), outs[0])


def test_noalloc_invariants_rejects_null(dg):
    grid, w, psi = _case(dg, 2, 4, 4, 1)
    L = dg.lib()
    rc = L.dg_invariants_noalloc(grid.handle, None, dg._vp(psi.data_ptr()),
                                 dg._vp(w.data_ptr()), dg._stream())
    assert rc == dg.DG_E_INVAL
