"""Batched form: every instance of a batch must give bitwise the same result
as the same instance stepped alone with dg_rk_step (same device code, same
blocks, same reduction order), with or without HIP graphs, and when the
batch changes between steps (continuous batching).  One batched instance
is also checked against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1311_7477_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (n, N, k0, seed): uneven mix with ragged sizes (not multiples of 64 or of
# the bracket kernel's tile) and every polynomial order
MEMBERS = [(2, 70, 4.0, 11), (3, 33, 5.0, 12), (4, 64, 6.0, 13), (5, 20, 4.0, 14),
           (4, 17, 3.0, 15), (2, 128, 8.0, 16), (3, 9, 2.0, 17), (5, 40, 6.0, 18)]


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1311_7477_amd import dg as _dg
    _dg.lib()
    return _dg


def _member(dg, n, N, k0, seed):
    w0, umax = I.random_spectrum(n, N, k0=k0, seed=seed, return_umax=True)
    dt = I.cfl_dt(n, N, umax, cfl=0.1)
    return dg.Grid(n, N, N), w0, dt


def _alone(dg, grid, w0, dt, D, steps, opts):
    ws, st = dg.Workspace(grid), dg.State(grid)
    w = torch.from_numpy(w0).cuda()
    its = []
    for _ in range(steps):
        its.append(dg.rk_step(grid, w, st, ws, dt, D, opts).cg_iters)
    return w.cpu().numpy(), st.psi().cpu().numpy(), its


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_bitwise_equals_alone(dg, graphs):
    print(f"batch bitwise graphs={graphs}", flush=True)
    D, steps, opts = 1e-4, 2, dg.cg_opts(rtol=1e-11)
    batch = dg.Batch(len(MEMBERS) + 2, use_graphs=graphs)
    inst = []
    for (n, N, k0, seed) in MEMBERS:
        grid, w0, dt = _member(dg, n, N, k0, seed)
        w = torch.from_numpy(w0).cuda()
        slot = batch.attach(grid, w, dt, D)
        inst.append((slot, grid, w0, dt, w))
    its_b = []
    for _ in range(steps):
        its, ok = batch.rk_step(opts)
        assert ok
        its_b.append(its)
    for (slot, grid, w0, dt, w) in inst:
        wa, pa, its_a = _alone(dg, grid, w0, dt, D, steps, opts)
        wb, pb = w.cpu().numpy(), batch.psi(slot).cpu().numpy()
        same_w, same_p = bool(np.array_equal(wb, wa)), bool(np.array_equal(pb, pa))
        assert same_w, f"slot {slot} omega differs by {np.abs(wb - wa).max():.3e}"
        assert same_p, f"slot {slot} psi differs by {np.abs(pb - pa).max():.3e}"
        assert [its_b[s][slot] for s in range(steps)] == its_a
        assert batch.time(slot) == pytest.approx(steps * dt, rel=1e-14)


def test_batch_attach_detach_between_steps(dg):
    D, opts = 1e-4, dg.cg_opts(rtol=1e-11)
    batch = dg.Batch(4)
    g1, w1, dt1 = _member(dg, 3, 40, 4.0, 21)
    g2, w2, dt2 = _member(dg, 4, 24, 3.0, 22)
    g3, w3, dt3 = _member(dg, 2, 50, 5.0, 23)
    t1, t2, t3 = (torch.from_numpy(a).cuda() for a in (w1, w2, w3))
    s1 = batch.attach(g1, t1, dt1, D)
    s2 = batch.attach(g2, t2, dt2, D)
    batch.rk_step(opts)
    batch.detach(s2)                       # leaves after one step
    s3 = batch.attach(g3, t3, dt3, D)      # joins for two steps
    batch.rk_step(opts)
    batch.rk_step(opts)
    for t, (g, w0, dt), steps in ((t1, (g1, w1, dt1), 3), (t2, (g2, w2, dt2), 1),
                                  (t3, (g3, w3, dt3), 2)):
        got, ref = t.cpu().numpy(), _alone(dg, g, w0, dt, D, steps, opts)[0]
        same = bool(np.array_equal(got, ref))
        assert same, f"differs by {np.abs(got - ref).max():.3e}"
    # the freed slot is reused by the newcomer
    assert s3 == s2 and sorted(batch.members) == sorted({s1, s3})


def test_batch_member_matches_oracle(dg):
    n, N, D, dt = 3, 24, 1e-3, 1e-3
    w0 = I.taylor_green_noise(n, N, seed=5)
    grid = dg.Grid(n, N, N)
    batch = dg.Batch(2)
    w = torch.from_numpy(w0).cuda()
    batch.attach(grid, w, dt, D)
    g = O.Grid2D(n, N, N)
    wr, t, hist = w0.copy(), 0.0, O.PsiHistory()
    for _ in range(3):
        batch.rk_step(dg.cg_opts(rtol=1e-14))
        wr, _ = O.rk3_step(g, wr, t, dt, D, hist, rtol=1e-14)
        t += dt
    e = w.cpu().numpy() - wr
    assert math.sqrt(O.inner(g, e, e) / O.inner(g, wr, wr)) <= 1e-12


def test_batch_errors(dg):
    batch = dg.Batch(1)
    g, w0, dt = _member(dg, 2, 16, 3.0, 1)
    w = torch.from_numpy(w0).cuda()
    batch.attach(g, w, dt, 0.0)
    with pytest.raises(dg.DgError):
        batch.attach(g, torch.from_numpy(w0).cuda(), dt, 0.0)     # full
    with pytest.raises(dg.DgError) as ei:
        batch.rk_step(dg.cg_opts(precision=dg.DG_PREC_MIXED))
    assert ei.value.code == dg.DG_E_UNSUPPORTED
    with pytest.raises(dg.DgError):
        batch.detach(5)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp64-products"])
def test_preconditioned_batch_bitwise_equals_alone(dg, precision):
    # Members of a batch made with dg_batch_use_precond take preconditioned
    # steps (each through dg_rk_step on the batch's stream): bitwise the same
    # omega and psi as the instance stepped alone with the same options, on
    # both transform paths (45 and 20 cells: folded products; 48 and 600:
    # FFTs), with iteration counts reported per stage.
    print(f"preconditioned batch {precision}", flush=True)
    members = [(2, 45, 4.0, 21), (4, 48, 6.0, 22), (3, 600, 8.0, 23), (5, 20, 4.0, 24)]
    prec = dg.DG_PREC_MIXED if precision == "mixed" else dg.DG_PREC_FP64
    # fp64-products: every member's preconditioner on the folded products
    fd = dg.DG_WS_FD | (dg.DG_WS_FD_PRODUCTS if precision.endswith("products") else 0)
    D, steps = 1e-4, 2
    opts = dg.cg_opts(rtol=1e-11, precond=dg.DG_PRECOND_FD, precision=prec)
    batch = dg.Batch(len(members))
    batch.use_precond(fd)
    inst = []
    for (n, N, k0, seed) in members:
        grid, w0, dt = _member(dg, n, N, k0, seed)
        w = torch.from_numpy(w0).cuda()
        inst.append((batch.attach(grid, w, dt, D), grid, w0, dt, w))
    its_b = []
    for _ in range(steps):
        its, ok = batch.rk_step(opts)
        assert ok
        its_b.append(its)
    for slot, grid, w0, dt, w in inst:
        assert batch.converged(slot)
        assert abs(batch.time(slot) - steps * dt) <= 1e-15 * steps * dt
        ws = dg.Workspace(grid, dg.DG_PREC_FP64 | fd)
        st = dg.State(grid)
        wa = torch.from_numpy(w0).cuda()
        its_a = [dg.rk_step(grid, wa, st, ws, dt, D, opts).cg_iters for _ in range(steps)]
        assert np.array_equal(w.cpu().numpy(), wa.cpu().numpy())
        assert np.array_equal(batch.psi(slot).cpu().numpy(), st.psi().cpu().numpy())
        assert [tuple(i[slot]) for i in its_b] == [tuple(i) for i in its_a]
        assert all(1 <= k <= 4 for i in its_a for k in i)
