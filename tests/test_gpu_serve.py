"""Serving loop: requests that arrive while others run are admitted between
steps (continuous batching), every result equals the same request run
alone (bitwise, since a batch runs each instance with the stand-alone
device code), and a small HBM budget forces queueing instead of failure;
the same for the stream-per-request server with the FP32-preconditioned CG
(its results equal the stand-alone steps bitwise too)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_1311_7477_amd import dg, serve as _serve
    dg.lib()
    return _serve


def _stream(serve, count=6, rate=50.0):
    return serve.draw_requests(count, seed=4, rate=rate, N_range=(16, 48),
                               k0_range=(2.0, 5.0), steps=3)


def test_mixed_stream_equals_alone(serve):
    from paper_1311_7477_amd import dg
    opts = dg.cg_opts(rtol=1e-10)
    reqs = _stream(serve)
    srv = serve.Server(capacity=8, opts=opts)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.max_active > 1            # requests overlapped on the device
    assert all(v[0] in (4, 8, 16) and v[1] in (8, 16) for v in srv.tiles.values())
    for r in done:
        alone = serve.run_alone(r, opts, srv.tiles.get((r.n, r.N)))
        same = bool(np.array_equal(r.result, alone))
        assert same, f"request {r.rid}: differs by {np.abs(r.result - alone).max():.3e}"
        assert r.latency > 0 and r.admitted >= r.arrival
    s = serve.summarize(done, max(r.finished for r in done))
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert s["aggregate_cell_updates_per_s"] > 0


def test_small_budget_queues_requests(serve):
    from paper_1311_7477_amd import dg
    reqs = _stream(serve, count=4, rate=1000.0)
    biggest = max(serve.member_bytes(r.n, r.N) for r in reqs)
    srv = serve.Server(capacity=8, hbm_budget=biggest, opts=dg.cg_opts(rtol=1e-8))
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.peak_used <= biggest      # the budget was never exceeded
    assert srv.max_active < len(reqs)    # so some requests had to wait
    # FIFO order under queueing
    order = [r.rid for r in sorted(done, key=lambda r: r.admitted)]
    assert order == sorted(order)


def test_oversized_request_is_rejected(serve):
    from paper_1311_7477_amd import dg
    reqs = _stream(serve, count=2)
    srv = serve.Server(capacity=2, hbm_budget=1024, opts=dg.cg_opts(rtol=1e-8))
    done = srv.run(reqs)
    assert done == [] and len(srv.rejected) == 2
    assert all(math.isnan(r.finished) for r in reqs)


def test_stream_server_pcg_equals_alone(serve):
    # one stream per request, the FP32-preconditioned CG, steps issued from
    # worker threads: every result equals the same request run alone
    from paper_1311_7477_amd import dg
    reqs = serve.draw_requests(8, seed=5, rate=200.0, N_range=(16, 96),
                               k0_range=(2.0, 5.0), steps=4)
    srv = serve.StreamServer(capacity=8, workers=4)
    assert srv.opts.precond == dg.DG_PRECOND_FD and srv.opts.precision == dg.DG_PREC_MIXED
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.max_active > 1
    for r in done:
        assert all(1 <= k <= 4 for k in r.cg_iters), r.cg_iters
        alone = serve.run_alone(r, srv.opts)
        assert np.array_equal(r.result, alone), \
            f"request {r.rid}: differs by {np.abs(r.result - alone).max():.3e}"
    assert not srv.active and srv.used == 0


def test_stream_server_budget_queues(serve):
    reqs = serve.draw_requests(4, seed=6, rate=1000.0, N_range=(16, 48),
                               k0_range=(2.0, 5.0), steps=2)
    from paper_1311_7477_amd import dg
    # the budget fits the largest request's real footprint (workspace with
    # its library buffers, state and omega), not two of them
    held = []
    for r in reqs:
        g = dg.Grid(r.n, r.N, r.N)
        held.append(dg.Workspace(g, dg.DG_PREC_FP64 | dg.DG_WS_FD).held_bytes()
                    + serve.STATE_FIELDS * g.elems * 8)
    biggest = max(held)
    assert 2 * min(held) > biggest
    srv = serve.StreamServer(capacity=8, hbm_budget=biggest, workers=2)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.peak_used <= biggest and srv.max_active < len(reqs)
    order = [r.rid for r in sorted(done, key=lambda r: r.admitted)]
    assert order == sorted(order)


def test_stream_server_retires_a_failing_request_alone(serve):
    # one request capped at one CG iteration (the FP32-preconditioned solve
    # needs at least two at rtol 1e-10 from a zero guess): it is retired
    # with an error, the others finish and equal their stand-alone runs
    reqs = serve.draw_requests(5, seed=7, rate=500.0, N_range=(16, 64),
                               k0_range=(2.0, 5.0), steps=3)
    reqs[1].max_iter = 1
    srv = serve.StreamServer(capacity=8)
    done = srv.run(reqs)
    assert [r.rid for r in srv.failed] == [reqs[1].rid]
    assert "did not converge" in reqs[1].error
    assert {r.rid for r in done} == {r.rid for r in reqs} - {reqs[1].rid}
    for r in done:
        assert np.array_equal(r.result, serve.run_alone(r, srv.opts))
    assert not srv.active and srv.used == 0


def test_batched_server_retires_non_converging_members(serve):
    from paper_1311_7477_amd import dg
    reqs = _stream(serve, count=3)
    srv = serve.Server(capacity=4, opts=dg.cg_opts(rtol=1e-12, max_iter=1), tune=False)
    done = srv.run(reqs)
    assert done == [] and len(srv.failed) == 3
    assert all(r.error and r.done_steps == 1 for r in reqs)
    assert not srv.active and srv.used == 0


def test_workspace_held_bytes_cover_library_buffers(serve):
    # FFT-path grids (both counts even, beyond 512 cells) and a
    # matrix-product one: the workspace reports at least the pre-creation
    # figure (the difference is rocFFT's work buffer and rocBLAS's memory)
    from paper_1311_7477_amd import dg
    for n, N in ((2, 1040), (2, 520), (3, 64)):
        g = dg.Grid(n, N, N)
        ws = dg.Workspace(g, dg.DG_PREC_FP64 | dg.DG_WS_FD)
        est = g.workspace_bytes(dg.DG_PREC_FP64 | dg.DG_WS_FD)
        held = ws.held_bytes()
        print(f"n={n} N={N}: estimate {est} B, held {held} B", flush=True)
        assert held >= est
        plain = dg.Workspace(g)
        assert plain.held_bytes() == g.workspace_bytes(dg.DG_PREC_FP64)
