"""Host logic of the serving loop, without a GPU: the seeded request
stream, and the admission loop of Server.run (FIFO order, the HBM budget,
the slot capacity, rejection of requests larger than the budget) driven by
an engine that only counts steps."""
import math

import numpy as np
import pytest

from paper_1311_7477_amd import serve


class CountingServer(serve.Server):
    """Server.run with the device work replaced by bookkeeping: a request's
    footprint is 8 N^2 bytes and each tick advances every active request by
    one step."""

    def __init__(self, capacity, budget):
        super().__init__(capacity=capacity, hbm_budget=budget, opts=None, tune=False)
        self.log = []

    def _engine(self):
        return None

    def request_bytes(self, req):
        return 8 * req.N * req.N

    def admit(self, req, now):
        req.admitted = now
        self.used += req.bytes
        self.peak_used = max(self.peak_used, self.used)
        self.active[req.rid] = req
        self.max_active = max(self.max_active, len(self.active))
        self.log.append(("admit", req.rid, self.used))

    def retire(self, req, now):
        self.used -= req.bytes
        del self.active[req.rid]
        req.finished = now
        self.log.append(("retire", req.rid, self.used))

    def tick(self, now_fn):
        self.ticks += 1
        for req in list(self.active.values()):
            req.done_steps += 1
            if req.done_steps >= req.steps:
                self.retire(req, now_fn())


def test_request_stream_is_seeded_and_in_range():
    a = serve.draw_requests(200, seed=3, rate=50.0, N_range=(128, 2048), steps=7)
    b = serve.draw_requests(200, seed=3, rate=50.0, N_range=(128, 2048), steps=7)
    assert [(r.arrival, r.n, r.N, r.k0, r.seed) for r in a] == \
           [(r.arrival, r.n, r.N, r.k0, r.seed) for r in b]
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    # exponential gaps of mean 1 / rate (200 samples: within 25%)
    assert abs(np.mean(np.diff(arr)) - 1 / 50.0) < 0.25 / 50.0
    assert {r.n for r in a} <= {2, 3, 4, 5} and len({r.n for r in a}) == 4
    assert all(128 <= r.N <= 2048 and 4.0 <= r.k0 <= 16.0 and r.steps == 7 for r in a)
    # log-uniform sizes: about half below the geometric mean of the range
    below = np.mean([r.N < math.sqrt(128 * 2048) for r in a])
    assert 0.35 < below < 0.65
    assert all(r.cell_updates == 3.0 * 7 * r.N * r.N for r in a)


@pytest.mark.parametrize("capacity,budget_cells", [(8, 10 ** 9), (2, 10 ** 9), (8, 3 * 64 ** 2)])
def test_admission_fifo_budget_and_capacity(capacity, budget_cells):
    reqs = serve.draw_requests(12, seed=8, rate=1e6, N_range=(16, 64), steps=3)
    budget = 8 * budget_cells
    srv = CountingServer(capacity, budget)
    done = srv.run(reqs)
    assert len(done) == len(reqs) and not srv.rejected
    assert srv.peak_used <= budget and srv.max_active <= capacity
    assert srv.used == 0 and not srv.active
    admitted = [rid for kind, rid, _ in srv.log if kind == "admit"]
    assert admitted == sorted(admitted)                # FIFO
    assert all(r.admitted >= r.arrival and r.finished >= r.admitted for r in done)
    assert all(r.done_steps == r.steps for r in done)
    if capacity == 2 or budget_cells < 10 ** 9:
        assert srv.max_active < len(reqs)              # some requests waited


def test_requests_beyond_the_budget_are_rejected():
    reqs = serve.draw_requests(6, seed=9, rate=1e6, N_range=(16, 64), steps=1)
    cut = sorted(8 * r.N * r.N for r in reqs)[2]
    srv = CountingServer(8, cut)
    done = srv.run(reqs)
    assert {r.rid for r in srv.rejected} == {r.rid for r in reqs if 8 * r.N * r.N > cut}
    assert {r.rid for r in done} == {r.rid for r in reqs if 8 * r.N * r.N <= cut}
    assert all(math.isnan(r.finished) for r in srv.rejected)


def test_summary_percentiles():
    reqs = serve.draw_requests(4, seed=1, rate=10.0, N_range=(16, 32), steps=2)
    for i, r in enumerate(reqs):
        r.arrival, r.finished = 0.0, float(i + 1)
        r.cg_iters = [i, i]
    s = serve.summarize(reqs, makespan=4.0)
    assert s["p50_latency_s"] == 2.0 and s["p99_latency_s"] == 4.0
    assert s["mean_latency_s"] == 2.5 and s["requests"] == 4
    assert s["aggregate_cell_updates_per_s"] == sum(r.cell_updates for r in reqs) / 4.0
    assert s["mean_cg_iters_per_rhs"] == 1.5


class FailingCountingServer(CountingServer):
    """The batched engine's tick with one request whose solve never
    converges: it must be retired with an error while the others finish."""

    def __init__(self, capacity, budget, bad):
        super().__init__(capacity, budget)
        self.bad = bad

    def tick(self, now_fn):
        self.ticks += 1
        for req in list(self.active.values()):
            req.done_steps += 1
            if req.rid == self.bad:
                req.error = f"request {req.rid}: a solve did not converge"
                self.retire(req, now_fn())
            elif req.done_steps >= req.steps:
                self.retire(req, now_fn())


def test_failed_request_is_retired_alone():
    reqs = serve.draw_requests(6, seed=2, rate=1e6, N_range=(16, 64), steps=4)
    srv = FailingCountingServer(8, 10 ** 12, bad=reqs[2].rid)
    done = srv.run(reqs)
    assert [r.rid for r in srv.failed] == [reqs[2].rid]
    assert {r.rid for r in done} == {r.rid for r in reqs} - {reqs[2].rid}
    assert all(r.done_steps == r.steps and r.error is None for r in done)
    assert srv.used == 0 and not srv.active


class SleepyStreamServer(serve.StreamServer):
    """StreamServer's scheduling (a worker per request, no step barrier,
    per-request failure) with the device step replaced by a sleep of
    N / 16000 s; a request with max_iter = 1 'does not converge' in its
    second step."""

    def __init__(self, capacity, budget):
        super().__init__(capacity=capacity, hbm_budget=budget, opts=None, workers=capacity)

    def request_bytes(self, req):
        return 8 * req.N * req.N

    def admit(self, req, now):
        self._launch(req, now)
        return True

    def _step_once(self, req, opts):
        import time as _t
        _t.sleep(req.N / 16000.0)
        return (1, 1, 1), not (req.max_iter == 1 and req.done_steps >= 1)

    def retire(self, req, now):
        self.used -= req.bytes
        del self.active[req.slot]
        self.futures.pop(req.slot, None)
        req.finished = req.done_at


def test_stream_engine_has_no_step_barrier_and_retires_failures_alone():
    # a large request (N = 1600: 0.1 s per step) and small ones (N = 16:
    # 1 ms per step) admitted together: the small ones finish long before
    # the large one although every request has 8 steps; one small request
    # fails in its second step and is retired alone
    reqs = serve.draw_requests(5, seed=3, rate=1e6, N_range=(16, 17), steps=8)
    reqs[0].N = 1600
    reqs[3].max_iter = 1
    srv = SleepyStreamServer(8, 10 ** 12)
    done = srv.run(reqs)
    assert [r.rid for r in srv.failed] == [reqs[3].rid]
    assert reqs[3].done_steps == 2 and reqs[3].error
    assert {r.rid for r in done} == {r.rid for r in reqs} - {reqs[3].rid}
    big = reqs[0]
    smalls = [r for r in done if r.rid != big.rid]
    assert all(r.done_steps == 8 for r in done)
    assert max(r.finished for r in smalls) < 0.5 * big.finished
    assert srv.used == 0 and not srv.active and not srv.futures
