"""Serving loop: simulation-step requests admitted into a device batch.

A request asks for `steps` SSP-RK3 steps of one instance (polynomial order
n, an N x N periodic grid, an initial vorticity).  The server keeps every
admitted request's state resident on the device and advances all of them
together, one batched RK3 step per tick (dg_batch_rk_step: one persistent
launch per kernel kind and polynomial order, graph-replayed).  Requests that
arrive while others run wait in a FIFO queue and are admitted between ticks
as soon as a slot is free and their device footprint
(dg_batch_member_bytes + the omega field) fits the HBM budget: continuous
batching.  Finished requests leave the batch at once and free their memory.

Because a batch runs every instance with the same device code and block
decomposition as a stand-alone run, a request's result is bitwise the same
whatever else was in flight.

StreamServer runs the same loop with another engine: every admitted request
owns a workspace with the fast-diagonalisation preconditioner and a HIP
stream, and a tick issues one dg_rk_step per active request from a pool of
host threads, so the requests' kernels overlap on the device; the solve is
the preconditioned CG with its preconditioner applied in FP32 under the FP64
iteration (rtol 1e-10 by default).  A request again gets the result of the
same steps run alone.  All scheduling is host logic here; every computation
runs in the HIP library.
"""
from __future__ import annotations

import collections
import math
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import dg, inputs


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    n: int
    N: int
    k0: float
    seed: int
    steps: int
    D: float = 1e-4
    # filled by the server
    dt: float = 0.0
    bytes: int = 0
    admitted: float = math.nan
    finished: float = math.nan
    cg_iters: list = field(default_factory=list)
    omega: object = None      # device tensor while resident
    result: object = None     # host copy of the final omega
    grid: object = None
    slot: int = -1
    done_steps: int = 0
    ws: object = None         # StreamServer: workspace, state and stream
    state: object = None
    stream: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def cell_updates(self) -> float:
        return 3.0 * self.steps * self.N * self.N


def draw_requests(count, seed, rate, n_choices=(2, 3, 4, 5), N_range=(128, 2048),
                  k0_range=(4.0, 16.0), steps=100, D=1e-4):
    """Seeded Poisson arrival stream: exponential inter-arrival times with
    the given rate (1/s), n uniform over n_choices, N log-uniform over
    N_range, spectrum peak k0 uniform over k0_range."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(n_choices))
        N = int(round(math.exp(rng.uniform(math.log(N_range[0]), math.log(N_range[1])))))
        k0 = float(rng.uniform(*k0_range))
        out.append(Request(i, t, n, N, k0, int(rng.integers(1 << 30)), steps, D))
    return out


def member_bytes(n, N):
    """Device bytes one admitted request holds: library state + omega."""
    g = dg.Grid(n, N, N)
    return dg.batch_member_bytes(g) + g.elems * 8


def prepare(req: Request):
    """Host part of admission: the initial field and the CFL time step."""
    w0, umax = inputs.random_spectrum(req.n, req.N, k0=req.k0, seed=req.seed,
                                      return_umax=True)
    req.dt = inputs.cfl_dt(req.n, req.N, umax, cfl=0.1)
    return w0


class Server:
    """Continuous-batching request loop.  With tune=True the tile shapes of
    each (n, N) are chosen once by the library's tile autotuner (on the first
    admitted request of that shape) and reused for later ones."""

    def __init__(self, capacity=64, hbm_budget=None, opts=None, tune=True):
        import torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = hbm_budget
        self.capacity = capacity
        self.opts = opts if opts is not None else dg.cg_opts(rtol=1e-10)
        self.batch = self._engine()
        self.used = 0
        self.active = {}
        self.ticks = 0
        self.max_active = 0
        self.peak_used = 0
        self.rejected = []
        self.tune = tune
        self.tiles = {}           # (n, N) -> (cell tile height, bracket tile height)

    def _engine(self):
        return dg.Batch(self.capacity)

    def request_bytes(self, req: Request) -> int:
        return member_bytes(req.n, req.N)

    def fits(self, req: Request) -> bool:
        return (len(self.active) < self.capacity and
                self.used + req.bytes <= self.budget)

    def admit(self, req: Request, now: float):
        import torch
        w0 = prepare(req)
        req.grid = dg.Grid(req.n, req.N, req.N)
        req.omega = torch.from_numpy(w0).cuda()
        key = (req.n, req.N)
        if self.tune and key not in self.tiles:
            self.tiles[key] = req.grid.tune(req.omega, reps=5)[0]
        if key in self.tiles:
            req.grid.set_tiles(*self.tiles[key])
        req.slot = self.batch.attach(req.grid, req.omega, req.dt, req.D)
        req.admitted = now
        self.used += req.bytes
        self.peak_used = max(self.peak_used, self.used)
        self.active[req.slot] = req
        self.max_active = max(self.max_active, len(self.active))

    def retire(self, req: Request, now: float):
        req.result = req.omega.cpu().numpy()
        self.batch.detach(req.slot)
        self.used -= req.bytes
        del self.active[req.slot]
        req.omega, req.grid = None, None
        req.finished = now

    def tick(self, now_fn):
        its, ok = self.batch.rk_step(self.opts)
        self.ticks += 1
        for slot, req in list(self.active.items()):
            req.cg_iters.extend(its[slot])
            req.done_steps += 1
            if req.done_steps >= req.steps:
                self.retire(req, now_fn())

    def run(self, requests, log=None):
        """Serve an arrival stream in real time; returns the finished
        requests.  Requests larger than the whole budget are rejected."""
        for r in requests:
            r.bytes = self.request_bytes(r)
        reqs = sorted(requests, key=lambda r: r.arrival)
        rejected = [r for r in reqs if r.bytes > self.budget]
        todo = collections.deque(r for r in reqs if r.bytes <= self.budget)
        queue = collections.deque()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while todo or queue or self.active:
            t = now()
            while todo and todo[0].arrival <= t:
                queue.append(todo.popleft())
            while queue and self.fits(queue[0]):
                self.admit(queue.popleft(), now())
            if self.active:
                self.tick(now)
                if log:
                    done = sum(not math.isnan(r.finished) for r in reqs)
                    log(f"tick {self.ticks}: active {len(self.active)} queued "
                        f"{len(queue)} done {done} t={now():.2f}s")
            elif todo:
                time.sleep(max(0.0, min(todo[0].arrival - now(), 0.05)))
        self.rejected = rejected
        return [r for r in reqs if not math.isnan(r.finished)]


class StreamServer(Server):
    """The request loop of Server with one stream per request: admission
    creates the request's grid, a DG_WS_FD workspace (the preconditioner's
    bases and plans), its state and a HIP stream; a tick runs one
    dg_rk_step of every active request, each issued from a worker thread
    on that request's stream (the library's calls release the GIL, and each
    one waits only for its own stream).  Default solve: CG preconditioned by
    fast diagonalisation, the preconditioner in FP32 under the FP64
    iteration, rtol 1e-10."""

    def __init__(self, capacity=64, hbm_budget=None, opts=None, tune=False, workers=16):
        if opts is None:
            opts = dg.cg_opts(rtol=1e-10, precond=dg.DG_PRECOND_FD,
                              precision=dg.DG_PREC_MIXED)
        self.workers = workers
        super().__init__(capacity, hbm_budget, opts, tune)

    def _engine(self):
        return ThreadPoolExecutor(self.workers)

    def request_bytes(self, req: Request) -> int:
        """Workspace (with the preconditioner), state (three fields) and
        omega; rocBLAS and rocFFT keep their work buffers on top."""
        g = dg.Grid(req.n, req.N, req.N)
        return g.workspace_bytes(dg.DG_PREC_FP64 | dg.DG_WS_FD) + 4 * g.elems * 8

    def admit(self, req: Request, now: float):
        import torch
        w0 = prepare(req)
        req.grid = dg.Grid(req.n, req.N, req.N)
        key = (req.n, req.N)
        req.stream = torch.cuda.Stream()
        with torch.cuda.stream(req.stream):
            req.omega = torch.from_numpy(w0).cuda()
            if self.tune and key not in self.tiles:
                self.tiles[key] = req.grid.tune(req.omega, reps=5)[0]
            if key in self.tiles:
                req.grid.set_tiles(*self.tiles[key])
            req.ws = dg.Workspace(req.grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
            req.state = dg.State(req.grid)
        req.slot = req.rid
        req.admitted = now
        self.used += req.bytes
        self.peak_used = max(self.peak_used, self.used)
        self.active[req.slot] = req
        self.max_active = max(self.max_active, len(self.active))

    def retire(self, req: Request, now: float):
        req.stream.synchronize()
        req.result = req.omega.cpu().numpy()
        self.used -= req.bytes
        del self.active[req.slot]
        req.omega = req.grid = req.ws = req.state = req.stream = None
        req.finished = now

    def _step(self, req: Request):
        import torch
        with torch.cuda.stream(req.stream):
            r = dg.rk_step(req.grid, req.omega, req.state, req.ws, req.dt, req.D, self.opts)
        if not r.converged:
            raise RuntimeError(f"request {req.rid}: the solve did not converge")
        return r

    def tick(self, now_fn):
        futures = {slot: self.batch.submit(self._step, req)
                   for slot, req in self.active.items()}
        self.ticks += 1
        for slot, f in futures.items():
            r = f.result()
            req = self.active[slot]
            req.cg_iters.extend(r.cg_iters)
            req.done_steps += 1
            if req.done_steps >= req.steps:
                self.retire(req, now_fn())


def summarize(done, makespan):
    lat = sorted(r.latency for r in done)

    def pct(q):
        return lat[min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))]

    return {
        "requests": len(done),
        "p50_latency_s": pct(0.50),
        "p99_latency_s": pct(0.99),
        "mean_latency_s": float(np.mean(lat)),
        "aggregate_cell_updates_per_s": sum(r.cell_updates for r in done) / makespan,
        "mean_cg_iters_per_rhs": float(np.mean([i for r in done for i in r.cg_iters])),
    }


def run_alone(req: Request, opts=None, tiles=None):
    """The same request stepped alone with dg_rk_step (for the alone-vs-mix
    check), with the tile shapes the server used: returns the final omega on
    the host."""
    import torch
    w0 = prepare(req)
    grid = dg.Grid(req.n, req.N, req.N)
    if tiles is not None:
        grid.set_tiles(*tiles)
    precond = opts is not None and opts.precond != dg.DG_PRECOND_NONE
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | (dg.DG_WS_FD if precond else 0))
    st = dg.State(grid)
    w = torch.from_numpy(w0).cuda()
    for _ in range(req.steps):
        dg.rk_step(grid, w, st, ws, req.dt, req.D,
                   opts if opts is not None else dg.cg_opts(rtol=1e-10))
    return w.cpu().numpy()
