"""Serving loop: simulation-step requests admitted into a device batch.

A request asks for `steps` SSP-RK3 steps of one instance (polynomial order
n, an N x N periodic grid, an initial vorticity).  The server keeps every
admitted request's state resident on the device and advances all of them
together, one batched RK3 step per tick (dg_batch_rk_step: one fused
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
stream, and a host worker thread runs all of that request's steps
(dg_rk_step on its own stream) back to back, so the requests' kernels
overlap on the device and no request waits for another's step: a small
request admitted beside a large one finishes on its own clock.  The solve
is the preconditioned CG with its preconditioner applied in FP32 under the
FP64 iteration (rtol 1e-10 by default).  A request again gets the result of
the same steps run alone.

A request whose solve does not converge (DG_E_NOCONV) or whose step fails
otherwise is retired with `error` set while the others continue; run()
returns the requests that finished and lists the failed ones in `failed`.
All scheduling is host logic here; every computation runs in the HIP
library.
"""
from __future__ import annotations

import collections
import math
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np

from . import dg, inputs


# device fields a stream-served request holds besides its workspace: the
# five of its dg_state and omega
STATE_FIELDS = 6


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
    max_iter: int = 0         # StreamServer: per-request CG iteration cap (0: the server's)
    error: str = None         # set when the request failed (e.g. a solve did not converge)
    done_at: float = math.nan  # StreamServer: when its last step returned

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
        self.failed = []
        self.tune = tune
        self.tiles = {}           # (n, N) -> (cell tile height, bracket tile height)
        self.shape_bytes = {}     # (n, N) -> device bytes measured at an admission

    def _engine(self):
        return dg.Batch(self.capacity)

    def request_bytes(self, req: Request) -> int:
        return member_bytes(req.n, req.N)

    def fits(self, req: Request) -> bool:
        need = self.shape_bytes.get((req.n, req.N), req.bytes)
        return (len(self.active) < self.capacity and
                self.used + need <= self.budget)

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
        """One batched RK3 step of every member; a member whose solve did
        not converge is retired with an error, the others go on."""
        its, ok = self.batch.rk_step(self.opts)
        self.ticks += 1
        for slot, req in list(self.active.items()):
            req.cg_iters.extend(its[slot])
            req.done_steps += 1
            if not ok and not self.batch.converged(slot):
                req.error = (f"request {req.rid}: a solve did not converge in step "
                             f"{req.done_steps}")
                self.retire(req, now_fn())
            elif req.done_steps >= req.steps:
                self.retire(req, now_fn())

    def advance(self, now_fn, wait_s):
        """Make progress on the active requests: here one batched tick
        (wait_s, the time to the next arrival, is not needed)."""
        self.tick(now_fn)

    def run(self, requests, log=None):
        """Serve an arrival stream in real time; returns the requests that
        finished without error (failed ones are in self.failed).  Requests
        larger than the whole budget are rejected."""
        for r in requests:
            r.bytes = self.request_bytes(r)
        reqs = sorted(requests, key=lambda r: r.arrival)
        rejected = [r for r in reqs if r.bytes > self.budget]
        todo = collections.deque(r for r in reqs if r.bytes <= self.budget)
        queue = collections.deque()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        self._now = now
        while todo or queue or self.active:
            t = now()
            while todo and todo[0].arrival <= t:
                queue.append(todo.popleft())
            while queue and self.fits(queue[0]):
                req = queue.popleft()
                if self.admit(req, now()) is False:
                    # its measured footprint does not fit after all
                    if req.bytes > self.budget:
                        rejected.append(req)
                        continue
                    queue.appendleft(req)
                    break
            if self.active:
                self.advance(now, (todo[0].arrival - now()) if todo else None)
                if log:
                    done = sum(not math.isnan(r.finished) for r in reqs)
                    log(f"step {self.ticks}: active {len(self.active)} queued "
                        f"{len(queue)} done {done} t={now():.2f}s")
            elif todo:
                time.sleep(max(0.0, min(todo[0].arrival - now(), 0.05)))
        self.rejected = rejected
        self.failed = [r for r in reqs if r.error is not None]
        return [r for r in reqs if not math.isnan(r.finished) and r.error is None]


# Preconditioner workspaces of requests with at most this many cells per
# axis transform with the folded matrix products (DG_WS_FD_PRODUCTS): a
# request is about 100 steps, and the rocFFT plans of a new grid size (kernels
# compiled per transform length: 1-2 s) cost more there than the products
# lose per step (n = 4, 338^2: 1.3 s of set-up, against 0.46 ms per step that
# the products lose).
PRODUCTS_MAX_CELLS = 512


def ws_mode(N, precond=True):
    """Workspace mode of a request on an N x N grid."""
    if not precond:
        return dg.DG_PREC_FP64
    mode = dg.DG_PREC_FP64 | dg.DG_WS_FD
    return mode | dg.DG_WS_FD_PRODUCTS if N <= PRODUCTS_MAX_CELLS else mode


class StreamServer(Server):
    """The request loop of Server with one stream and one host worker per
    request: admission creates the request's grid, a DG_WS_FD workspace (the
    preconditioner's bases and plans; the folded products up to
    PRODUCTS_MAX_CELLS cells per axis), its state and a HIP stream, then
    hands the request to a worker thread that runs all of its steps on that
    stream (the library's calls release the GIL and each waits only for its
    own stream).  The main loop never waits for a step: it retires requests
    as their workers finish and admits queued ones as memory and slots free
    up.  Admission charges the bytes the workspace really holds (library
    work buffers included) once it exists; a request that then does not fit
    goes back to the head of the queue.  Default solve: CG preconditioned by
    fast diagonalisation, the preconditioner in FP32 under the FP64
    iteration, rtol 1e-10."""

    def __init__(self, capacity=64, hbm_budget=None, opts=None, tune=False, workers=None):
        if opts is None:
            opts = dg.cg_opts(rtol=1e-10, precond=dg.DG_PRECOND_FD,
                              precision=dg.DG_PREC_MIXED)
        self.workers = capacity if workers is None else workers
        super().__init__(capacity, hbm_budget, opts, tune)
        self.futures = {}

    def _engine(self):
        return ThreadPoolExecutor(self.workers)

    def request_bytes(self, req: Request) -> int:
        """Estimate before admission: workspace (with the preconditioner),
        state (five fields) and omega; admission replaces it by the bytes
        the workspace reports once created."""
        g = dg.Grid(req.n, req.N, req.N)
        return g.workspace_bytes(ws_mode(req.N)) + STATE_FIELDS * g.elems * 8

    def admit(self, req: Request, now: float):
        import torch
        req.grid = dg.Grid(req.n, req.N, req.N)
        key = (req.n, req.N)
        req.stream = torch.cuda.Stream()
        try:
            with torch.cuda.stream(req.stream):
                req.ws = dg.Workspace(req.grid, ws_mode(req.N))
        except dg.DgError as e:
            req.grid = req.ws = req.stream = None
            if e.code != dg.DG_E_NOMEM or not self.active:
                raise
            return False              # the device is full now: retry later
        held = req.ws.held_bytes() + STATE_FIELDS * req.grid.elems * 8
        self.shape_bytes[key] = held
        if self.used + held > self.budget:
            req.bytes = held
            req.grid = req.ws = req.stream = None
            return False
        req.bytes = held
        w0 = prepare(req)
        with torch.cuda.stream(req.stream):
            req.omega = torch.from_numpy(w0).cuda()
            if self.tune and key not in self.tiles:
                self.tiles[key] = req.grid.tune(req.omega, reps=5)[0]
            if key in self.tiles:
                req.grid.set_tiles(*self.tiles[key])
            req.state = dg.State(req.grid)
        self._launch(req, now)
        return True

    def _launch(self, req: Request, now: float):
        """Book an admitted request and hand it to a worker thread."""
        req.slot = req.rid
        req.admitted = now
        self.used += req.bytes
        self.peak_used = max(self.peak_used, self.used)
        self.active[req.slot] = req
        self.max_active = max(self.max_active, len(self.active))
        self.futures[req.slot] = self.batch.submit(self._run_request, req, self._now)

    def retire(self, req: Request, now: float):
        if req.stream is not None:
            req.stream.synchronize()
        if req.error is None:
            req.result = req.omega.cpu().numpy()
        self.used -= req.bytes
        del self.active[req.slot]
        self.futures.pop(req.slot, None)
        req.omega = req.grid = req.ws = req.state = req.stream = None
        req.finished = req.done_at if not math.isnan(req.done_at) else now

    def _step_once(self, req: Request, opts):
        """One SSP-RK3 step of the request on its stream: (iterations of the
        three solves, whether all converged)."""
        import torch
        with torch.cuda.stream(req.stream):
            r = dg.rk_step(req.grid, req.omega, req.state, req.ws, req.dt, req.D, opts)
        return r.cg_iters, r.converged

    def _run_request(self, req: Request, now_fn):
        """Worker: every step of one request, back to back."""
        opts = self.opts
        if opts is not None and req.max_iter:
            opts = dg.cg_opts(opts.rtol, req.max_iter, opts.precision, opts.precond,
                              opts.check_every)
        try:
            while req.done_steps < req.steps:
                its, ok = self._step_once(req, opts)
                req.cg_iters.extend(its)
                req.done_steps += 1
                if not ok:
                    req.error = (f"request {req.rid}: a solve did not converge in "
                                 f"step {req.done_steps}")
                    break
            if req.stream is not None:
                req.stream.synchronize()
        except Exception as e:          # a failed step retires this request only
            req.error = f"request {req.rid}: {e}"
        req.done_at = now_fn()

    def advance(self, now_fn, wait_s):
        """Retire the requests whose workers finished; wait for the first
        one at most until the next arrival."""
        timeout = 0.05 if wait_s is None else max(0.0, min(wait_s, 0.05))
        done, _ = wait(list(self.futures.values()), timeout=timeout,
                       return_when=FIRST_COMPLETED)
        self.ticks += 1
        for slot, f in list(self.futures.items()):
            if f in done:
                f.result()
                self.retire(self.active[slot], now_fn())

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
    ws = dg.Workspace(grid, ws_mode(req.N, precond))
    st = dg.State(grid)
    w = torch.from_numpy(w0).cuda()
    for _ in range(req.steps):
        r = dg.rk_step(grid, w, st, ws, req.dt, req.D,
                       opts if opts is not None else dg.cg_opts(rtol=1e-10))
        if not r.converged:
            raise RuntimeError(f"request {req.rid} alone: a solve did not converge")
    return w.cpu().numpy()
