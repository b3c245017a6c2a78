"""Benchmark: DG cell-updates/s per RHS (bracket + CG) on one MI355X.

Workload: periodic [0, 2pi]^2, n = 4 Legendre coefficients per direction,
512 x 512 cells; decaying 2D turbulence from a seeded random-spectrum
vorticity (peak |k| = 10, zero mean, energy 1/2), D = 1e-4, dt from CFL 0.1,
CG rtol 1e-12 with the extrapolated initial guess.  A step is one SSP-RK3
step = three right-hand sides (each: CG setup, CG iterations, fused
bracket/viscous/stage kernel).  value = Nx * Ny * RHS / second.

Also reported: p50/p99 of the per-RHS device time (HIP events), CG
iterations per RHS, the roofline figure of the dominant kernel (the CG
direction-update kernel, timed live with HIP events on the solve stream),
and the FP64 oracle timed on the host on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("DG cell-updates/s per RHS (bracket+CG) at n=4, 512², 1 GPU; "
          "p50/p99 latency")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_dir_traffic_n4_512.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1311_7477_amd", "csrc", f)
               for f in ("cg_kernels.hip", "cg_body.h", "dg_device.h")]


def kernel_source_hash():
    """sha256 (first 16 hex digits) of the sources the CG kernels are
    compiled from, concatenated."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(F_bytes, cw):
    """HBM bytes per launch of the direction kernel with cell tiles of cw
    waves, from committed rocprofv3 FETCH_SIZE/WRITE_SIZE counters, or None
    when they are missing or were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch_by_cw", {}).get(str(cw))


def cpu_baseline(n, N, omega0, psi0, D, dt, iters_per_rhs):
    """Time the oracle on the host on a bounded sample of the workload: one
    bracket + viscous evaluation, one CG setup and a few CG iterations at the
    full 512 x 512 size; per-RHS time = rhs + setup + k * iteration with k
    the GPU's mean CG iterations per RHS (a full oracle solve at this size
    takes tens of minutes)."""
    import oracle as O
    g = O.Grid2D(n, N, N)
    t0 = time.perf_counter()
    O.rhs(g, omega0, psi0, D)
    t_rhs = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.cg_poisson(g, omega0, psi0, rtol=1e-12, max_iter=0)
    t_setup = time.perf_counter() - t0
    k = 8
    t0 = time.perf_counter()
    O.cg_poisson(g, omega0, psi0, rtol=1e-30, max_iter=k)
    t_iter = max(time.perf_counter() - t0 - t_setup, 1e-9) / k
    t_per_rhs = t_rhs + t_setup + iters_per_rhs * t_iter
    return {
        "value": N * N / t_per_rhs,
        "unit": "cell-updates/s",
        # scipy's sparse products and numpy's elementwise operations run on
        # one thread (the oracle makes no BLAS calls)
        "cores": 1,
        "host_cpu_count": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": (f"numpy/scipy FP64 oracle at n={n}, {N}x{N}: 1 bracket+viscous "
                   f"({t_rhs:.2f} s), 1 CG setup ({t_setup:.2f} s), {k} CG iterations "
                   f"({t_iter * 1e3:.0f} ms each); per RHS = rhs + setup + "
                   f"{iters_per_rhs:.0f} x iteration, with the GPU's mean iterations per "
                   f"RHS (the oracle's own count agrees within 2 wherever both solve, "
                   f"but a full oracle solve at this size would take about "
                   f"{iters_per_rhs * t_iter / 60:.0f} minutes)"),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def form_batch(args):
    """Batched form: 64 instances with n uniform over {2..5}, N log-uniform
    over [64, N_max], random spectra with peak k0 uniform over [4, 16]; the
    same members stepped one by one with dg_rk_step and together in one
    batch (fused launches, graph replay).  Reports aggregate
    cell-updates/s per RHS of both and checks bitwise equality.  With
    --batch-precond fd or fd-products the members hold the fast-
    diagonalisation preconditioner (with fd-products on the folded matrix
    products, no FFT plans) and the batch steps them one after the other
    through dg_rk_step, so the two runs differ only in the loop's place."""
    import numpy as np
    import torch
    from paper_1311_7477_amd import dg, inputs
    rng = np.random.default_rng(2)
    members = []
    for _ in range(args.members):
        n = int(rng.integers(2, 6))
        N = int(round(math.exp(rng.uniform(math.log(64), math.log(args.N_max)))))
        k0 = float(rng.uniform(4.0, 16.0))
        w0, umax = inputs.random_spectrum(n, N, k0=k0, seed=int(rng.integers(1 << 30)),
                                          return_umax=True)
        members.append((n, N, w0, inputs.cfl_dt(n, N, umax, cfl=0.1)))
    fd_flags = {"none": 0, "fd": dg.DG_WS_FD,
                "fd-products": dg.DG_WS_FD | dg.DG_WS_FD_PRODUCTS}[args.batch_precond]
    opts = dg.cg_opts(rtol=args.rtol,
                      precond=dg.DG_PRECOND_FD if fd_flags else dg.DG_PRECOND_NONE)
    cells = sum(N * N for (_, N, _, _) in members)
    steps = args.steps

    # tile shapes from the tuner, once per (n, N), shared by both runs
    shapes = {}
    for (n, N, w0, dt) in members:
        if (n, N) not in shapes:
            g = dg.Grid(n, N, N)
            shapes[(n, N)] = g.tune(torch.from_numpy(w0).cuda(), reps=5)[0]

    # one by one
    singles = []
    for (n, N, w0, dt) in members:
        g = dg.Grid(n, N, N)
        g.set_tiles(*shapes[(n, N)])
        singles.append((g, dg.Workspace(g, dg.DG_PREC_FP64 | fd_flags), dg.State(g),
                        torch.from_numpy(w0).cuda(), dt))
    print(f"[batch] {len(members)} members, {cells} cells, {len(shapes)} tuned shapes",
          file=sys.stderr, flush=True)
    for (g, ws, st, w, dt) in singles:            # warm-up step
        dg.rk_step(g, w, st, ws, dt, args.D, opts)
    torch.cuda.synchronize()
    print("[batch] one-by-one warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(steps):
        for (g, ws, st, w, dt) in singles:
            dg.rk_step(g, w, st, ws, dt, args.D, opts)
        torch.cuda.synchronize()
        print(f"[batch] one-by-one step {k} at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_single = time.perf_counter() - t0

    # batched
    batch = dg.Batch(len(members))
    if fd_flags:
        batch.use_precond(fd_flags)
    bw = []
    for (n, N, w0, dt) in members:
        g = dg.Grid(n, N, N)
        g.set_tiles(*shapes[(n, N)])
        w = torch.from_numpy(w0).cuda()
        batch.attach(g, w, dt, args.D)
        bw.append((g, w))
    batch.rk_step(opts)                            # warm-up step (+ capture)
    torch.cuda.synchronize()
    print("[batch] batched warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(steps):
        batch.rk_step(opts)
        torch.cuda.synchronize()
        print(f"[batch] batched step {k} at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    t_batch = time.perf_counter() - t0
    same = all(bool(torch.equal(w, s[3])) for (g, w), s in zip(bw, singles))
    rhs = 3 * steps
    print(json.dumps({
        "metric": "batched DG cell-updates/s per RHS (64 uneven instances)",
        "value": cells * rhs / t_batch, "unit": "cell-updates/s",
        "one_by_one_value": cells * rhs / t_single, "speedup": t_single / t_batch,
        "bitwise_equal_to_one_by_one": same, "steps": steps, "warmup": 1,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.members} instances, n~U{{2..5}}, N log-uniform "
                               f"[64,{args.N_max}], k0~U[4,16], D={args.D}, CFL 0.1, "
                               f"CG rtol {args.rtol}, seed 2",
                   "total_cells": cells, "graphs": not fd_flags,
                   "precond": args.batch_precond},
    }), flush=True)


def form_mixed(args):
    """Mixed precision (FP32-stored CG recurrences, FP64 arithmetic, solution
    and residual replacement) against the FP64 CG -- and the CG preconditioned
    by fast diagonalisation, with the preconditioner applied in FP64 and in
    FP32 (the mixed-precision PCG) -- on the double shear layer at
    n = 5: one Poisson solve of the initial vorticity from a zero guess per
    variant (time, iterations, true FP64 residual recomputed on the device),
    then RK3 steps with each solver (time per RHS, difference of the final
    vorticity and streamfunction to the FP64 run)."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    n, N = 5, args.N
    w0, umax = inputs.double_shear_layer(n, N)
    dt = inputs.cfl_dt(n, N, umax, cfl=0.1)
    g = dg.Grid(n, N, N)
    ws = dg.Workspace(g, dg.DG_PREC_MIXED | dg.DG_WS_FD)
    w = torch.from_numpy(w0).cuda()
    xi_w = g.tables()[n:2 * n]
    h = 2 * math.pi / N
    wc = torch.tensor(xi_w, dtype=torch.float64, device="cuda") * (h / 2)
    Wt = (wc[:, None] * wc[None, :]).expand(N, N, n, n)
    b = w - (Wt * w).sum() / Wt.sum()

    def wnorm(u):
        return math.sqrt(float((Wt * u * u).sum()))

    variants = {"fp64": dg.cg_opts(rtol=1e-10),
                "mixed": dg.cg_opts(rtol=1e-10, precision=dg.DG_PREC_MIXED),
                "fp64_precond": dg.cg_opts(rtol=1e-10, precond=dg.DG_PRECOND_FD),
                "mixed_precond": dg.cg_opts(rtol=1e-10, precision=dg.DG_PREC_MIXED,
                                            precond=dg.DG_PRECOND_FD)}
    ref = args.reference
    if ref not in ("fp64", "fp64_precond"):
        raise SystemExit("--reference must be fp64 or fp64_precond (an all-FP64 solve)")
    keep = {ref} | set(args.variants.split(","))
    variants = {k: v for k, v in variants.items() if k in keep}
    others = [k for k in ("mixed", "fp64_precond", "mixed_precond") if k in variants and k != ref]
    if not others:
        raise SystemExit("--variants must name at least one of mixed, fp64_precond, "
                         "mixed_precond besides the reference")
    solves, psis = {}, {}
    for name, opts in variants.items():
        psi = torch.zeros_like(w)
        dg.cg_solve_poisson(g, w, torch.zeros_like(w), ws, opts)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dg.cg_solve_poisson(g, w, psi, ws, opts)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res = b + dg.laplace_apply(g, psi)
        solves[name] = {"ms": t * 1e3, "iters": r.iters, "replacements": r.outer_iters,
                        "status": ("converged" if not r.stalled else "attainable accuracy")
                        if r.converged else "not converged",
                        "true_rel_residual": wnorm(res) / wnorm(b)}
        psis[name] = psi
        print(f"[mixed] solve {name}: {solves[name]}", file=sys.stderr, flush=True)
    for name in others:
        solves[name]["rel_diff_psi_vs_ref"] = wnorm(psis[name] - psis[ref]) / wnorm(psis[ref])

    steps = {}
    for name, opts in variants.items():
        st = dg.State(g)
        wv = torch.from_numpy(w0).cuda()
        dg.rk_step(g, wv, st, ws, dt, 5e-5, opts)                    # warm-up step
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, stalled, failed = [], 0, 0
        for _ in range(args.steps):
            r = dg.rk_step(g, wv, st, ws, dt, 5e-5, opts)
            its += r.cg_iters
            stalled += r.stalled
            failed += not r.converged
        torch.cuda.synchronize()
        steps[name] = ((time.perf_counter() - t0) / (3 * args.steps), wv, st.psi(), its,
                       stalled, failed)
    rel = {}
    for name in others:
        rel[name] = {
            "rel_err_omega_vs_ref": wnorm(steps[name][1] - steps[ref][1]) / wnorm(steps[ref][1]),
            "rel_err_psi_vs_ref": wnorm(steps[name][2] - steps[ref][2]) / wnorm(steps[ref][2]),
            "cell_updates_per_s": N * N / steps[name][0],
            "speedup_vs_ref": steps[ref][0] / steps[name][0],
            "iters_per_rhs": statistics.mean(steps[name][3]),
            "steps_stopped_at_attainable_accuracy": steps[name][4],
            "steps_not_converged": steps[name][5]}
    head = "mixed" if "mixed" in steps else others[-1]
    print(json.dumps({
        "metric": f"mixed-precision CG vs FP64 CG: DG cell-updates/s per RHS ({head})",
        "value": N * N / steps[head][0], "unit": "cell-updates/s",
        "reference": ref, "ref_value": N * N / steps[ref][0],
        "ref_iters_per_rhs": statistics.mean(steps[ref][3]),
        "ref_steps_not_converged": steps[ref][5],
        **{k: rel[k] for k in others},
        "single_solve_from_zero": solves,
        "steps": args.steps, "warmup": 1,
        "dtype": "f32-stored r, p / f64 arithmetic and solution", "data": "synthetic",
        "config": {"workload": f"double shear layer, n=5, {N}x{N}, D=5e-5, CFL 0.1, "
                               "rtol 1e-10 (mixed: on the FP64 residual, or the "
                               "attainable FP64 accuracy)"},
    }), flush=True)


def form_lamb(args):
    """Table 4 of the paper on the GPU: the Lamb dipole (P = 1, N = 200, box
    1 x 1, U = 1, R = 0.1, D = 0) integrated to t = 0.01 with the K-step
    Adams-Bashforth method, K = 1..4, 10/20/40/80 steps (PCG, rtol 1e-14);
    relative enstrophy and energy errors, their orders, and the time."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    n, N = 1, 200
    grid = dg.Grid(n, N, N, 0.0, 1.0, 0.0, 1.0)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    opts = dg.cg_opts(rtol=1e-14, precond=dg.DG_PRECOND_FD)
    w0 = torch.from_numpy(inputs.lamb_dipole(n, N)).cuda()
    p0 = torch.zeros_like(w0)
    dg.cg_solve_poisson(grid, w0, p0, ws, opts)
    V0, E0, Om0 = dg.invariants(grid, w0, p0, ws)
    rows = []
    for K in (1, 2, 3, 4):
        prev = None
        for steps in (10, 20, 40, 80):
            ab = dg.AbState(grid, K)
            w = w0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                dg.ab_step(grid, w, ab, ws, 0.01 / steps, 0.0, opts)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            psi = ab.psi()
            dg.cg_solve_poisson(grid, w, psi, ws, opts)
            V, E, Om = dg.invariants(grid, w, psi, ws)
            eo, ee = abs((Om - Om0) / Om0), abs((E - E0) / E0)
            row = {"K": K, "steps": steps, "eps_V": abs(V), "eps_Omega": eo, "eps_E": ee,
                   "order_Omega": math.log2(prev[0] / eo) if prev else None,
                   "order_E": math.log2(prev[1] / ee) if prev else None,
                   "ms_per_step": t / steps * 1e3}
            prev = (eo, ee)
            rows.append(row)
            print(f"[lamb] {row}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "Table 4: Lamb dipole conservation errors, K-step Adams-Bashforth",
                      "rows": rows, "data": "synthetic (analytic Lamb dipole)", "dtype": "f64",
                      "config": {"workload": "P=1, 200x200 cells, [0,1]^2, U=1, R=0.1, D=0, "
                                             "t in [0, 0.01], PCG rtol 1e-14"}}), flush=True)


# Table 3 of the paper: printed L2 errors at t = 2 (columns: D = 0 periodic,
# D = 0 Dirichlet, D = 0.01 periodic, D = 0.01 Dirichlet), P = 1..4,
# N = 16, 32, 64, 128.
TABLE3_PRINTED = {
    1: [(0.0, 4.00e-01, 2.63e-03, 3.79e-01), (0.0, 3.30e-01, 6.59e-04, 3.07e-01),
        (0.0, 2.00e-01, 1.79e-04, 1.90e-01), (0.0, 1.10e-01, 4.48e-05, 1.00e-01)],
    2: [(5.96e-02, 5.46e-02, 5.63e-02, 5.71e-02), (1.48e-02, 1.38e-02, 1.49e-02, 1.51e-02),
        (3.74e-03, 3.60e-03, 3.83e-03, 3.87e-03), (9.44e-04, 9.20e-04, 9.74e-04, 9.80e-04)],
    3: [(2.59e-03, 2.47e-03, 1.80e-03, 1.69e-03), (3.36e-04, 3.27e-04, 2.32e-04, 2.25e-04),
        (4.34e-05, 4.28e-05, 2.95e-05, 2.91e-05), (5.51e-06, 5.47e-06, 3.73e-06, 3.70e-06)],
    4: [(3.16e-05, 3.33e-05, 4.33e-05, 4.49e-05), (1.84e-06, 1.91e-06, 2.78e-06, 2.84e-06),
        (1.11e-07, 1.13e-07, 1.76e-07, 1.78e-07), (6.79e-09, 6.84e-09, 1.11e-08, 1.12e-08)],
}


def _lap_max(dg, grid, ws_like, iters=80):
    """Largest |eigenvalue| of Lap_h by power iteration on the device (a
    lower estimate; the caller keeps a margin)."""
    import torch
    v = torch.randn(grid.shape, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5))
    lam = 0.0
    for _ in range(iters):
        u = dg.laplace_apply(grid, v)
        lam = float(u.norm() / v.norm())
        v = u / u.norm()
    return lam


def form_table3(args):
    """Table 3 of the paper on the GPU: omega = 2 sin x sin y on [0, 2 pi]^2
    (exact: 2 sin x sin y exp(-2 D t) for periodic and homogeneous Dirichlet
    boundaries) integrated to t = 2 with the three-step Adams-Bashforth
    method (SSP-RK3 start), dt = min(0.1 h / P, 0.3 / (D |lambda_max|));
    L2 error against the exact solution at the Gauss nodes, for every entry
    of the printed table.  Poisson solves: CG preconditioned by fast
    diagonalisation (factored Bloch bases on periodic grids, dense
    eigenbases on Dirichlet grids; rtol 1e-12, the errors are those of the
    spatial discretisation)."""
    import numpy as np
    import torch
    from numpy.polynomial.legendre import leggauss
    from paper_1311_7477_amd import dg, inputs
    rows, t_all = [], time.perf_counter()
    Ns = (16, 32, 64, 128)
    for P in (1, 2, 3, 4):
        for i, N in enumerate(Ns):
            for col, (D, bc) in enumerate(((0.0, 0), (0.0, 1), (0.01, 0), (0.01, 1))):
                t0 = time.perf_counter()
                grid = dg.Grid(P, N, N, bc_x=bc, bc_y=bc)
                ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
                X, Y = inputs.node_coords(P, N, N)
                w0 = 2.0 * np.sin(X) * np.sin(Y)
                h = 2.0 * math.pi / N
                dt = 0.1 * h / P
                if D > 0:
                    dt = min(dt, 0.3 / (D * 1.25 * _lap_max(dg, grid, ws)))
                steps = int(math.ceil(2.0 / dt))
                dt = 2.0 / steps
                opts = dg.cg_opts(rtol=1e-12, precond=dg.DG_PRECOND_FD)
                ab, w = dg.AbState(grid, 3), torch.from_numpy(w0).cuda()
                iters, t_print = 0, time.perf_counter()
                for k in range(steps):
                    r = dg.ab_step(grid, w, ab, ws, dt, D, opts)
                    iters += sum(r.cg_iters)
                    if time.perf_counter() - t_print > 30.0:
                        t_print = time.perf_counter()
                        print(f"[table3] P={P} N={N} D={D} bc={bc}: step {k + 1}/{steps}",
                              file=sys.stderr, flush=True)
                d = w.cpu().numpy() - w0 * math.exp(-2.0 * D * 2.0)
                wg = 0.5 * h * leggauss(P)[1]           # Gauss weights of one cell
                wq = (wg[:, None] * wg[None, :])[None, None]
                err = math.sqrt(float(np.sum(wq * d * d)))
                printed = TABLE3_PRINTED[P][i][col]
                rows.append({"P": P, "N": N, "D": D, "bc": "dirichlet" if bc else "periodic",
                             "error": err, "printed": printed,
                             "ratio": err / printed if printed else None,
                             "steps": steps, "cg_iters": iters,
                             "seconds": time.perf_counter() - t0})
                print(f"[table3] {rows[-1]}", file=sys.stderr, flush=True)
    dev = [abs(r["ratio"] - 1.0) for r in rows
           if r["ratio"] is not None and (r["P"] > 1 or r["bc"] == "dirichlet")]
    print(json.dumps({"metric": "Table 3: L2 errors at t = 2 vs the printed ones",
                      "rows": rows, "max_rel_deviation_P2to4_and_P1_dirichlet": max(dev),
                      "seconds": time.perf_counter() - t_all, "dtype": "f64",
                      "data": "analytic (2 sin x sin y)"}), flush=True)


def form_tune(args):
    """Tile autotuner sweep: for n in {2,3,4,5} and N in {64, 256, 512, 1024},
    dg_grid_tune on a random-spectrum field; prints one line per case with
    the chosen shapes and the per-shape times (CG iteration, bracket)."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    rows = []
    for n in (2, 3, 4, 5):
        for N in (64, 256, 512, 1024):
            w0 = inputs.random_spectrum(n, N, k0=8.0, seed=1)
            g = dg.Grid(n, N, N)
            (cw, rw), ms = g.tune(torch.from_numpy(w0).cuda(), reps=10)
            F = 8 * N * N * n * n
            rows.append({"n": n, "N": N, "cw": cw, "rw": rw,
                         "cg_iter_ms": dict(zip(("cw4", "cw8", "cw16"), ms[:3])),
                         "bracket_ms": dict(zip(("rw8", "rw16"), ms[3:])),
                         "cg_GBps_at_8F": 8 * F / (ms[(4, 8, 16).index(cw)] * 1e-3) / 1e9})
            print(f"[tune] {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "tile autotuner sweep", "cases": rows,
                      "data": "synthetic", "dtype": "f64"}), flush=True)


def form_serve(args):
    """Serving: a seeded Poisson stream of requests (n uniform over {2..5},
    N log-uniform over [N_min, N_max], random spectra), continuous batching
    under an HBM budget; latency percentiles, aggregate throughput and an
    alone-vs-mix check.  --serve-solver batch: the fused batched launches
    with the plain FP64 CG; pcg: a stream and a worker per request with the
    CG preconditioned by fast diagonalisation, its preconditioner in FP32
    under the FP64 iteration.  With --rate 0 the stream runs once per load
    factor in --loads, the arrival rate set to that factor x the measured
    capacity (cell-updates/s of the first four requests run alone, divided
    by the mean request size); --replay requests of each run are then run
    alone again and compared bit for bit."""
    import numpy as np
    from paper_1311_7477_amd import dg, serve

    def stream():
        return serve.draw_requests(args.requests, seed=4, rate=1.0,
                                   N_range=(args.N_min, args.N_max), steps=args.req_steps)

    def server():
        if args.serve_solver == "pcg":
            return serve.StreamServer(capacity=64)
        return serve.Server(capacity=64, opts=dg.cg_opts(rtol=1e-10))

    reqs = stream()
    opts = server().opts
    # capacity estimate: the first four requests run alone, one after another
    t_alone = 0.0
    serve.run_alone(reqs[0], opts, None)                     # warm-up
    for r in reqs[:4]:
        t0 = time.perf_counter()
        serve.run_alone(r, opts, None)
        t_alone += time.perf_counter() - t0
        print(f"[serve] alone: request {r.rid} n={r.n} N={r.N} done", file=sys.stderr,
              flush=True)
    capacity = sum(r.cell_updates for r in reqs[:4]) / t_alone
    mean_size = float(np.mean([r.cell_updates for r in reqs]))
    loads = [float(x) for x in args.loads.split(",")] if args.rate <= 0 else [None]
    runs = []
    for load in loads:
        reqs = stream()
        rate = args.rate if load is None else load * capacity / mean_size
        for r in reqs:
            r.arrival /= rate
        srv = server()
        t0 = time.perf_counter()
        done = srv.run(reqs, log=lambda m: print("[serve] " + m, file=sys.stderr, flush=True))
        makespan = time.perf_counter() - t0
        s = serve.summarize(done, makespan)
        print(f"[serve] load {load}: {s}", file=sys.stderr, flush=True)
        # alone vs in the mix: the first `replay` finished requests again,
        # alone, with the tile shapes the server used
        same = [bool(np.array_equal(r.result, serve.run_alone(r, srv.opts,
                                                              srv.tiles.get((r.n, r.N)))))
                for r in done[:args.replay]]
        s.update({"load": load, "arrival_rate_per_s": rate, "makespan_s": makespan,
                  "max_concurrent": srv.max_active, "failed": len(srv.failed),
                  "rejected": len(srv.rejected), "peak_budgeted_bytes": srv.peak_used,
                  "budget_bytes": srv.budget, "alone_equals_mix": same})
        runs.append(s)
    out = {
        "metric": "served DG cell-updates/s (aggregate) with p50/p99 request latency",
        "value": runs[0]["aggregate_cell_updates_per_s"], "unit": "cell-updates/s",
        "runs": runs, "capacity_cell_updates_per_s_alone": capacity,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.requests} requests, Poisson arrivals (seed 4), "
                               f"n~U{{2..5}}, N log-uniform [{args.N_min},{args.N_max}], "
                               f"{args.req_steps} RK3 steps each, k0~U[4,16], D=1e-4, "
                               f"rtol 1e-10, HBM budget 80% of free memory",
                   "solver": ("stream and worker per request, CG preconditioned by fast "
                              "diagonalisation (FP32 preconditioner, FP64 iteration)"
                              if args.serve_solver == "pcg" else
                              "batched fused launches, plain FP64 CG")},
    }
    print(json.dumps(out), flush=True)


def _dipole_wake(n, N, w):
    """Fraction of the W-norm of omega lying farther than 1.5 R = 0.15 from
    the dipole centre, taken as the periodic midpoint of the nodes of
    largest and smallest omega (box [0, 1]^2): the vorticity the scheme
    sheds outside the dipole."""
    import numpy as np
    from paper_1311_7477_amd import inputs
    X, Y = inputs.node_coords(n, N, N, 0.0, 1.0, 0.0, 1.0)
    a, b = np.unravel_index(np.argmax(w), w.shape), np.unravel_index(np.argmin(w), w.shape)

    def mid(u, v):
        d = (v - u + 0.5) % 1.0 - 0.5
        return (u + 0.5 * d) % 1.0

    cx, cy = mid(X[a], X[b]), mid(Y[a], Y[b])
    dx = (X - cx + 0.5) % 1.0 - 0.5
    dy = (Y - cy + 0.5) % 1.0 - 0.5
    xi, wq = np.polynomial.legendre.leggauss(n)
    W = np.broadcast_to((wq[:, None] * wq[None, :])[None, None], w.shape)
    far = np.hypot(dx, dy) > 0.15
    return float(np.sqrt(np.sum(W * w * w * far) / np.sum(W * w * w))), (float(cx), float(cy))


def form_dipole(args):
    """Sec. 6.2, Figs. 1-2: the Lamb dipole (box [0,1]^2, U = 1, R = 0.1,
    D = 0) advanced to t = 0.5 with the paper's three-step Adams-Bashforth
    method, once with the conservative bracket J = (J++ + J+x + Jx+)/3 and
    once with J++ alone, at P = 1, N = 100 (Fig. 1) and P = 4, N = 50
    (Fig. 2), each at two time steps dt and dt/2.  Reports eps_V, eps_E,
    eps_Omega at t = 0.5 and their ratio between the two time steps (about
    8 where only the third-order time stepping changes E and Omega, about 1
    where the bracket itself does), and the share of the vorticity norm
    shed outside the dipole."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    T = 0.5
    cases = [(1, 100, 5e-4), (4, 50, 2e-4)]
    rows = []
    for (n, N, dt0) in cases:
        grid = dg.Grid(n, N, N, 0.0, 1.0, 0.0, 1.0)
        ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
        opts = dg.cg_opts(rtol=1e-13, precond=dg.DG_PRECOND_FD)
        w0 = torch.from_numpy(inputs.lamb_dipole(n, N)).cuda()
        p0 = torch.zeros_like(w0)
        dg.cg_solve_poisson(grid, w0, p0, ws, opts)
        V0, E0, Om0 = dg.invariants(grid, w0, p0, ws)
        for form_name, form in (("J", dg.DG_FORM_ARAKAWA), ("J++", dg.DG_FORM_PP)):
            res = []
            for dt in (dt0, dt0 / 2):
                steps = int(round(T / dt))
                ab = dg.AbState(grid, 3)
                w = w0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ok = True
                for _ in range(steps):
                    ok = dg.ab_step(grid, w, ab, ws, dt, 0.0, opts, form=form).converged and ok
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                psi = ab.psi()
                dg.cg_solve_poisson(grid, w, psi, ws, opts)
                V, E, Om = dg.invariants(grid, w, psi, ws)
                wake, centre = _dipole_wake(n, N, w.cpu().numpy())
                res.append({"dt": dt, "steps": steps, "eps_V": abs(V),
                            "eps_E": abs((E - E0) / E0), "eps_Omega": abs((Om - Om0) / Om0),
                            "wake_fraction": wake, "centre": centre,
                            "all_converged": ok, "ms_per_step": el / steps * 1e3})
                print(f"[dipole] P={n} N={N} {form_name} {res[-1]}", file=sys.stderr,
                      flush=True)
            rows.append({"P": n, "N": N, "bracket": form_name, "runs": res,
                         "ratio_eps_E_dt_over_dt2": res[0]["eps_E"] / res[1]["eps_E"],
                         "ratio_eps_Omega_dt_over_dt2":
                             res[0]["eps_Omega"] / res[1]["eps_Omega"]})
    print(json.dumps({"metric": "Lamb dipole at t = 0.5: conservation of the average "
                                "bracket J against J++ (Sec. 6.2, Figs. 1-2)",
                      "rows": rows, "data": "synthetic (analytic Lamb dipole)", "dtype": "f64",
                      "config": {"workload": "box [0,1]^2, U=1, R=0.1, D=0, t in [0, 0.5], "
                                             "three-step Adams-Bashforth, PCG rtol 1e-13; "
                                             "P=1 N=100 and P=4 N=50"}}), flush=True)


def form_paper(args):
    """The paper's timing shape (Table 1): one bracket evaluation, N = 100,
    P = 1..4, FP64, beside the printed GTX 570 times (context only)."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    printed = {1: 0.05, 2: 0.26, 3: 0.71, 4: 1.47}
    rows = []
    for n in (1, 2, 3, 4):
        g = dg.Grid(n, 100, 100)
        f = torch.from_numpy(inputs.white_noise(n, 100, 100, 1)).cuda()
        h = torch.from_numpy(inputs.white_noise(n, 100, 100, 2)).cuda()
        out = torch.empty_like(f)
        for _ in range(10):
            dg.poisson_bracket(g, f, h, out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(200):
            dg.poisson_bracket(g, f, h, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 200
        rows.append({"P": n, "ms": ms, "paper_gtx570_ms": printed[n],
                     "ratio": printed[n] / ms})
    print(json.dumps({"metric": "bracket time, N=100 (Table 1 shape)", "unit": "ms",
                      "rows": rows, "higher_is_better": False, "dtype": "f64",
                      "data": "synthetic"}), flush=True)


def form_dirichlet(args):
    """The Poisson solve on a grid with homogeneous Dirichlet boundaries on
    both axes (n = 4, 512^2 cells by default, [0, 2 pi]^2, random-spectrum
    right-hand side): the preconditioner's setup (dense eigenbases, one
    rocSOLVER eigensolve per distinct axis), single solves from a zero guess
    with plain CG, PCG and the FP32-preconditioned PCG (rtol 1e-10), and
    SSP-RK3 steps with each solver."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    n, N = args.n, args.N
    omega0, umax = inputs.random_spectrum(n, N, k0=10.0, seed=1, return_umax=True)
    dt = inputs.cfl_dt(n, N, umax, cfl=0.1)
    grid = dg.Grid(n, N, N, bc_x=dg.DG_BC_DIRICHLET, bc_y=dg.DG_BC_DIRICHLET)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    setup_s = time.perf_counter() - t0
    print(f"[dirichlet] workspace with dense eigenbases: {setup_s:.2f} s", file=sys.stderr,
          flush=True)
    w = torch.from_numpy(omega0).cuda()
    variants = {"plain_fp64": dg.cg_opts(rtol=1e-10),
                "precond_fp64": dg.cg_opts(rtol=1e-10, precond=dg.DG_PRECOND_FD),
                "precond_mixed": dg.cg_opts(rtol=1e-10, precond=dg.DG_PRECOND_FD,
                                            precision=dg.DG_PREC_MIXED)}
    solves, ref = {}, None
    for name, opts in variants.items():
        best = None
        for _ in range(3):
            psi = torch.zeros_like(w)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = dg.cg_solve_poisson(grid, w, psi, ws, opts)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        if ref is None:
            ref = psi
        solves[name] = {"ms": best * 1e3, "iters": res.iters, "converged": res.converged,
                        "rel_diff_vs_plain": float((psi - ref).norm() / ref.norm())}
        print(f"[dirichlet] solve {name}: {solves[name]}", file=sys.stderr, flush=True)
    steps = {}
    for name in ("plain_fp64", "precond_fp64", "precond_mixed"):
        st, wk = dg.State(grid), torch.from_numpy(omega0).cuda()
        k_steps = 2 if name == "plain_fp64" else 50
        dg.rk_step(grid, wk, st, ws, dt, 1e-4, variants[name])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for _ in range(k_steps):
            r = dg.rk_step(grid, wk, st, ws, dt, 1e-4, variants[name])
            its += r.cg_iters
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        steps[name] = {"value": N * N * 3 * k_steps / T, "unit": "cell-updates/s",
                       "steps": k_steps, "cg_iters_per_rhs": statistics.mean(its)}
        print(f"[dirichlet] rk3 {name}: {steps[name]}", file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "Poisson solve and RK3 steps on a Dirichlet grid", "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"n={n}, {N}x{N} cells, [0,2pi]^2, homogeneous Dirichlet on "
                                f"both axes, random-spectrum omega0 (k0=10, seed 1), rtol "
                                f"1e-10, D=1e-4, dt={dt:.4e}")},
        "setup_seconds": setup_s,
        "workspace_bytes": grid.workspace_bytes(dg.DG_PREC_FP64 | dg.DG_WS_FD),
        "precond_flops_per_apply": 2 * (n * N) ** 2 * (2 * n * N) * 2,
        "solves": solves, "rk3": steps}), flush=True)


def form_turbulence(args):
    print(json.dumps(turbulence_runs(args)), flush=True)


def turbulence_runs(args):
    """The full decaying-turbulence run: n = 4, 512^2 periodic cells,
    random-spectrum omega0 (k0 = 10, seed 1), CFL 0.1, `--run-steps` SSP-RK3
    steps (default 2000) for D = 0 and D = 1e-4 after 50 warm-up steps, CG
    preconditioned by the exact fast-diagonalisation inverse (rtol 1e-12,
    extrapolated guess); per-RHS device times over every RHS of the run.
    Reports the invariants V = int omega, E = 1/2 int psi omega and
    Omega = 1/2 int omega^2 along the run: with D = 0 the scheme conserves E
    and Omega up to the RK3 time error and the CG tolerance, with D > 0 they
    decay."""
    import torch
    from paper_1311_7477_amd import dg, inputs
    n, N = args.n, args.N
    omega0, umax = inputs.random_spectrum(n, N, k0=10.0, seed=1, return_umax=True)
    dt = inputs.cfl_dt(n, N, umax, cfl=0.1)
    grid = dg.Grid(n, N, N)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    opts = dg.cg_opts(rtol=args.rtol, precond=dg.DG_PRECOND_FD)
    every = max(1, args.run_steps // 8)
    runs = []
    for D in (0.0, 1e-4):
        # 50 warm-up steps on a copy, then the run from omega0
        st = dg.State(grid)
        w = torch.from_numpy(omega0).cuda()
        for _ in range(50):
            dg.rk_step(grid, w, st, ws, dt, D, opts)
        st = dg.State(grid)
        w = torch.from_numpy(omega0).cuda()
        psi = torch.zeros_like(w)
        dg.cg_solve_poisson(grid, w, psi, ws, opts)
        V0, E0, Om0 = dg.invariants(grid, w, psi, ws)
        track = [{"step": 0, "t": 0.0, "V": V0, "E": E0, "Omega": Om0}]
        iters, stage_ms, busy, last = [], [], 0.0, time.perf_counter()
        for k in range(1, args.run_steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = dg.rk_step(grid, w, st, ws, dt, D, opts, record_times=True)
            torch.cuda.synchronize()
            busy += time.perf_counter() - t0
            if not r.converged:
                raise RuntimeError(f"CG did not converge at step {k} (D={D})")
            iters.extend(r.cg_iters)
            stage_ms.extend(r.stage_ms)
            if k % every == 0 or k == args.run_steps:
                psi = torch.zeros_like(w)
                dg.cg_solve_poisson(grid, w, psi, ws, opts)
                V, E, Om = dg.invariants(grid, w, psi, ws)
                track.append({"step": k, "t": k * dt, "V": V, "E": E, "Omega": Om,
                              "dE_rel": (E - E0) / E0, "dOmega_rel": (Om - Om0) / Om0})
            if time.perf_counter() - last > 20 or k == args.run_steps:
                last = time.perf_counter()
                print(f"[turbulence] D={D} step {k}/{args.run_steps} "
                      f"{track[-1]}", file=sys.stderr, flush=True)
        srt = sorted(stage_ms)
        runs.append({"D": D, "steps": args.run_steps, "t_end": args.run_steps * dt,
                     "value": N * N * 3 * args.run_steps / busy,
                     "ms_per_step": busy / args.run_steps * 1e3,
                     "latency_ms_per_rhs": {
                         "p50": srt[len(srt) // 2],
                         "p99": srt[min(len(srt) - 1, int(math.ceil(0.99 * len(srt))) - 1)],
                         "mean": statistics.mean(stage_ms)},
                     "cg_iters_per_rhs": {"mean": statistics.mean(iters), "max": max(iters)},
                     "invariants": track})
    return {
        "metric": "decaying turbulence run: invariants and throughput",
        "unit": "cell-updates/s", "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"decaying 2D turbulence, periodic [0,2pi]^2, n={n}, "
                                f"{N}x{N} cells, random-spectrum omega0 (k0=10, seed 1), "
                                f"dt={dt:.4e} (CFL 0.1), SSP-RK3, {args.run_steps} steps "
                                f"after 50 warm-up steps, PCG (fast diagonalisation) rtol "
                                f"{args.rtol}, extrapolated guess"),
                   "n": n, "Nx": N, "Ny": N},
        "runs": runs}


def check_solve(grid, omega, guess, ws, opts):
    """One more solve of the kind the timed steps make (the final omega,
    from the newest psi as guess), outside the timed region, with its true
    relative residual ||b + Lap_h psi||_W / ||b||_W recomputed on the device
    by the library's Laplacian: the recursive residual the CG stops on
    can fall below what FP64 can confirm."""
    import torch
    from paper_1311_7477_amd import dg
    n = grid.n
    psi = guess.clone()
    r = dg.cg_solve_poisson(grid, omega, psi, ws, opts)
    xw = grid.tables()[n:2 * n]
    hx, hy = 2 * math.pi / grid.nx, 2 * math.pi / grid.ny
    w1 = torch.tensor(xw, dtype=torch.float64, device="cuda")
    W = ((w1 * hy / 2)[:, None] * (w1 * hx / 2)[None, :]).expand(grid.shape)
    b = omega - (W * omega).sum() / W.sum()
    res = b + dg.laplace_apply(grid, psi)
    true_rel = math.sqrt(float((W * res * res).sum()) / float((W * b * b).sum()))
    return {"iters": r.iters, "converged": r.converged, "rtol": opts.rtol,
            "recursive_rel_residual": r.rel_residual, "true_rel_residual": true_rel}


def precond_leg(args, omega0, dt, tiles):
    """The same workload (fresh from omega0) with CG preconditioned by the
    exact fast-diagonalisation inverse of -Lap_h: W warm-up steps, then K
    timed steps; per-RHS latency from HIP events around each stage."""
    import torch
    from paper_1311_7477_amd import dg
    n, N = args.n, args.N
    grid = dg.Grid(n, N, N)
    grid.set_tiles(*tiles)
    ws = dg.Workspace(grid, dg.DG_PREC_FP64 | dg.DG_WS_FD)
    st = dg.State(grid)
    w = torch.from_numpy(omega0).cuda()
    opts = dg.cg_opts(rtol=args.rtol, precond=dg.DG_PRECOND_FD)
    for _ in range(args.warmup):
        dg.rk_step(grid, w, st, ws, dt, args.D, opts)
    stage_ms, iters = [], []
    all_conv = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = dg.rk_step(grid, w, st, ws, dt, args.D, opts, record_times=True)
        stage_ms.extend(r.stage_ms)
        iters.extend(r.cg_iters)
        all_conv = all_conv and r.converged
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    print(f"[bench] preconditioned: iters {iters} ms {[round(x, 3) for x in stage_ms]}",
          file=sys.stderr, flush=True)
    check = check_solve(grid, w, st.psi(), ws, opts)
    srt = sorted(stage_ms)
    return {
        "value": N * N * 3 * args.steps / T, "unit": "cell-updates/s",
        "ms_per_step": T / args.steps * 1e3,
        "latency_ms_per_rhs": {"p50": srt[len(srt) // 2], "p99": srt[-1],
                               "mean": statistics.mean(stage_ms)},
        "cg_iters_per_rhs": {"mean": statistics.mean(iters), "max": max(iters)},
        "all_converged": all_conv,
        "check_solve": check,
        "workspace_bytes": ws.held_bytes(),
        "precond_flops_per_apply": 4 * n * n * N * N * (N + N),
        "method": "PCG, M = exact (-Lap_h)^+ by fast diagonalisation: separable "
                  "Bloch eigenbases in factored form (FP64 cell Fourier transforms by "
                  "half-length FFTs when both cell counts are even and an axis exceeds "
                  "32 cells, else as folded matrix products; 2n x 2n mixing per wave "
                  "number)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--D", type=float, default=1e-4)
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile shapes instead of running the tuner")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the fast-diagonalisation preconditioned leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 plain 256 MiB device copies (torch copy_) whose "
                         "HBM counters calibrate the profiler's FETCH/WRITE_SIZE")
    ap.add_argument("--form", default="rhs",
                    choices=["rhs", "batch", "mixed", "serve", "paper", "tune", "lamb",
                             "table3", "turbulence", "dirichlet", "dipole"],
                    help="rhs: the headline metric (default); the others measure "
                         "the batched, mixed-precision and served forms and the "
                         "paper's bracket-timing shape")
    ap.add_argument("--variants", default="fp64,mixed,fp64_precond,mixed_precond",
                    help="--form mixed: the solver variants to run (fp64 is always run); "
                         "the plain mixed form does not reach rtol 1e-10 beyond 128^2 "
                         "cells at n = 5")
    ap.add_argument("--reference", default="fp64",
                    help="--form mixed: the all-FP64 solve the others are compared with "
                         "(fp64: plain CG; fp64_precond: the FP64 preconditioned CG)")
    ap.add_argument("--run-steps", dest="run_steps", type=int, default=2000,
                    help="RK3 steps of the full decaying-turbulence runs (--form turbulence, "
                         "and the preconditioned full-run leg of the default form; 0 skips "
                         "that leg)")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--N-max", dest="N_max", type=int, default=256)
    ap.add_argument("--N-min", dest="N_min", type=int, default=32,
                    help="--form serve: smallest grid of the request stream")
    ap.add_argument("--batch-precond", dest="batch_precond", default="none",
                    choices=["none", "fd", "fd-products"],
                    help="--form batch: members with the fast-diagonalisation "
                         "preconditioner (fd-products: on the folded matrix products)")
    ap.add_argument("--serve-solver", dest="serve_solver", default="batch",
                    choices=["batch", "pcg"],
                    help="--form serve: batched plain CG, or a stream per request with "
                         "the FP32-preconditioned CG")
    ap.add_argument("--requests", type=int, default=16)
    ap.add_argument("--rate", type=float, default=20.0,
                    help="--form serve: arrivals per second (0: 0.7 x measured capacity)")
    ap.add_argument("--req-steps", dest="req_steps", type=int, default=10)
    ap.add_argument("--loads", default="0.7,0.9",
                    help="--form serve with --rate 0: arrival rates as fractions of "
                         "the measured capacity, one run each")
    ap.add_argument("--replay", type=int, default=8,
                    help="--form serve: finished requests rerun alone and compared")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the single-instance RHS is not "
              "sharded across GPUs in this build (see the design notes for the "
              "domain-decomposition plan).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1311_7477_amd import dg, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.form != "rhs":
        {"batch": form_batch, "mixed": form_mixed, "serve": form_serve,
         "paper": form_paper, "tune": form_tune, "lamb": form_lamb,
         "table3": form_table3, "turbulence": form_turbulence,
         "dirichlet": form_dirichlet, "dipole": form_dipole}[args.form](args)
        return
    n, N = args.n, args.N
    omega0, umax = inputs.random_spectrum(n, N, k0=10.0, seed=1, return_umax=True)
    dt = inputs.cfl_dt(n, N, umax, cfl=0.1)
    grid = dg.Grid(n, N, N)
    w = torch.from_numpy(omega0).cuda()
    tiles, tune_ms = (grid.tiles(), None) if args.no_tune else grid.tune(w)
    ws = dg.Workspace(grid)
    st = dg.State(grid)
    opts = dg.cg_opts(rtol=args.rtol)
    print(f"[bench] n={n} N={N} D={args.D} dt={dt:.3e} warmup={args.warmup} "
          f"steps={args.steps} tiles={tiles} tune_ms={tune_ms}", file=sys.stderr, flush=True)

    for k in range(args.warmup):
        r = dg.rk_step(grid, w, st, ws, dt, args.D, opts, record_times=True)
        print(f"[bench] warmup step {k}: iters {r.cg_iters} ms {r.stage_ms}",
              file=sys.stderr, flush=True)

    ws.read_profile()           # reset
    ws.profile(True)
    stage_ms, iters = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_conv = True
    for k in range(args.steps):
        r = dg.rk_step(grid, w, st, ws, dt, args.D, opts, record_times=True)
        stage_ms.extend(r.stage_ms)
        iters.extend(r.cg_iters)
        all_conv = all_conv and r.converged
        print(f"[bench] step {k}: iters {r.cg_iters} ms "
              f"{[round(x, 2) for x in r.stage_ms]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    ws.profile(False)
    ms_dir, n_dir, ms_res, n_res = ws.read_profile()
    check = check_solve(grid, w, st.psi(), ws, opts)

    # achievable-bandwidth reference outside the timed region: a plain
    # 256 MiB device-to-device copy (torch copy_), timed with events
    src = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    del src, dst

    rhs = 3 * args.steps
    value = N * N * rhs / T
    F = 8 * N * N * n * n
    # algorithmic bytes per direction-update launch, averaged over both
    # parities (the live timing samples both alike): odd k reads r, p_{k-1}
    # and writes p_k (3 fields); even k also reads p_{k-2} and x and writes
    # x (6 fields)
    alg_bytes = 4.5 * F
    achieved = alg_bytes / (ms_dir * 1e-3) / 1e9
    traffic = measured_traffic(F, tiles[0])
    srt = sorted(stage_ms)

    def pct(q):
        return srt[min(len(srt) - 1, int(math.ceil(q * len(srt))) - 1)]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"decaying 2D turbulence, periodic [0,2pi]^2, n={n}, "
                         f"{N}x{N} cells, random-spectrum omega0 (k0=10, seed 1), "
                         f"D={args.D}, dt={dt:.4e} (CFL 0.1), SSP-RK3, CG rtol "
                         f"{args.rtol}, extrapolated guess; step = 1 RK3 step = 3 RHS"),
            "n": n, "Nx": N, "Ny": N, "rhs_per_step": 3,
            "tiles": {"cell_tile": [64, tiles[0]], "bracket_tile_rows": tiles[1],
                      "tuner_ms": tune_ms},
        },
        "latency_ms_per_rhs": {"p50": pct(0.50), "p99": pct(0.99),
                               "mean": statistics.mean(stage_ms)},
        "cg_iters_per_rhs": {"mean": statistics.mean(iters), "max": max(iters)},
        "all_converged": all_conv,
        "check_solve": check,
        "roofline": {
            "kernel": ("k_cg_dir (CG direction update: p = r + b p, <p, A p>; x += the "
                       "last two a p every other launch)"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": ms_dir,
            "samples": n_dir,
            "residual_kernel_avg_ms": ms_res,
            "algorithmic_bytes_per_launch": alg_bytes,
            "copy_GBps": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "cache_note": ("the CG vectors (3 fields, %.0f MB) fit the 256 MB Infinity "
                           "Cache at this size, so this is effective bandwidth; the "
                           "HBM-bound figure is profiled at n=5, 1024^2" % (3 * F / 1e6)),
        },
    }
    if not args.no_precond:
        out["preconditioned"] = precond_leg(args, omega0, dt, tiles)
        if args.run_steps > 0:
            # the whole run (2000 steps by default, for D = 0 and D = 1e-4)
            # with the preconditioned solve: per-RHS device times over every
            # RHS, and the invariant drift
            out["full_run_preconditioned"] = turbulence_runs(args)
    if not args.no_cpu_baseline:
        psi0 = st.psi().cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(n, N, w.cpu().numpy(), psi0, args.D, dt,
                                           statistics.mean(iters))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
