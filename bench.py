"""Benchmark: split time steps of the full-sphere global workload on one GPU.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu] [--config R,SR,ST,PM]
    python bench.py --ensemble [--members 64] [--steps 3] [--warmup 1]

Workload: 512 (phi, periodic) x 256 (theta, poles) x 128 (r) cells over a
10 km shell, FP64, K = 3 nonlinear iterations per split step, Mach 1e-4,
seeded synthetic initial data (hydrostatic isothermal atmosphere, Gaussian
potential-temperature bubble, seeded velocity noise).  A "step" is one call of
dsw_split_step (K x (residual + three line sweeps)); inputs are resident in
HBM before the timed region.  Prints one JSON line: the step rate, the
roofline of the dominant pass (algorithmic bytes of the fixed four-pass
model per launch over its average launch time, HIP events on the launch
stream; HBM bytes from committed counter summaries when they match the
kernel sources), the adjoint/forward time on the adjoint workload, and the
CPU oracle built for the host, on all its cores at full size and on one core
on a slab.

--sweeps measures the line solves alone and the split step's passes on the
1024 x 512 x 64 sector; --adjoint the adjoint step against the forward step
on the 256 x 128 x 64 sector; --forced the forced split step (source term,
wall velocities, new Dirichlet data) against the plain one on the
1024 x 512 x 64 sector.

--ensemble measures the 64-member ensemble of uneven regional grids instead:
the autotuner picks the launch shapes, then the batched step (one launch per
pass over all members, replayed from one HIP graph) is timed against the same
step done as one dsw_split_step call per member on one stream, from the same
initial states, and the two final states are compared.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s
WORKLOAD = "global"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha():
    h = hashlib.sha256()
    for f in ("dsw_common.hpp", "dsw_internal.hpp", "rows.hpp", "residual.hip", "sweeps.hip",
              "rt_part.hip", "phi_part.hip", "api.hip"):
        with open(os.path.join(ROOT, "paper_2004_13887_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(counts, K):
    """Algorithmic bytes per split step of each pass, the fixed four-pass model
    of the method (one read of every input state and one write of every output
    state per pass; neighbour re-reads and this implementation's extra
    buffers not counted); S = one five-field state at its real array sizes:
      residual   k=0: U^n -> R (2S; Ubar = U^k = U^n);  k>0: U^n, U^k -> Ubar, R (4S)
      sweep r    Ubar, R -> X1 (3S);  sweep theta: Ubar, X1 -> X2 (3S)
      sweep phi  k=0: Ubar = U^k = U^n, X2 -> U^1 (3S);  k>0: Ubar, X2, U^k -> U^{k+1} (4S)
    i.e. 55 + 70 (K - 1) doubles per cell and step."""
    S = 8 * sum(counts)
    return {"residual": 2 * S + 4 * S * (K - 1), "sweep_r": 3 * S * K, "sweep_theta": 3 * S * K,
            "sweep_phi_update": 3 * S + 4 * S * (K - 1), "boundary_copy": 0}


def implementation_bytes(counts, K):
    """The arrays this implementation's passes actually read and write once
    each, per split step (S as above): the residual reads the resident
    midpoint and forms -(U^k - U^n), and the phi pass also writes the next
    iteration's midpoint (and reads U^n for it):
      residual   k=0: U^n -> R (2S);  k>0: Ubar, U^k, U^n -> R (4S)
      sweeps     3S each
      sweep phi  k=0: U^n, X2 -> U^1, Ubar^1 (4S);  0<k<K-1: Ubar, X2, U^k, U^n
                 -> U^{k+1}, Ubar^{k+1} (6S);  k=K-1>0: Ubar, X2, U^k -> U^K (4S)"""
    S = 8 * sum(counts)
    phi = 0
    for k in range(K):
        last = k == K - 1
        phi += ((3 if last else 4) if k == 0 else (4 if last else 6)) * S
    return {"residual": 2 * S + 4 * S * (K - 1), "sweep_r": 3 * S * K, "sweep_theta": 3 * S * K,
            "sweep_phi_update": phi, "boundary_copy": 0}


def measured_traffic(kind, sha):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only if
    they were taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    e = t.get(kind)
    if not e or e.get("source_sha") != sha:
        return None
    return e.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The oracle timed on the host: built for this host (-O3 -march=native,
    no FMA contraction, no fast-math), one split step (K = 3) of the global
    workload at full size on all host cores, and on one core a bounded slab
    of the same recipe (512 x 256 x 8 cells; about half a minute each)."""
    import oracle
    from paper_2004_13887_amd import inputs as I
    L = oracle.lib_bench()
    oracle._lib = L  # the oracle calls below run the host-tuned build
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count()
    if os.environ.get("OMP_NUM_THREADS"):
        ncores = min(ncores, int(os.environ["OMP_NUM_THREADS"]))

    def one_step(w, threads):
        U0, tau = I.initial_state(w)
        g = oracle.Grid(*w.grid.args())
        m = oracle.Material(*w.material.astuple())
        L.orc_set_threads(threads)
        t0 = time.perf_counter()
        oracle.split_step(g, m, U0, tau, w.K)
        return time.perf_counter() - t0

    w_all = I.WORKLOADS[WORKLOAD]
    log(f"[bench] oracle: one step of {w_all.grid.ncells} cells on {ncores} threads")
    dt_all = one_step(w_all, ncores)
    w_one = I.scaled(w_all, 8, 256, 512, name="global-8-levels")
    log(f"[bench] oracle: one step of {w_one.grid.ncells} cells on 1 thread")
    dt_one = one_step(w_one, 1)
    L.orc_set_threads(ncores)
    return {"value": w_all.grid.ncells / dt_all, "unit": "grid-point updates/s", "cores": ncores,
            "kind": "oracle",
            "sample": f"one split step (K={w_all.K}) of the global workload at full size "
                      f"(512x256x128, {w_all.grid.ncells} cells), {dt_all:.1f} s wall on {ncores} threads",
            "one_core": {"value": w_one.grid.ncells / dt_one, "unit": "grid-point updates/s", "cores": 1,
                         "sample": f"one split step (K={w_one.K}) of the global recipe on a 512x256x8 slab "
                                   f"({w_one.grid.ncells} cells), {dt_one:.1f} s wall"},
            "build": "gcc -O3 -march=native -fopenmp -ffp-contract=off -fno-fast-math",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def adjoint_ratio(steps=5, warmup=2):
    """adjoint / forward time on the adjoint workload (256 x 128 x 64 sector):
    one dsw_adjoint_step (its forward recompute included) and the reverse pass
    through the workload's steps from per-step checkpoints, each against one
    dsw_split_step"""
    import numpy as np
    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    w = I.WORKLOADS["adjoint"]
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(w.grid, w.material)
    A, B, out = dsw.to_device(U0), grid.empty(), grid.empty()
    rng = np.random.Generator(np.random.PCG64(7))
    lam = {k: torch.as_tensor(rng.uniform(-1.0, 1.0, v.shape), device="cuda") for k, v in U0.items()}
    stream = torch.cuda.current_stream()
    ck = [A]
    for n in range(w.steps - 1):
        nxt = grid.empty()
        grid.split_step(ck[-1], nxt, tau, w.K, stream)
        ck.append(nxt)

    def timed(fn, n):
        for q in range(warmup):
            fn(q)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for q in range(n):
            fn(warmup + q)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    fwd = timed(lambda q: grid.split_step(A if q % 2 == 0 else B, B if q % 2 == 0 else A, tau, w.K, stream),
                steps)
    adj = timed(lambda q: grid.adjoint_step(A, tau, w.K, lam, out, stream), steps)
    traj = timed(lambda q: grid.adjoint_trajectory(ck, tau, w.K, lam, out, stream), 2) / w.steps
    grid.get_status()
    return {"workload": f"adjoint: 256x128x64 sector, K={w.K}, {w.steps} checkpointed steps",
            "forward_ms": fwd, "adjoint_step_ms": adj, "adjoint_step_over_forward": adj / fwd,
            "trajectory_ms_per_step": traj, "trajectory_over_forward": traj / fwd}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward measurement")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (to scale hardware byte counters)")
    ap.add_argument("--config", default=None,
                    help="launch shapes residual_block,sweep_block_r,sweep_block_theta,phi_rows_per_thread[,rows_per_thread_r,rows_per_thread_theta]")
    ap.add_argument("--ensemble", action="store_true", help="measure the batched ensemble instead")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--adjoint", action="store_true",
                    help="measure the adjoint step against the forward step instead")
    ap.add_argument("--sweeps", action="store_true",
                    help="measure the line solves and the split step's passes on the sweeps workload")
    ap.add_argument("--forced", action="store_true",
                    help="measure the forced split step against the plain one on the sweeps workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library runs one "
              "grid or ensemble per GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.ensemble:
        return bench_ensemble(args)
    if args.adjoint:
        return bench_adjoint(args)
    if args.forced:
        return bench_forced(args)
    if args.sweeps:
        return bench_sweeps(args)

    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    w = I.WORKLOADS[WORKLOAD]
    log(f"[bench] generating {w.name}: {w.grid.np}x{w.grid.nt}x{w.grid.nr} cells")
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(w.grid, w.material)
    if args.config:
        grid.set_config(*(int(x) for x in args.config.split(",")))
    bufs = [dsw.to_device(U0), grid.empty()]
    counts = [v.numel() for v in bufs[0].values()]
    stream = torch.cuda.current_stream()

    def step(n):
        src, dst = bufs[n % 2], bufs[(n + 1) % 2]
        grid.split_step(src, dst, tau, w.K, stream)

    if args.calib:  # known traffic: 1 GiB read + 1 GiB written
        a = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"[bench] warmup {args.warmup} steps (tau = {tau:.4f} s, K = {w.K})")
    for n in range(args.warmup):
        step(n)
    torch.cuda.synchronize()
    grid.get_status()

    grid.set_timing(True)
    grid.read_timing(stream)  # clear
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for n in range(args.steps):
        step(args.warmup + n)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_kernel = grid.read_timing(stream)
    grid.set_timing(False)
    grid.get_status()
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    log(f"[bench] {args.steps} steps: {gpu_ms:.2f} ms GPU, {wall * 1e3:.2f} ms wall")

    cells = w.grid.ncells
    value = cells * args.steps / (gpu_ms * 1e-3)
    alg = algorithmic_bytes(counts, w.K)  # per step
    impl = implementation_bytes(counts, w.K)
    kstats = {}
    for k, (ms, n) in per_kernel.items():
        if n:
            avg = ms / n * 1e-3
            per_launch = alg[k] * args.steps / n  # average algorithmic bytes per launch
            kstats[k] = {"avg_ms": avg * 1e3, "launches": n, "total_ms": ms,
                         "bytes_per_launch": per_launch, "GBps": per_launch / avg / 1e9,
                         "implementation_bytes_per_launch": impl[k] * args.steps / n}
            log(f"[bench] {k:17s} {n:4d} launches, avg {avg * 1e3:8.3f} ms, "
                f"{per_launch / avg / 1e9:8.1f} GB/s algorithmic")
    dom = max(kstats, key=lambda k: kstats[k]["total_ms"])
    sha = kernel_sources_sha()
    achieved = kstats[dom]["GBps"]
    traffic = measured_traffic(dom, sha)
    step_bytes = sum(alg.values())
    out = {
        "metric": "grid-point updates/s per split step (FP64) + % HBM roofline; adjoint/forward time",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "global: 512 (phi, periodic) x 256 (theta) x 128 (r) full sphere, "
                               "10 km shell, K=3, Mach 1e-4, seeded bubble + noise",
                   "cells": cells, "K": w.K, "tau_s": tau,
                   "launch_config": dict(zip(("residual_block", "sweep_block_r", "sweep_block_theta",
                                              "phi_rows_per_thread", "rows_per_thread_r",
                                              "rows_per_thread_theta"), grid.get_config()))},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": achieved / (PEAK_HBM / 1e9), "traffic": traffic,
                     "bytes_per_launch": kstats[dom]["bytes_per_launch"],
                     "avg_launch_ms": kstats[dom]["avg_ms"],
                     "implementation_bytes_per_launch": kstats[dom]["implementation_bytes_per_launch"],
                     "source_sha": sha},
        "step_algorithmic_GBps": step_bytes / (ms_per_step * 1e-3) / 1e9,
        "step_frac": step_bytes / (ms_per_step * 1e-3) / PEAK_HBM,
        "kernels": kstats,
    }
    if not args.no_adjoint:
        log("[bench] adjoint / forward on the adjoint workload")
        del bufs
        torch.cuda.empty_cache()
        out["adjoint"] = adjoint_ratio()
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """adjoint workload (64 x 128 x 256 sector, 100 m, Mach 1e-2, K = 3): time
    of dsw_adjoint_step (forward recompute from the checkpoint included)
    against dsw_split_step; also the taped pair (dsw_split_step_taped, then
    dsw_adjoint_step_taped without the recompute) and the reverse pass
    through the workload's 10 steps from per-step checkpoints
    (dsw_adjoint_trajectory, every step's recompute included)"""
    import numpy as np
    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    w = I.WORKLOADS["adjoint"]
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(w.grid, w.material)
    if args.config:
        grid.set_config(*(int(x) for x in args.config.split(",")))
    A, B = dsw.to_device(U0), grid.empty()
    rng = np.random.Generator(np.random.PCG64(7))
    lam = {k: torch.as_tensor(rng.uniform(-1.0, 1.0, v.shape), device="cuda") for k, v in U0.items()}
    out = grid.empty()
    stream = torch.cuda.current_stream()
    tape = grid.new_tape(w.K)
    times = {}
    for name in ("forward", "adjoint", "forward_taped", "adjoint_taped"):
        def one(n):
            if name == "forward":
                src, dst = (A, B) if n % 2 == 0 else (B, A)
                grid.split_step(src, dst, tau, w.K, stream)
            elif name == "adjoint":
                grid.adjoint_step(A, tau, w.K, lam, out, stream)
            elif name == "forward_taped":
                grid.split_step_taped(A, B, tau, w.K, tape, stream)
            else:
                grid.adjoint_step_taped(A, tau, w.K, tape, lam, out, stream)
        for n in range(args.warmup):
            one(n)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for n in range(args.steps):
            one(args.warmup + n)
        ev1.record(stream)
        torch.cuda.synchronize()
        times[name] = ev0.elapsed_time(ev1) / args.steps
        log(f"[adjoint] {name}: {times[name]:.3f} ms per step")
    # the adjoint workload's reverse pass: w.steps steps from per-step
    # checkpoints (computed before the timed region), one call per pass
    ck = [A]
    for n in range(w.steps - 1):
        nxt = grid.empty()
        grid.split_step(ck[-1], nxt, tau, w.K, stream)
        ck.append(nxt)
    ntraj = max(1, args.steps // 5)
    for n in range(max(1, args.warmup // 2)):
        grid.adjoint_trajectory(ck, tau, w.K, lam, out, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for n in range(ntraj):
        grid.adjoint_trajectory(ck, tau, w.K, lam, out, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    traj_ms = ev0.elapsed_time(ev1) / (ntraj * w.steps)
    log(f"[adjoint] trajectory of {w.steps} steps: {traj_ms:.3f} ms per step ({ntraj} passes)")
    grid.get_status()
    out_line = {
        "metric": "adjoint step time / forward step time (reverse pass through the workload's steps "
                  "from per-step checkpoints, every step's forward recompute included)",
        "value": traj_ms / times["forward"],
        "unit": "ratio",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": traj_ms,
        "forward_ms_per_step": times["forward"],
        "single_step": {"adjoint_ms": times["adjoint"], "adjoint_over_forward": times["adjoint"] / times["forward"]},
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"adjoint: 256 (phi) x 128 (theta) x 64 (r) sector, 100 m horizontal, "
                               f"K=3, Mach 1e-2, seeded bubble + noise, {w.steps} steps checkpointed",
                   "cells": w.grid.ncells, "K": w.K},
        "taped": {"forward_taped_ms": times["forward_taped"], "adjoint_taped_ms": times["adjoint_taped"],
                  "adjoint_taped_over_forward": times["adjoint_taped"] / times["forward"],
                  "tape_bytes": grid.tape_bytes(w.K)},
        "trajectory": {"steps": w.steps, "passes": ntraj, "adjoint_ms_per_step": traj_ms,
                       "adjoint_over_forward": traj_ms / times["forward"]},
    }
    print(json.dumps(out_line), flush=True)


def bench_sweeps(args):
    """sweeps workload (1024 x 512 x 64 sector, 100 m, Mach 1e-6, K = 3): GB/s
    of each pass of the split step (HIP events around every launch) and of
    the three exported line solves alone, dsw_line_solve_{r,theta,phi} on
    (Ubar = U^n, rhs = the first residual); algorithmic bytes: 3 states per
    line solve (reads Ubar and rhs, writes x)"""
    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    w = I.WORKLOADS["sweeps"]
    log(f"[sweeps] generating {w.name}: {w.grid.np}x{w.grid.nt}x{w.grid.nr} cells")
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(w.grid, w.material)
    if args.config:
        grid.set_config(*(int(x) for x in args.config.split(",")))
    A, B = dsw.to_device(U0), grid.empty()
    counts = [v.numel() for v in A.values()]
    S = 8 * sum(counts)
    stream = torch.cuda.current_stream()
    # split-step passes
    for n in range(args.warmup):
        grid.split_step(A if n % 2 == 0 else B, B if n % 2 == 0 else A, tau, w.K, stream)
    torch.cuda.synchronize()
    grid.set_timing(True)
    grid.read_timing(stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for n in range(args.steps):
        q = args.warmup + n
        grid.split_step(A if q % 2 == 0 else B, B if q % 2 == 0 else A, tau, w.K, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    per_kernel = grid.read_timing(stream)
    grid.set_timing(False)
    step_ms = ev0.elapsed_time(ev1) / args.steps
    alg = algorithmic_bytes(counts, w.K)
    passes = {}
    for k, (ms, n) in per_kernel.items():
        if n and alg[k]:
            avg = ms / n * 1e-3
            per_launch = alg[k] * args.steps / n
            passes[k] = {"avg_ms": avg * 1e3, "GBps": per_launch / avg / 1e9}
            log(f"[sweeps] split-step {k:17s} avg {avg * 1e3:7.3f} ms, {per_launch / avg / 1e9:7.1f} GB/s")
    # the exported line solves alone
    R, Ub, X = grid.empty(), grid.empty(), grid.empty()
    grid.residual(A, A, tau, R, Ub, stream)
    solves = {}
    for d, name in enumerate(("r", "theta", "phi")):
        for _ in range(args.warmup):
            grid.line_solve(d, Ub, tau, R, X, stream)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            grid.line_solve(d, Ub, tau, R, X, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        solves[name] = {"avg_ms": ms, "GBps": 3 * S / (ms * 1e-3) / 1e9}
        log(f"[sweeps] dsw_line_solve_{name:5s} {ms:7.3f} ms, {3 * S / (ms * 1e-3) / 1e9:7.1f} GB/s")
    grid.get_status()
    model_bytes = sum(alg.values())
    out = {
        "metric": "GB/s per line solve (FP64, algorithmic bytes)",
        "value": min(v["GBps"] for v in solves.values()),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sweeps: 1024 (phi) x 512 (theta) x 64 (r) sector, 100 m horizontal, K=3, "
                               "Mach 1e-6, seeded bubble + noise", "cells": w.grid.ncells, "K": w.K},
        "line_solves": solves,
        "split_step_passes": passes,
        "split_step_model_GBps": model_bytes / (step_ms * 1e-3) / 1e9,
    }
    print(json.dumps(out), flush=True)


def bench_forced(args):
    """sweeps workload (1024 x 512 x 64 sector: walls on every side), K = 3:
    dsw_split_step_forced with a seeded source term, seeded wall velocities
    on all twelve wall arrays at t^n and t^{n+1}, and new Dirichlet data, against dsw_split_step
    on the same grid; ms per step and grid-point updates/s of each"""
    import numpy as np
    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    w = I.WORKLOADS["sweeps"]
    g = w.grid
    log(f"[forced] generating {w.name}: {g.np}x{g.nt}x{g.nr} cells")
    U0, tau = I.initial_state(w)
    grid = dsw.Grid.from_spec(g, w.material)
    if args.config:
        grid.set_config(*(int(x) for x in args.config.split(",")))
    rng = np.random.Generator(np.random.PCG64(200413899))
    us = w.mach * 347.0
    src = {"p": 1e-6 * np.mean(U0["p"]) / tau * rng.uniform(-1, 1, U0["p"].shape),
           "ur": us / tau * rng.uniform(-1, 1, U0["ur"].shape),
           "ut": us / tau * rng.uniform(-1, 1, U0["ut"].shape),
           "uf": us / tau * rng.uniform(-1, 1, U0["uf"].shape),
           "T": 1e-6 * np.mean(U0["T"]) / tau * rng.uniform(-1, 1, U0["T"].shape)}
    shp = {"ur_t1": (g.nr + 1, g.np), "ur_t2": (g.nr + 1, g.np), "ur_p1": (g.nr + 1, g.nt),
           "ur_p2": (g.nr + 1, g.nt), "ut_r1": (g.nt + 1, g.np), "ut_r2": (g.nt + 1, g.np),
           "ut_p1": (g.nr, g.nt + 1), "ut_p2": (g.nr, g.nt + 1), "uf_r1": (g.nt, g.npf),
           "uf_r2": (g.nt, g.npf), "uf_t1": (g.nr, g.npf), "uf_t2": (g.nr, g.npf)}
    wall = {k: us * rng.uniform(-1, 1, s) for k, s in shp.items()}
    bnd = {k: U0[k] + us * rng.uniform(-1, 1, U0[k].shape) for k in ("ur", "ut", "uf")}
    # the wall velocities at t^{n+1}: those at t^n plus a seeded change
    wall1 = {k: v + 0.1 * us * rng.uniform(-1, 1, v.shape) for k, v in wall.items()}
    dsrc, dwall, dwall1, dbnd = (dsw.to_device(src), dsw.to_device(wall), dsw.to_device(wall1),
                                 dsw.to_device(bnd))
    del src, bnd, wall1
    A, B = dsw.to_device(U0), grid.empty()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run(forced):
        X, Y = A, B
        for n in range(args.warmup + args.steps):
            if n == args.warmup:
                torch.cuda.synchronize()
                ev0.record(stream)
            if forced:
                grid.split_step_forced(X, Y, tau, w.K, src=dsrc, wall0=dwall, wall1=dwall1, bnd=dbnd,
                                       stream=stream)
            else:
                grid.split_step(X, Y, tau, w.K, stream)
            X, Y = Y, X
        ev1.record(stream)
        torch.cuda.synchronize()
        grid.get_status()
        return ev0.elapsed_time(ev1) / args.steps

    U0d = dsw.to_device(U0)
    plain_ms = run(False)
    for k in A:
        A[k].copy_(U0d[k])
    forced_ms = run(True)
    log(f"[forced] plain {plain_ms:.3f} ms, forced {forced_ms:.3f} ms per step")
    out = {
        "metric": "grid-point updates/s per forced split step (FP64)",
        "value": g.ncells / (forced_ms * 1e-3),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": forced_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "forced: 1024 (phi) x 512 (theta) x 64 (r) sector, 100 m horizontal, K=3, "
                               "Mach 1e-6, seeded source, wall velocities and Dirichlet data",
                   "cells": g.ncells, "K": w.K},
        "plain": {"ms_per_step": plain_ms, "value": g.ncells / (plain_ms * 1e-3)},
        "forced_over_plain": forced_ms / plain_ms,
    }
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    import torch
    from paper_2004_13887_amd import dsw
    from paper_2004_13887_amd import inputs as I

    ws = I.ensemble_members(n=args.members)
    cells = sum(w.grid.ncells for w in ws)
    K = ws[0].K
    log(f"[ensemble] {len(ws)} members, {cells} cells; generating inputs")
    t0 = time.perf_counter()
    E = dsw.Ensemble([w.grid for w in ws], [w.material for w in ws])
    U0, taus = [], []
    for w in ws:
        u, tau = I.initial_state(w)
        U0.append(dsw.to_device(u))
        taus.append(tau)
        del u
    A = [g.empty() for g in E.members]
    B = [g.empty() for g in E.members]
    keep = [g.empty() for g in E.members]
    log(f"[ensemble] inputs resident after {time.perf_counter() - t0:.1f} s; tuning")
    stream = torch.cuda.current_stream()

    def reset():
        for a, u in zip(A, U0):
            for k in a:
                a[k].copy_(u[k])

    reset()
    if args.config:
        cfg = tuple(int(x) for x in args.config.split(","))
        E.set_config(*cfg)
        log(f"[ensemble] launch shapes {cfg} (given)")
    else:
        # three timed runs per candidate: with one, timing noise between
        # close candidates flipped the choice from run to run
        cfg = E.ensemble_tune(A, B, taus, K, reps=3, stream=stream)
        log(f"[ensemble] tuned launch shapes {cfg}")
    # the per-member calls take the same launch shapes, so that both paths
    # run the same arithmetic (the phi solver's partition depends on them)
    for g in E.members:
        g.set_config(*cfg)

    def run(step_fn, n0, n):
        for q in range(n0, n0 + n):
            src, dst = (A, B) if q % 2 == 0 else (B, A)
            step_fn(src, dst)

    def batched(src, dst):
        E.ensemble_step(src, dst, taus, K, stream)

    def per_member(src, dst):
        for m, g in enumerate(E.members):
            g.split_step(src[m], dst[m], taus[m], K, stream)

    times = {}
    for name, fn in (("batched_graph", batched), ("per_member", per_member)):
        reset()
        run(fn, 0, args.warmup)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        run(fn, args.warmup, args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        times[name] = ev0.elapsed_time(ev1) / args.steps
        log(f"[ensemble] {name}: {times[name]:.2f} ms per step")
        final = A if (args.warmup + args.steps) % 2 == 0 else B
        if name == "batched_graph":
            for kk, f in zip(keep, final):
                for k in kk:
                    kk[k].copy_(f[k])
    E.get_status()
    final = A if (args.warmup + args.steps) % 2 == 0 else B
    diff = 0.0
    for kk, f in zip(keep, final):
        for k in kk:
            n = float(torch.linalg.vector_norm(f[k]))
            d = float(torch.linalg.vector_norm(kk[k] - f[k]))
            diff = max(diff, d / n if n > 0 else d)
    ms = times["batched_graph"]
    out = {
        "metric": "grid-point updates/s per ensemble split step (FP64)",
        "value": cells / (ms * 1e-3),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble: {len(ws)} regional members, sizes U{{64..256}} per "
                               "direction, 100 m horizontal, K=3, seeded", "members": len(ws),
                   "cells": cells, "K": K,
                   "launch_config": dict(zip(("residual_block", "sweep_block_r", "sweep_block_theta",
                                              "phi_rows_per_thread", "rows_per_thread_r",
                                              "rows_per_thread_theta"), cfg))},
        "per_member": {"value": cells / (times["per_member"] * 1e-3),
                       "ms_per_step": times["per_member"]},
        "speedup_vs_per_member": times["per_member"] / ms,
        "max_rel_l2_vs_per_member": diff,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
