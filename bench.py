#!/usr/bin/env python3
"""Benchmark of the MacCormack-TVD step on one MI355X.

Workload (default): the largest single-GPU case, the 3D 1024 x 1024 x 256
box (FP64, gamma 1.4, Pr 1, Ra 1e9, plates at T = 1 and 0.5, periodic in x
and y, seeded +-1e-3 T noise).  The state is synthetic (generated on the GPU
by mtvd_init_state) and resident in HBM before the timed region.

Prints ONE JSON line: cell-updates/s (the median of several repetitions of
K steps, each bracketed by device synchronisations), the roofline of the
dominant sweep kernel (bytes of the per-sweep model: read and write every
field once per node, over its average duration from HIP events recorded on
the library's stream) against the HBM peak and against a measured device
copy, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 MacCormack-TVD cell-updates/s, % HBM roofline; adjoint cost/forward"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
AXES = {0: "sweep_x", 1: "sweep_y", 2: "sweep_z"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the files a sweep kernel's binary and launch shape depend on (the build
# script holds its compiler flags, mtvd_rows.h the default rows per wave)
KERNEL_SOURCES = {2: ("mtvd_2d.hip", "mtvd_device.h", "mtvd_rows.h", "../build.py"),
                  3: ("mtvd_3d.h", "mtvd_3d_x.hip", "mtvd_3d_y.hip", "mtvd_3d_z.hip",
                      "mtvd_device.h", "mtvd_rows.h", "../build.py")}


def source_hash(files=None) -> str:
    """Hash of the kernel sources (all of them, or the named files, relative
    to the package's csrc/)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_10372_amd", "csrc")
    names = sorted(files) if files else sorted(
        f for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    for f in names:
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str, shash: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != shash:
        return None
    return d.get("hbm_bytes_per_launch")


def copy_ref() -> int:
    """A plain 256 MiB device-to-device copy, three times: the dispatch whose
    counter readings scale FETCH_SIZE and WRITE_SIZE to bytes in the
    rocprofv3 summaries.  Returns the bytes one copy moves."""
    import torch
    a = torch.empty(32 << 20, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return 2 * a.numel() * 8


def cpu_model() -> str:
    """The host CPU's model name (lscpu's, from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate_full(kw: dict, budget_s: float, threads: int):
    """Full oracle steps from the initial state, as many as fit in about
    budget_s: (cell-updates/s, steps, seconds)."""
    import oracle
    p = oracle.Params(**kw, nthreads=threads)
    X = oracle.init(p)
    nodes = p.nx * (p.ny if p.ndim == 3 else 1) * p.nz
    t0 = time.perf_counter()
    X, _, _ = oracle.step(p, X, 1)
    one = time.perf_counter() - t0
    extra = max(0, int(budget_s / max(one, 1e-9)) - 1)
    t1 = time.perf_counter()
    if extra:
        X, _, _ = oracle.step(p, X, extra)
    tot = one + (time.perf_counter() - t1)
    return nodes * (1 + extra) / tot, 1 + extra, tot


def _oracle_rate_patches(kw: dict, budget_s: float, threads: int, side: int = 68):
    """The oracle's box operators on sampled column patches of a 3D grid
    (side x side columns, all rows, a two-column halo each way): the six
    operators of a step applied to each patch, patches taken at seeded
    positions until about budget_s have passed.  Rate = inner nodes of the
    patches times operators / 6 over the time: (cell-updates/s, patches,
    seconds)."""
    import numpy as np
    import oracle
    p = oracle.Params(**kw, nthreads=threads)
    rng = np.random.default_rng(12)
    X0 = oracle.init_box(p, 0, 0, side, side)
    # dt of the first patch: a grid of side x side columns with the same
    # spacings as the whole one
    pb = oracle.Params(**{**kw, "nx": side, "ny": side,
                          "aspect": kw["aspect"] * side / kw["nx"]}, nthreads=threads)
    assert kw["nx"] == kw["ny"]
    tau = 0.5 * oracle.dt(pb, X0)
    inner = (side - 4) * (side - 4) * p.nz
    order = (2, 1, 0, 2, 1, 0)
    done, tot = 0, 0.0
    while True:
        i0, j0 = int(rng.integers(0, p.nx)), int(rng.integers(0, p.ny))
        B = oracle.init_box(p, i0, j0, side, side)
        t0 = time.perf_counter()
        for a in order:
            B = oracle.sweep_box(p, a, tau, B)
        tot += time.perf_counter() - t0
        done += 1
        if tot >= budget_s:
            break
    return inner * done / tot, done, tot


def cpu_baseline(kw: dict, budget_s: float):
    """The CPU oracle, as it stands (gcc -O2, no fast-math, OpenMP over
    rows), on a bounded sample of the workload, single-threaded and on all
    host cores.  2D: full steps from the initial state.  3D: the six box
    operators of a step on sampled 68 x 68-column patches (all rows), since
    a full step of the 1024 x 1024 x 256 grid takes minutes."""
    import oracle
    allc = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    share = 0.25 if kw["ndim"] == 3 else 0.3
    if kw["ndim"] == 3:
        r1, n1, s1 = _oracle_rate_patches(kw, share * budget_s, 1)
        rn, nn, sn = _oracle_rate_patches(kw, (1 - share) * budget_s, allc)
        what = (f"sampled: the 6 box operators of one step on {nn} seeded 68x68-column "
                f"patches of all {kw['nz']} rows ({nn * 64 * 64 * kw['nz']} inner nodes, "
                f"{sn:.1f} s, {allc} threads); single thread {n1} patches in {s1:.1f} s")
    else:
        r1, n1, s1 = _oracle_rate_full(kw, share * budget_s, 1)
        rn, nn, sn = _oracle_rate_full(kw, (1 - share) * budget_s, allc)
        what = (f"{nn} full steps of the same workload from its initial state "
                f"({sn:.1f} s, {allc} threads); single thread {n1} steps in {s1:.1f} s")
    del oracle
    return {"value": rn, "unit": "cell-updates/s", "cores": allc, "kind": "oracle",
            "sample": what, "single_thread_value": r1, "cpu_model": cpu_model()}


def copy_bandwidth(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """GB/s of a plain device-to-device copy of nbytes (read + write bytes
    over the median time of reps copies, timed with events on torch's
    stream)."""
    import statistics

    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / statistics.median(ts) / 1e9


def bench_batch(args):
    """The 64-box batch: batched throughput over all boxes (graph-replayed
    step pairs, rows per wave from the autotuner) next to the same boxes
    advanced one after another with the plain single-box step."""
    import torch
    import paper_2411_10372_amd as mtvd
    from paper_2411_10372_amd.workloads import batch_boxes

    fields = mtvd.Params.__dataclass_fields__
    ps = [mtvd.Params(**{k: v for k, v in kw.items() if k in fields}) for kw in batch_boxes()]
    nodes = sum(p.nodes for p in ps)
    K, W = args.steps, args.warmup
    torch.cuda.set_device(0)
    b = mtvd.Batch(ps, device="cuda:0")
    b.init_state()
    t0 = time.perf_counter()
    if args.batch_rows:
        # rows per wave given per box size (as a previous run's autotuner
        # chose them): no trial launches, e.g. inside a profiler's window
        rows = json.loads(args.batch_rows)
        for i, p in enumerate(ps):
            rx, rz = rows[f"{p.nx}x{p.nz}"]
            b.set_tiling(i, rx, rz)
    else:
        b.autotune(trial_steps=4)
    t_tune = time.perf_counter() - t0
    b.step(W)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    ev[0].record()
    b.step(K)
    ev[1].record()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    gpu_ms = ev[0].elapsed_time(ev[1])
    # plain single-box steps, one box after another, on the same GPU
    kp = max(2, min(K, 50))
    solvers = [mtvd.Solver(p, device="cuda:0") for p in ps]
    for s in solvers:
        s.init_state()
        s.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(kp)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    tiles = {}
    for i, p in enumerate(ps):
        tiles[f"{p.nx}x{p.nz}"] = b.tiling(i)
    launch_bytes = nodes * 2 * 4 * 8
    per_launch_s = 1e-3 * gpu_ms / (4 * K)
    achieved = launch_bytes / per_launch_s / 1e9
    shash = source_hash(KERNEL_SOURCES[2])
    traffic = load_traffic("batch_64_mixed_2d", "sweep_batch2d", shash)
    out = {
        "metric": METRIC, "value": nodes * K / t_b, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": 1e3 * t_b / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded initial states generated on the GPU)",
        "config": {"workload": "batch_64_mixed_2d", "boxes": len(ps), "nodes": nodes,
                   "sizes": sorted(set(f"{p.nx}x{p.nz}" for p in ps)),
                   "Ra_range": [min(p.Ra for p in ps), max(p.Ra for p in ps)]},
        "roofline": {"bound": "hbm", "kernel": "sweep_batch2d", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": launch_bytes,
                     "note": "average over the 4 operator launches of a step (graph replay)"},
        "plain_sequential_value": nodes * kp / t_p,
        "speedup_vs_plain_sequential": (nodes * K / t_b) / (nodes * kp / t_p),
        "autotune_s": t_tune, "rows_per_wave_x_z": tiles,
        "source_hash": shash,
    }
    if args.copy_ref:
        out["copy_ref_bytes"] = copy_ref()
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Cost of the gradient of the time-averaged Nu-bar (checkpointed forward
    pass + backward pass) as a multiple of the plain forward run of the same
    steps on the same GPU.  --steps counts gradient evaluations here (at most
    10); each covers the workload's 500 steps."""
    import numpy as np
    import torch
    import paper_2411_10372_amd as mtvd
    from paper_2411_10372_amd.workloads import WORKLOADS, params_dict

    wl = WORKLOADS[args.workload]
    p = mtvd.Params(**params_dict(args.workload))
    N, E = wl["steps"], wl["adjoint_every"]
    if args.adjoint_steps:          # a shorter gradient (counter runs)
        N = args.adjoint_steps
    reps = max(1, min(args.steps, 10))
    torch.cuda.set_device(0)
    rng = np.random.default_rng(wl["theta_seed"])
    theta = torch.tensor(wl["theta_amp"] * rng.uniform(-1.0, 1.0, size=(p.nz, p.nx)),
                         device="cuda:0")
    a = mtvd.Adjoint(p, N, E, device="cuda:0")
    J, dt = a.forward(theta, 0.0)
    a.backward(1.0)
    # the plain step of the same box with the same frozen dt, N steps
    s = mtvd.Solver(p, device="cuda:0")
    s.init_state()
    s.step(max(1, args.warmup))
    s.sync()
    tf, tb, tp = [], [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(N)
        s.sync()
        t1 = time.perf_counter()
        a.forward(theta, dt)
        t2 = time.perf_counter()
        a.backward(1.0)
        t3 = time.perf_counter()
        tp.append(t1 - t0)
        tf.append(t2 - t1)
        tb.append(t3 - t2)
    t_plain, t_fwd, t_bwd = (float(np.median(v)) for v in (tp, tf, tb))
    nodes = p.nodes
    # algorithmic bytes of the backward pass per node and step: every
    # operator's input recomputed once (read + write the state, 64 B) and
    # reversed once (read X and the output cotangent, write the input
    # cotangent, 96 B)
    bwd_bytes = nodes * N * 4 * (64 + 96)
    achieved = bwd_bytes / t_bwd / 1e9
    out = {
        "metric": "adjoint cost/forward", "value": (t_fwd + t_bwd) / t_plain, "unit": "x",
        "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": 1e3 * (t_fwd + t_bwd) / N, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded temperature perturbation)",
        "config": {"workload": args.workload, "nx": p.nx, "nz": p.nz, "Ra": p.Ra,
                   "steps_per_gradient": N, "checkpoint_every": E, "dt": dt},
        "plain_forward_ms": 1e3 * t_plain, "adjoint_forward_ms": 1e3 * t_fwd,
        "adjoint_backward_ms": 1e3 * t_bwd, "backward_over_plain": t_bwd / t_plain,
        "roofline": {"bound": "hbm", "kernel": "backward pass (reverse and recompute kernels)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_gradient": bwd_bytes},
        "J": J, "workspace_MiB": a.workspace_bytes / 2 ** 20,
        "source_hash": source_hash(),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="steps per timed repetition (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions (median reported)")
    ap.add_argument("--workload", default="3d_1024x1024x256_ra1e9")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM counters)")
    ap.add_argument("--rows", type=int, nargs=2, default=None,
                    help="rows per wave for the x and z sweeps (default: library choice)")
    ap.add_argument("--adjoint-steps", type=int, default=0,
                    help="adjoint workload: steps per gradient instead of the workload's "
                         "(for profiling runs; the reported value is then of that shorter run)")
    ap.add_argument("--batch-rows", default=None,
                    help='batch: rows per wave per box size as JSON, e.g. '
                         '\'{"128x32": [4, 32], ...}\' (default: run the autotuner)')
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import statistics

    import torch
    import paper_2411_10372_amd as mtvd
    from paper_2411_10372_amd.workloads import WORKLOADS, params_dict

    wl = WORKLOADS[args.workload]
    if not args.steps:
        args.steps = wl.get("steps", 100)
    if "boxes" in wl:
        return bench_batch(args)
    if "adjoint_every" in wl:
        return bench_adjoint(args)
    kw = params_dict(args.workload)
    p = mtvd.Params(**kw)
    diag_every = wl.get("diag_every", 0)
    K, W, R = args.steps, args.warmup, max(1, args.reps)
    nodes = p.nodes
    sweeps = 6 if p.ndim == 3 else 4

    torch.cuda.set_device(0)
    copy_gbs = copy_bandwidth()
    s = mtvd.Solver(p, device="cuda:0")
    if args.rows:
        s.set_tiling(*args.rows)
    s.init_state()
    s.step(W)
    s.sync()
    torch.cuda.synchronize()

    # timed region: R repetitions of K steps, each bracketed by device
    # synchronisations; diagnostics every diag_every steps where the
    # workload asks for them (they synchronise with the host, as a
    # production run would)
    log(f"timing {R} x {K} steps of {args.workload} ({nodes} nodes)")
    reps, done = [], 0
    for _ in range(R):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = 0
        while k < K:
            n = K - k
            if diag_every:
                n = min(n, diag_every - done % diag_every)
            s.step(n)
            k += n
            done += n
            if diag_every and done % diag_every == 0:
                s.diagnostics()
        s.sync()
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
    t_med = statistics.median(reps)

    value_no_diag = None
    if diag_every:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(K)
        s.sync()
        torch.cuda.synchronize()
        value_no_diag = nodes * K / (time.perf_counter() - t0)

    # and again with HIP events around every sweep launch on the library's
    # stream (per-kernel durations for the roofline; the events themselves
    # cost time between launches, so this pass is not used for `value`)
    s.set_timing(True)
    s.step(K)
    s.sync()
    s.set_timing(False)
    ms, cnt = s.kernel_times()
    dfin = s.diagnostics()

    kern = {AXES[a]: {"avg_us": 1e3 * ms[a] / cnt[a], "launches": cnt[a]}
            for a in range(3) if cnt[a]}
    dom = max(range(3), key=lambda a: ms[a])
    per_launch_bytes = nodes * 2 * p.nf * 8      # read + write every field once
    avg_s = 1e-3 * ms[dom] / cnt[dom]
    achieved = per_launch_bytes / avg_s / 1e9
    shash = source_hash(KERNEL_SOURCES[p.ndim])
    traffic = load_traffic(args.workload, AXES[dom], shash)
    value = nodes * K / t_med
    step_bytes_sweep = sweeps * 2 * p.nf * 8     # per cell-update, per-sweep model
    step_bytes_floor = 2 * p.nf * 8              # per cell-update, one pass per step
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * t_med / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded initial state generated on the GPU)",
        "config": {"workload": args.workload, "ndim": p.ndim, "nx": p.nx, "ny": p.ny,
                   "nz": p.nz, "Ra": p.Ra, "Pr": p.Pr, "gamma": p.gamma, "eps": p.eps,
                   "D": p.D, "cfl": p.cfl, "stretch": p.stretch, "diag_every": diag_every},
        "roofline": {"bound": "hbm", "kernel": AXES[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": per_launch_bytes,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "repetitions_s": reps,
        "step_roofline": {
            "per_sweep_model_frac": value * step_bytes_sweep / 1e9 / HBM_PEAK_GBS,
            "floor_model_frac": value * step_bytes_floor / 1e9 / HBM_PEAK_GBS,
            "per_sweep_model_frac_of_copy": value * step_bytes_sweep / 1e9 / copy_gbs,
            "bytes_per_cell_update": {"per_sweep": step_bytes_sweep, "floor": step_bytes_floor}},
        "kernels": kern,
        "final": {"step": dfin["step"], "time": dfin["time"], "mass": dfin["mass"],
                  "nu_mean": dfin["nu_mean"], "nu_bulk": dfin["nu_bulk"]},
        "source_hash": shash,
    }
    if value_no_diag is not None:
        out["value_no_diag"] = value_no_diag
    if args.copy_ref:
        out["copy_ref_bytes"] = copy_ref()
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(kw, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
