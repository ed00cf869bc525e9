"""Benchmark of the landscape-evolution hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one time step of the method (receivers, donors, levels, drainage
area, uplift, erosion) over the whole grid.  The default workload is the
10000 x 10000 FP64 grid (30 m cells, U = 1e-3, K = 2e-5, m = 0.45,
dt = 500 yr) for its 50 steps, from seeded Uniform[0,1) heights already
resident in HBM.  Prints one JSON line with cell-updates/s, the roofline of
the dominant kernel (measured live with HIP events on the library's stream)
and the serial CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

# Algorithmic bytes per cell-update.
#  - The whole step, counted as the level-queue formulation of the method
#    moves it: each per-cell array written once and read once by each
#    consuming phase at its minimal width (h 32 B, receiver code 2, donor
#    mask 3, queue 16, counts 12; +8 per K or U field): 65 B.
#  - k_tile_step (the fused tile pass): read h, write h, write the donor mask
#    (8 + 8 + 1 B; +8 per K or U field read).
#  - k_global_levels: the 65 B formulation minus the receiver sweep's h read
#    and the code/mask writes (55 B), for each cell of a tree that crosses a
#    tile edge.
ALG_BYTES_STEP = 65
ALG_BYTES_TILE = 17
ALG_BYTES_GLOBAL = 55
ALG_BYTES_FIELD = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=W.LARGE_10000.name,
                    choices=sorted(W.WORKLOADS) + [BATCH_NAME, SWEEP_NAME])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--repeats", type=int, default=1)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device-to-device copy of 2 GiB (three times) "
                         "whose HBM counters calibrate FETCH_SIZE and WRITE_SIZE")
    return ap.parse_args()


BATCH_NAME = "batch-512-realizations-fp64"
SWEEP_NAME = "size-sweep-100-16000"
# Square edge lengths of the size sweep; the regions (upper edge length)
# follow the GPU scaling table of the paper (section on GPU performance),
# whose wall-time exponents x (wall ~ N^x) are quoted beside the fit.
SWEEP_EDGES = (100, 141, 200, 283, 400, 500, 632, 800, 1000, 1250, 1581, 2000, 2500, 3536,
               5000, 7071, 10000, 12649, 16000)
SWEEP_REGIONS = (("A", 100, 400, 0.33), ("B", 400, 1000, 0.16), ("C", 1000, 2500, 0.42),
                 ("D", 2500, 16000, 0.92))


def bench_batch(args):
    """512 independent realizations (sizes 128..1024, per-realization K, U, m)
    advanced together for 500 steps; compared with the same grids run one by
    one through the single-grid path on the same GPU."""
    import torch

    from paper_1803_02977_amd import Batch, Solver
    reals = W.batch_realizations(512, seed=args.seed)
    steps = args.steps or 500
    dev = torch.device("cuda:0")
    h0 = torch.from_numpy(W.batch_initial_heights(reals)).to(dev)
    h = h0.clone()
    b = Batch(reals, device=dev)
    if args.warmup > 0:
        b.run(h, args.warmup)
        b.sync()
    h.copy_(h0)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.run(h, steps)
    ev1.record(b.stream)
    b.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    st = b.stats()
    b.close()
    cells = sum(r.ny * r.nx for r in reals)
    value = cells * steps / (ms / 1e3)
    # The same grids one at a time through the single-grid path (fewer steps).
    one_steps = max(1, min(steps, 20))
    solvers = [Solver(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, r.U, r.K, device=dev) for r in reals]
    views = [h0[sum(q.ny * q.nx for q in reals[:i]):][: r.ny * r.nx].clone().view(r.ny, r.nx)
             for i, r in enumerate(reals)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s_, v in zip(solvers, views):
        s_.run(v, one_steps)
    torch.cuda.synchronize()
    one_wall = time.perf_counter() - t1
    for s_ in solvers:
        s_.close()
    one_value = cells * one_steps / one_wall
    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": BATCH_NAME, "realizations": len(reals), "cells": cells,
                   "sizes": "square, uniform over {128,192,...,1024}",
                   "K": "logUniform[1e-6,1e-4]", "U": "Uniform[1e-4,2e-3]",
                   "m": "Uniform[0.35,0.6]", "dt": 1000.0, "dx": 100.0, "seed": args.seed},
        "wall_s": wall,
        "crossing_frac": round(st.crossing_run / steps / cells, 4),
        "grid_by_grid": {"value": one_value, "unit": "cell-updates/s", "steps": one_steps,
                         "note": "same realizations, one single-grid context each, run "
                                 "one after another on the same GPU"},
        "batch_speedup_vs_grid_by_grid": round(value / one_value, 2),
        "roofline": None,
    }
    if not args.no_cpu:
        import oracle
        sample = reals[:3]
        t = time.perf_counter()
        for r in sample:
            p = oracle.Params(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, 1.0, r.U, r.K)
            oracle.run(W.initial_heights(r.ny, r.nx, r.seed), p, 10)
        dt_ = time.perf_counter() - t
        c = sum(r.ny * r.nx for r in sample) * 10
        out["cpu_baseline"] = dict(value=c / dt_, unit="cell-updates/s", cores=1, kind="oracle",
                                   sample=f"10 steps of each of the first 3 realizations "
                                          f"({[r.ny for r in sample]} square), serial C oracle, "
                                          f"{dt_:.2f} s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """Wall time per step against grid size: seeded Uniform[0,1) square
    rasters (100 m cells, U = 5e-4, K = 1e-5, m = 0.5, dt = 1000 yr), the
    same number of steps at every size, and a least-squares fit of
    log(ms per step) against log(cells) in each region."""
    import torch

    from paper_1803_02977_amd import Solver
    dev = torch.device("cuda:0")
    steps = args.steps or 50
    rows = []
    for e in SWEEP_EDGES:
        h0 = torch.from_numpy(W.initial_heights(e, e, args.seed)).to(dev)
        h = h0.clone()
        s = Solver(e, e, 100.0, 100.0, 1000.0, 0.5, 5e-4, 1e-5, device=dev)
        if args.warmup > 0:
            s.run(h, args.warmup)
            s.sync()
        best = None
        for _ in range(max(3, args.repeats)):
            h.copy_(h0)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(s.stream)
            s.run(h, steps)
            ev1.record(s.stream)
            s.sync()
            ms = ev0.elapsed_time(ev1) / steps
            best = ms if best is None else min(best, ms)
        st = s.stats()
        rows.append(dict(edge=e, cells=e * e, ms_per_step=round(best, 5),
                         cell_updates_per_s=e * e / (best * 1e-3),
                         max_levels=int(st.max_nlevels)))
        print(f"[sweep] {e}x{e}: {best:.4f} ms/step, {e * e / (best * 1e-3):.3e} cell-updates/s",
              file=sys.stderr, flush=True)
        s.close()
        del h, h0
        torch.cuda.empty_cache()
    fits = []
    for name, lo, hi, paper_x in SWEEP_REGIONS:
        pts = [(np.log(r["cells"]), np.log(r["ms_per_step"])) for r in rows if lo <= r["edge"] <= hi]
        x = float(np.polyfit([p[0] for p in pts], [p[1] for p in pts], 1)[0]) if len(pts) >= 2 else None
        fits.append(dict(region=name, edge_lo=lo, edge_hi=hi, x=None if x is None else round(x, 3),
                         paper_x=paper_x, points=len(pts)))
    big = rows[-1]
    print(json.dumps({
        "metric": "cell-updates/s", "value": big["cell_updates_per_s"], "unit": "cell-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": big["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": SWEEP_NAME, "edges": list(SWEEP_EDGES), "dx": 100.0, "dt": 1000.0,
                   "m": 0.5, "U": 5e-4, "K": 1e-5, "seed": args.seed},
        "sweep": rows, "fit": fits, "roofline": None, "cpu_baseline": None}), flush=True)


def cpu_baseline(w, h0, K, steps):
    """The serial oracle (one host thread) on ``steps`` steps of the workload."""
    import oracle
    p = oracle.Params(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K)
    t = time.perf_counter()
    oracle.run(h0, p, steps, K=K)
    dt = time.perf_counter() - t
    return dict(value=w.cells * steps / dt, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{steps} step(s) of the full {w.ny}x{w.nx} grid from its initial "
                       f"heights, serial C oracle, {dt:.2f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU sharding design is described but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == BATCH_NAME:
        bench_batch(args)
        return
    if args.workload == SWEEP_NAME:
        bench_sweep(args)
        return
    import torch

    from paper_1803_02977_amd import LEM_F_PHASE_TIMERS, Solver

    w = W.WORKLOADS[args.workload]
    steps = args.steps or w.steps
    dev = torch.device("cuda:0")
    h0_np, K_np, _ = W.make_inputs(w, args.seed)
    h0 = torch.from_numpy(h0_np).to(dev)
    Kt = None if K_np is None else torch.from_numpy(K_np).to(dev)
    h = h0.clone()
    solver = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev)
    stream = solver.stream

    # Warm-up on a copy, then restore the initial heights (not timed).
    if args.warmup > 0:
        solver.run(h, args.warmup, K=Kt)
        solver.sync()
    best = None
    for _ in range(max(1, args.repeats)):
        h.copy_(h0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        solver.run(h, steps, K=Kt)
        ev1.record(stream)
        solver.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        if best is None or ms < best[0]:
            best = (ms, wall)
    ms, wall = best
    levels = solver.level_history(steps)
    solver.close()

    # Per-kernel device time, measured live with HIP events on the library's
    # stream in a separate run with phase timers on (same inputs, same steps).
    h.copy_(h0)
    tsolver = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev,
                     flags=LEM_F_PHASE_TIMERS)
    tsolver.run(h, steps, K=Kt)
    tsolver.sync()
    st = tsolver.stats()
    tsolver_crossing = st.crossing_run / steps
    tsolver.close()
    tile_ms = st.kernel_ms[0] / steps
    global_ms = st.kernel_ms[1] / steps
    crossing = tsolver_crossing

    cells = w.cells
    value = cells * steps / (ms / 1e3)
    fields = (Kt is not None)
    alg_step = ALG_BYTES_STEP + ALG_BYTES_FIELD * fields
    alg_tile = ALG_BYTES_TILE + ALG_BYTES_FIELD * fields
    if tile_ms >= global_ms:
        kname, kms, kbytes = "k_tile_step", tile_ms, alg_tile * cells
        per_unit = f"{alg_tile} B per cell"
    else:
        kname, kms, kbytes = "k_global_levels", global_ms, ALG_BYTES_GLOBAL * crossing
        per_unit = f"{ALG_BYTES_GLOBAL} B per crossing-tree cell"
    achieved = kbytes / (kms / 1e3) / 1e9
    roofline = dict(bound="hbm", kernel=kname, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    alg_bytes=per_unit, avg_launch_ms=round(kms, 4))
    out = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "ny": w.ny, "nx": w.nx, "dx": w.dx, "dt": w.dt,
                   "m": w.m, "n": 1.0, "U": w.U, "K": w.K,
                   "K_field": "lognormal" if Kt is not None else "scalar", "seed": args.seed},
        "roofline": roofline,
        "hbm_roofline_frac_65B": round(value * alg_step / (HBM_PEAK_GBS * 1e9), 4),
        "wall_s": wall,
        "levels": {"min": int(levels.min()), "max": int(levels.max()),
                   "mean": float(levels.mean())} if len(levels) else None,
        "kernel_ms_per_step": {"k_tile_step": tile_ms, "k_global_levels": global_ms},
        "global_phase_ms_per_step": {"order": st.phase_ms[1] / steps,
                                     "accumulate": st.phase_ms[2] / steps,
                                     "erode": st.phase_ms[3] / steps},
        "crossing_cells_per_step": crossing,
        "crossing_frac": round(crossing / cells, 4),
    }
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes_each_way"] = src.numel() * 8
        del src, dst
    if not args.no_cpu:
        cpu_steps = args.cpu_steps or (2 if cells >= 10 ** 8 else max(1, min(steps, int(2e8 // cells))))
        out["cpu_baseline"] = cpu_baseline(w, h0_np, K_np, cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
