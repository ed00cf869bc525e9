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
#  - k_chunk_trees: the same trees with the queue, counts and queue-order
#    heights in LDS: read the donor mask and h, write h (1 + 8 + 8 B per
#    crossing-tree cell; +8 per K or U field read).
ALG_BYTES_STEP = 65
ALG_BYTES_TILE = 17
ALG_BYTES_GLOBAL = 55
ALG_BYTES_CHUNK = 17
ALG_BYTES_FIELD = 8


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm-traffic-plain-10000x10000.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1803_02977_amd", "csrc", "lem_kernels.hip")


def _profile_block(path):
    """The JSON block of a committed counter summary, or None when the kernel
    source has changed since the counters were taken (the summary records
    the source's SHA-256)."""
    import hashlib
    try:
        text = open(path).read()
        data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, IndexError, ValueError):
        return None
    return data if data.get("source_sha256") == digest else None


MFD_PROFILE = os.path.join(ROOT, "profiles", "k_mfd_levels-mfd-10000x10000.md")
BATCH_PROFILE = os.path.join(ROOT, "profiles", "k_grid_levels-batch-512-realizations.md")


def measured_traffic(kernel, path=TRAFFIC_PROFILE):
    """HBM bytes per launch of `kernel` from a committed FETCH_SIZE /
    WRITE_SIZE summary, or None (see _profile_block)."""
    data = _profile_block(path)
    return data.get("bytes_per_launch", {}).get(kernel) if data else None


SQ_PROFILE = os.path.join(ROOT, "profiles", "k_tile_step-sq-counters-plain-10000x10000.md")
# Issue peak of wave64 VALU instructions: 256 CUs x 4 SIMDs, one instruction
# per 4 cycles each (16 lanes), 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def measured_valu(kernel):
    """VALU wave-instructions per launch of `kernel` from the committed
    instruction-counter summary, or None (see _profile_block)."""
    data = _profile_block(SQ_PROFILE)
    return data.get("valu_wave_instructions_per_launch", {}).get(kernel) if data else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=W.LARGE_10000.name,
                    choices=sorted(W.WORKLOADS) + [BATCH_NAME, SWEEP_NAME, WARM_NAME, NET_NAME,
                                                   MFD_NAME])
    ap.add_argument("--grids", type=int, default=100, help="held-out grids (warm-start workload)")
    ap.add_argument("--plain-sample", type=int, default=10,
                    help="warm-start workload: realizations timed through the plain solver")
    ap.add_argument("--streams", type=int, default=4,
                    help="batch workload: also run the realizations as this many batches on "
                         "their own HIP streams, concurrently (0 or 1: one batch only)")
    ap.add_argument("--stream-split", choices=("deal", "size"), default="size",
                    help="batch workload with --streams: deal the realizations round robin by "
                         "size, or group them by size")
    ap.add_argument("--level-pass", type=int, default=0,
                    help="batch workload: 0 automatic, 1 one device-wide pass, 2 one workgroup "
                         "per grid")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch workload: skip the grid-by-grid comparison (counter runs)")
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of the K steps (each from the same initial heights); "
                         "the median is reported")
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip the timed 2 GiB device-to-device copy (achievable HBM GB/s)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the serial oracle over the full length of the 256x256 and "
                         "2048x2048 workloads (and, with --workload plain-10000x10000-fp64, "
                         "over its 50 steps) instead of running the GPU benchmark")
    return ap.parse_args()


BATCH_NAME = "batch-512-realizations-fp64"
SWEEP_NAME = "size-sweep-100-16000"
WARM_NAME = "warmstart-100x256x256-fp64"
NET_NAME = "warmstart-network-b16-256x256-bf16"
MFD_NAME = "mfd-10000x10000-fp64"
# Algorithmic bytes per cell-update of a multiple-flow-direction step:
# routing (k_mfd_route: read h, write the one-byte receiver counter and the
# weight sum: 17 B), then k_mfd_levels: levels (queue read and append,
# counter update, h: 18 B), areas (queue, h, donors' weight sums and areas,
# area write: 36 B), erosion (queue, h, weight sum, area, new height written
# and read as a receiver's: 44 B).
ALG_BYTES_MFD_ROUTE = 17
ALG_BYTES_MFD_LEVELS = 98
# Square edge lengths of the size sweep; the regions (upper edge length)
# follow the GPU scaling table of the paper (section on GPU performance),
# whose wall-time exponents x (wall ~ N^x) are quoted beside the fit.
SWEEP_EDGES = (100, 141, 200, 283, 400, 500, 632, 800, 1000, 1250, 1581, 2000, 2500, 3536,
               5000, 7071, 10000, 12649, 16000)
SWEEP_REGIONS = (("A", 100, 400, 0.33), ("B", 400, 1000, 0.16), ("C", 1000, 2500, 0.42),
                 ("D", 2500, 16000, 0.92))


def _batch_tuning(args):
    """The tuned launch settings for a batch of this size (tuning.json), with
    the level pass forced by --level-pass when it is given."""
    from paper_1803_02977_amd import tune
    t = tune.lookup(sum(r.ny * r.nx for r in W.batch_realizations(512)), batch=True) or {}
    if args.level_pass:
        t = {**t, "level_pass": args.level_pass}
        if args.level_pass == 1:
            t["level_threads"] = 0
    return t


def run_streams(args, reals, steps, h_ref, tuning):
    """The same realizations as `args.streams` batches (sizes dealt round
    robin, largest first, or grouped by size), each with its own context on
    its own HIP stream, run concurrently: while one batch's level pass keeps a
    few CUs busy with its deepest grids, the others' tile passes could fill
    the rest.  Every grid must end bit-identical to the one-batch run
    (`h_ref`)."""
    import torch

    from paper_1803_02977_amd import Batch
    dev = h_ref.device
    k = args.streams
    offs = np.cumsum([0] + [r.ny * r.nx for r in reals])
    order = sorted(range(len(reals)), key=lambda i: -reals[i].ny * reals[i].nx)
    if args.stream_split == "deal":
        groups = [order[j::k] for j in range(k)]
    else:  # contiguous by size: the largest grids together, the smallest together
        groups = [order[j * len(order) // k:(j + 1) * len(order) // k] for j in range(k)]
    runs = []
    for g in groups:
        st = torch.cuda.Stream(device=dev)
        rs = [reals[i] for i in g]
        hg0 = torch.from_numpy(W.batch_initial_heights(rs)).to(dev)
        b = Batch(rs, device=dev, stream=st, tuning=None)
        b.set_tuning(**tuning)  # the one batch's setting
        runs.append((b, st, hg0, hg0.clone(), g))
    if args.warmup > 0:
        for b, st, hg0, hg, g in runs:
            b.run(hg, args.warmup)
        torch.cuda.synchronize()
    for b, st, hg0, hg, g in runs:
        hg.copy_(hg0)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    start.record(runs[0][1])
    ends = []
    t0 = time.perf_counter()
    for b, st, hg0, hg, g in runs:
        if st is not runs[0][1]:
            st.wait_event(start)
        b.run(hg, steps)
        e = torch.cuda.Event(enable_timing=True)
        e.record(st)
        ends.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = max(start.elapsed_time(e) for e in ends)
    equal = True
    for b, st, hg0, hg, g in runs:
        o = 0
        for i in g:
            n = reals[i].ny * reals[i].nx
            equal &= bool(torch.equal(hg[o:o + n], h_ref[offs[i]:offs[i] + n]))
            o += n
        b.close()
    cells = int(offs[-1])
    return {"streams": k, "value": cells * steps / (ms / 1e3), "ms_per_step": ms / steps,
            "wall_s": wall, "bit_identical_to_one_batch": equal,
            "batch_cells": [int(sum(reals[i].ny * reals[i].nx for i in g)) for g in groups]}


def bench_batch(args):
    """512 independent realizations (sizes 128..1024, per-realization K, U, m)
    advanced together for 500 steps; compared with the same grids run one by
    one through the single-grid path on the same GPU."""
    import torch

    from paper_1803_02977_amd import LEM_F_PHASE_TIMERS, LEM_F_TILE_CLOCKS, Batch, Solver
    reals = W.batch_realizations(512, seed=args.seed)
    steps = args.steps or 500
    dev = torch.device("cuda:0")
    h0 = torch.from_numpy(W.batch_initial_heights(reals)).to(dev)
    h = h0.clone()
    b = Batch(reals, device=dev)
    applied = b.set_tuning(**_batch_tuning(args))
    mode = applied["level_pass"]
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
    # Kernel times with the library's HIP events on its stream: a second run
    # of the same steps with phase timers (slower by one sync per step).
    bt = Batch(reals, flags=LEM_F_PHASE_TIMERS, device=dev)
    bt.set_tuning(**_batch_tuning(args))
    h.copy_(h0)
    bt.run(h, steps)
    bt.sync()
    stt = bt.stats()
    bt.close()
    # Device clocks per phase inside every tile workgroup (a run of its own).
    bc = Batch(reals, flags=LEM_F_TILE_CLOCKS, device=dev)
    bc.set_tuning(**_batch_tuning(args))
    h.copy_(h0)
    bc.run(h, steps)
    bc.sync()
    tile_phase_ms = list(bc.stats().tile_phase_ms)
    bc.close()
    tile_ms = stt.kernel_ms[0] / steps
    chunk_ms = stt.kernel_ms[2] / steps
    level_ms = (stt.kernel_ms[1] - stt.kernel_ms[2]) / steps
    cross = stt.crossing_run / steps
    streams = run_streams(args, reals, steps, h, applied) if args.streams > 1 else None
    level_name = "k_grid_levels" if mode == 2 else "k_global_levels"
    if level_ms >= max(tile_ms, chunk_ms):
        roof = {"bound": "hbm", "kernel": level_name,
                "achieved": ALG_BYTES_GLOBAL * cross / (level_ms * 1e-3) / 1e9,
                "alg_bytes": f"{ALG_BYTES_GLOBAL} B per crossing-tree cell",
                "avg_launch_ms": level_ms}
    elif chunk_ms >= tile_ms:
        roof = {"bound": "hbm", "kernel": "k_chunk_trees",
                "achieved": ALG_BYTES_CHUNK * cross / (chunk_ms * 1e-3) / 1e9,
                "alg_bytes": f"{ALG_BYTES_CHUNK} B per crossing-tree cell",
                "avg_launch_ms": chunk_ms}
    else:
        roof = {"bound": "hbm", "kernel": "k_tile_step",
                "achieved": ALG_BYTES_TILE * cells / (tile_ms * 1e-3) / 1e9,
                "alg_bytes": f"{ALG_BYTES_TILE} B per cell", "avg_launch_ms": tile_ms}
    roof.update(peak=HBM_PEAK_GBS, unit="GB/s", frac=roof["achieved"] / HBM_PEAK_GBS,
                traffic=measured_traffic(roof["kernel"], BATCH_PROFILE)
                if args.seed == 0 else None)
    one_value = None
    if not args.no_compare:
        # The same grids one at a time through the single-grid path (fewer steps).
        one_steps = max(1, min(steps, 20))
        solvers = [Solver(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, r.U, r.K, device=dev)
                   for r in reals]
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
    # The faster schedule is the workload's figure (both give the same bits).
    one_batch = {"value": value, "ms_per_step": ms / steps}
    schedule = "one batch"
    if streams and streams["bit_identical_to_one_batch"] and streams["value"] > value:
        value, ms = streams["value"], streams["ms_per_step"] * steps
        schedule = f"{streams['streams']} concurrent batches on their own streams"
    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": ms / steps,
        "schedule": schedule, "one_batch": one_batch,
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
                                 "one after another on the same GPU"} if one_value else None,
        "batch_speedup_vs_grid_by_grid": round(value / one_value, 2) if one_value else None,
        "level_pass": "one workgroup per grid" if mode == 2 else "one device-wide pass",
        "kernel_ms_per_step": {"k_tile_step": tile_ms, "k_chunk_trees": chunk_ms,
                               level_name: level_ms},
        # Device clock of a tile workgroup, mean over workgroups, per phase.
        "tile_wg_phase_us_per_step": {
            k: round(tile_phase_ms[i] / steps * 1e3, 3)
            for i, k in enumerate(("stage", "receivers", "donors_walks", "clean",
                                   "erosion", "writeback"))},
        "levels_max": int(stt.max_nlevels),
        "concurrent_batches": streams,
        # Crossing-tree phases by the device clock (per-grid level pass: the
        # longest workgroup of each phase, per step).
        "crossing_phase_ms_per_step": {"order": stt.phase_ms[1] / steps,
                                       "accumulate": stt.phase_ms[2] / steps,
                                       "erode": stt.phase_ms[3] / steps},
        "tuning": applied,
        "roofline": roof,
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


def _network_throughput(net, dev, side, steps=20):
    """Forward pass and training step (forward, backward, Adam) of the
    warm-start network at its context's batch, timed with HIP events on its
    stream; FLOPs count the fourteen 3x3 convolutions (2 per multiply-add),
    the backward pass twice the forward minus the skipped input gradient of
    the first layer."""
    import torch

    from paper_1803_02977_amd import warmstart as WS
    from paper_1803_02977_amd.surrogate import layer
    B = net.batch
    levels = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0]
    fwd = sum(2.0 * B * (side >> lv) ** 2 * 9 * layer(i)[0] * layer(i)[1]
              for i, lv in enumerate(levels))
    bwd = 2 * fwd - 2.0 * B * side * side * 9 * layer(0)[0] * layer(0)[1]
    K, U, h0 = WS.make_dataset(B, W.WARMSTART_TEST_SEED, dev)
    tgt = h0 * 100.0
    stream = net.stream
    for _ in range(3):
        net.train_step(K, U, h0, tgt, lr=1e-6, want_loss=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        net.predict(K, U, h0)
    e1.record(stream)
    net.sync()
    ms_fwd = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        net.train_step(K, U, h0, tgt, lr=1e-6, want_loss=False)
    e1.record(stream)
    net.sync()
    ms_train = e0.elapsed_time(e1) / steps
    return {"batch": B, "forward_ms": ms_fwd, "train_step_ms": ms_train, "fwd_flop": fwd,
            "bwd_flop": bwd}


def bench_mfd(args):
    """Multiple-flow-direction routing on the 10000 x 10000 workload (same
    grid, parameters and initial heights as the default benchmark, flow
    shared in proportion to the slope)."""
    import torch

    from paper_1803_02977_amd import LEM_F_PHASE_TIMERS, MfdSolver
    w = W.LARGE_10000
    steps = args.steps or 10
    dev = torch.device("cuda:0")
    h0 = torch.from_numpy(W.initial_heights(w.ny, w.nx, args.seed)).to(dev)
    h = h0.clone()
    s = MfdSolver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev)
    if args.warmup > 0:
        s.run(h, args.warmup)
        s.sync()
    h.copy_(h0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(h, steps)
    e1.record(s.stream)
    s.sync()
    ms = e0.elapsed_time(e1)
    nl = s.export()["nlevels"]
    s.close()
    # Phase timers synchronise after every step: a run of its own, not the timed one.
    st = MfdSolver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, flags=LEM_F_PHASE_TIMERS,
                   device=dev)
    h.copy_(h0)
    st.run(h, steps)
    st.sync()
    stats = st.stats()
    route_ms, levels_ms = stats.kernel_ms[0] / steps, stats.kernel_ms[1] / steps
    phases = {"levels": stats.phase_ms[1] / steps, "areas": stats.phase_ms[2] / steps,
              "erosion": stats.phase_ms[3] / steps}
    st.close()
    cells = w.cells
    achieved = ALG_BYTES_MFD_LEVELS * cells / (levels_ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu:
        import oracle
        side, csteps = 2048, 3
        hc = W.initial_heights(side, side, args.seed)
        p = oracle.Params(side, side, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K)
        t0 = time.perf_counter()
        oracle.mfd_run(hc, p, csteps)
        dt = time.perf_counter() - t0
        cpu = {"value": side * side * csteps / dt, "unit": "cell-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{csteps} steps of a {side}x{side} grid with the same parameters, "
                         f"serial C oracle (cells in height order), {dt:.2f} s"}
    print(json.dumps({
        "metric": "cell-updates/s", "value": cells * steps / (ms * 1e-3),
        "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": MFD_NAME, "ny": w.ny, "nx": w.nx, "dx": w.dx, "dt": w.dt,
                   "m": w.m, "U": w.U, "K": w.K, "exponent": 1.0, "seed": args.seed},
        "levels": nl,
        "roofline": {"bound": "hbm", "kernel": "k_mfd_levels", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_mfd_levels", MFD_PROFILE)
                     if args.seed == 0 else None,
                     "alg_bytes": f"{ALG_BYTES_MFD_LEVELS} B per cell",
                     "avg_launch_ms": levels_ms},
        "kernel_ms_per_step": {"k_mfd_route": route_ms, "k_mfd_levels": levels_ms},
        "levels_kernel_phase_ms_per_step": phases,
        "cpu_baseline": cpu}), flush=True)


def bench_network(args):
    """The warm-start network alone: training steps and forward passes at
    batch 16 on 256 x 256 inputs (the convolutions run on MFMA)."""
    import torch

    from paper_1803_02977_amd import warmstart as WS
    from paper_1803_02977_amd.surrogate import Surrogate, load_params
    dev = torch.device("cuda:0")
    side = W.WARMSTART_SIDE
    net = Surrogate(16, side, side, device=dev)
    net.set_params(load_params(WS.WEIGHTS_PATH))
    nt = _network_throughput(net, dev, side, steps=args.steps or 20)
    net.close()
    train_tf = (nt["fwd_flop"] + nt["bwd_flop"]) / (nt["train_step_ms"] * 1e-3) / 1e12
    fwd_tf = nt["fwd_flop"] / (nt["forward_ms"] * 1e-3) / 1e12
    print(json.dumps({
        "metric": "conv TFLOP/s (training step)", "value": train_tf, "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps or 20, "warmup": 3, "ms_per_step": nt["train_step_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": NET_NAME, "batch": 16, "side": side},
        "forward_ms": nt["forward_ms"], "forward_tflops": fwd_tf,
        "conv_gflop": {"forward": nt["fwd_flop"] / 1e9, "backward": nt["bwd_flop"] / 1e9},
        "roofline": {"bound": "mfma", "achieved": fwd_tf, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": fwd_tf / 2500.0, "traffic": None,
                     "kernel": "k_conv3x3 (forward pass, all fourteen convolutions)"},
        "cpu_baseline": None}), flush=True)


def bench_warmstart(args):
    """Time to steady state (no cell changing by more than 1e-6 of its
    grid's largest height in one step, dt = 1000 yr) of held-out 256 x 256
    realizations, as one batch, from the noise surface (cold) and from the
    network's prediction (warm start, prediction time included), each by the
    method's steps alone and by steady-state projections then steps; against
    the plain solver (single-grid steps from the noise surface, grid after
    grid); plus the network's own throughput: a training step (forward,
    backward, Adam) and a forward pass at batch 16, whose convolutions run on
    MFMA.  The reported value is the warm start with projections."""
    import torch

    from paper_1803_02977_amd import warmstart as WS
    from paper_1803_02977_amd.surrogate import Surrogate, layer, load_params
    dev = torch.device("cuda:0")
    side = W.WARMSTART_SIDE
    net = Surrogate(16, side, side, device=dev)
    net.set_params(load_params(WS.WEIGHTS_PATH))
    r = WS.evaluate(net, args.grids, batch=16, chunk=2000, plain_sample=args.plain_sample,
                    project=True)
    plain_s = r["plain"]["s_per_realization"] * args.grids
    pc, pw = r["projected"]["cold"], r["projected"]["warm"]
    # Network throughput (training changes the parameters, so it runs after
    # the evaluation).
    nt = _network_throughput(net, dev, side)
    net.close()
    ms_fwd, ms_train, fwd, bwd = nt["forward_ms"], nt["train_step_ms"], nt["fwd_flop"], nt["bwd_flop"]
    B = nt["batch"]
    fwd_tflops = fwd / (ms_fwd * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        import oracle
        Kc, Uc, hc = W.warmstart_inputs(1, W.WARMSTART_TEST_SEED)
        p = oracle.Params(side, side, WS.DX, WS.DX, WS.DT, WS.M, 1.0, float(Uc[0, 0, 0]), 1e-5)
        steps = args.cpu_steps or 300
        t0 = time.perf_counter()
        oracle.run(hc[0], p, steps, K=Kc[0], U=Uc[0])
        dt = time.perf_counter() - t0
        cpu = {"value": side * side * steps / dt, "unit": "cell-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{steps} cold-start steps of held-out realization 0 ({side}x{side}, "
                         f"K and U fields), serial C oracle, {dt:.2f} s; the cold runs above "
                         f"take {r['cold_steps_mean']:.0f} steps per grid on average"}
    print(json.dumps({
        "metric": "time to steady state", "value": pw["s"], "unit": "s",
        "n_gpus": 1, "steps": int(round(pw["projections_mean"] * args.grids)), "warmup": 0,
        "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 solver, bf16/f32 network", "data": "synthetic",
        "config": {"workload": WARM_NAME, "grids": args.grids, "side": side, "dt": WS.DT,
                   "rtol": WS.RTOL, "K": "lognormal per cell, median 1e-5, sigma_ln 0.5",
                   "U": "Uniform[1e-4,2e-3] per grid", "m": WS.M, "dx": WS.DX,
                   "seeds": f"{W.WARMSTART_TEST_SEED}+ (held out)"},
        "plain_solver_s": plain_s, "speedup_vs_plain": plain_s / pw["s"],
        "batched_s": {"cold_steps": r["cold_s"], "warm_steps": r["warm_s"],
                      "cold_projections_then_steps": pc["s"],
                      "warm_projections_then_steps": pw["s"]},
        "projections": {"cold": {k: pc[k] for k in ("projections_mean", "projections_max",
                                                    "steps_after_max", "project_s", "steps_s")},
                        "warm": {k: pw[k] for k in ("projections_mean", "projections_max",
                                                    "steps_after_max", "project_s", "steps_s")},
                        "steady_rel_l2_vs_cold_steps": {"cold": pc["rel_l2_vs_cold_steady"],
                                                        "warm": pw["rel_l2_vs_cold_steady"]}},
        "warm_over_cold_time": {"steps": r["warm_s"] / r["cold_s"],
                                "projections_then_steps": pw["s"] / pc["s"]},
        "plain_solver": {"s_per_realization": r["plain"]["s_per_realization"],
                         "sample": f"first {args.plain_sample} realizations from the noise "
                                   "surface, one after another through the single-grid path "
                                   f"(a batch of one), scaled to {args.grids}",
                         "steps_equal_batched": r["plain"]["steps_match_batch"]},
        "batched_cold_s": r["cold_s"], "batched_warm_s": r["warm_s"],
        "surrogate_speedup_in_batch": r["cold_s"] / r["warm_s"],
        "steps_mean": {"cold": r["cold_steps_mean"], "warm": r["warm_steps_mean"]},
        "steps_pct_10_50_90_100": {"cold": r["cold_steps_pct"], "warm": r["warm_steps_pct"]},
        "steps_ratio_warm_over_cold": r["steps_ratio_warm_over_cold"],
        "warm_fewer_steps_frac": r["warm_fewer_steps_frac"],
        "all_converged": r["all_converged"], "predict_s": r["predict_s"],
        "prediction_rel_l2_vs_cold_steady": r["prediction_rel_l2_vs_cold_steady"],
        "noise_rel_l2_vs_cold_steady": r["noise_rel_l2_vs_cold_steady"],
        "network": {"batch": B, "forward_ms": ms_fwd, "train_step_ms": ms_train,
                    "conv_gflop_forward": fwd / 1e9,
                    "train_tflops": (fwd + bwd) / (ms_train * 1e-3) / 1e12},
        "roofline": {"bound": "mfma", "achieved": fwd_tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": fwd_tflops / 2500.0, "traffic": None,
                     "kernel": "k_conv3x3 (forward pass, all fourteen convolutions)"},
        "cpu_baseline": cpu}), flush=True)


def host_cpu():
    """Model name of the host CPU and the number of online cores."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, h0, K, steps):
    """The serial oracle (one host thread) on ``steps`` steps of the workload."""
    import oracle
    p = oracle.Params(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K)
    t = time.perf_counter()
    oracle.run(h0, p, steps, K=K)
    dt = time.perf_counter() - t
    model, nproc = host_cpu()
    return dict(value=w.cells * steps / dt, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{steps} of the {w.steps} step(s) of the full {w.ny}x{w.nx} grid from "
                       f"its initial heights, serial C oracle, {dt:.2f} s",
                cpu_model=model, nproc=nproc, seconds=round(dt, 2), steps=steps)


def cpu_full(args):
    """The serial oracle over whole workloads (one JSON line each).  The steps
    run in segments of about 30 s, each continuing from the last one's
    heights (the same result as one call), with a progress line after each."""
    import oracle
    names = [W.SMALL_256.name, W.MEDIUM_2048.name]
    if args.workload == W.LARGE_10000.name:
        names.append(W.LARGE_10000.name)
    model, nproc = host_cpu()
    for name in names:
        w = W.WORKLOADS[name]
        h, K, _ = W.make_inputs(w, args.seed)
        p = oracle.Params(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K)
        seg = max(1, int(30 * 1.5e7 // w.cells))
        done, total = 0, 0.0
        while done < w.steps:
            k = min(seg, w.steps - done)
            t = time.perf_counter()
            h = oracle.run(h, p, k, K=K)["h"]
            total += time.perf_counter() - t
            done += k
            print(f"[cpu-full] {name}: {done}/{w.steps} steps, {total:.1f} s", file=sys.stderr,
                  flush=True)
        r = dict(workload=name, value=w.cells * w.steps / total, unit="cell-updates/s", cores=1,
                 kind="oracle", steps=w.steps, seconds=round(total, 2),
                 seconds_per_step=round(total / w.steps, 4), cpu_model=model, nproc=nproc,
                 sample=f"all {w.steps} steps of the {w.ny}x{w.nx} grid, serial C oracle")
        print(json.dumps(r), flush=True)


def copy_probe(dev, reps=5):
    """Achievable HBM bandwidth on this GPU: a plain 2 GiB device-to-device
    copy (2 GiB read + 2 GiB written), median of ``reps`` timed copies."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    nbytes = 2 * src.numel() * 8
    del src, dst
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    med = float(np.median(times))
    return {"bytes_per_copy": nbytes, "ms_median": round(med, 4),
            "gbs": round(nbytes / (med * 1e-3) / 1e9, 1),
            "note": "torch copy_ of 2 GiB float64 on the GPU (read + write counted)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); sharding over "
              "several GPUs is designed (row strips, boundary graphs) but not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.cpu_full:
        cpu_full(args)
        return
    if args.workload == BATCH_NAME:
        bench_batch(args)
        return
    if args.workload == SWEEP_NAME:
        bench_sweep(args)
        return
    if args.workload == WARM_NAME:
        bench_warmstart(args)
        return
    if args.workload == NET_NAME:
        bench_network(args)
        return
    if args.workload == MFD_NAME:
        bench_mfd(args)
        return
    import torch

    from paper_1803_02977_amd import LEM_F_PHASE_TIMERS, LEM_F_TILE_CLOCKS, Solver

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
    runs = []
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
        runs.append((ev0.elapsed_time(ev1), time.perf_counter() - t0))
    runs.sort()
    ms, wall = runs[len(runs) // 2]  # the median run (the middle one for an odd count)
    run_ms = [r[0] / steps for r in runs]
    levels = solver.level_history(steps)
    # Level-size histogram of the last timed step (cells per level of Alg 3,
    # whole grid: trees inside a tile and crossing trees together).
    offsets = solver.routing()["offsets"]
    level_sizes = np.diff(np.asarray(offsets, dtype=np.int64)).tolist()
    from paper_1803_02977_amd import lem as L
    tq = L.lem_get_tuning(solver.ctx)
    applied = {name: getattr(tq, name) for name, _ in L.lem_tuning._fields_}
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
    # Device clocks per phase inside every tile workgroup: a run of its own,
    # since they slow the tile pass that the run above times.
    h.copy_(h0)
    csolver = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev,
                     flags=LEM_F_TILE_CLOCKS)
    csolver.run(h, steps, K=Kt)
    csolver.sync()
    tile_phase_ms = list(csolver.stats().tile_phase_ms)
    csolver.close()
    tile_ms = st.kernel_ms[0] / steps
    chunk_ms = st.kernel_ms[2] / steps
    global_ms = (st.kernel_ms[1] - st.kernel_ms[2]) / steps
    crossing = tsolver_crossing
    # The level pass after the chunk stage: device-wide, or one workgroup per grid.
    level_name = "k_grid_levels" if applied["level_pass"] == 2 else "k_global_levels"

    cells = w.cells
    value = cells * steps / (ms / 1e3)
    fields = (Kt is not None)
    alg_step = ALG_BYTES_STEP + ALG_BYTES_FIELD * fields
    alg_tile = ALG_BYTES_TILE + ALG_BYTES_FIELD * fields
    if tile_ms >= max(global_ms, chunk_ms):
        kname, kms, kbytes = "k_tile_step", tile_ms, alg_tile * cells
        per_unit = f"{alg_tile} B per cell"
    elif chunk_ms >= global_ms:
        alg_chunk = ALG_BYTES_CHUNK + ALG_BYTES_FIELD * fields
        kname, kms, kbytes = "k_chunk_trees", chunk_ms, alg_chunk * crossing
        per_unit = f"{alg_chunk} B per crossing-tree cell"
    else:
        kname, kms, kbytes = level_name, global_ms, ALG_BYTES_GLOBAL * crossing
        per_unit = f"{ALG_BYTES_GLOBAL} B per crossing-tree cell"
    achieved = kbytes / (kms / 1e3) / 1e9
    roofline = dict(bound="hbm", kernel=kname, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(kname) if w.name == W.LARGE_10000.name else None,
                    alg_bytes=per_unit, avg_launch_ms=round(kms, 4))
    valu = measured_valu(kname) if w.name == W.LARGE_10000.name else None
    if valu:
        # The tile kernel is bound by instruction issue more than by HBM: the
        # counted VALU instructions over the live launch time, against the peak.
        rate = valu / (kms / 1e3)
        roofline["valu_issue"] = {"wave_instructions_per_launch": valu,
                                  "achieved_per_s": round(rate, -6),
                                  "peak_per_s": VALU_ISSUE_PEAK,
                                  "frac": round(rate / VALU_ISSUE_PEAK, 4)}
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
        "repeats": {"count": len(runs), "reported": "median",
                    "ms_per_step_min_median_max": [round(run_ms[0], 4),
                                                   round(run_ms[len(run_ms) // 2], 4),
                                                   round(run_ms[-1], 4)]},
        "wall_s": wall,
        "levels": {"min": int(levels.min()), "max": int(levels.max()),
                   "mean": float(levels.mean()), "per_step": [int(x) for x in levels],
                   "last_step_level_sizes": level_sizes} if len(levels) else None,
        "kernel_ms_per_step": {"k_tile_step": tile_ms, "k_chunk_trees": chunk_ms,
                               level_name: global_ms},
        # Device clock of the first workgroup of the crossing-tree work (the
        # chunk stage's when it runs): its time in each phase per step.
        "crossing_wg0_phase_ms_per_step": {"order": st.phase_ms[1] / steps,
                                           "accumulate": st.phase_ms[2] / steps,
                                           "erode": st.phase_ms[3] / steps},
        # Device clock of a tile workgroup, mean over workgroups, per phase.
        "tile_wg_phase_us_per_step": {
            k: round(tile_phase_ms[i] / steps * 1e3, 3)
            for i, k in enumerate(("stage", "receivers", "donors_walks", "clean",
                                   "erosion", "writeback"))},
        "tuning": applied,
        "crossing_cells_per_step": crossing,
        "crossing_frac": round(crossing / cells, 4),
    }
    roofline["frac_whole_step_65B"] = out["hbm_roofline_frac_65B"]
    if not args.no_copy_probe:
        del h, h0, Kt
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        probe = copy_probe(dev)
        out["copy_probe"] = probe
        roofline["frac_of_copy_probe"] = round(achieved / probe["gbs"], 4)
    if not args.no_cpu:
        cpu_steps = args.cpu_steps or (2 if cells >= 10 ** 8 else max(1, min(steps, int(2e8 // cells))))
        out["cpu_baseline"] = cpu_baseline(w, h0_np, K_np, cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def release_gpu():
    """Frees what the run still holds on the GPU before the interpreter exits:
    every library context is closed where it was used; this drops the last
    tensors and torch's cached blocks so that nothing is torn down by
    finalizers after a profiler has detached."""
    if "torch" not in sys.modules:
        return
    import gc

    import torch
    gc.collect()
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
    release_gpu()
