"""Launch tuner for the level pass of trees that cross tile edges.

For each grid-size bucket it times candidate settings (workgroups of the
cooperative level kernel, and the level size below which one workgroup works
alone) on a representative synthetic workload and stores the fastest in
``tuning.json`` next to this file.  Settings change only the schedule: the
results are bit-identical for every candidate (a GPU test checks this).

    python -m paper_1803_02977_amd.tune            # tune and write tuning.json

``lookup(cells)`` returns the stored setting for a grid (or batch) of that
many cells; ``Solver`` and ``Batch`` apply it when ``tuning="auto"``.
"""
from __future__ import annotations

import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "tuning.json")

# Buckets by cell count: [lo, hi).
BUCKETS = [(0, 1 << 18), (1 << 18, 1 << 22), (1 << 22, 1 << 25), (1 << 25, 1 << 31)]
# A representative square grid per bucket (side length).
BUCKET_SIDES = [256, 1024, 4096, 10000]
CANDIDATES = [(g, t) for g in (16, 32, 64, 96, 128, 160, 192, 256) for t in (512, 2048, 8192)]


def _bucket(cells: int) -> int:
    for i, (lo, hi) in enumerate(BUCKETS):
        if lo <= cells < hi:
            return i
    return len(BUCKETS) - 1


def load(path: str = TUNING_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def lookup(cells: int, table=None):
    """(global_workgroups, tail_level) for a run of `cells` cells, or None."""
    table = table if table is not None else load()
    if not table:
        return None
    for entry in table.get("buckets", []):
        if entry["lo"] <= cells < entry["hi"]:
            return entry["global_workgroups"], entry["tail_level"]
    return None


def time_candidates(make_runner, steps: int, candidates=CANDIDATES, repeats: int = 3):
    """Times each candidate; make_runner() -> (set_tuning, run(steps), sync,
    level_ms()), level_ms() giving the level kernel's HIP-event milliseconds
    summed over the last run.  Settings only change that kernel's schedule,
    so its own time ranks them (host clocks around whole steps proved too
    noisy to separate settings a few percent apart)."""
    set_tuning, run, sync, level_ms = make_runner()
    run(2)
    sync()
    out = []
    for g, t in candidates:
        set_tuning(g, t)
        best = None
        for _ in range(repeats):
            run(steps)
            sync()
            dt = level_ms() / steps / 1e3
            best = dt if best is None else min(best, dt)
        out.append(((g, t), best))
    return out


def tune(steps: int = 10, path: str = TUNING_PATH, verbose: bool = True):
    import torch

    import workloads as W
    from . import LEM_F_PHASE_TIMERS, Solver
    table = {"note": "level-kernel ms per step of candidate settings, per grid-size bucket; "
                     "fastest kept",
             "buckets": []}
    dev = torch.device("cuda:0")
    for (lo, hi), side in zip(BUCKETS, BUCKET_SIDES):
        w = W.LARGE_10000 if side == 10000 else W.SMALL_256.with_(ny=side, nx=side)
        h0 = torch.from_numpy(W.initial_heights(w.ny, w.nx, 0)).to(dev)
        h = h0.clone()
        s = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev, tuning=None,
                   flags=LEM_F_PHASE_TIMERS)

        def make():
            def run(k):  # every timed run starts from the same heights
                h.copy_(h0)
                s.run(h, k)

            return (lambda g, t: s.set_tuning(g, t), run, s.sync,
                    lambda: s.stats().kernel_ms[1])

        res = time_candidates(make, steps)
        s.close()
        (g, t), best = min(res, key=lambda r: r[1])
        entry = {"lo": lo, "hi": hi, "side": side, "global_workgroups": g, "tail_level": t,
                 "ms_per_step": round(best * 1e3, 4),
                 "timings_ms": {f"{c[0]}/{c[1]}": round(v * 1e3, 4) for c, v in res}}
        table["buckets"].append(entry)
        if verbose:
            print(json.dumps(entry), flush=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    tune()
