"""Launch tuner for the stages that resolve trees crossing tile edges.

The settings of ``lem_tuning`` change only the schedule, never the results
(GPU tests check them bit for bit):

- ``chunk_pass`` / ``chunk_roots``: the chunk stage (trees finished in LDS, a
  chunk of roots per workgroup) on or off, and the roots per chunk;
- ``level_pass``: trees the chunk stage hands on go to one device-wide pass
  or to one workgroup per grid; ``level_threads``: that workgroup's size;
- ``global_workgroups`` / ``tail_level``: workgroups of the device-wide pass
  and the level size below which one workgroup works alone.

Two tables are kept in ``tuning.json`` next to this file:

- ``single``: one grid, by cell-count bucket; a square noise raster per
  bucket, timed from its initial surface (the regime of the benchmark runs);
- ``batch``: batches of independent realizations, by total-cell bucket; a
  batch of the benchmark's realization mix, evolved for ``EVOLVE`` steps
  first (runs of batches spend most of their steps on evolved landscapes,
  whose trees are deep and often too large for a chunk).

Each candidate is timed by the crossing-tree kernels' own HIP events
(``lem_stats.kernel_ms[1]``), over the same steps from the same heights.

    python -m paper_1803_02977_amd.tune            # tune and write tuning.json

``lookup(cells, batch)`` returns the stored setting as a dict of
``lem_tuning`` fields; ``Solver`` and ``Batch`` apply it when
``tuning="auto"``.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "tuning.json")

# Single grids: buckets by cell count [lo, hi) and a square side per bucket.
SINGLE_BUCKETS = [(0, 1 << 18), (1 << 18, 1 << 22), (1 << 22, 1 << 25), (1 << 25, 1 << 31)]
SINGLE_SIDES = [256, 1024, 4096, 10000]
# Device-wide pass: workgroups x one-workgroup level threshold.
LEVEL_CANDIDATES = [(g, t) for g in (16, 32, 64, 96, 128, 160, 192, 256)
                    for t in (512, 2048, 8192)]
CHUNK_ROOTS = (4, 8, 16, 32, 64, 128, 256)
# Batches: buckets by total cells and the number of realizations of the
# benchmark's mix (edges 128..1024) that represents each.
BATCH_BUCKETS = [(0, 1 << 22), (1 << 22, 1 << 26), (1 << 26, 1 << 31)]
BATCH_GRIDS = [8, 64, 512]
EVOLVE = 100

LEVELS_GLOBAL, LEVELS_PER_GRID = 1, 2
CHUNKS_ON, CHUNKS_OFF = 1, 2
FIELDS = ("global_workgroups", "tail_level", "level_pass", "level_threads", "chunk_pass",
          "chunk_roots")


def load(path: str = TUNING_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def lookup(cells: int, batch: bool = False, table=None):
    """The stored setting (dict of lem_tuning fields) for a single grid or a
    batch of `cells` cells in all, or None."""
    table = table if table is not None else load()
    if not table:
        return None
    for entry in table.get("batch" if batch else "single", []):
        if entry["lo"] <= cells < entry["hi"]:
            return {k: entry["setting"][k] for k in FIELDS}
    return None


def setting(global_workgroups=0, tail_level=0, level_pass=0, level_threads=0, chunk_pass=0,
            chunk_roots=0):
    return dict(global_workgroups=global_workgroups, tail_level=tail_level,
                level_pass=level_pass, level_threads=level_threads, chunk_pass=chunk_pass,
                chunk_roots=chunk_roots)


def _label(s):
    if s["chunk_pass"] == CHUNKS_OFF:
        chunk = "chunks off"
    else:
        chunk = f"chunks {s['chunk_roots'] or 'default'}"
    if s["level_pass"] == LEVELS_PER_GRID:
        level = f"per-grid {s['level_threads'] or 'default'}"
    else:
        level = f"global {s['global_workgroups'] or 'max'}/{s['tail_level'] or 'default'}"
    return f"{chunk}, {level}"


def time_candidates(ctx_obj, h, h0, candidates, steps, repeats=3):
    """Crossing-tree milliseconds per step of each candidate (best of
    `repeats` runs of `steps` steps, each from the heights h0)."""
    out = []
    for cand in candidates:
        got = ctx_obj.set_tuning(**cand)
        best = None
        for _ in range(repeats):
            h.copy_(h0)
            ctx_obj.run(h, steps)
            ctx_obj.sync()
            ms = ctx_obj.stats().kernel_ms[1] / steps
            best = ms if best is None else min(best, ms)
        out.append((cand, got, best))
    return out


def _entry(lo, hi, what, res):
    cand, got, best = min(res, key=lambda r: r[2])
    return {"lo": lo, "hi": hi, "workload": what,
            "setting": {k: int(got[k]) for k in FIELDS}, "ms_per_step": round(best, 4),
            "timings_ms": {_label(c): round(v, 4) for c, _, v in res}}


def tune_single(steps=10, verbose=True):
    import torch

    import workloads as W
    from . import LEM_F_PHASE_TIMERS, Solver
    dev = torch.device("cuda:0")
    entries = []
    for (lo, hi), side in zip(SINGLE_BUCKETS, SINGLE_SIDES):
        w = W.LARGE_10000 if side == 10000 else W.SMALL_256.with_(ny=side, nx=side)
        h0 = torch.from_numpy(W.initial_heights(w.ny, w.nx, 0)).to(dev)
        h = h0.clone()
        s = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev, tuning=None,
                   flags=LEM_F_PHASE_TIMERS)
        s.run(h, 2)
        s.sync()
        # The device-wide pass alone (chunk stage off), then the chunk stage
        # in front of the best of it.
        res = time_candidates(s, h, h0, [setting(g, t, LEVELS_GLOBAL, 0, CHUNKS_OFF)
                                         for g, t in LEVEL_CANDIDATES], steps)
        best = min(res, key=lambda r: r[2])[1]
        g, t = best["global_workgroups"], best["tail_level"]
        res += time_candidates(s, h, h0, [setting(g, t, LEVELS_GLOBAL, 0, CHUNKS_ON, r)
                                          for r in CHUNK_ROOTS], steps)
        s.close()
        e = _entry(lo, hi, f"{side}x{side} noise raster ({w.name} parameters), {steps} steps "
                           "from the initial surface", res)
        entries.append(e)
        if verbose:
            print(json.dumps({k: e[k] for k in ("lo", "hi", "setting", "ms_per_step")}),
                  flush=True)
    return entries


def tune_batch(steps=10, verbose=True):
    import torch

    import workloads as W
    from . import LEM_F_PHASE_TIMERS, Batch
    dev = torch.device("cuda:0")
    entries = []
    for (lo, hi), n in zip(BATCH_BUCKETS, BATCH_GRIDS):
        reals = W.batch_realizations(n, seed=0)
        cells = sum(r.ny * r.nx for r in reals)
        h0 = torch.from_numpy(W.batch_initial_heights(reals)).to(dev)
        b = Batch(reals, flags=LEM_F_PHASE_TIMERS, device=dev, tuning=None)
        b.run(h0, EVOLVE)  # the evolved landscapes the candidates start from
        b.sync()
        h = h0.clone()
        cands = []
        for chunk, roots in [(CHUNKS_OFF, 0)] + [(CHUNKS_ON, r) for r in CHUNK_ROOTS]:
            cands.append(setting(0, 0, LEVELS_PER_GRID, 1024, chunk, roots))
            cands.append(setting(0, 0, LEVELS_PER_GRID, 256, chunk, roots))
            cands.append(setting(0, 0, LEVELS_GLOBAL, 0, chunk, roots))
        res = time_candidates(b, h, h0, cands, steps)
        b.close()
        e = _entry(lo, hi, f"{n} realizations of the batch benchmark's mix ({cells} cells), "
                           f"{steps} steps after {EVOLVE} steps of evolution", res)
        entries.append(e)
        if verbose:
            print(json.dumps({k: e[k] for k in ("lo", "hi", "setting", "ms_per_step")}),
                  flush=True)
    return entries


def tune(steps: int = 10, path: str = TUNING_PATH, verbose: bool = True):
    table = {"note": "crossing-tree kernel ms per step of candidate settings; fastest kept",
             "single": tune_single(steps, verbose), "batch": tune_batch(steps, verbose)}
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    tune()
