"""Write the stored oracle results of the full-length headline workloads.

Calls only the oracle (``oracle/``) and the seeded input generators
(``workloads``).  For each workload the oracle runs every step of it from the
seeded initial heights and this script writes, next to itself:

  <name>.json          the command, seed, step count and SHA-256 digests of the
                       last step's receivers, levels, counts and level offsets
                       (the routing of the heights the last step started from)
                       and of the final heights' bit patterns;
  <name>-hsample.npy   the oracle's final heights at SAMPLE_CELLS cells drawn
                       without replacement by default_rng(SAMPLE_SEED).

    python tests/golden/make_headline_goldens.py [plain-2048x2048-fp64-lognormalK]
                                                 [plain-10000x10000-fp64]

The 10000x10000 run takes about five minutes on one core and about 7 GB of
host memory; the 2048x2048 run about a minute.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

SAMPLE_CELLS = 1 << 20
SAMPLE_SEED = 20180308
HEADLINE = (W.MEDIUM_2048, W.LARGE_10000)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sample_cells(n: int) -> np.ndarray:
    """The sampled cell indices (sorted), identical for writer and reader."""
    k = min(SAMPLE_CELLS, n)
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=k, replace=False))


def paths(name: str):
    return os.path.join(HERE, name + ".json"), os.path.join(HERE, name + "-hsample.npy")


def write(w: W.Workload, seed: int = 0) -> None:
    h0, K, U = W.make_inputs(w, seed)
    p = oracle.Params(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.n, w.U, w.K)
    t0 = time.perf_counter()
    ref = oracle.run(h0, p, w.steps, K=K, U=U)
    secs = time.perf_counter() - t0
    h = ref["h"]
    idx = sample_cells(h.size)
    meta = {
        "workload": w.name,
        "command": "python tests/golden/make_headline_goldens.py " + w.name,
        "seed": seed,
        "steps": w.steps,
        "ny": w.ny,
        "nx": w.nx,
        "sample_cells": int(idx.size),
        "sample_seed": SAMPLE_SEED,
        "nlevels_last_step": int(ref["nlevels"]),
        "sha256": {
            "rec_int32": digest(ref["rec"].astype(np.int32)),
            "depth_int32": digest(ref["depth"].astype(np.int32)),
            "count_uint32": digest(ref["count"].astype(np.uint32)),
            "offsets_int64": digest(np.asarray(ref["offsets"], np.int64)),
            "h_float64": digest(h.astype(np.float64)),
        },
        "oracle_seconds": round(secs, 1),
        "h_checksum": {"sum": float(h.sum()), "max": float(h.max())},
    }
    jpath, npath = paths(w.name)
    np.save(npath, h.ravel()[idx])
    with open(jpath, "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    print(f"{w.name}: {w.steps} steps in {secs:.1f} s, {ref['nlevels']} levels", flush=True)


def main(argv):
    names = argv or [w.name for w in HEADLINE]
    for name in names:
        write(W.WORKLOADS[name])


if __name__ == "__main__":
    main(sys.argv[1:])
