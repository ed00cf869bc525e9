"""GPU: the 2048x2048 (lognormal K, 200 steps) and 10000x10000 (50 steps)
workloads over their full length against stored oracle results.

The stored results were written by ``tests/golden/make_headline_goldens.py``,
which runs only the oracle: SHA-256 digests of the last step's receivers,
levels, counts and level offsets (compared bit for bit) and the final heights
at 2^20 seeded sample cells (compared within 1e-12 relative, 1 m floor).
Whether every height is also bit-identical is printed."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import assert_heights_close, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SAMPLE_SEED = 20180308


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        meta = json.load(f)
    hs = np.load(os.path.join(GOLDEN, name + "-hsample.npy"), allow_pickle=False)
    return meta, hs


@pytest.mark.parametrize("w", [W.MEDIUM_2048, W.LARGE_10000], ids=lambda w: w.name)
def test_full_length_against_stored_oracle(w):
    torch = require_gpu()
    from paper_1803_02977_amd import Solver
    meta, hs = _golden(w.name)
    assert meta["steps"] == w.steps and meta["ny"] == w.ny and meta["nx"] == w.nx
    assert meta["sample_seed"] == SAMPLE_SEED
    print(f"[gpu] {w.name}: {w.steps} steps against the stored oracle results", flush=True)
    h0, K, U = W.make_inputs(w, meta["seed"])
    dev = torch.device("cuda:0")
    h = torch.from_numpy(h0).to(dev)
    s = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev)
    s.run(h, w.steps, K=None if K is None else torch.from_numpy(K).to(dev))
    s.sync()
    r = s.routing()
    got = h.cpu().numpy()
    s.close()
    d = meta["sha256"]
    assert _digest(r["rec"].cpu().numpy().astype(np.int32)) == d["rec_int32"], "receivers"
    assert _digest(r["depth"].cpu().numpy().astype(np.int32)) == d["depth_int32"], "levels"
    assert _digest(r["count"].cpu().numpy().view(np.uint32)) == d["count_uint32"], "counts"
    assert _digest(np.asarray(r["offsets"], np.int64)) == d["offsets_int64"], "level offsets"
    assert r["nlevels"] == meta["nlevels_last_step"]
    n = w.ny * w.nx
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=hs.size, replace=False))
    assert_heights_close(got.ravel()[idx], hs)
    same = _digest(got.astype(np.float64)) == d["h_float64"]
    print(f"[gpu] {w.name}: routing bit-exact, {hs.size} sampled heights within 1e-12; "
          f"all heights bit-identical: {same}", flush=True)
