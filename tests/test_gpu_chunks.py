"""GPU: the chunk stage for trees that cross tile edges.

Workgroups take chunks of crossing roots and finish those trees in LDS; a
chunk whose trees need more than the stage holds (cells or levels) is handed
to the level pass that follows.  Results must not depend on any of this:
heights and routing are bit-identical with the stage on or off and for any
chunk size, and match the oracle (routing bit-exact, heights within 1e-12).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, assert_routing_equal, oracle_params, require_gpu

pytestmark = pytest.mark.gpu

CHUNKS_ON, CHUNKS_OFF = 1, 2
LEVELS_PER_GRID = 2


def _pyramid(ny, nx, seed, scale=1.0):
    """Heights rising with the distance to the nearest edge (plus a little
    noise): every tree is a long fan draining straight to the perimeter, so
    trees cross many tiles and run as deep as half the shorter side."""
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    d = np.minimum(np.minimum(y, ny - 1 - y), np.minimum(x, nx - 1 - x)).astype(np.float64)
    h = scale * d + 0.01 * np.random.default_rng(seed).random((ny, nx))
    h[0, :] = h[-1, :] = 0.0
    h[:, 0] = h[:, -1] = 0.0
    return h


def _run(torch, w, h0, steps, **tuning):
    from paper_1803_02977_amd import Solver
    ny, nx = h0.shape
    s = Solver(ny, nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=torch.device("cuda:0"),
               tuning=None)
    got = s.set_tuning(**tuning) if tuning else None
    h = torch.from_numpy(np.ascontiguousarray(h0)).to("cuda:0")
    s.run(h, steps)
    s.sync()
    r = s.routing()
    st = s.stats()
    out = h.cpu().numpy()
    s.close()
    return out, r, st, got


@pytest.mark.parametrize("roots", [1, 7, 128, 256])
def test_chunk_sizes_match_stage_off_and_oracle(roots):
    torch = require_gpu()
    w = W.SMALL_256
    h0 = W.initial_heights(500, 700, 21)
    print(f"[gpu] chunk stage 500x700 roots {roots}", flush=True)
    ref_h, ref_r, _, got = _run(torch, w, h0, 12, chunk_pass=CHUNKS_OFF)
    assert got["chunk_pass"] == CHUNKS_OFF
    h, r, st, got = _run(torch, w, h0, 12, chunk_pass=CHUNKS_ON, chunk_roots=roots)
    assert got["chunk_pass"] == CHUNKS_ON and got["chunk_roots"] == roots
    assert np.array_equal(h, ref_h)
    for k in ("rec", "depth", "count"):
        assert torch.equal(r[k], ref_r[k]), k
    assert r["nlevels"] == ref_r["nlevels"]
    assert st.crossing_last > 0
    ref = oracle.run(h0, oracle_params(w, 500, 700), 12)
    assert_routing_equal(r, ref)
    assert_heights_close(h, ref["h"])


@pytest.mark.parametrize("shape,roots", [((300, 340), 128), ((200, 220), 1), ((640, 600), 4)])
def test_chunks_that_do_not_fit_go_to_the_level_pass(shape, roots):
    """Pyramids: fans of about 150 cells per root overflow a 128-root chunk's
    cell capacity; at 600 cells a side they run deeper than the stage's
    level limit.  One root per chunk at 200 cells a side fits."""
    torch = require_gpu()
    w = W.SMALL_256
    ny, nx = shape
    h0 = _pyramid(ny, nx, 5, scale=0.5)
    print(f"[gpu] pyramid {ny}x{nx} roots {roots}", flush=True)
    h, r, st, _ = _run(torch, w, h0, 4, chunk_pass=CHUNKS_ON, chunk_roots=roots)
    ref = oracle.run(h0, oracle_params(w, ny, nx), 4)
    assert_routing_equal(r, ref)
    assert_heights_close(h, ref["h"])
    assert st.crossing_last > 0
    off_h, off_r, _, _ = _run(torch, w, h0, 4, chunk_pass=CHUNKS_OFF)
    assert np.array_equal(h, off_h)
    # The overflow of a single grid ordered by its one workgroup instead of
    # the device-wide pass.
    print(f"[gpu] pyramid {ny}x{nx} roots {roots} per-grid level pass", flush=True)
    pg_h, pg_r, _, got = _run(torch, w, h0, 4, chunk_pass=CHUNKS_ON, chunk_roots=roots,
                              level_pass=LEVELS_PER_GRID, level_threads=1024)
    assert got["level_pass"] == LEVELS_PER_GRID
    assert np.array_equal(h, pg_h)
    for k in ("rec", "depth", "count"):
        assert torch.equal(r[k], pg_r[k]), k
    assert r["nlevels"] == pg_r["nlevels"]


def test_batch_chunk_overflow_to_per_grid_pass():
    """A batch mixing pyramids (chunks overflow to the per-grid pass) and
    random grids (chunks fit): every grid equals the oracle."""
    torch = require_gpu()
    from paper_1803_02977_amd import LEM_LEVELS_GLOBAL, LEM_LEVELS_PER_GRID, Batch
    spec = [(300, 320, "pyr"), (130, 200, "rand"), (64, 64, "rand"), (400, 260, "pyr"),
            (257, 129, "rand")]
    grids, h0s = [], []
    for i, (ny, nx, kind) in enumerate(spec):
        grids.append(W.Realization(ny, nx, 100.0, 100.0, 1000.0, 0.5, 3e-4 * (1 + i),
                                   1e-5 * (1 + 0.5 * i), 70 + i))
        h0s.append(_pyramid(ny, nx, i, 0.3) if kind == "pyr" else W.initial_heights(ny, nx, 70 + i))
    h0 = np.concatenate([a.ravel() for a in h0s])
    results = {}
    for mode in (LEM_LEVELS_PER_GRID, LEM_LEVELS_GLOBAL):
        print(f"[gpu] batch chunk overflow, level pass {mode}", flush=True)
        b = Batch(grids, device=torch.device("cuda:0"), tuning=None)
        b.set_tuning(level_pass=mode, chunk_pass=CHUNKS_ON, chunk_roots=64)
        h = torch.from_numpy(h0.copy()).to("cuda:0")
        b.run(h, 5)
        b.sync()
        results[mode] = (h.cpu().numpy(), [b.routing(g) for g in range(len(grids))])
        b.close()
    hp, rp = results[LEM_LEVELS_PER_GRID]
    hg, rg = results[LEM_LEVELS_GLOBAL]
    assert np.array_equal(hp, hg)
    off = 0
    for g, r in enumerate(grids):
        ref = oracle.run(h0s[g], oracle.Params(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, 1.0, r.U, r.K), 5)
        assert_routing_equal(rp[g], ref)
        for k in ("rec", "depth", "count"):
            assert torch.equal(rp[g][k], rg[g][k]), (g, k)
        assert_heights_close(hp[off:off + r.ny * r.nx].reshape(r.ny, r.nx), ref["h"])
        off += r.ny * r.nx
