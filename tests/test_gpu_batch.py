"""GPU: batched realizations (many grids per launch) against single-grid
runs (bit-identical) and against the oracle; the run-to-steady-state driver."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, require_gpu

pytestmark = pytest.mark.gpu


def _grids():
    # Mixed sizes (smaller than a tile, ragged, several tiles), parameters,
    # exponents (sqrt path, pow path, m = 1) and one grid with dx != dy.
    out = []
    spec = [(3, 3, 0.5), (5, 7, 0.45), (64, 64, 0.5), (70, 130, 0.4), (130, 70, 1.0),
            (200, 200, 0.55), (129, 257, 0.5), (33, 300, 0.35), (96, 96, 0.6)]
    for i, (ny, nx, m) in enumerate(spec):
        dy = 100.0 if i != 6 else 60.0
        out.append(W.Realization(ny, nx, 100.0, dy, 1000.0 * (1 + i % 3), m,
                                 2e-4 * (1 + i), 1e-5 * (1 + 0.3 * i), 40 + i))
    return out


def _batch(torch, grids, flags=0):
    from paper_1803_02977_amd import Batch
    return Batch(grids, flags=flags, device=torch.device("cuda:0"))


def _single(torch, r, h0, steps):
    from paper_1803_02977_amd import Solver
    h = torch.from_numpy(h0).to("cuda:0")
    s = Solver(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, r.U, r.K, device=torch.device("cuda:0"))
    s.run(h, steps)
    s.sync()
    rt = s.routing()
    out = h.cpu().numpy()
    s.close()
    return out, rt


def test_batch_equals_each_grid_alone():
    torch = require_gpu()
    grids = _grids()
    h0 = W.batch_initial_heights(grids)
    b = _batch(torch, grids)
    h = torch.from_numpy(h0).to("cuda:0")
    b.run(h, 15)
    b.sync()
    for g, r in enumerate(grids):
        print(f"[gpu] batch grid {g}: {r.ny}x{r.nx}", flush=True)
        ref_h, ref_r = _single(torch, r, W.initial_heights(r.ny, r.nx, r.seed), 15)
        assert np.array_equal(b.view(h, g).cpu().numpy(), ref_h), g
        rt = b.routing(g)
        for k in ("rec", "depth", "count"):
            assert torch.equal(rt[k], ref_r[k]), (g, k)
        assert rt["nlevels"] == ref_r["nlevels"]
        assert np.array_equal(rt["offsets"], ref_r["offsets"])
    b.close()


def test_batch_matches_oracle():
    torch = require_gpu()
    grids = _grids()
    h0 = W.batch_initial_heights(grids)
    b = _batch(torch, grids)
    h = torch.from_numpy(h0).to("cuda:0")
    b.run(h, 12)
    b.sync()
    for g, r in enumerate(grids):
        p = oracle.Params(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, 1.0, r.U, r.K)
        ref = oracle.run(W.initial_heights(r.ny, r.nx, r.seed), p, 12)
        rt = b.routing(g)
        assert np.array_equal(rt["rec"].cpu().numpy(), ref["rec"]), g
        assert np.array_equal(rt["depth"].cpu().numpy(), ref["depth"]), g
        assert np.array_equal(rt["count"].cpu().numpy().view(np.uint32), ref["count"]), g
        assert_heights_close(b.view(h, g).cpu().numpy(), ref["h"], what=f"grid {g}")
    b.close()


def test_run_to_steady_state_matches_oracle():
    """Every grid stops at the first check after which its last step changed
    no cell by more than rtol*max|h|; the oracle run for the same number of
    steps gives the same heights, and its next step is below tolerance."""
    torch = require_gpu()
    grids = [W.Realization(s, s, 100.0, 100.0, 2e4, m, 1e-3, k, 7 + i)
             for i, (s, m, k) in enumerate([(20, 0.5, 5e-5), (33, 0.45, 1e-4), (48, 0.5, 2e-4),
                                            (17, 0.6, 5e-4)])]
    h0 = W.batch_initial_heights(grids)
    b = _batch(torch, grids)
    h = torch.from_numpy(h0).to("cuda:0")
    steps = b.run_to_steady(h, rtol=1e-6, check_every=5, max_steps=20000)
    assert np.all(steps > 0), steps
    assert np.all(steps % 5 == 0)
    for g, r in enumerate(grids):
        p = oracle.Params(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, 1.0, r.U, r.K)
        hg = W.initial_heights(r.ny, r.nx, r.seed)
        before = oracle.run(hg, p, int(steps[g]) - 1)["h"]
        ref = oracle.run(before, p, 1)["h"]
        got = b.view(h, g).cpu().numpy()
        assert_heights_close(got, ref, rtol=1e-10, what=f"grid {g}")
        assert np.abs(ref - before).max() <= 1e-6 * np.abs(ref).max()
        # One check earlier the grid had not converged yet.
        if steps[g] > 5:
            prev = oracle.run(hg, p, int(steps[g]) - 6)["h"]
            prev2 = oracle.run(prev, p, 1)["h"]
            assert np.abs(prev2 - prev).max() > 1e-6 * np.abs(prev2).max()
    b.close()


def test_batch_of_one_and_argument_errors():
    torch = require_gpu()
    from paper_1803_02977_amd import LemError, lem
    r = W.Realization(90, 110, 100.0, 100.0, 1000.0, 0.5, 5e-4, 1e-5, 3)
    h0 = W.initial_heights(r.ny, r.nx, r.seed)
    b = _batch(torch, [r])
    h = torch.from_numpy(h0.ravel().copy()).to("cuda:0")
    b.run(h, 9)
    b.sync()
    ref_h, _ = _single(torch, r, h0, 9)
    assert np.array_equal(b.view(h, 0).cpu().numpy(), ref_h)
    with pytest.raises(LemError):
        b.routing(1)
    with pytest.raises(LemError):
        b.run(torch.zeros(10, dtype=torch.float64, device="cuda:0"), 1)
    b.close()
    bad = [lem.lem_grid(10, 10, 1.0, 1.0, 1.0, 0.5, 0.0, 0.0, 1.0, 1e-12, 100, 0, 5)]
    assert lem.lem_batch_workspace_bytes(bad) == 0


def test_batch_with_fields_equals_each_grid_alone():
    """Per-cell K and U fields laid out like the batch heights."""
    torch = require_gpu()
    grids = _grids()[2:6]
    h0 = W.batch_initial_heights(grids)
    rng = np.random.default_rng(5)
    K = 1e-5 * np.exp(0.5 * rng.standard_normal(h0.size))
    U = rng.uniform(1e-4, 2e-3, h0.size)
    b = _batch(torch, grids)
    h = torch.from_numpy(h0).to("cuda:0")
    b.run(h, 10, K=torch.from_numpy(K).to("cuda:0"), U=torch.from_numpy(U).to("cuda:0"))
    b.sync()
    from paper_1803_02977_amd import Solver
    for g, r in enumerate(grids):
        o, n = b.offsets[g], r.ny * r.nx
        hs = torch.from_numpy(W.initial_heights(r.ny, r.nx, r.seed)).to("cuda:0")
        s = Solver(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, r.U, r.K, device=torch.device("cuda:0"))
        s.run(hs, 10, K=torch.from_numpy(K[o:o + n].reshape(r.ny, r.nx)).to("cuda:0"),
              U=torch.from_numpy(U[o:o + n].reshape(r.ny, r.nx)).to("cuda:0"))
        s.sync()
        s.close()
        assert np.array_equal(b.view(h, g).cpu().numpy(), hs.cpu().numpy()), g
    b.close()


def test_run_to_steady_in_chunks_equals_one_call():
    """A run split over calls (grids steady on entry are skipped) gives the
    same heights and step counts as one call."""
    torch = require_gpu()
    grids = [W.Realization(s, s, 100.0, 100.0, 2e4, m, 1e-3, k, 17 + i)
             for i, (s, m, k) in enumerate([(20, 0.5, 5e-5), (33, 0.45, 1e-4), (48, 0.5, 2e-4),
                                            (17, 0.6, 5e-4)])]
    h0 = W.batch_initial_heights(grids)
    b = _batch(torch, grids)
    h1 = torch.from_numpy(h0).to("cuda:0")
    one = b.run_to_steady(h1, rtol=1e-6, check_every=5, max_steps=20000)
    h2 = torch.from_numpy(h0).to("cuda:0")
    seen = []
    many = b.run_to_steady(h2, rtol=1e-6, check_every=5, max_steps=20000, chunk=15,
                           progress=lambda s, c: seen.append((s, c)))
    assert np.array_equal(one, many), (one, many)
    assert torch.equal(h1, h2)
    assert seen and seen[-1][1] == len(grids)
    b.close()


def test_level_pass_modes_give_identical_results():
    """The crossing trees of a batch ordered by one device-wide pass or by
    one workgroup per grid: heights, routing and level history identical."""
    torch = require_gpu()
    from paper_1803_02977_amd import LEM_LEVELS_GLOBAL, LEM_LEVELS_PER_GRID
    grids = _grids()
    h0 = W.batch_initial_heights(grids)
    out = {}
    settings = [(LEM_LEVELS_GLOBAL, 0), (LEM_LEVELS_PER_GRID, 1024), (LEM_LEVELS_PER_GRID, 256)]
    for mode, threads in settings:
        print(f"[gpu] batch level pass mode {mode} threads {threads}", flush=True)
        b = _batch(torch, grids)
        got = b.set_tuning(level_pass=mode, level_threads=threads)
        assert got["level_pass"] == mode
        h = torch.from_numpy(h0).to("cuda:0")
        b.run(h, 25)
        b.sync()
        routes = [b.routing(g) for g in range(len(grids))]
        out[(mode, threads)] = (h.cpu().numpy(), routes, b.stats().max_nlevels)
        b.close()
    ha, ra, la = out[settings[0]]
    for cfg in settings[1:]:
        hb, rb, lb = out[cfg]
        assert np.array_equal(ha, hb), cfg
        assert la == lb, cfg
        for g in range(len(grids)):
            for k in ("rec", "depth", "count"):
                assert torch.equal(ra[g][k], rb[g][k]), (cfg, g, k)
            assert ra[g]["nlevels"] == rb[g]["nlevels"]
            assert np.array_equal(np.asarray(ra[g]["offsets"]), np.asarray(rb[g]["offsets"]))


def test_full_size_batch_sampled_realizations_match_oracle():
    """The 512-realization benchmark batch (square grids of 128 to 1024 cells
    a side, 2.16e8 cells, per-grid level pass chosen as the benchmark runs it),
    3 steps: the smallest, a middle and the largest realization have the
    oracle's routing exactly and its heights within 1e-12."""
    torch = require_gpu()
    from tests.gpu_util import assert_routing_equal
    grids = W.batch_realizations()
    print(f"[gpu] full batch: {len(grids)} grids, 3 steps", flush=True)
    b = _batch(torch, grids)
    h = torch.from_numpy(W.batch_initial_heights(grids)).to("cuda:0")
    b.run(h, 3)
    b.sync()
    sizes = [r.ny * r.nx for r in grids]
    for g in (int(np.argmin(sizes)), len(grids) // 2, int(np.argmax(sizes))):
        r = grids[g]
        print(f"[gpu] full batch grid {g}: {r.ny}x{r.nx}", flush=True)
        p = oracle.Params(r.ny, r.nx, r.dx, r.dy, r.dt, r.m, 1.0, r.U, r.K)
        ref = oracle.run(W.initial_heights(r.ny, r.nx, r.seed), p, 3)
        assert_routing_equal(b.routing(g), ref)
        assert_heights_close(b.view(h, g).cpu().numpy(), ref["h"])


def test_run_to_steady_reports_heights_that_stop_being_finite():
    """A NaN in one grid's heights (no input validation) never passes for a
    steady state: the call ends with LEM_E_NONFINITE instead."""
    torch = require_gpu()
    from paper_1803_02977_amd.lem import LEM_E_NONFINITE, LemError
    grids = [W.Realization(s, s, 100.0, 100.0, 2e4, 0.5, 1e-3, 5e-5, 70 + i)
             for i, s in enumerate((24, 40))]
    h0 = W.batch_initial_heights(grids)
    h0[24 * 24 + 40 * 7 + 9] = np.nan
    b = _batch(torch, grids)
    h = torch.from_numpy(h0).to("cuda:0")
    print("[gpu] run_to_steady with a NaN height", flush=True)
    with pytest.raises(LemError) as e:
        b.run_to_steady(h, rtol=1e-6, check_every=5, max_steps=200)
    assert e.value.status == LEM_E_NONFINITE, e.value
    b.close()
