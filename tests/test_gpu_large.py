"""GPU at the full sizes the benchmark times: the 10000x10000 workload.

One step from the seeded initial heights is compared cell by cell with the
oracle.  After the benchmark's 50 steps, properties that hold at any size are
checked on every cell: receivers of sampled row bands against the oracle,
the drainage-count recursion and total, the level recursion, and the
implicit-update identity of the last step."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import H_RTOL, assert_heights_close, assert_routing_equal, oracle_params, require_gpu

pytestmark = pytest.mark.gpu

W3 = W.LARGE_10000


def _solver(torch):
    from paper_1803_02977_amd import Solver
    return Solver(W3.ny, W3.nx, W3.dx, W3.dy, W3.dt, W3.m, W3.U, W3.K, device=torch.device("cuda:0"))


def test_large_grid_first_step_matches_oracle():
    torch = require_gpu()
    h0 = W.initial_heights(W3.ny, W3.nx, 0)
    print("[gpu] 10000x10000 one step vs oracle", flush=True)
    h = torch.from_numpy(h0).to("cuda:0")
    s = _solver(torch)
    s.run(h, 1)
    s.sync()
    r = s.routing()
    got = h.cpu().numpy()
    s.close()
    ref = oracle.run(h0, oracle_params(W3), 1)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_large_grid_properties_after_benchmark_steps():
    torch = require_gpu()
    steps = W3.steps
    print(f"[gpu] 10000x10000 {steps} steps, properties", flush=True)
    h = torch.from_numpy(W.initial_heights(W3.ny, W3.nx, 0)).to("cuda:0")
    s = _solver(torch)
    s.run(h, steps - 1)
    s.sync()
    before = h.cpu().numpy()
    s.run(h, 1)
    s.sync()
    r = s.routing()
    after = h.cpu().numpy()
    rec = r["rec"].cpu().numpy().ravel().astype(np.int64)
    depth = r["depth"].cpu().numpy().ravel()
    count = r["count"].cpu().numpy().view(np.uint32).ravel().astype(np.int64)
    s.close()
    n = W3.ny * W3.nx
    ny, nx = W3.ny, W3.nx
    # Receivers of sampled row bands, computed by the oracle from the heights
    # the last step started from.
    rng = np.random.default_rng(0)
    for row in rng.integers(1, ny - 1, size=24):
        band = before[row - 1: row + 2]
        exp = oracle.receivers(band, W3.dx, W3.dy)[1] - nx + row * nx
        exp[0] = row * nx
        exp[-1] = row * nx + nx - 1
        assert np.array_equal(rec[row * nx: (row + 1) * nx], exp), row
    # Forest: roots have level 0; every other cell is one level below its
    # receiver; counts are 1 plus the donors' counts and sum to N over roots.
    idx = np.arange(n)
    roots = rec == idx
    assert np.all(depth[roots] == 0)
    nr = ~roots
    assert np.all(depth[nr] == depth[rec[nr]] + 1)
    inflow = np.bincount(rec[nr], weights=count[nr], minlength=n).astype(np.int64)
    assert np.array_equal(count, 1 + inflow)
    assert count[roots].sum() == n
    hist = np.bincount(depth, minlength=r["nlevels"])
    assert np.array_equal(np.asarray(r["offsets"]), np.concatenate([[0], np.cumsum(hist)]))
    # Heights: interior roots are uplifted, the perimeter is unchanged and
    # every eroding cell satisfies (1 + F) h'_c - F h'_r = h_c + U dt.
    b = before.ravel()
    a = after.ravel()
    yy, xx = np.divmod(idx, nx)
    perim = (yy == 0) | (xx == 0) | (yy == ny - 1) | (xx == nx - 1)
    assert np.array_equal(a[perim], b[perim])
    udt = W3.U * W3.dt
    sinks = roots & ~perim
    assert np.array_equal(a[sinks], b[sinks] + udt)
    ry, rx = np.divmod(rec[nr], nx)
    diag = (ry != yy[nr]) & (rx != xx[nr])
    d = np.where(diag, np.sqrt(W3.dx ** 2 + W3.dy ** 2), np.where(ry != yy[nr], W3.dy, W3.dx))
    F = W3.K * W3.dt * (count[nr] * W3.dx * W3.dy) ** W3.m / d
    lhs = (1 + F) * a[nr] - F * a[rec[nr]]
    rhs = b[nr] + udt
    scale = np.maximum(np.abs(rhs), 1.0) * (1 + 2 * F)
    assert np.all(np.abs(lhs - rhs) <= 4 * H_RTOL * scale)


@pytest.mark.parametrize("edge", [12649, 16000])
def test_size_sweep_region_d_first_step_matches_oracle(edge):
    """The two largest rasters of the size sweep (region D of the paper's GPU
    scaling table: 1.6e8 and 2.56e8 cells), one step from seeded noise with
    the sweep's parameters, every cell against the oracle."""
    torch = require_gpu()
    from paper_1803_02977_amd import Solver
    w = W.SMALL_256.with_(ny=edge, nx=edge)
    h0 = W.initial_heights(edge, edge, 0)
    print(f"[gpu] {edge}x{edge} one step vs oracle", flush=True)
    h = torch.from_numpy(h0).to("cuda:0")
    s = Solver(edge, edge, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=torch.device("cuda:0"))
    s.run(h, 1)
    s.sync()
    r = s.routing()
    got = h.cpu().numpy()
    s.close()
    del h
    ref = oracle.run(h0, oracle_params(w), 1)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])
