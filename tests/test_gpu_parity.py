"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Receivers, levels, level offsets and drainage counts must be bit-exact; FP64
heights must agree within 1e-12 relative (1 m floor).  Inputs come from the
seeded generators in ``workloads``; the oracle runs on the same arrays.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, assert_routing_equal, oracle_params, require_gpu

pytestmark = pytest.mark.gpu


def _solver(torch, w, ny=None, nx=None, flags=0):
    from paper_1803_02977_amd import Solver
    return Solver(ny or w.ny, nx or w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, flags=flags,
                  device=torch.device("cuda:0"))


def _to_dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _run_gpu(torch, w, h0, steps, K=None, U=None):
    ny, nx = h0.shape
    h = _to_dev(torch, h0)
    s = _solver(torch, w, ny, nx)
    s.run(h, steps, K=_to_dev(torch, K), U=_to_dev(torch, U))
    s.sync()
    r = s.routing()
    hist = s.level_history(max(steps, 1))
    out = h.cpu().numpy()
    s.close()
    return out, r, hist


@pytest.mark.parametrize("steps", [1, 2, 10])
def test_small_grid_steps(steps):
    torch = require_gpu()
    w = W.SMALL_256
    h0 = W.initial_heights(w.ny, w.nx, 0)
    print(f"[gpu] 256x256 seed 0 steps {steps}", flush=True)
    got, r, _ = _run_gpu(torch, w, h0, steps)
    ref = oracle.run(h0, oracle_params(w), steps)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


@pytest.mark.parametrize("seed", range(10))
def test_small_grid_full_run(seed):
    """The 256x256 workload, all 100 steps, ten seeds."""
    torch = require_gpu()
    w = W.SMALL_256
    h0 = W.initial_heights(w.ny, w.nx, seed)
    print(f"[gpu] 256x256 seed {seed} steps {w.steps}", flush=True)
    got, r, _ = _run_gpu(torch, w, h0, w.steps)
    ref = oracle.run(h0, oracle_params(w), w.steps)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_level_count_of_every_step():
    torch = require_gpu()
    w = W.SMALL_256
    h0 = W.initial_heights(w.ny, w.nx, 4)
    steps = 30
    _, _, hist = _run_gpu(torch, w, h0, steps)
    h = h0
    expect = []
    for _ in range(steps):
        ref = oracle.run(h, oracle_params(w), 1)
        expect.append(ref["nlevels"])
        h = ref["h"]
    assert hist.tolist() == expect


SHAPES = [(3, 3), (3, 4), (4, 3), (3, 17), (17, 3), (5, 5), (7, 130), (129, 65), (33, 1000),
          (257, 255), (64, 64), (1000, 7)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_ragged_and_tiny_grids(shape, kind):
    """Grids smaller than one workgroup, ragged edges, and heights quantised
    to four values so that exact slope ties and flats are everywhere."""
    torch = require_gpu()
    ny, nx = shape
    w = W.SMALL_256.with_(ny=ny, nx=nx)
    h0 = (W.initial_heights(ny, nx, 7) if kind == "uniform"
          else W.quantised_heights(ny, nx, 4, seed=7))
    print(f"[gpu] {ny}x{nx} {kind}", flush=True)
    for steps in (1, 5):
        got, r, _ = _run_gpu(torch, w, h0, steps)
        ref = oracle.run(h0, oracle_params(w, ny, nx), steps)
        assert_routing_equal(r, ref)
        assert_heights_close(got, ref["h"])


@pytest.mark.parametrize("m", [0.0, 0.35, 0.45, 0.6, 1.0])
def test_area_exponents(m):
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=96, nx=120, m=m)
    h0 = W.initial_heights(w.ny, w.nx, 12)
    got, r, _ = _run_gpu(torch, w, h0, 20)
    ref = oracle.run(h0, oracle_params(w), 20)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_rectangular_cells_and_fields():
    """dx != dy, a per-cell K field and a per-cell U field."""
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=150, nx=90, dx=30.0, dy=55.0, m=0.45)
    h0 = W.initial_heights(w.ny, w.nx, 5)
    rng = np.random.default_rng(99)
    K = 1e-5 * np.exp(0.5 * rng.standard_normal(h0.shape))
    U = rng.uniform(1e-4, 2e-3, h0.shape)
    got, r, _ = _run_gpu(torch, w, h0, 25, K=K, U=U)
    ref = oracle.run(h0, oracle_params(w), 25, K=K, U=U)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_medium_grid_with_k_field():
    """The 2048x2048 workload with its lognormal K field (first 40 steps)."""
    torch = require_gpu()
    w = W.MEDIUM_2048
    h0, K, _ = W.make_inputs(w, 0)
    steps = 40
    print(f"[gpu] 2048x2048 lognormal K, {steps} steps", flush=True)
    got, r, _ = _run_gpu(torch, w, h0, steps, K=K)
    ref = oracle.run(h0, oracle_params(w), steps, K=K)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_deterministic_and_resumable():
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=300, nx=200)
    h0 = W.initial_heights(w.ny, w.nx, 8)
    a, ra, _ = _run_gpu(torch, w, h0, 60)
    b, rb, _ = _run_gpu(torch, w, h0, 60)
    assert np.array_equal(a, b)
    for k in ("rec", "depth", "count"):
        assert torch.equal(ra[k], rb[k])
    half, _, _ = _run_gpu(torch, w, h0, 30)
    c, rc, _ = _run_gpu(torch, w, half, 30)
    assert np.array_equal(a, c)
    assert torch.equal(ra["count"], rc["count"])


def test_zero_steps_is_a_no_op():
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=40, nx=40)
    h0 = W.initial_heights(40, 40, 1)
    h = _to_dev(torch, h0)
    s = _solver(torch, w)
    s.run(h, 0)
    s.sync()
    assert np.array_equal(h.cpu().numpy(), h0)
    from paper_1803_02977_amd import LemError
    with pytest.raises(LemError):
        s.routing()
    s.close()


@pytest.mark.parametrize("tuning", [(0, 0), (1, 1), (16, 1 << 30), (256, 64), (3, 5000), (0, 0, 2)])
def test_tuning_does_not_change_results(tuning):
    """Workgroup count and the one-workgroup level threshold of the global
    pass change only the schedule: heights and routing stay bit-identical."""
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=500, nx=700)
    h0 = W.initial_heights(w.ny, w.nx, 21)
    ref_h, ref_r, _ = _run_gpu(torch, w, h0, 12)
    h = _to_dev(torch, h0)
    s = _solver(torch, w)
    got = s.set_tuning(*tuning)
    assert got["global_workgroups"] >= 1 and got["tail_level"] >= 1
    s.run(h, 12)
    s.sync()
    r = s.routing()
    assert np.array_equal(h.cpu().numpy(), ref_h)
    for k in ("rec", "depth", "count"):
        assert torch.equal(r[k], ref_r[k])
    s.close()
