"""GPU: the slope exponent n != 1 (the Newton-Raphson loop of Algorithm 6)
against the oracle's Newton loop, single grids and a batch of mixed n.

Receivers, levels and counts must be bit-exact; heights within 1e-12
relative (1 m floor).  Both sides take the same number of iterations except
where an iterate difference lands within rounding of eps; the extra
iteration then moves the height by less than eps.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, assert_routing_equal, require_gpu

pytestmark = pytest.mark.gpu


def _gpu(torch, w, nexp, h0, steps, K=None, eps=1e-12, max_newton=100):
    from paper_1803_02977_amd import Solver
    ny, nx = h0.shape
    h = torch.from_numpy(h0.copy()).to("cuda:0")
    s = Solver(ny, nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, n=nexp, eps=eps, max_newton=max_newton,
               device=torch.device("cuda:0"))
    s.run(h, steps, K=None if K is None else torch.from_numpy(K).to("cuda:0"))
    s.sync()
    r = s.routing()
    out = h.cpu().numpy()
    s.close()
    return out, r


def _params(w, ny, nx, nexp, eps=1e-12, max_newton=100):
    return oracle.Params(ny, nx, w.dx, w.dy, w.dt, w.m, nexp, w.U, w.K, eps=eps,
                         max_newton=max_newton)


@pytest.mark.parametrize("nexp", [0.7, 1.5, 2.0, 4.0])
def test_newton_exponents(nexp):
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=150, nx=170, m=0.45)
    h0 = W.initial_heights(w.ny, w.nx, 31) * 20.0
    print(f"[gpu] newton n={nexp} 150x170 20 steps", flush=True)
    got, r = _gpu(torch, w, nexp, h0, 20)
    ref = oracle.run(h0, _params(w, w.ny, w.nx, nexp), 20)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_newton_with_k_field_rectangular_cells_and_iteration_limit():
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=97, nx=131, dx=30.0, dy=45.0, m=0.5)
    h0 = W.initial_heights(w.ny, w.nx, 32) * 5.0
    K = 1e-5 * np.exp(0.5 * np.random.default_rng(3).standard_normal(h0.shape))
    for eps, max_newton in ((1e-12, 100), (1e-6, 3), (1e-9, 1)):
        print(f"[gpu] newton n=2 K field eps={eps} max={max_newton}", flush=True)
        got, r = _gpu(torch, w, 2.0, h0, 15, K=K, eps=eps, max_newton=max_newton)
        ref = oracle.run(h0, _params(w, w.ny, w.nx, 2.0, eps, max_newton), 15, K=K)
        assert_routing_equal(r, ref)
        assert_heights_close(got, ref["h"])


def test_newton_large_grid_crossing_trees():
    """512x640 (many tiles; trees crossing tile edges run in the global pass)."""
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=512, nx=640, m=0.5)
    h0 = W.initial_heights(w.ny, w.nx, 33) * 10.0
    print("[gpu] newton n=1.5 512x640 12 steps", flush=True)
    got, r = _gpu(torch, w, 1.5, h0, 12)
    ref = oracle.run(h0, _params(w, w.ny, w.nx, 1.5), 12)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])


def test_batch_of_mixed_exponents_equals_each_grid_alone():
    torch = require_gpu()
    from paper_1803_02977_amd import Batch
    grids = [dict(ny=ny, nx=nx, dx=100.0, dy=100.0, dt=1000.0, m=0.5, U=5e-4, K=1e-5, n=n,
                  eps=1e-12, max_newton=100, seed=50 + i)
             for i, (ny, nx, n) in enumerate([(70, 90, 1.0), (130, 64, 2.0), (65, 200, 0.8),
                                               (128, 128, 1.0), (33, 77, 3.0)])]
    h0 = np.concatenate([W.initial_heights(g["ny"], g["nx"], g["seed"]).ravel() * 10.0
                         for g in grids])
    b = Batch(grids, device=torch.device("cuda:0"))
    h = torch.from_numpy(h0).to("cuda:0")
    b.run(h, 10)
    b.sync()
    for i, g in enumerate(grids):
        w = W.SMALL_256.with_(ny=g["ny"], nx=g["nx"])
        hs = W.initial_heights(g["ny"], g["nx"], g["seed"]) * 10.0
        single, _ = _gpu(torch, w, g["n"], hs, 10)
        assert np.array_equal(b.view(h, i).cpu().numpy(), single), i
        ref = oracle.run(hs, _params(w, g["ny"], g["nx"], g["n"]), 10)
        assert_heights_close(single, ref["h"])
    b.close()


def test_newton_below_one_with_overshooting_iterates():
    """n = 0.5 with a large K*dt: Newton overshoots below the receiver for many
    cells and both sides replace such iterates by the midpoint towards the
    receiver (Algorithm 6 with the safeguard); 300x260 spans several tiles."""
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=300, nx=260, m=0.5, dt=5e4, K=4e-5, U=1e-4)
    h0 = W.initial_heights(w.ny, w.nx, 34) * 30.0
    print("[gpu] newton n=0.5 overshoot 300x260 6 steps", flush=True)
    got, r = _gpu(torch, w, 0.5, h0, 6, eps=1e-13, max_newton=200)
    ref = oracle.run(h0, _params(w, w.ny, w.nx, 0.5, 1e-13, 200), 6)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])
