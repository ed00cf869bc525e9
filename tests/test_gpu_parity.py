"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Receivers, levels, level offsets and drainage counts must be bit-exact; FP64
heights must agree within 1e-12 relative (1 m floor).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, assert_routing_equal, oracle_params, require_gpu

pytestmark = pytest.mark.gpu


def _run_gpu(torch, w, h0, steps, K=None, U=None, ny=None, nx=None):
    from paper_1803_02977_amd import Solver
    ny = ny or w.ny
    nx = nx or w.nx
    dev = torch.device("cuda:0")
    h = torch.from_numpy(np.ascontiguousarray(h0)).to(dev)
    Kt = None if K is None else torch.from_numpy(K).to(dev)
    Ut = None if U is None else torch.from_numpy(U).to(dev)
    s = Solver(ny, nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev)
    s.run(h, steps, K=Kt, U=Ut)
    s.sync()
    r = s.routing()
    out = h.cpu().numpy()
    s.close()
    return out, r


@pytest.mark.parametrize("steps", [1, 2, 10])
def test_small_grid_steps(steps):
    torch = require_gpu()
    w = W.SMALL_256
    h0 = W.initial_heights(w.ny, w.nx, 0)
    print(f"[gpu] 256x256 seed 0 steps {steps}", flush=True)
    got, r = _run_gpu(torch, w, h0, steps)
    ref = oracle.run(h0, oracle_params(w), steps)
    assert_routing_equal(r, ref)
    assert_heights_close(got, ref["h"])
