"""GPU: fixed routing (1-D channel, cycles, bad codes), input validation."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, oracle_params, require_gpu

pytestmark = pytest.mark.gpu

# Receiver code of each neighbour offset (dy, dx).
CODE = {(-1, -1): 0, (-1, 0): 1, (-1, 1): 2, (0, -1): 3, (0, 1): 4, (1, -1): 5, (1, 0): 6,
        (1, 1): 7}


def _solver(torch, w, flags=0):
    from paper_1803_02977_amd import Solver
    return Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, flags=flags,
                  device=torch.device("cuda:0"))


def _codes_from_rec(rec):
    ny, nx = rec.shape
    codes = np.full((ny, nx), 8, np.uint8)
    for y in range(ny):
        for x in range(nx):
            r = rec[y, x]
            if r != y * nx + x:
                codes[y, x] = CODE[(r // nx - y, r % nx - x)]
    return codes


def test_fixed_routing_channel_matches_oracle():
    """A 1-D channel: every interior cell of the middle row drains left."""
    torch = require_gpu()
    w = W.SMALL_256.with_(ny=3, nx=300)
    rec = np.arange(w.ny * w.nx, dtype=np.int32).reshape(w.ny, w.nx)
    for x in range(1, w.nx - 1):
        rec[1, x] = w.nx + x - 1
    h0 = W.initial_heights(w.ny, w.nx, 2)
    ref = oracle.run_fixed_routing(h0, rec, oracle_params(w), 40)
    h = torch.from_numpy(h0).to("cuda:0")
    s = _solver(torch, w)
    s.run_fixed_routing(h, torch.from_numpy(_codes_from_rec(rec)).to("cuda:0"), 40)
    s.sync()
    r = s.routing()
    assert np.array_equal(r["depth"].cpu().numpy(), ref["depth"])
    assert np.array_equal(r["count"].cpu().numpy().view(np.uint32), ref["count"])
    assert_heights_close(h.cpu().numpy(), ref["h"])
    # m = 0.5 uses a correctly rounded square root on both sides: bit-exact.
    assert np.array_equal(h.cpu().numpy(), ref["h"])
    s.close()


def test_fixed_routing_spiral_is_one_deep_chain():
    """Every interior cell in one chain: as many levels as interior cells."""
    torch = require_gpu()
    ny, nx = 12, 14
    w = W.SMALL_256.with_(ny=ny, nx=nx)
    path = []
    top, bot, lef, rig = 1, ny - 2, 1, nx - 2
    while top <= bot and lef <= rig:
        path += [(top, x) for x in range(lef, rig + 1)]
        path += [(y, rig) for y in range(top + 1, bot + 1)]
        if top < bot:
            path += [(bot, x) for x in range(rig - 1, lef - 1, -1)]
        if lef < rig:
            path += [(y, lef) for y in range(bot - 1, top, -1)]
        top, bot, lef, rig = top + 1, bot - 1, lef + 1, rig - 1
    rec = np.arange(ny * nx, dtype=np.int32).reshape(ny, nx)
    rec[path[0]] = 0 * nx + 1  # the first cell drains to the perimeter
    for a, b in zip(path[1:], path[:-1]):
        rec[a] = b[0] * nx + b[1]
    h0 = W.initial_heights(ny, nx, 3)
    ref = oracle.run_fixed_routing(h0, rec, oracle_params(w), 3)
    h = torch.from_numpy(h0).to("cuda:0")
    s = _solver(torch, w)
    s.run_fixed_routing(h, torch.from_numpy(_codes_from_rec(rec)).to("cuda:0"), 3)
    s.sync()
    r = s.routing()
    assert r["nlevels"] == len(path) + 1
    assert np.array_equal(r["depth"].cpu().numpy(), ref["depth"])
    assert np.array_equal(r["count"].cpu().numpy().view(np.uint32), ref["count"])
    assert_heights_close(h.cpu().numpy(), ref["h"])
    s.close()


def test_fixed_routing_cycle_is_reported():
    torch = require_gpu()
    from paper_1803_02977_amd import LEM_E_CYCLE, LemError
    w = W.SMALL_256.with_(ny=6, nx=6)
    codes = np.full((6, 6), 8, np.uint8)
    codes[2, 2] = CODE[(0, 1)]   # (2,2) -> (2,3)
    codes[2, 3] = CODE[(0, -1)]  # (2,3) -> (2,2)
    h = torch.from_numpy(W.initial_heights(6, 6, 0)).to("cuda:0")
    s = _solver(torch, w)
    s.run_fixed_routing(h, torch.from_numpy(codes).to("cuda:0"), 1)
    with pytest.raises(LemError) as e:
        s.sync()
    assert e.value.status == LEM_E_CYCLE
    s.sync()  # the error was cleared
    s.close()


def test_fixed_routing_bad_code_is_reported():
    torch = require_gpu()
    from paper_1803_02977_amd import LEM_E_ARG, LemError
    w = W.SMALL_256.with_(ny=6, nx=6)
    codes = np.full((6, 6), 8, np.uint8)
    codes[0, 3] = CODE[(1, 0)]  # a perimeter cell may not have a receiver
    codes[3, 3] = 200           # not a code
    h = torch.from_numpy(W.initial_heights(6, 6, 0)).to("cuda:0")
    s = _solver(torch, w)
    s.run_fixed_routing(h, torch.from_numpy(codes).to("cuda:0"), 1)
    with pytest.raises(LemError) as e:
        s.sync()
    assert e.value.status == LEM_E_ARG
    s.close()


def test_validate_rejects_non_finite_inputs_and_leaves_h_untouched():
    torch = require_gpu()
    from paper_1803_02977_amd import LEM_E_NONFINITE, LEM_F_VALIDATE, LemError
    w = W.SMALL_256.with_(ny=50, nx=60)
    h0 = W.initial_heights(50, 60, 0)
    h0[20, 30] = np.nan
    h = torch.from_numpy(h0).to("cuda:0")
    s = _solver(torch, w, flags=LEM_F_VALIDATE)
    with pytest.raises(LemError) as e:
        s.run(h, 3)
    assert e.value.status == LEM_E_NONFINITE
    assert np.array_equal(h.cpu().numpy(), h0, equal_nan=True)
    K = np.full((50, 60), 1e-5)
    K[1, 1] = np.inf
    h0[20, 30] = 0.5
    h = torch.from_numpy(h0).to("cuda:0")
    with pytest.raises(LemError):
        s.run(h, 3, K=torch.from_numpy(K).to("cuda:0"))
    s.run(h, 3)
    s.sync()
    s.close()


def test_argument_errors_on_the_device_path():
    torch = require_gpu()
    from paper_1803_02977_amd import LemError, lem
    w = W.SMALL_256.with_(ny=20, nx=20)
    s = _solver(torch, w)
    h = torch.zeros((20, 21), dtype=torch.float64, device="cuda:0")
    with pytest.raises(LemError):
        s.run(h, 1)
    with pytest.raises(LemError):
        lem.lem_run(s.ctx, None, None, None, 1)
    with pytest.raises(LemError):
        lem.lem_run(s.ctx, torch.zeros((20, 20), dtype=torch.float64, device="cuda:0").data_ptr(),
                    None, None, -1)
    s.close()
