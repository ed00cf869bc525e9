"""GPU: multiple-flow-direction routing (lem_mfd_create) against the oracle's
height-ordered implementation on the same seeded inputs.

Levels (longest path to a root) must be identical.  With shares in
proportion to the slope (exponent 1) and m = 0.5 both sides perform the same
correctly rounded operations in the same order, so areas and heights must be
bit-identical; other exponents and m go through each platform's pow, so
areas and heights are compared within 1e-13 and 1e-12 relative.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, require_gpu

pytestmark = pytest.mark.gpu


def _gpu(torch, h0, steps, dx=100.0, dy=100.0, dt=1000.0, m=0.5, U=5e-4, K=1e-5, exponent=1.0,
         Kf=None, Uf=None):
    from paper_1803_02977_amd import MfdSolver
    ny, nx = h0.shape
    dev = torch.device("cuda:0")
    h = torch.from_numpy(np.ascontiguousarray(h0)).to(dev)
    s = MfdSolver(ny, nx, dx, dy, dt, m, U, K, exponent=exponent, device=dev)
    s.run(h, steps, K=None if Kf is None else torch.from_numpy(Kf).to(dev),
          U=None if Uf is None else torch.from_numpy(Uf).to(dev))
    s.sync()
    e = s.export()
    out = (h.cpu().numpy(), e["area"].cpu().numpy(), e["level"].cpu().numpy(), e["nlevels"])
    s.close()
    return out


def _ref(h0, steps, dx=100.0, dy=100.0, dt=1000.0, m=0.5, U=5e-4, K=1e-5, exponent=1.0,
         Kf=None, Uf=None):
    ny, nx = h0.shape
    p = oracle.Params(ny, nx, dx, dy, dt, m, 1.0, U, K)
    return oracle.mfd_run(h0, p, steps, pexp=exponent, K=Kf, U=Uf)


@pytest.mark.parametrize("steps", [1, 5, 20])
def test_mfd_bit_identical_to_oracle(steps):
    torch = require_gpu()
    h0 = W.initial_heights(150, 170, 3)
    print(f"[gpu] mfd 150x170 steps {steps}", flush=True)
    h, area, level, nl = _gpu(torch, h0, steps)
    ref = _ref(h0, steps)
    assert np.array_equal(level, ref["level"]) and nl == ref["nlevels"]
    assert np.array_equal(area, ref["area"])
    assert np.array_equal(h, ref["h"])


@pytest.mark.parametrize("shape", [(3, 3), (5, 7), (64, 200), (129, 65)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("kind", ["uniform", "ties"])
def test_mfd_ragged_grids_and_ties(shape, kind):
    torch = require_gpu()
    ny, nx = shape
    h0 = (W.initial_heights(ny, nx, 11) if kind == "uniform"
          else W.quantised_heights(ny, nx, 4, seed=11))
    print(f"[gpu] mfd {ny}x{nx} {kind}", flush=True)
    h, area, level, nl = _gpu(torch, h0, 4)
    ref = _ref(h0, 4)
    assert np.array_equal(level, ref["level"]) and nl == ref["nlevels"]
    assert np.array_equal(area, ref["area"])
    assert np.array_equal(h, ref["h"])


def test_mfd_exponent_fields_and_rectangular_cells():
    torch = require_gpu()
    h0 = W.initial_heights(97, 131, 7) * 5.0
    rng = np.random.default_rng(8)
    Kf = 1e-5 * np.exp(0.5 * rng.standard_normal(h0.shape))
    Uf = rng.uniform(1e-4, 2e-3, h0.shape)
    kw = dict(dx=30.0, dy=45.0, m=0.45, exponent=1.3, Kf=Kf, Uf=Uf)
    h, area, level, nl = _gpu(torch, h0, 12, **kw)
    ref = _ref(h0, 12, **kw)
    assert np.array_equal(level, ref["level"]) and nl == ref["nlevels"]
    assert np.allclose(area, ref["area"], rtol=1e-13, atol=0)
    assert_heights_close(h, ref["h"])


@pytest.mark.parametrize("kind", ["cone", "ramp-north", "ramp-west", "ramp-south-east"])
def test_mfd_long_paths_across_many_tiles(kind):
    """Flow paths of a few hundred cells that cross many tiles, including
    ramps whose areas must travel against the order in which tiles are
    visited: every cell still gets the oracle's value."""
    torch = require_gpu()
    ny, nx = 203, 261
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    base = {"cone": np.minimum(np.minimum(yy, ny - 1 - yy), np.minimum(xx, nx - 1 - xx)),
            "ramp-north": yy, "ramp-west": xx, "ramp-south-east": (ny - 1 - yy) + (nx - 1 - xx)}[kind]
    rng = np.random.default_rng(21)
    h0 = 0.5 * base + rng.uniform(0.0, 0.01, (ny, nx))
    h0[0, :] = h0[-1, :] = h0[:, 0] = h0[:, -1] = 0.0
    print(f"[gpu] mfd {kind} {ny}x{nx}", flush=True)
    h, area, level, nl = _gpu(torch, h0, 3)
    ref = _ref(h0, 3)
    assert ref["nlevels"] > 90
    assert np.array_equal(level, ref["level"]) and nl == ref["nlevels"]
    assert np.array_equal(area, ref["area"])
    assert np.array_equal(h, ref["h"])


def test_mfd_large_grid_and_determinism():
    torch = require_gpu()
    h0 = W.initial_heights(1024, 1536, 5)
    print("[gpu] mfd 1024x1536 3 steps", flush=True)
    a = _gpu(torch, h0, 3)
    b = _gpu(torch, h0, 3)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))
    ref = _ref(h0, 3)
    assert np.array_equal(a[2], ref["level"])
    assert np.array_equal(a[1], ref["area"])
    assert np.array_equal(a[0], ref["h"])


def test_mfd_context_rejects_d8_only_calls():
    torch = require_gpu()
    from paper_1803_02977_amd import LemError, MfdSolver, lem
    s = MfdSolver(40, 50, device=torch.device("cuda:0"))
    with pytest.raises(LemError):
        s.export()  # no step yet
    h = torch.from_numpy(W.initial_heights(40, 50, 1)).to("cuda:0")
    s.run(h, 2)
    s.sync()
    with pytest.raises(LemError):
        lem.lem_routing(s.ctx, None, None, None, 0)
    s.close()
