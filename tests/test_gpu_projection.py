"""GPU: steady-state projections (an accelerator of runs to steady state, not
a step of the paper's method) through the C ABI against the oracle's, and
what they are for: once projections stop changing the heights, the method's
own steps confirm a steady state almost at once."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_util import assert_heights_close, require_gpu

pytestmark = pytest.mark.gpu


def _grids():
    # Ragged sizes, several tiles, a K and a U field, n = 1 and n = 1.5.
    spec = [(64, 64, 0.5, 1.0), (130, 200, 0.45, 1.0), (97, 61, 0.5, 1.5), (200, 170, 0.4, 1.0)]
    out = []
    for i, (ny, nx, m, n) in enumerate(spec):
        out.append(dict(ny=ny, nx=nx, dx=100.0, dy=80.0 if i == 1 else 100.0, dt=1e4, m=m, n=n,
                        U=3e-4 * (1 + i), K=1e-5 * (1 + 0.4 * i), seed=90 + i))
    return out


def _batch(torch, specs):
    from paper_1803_02977_amd import Batch
    return Batch(specs, device=torch.device("cuda:0"), tuning=None)


def _fields(specs):
    rng = np.random.default_rng(3)
    h0 = [W.initial_heights(d["ny"], d["nx"], d["seed"]) * 5.0 for d in specs]
    K = [d["K"] * np.exp(0.5 * rng.standard_normal((d["ny"], d["nx"]))) for d in specs]
    U = [rng.uniform(0.5, 1.5) * d["U"] * np.ones((d["ny"], d["nx"])) for d in specs]
    return h0, K, U


def test_projections_match_oracle():
    torch = require_gpu()
    specs = _grids()
    h0, K, U = _fields(specs)
    cat = lambda xs: torch.from_numpy(np.concatenate([x.ravel() for x in xs])).to("cuda:0")
    for iters in (1, 6):
        print(f"[gpu] projection x{iters} against the oracle", flush=True)
        b = _batch(torch, specs)
        h, Kd, Ud = cat(h0), cat(K), cat(U)
        got = b.project_to_steady(h, rtol=1e-300, check_every=iters, max_iters=iters, K=Kd, U=Ud)
        b.sync()
        assert np.all(got == -1)
        out = h.cpu().numpy()
        b.close()
        off = 0
        for i, d in enumerate(specs):
            p = oracle.Params(d["ny"], d["nx"], d["dx"], d["dy"], d["dt"], d["m"], d["n"], 0.0,
                              d["K"])
            ref = oracle.project(h0[i], p, iters, K=K[i], U=U[i])
            cells = d["ny"] * d["nx"]
            rtol = 1e-12 if d["n"] == 1.0 else 1e-11
            assert_heights_close(out[off:off + cells].reshape(d["ny"], d["nx"]), ref["h"], rtol,
                                 what=f"grid {i} after {iters}")
            off += cells


def test_projection_then_steps_reach_steady_state():
    """Projections from noise to a fixed point, then the method's own steps:
    every grid is confirmed steady at the first check."""
    torch = require_gpu()
    specs = [dict(ny=128, nx=128, dx=100.0, dy=100.0, dt=1e4, m=0.5, n=1.0, U=5e-4, K=1e-5,
                  seed=7),
             dict(ny=96, nx=160, dx=100.0, dy=100.0, dt=1e4, m=0.45, n=1.0, U=1e-3, K=2e-5,
                  seed=8)]
    b = _batch(torch, specs)
    h = torch.from_numpy(np.concatenate([W.initial_heights(d["ny"], d["nx"], d["seed"]).ravel()
                                         for d in specs])).to("cuda:0")
    its = b.project_to_steady(h, rtol=1e-6, check_every=1, max_iters=2000)
    assert np.all(its > 0), its
    steps = b.run_to_steady(h, rtol=1e-6, check_every=1, max_steps=50)
    print(f"[gpu] projections {its.tolist()}, then steps {steps.tolist()}", flush=True)
    assert np.all((steps >= 0) & (steps <= 2)), steps
    b.close()


def test_projection_rejected_on_multiple_flow_directions():
    torch = require_gpu()
    from paper_1803_02977_amd import LemError, MfdSolver, lem
    s = MfdSolver(32, 32, device=torch.device("cuda:0"))
    h = torch.zeros(32 * 32, dtype=torch.float64, device="cuda:0")
    with pytest.raises(LemError):
        lem.lem_batch_project_to_steady(s.ctx, h.data_ptr(), None, None, 1e-6, 1, 1, 1)
    s.close()
