"""GPU: lem_run_static (no device allocation; its workspace is a device array
inside the library) gives the same heights as lem_run over a caller's
workspace, on two calls in a row, the second on a smaller grid with a K
field, and rejects a grid whose workspace does not fit the array."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _static(torch, lem, w, h0, steps, K=None):
    p = lem.lem_params(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K, 1e-12, 100, 0)
    h = torch.from_numpy(h0).to("cuda:0")
    Kt = None if K is None else torch.from_numpy(K).to("cuda:0")
    lem.lem_run_static(p, h.data_ptr(), None if Kt is None else Kt.data_ptr(), None, steps,
                       torch.cuda.current_stream().cuda_stream)
    return h.cpu().numpy()


def _ctx(torch, w, h0, steps, K=None):
    from paper_1803_02977_amd import Solver
    s = Solver(w.ny, w.nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=torch.device("cuda:0"))
    h = torch.from_numpy(h0).to("cuda:0")
    s.run(h, steps, K=None if K is None else torch.from_numpy(K).to("cuda:0"))
    s.sync()
    s.close()
    return h.cpu().numpy()


def test_static_workspace_run_equals_caller_workspace_run():
    torch = require_gpu()
    from paper_1803_02977_amd import lem
    cases = [(W.SMALL_256.with_(ny=512, nx=512), 7, None),
             (W.SMALL_256.with_(ny=200, nx=300, dx=30.0, dy=45.0, m=0.45), 5, "K")]
    for w, steps, kf in cases:
        h0 = W.initial_heights(w.ny, w.nx, 40 + w.ny) * 5.0
        K = None if kf is None else 1e-5 * np.exp(
            0.5 * np.random.default_rng(w.nx).standard_normal((w.ny, w.nx)))
        print(f"[gpu] lem_run_static {w.ny}x{w.nx} {steps} steps K field={kf}", flush=True)
        got = _static(torch, lem, w, h0, steps, K)
        ref = _ctx(torch, w, h0, steps, K)
        assert np.array_equal(got, ref), np.abs(got - ref).max()
    big = W.SMALL_256.with_(ny=1024, nx=1024)
    print("[gpu] lem_run_static 1024x1024 rejected", flush=True)
    with pytest.raises(lem.LemError) as e:
        _static(torch, lem, big, W.initial_heights(1024, 1024, 1), 1)
    assert e.value.status == lem.LEM_E_WORKSPACE
