"""Helpers for the GPU parity tests (inputs from ``workloads``, oracle on CPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

# Heights: |h_gpu - h_oracle| <= 1e-12 * max(|h_oracle|, 1 m).
H_RTOL = 1e-12


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_params(w, ny=None, nx=None):
    return oracle.Params(ny or w.ny, nx or w.nx, w.dx, w.dy, w.dt, w.m, 1.0, w.U, w.K)


def assert_heights_close(got, ref, rtol=H_RTOL, what="h"):
    tol = rtol * np.maximum(np.abs(ref), 1.0)
    err = np.abs(got - ref)
    bad = err > tol
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {int(bad.sum())} cells out of tolerance; first {idx.tolist()}"
                             f" max err {float(err.max()):.3e}")


def assert_routing_equal(r, ref):
    rec = r["rec"].cpu().numpy()
    depth = r["depth"].cpu().numpy()
    count = r["count"].cpu().numpy().view(np.uint32)
    assert np.array_equal(rec, ref["rec"]), f"receivers differ at {np.argwhere(rec != ref['rec'])[:5].tolist()}"
    assert np.array_equal(depth, ref["depth"]), f"levels differ at {np.argwhere(depth != ref['depth'])[:5].tolist()}"
    assert np.array_equal(count, ref["count"]), f"counts differ at {np.argwhere(count != ref['count'])[:5].tolist()}"
    assert r["nlevels"] == ref["nlevels"]
    assert np.array_equal(np.asarray(r["offsets"]), ref["offsets"])
