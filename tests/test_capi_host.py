"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/lem.h declares, and rejects bad arguments before it
touches the device."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import torch

import pytest

import paper_1803_02977_amd as pkg
from paper_1803_02977_amd import lem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(lem_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    names = declared_entry_points()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), f"{n} is declared but not exported"
    assert set(names) >= set(lem.EXPORTS)


def _params(**kw):
    base = dict(ny=256, nx=256, dx=100.0, dy=100.0, dt=1000.0, m=0.5, n=1.0, U=5e-4, K=1e-5,
                eps=1e-12, max_newton=100, flags=0)
    base.update(kw)
    return lem.lem_params(**base)


def test_slope_exponent_is_accepted_with_a_tolerance():
    assert lem.lem_workspace_bytes(_params(n=2.0)) > 0
    assert lem.lem_workspace_bytes(_params(n=0.7, eps=1e-9, max_newton=5)) > 0
    # n = 1 ignores eps and max_newton (closed form).
    assert lem.lem_workspace_bytes(_params(eps=0.0, max_newton=0)) > 0


def test_workspace_bytes():
    small = lem.lem_workspace_bytes(_params())
    big = lem.lem_workspace_bytes(_params(ny=2048, nx=2048))
    assert small > 256 * 256 * 20
    assert big > small
    assert (big - small) / (2048 * 2048 - 256 * 256) < 64


@pytest.mark.parametrize("kw,status", [
    (dict(ny=2), lem.LEM_E_SIZE), (dict(nx=0), lem.LEM_E_SIZE),
    (dict(ny=50000, nx=50000), lem.LEM_E_SIZE),
    (dict(dx=0.0), lem.LEM_E_ARG), (dict(dy=-1.0), lem.LEM_E_ARG),
    (dict(dt=float("nan")), lem.LEM_E_ARG), (dict(m=-0.1), lem.LEM_E_ARG),
    (dict(n=0.0), lem.LEM_E_ARG), (dict(n=float("nan")), lem.LEM_E_ARG),
    (dict(n=2.0, eps=0.0), lem.LEM_E_ARG), (dict(n=2.0, max_newton=0), lem.LEM_E_ARG),
    (dict(K=-1e-5), lem.LEM_E_ARG),
    (dict(U=float("inf")), lem.LEM_E_ARG), (dict(flags=0x80), lem.LEM_E_ARG),
])
def test_bad_parameters_are_rejected_on_the_host(kw, status):
    p = _params(**kw)
    assert lem.lem_workspace_bytes(p) == 0
    lib = pkg.load()
    ctx = C.c_void_p()
    assert lib.lem_create(C.byref(p), C.c_void_p(1 << 20), 1 << 40, None, C.byref(ctx)) == status
    assert ctx.value is None


def test_workspace_is_checked_before_the_device():
    lib = pkg.load()
    p = _params()
    need = lem.lem_workspace_bytes(p)
    ctx = C.c_void_p()
    assert lib.lem_create(C.byref(p), None, need, None, C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_create(C.byref(p), C.c_void_p(4096 + 8), need, None,
                          C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_create(C.byref(p), C.c_void_p(4096), need - 1, None,
                          C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_create(C.byref(p), C.c_void_p(4096), need, None, None) == lem.LEM_E_ARG


def test_null_context_calls():
    lib = pkg.load()
    assert lib.lem_run(None, None, None, None, 1) == lem.LEM_E_ARG
    assert lib.lem_sync(None) == lem.LEM_E_ARG
    assert lib.lem_destroy(None) == lem.LEM_OK
    assert lib.lem_last_error(None) == b""
    for s in range(8):
        assert lib.lem_status_str(s).startswith(b"LEM_")


def test_surrogate_layer_table_matches_the_reference_network():
    from oracle import surrogate as S
    from paper_1803_02977_amd import surrogate as sur
    layout, total = S.param_layout()
    assert sur.param_count() == total
    for i, (name, cin, cout) in enumerate(S.layer_table()):
        assert sur.layer(i) == (cin, cout, layout[name][0]), name
    assert sur.layer(14) == (32, 1, layout["head"][0])
    with pytest.raises(lem.LemError):
        sur.layer(15)


@pytest.mark.parametrize("shape", [(0, 64, 64), (1, 60, 64), (1, 64, 4), (2, 7, 8)])
def test_surrogate_shapes_are_checked_on_the_host(shape):
    from paper_1803_02977_amd import surrogate as sur
    assert sur.workspace_bytes(*shape) == 0
    lib = sur.load()
    ctx = C.c_void_p()
    assert lib.lem_sur_create(*shape, C.c_void_p(4096), 1 << 40, None, C.byref(ctx)) == lem.LEM_E_SIZE


def test_surrogate_workspace_is_checked_before_the_device():
    from paper_1803_02977_amd import surrogate as sur
    lib = sur.load()
    need = sur.workspace_bytes(2, 64, 64)
    assert need > 0
    ctx = C.c_void_p()
    assert lib.lem_sur_create(2, 64, 64, None, need, None, C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_sur_create(2, 64, 64, C.c_void_p(4096 + 8), need, None,
                              C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_sur_create(2, 64, 64, C.c_void_p(4096), need - 1, None,
                              C.byref(ctx)) == lem.LEM_E_WORKSPACE


def test_surrogate_parameters_round_trip_through_storage(tmp_path):
    from paper_1803_02977_amd import surrogate as sur
    p = sur.init_params(3)
    p[sur.bias_mask()] = np.linspace(-1, 1, int(sur.bias_mask().sum()), dtype=np.float32)
    sur.save_params(str(tmp_path / "w.npz"), p)
    q = sur.load_params(str(tmp_path / "w.npz"))
    m = sur.bias_mask()
    assert np.array_equal(q[m], p[m])
    assert np.array_equal(q[~m], torch.from_numpy(p[~m]).to(torch.bfloat16).float().numpy())


def test_stored_warm_start_weights_have_the_network_shape():
    from paper_1803_02977_amd import surrogate as sur, warmstart as WS
    p = sur.load_params(WS.WEIGHTS_PATH)
    assert p.shape == (sur.param_count(),) and np.all(np.isfinite(p))


def test_mfd_workspace_and_arguments_are_checked_on_the_host():
    p = _params()
    d8 = lem.lem_workspace_bytes(p)
    mfd = lem.lem_mfd_workspace_bytes(p)
    assert mfd >= d8 + 8 * 256 * 256  # one more FP64 array per cell
    assert lem.lem_mfd_workspace_bytes(_params(n=2.0)) == 0
    lib = pkg.load()
    ctx = C.c_void_p()
    for exponent in (0.0, -1.0, float("nan"), float("inf")):
        assert lib.lem_mfd_create(C.byref(p), exponent, C.c_void_p(1 << 20), 1 << 40, None,
                                  C.byref(ctx)) == lem.LEM_E_ARG
    q = _params(n=2.0)
    assert lib.lem_mfd_create(C.byref(q), 1.0, C.c_void_p(1 << 20), 1 << 40, None,
                              C.byref(ctx)) == lem.LEM_E_ARG
    assert lib.lem_mfd_create(C.byref(p), 1.0, C.c_void_p(4096), mfd - 1, None,
                              C.byref(ctx)) == lem.LEM_E_WORKSPACE
    assert lib.lem_mfd_export(None, None, None, None) == lem.LEM_E_ARG


def test_static_entry_point_rejects_oversized_grids_on_the_host():
    """lem_run_static checks the grid against its fixed workspace before any
    device call (the heights pointer is never used here)."""
    from paper_1803_02977_amd import lem
    lib = lem.load()
    big = lem.lem_params(1024, 1024, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 1e-5, 1e-12, 100, 0)
    assert lem.lem_workspace_bytes(big) > lem.LEM_STATIC_WORKSPACE_BYTES
    assert lib.lem_run_static(C.byref(big), 256, None, None, 1, None) == lem.LEM_E_WORKSPACE
    fits = lem.lem_params(512, 512, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 1e-5, 1e-12, 100, 0)
    assert lem.lem_workspace_bytes(fits) <= lem.LEM_STATIC_WORKSPACE_BYTES
    bad = lem.lem_params(2, 512, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 1e-5, 1e-12, 100, 0)
    assert lib.lem_run_static(C.byref(bad), 256, None, None, 1, None) == lem.LEM_E_ARG
    timers = lem.lem_params(64, 64, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 1e-5, 1e-12, 100,
                            lem.LEM_F_PHASE_TIMERS)
    assert lib.lem_run_static(C.byref(timers), 256, None, None, 1, None) == lem.LEM_E_ARG
    clocks = lem.lem_params(64, 64, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 1e-5, 1e-12, 100,
                            lem.LEM_F_TILE_CLOCKS)
    assert lib.lem_run_static(C.byref(clocks), 256, None, None, 1, None) == lem.LEM_E_ARG
    assert lib.lem_run_static(None, 256, None, None, 1, None) == lem.LEM_E_ARG
