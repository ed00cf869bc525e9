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


_DY = (-1, -1, -1, 0, 0, 1, 1, 1)
_DX = (-1, 0, 1, -1, 1, -1, 0, 1)


def test_mfd_full_size_conservation_and_sampled_cells():
    """The 10000 x 10000 benchmark grid, second step: all drainage area ends
    at cells without receivers, and 2000 sampled cells have exactly the
    level, drainage area and new height that the definitions give from their
    neighbours' exported values (levels and areas bit for bit; heights within
    1e-12, since m = 0.45 goes through each platform's pow)."""
    torch = require_gpu()
    from paper_1803_02977_amd import MfdSolver
    w = W.LARGE_10000
    ny, nx = w.ny, w.nx
    dev = torch.device("cuda:0")
    print("[gpu] mfd 10000x10000 two steps, conservation and samples", flush=True)
    h = torch.from_numpy(W.initial_heights(ny, nx, 0)).to(dev)
    s = MfdSolver(ny, nx, w.dx, w.dy, w.dt, w.m, w.U, w.K, device=dev)
    s.run(h, 1)
    s.sync()
    hs = h.cpu().numpy()  # heights at the start of the checked step
    s.run(h, 1)
    s.sync()
    e = s.export()
    area = e["area"].cpu().numpy()
    lev = e["level"].cpu().numpy()
    hn = h.cpu().numpy()
    nlevels = e["nlevels"]
    s.close()

    # Cells with at least one strictly lower neighbour (interior cells only).
    inner = hs[1:-1, 1:-1]
    lower = np.zeros(inner.shape, bool)
    for dy, dx in zip(_DY, _DX):
        lower |= inner - hs[1 + dy:ny - 1 + dy, 1 + dx:nx - 1 + dx] > 0.0
    sink = np.ones((ny, nx), bool)
    sink[1:-1, 1:-1] = ~lower
    del lower, inner
    total = float(np.sum(area[sink], dtype=np.float64))
    assert abs(total - ny * nx * w.dx * w.dy) <= 1e-9 * ny * nx * w.dx * w.dy
    assert nlevels == int(lev.max()) + 1
    assert np.all(lev[sink] == 0)

    dd = float(np.sqrt(w.dx * w.dx + w.dy * w.dy))
    dist = [dd if (_DY[k] and _DX[k]) else (w.dy if _DY[k] else w.dx) for k in range(8)]

    def interior(y, x):
        return 0 < y < ny - 1 and 0 < x < nx - 1

    def receivers(y, x):
        if not interior(y, x):
            return []
        return [k for k in range(8) if float(hs[y, x]) - float(hs[y + _DY[k], x + _DX[k]]) > 0.0]

    def wsum(y, x):
        t = 0.0
        for k in receivers(y, x):
            t += (float(hs[y, x]) - float(hs[y + _DY[k], x + _DX[k]])) / dist[k]
        return t

    rng = np.random.default_rng(17)
    ys = rng.integers(0, ny, 2000)
    xs = rng.integers(0, nx, 2000)
    ys[:8] = [0, ny - 1, 0, ny - 1, 0, 5, ny - 1, 7]  # a few perimeter cells
    xs[:8] = [0, nx - 1, 9, 11, nx - 1, 0, 3, nx - 1]
    dxdy, udt, kdt = w.dx * w.dy, w.U * w.dt, w.K * w.dt
    for y, x in zip(ys.tolist(), xs.tolist()):
        hc = float(hs[y, x])
        rec = receivers(y, x)
        want_level = 1 + max(int(lev[y + _DY[k], x + _DX[k]]) for k in rec) if rec else 0
        assert lev[y, x] == want_level, (y, x)
        acc = dxdy
        for k in range(8):
            yy, xx = y + _DY[k], x + _DX[k]
            if not interior(yy, xx):
                continue
            hd = float(hs[yy, xx])
            if hd - hc > 0.0:
                acc += ((hd - hc) / dist[k]) / wsum(yy, xx) * float(area[yy, xx])
        assert area[y, x] == acc, (y, x, float(area[y, x]), acc)
        if not interior(y, x):
            assert hn[y, x] == hs[y, x]
            continue
        hup = hc + udt
        if not rec:
            want = hup
        else:
            wc, ac = wsum(y, x), float(area[y, x])
            sumf = sumfh = 0.0
            for k in rec:
                yy, xx = y + _DY[k], x + _DX[k]
                share = ((hc - float(hs[yy, xx])) / dist[k]) / wc
                f = (kdt * (share * ac) ** w.m) / dist[k]
                sumf += f
                sumfh += f * float(hn[yy, xx])
            want = (hup + sumfh) / (1.0 + sumf)
        assert abs(float(hn[y, x]) - want) <= 1e-12 * max(abs(want), 1.0), (y, x)
