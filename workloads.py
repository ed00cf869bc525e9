"""Seeded synthetic inputs for the landscape-evolution workloads.

Shared by the tests, the benchmark, the GPU library's users and the oracle's
callers.  It holds no arithmetic of the method: it only draws the initial
heights and the parameter fields.  The paper's test data are square rasters
whose cells are drawn uniformly from [0, 1] with a fixed seed (section "Test
Data"); the perimeter is the fixed base level (section "The Equation"), so it
is set to 0 here.  Random numbers come from NumPy's PCG64 ``default_rng``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One configuration: grid, cell size, time step, exponents, U, K, steps."""
    name: str
    ny: int
    nx: int
    dx: float
    dy: float
    dt: float
    m: float
    U: float
    K: float
    steps: int
    n: float = 1.0
    k_lognormal_sigma: Optional[float] = None  # per-cell K = K * exp(sigma * N(0,1))
    seeds: tuple = field(default=(0,))

    @property
    def cells(self) -> int:
        return self.ny * self.nx

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# 256 x 256, 100 m cells, scalar U and K, m = 0.5, dt = 1000 yr, 100 steps.
SMALL_256 = Workload("plain-256x256-fp64", 256, 256, 100.0, 100.0, 1000.0, 0.5, 5e-4, 1e-5,
                     100, seeds=tuple(range(10)))
# 2048 x 2048, 100 m cells, lognormal K per cell (median 1e-5, sigma_ln 0.5), 200 steps.
MEDIUM_2048 = Workload("plain-2048x2048-fp64-lognormalK", 2048, 2048, 100.0, 100.0, 1000.0,
                       0.5, 5e-4, 1e-5, 200, k_lognormal_sigma=0.5)
# 10000 x 10000 (1e8 cells), 30 m cells, U = 1e-3, K = 2e-5, m = 0.45, dt = 500, 50 steps.
LARGE_10000 = Workload("plain-10000x10000-fp64", 10000, 10000, 30.0, 30.0, 500.0, 0.45, 1e-3,
                       2e-5, 50)

WORKLOADS = {w.name: w for w in (SMALL_256, MEDIUM_2048, LARGE_10000)}


def initial_heights(ny: int, nx: int, seed: int = 0) -> np.ndarray:
    """Uniform[0,1) heights from ``default_rng(seed)``, perimeter set to 0."""
    h = np.random.default_rng(seed).random((ny, nx))
    h[0, :] = 0.0
    h[-1, :] = 0.0
    h[:, 0] = 0.0
    h[:, -1] = 0.0
    return h


def k_field(w: Workload, seed: int = 0) -> Optional[np.ndarray]:
    """Per-cell erodibility, lognormal around ``w.K``, or None for scalar K."""
    if w.k_lognormal_sigma is None:
        return None
    z = np.random.default_rng(seed + 1).standard_normal((w.ny, w.nx))
    return w.K * np.exp(w.k_lognormal_sigma * z)


def make_inputs(w: Workload, seed: int = 0):
    """(h0, K field or None, U field or None) for workload ``w``."""
    return initial_heights(w.ny, w.nx, seed), k_field(w, seed), None


def quantised_heights(ny: int, nx: int, levels: int, seed: int) -> np.ndarray:
    """Heights drawn from {0, 1, ..., levels-1}: many exact ties and flats."""
    h = np.random.default_rng(seed).integers(0, levels, size=(ny, nx)).astype(np.float64)
    h[0, :] = 0.0
    h[-1, :] = 0.0
    h[:, 0] = 0.0
    h[:, -1] = 0.0
    return h


# Batched realizations: square sizes from {128, 192, ..., 1024}, per-realization
# K ~ logUniform[1e-6, 1e-4], U ~ Uniform[1e-4, 2e-3], m ~ Uniform[0.35, 0.6],
# dt = 1000 yr, 100 m cells, h0 ~ Uniform[0,1) with the perimeter at 0.
BATCH_SIZES = tuple(range(128, 1025, 64))


@dataclass(frozen=True)
class Realization:
    ny: int
    nx: int
    dx: float
    dy: float
    dt: float
    m: float
    U: float
    K: float
    seed: int


def batch_realizations(count: int = 512, seed: int = 0, sizes=BATCH_SIZES,
                       dx: float = 100.0, dt: float = 1000.0):
    """Draw ``count`` independent realizations (sizes and parameters)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = int(rng.choice(np.asarray(sizes)))
        k = float(10.0 ** rng.uniform(-6.0, -4.0))
        u = float(rng.uniform(1e-4, 2e-3))
        m = float(rng.uniform(0.35, 0.6))
        out.append(Realization(s, s, dx, dx, dt, m, u, k, seed * 100003 + i))
    return out


def batch_initial_heights(realizations) -> np.ndarray:
    """Initial heights of a batch, grid after grid (each from its own seed)."""
    return np.concatenate([initial_heights(r.ny, r.nx, r.seed).ravel() for r in realizations])


# Learned warm start: 256 x 256 grids, 100 m cells, m = 0.5, dt = 1000 yr,
# per-cell K lognormal (median 1e-5, sigma_ln 0.5), U ~ Uniform[1e-4, 2e-3]
# per grid (a uniform field), h0 ~ Uniform[0,1) with the perimeter at 0.
# Training realizations use seeds from WARMSTART_TRAIN_SEED, held-out ones
# from WARMSTART_TEST_SEED.
WARMSTART_SIDE = 256
WARMSTART_TRAIN_SEED = 1_000_000
WARMSTART_TEST_SEED = 9_000_000


def warmstart_inputs(count: int, first_seed: int, ny: int = WARMSTART_SIDE,
                     nx: int = WARMSTART_SIDE):
    """(K, U, h0), each float64 [count, ny, nx], for realizations
    first_seed, first_seed + 1, ...; realization s draws K and U from
    default_rng(s) and h0 from initial_heights(ny, nx, s)."""
    K = np.empty((count, ny, nx))
    U = np.empty((count, ny, nx))
    h0 = np.empty((count, ny, nx))
    for i in range(count):
        s = first_seed + i
        rng = np.random.default_rng(s)
        K[i] = 1e-5 * np.exp(0.5 * rng.standard_normal((ny, nx)))
        U[i] = rng.uniform(1e-4, 2e-3)
        h0[i] = initial_heights(ny, nx, s)
    return K, U, h0
