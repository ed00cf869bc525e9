"""Serial CPU oracle of the landscape-evolution hot path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or runs anything in this package, and this package imports nothing from it.

The arithmetic lives in ``lem_oracle.c`` (plain serial C, FP64, built with
``-O2 -ffp-contract=off``, no fast-math); this module only compiles it and
marshals NumPy arrays through ctypes.  Every function cites the passage of
Barnes, "Accelerating a Landscape Evolution Model with Parallelism"
(arXiv:1803.02977) that it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "lem_oracle.c")
LIB_PATH = os.path.join(_HERE, "liblemoracle.so")

# Compiler flags: no contraction of a*b+c into FMA and no fast-math, so every
# expression rounds exactly as written.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]

LEMO_OK, LEMO_E_ARG, LEMO_E_ALLOC, LEMO_E_CYCLE = 0, 1, 2, 5


def build(source: str = SOURCE, out: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", *CFLAGS, *extra_flags, "-I", os.path.dirname(os.path.abspath(source)),
           source, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Params(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double),
                ("dy", C.c_double), ("dt", C.c_double), ("m", C.c_double),
                ("n", C.c_double), ("U", C.c_double), ("K", C.c_double),
                ("eps", C.c_double), ("max_newton", C.c_int32)]


_P = C.c_void_p


def _declare(lib):
    lib.lemo_receivers.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, _P, _P]
    lib.lemo_receivers.restype = None
    lib.lemo_donors.argtypes = [C.c_int32, C.c_int32, _P, _P, _P]
    lib.lemo_donors.restype = None
    lib.lemo_stack_order.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P]
    lib.lemo_stack_order.restype = C.c_int64
    lib.lemo_bfs_queue.argtypes = [C.c_int64, _P, _P, _P, _P, _P]
    lib.lemo_bfs_queue.restype = C.c_int64
    lib.lemo_graph_order.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.lemo_graph_order.restype = C.c_int64
    lib.lemo_run.argtypes = [C.POINTER(_Params), _P, _P, _P, C.c_int64, _P, _P, _P, _P,
                             C.c_int64, _P]
    lib.lemo_run.restype = C.c_int
    lib.lemo_run_fixed_routing.argtypes = [C.POINTER(_Params), _P, _P, _P, _P, C.c_int64,
                                           _P, _P]
    lib.lemo_project.argtypes = [C.POINTER(_Params), _P, _P, _P, C.c_int64, _P, _P, _P]
    lib.lemo_project.restype = C.c_int
    lib.lemo_run_fixed_routing.restype = C.c_int
    lib.lemo_routing.argtypes = [C.POINTER(_Params), _P, _P, _P, _P, _P, C.c_int64, _P]
    lib.lemo_mfd_run.argtypes = [C.POINTER(_Params), C.c_double, _P, _P, _P, C.c_int64, _P, _P,
                                 _P]
    lib.lemo_mfd_run.restype = C.c_int
    lib.lemo_routing.restype = C.c_int
    return lib


_LIB = None


def load(path: str = LIB_PATH):
    """Load the compiled oracle (building it first only if it is missing)."""
    global _LIB
    if path == LIB_PATH and _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        build(out=path)
    lib = _declare(C.CDLL(path))
    if path == LIB_PATH:
        _LIB = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Params:
    """Problem statement: grid, cell size, time step, exponents, U and K."""
    ny: int
    nx: int
    dx: float = 100.0
    dy: float = 100.0
    dt: float = 1000.0
    m: float = 0.5
    n: float = 1.0
    U: float = 5e-4
    K: float = 1e-5
    eps: float = 1e-12
    max_newton: int = 100

    def c(self) -> _Params:
        return _Params(self.ny, self.nx, self.dx, self.dy, self.dt, self.m, self.n,
                       self.U, self.K, self.eps, self.max_newton)


def receivers(h, dx=100.0, dy=100.0, lib=None):
    """Step 2, Algorithm 1: receiver index of every cell (self for NoFlow)."""
    lib = lib or load()
    h = _f64(h)
    ny, nx = h.shape
    rec = np.empty((ny, nx), np.int32)
    lib.lemo_receivers(ny, nx, dx, dy, _ptr(h), _ptr(rec))
    return rec


def donors(rec, lib=None):
    """Step 3, Algorithm 2 over every cell: (donor[N, 8], dnum[N])."""
    lib = lib or load()
    rec = np.ascontiguousarray(rec, np.int32)
    ny, nx = rec.shape
    donor = np.full((ny * nx, 8), -1, np.int32)
    dnum = np.empty(ny * nx, np.uint8)
    lib.lemo_donors(ny, nx, _ptr(rec), _ptr(donor), _ptr(dnum))
    return donor, dnum


def stack_order(rec, donor, dnum, lib=None):
    """Depth-first stack order and depth (figure "Stack vs. queue" (a))."""
    lib = lib or load()
    rec = np.ascontiguousarray(rec, np.int32).ravel()
    n = rec.size
    order = np.empty(n, np.int32)
    depth = np.empty(n, np.int32)
    stack = np.empty(max(n, 1), np.int32)
    emitted = lib.lemo_stack_order(n, _ptr(rec), _ptr(donor), _ptr(dnum), _ptr(order),
                                   _ptr(depth), _ptr(stack))
    return order[:emitted], depth, emitted


def bfs_queue(rec, donor, dnum, lib=None):
    """Algorithm 3 (Generate Queue): (queue, levels) with Levels[0] = 0."""
    lib = lib or load()
    rec = np.ascontiguousarray(rec, np.int32).ravel()
    n = rec.size
    queue = np.empty(n, np.int32)
    levels = np.empty(n + 2, np.int64)
    nl = lib.lemo_bfs_queue(n, _ptr(rec), _ptr(donor), _ptr(dnum), _ptr(queue), _ptr(levels))
    return queue, levels[: nl + 1]


def graph_order(rec, lib=None):
    """Steps 3-5 on an arbitrary forest (Table 1's worked example).

    ``rec[c] == c`` marks a node without receiver.  Returns a dict with the
    donor lists, Dnum, the breadth-first Queue and Levels, the depth-first
    stack order, the depth and the unit-area accumulation of every node.
    """
    lib = lib or load()
    rec = np.ascontiguousarray(rec, np.int32)
    n = rec.size
    donor = np.full((n, 8), -1, np.int32)
    dnum = np.empty(n, np.uint8)
    queue = np.empty(n, np.int32)
    levels = np.empty(n + 2, np.int64)
    order = np.empty(n, np.int32)
    depth = np.empty(n, np.int32)
    count = np.empty(n, np.uint32)
    nl = lib.lemo_graph_order(n, _ptr(rec), _ptr(donor), _ptr(dnum), _ptr(queue),
                              _ptr(levels), _ptr(order), _ptr(depth), _ptr(count))
    if nl < 0:
        raise ValueError("receivers contain a cycle or a node has more than 8 donors")
    return dict(donor=donor, dnum=dnum, queue=queue, levels=levels[: nl + 1],
                stack_order=order, depth=depth, count=count)


def _check(st):
    if st == LEMO_E_CYCLE:
        raise ValueError("oracle: receivers contain a cycle")
    if st != LEMO_OK:
        raise ValueError(f"oracle: status {st}")


def run(h0, params: Params, steps: int, K=None, U=None, lib=None):
    """Run ``steps`` time steps (Steps 2-7, repeated) on a copy of ``h0``.

    Returns a dict: ``h`` (final heights) and the routing of the last step
    (``rec``, ``depth``, ``count``, ``offsets``, ``nlevels``).
    """
    lib = lib or load()
    h = np.array(h0, dtype=np.float64, copy=True, order="C")
    ny, nx = h.shape
    assert (ny, nx) == (params.ny, params.nx)
    K = _f64(K)
    U = _f64(U)
    rec = np.empty((ny, nx), np.int32)
    depth = np.empty((ny, nx), np.int32)
    count = np.empty((ny, nx), np.uint32)
    offsets = np.empty(ny * nx + 2, np.int64)
    nlev = C.c_int64(0)
    p = params.c()
    _check(lib.lemo_run(C.byref(p), _ptr(h), _ptr(K), _ptr(U), int(steps), _ptr(rec),
                        _ptr(depth), _ptr(count), _ptr(offsets), offsets.size,
                        C.byref(nlev)))
    return dict(h=h, rec=rec, depth=depth, count=count,
                offsets=offsets[: nlev.value + 1].copy(), nlevels=nlev.value)


def project(h0, params: Params, iters: int, K=None, U=None, lib=None):
    """Steady-state projections (an accelerator of runs to steady state, not
    a step of the paper's method): each computes the routing of the current
    heights as Steps 2-5 do, uplifts as Step 6 (Algorithm 5) does, then gives
    every cell with a receiver the height at which Algorithm 6 would leave it
    unchanged: h_c = h_r + U_c*dt/F (n = 1) or h_r + (U_c*dt/F)^(1/n), in
    receiver-first order.  Returns the heights and the last routing."""
    lib = lib or load()
    h = np.array(h0, dtype=np.float64, copy=True, order="C")
    rec = np.empty(h.shape, np.int32)
    depth = np.empty(h.shape, np.int32)
    count = np.empty(h.shape, np.uint32)
    p = params.c()
    _check(lib.lemo_project(C.byref(p), _ptr(h), _ptr(_f64(K)), _ptr(_f64(U)), int(iters),
                            _ptr(rec), _ptr(depth), _ptr(count)))
    return dict(h=h, rec=rec, depth=depth, count=count)


def run_fixed_routing(h0, rec, params: Params, steps: int, K=None, U=None, lib=None):
    """Steps 3-7 repeated with the receivers held fixed (no Step 2)."""
    lib = lib or load()
    h = np.array(h0, dtype=np.float64, copy=True, order="C")
    rec = np.ascontiguousarray(rec, np.int32)
    depth = np.empty(h.shape, np.int32)
    count = np.empty(h.shape, np.uint32)
    p = params.c()
    _check(lib.lemo_run_fixed_routing(C.byref(p), _ptr(h), _ptr(rec), _ptr(_f64(K)),
                                      _ptr(_f64(U)), int(steps), _ptr(depth), _ptr(count)))
    return dict(h=h, depth=depth, count=count)


def routing(h, params: Params, lib=None):
    """Steps 2-5 for the given heights (receivers, depth, counts, levels)."""
    lib = lib or load()
    h = _f64(h)
    ny, nx = h.shape
    rec = np.empty((ny, nx), np.int32)
    depth = np.empty((ny, nx), np.int32)
    count = np.empty((ny, nx), np.uint32)
    offsets = np.empty(ny * nx + 2, np.int64)
    nlev = C.c_int64(0)
    p = params.c()
    _check(lib.lemo_routing(C.byref(p), _ptr(h), _ptr(rec), _ptr(depth), _ptr(count),
                            _ptr(offsets), offsets.size, C.byref(nlev)))
    return dict(rec=rec, depth=depth, count=count,
                offsets=offsets[: nlev.value + 1].copy(), nlevels=nlev.value)


def mfd_run(h0, params: Params, steps: int, pexp: float = 1.0, K=None, U=None, lib=None):
    """``steps`` time steps with multiple-flow-direction routing (section
    "Multiple Flow Directions"): every strictly lower neighbour receives a
    share of the flow proportional to slope**pexp.  Returns ``h`` and the last
    step's drainage ``area`` (m^2), ``level`` (longest path to a root) and
    ``nlevels``."""
    lib = lib or load()
    h = np.array(h0, dtype=np.float64, copy=True, order="C")
    ny, nx = h.shape
    area = np.empty((ny, nx), np.float64)
    level = np.empty((ny, nx), np.int32)
    nlev = C.c_int64(0)
    p = params.c()
    _check(lib.lemo_mfd_run(C.byref(p), float(pexp), _ptr(h), _ptr(_f64(K)), _ptr(_f64(U)),
                            int(steps), _ptr(area), _ptr(level), C.byref(nlev)))
    return dict(h=h, area=area, level=level, nlevels=nlev.value)
