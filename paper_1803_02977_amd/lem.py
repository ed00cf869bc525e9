"""ctypes binding of the C ABI in ``include/lem.h`` (argument marshalling only).

Every function has the name of the C entry point it wraps.  ``Solver`` is a
convenience wrapper that takes torch tensors on the ROCm device (torch is used
for device memory and streams only) and calls the same entry points.  Nothing
here computes any step of the method; if ``liblem.so`` is missing, loading
fails with an error instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblem.so")

LEM_OK, LEM_E_ARG, LEM_E_SIZE, LEM_E_WORKSPACE = 0, 1, 2, 3
LEM_E_NONFINITE, LEM_E_CYCLE, LEM_E_HIP, LEM_E_STATE = 4, 5, 6, 7
LEM_F_VALIDATE, LEM_F_PHASE_TIMERS, LEM_F_TILE_CLOCKS = 0x1, 0x2, 0x4

# Symbols declared in include/lem.h.
EXPORTS = ("lem_workspace_bytes", "lem_create", "lem_run", "lem_run_fixed_routing",
           "lem_sync", "lem_routing", "lem_batch_workspace_bytes", "lem_batch_create",
           "lem_batch_run", "lem_batch_run_to_steady", "lem_batch_project_to_steady",
           "lem_batch_routing",
           "lem_level_history", "lem_stats", "lem_set_tuning", "lem_get_tuning", "lem_destroy",
           "lem_status_str", "lem_last_error", "lem_mfd_workspace_bytes", "lem_mfd_create",
           "lem_mfd_export")


class lem_params(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dt", C.c_double), ("m", C.c_double), ("n", C.c_double), ("U", C.c_double),
                ("K", C.c_double), ("eps", C.c_double), ("max_newton", C.c_int32),
                ("flags", C.c_uint32)]


class lem_stats_t(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("last_nlevels", C.c_int64),
                ("max_nlevels", C.c_int64), ("last_run_steps", C.c_int64),
                ("phase_ms", C.c_double * 4), ("kernel_ms", C.c_double * 3),
                ("crossing_last", C.c_int64), ("crossing_run", C.c_int64),
                ("tile_phase_ms", C.c_double * 6)]


class lem_grid(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dt", C.c_double), ("m", C.c_double), ("U", C.c_double), ("K", C.c_double),
                ("n", C.c_double), ("eps", C.c_double), ("max_newton", C.c_int32),
                ("pad", C.c_int32), ("offset", C.c_int64)]


LEM_LEVELS_AUTO, LEM_LEVELS_GLOBAL, LEM_LEVELS_PER_GRID = 0, 1, 2
LEM_CHUNKS_AUTO, LEM_CHUNKS_ON, LEM_CHUNKS_OFF = 0, 1, 2


class lem_tuning(C.Structure):
    _fields_ = [("global_workgroups", C.c_int32), ("tail_level", C.c_int32),
                ("level_pass", C.c_int32), ("level_threads", C.c_int32),
                ("chunk_pass", C.c_int32), ("chunk_roots", C.c_int32)]


class LemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


_LIB = None
_P = C.c_void_p


def load(path: str = LIB_PATH):
    """Load ``liblem.so``; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python paper_1803_02977_amd/build_lib.py` (hipcc --offload-arch=gfx950)")
    lib = C.CDLL(path)
    lib.lem_workspace_bytes.argtypes = [C.POINTER(lem_params)]
    lib.lem_workspace_bytes.restype = C.c_size_t
    lib.lem_create.argtypes = [C.POINTER(lem_params), _P, C.c_size_t, _P, C.POINTER(_P)]
    lib.lem_create.restype = C.c_int
    lib.lem_run.argtypes = [_P, _P, _P, _P, C.c_int64]
    lib.lem_run.restype = C.c_int
    lib.lem_run_fixed_routing.argtypes = [_P, _P, _P, _P, _P, C.c_int64]
    lib.lem_run_fixed_routing.restype = C.c_int
    lib.lem_sync.argtypes = [_P]
    lib.lem_sync.restype = C.c_int
    lib.lem_routing.argtypes = [_P, _P, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]
    lib.lem_routing.restype = C.c_int
    lib.lem_level_history.argtypes = [_P, _P, C.c_int64, C.POINTER(C.c_int64)]
    lib.lem_level_history.restype = C.c_int
    lib.lem_stats.argtypes = [_P, C.POINTER(lem_stats_t)]
    lib.lem_stats.restype = C.c_int
    lib.lem_batch_workspace_bytes.argtypes = [C.POINTER(lem_grid), C.c_int32]
    lib.lem_batch_workspace_bytes.restype = C.c_size_t
    lib.lem_batch_create.argtypes = [C.POINTER(lem_grid), C.c_int32, C.c_uint32, _P, C.c_size_t,
                                     _P, C.POINTER(_P)]
    lib.lem_batch_create.restype = C.c_int
    lib.lem_batch_run.argtypes = [_P, _P, _P, _P, C.c_int64]
    lib.lem_batch_run.restype = C.c_int
    lib.lem_batch_run_to_steady.argtypes = [_P, _P, _P, _P, C.c_double, C.c_int64, C.c_int64, _P]
    lib.lem_batch_run_to_steady.restype = C.c_int
    lib.lem_batch_project_to_steady.argtypes = [_P, _P, _P, _P, C.c_double, C.c_int64,
                                                C.c_int64, _P]
    lib.lem_batch_project_to_steady.restype = C.c_int
    lib.lem_batch_routing.argtypes = [_P, C.c_int32, _P, _P, _P, _P, C.c_int64,
                                      C.POINTER(C.c_int64)]
    lib.lem_batch_routing.restype = C.c_int
    lib.lem_set_tuning.argtypes = [_P, C.POINTER(lem_tuning)]
    lib.lem_set_tuning.restype = C.c_int
    lib.lem_get_tuning.argtypes = [_P, C.POINTER(lem_tuning)]
    lib.lem_get_tuning.restype = C.c_int
    lib.lem_destroy.argtypes = [_P]
    lib.lem_destroy.restype = C.c_int
    lib.lem_mfd_workspace_bytes.argtypes = [C.POINTER(lem_params)]
    lib.lem_mfd_workspace_bytes.restype = C.c_size_t
    lib.lem_mfd_create.argtypes = [C.POINTER(lem_params), C.c_double, _P, C.c_size_t, _P,
                                   C.POINTER(_P)]
    lib.lem_mfd_create.restype = C.c_int
    lib.lem_mfd_export.argtypes = [_P, _P, _P, C.POINTER(C.c_int64)]
    lib.lem_mfd_export.restype = C.c_int
    lib.lem_status_str.argtypes = [C.c_int]
    lib.lem_status_str.restype = C.c_char_p
    lib.lem_last_error.argtypes = [_P]
    lib.lem_last_error.restype = C.c_char_p
    lib.lem_run_static.argtypes = [C.POINTER(lem_params), _P, _P, _P, C.c_int64, _P]
    lib.lem_run_static.restype = C.c_int
    _LIB = lib
    return lib


def _check(st: int, ctx=None):
    if st != LEM_OK:
        lib = load()
        msg = lib.lem_status_str(st).decode()
        if ctx:
            detail = lib.lem_last_error(ctx).decode()
            if detail:
                msg = f"{msg} ({detail})"
        raise LemError(st, msg)


# --- one wrapper per C entry point ------------------------------------------------

# Size of the library's own device workspace array used by lem_run_static.
LEM_STATIC_WORKSPACE_BYTES = 16 << 20


def lem_run_static(p: lem_params, d_h: int, d_K, d_U, steps: int, hip_stream: int) -> None:
    """Steps over the library's static device workspace (no device allocation)."""
    st = load().lem_run_static(C.byref(p), d_h, d_K, d_U, steps, hip_stream)
    if st == LEM_E_WORKSPACE:
        raise LemError(st, f"LEM_E_WORKSPACE (the grid needs {lem_workspace_bytes(p)} bytes of "
                           f"workspace; the static workspace holds {LEM_STATIC_WORKSPACE_BYTES})")
    _check(st)


def lem_workspace_bytes(p: lem_params) -> int:
    return int(load().lem_workspace_bytes(C.byref(p)))


def lem_create(p: lem_params, d_workspace: int, ws_bytes: int, hip_stream: int) -> int:
    ctx = _P()
    _check(load().lem_create(C.byref(p), d_workspace, ws_bytes, hip_stream, C.byref(ctx)))
    return ctx.value


def lem_run(ctx: int, d_h: int, d_K, d_U, steps: int) -> None:
    _check(load().lem_run(ctx, d_h, d_K, d_U, steps), ctx)


def lem_run_fixed_routing(ctx: int, d_h: int, d_rcode: int, d_K, d_U, steps: int) -> None:
    _check(load().lem_run_fixed_routing(ctx, d_h, d_rcode, d_K, d_U, steps), ctx)


def lem_sync(ctx: int) -> None:
    _check(load().lem_sync(ctx), ctx)


def lem_routing(ctx: int, d_rec, d_depth, d_count, cap: int):
    import numpy as np
    offsets = np.zeros(max(cap, 1), np.int64)
    nl = C.c_int64(0)
    _check(load().lem_routing(ctx, d_rec, d_depth, d_count,
                              offsets.ctypes.data_as(_P), cap, C.byref(nl)), ctx)
    return offsets[: nl.value + 1] if cap >= nl.value + 1 else None, nl.value


def lem_batch_workspace_bytes(grids) -> int:
    arr = (lem_grid * len(grids))(*grids)
    return int(load().lem_batch_workspace_bytes(arr, len(grids)))


def lem_batch_create(grids, flags: int, d_workspace: int, ws_bytes: int, hip_stream: int) -> int:
    arr = (lem_grid * len(grids))(*grids)
    ctx = _P()
    _check(load().lem_batch_create(arr, len(grids), flags, d_workspace, ws_bytes, hip_stream,
                                   C.byref(ctx)))
    return ctx.value


def lem_batch_run(ctx: int, d_h: int, d_K, d_U, steps: int) -> None:
    _check(load().lem_batch_run(ctx, d_h, d_K, d_U, steps), ctx)


def lem_batch_run_to_steady(ctx: int, d_h: int, d_K, d_U, rtol: float, check_every: int,
                            max_steps: int, count: int, steps_in=None):
    import numpy as np
    out = (np.full(count, -1, np.int64) if steps_in is None
           else np.ascontiguousarray(steps_in, np.int64).copy())
    _check(load().lem_batch_run_to_steady(ctx, d_h, d_K, d_U, rtol, check_every, max_steps,
                                          out.ctypes.data_as(_P)), ctx)
    return out


def lem_batch_project_to_steady(ctx: int, d_h: int, d_K, d_U, rtol: float, check_every: int,
                                max_iters: int, count: int, iters_in=None):
    import numpy as np
    out = (np.full(count, -1, np.int64) if iters_in is None
           else np.ascontiguousarray(iters_in, np.int64).copy())
    _check(load().lem_batch_project_to_steady(ctx, d_h, d_K, d_U, rtol, check_every, max_iters,
                                              out.ctypes.data_as(_P)), ctx)
    return out


def lem_batch_routing(ctx: int, grid: int, d_rec, d_depth, d_count, cap: int):
    import numpy as np
    offsets = np.zeros(max(cap, 1), np.int64)
    nl = C.c_int64(0)
    _check(load().lem_batch_routing(ctx, grid, d_rec, d_depth, d_count,
                                    offsets.ctypes.data_as(_P), cap, C.byref(nl)), ctx)
    return offsets[: nl.value + 1] if cap >= nl.value + 1 else None, nl.value


def lem_level_history(ctx: int, cap: int):
    import numpy as np
    out = np.zeros(max(cap, 1), np.int32)
    n = C.c_int64(0)
    _check(load().lem_level_history(ctx, out.ctypes.data_as(_P), cap, C.byref(n)), ctx)
    return out[: min(n.value, cap)]


def lem_stats(ctx: int) -> lem_stats_t:
    s = lem_stats_t()
    _check(load().lem_stats(ctx, C.byref(s)), ctx)
    return s


def lem_set_tuning(ctx: int, t: lem_tuning) -> None:
    _check(load().lem_set_tuning(ctx, C.byref(t)), ctx)


def lem_get_tuning(ctx: int) -> lem_tuning:
    t = lem_tuning()
    _check(load().lem_get_tuning(ctx, C.byref(t)), ctx)
    return t


def lem_destroy(ctx: int) -> None:
    _check(load().lem_destroy(ctx))


def lem_status_str(st: int) -> str:
    return load().lem_status_str(st).decode()


def lem_last_error(ctx: int) -> str:
    return load().lem_last_error(ctx).decode()


# --- torch convenience -----------------------------------------------------------

def _dptr(t):
    return None if t is None else t.data_ptr()


def _set_tuning(ctx, *fields):
    lem_set_tuning(ctx, lem_tuning(*fields))
    t = lem_get_tuning(ctx)
    return {name: getattr(t, name) for name, _ in lem_tuning._fields_}


def _apply_tuning(obj, cells, tuning, batch=False):
    """tuning: None (library defaults), "auto" (tuning.json's setting for a
    single grid or a batch of that many cells, if present), a tuple of
    lem_tuning fields in order or a dict of them by name."""
    if tuning is None:
        return
    if tuning == "auto":
        from . import tune
        tuning = tune.lookup(cells, batch)
        if tuning is None:
            return
    if isinstance(tuning, dict):
        obj.set_tuning(**tuning)
    else:
        obj.set_tuning(*tuning)


class Solver:
    """A context plus its workspace, for torch tensors on one ROCm device.

    ``run(h, steps, K=None, U=None)`` updates ``h`` (float64, contiguous,
    shape (ny, nx), on the device) in place on the current torch stream.
    """

    def __init__(self, ny, nx, dx=100.0, dy=100.0, dt=1000.0, m=0.5, U=5e-4, K=1e-5,
                 n=1.0, flags=0, device=None, stream=None, tuning="auto", eps=1e-12,
                 max_newton=100):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.params = lem_params(ny, nx, dx, dy, dt, m, n, U, K, eps, max_newton, flags)
        nbytes = lem_workspace_bytes(self.params)
        if nbytes == 0:
            raise LemError(LEM_E_ARG, "invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.ctx = lem_create(self.params, self.workspace.data_ptr(), nbytes,
                                  self.stream.cuda_stream)
        _apply_tuning(self, ny * nx, tuning)

    def _check_field(self, t, name):
        torch = self.torch
        if t is None:
            return None
        shape = (self.params.ny, self.params.nx)
        if (t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous()
                or t.device != self.device):
            raise LemError(LEM_E_ARG, f"{name} must be a contiguous float64 {shape} tensor "
                                      f"on {self.device}")
        return t

    def run(self, h, steps, K=None, U=None):
        self._check_field(h, "h")
        lem_run(self.ctx, h.data_ptr(), _dptr(self._check_field(K, "K")),
                _dptr(self._check_field(U, "U")), int(steps))

    def run_fixed_routing(self, h, rcode, steps, K=None, U=None):
        torch = self.torch
        self._check_field(h, "h")
        if (rcode.dtype != torch.uint8 or tuple(rcode.shape) != tuple(h.shape)
                or not rcode.is_contiguous() or rcode.device != self.device):
            raise LemError(LEM_E_ARG, "rcode must be a contiguous uint8 tensor like h")
        lem_run_fixed_routing(self.ctx, h.data_ptr(), rcode.data_ptr(),
                              _dptr(self._check_field(K, "K")),
                              _dptr(self._check_field(U, "U")), int(steps))

    def sync(self):
        lem_sync(self.ctx)

    def routing(self):
        """Routing of the last step: rec, depth, count (device tensors), offsets."""
        torch = self.torch
        shape = (self.params.ny, self.params.nx)
        rec = torch.empty(shape, dtype=torch.int32, device=self.device)
        depth = torch.empty(shape, dtype=torch.int32, device=self.device)
        count = torch.empty(shape, dtype=torch.int32, device=self.device)  # holds uint32 bits
        offsets, nl = lem_routing(self.ctx, rec.data_ptr(), depth.data_ptr(),
                                  count.data_ptr(), 0)
        offsets, _ = lem_routing(self.ctx, None, None, None, nl + 1)
        return dict(rec=rec, depth=depth, count=count, offsets=offsets, nlevels=nl)

    def level_history(self, cap=1 << 16):
        return lem_level_history(self.ctx, cap)

    def stats(self) -> lem_stats_t:
        return lem_stats(self.ctx)

    def set_tuning(self, global_workgroups=0, tail_level=0, level_pass=0, level_threads=0,
                   chunk_pass=0, chunk_roots=0):
        return _set_tuning(self.ctx, global_workgroups, tail_level, level_pass, level_threads,
                           chunk_pass, chunk_roots)

    def close(self):
        if getattr(self, "ctx", None):
            lem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent grids advanced together (one context, one buffer).

    ``grids`` is a list of dicts or objects with ny, nx, dx, dy, dt, m, U, K.
    ``h`` is a float64 device tensor of ``total_cells`` elements holding the
    grids back to back; ``view(h, g)`` returns grid g as an (ny, nx) view.
    """

    def __init__(self, grids, flags=0, device=None, stream=None, tuning="auto"):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        descs, off = [], 0
        for g in grids:
            def get(k, default=None, g=g):
                if isinstance(g, dict):
                    return g.get(k, default)
                return getattr(g, k, default)
            d = lem_grid(int(get("ny")), int(get("nx")), float(get("dx")), float(get("dy")),
                         float(get("dt")), float(get("m")), float(get("U")), float(get("K")),
                         float(get("n", 1.0)), float(get("eps", 1e-12)),
                         int(get("max_newton", 100)), 0, off)
            descs.append(d)
            off += d.ny * d.nx
        self.descs = descs
        self.offsets = [d.offset for d in descs]
        self.shapes = [(d.ny, d.nx) for d in descs]
        self.total_cells = off
        nbytes = lem_batch_workspace_bytes(descs)
        if nbytes == 0:
            raise LemError(LEM_E_ARG, "invalid grid descriptors")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.ctx = lem_batch_create(descs, flags, self.workspace.data_ptr(), nbytes,
                                        self.stream.cuda_stream)
        _apply_tuning(self, self.total_cells, tuning, batch=len(descs) > 1)

    def _check_h(self, h):
        torch = self.torch
        if (h.dtype != torch.float64 or h.numel() != self.total_cells or not h.is_contiguous()
                or h.device != self.device):
            raise LemError(LEM_E_ARG, f"h must be a contiguous float64 tensor of "
                                      f"{self.total_cells} elements on {self.device}")

    def view(self, h, g):
        ny, nx = self.shapes[g]
        o = self.offsets[g]
        return h.view(-1)[o: o + ny * nx].view(ny, nx)

    def run(self, h, steps, K=None, U=None):
        self._check_h(h)
        for f in (K, U):
            if f is not None:
                self._check_h(f)
        lem_batch_run(self.ctx, h.data_ptr(), _dptr(K), _dptr(U), int(steps))

    def run_to_steady(self, h, rtol=1e-6, check_every=10, max_steps=100000, K=None, U=None,
                      chunk=None, progress=None):
        """Steps to convergence; returns steps per grid (-1: not converged).
        With ``chunk`` the run is split into calls of at most that many
        steps (grids that converged stay frozen) and ``progress(done_steps,
        converged)`` is called after each."""
        import numpy as np
        self._check_h(h)
        for f in (K, U):
            if f is not None:
                self._check_h(f)
        n = len(self.descs)
        if not chunk:
            return lem_batch_run_to_steady(self.ctx, h.data_ptr(), _dptr(K), _dptr(U),
                                           float(rtol), int(check_every), int(max_steps), n)
        if chunk % check_every:
            raise LemError(LEM_E_ARG, "chunk must be a multiple of check_every")
        total = np.full(n, -1, np.int64)
        done = 0
        while done < max_steps and (total < 0).any():
            k = min(int(chunk), int(max_steps) - done)
            got = lem_batch_run_to_steady(self.ctx, h.data_ptr(), _dptr(K), _dptr(U),
                                          float(rtol), int(check_every), k, n, steps_in=total)
            new = (total < 0) & (got >= 0)
            total[new] = got[new] + done
            done += k
            if progress:
                progress(done, int((total >= 0).sum()))
        return total

    def project_to_steady(self, h, rtol=1e-6, check_every=10, max_iters=100000, K=None, U=None):
        """Steady-state projections until every grid changes by at most rtol
        of its largest height (lem_batch_project_to_steady); returns the
        projections per grid (-1: not converged)."""
        self._check_h(h)
        for f in (K, U):
            if f is not None:
                self._check_h(f)
        return lem_batch_project_to_steady(self.ctx, h.data_ptr(), _dptr(K), _dptr(U),
                                           float(rtol), int(check_every), int(max_iters),
                                           len(self.descs))

    def sync(self):
        lem_sync(self.ctx)

    def routing(self, g):
        torch = self.torch
        if not 0 <= g < len(self.shapes):
            lem_batch_routing(self.ctx, g, None, None, None, 0)  # raises LEM_E_ARG
        shape = self.shapes[g]
        rec = torch.empty(shape, dtype=torch.int32, device=self.device)
        depth = torch.empty(shape, dtype=torch.int32, device=self.device)
        count = torch.empty(shape, dtype=torch.int32, device=self.device)
        _, nl = lem_batch_routing(self.ctx, g, rec.data_ptr(), depth.data_ptr(),
                                  count.data_ptr(), 0)
        offsets, _ = lem_batch_routing(self.ctx, g, None, None, None, nl + 1)
        return dict(rec=rec, depth=depth, count=count, offsets=offsets, nlevels=nl)

    def set_tuning(self, global_workgroups=0, tail_level=0, level_pass=0, level_threads=0,
                   chunk_pass=0, chunk_roots=0):
        return _set_tuning(self.ctx, global_workgroups, tail_level, level_pass, level_threads,
                           chunk_pass, chunk_roots)

    def stats(self) -> lem_stats_t:
        return lem_stats(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lem_mfd_workspace_bytes(p: lem_params) -> int:
    return int(load().lem_mfd_workspace_bytes(C.byref(p)))


class MfdSolver:
    """Multiple-flow-direction routing (``lem_mfd_create``) for torch tensors:
    ``run(h, steps, K=None, U=None)`` updates ``h`` in place, ``export()``
    returns the last step's drainage area, levels and level count."""

    def __init__(self, ny, nx, dx=100.0, dy=100.0, dt=1000.0, m=0.5, U=5e-4, K=1e-5,
                 exponent=1.0, flags=0, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.params = lem_params(ny, nx, dx, dy, dt, m, 1.0, U, K, 1e-12, 100, flags)
        nbytes = lem_mfd_workspace_bytes(self.params)
        if nbytes == 0:
            raise LemError(LEM_E_ARG, "invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        ctx = _P()
        _check(load().lem_mfd_create(C.byref(self.params), float(exponent),
                                     _P(self.workspace.data_ptr()), nbytes,
                                     _P(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx.value
        self.shape = (ny, nx)

    def _check_f(self, name, t):
        torch = self.torch
        if t is None:
            return None
        if (t.dtype != torch.float64 or tuple(t.shape) != self.shape or not t.is_contiguous()
                or t.device != self.device):
            raise LemError(LEM_E_ARG, f"{name} must be a contiguous float64 {self.shape} tensor "
                                      f"on {self.device}")
        return t.data_ptr()

    def run(self, h, steps, K=None, U=None):
        _check(load().lem_run(self.ctx, self._check_f("h", h), self._check_f("K", K),
                              self._check_f("U", U), int(steps)), self.ctx)

    def sync(self):
        lem_sync(self.ctx)

    def export(self):
        torch = self.torch
        area = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        level = torch.empty(self.shape, dtype=torch.int32, device=self.device)
        nl = C.c_int64()
        _check(load().lem_mfd_export(self.ctx, _P(area.data_ptr()), _P(level.data_ptr()),
                                     C.byref(nl)), self.ctx)
        return dict(area=area, level=level, nlevels=nl.value)

    def stats(self) -> lem_stats_t:
        return lem_stats(self.ctx)

    def set_tuning(self, global_workgroups=0, tail_level=0):
        lem_set_tuning(self.ctx, lem_tuning(global_workgroups, tail_level, 0, 0))
        t = lem_get_tuning(self.ctx)
        return dict(global_workgroups=t.global_workgroups)

    def close(self):
        if getattr(self, "ctx", None):
            lem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
