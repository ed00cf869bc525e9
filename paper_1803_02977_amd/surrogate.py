"""ctypes binding of the warm-start network (``include/lem_surrogate.h``).

Argument marshalling only: the forward pass, the backward pass and the Adam
step all run in the library's HIP kernels.  ``Surrogate`` owns a device
workspace (a torch tensor) and enqueues on the current torch stream.

    net = Surrogate(batch=16, ny=256, nx=256)
    net.set_params(init_params(seed=0))          # float32 vector
    loss = net.train_step(K, U, h0, h_steady, lr=1e-3)
    h_warm = net.predict(K, U, h0)               # FP64 heights, perimeter 0

K, U, h0 and targets are float64 device tensors of shape (batch, ny, nx).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .lem import LEM_OK, LemError, load as _load_lem

_P = C.c_void_p
_SUR = None

SUR_EXPORTS = ("lem_sur_param_count", "lem_sur_layer", "lem_sur_workspace_bytes",
               "lem_sur_create", "lem_sur_set_params", "lem_sur_get_params", "lem_sur_predict",
               "lem_sur_loss_grad", "lem_sur_train_step", "lem_sur_activation", "lem_sur_sync",
               "lem_sur_destroy", "lem_sur_last_error")
NUM_LAYERS = 15  # fourteen 3x3 convolutions, then the 1x1 head


def load():
    global _SUR
    if _SUR is not None:
        return _SUR
    lib = _load_lem()
    lib.lem_sur_param_count.argtypes = []
    lib.lem_sur_param_count.restype = C.c_int64
    lib.lem_sur_layer.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64)]
    lib.lem_sur_layer.restype = C.c_int
    lib.lem_sur_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    lib.lem_sur_workspace_bytes.restype = C.c_size_t
    lib.lem_sur_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, _P, C.c_size_t, _P,
                                   C.POINTER(_P)]
    lib.lem_sur_create.restype = C.c_int
    lib.lem_sur_set_params.argtypes = [_P, _P]
    lib.lem_sur_set_params.restype = C.c_int
    lib.lem_sur_get_params.argtypes = [_P, _P]
    lib.lem_sur_get_params.restype = C.c_int
    lib.lem_sur_predict.argtypes = [_P, C.c_int32, _P, _P, _P, _P, _P]
    lib.lem_sur_predict.restype = C.c_int
    lib.lem_sur_loss_grad.argtypes = [_P, C.c_int32, _P, _P, _P, _P, _P, C.POINTER(C.c_double)]
    lib.lem_sur_loss_grad.restype = C.c_int
    lib.lem_sur_train_step.argtypes = [_P, C.c_int32, _P, _P, _P, _P, C.c_float,
                                       C.POINTER(C.c_double)]
    lib.lem_sur_train_step.restype = C.c_int
    lib.lem_sur_activation.argtypes = [_P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lem_sur_activation.restype = C.c_int
    lib.lem_sur_sync.argtypes = [_P]
    lib.lem_sur_sync.restype = C.c_int
    lib.lem_sur_destroy.argtypes = [_P]
    lib.lem_sur_destroy.restype = C.c_int
    lib.lem_sur_last_error.argtypes = [_P]
    lib.lem_sur_last_error.restype = C.c_char_p
    _SUR = lib
    return lib


def _check(st, ctx=None):
    if st != LEM_OK:
        lib = load()
        msg = lib.lem_status_str(st).decode()
        if ctx:
            detail = lib.lem_sur_last_error(ctx).decode()
            if detail:
                msg = f"{msg} ({detail})"
        raise LemError(st, msg)


def param_count() -> int:
    return int(load().lem_sur_param_count())


def layer(i: int):
    """(cin, cout, offset) of parameter block i (0..13 convolutions, 14 head)."""
    cin, cout, off = C.c_int32(), C.c_int32(), C.c_int64()
    _check(load().lem_sur_layer(i, C.byref(cin), C.byref(cout), C.byref(off)))
    return cin.value, cout.value, off.value


def workspace_bytes(batch: int, ny: int, nx: int) -> int:
    return int(load().lem_sur_workspace_bytes(batch, ny, nx))


def init_params(seed: int = 0, input_features: int = 3) -> np.ndarray:
    """He-normal weights (fan-in over the real input channels; padded input
    channels start at zero), zero biases, float32."""
    rng = np.random.default_rng(seed)
    p = np.zeros(param_count(), np.float32)
    for i in range(NUM_LAYERS):
        cin, cout, off = layer(i)
        if i == NUM_LAYERS - 1:
            p[off:off + cin] = rng.standard_normal(cin) * np.sqrt(1.0 / cin)
            continue
        real = input_features if i == 0 else cin
        w = rng.standard_normal((cout, 3, 3, cin)) * np.sqrt(2.0 / (9 * real))
        w[..., real:] = 0.0
        p[off:off + w.size] = w.ravel()
    return p


def bias_mask() -> np.ndarray:
    """True at the bias entries of the parameter vector."""
    mask = np.zeros(param_count(), bool)
    for i in range(NUM_LAYERS):
        cin, cout, off = layer(i)
        nw = cin if i == NUM_LAYERS - 1 else cout * 9 * cin
        mask[off + nw:off + nw + cout] = True
    return mask


def save_params(path, params):
    """Stores parameters as the network uses them: weights as bfloat16
    (nearest, ties to even) and biases as float32.  Loading gives a vector
    whose predictions equal those of the float32 original."""
    p = np.asarray(params, np.float32)
    u = p.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    mask = bias_mask()
    np.savez_compressed(path, weights_bf16=bits, biases=p[mask])


def load_params(path) -> np.ndarray:
    z = np.load(path, allow_pickle=False)
    p = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32).copy()
    p[bias_mask()] = z["biases"]
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Surrogate:
    """A network context for up to ``batch`` grids of ny x nx on one device."""

    def __init__(self, batch: int, ny: int, nx: int, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self.batch, self.ny, self.nx = batch, ny, nx
        nbytes = workspace_bytes(batch, ny, nx)
        if nbytes == 0:
            raise LemError(2, "invalid network shape (ny, nx >= 8 and divisible by 8)")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        ctx = _P()
        _check(load().lem_sur_create(batch, ny, nx, _P(self.workspace.data_ptr()), nbytes,
                                     _P(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx.value
        self.nparams = param_count()

    def _fields(self, *ts):
        n = None
        for t in ts:
            if t is None:
                continue
            if t.dtype != self.torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise LemError(1, "fields must be contiguous float64 tensors on the device")
            if t.dim() != 3 or tuple(t.shape[1:]) != (self.ny, self.nx):
                raise LemError(1, f"fields must have shape (batch, {self.ny}, {self.nx})")
            if n is not None and t.shape[0] != n:
                raise LemError(1, "fields must have the same batch")
            n = t.shape[0]
        return n

    def set_params(self, params):
        t = self.torch.as_tensor(np.asarray(params, np.float32)).to(self.device)
        if t.numel() != self.nparams:
            raise LemError(1, f"expected {self.nparams} parameters")
        _check(load().lem_sur_set_params(self.ctx, _ptr(t)), self.ctx)
        self.sync()

    def get_params(self):
        t = self.torch.empty(self.nparams, dtype=self.torch.float32, device=self.device)
        _check(load().lem_sur_get_params(self.ctx, _ptr(t)), self.ctx)
        self.sync()
        return t

    def predict(self, K, U, h0, want_y=False):
        n = self._fields(K, U, h0)
        h = self.torch.empty((n, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        y = (self.torch.empty((n, self.ny, self.nx), dtype=self.torch.float32, device=self.device)
             if want_y else None)
        _check(load().lem_sur_predict(self.ctx, n, _ptr(K), _ptr(U), _ptr(h0), _ptr(h), _ptr(y)),
               self.ctx)
        return (h, y) if want_y else h

    def loss_grad(self, K, U, h0, target):
        n = self._fields(K, U, h0, target)
        g = self.torch.empty(self.nparams, dtype=self.torch.float32, device=self.device)
        loss = C.c_double()
        _check(load().lem_sur_loss_grad(self.ctx, n, _ptr(K), _ptr(U), _ptr(h0), _ptr(target),
                                        _ptr(g), C.byref(loss)), self.ctx)
        return loss.value, g

    def train_step(self, K, U, h0, target, lr, want_loss=True):
        n = self._fields(K, U, h0, target)
        loss = C.c_double()
        _check(load().lem_sur_train_step(self.ctx, n, _ptr(K), _ptr(U), _ptr(h0), _ptr(target),
                                         float(lr), C.byref(loss) if want_loss else None),
               self.ctx)
        return loss.value if want_loss else None

    def activation(self, index, batch):
        """Activation map `index` of the last forward pass as float32
        (bfloat16 values), shape (batch, height, width, channels)."""
        ch, hh, ww = C.c_int32(), C.c_int32(), C.c_int32()
        lib = load()
        _check(lib.lem_sur_activation(self.ctx, index, batch, None, C.byref(ch), C.byref(hh),
                                      C.byref(ww)), self.ctx)
        t = self.torch.empty((batch, hh.value, ww.value, ch.value), dtype=self.torch.int16,
                             device=self.device)
        _check(lib.lem_sur_activation(self.ctx, index, batch, _ptr(t), None, None, None),
               self.ctx)
        self.sync()
        bits = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return bits.view(np.float32)

    def sync(self):
        _check(load().lem_sur_sync(self.ctx), self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            load().lem_sur_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
