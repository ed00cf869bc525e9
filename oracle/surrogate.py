"""FP64 CPU reference of the learned warm start (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite and the smoke check are the only
callers.  The GPU library never imports or runs this module, and this module
imports nothing from the library.

The warm start is not in the paper.  It predicts the steady state that the
paper's time loop (Steps 1-7, repeated until heights stop changing) reaches
from a given erodibility field, uplift field and initial surface, so that the
solver can start from the prediction instead of from the noise surface of the
paper's test data (section "Test Data").  At a steady state uplift balances
erosion, so the slope of every cell follows S = (U/K) A^-m (the n = 1 form of
the stream power law of section "The Equation"); heights therefore scale with
U/K, which sets the normalisation of the network's target below.

Network (all shapes NHWC, batch B, an H x W grid with H and W divisible by 8):

* features x0 (32 channels): (ln K - ln 1e-5)/0.5, U/1e-3, h0, then 29 zero
  channels;
* encoder level l = 0..3 with C = 32, 64, 128, 256 channels: two 3x3
  convolutions (zero padding 1, bias) each followed by ReLU; the input of
  level l > 0 is the 2x2 average pool of level l-1's output;
* decoder level l = 2, 1, 0: the channel concatenation [nearest 2x upsample
  of the level below, encoder output of level l] goes through two 3x3
  convolutions with ReLU (C_l output channels);
* head: a 1x1 convolution 32 -> 1 (weights and bias), giving y;
* predicted heights: y * (U/1e-3) * 100 m inside the grid, 0 on the perimeter
  (the fixed base level).

Parameters are one flat float32 vector: for each convolution in the order of
``layer_table()`` the weights [Cout][3][3][Cin] then the bias [Cout]; then the
head weights [32] and bias [1].  The GPU computes with bfloat16 copies of the
weights and bfloat16 activations and accumulates in float32.  ``bf16=True``
rounds, to the nearest bfloat16 (ties to even), exactly the values the GPU
stores in bfloat16: the features, the weights, every convolution output after
ReLU, every pooled map, and the gradient of each convolution's
pre-activation before it enters the weight and input gradients.  Everything
else is exact FP64.  ``bf16=False`` gives the plain FP64 network that the
finite-difference pins check.

Loss: mean over interior cells of (y - t)^2 with t = h_target / ((U/1e-3) 100).
Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (32, 64, 128, 256)
IN_CHANNELS = 32
K_REF = 1e-5
U_REF = 1e-3
H_REF = 100.0
LN_K_SIGMA = 0.5
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def layer_table():
    """(name, cin, cout) of the fourteen 3x3 convolutions, in parameter order."""
    c = CHANNELS
    t = [("enc0a", IN_CHANNELS, c[0]), ("enc0b", c[0], c[0])]
    for level in range(1, 4):
        t += [(f"enc{level}a", c[level - 1], c[level]), (f"enc{level}b", c[level], c[level])]
    for level in (2, 1, 0):
        t += [(f"dec{level}a", c[level + 1] + c[level], c[level]),
              (f"dec{level}b", c[level], c[level])]
    return t


def param_layout():
    """{name: (offset, cin, cout)} and the total parameter count."""
    off, out = 0, {}
    for name, cin, cout in layer_table():
        out[name] = (off, cin, cout)
        off += cout * 9 * cin + cout
    out["head"] = (off, CHANNELS[0], 1)
    off += CHANNELS[0] + 1
    return out, off


def unpack(params):
    """Views of the flat vector: {name: (W [cout,3,3,cin], b [cout])}."""
    layout, total = param_layout()
    p = np.asarray(params, dtype=np.float64)
    assert p.size == total, (p.size, total)
    out = {}
    for name, cin, cout in layer_table():
        off = layout[name][0]
        nw = cout * 9 * cin
        out[name] = (p[off:off + nw].reshape(cout, 3, 3, cin), p[off + nw:off + nw + cout])
    off = layout["head"][0]
    out["head"] = (p[off:off + CHANNELS[0]], p[off + CHANNELS[0]:off + CHANNELS[0] + 1])
    return out


def bf16_round(x):
    """Nearest bfloat16 value (8 significant bits, ties to even), in FP64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)            # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def features(K, U, h0):
    """The 32-channel input map of a batch (K, U, h0: [B, H, W] FP64)."""
    K, U, h0 = (np.asarray(a, dtype=np.float64) for a in (K, U, h0))
    x = np.zeros(K.shape + (IN_CHANNELS,))
    x[..., 0] = (np.log(K) - np.log(K_REF)) / LN_K_SIGMA
    x[..., 1] = U / U_REF
    x[..., 2] = h0
    return x


def target(h, U):
    """The normalised steady state the network is trained to output."""
    return np.asarray(h, np.float64) / ((np.asarray(U, np.float64) / U_REF) * H_REF)


def heights(y, U):
    """Predicted heights from the network output: scaled, perimeter at 0."""
    h = np.asarray(y, np.float64) * ((np.asarray(U, np.float64) / U_REF) * H_REF)
    h[:, 0, :] = 0.0
    h[:, -1, :] = 0.0
    h[:, :, 0] = 0.0
    h[:, :, -1] = 0.0
    return h


def interior_mask(shape):
    m = np.zeros(shape, bool)
    m[:, 1:-1, 1:-1] = True
    return m


def _im2col(x):
    B, H, W, C = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    cols = np.empty((B, H, W, 3, 3, C))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx, :] = xp[:, ky:ky + H, kx:kx + W, :]
    return cols.reshape(B * H * W, 9 * C)


def conv3x3(x, w, b):
    """out[p, co] = b[co] + sum_{ky,kx,ci} x[p + (ky-1, kx-1), ci] w[co,ky,kx,ci]
    with zeros outside the grid."""
    B, H, W, _ = x.shape
    cout = w.shape[0]
    return (_im2col(x) @ w.reshape(cout, -1).T).reshape(B, H, W, cout) + b


def conv3x3_backward(x, w, dz):
    """Weight and input gradients of conv3x3 for the output gradient dz."""
    B, H, W, C = x.shape
    cout = w.shape[0]
    dz2 = dz.reshape(-1, cout)
    dw = (dz2.T @ _im2col(x)).reshape(w.shape)
    dcols = (dz2 @ w.reshape(cout, -1)).reshape(B, H, W, 3, 3, C)
    dxp = np.zeros((B, H + 2, W + 2, C))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + W, :] += dcols[:, :, :, ky, kx, :]
    return dw, dxp[:, 1:-1, 1:-1, :]


def pool2(x):
    """2x2 average pool."""
    return (x[:, 0::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 0::2] + x[:, 1::2, 1::2]) * 0.25


def pool2_backward(g):
    B, H, W, C = g.shape
    out = np.empty((B, 2 * H, 2 * W, C))
    for a in (0, 1):
        for b in (0, 1):
            out[:, a::2, b::2] = 0.25 * g
    return out


def up2(x):
    """Nearest-neighbour 2x upsample."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(g):
    return g[:, 0::2, 0::2] + g[:, 0::2, 1::2] + g[:, 1::2, 0::2] + g[:, 1::2, 1::2]


def forward(params, K, U, h0, bf16=True):
    """All activations of the network and its output y [B, H, W]."""
    r = bf16_round if bf16 else (lambda v: v)
    P = unpack(params)
    Wr = {k: (r(w), b) for k, (w, b) in P.items()}
    act = {"x0": r(features(K, U, h0))}

    def block(x, la, lb):
        a = r(np.maximum(conv3x3(x, *Wr[la]), 0.0))
        e = r(np.maximum(conv3x3(a, *Wr[lb]), 0.0))
        return a, e

    x = act["x0"]
    for level in range(4):
        act[f"in_enc{level}"] = x
        act[f"a_enc{level}"], act[f"e{level}"] = block(x, f"enc{level}a", f"enc{level}b")
        if level < 3:
            x = r(pool2(act[f"e{level}"]))
    d = act["e3"]
    for level in (2, 1, 0):
        cat = np.concatenate([up2(d), act[f"e{level}"]], axis=-1)
        act[f"in_dec{level}"] = cat
        act[f"a_dec{level}"], d = block(cat, f"dec{level}a", f"dec{level}b")
        act[f"d{level}"] = d
    wh, bh = Wr["head"]
    act["y"] = d @ wh + bh[0]
    return act


def loss_and_grad(params, K, U, h0, h_target, bf16=True):
    """Mean squared error over interior cells and its gradient (flat FP64)."""
    r = bf16_round if bf16 else (lambda v: v)
    act = forward(params, K, U, h0, bf16)
    P = unpack(params)
    Wr = {k: r(w) for k, (w, _) in P.items()}
    y = act["y"]
    mask = interior_mask(y.shape)
    n = mask.sum()
    diff = np.where(mask, y - target(h_target, U), 0.0)
    loss = float((diff * diff).sum() / n)
    dy = 2.0 * diff / n
    grads = {}
    d0 = act["d0"]
    grads["head"] = ((d0 * dy[..., None]).sum(axis=(0, 1, 2)), np.array([dy.sum()]))
    g = dy[..., None] * Wr["head"][None, None, None, :]

    def block_bwd(x, a, e, ge, la, lb, need_dx=True):
        gz = ge * (e > 0)
        dwb, ga = conv3x3_backward(a, Wr[lb], r(gz))
        grads[lb] = (dwb, gz.sum(axis=(0, 1, 2)))
        gz = ga * (a > 0)
        dwa, gx = conv3x3_backward(x, Wr[la], r(gz))
        grads[la] = (dwa, gz.sum(axis=(0, 1, 2)))
        return gx if need_dx else None

    skip = {}
    for level in (0, 1, 2):
        gcat = block_bwd(act[f"in_dec{level}"], act[f"a_dec{level}"], act[f"d{level}"], g,
                         f"dec{level}a", f"dec{level}b")
        cu = CHANNELS[level + 1]
        g = up2_backward(gcat[..., :cu])
        skip[level] = gcat[..., cu:]
    for level in (3, 2, 1, 0):
        gx = block_bwd(act[f"in_enc{level}"], act[f"a_enc{level}"], act[f"e{level}"], g,
                       f"enc{level}a", f"enc{level}b", need_dx=level > 0)
        if level > 0:
            g = skip[level - 1] + pool2_backward(gx)
    layout, total = param_layout()
    flat = np.zeros(total)
    for name, cin, cout in layer_table():
        off = layout[name][0]
        nw = cout * 9 * cin
        flat[off:off + nw] = grads[name][0].ravel()
        flat[off + nw:off + nw + cout] = grads[name][1]
    off = layout["head"][0]
    flat[off:off + CHANNELS[0]] = grads["head"][0]
    flat[off + CHANNELS[0]] = grads["head"][1][0]
    return loss, flat


def adam(params, grad, m, v, t, lr):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return params - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
