"""GPU: the warm-start network's MFMA forward pass, gradients and Adam step
through the C ABI against the FP64 CPU reference (``oracle.surrogate``) with
bfloat16 rounding at the same points.

Tolerance.  Both sides round the same values to bfloat16, but the GPU sums in
float32 and the reference in FP64, so a value lying within float32 error of
a bfloat16 rounding boundary can round the other way: one bfloat16 step
(2^-8 relative) in that element, which then spreads through later layers.
Such flips are rare (float32 error ~1e-6 relative against a 4e-3 spacing),
so whole tensors agree to well under 1e-2 in relative L2 norm (measured:
2e-3 to 7e-3 for the output after fourteen layers); the bounds below are set
there.  The layer-by-layer test is the tight one: each layer recomputed by
the reference from the GPU's own bfloat16 input must match except for
one-step rounding flips in under 1% of the elements.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import surrogate as S
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

REL_Y = 1e-2       # relative L2 error of the network output
REL_GRAD = 2e-2    # relative L2 error of each parameter block's gradient
COS_GRAD = 0.9995  # cosine of the whole gradient vector


def _problem(seed, B, H, W):
    rng = np.random.default_rng(seed)
    from paper_1803_02977_amd import surrogate as sur
    p = sur.init_params(seed)
    # Nonzero biases so that they matter in the forward pass.
    layout, _ = S.param_layout()
    for name, cin, cout in S.layer_table():
        off = layout[name][0] + cout * 9 * cin
        p[off:off + cout] = (rng.standard_normal(cout) * 0.05).astype(np.float32)
    p[layout["head"][0] + 32] = np.float32(0.7)
    K = 1e-5 * np.exp(0.5 * rng.standard_normal((B, H, W)))
    U = np.repeat(rng.uniform(1e-4, 2e-3, B), H * W).reshape(B, H, W)
    h0 = rng.random((B, H, W))
    yy, xx = np.mgrid[0:H, 0:W]
    dome = np.minimum.reduce([yy, xx, H - 1 - yy, W - 1 - xx]).astype(np.float64)
    ht = (U / 1e-3) * 100.0 * (0.1 * dome[None] + 0.2 * rng.random((B, H, W)))
    return p, K, U, h0, ht


def _net(torch, B, H, W):
    from paper_1803_02977_amd.surrogate import Surrogate
    return Surrogate(B, H, W, device=torch.device("cuda:0"))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


SHAPES = [(2, 32, 48), (1, 64, 80), (3, 16, 16)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_forward_matches_reference(shape):
    torch = require_gpu()
    B, H, W = shape
    print(f"[gpu] surrogate forward {shape}", flush=True)
    p, K, U, h0, _ = _problem(1, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    h, y = net.predict(_dev(torch, K), _dev(torch, U), _dev(torch, h0), want_y=True)
    net.sync()
    y = y.cpu().numpy().astype(np.float64)
    ref = S.forward(p.astype(np.float64), K, U, h0, bf16=True)["y"]
    assert _rel(y, ref) < REL_Y, _rel(y, ref)
    # Heights from the GPU's own output follow the stated formula exactly.
    assert np.array_equal(h.cpu().numpy(), S.heights(y, U))
    net.close()


def test_full_batch_forward_equals_single_images_and_reference():
    """Batch 16 of 256 x 256, the benchmark's size: the level-0 convolutions
    have more tiles than resident workgroups, so each workgroup walks several
    tiles (a single image: one tile per workgroup).  The forward pass works
    image by image, so every image's output equals the same image run alone,
    bit for bit, and two of them match the reference."""
    torch = require_gpu()
    B, H, W = 16, 256, 256
    print(f"[gpu] surrogate forward, batch {B} of {H}x{W}", flush=True)
    p, K, U, h0, _ = _problem(5, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    dK, dU, dh = (_dev(torch, a) for a in (K, U, h0))
    _, y = net.predict(dK, dU, dh, want_y=True)
    y = y.cpu().numpy()
    for b in (0, 7, 15):
        sl = slice(b, b + 1)
        _, y1 = net.predict(dK[sl].contiguous(), dU[sl].contiguous(), dh[sl].contiguous(),
                            want_y=True)
        assert np.array_equal(y1.cpu().numpy()[0], y[b]), b
    for b in (0, 15):
        sl = slice(b, b + 1)
        ref = S.forward(p.astype(np.float64), K[sl], U[sl], h0[sl], bf16=True)["y"]
        assert _rel(y[sl].astype(np.float64), ref) < REL_Y, (b, _rel(y[sl], ref))
    net.close()


def test_batch_gradient_is_the_mean_of_single_image_gradients():
    """Batch 4 of 256 x 256: the weight gradient's splits then take several
    patches each (a single image: one patch per split).  The loss is a mean
    over all interior cells, so the batch's loss and gradient are the means of
    the four single-image ones; the output gradient of the batch is a single
    image's times exactly 1/4, so only the float32 summation order of the
    weight and bias gradients differs."""
    torch = require_gpu()
    B, H, W = 4, 256, 256
    print(f"[gpu] surrogate gradient, batch {B} of {H}x{W} against single images", flush=True)
    p, K, U, h0, ht = _problem(6, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    args = [_dev(torch, a) for a in (K, U, h0, ht)]
    loss, g = net.loss_grad(*args)
    g = g.cpu().numpy().astype(np.float64)
    losses, gsum = [], np.zeros_like(g)
    for b in range(B):
        lb, gb = net.loss_grad(*[a[b:b + 1].contiguous() for a in args])
        losses.append(lb)
        gsum += gb.cpu().numpy().astype(np.float64)
    gmean = gsum / B
    assert abs(loss - sum(losses) / B) <= 1e-12 * loss, (loss, losses)
    layout, _ = S.param_layout()
    for name, cin, cout in S.layer_table():
        off = layout[name][0]
        nw = cout * 9 * cin
        for part, (a, b) in (("w", (off, off + nw)), ("b", (off + nw, off + nw + cout))):
            r = _rel(g[a:b], gmean[a:b])
            assert r < 1e-4, (name, part, r)
    ho = layout["head"][0]
    assert _rel(g[ho:], gmean[ho:]) < 1e-4
    net.close()


@pytest.mark.parametrize("shape", SHAPES[:2], ids=lambda s: "x".join(map(str, s)))
def test_gradients_match_reference(shape):
    torch = require_gpu()
    B, H, W = shape
    print(f"[gpu] surrogate gradients {shape}", flush=True)
    p, K, U, h0, ht = _problem(2, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    args = [_dev(torch, a) for a in (K, U, h0, ht)]
    loss, g = net.loss_grad(*args)
    loss2, g2 = net.loss_grad(*args)
    g = g.cpu().numpy().astype(np.float64)
    assert loss == loss2 and np.array_equal(g, g2.cpu().numpy()), "not deterministic"
    ref_loss, ref_g = S.loss_and_grad(p.astype(np.float64), K, U, h0, ht, bf16=True)
    assert abs(loss - ref_loss) <= REL_Y * ref_loss, (loss, ref_loss)
    layout, _ = S.param_layout()
    blocks = [(n, layout[n][0], ci, co) for n, ci, co in S.layer_table()]
    for name, off, cin, cout in blocks:
        nw = cout * 9 * cin
        for part, (a, b) in (("w", (off, off + nw)), ("b", (off + nw, off + nw + cout))):
            r = _rel(g[a:b], ref_g[a:b])
            assert r < REL_GRAD, (name, part, r)
    ho = layout["head"][0]
    assert _rel(g[ho:], ref_g[ho:]) < REL_GRAD
    cos = float(g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g)))
    assert cos > COS_GRAD, cos
    # Padded input channels have exactly zero gradient.
    w0 = g[:32 * 9 * 32].reshape(32, 3, 3, 32)
    assert np.all(w0[..., 3:] == 0.0)
    net.close()


def _ulp_bf16(x):
    """Spacing of bfloat16 numbers at |x| (8 significant bits)."""
    x = np.abs(x)
    e = np.floor(np.log2(np.where(x > 0, x, 1.0)))
    return np.where(x > 0, 2.0 ** (e - 7), 0.0)


def _check_rounded(got, ref, what, max_frac=1e-2):
    """got (GPU, bfloat16 values) against ref (exact, rounded to bfloat16
    once): equal except where float32 summation put the value on the other
    side of a rounding boundary, which moves it by one bfloat16 step (or
    across zero by a negligible amount after ReLU)."""
    diff = np.abs(got - ref)
    bad = diff > 0
    scale = float(np.sqrt(np.mean(ref * ref))) + 1e-30
    big = np.maximum(np.abs(got), np.abs(ref))
    allowed = np.maximum(_ulp_bf16(big) * 1.0000001, 1e-5 * scale)
    assert np.all(diff <= allowed), (what, float((diff / np.maximum(allowed, 1e-300)).max()))
    frac = float(bad.mean())
    assert frac <= max_frac, (what, frac)
    return frac


@pytest.mark.parametrize("shape", [(2, 32, 48), (1, 64, 80)], ids=lambda s: "x".join(map(str, s)))
def test_each_layer_matches_reference_on_the_gpus_own_inputs(shape):
    """Every map of the forward pass recomputed by the reference from the
    GPU's own bfloat16 input of that layer: convolutions (with bias and
    ReLU), pooling, upsampling with concatenation, the head and the
    features."""
    torch = require_gpu()
    B, H, W = shape
    print(f"[gpu] surrogate layer by layer {shape}", flush=True)
    p, K, U, h0, _ = _problem(5, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    _, y = net.predict(_dev(torch, K), _dev(torch, U), _dev(torch, h0), want_y=True)
    net.sync()
    act = {i: net.activation(i, B).astype(np.float64) for i in range(21)}
    P = S.unpack(p.astype(np.float64))
    r = S.bf16_round
    fracs = {}
    fracs["features"] = _check_rounded(act[0], r(S.features(K, U, h0)), "features", 1e-3)

    def conv_check(name, src, dst):
        w, b = P[name]
        ref = r(np.maximum(S.conv3x3(act[src], r(w), b), 0.0))
        fracs[name] = _check_rounded(act[dst], ref, name)

    for level in range(4):
        conv_check(f"enc{level}a", 0 if level == 0 else 8 + level, 1 + 2 * level)
        conv_check(f"enc{level}b", 1 + 2 * level, 2 + 2 * level)
        if level < 3:
            fracs[f"pool{level}"] = _check_rounded(act[9 + level], r(S.pool2(act[2 + 2 * level])),
                                                   f"pool{level}", 1e-3)
    for k, level in enumerate((2, 1, 0)):
        low = act[8] if level == 2 else act[14 + 3 * (k - 1)]
        cat = np.concatenate([S.up2(low), act[2 + 2 * level]], axis=-1)
        assert np.array_equal(act[12 + 3 * k], cat), f"concatenation at level {level}"
        # The concatenation is assembled on request; a smaller batch gets the
        # same leading grids.
        assert np.array_equal(net.activation(12 + 3 * k, 1).astype(np.float64), cat[:1]), level
        conv_check(f"dec{level}a", 12 + 3 * k, 13 + 3 * k)
        conv_check(f"dec{level}b", 13 + 3 * k, 14 + 3 * k)
    wh, bh = P["head"]
    yref = act[20] @ r(wh) + bh[0]
    yg = y.cpu().numpy().astype(np.float64)
    assert np.allclose(yg, yref, rtol=1e-5, atol=1e-5 * np.abs(yref).max())
    print(f"[gpu] mismatch fractions {fracs}", flush=True)
    net.close()


def test_adam_steps_match_reference():
    """Two Adam steps on the GPU against the reference Adam fed the GPU's own
    gradients (the update rule alone: bias correction, moments, step)."""
    torch = require_gpu()
    B, H, W = 2, 32, 32
    p, K, U, h0, ht = _problem(3, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    args = [_dev(torch, a) for a in (K, U, h0, ht)]
    lr = 1e-3
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    cur = p.astype(np.float64)
    for t in (1, 2):
        _, g = net.loss_grad(*args)
        g = g.cpu().numpy().astype(np.float64)
        net.train_step(*args, lr=lr)
        got = net.get_params().cpu().numpy().astype(np.float64)
        ref, m, v = S.adam(cur, g, m, v, t, lr)
        err = np.abs(got - ref)
        assert np.all(err <= 1e-6 * np.abs(ref) + 2e-3 * lr), (t, float(err.max()))
        cur = got
    net.close()


def test_training_reduces_the_loss():
    torch = require_gpu()
    B, H, W = 4, 32, 32
    p, K, U, h0, ht = _problem(4, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    args = [_dev(torch, a) for a in (K, U, h0, ht)]
    first = net.train_step(*args, lr=2e-3)
    for _ in range(60):
        last = net.train_step(*args, lr=2e-3)
    assert np.isfinite(last) and last < 0.3 * first, (first, last)
    net.close()


def test_argument_errors():
    torch = require_gpu()
    from paper_1803_02977_amd import LemError
    net = _net(torch, 2, 16, 16)
    K = torch.ones((3, 16, 16), dtype=torch.float64, device="cuda:0")
    with pytest.raises(LemError):
        net.predict(K, K, K)          # batch above the context's
    with pytest.raises(LemError):
        net.predict(K[:, :8], K[:, :8], K[:, :8])
    with pytest.raises(LemError):
        net.set_params(np.zeros(10, np.float32))
    net.close()


def _gamma(n):
    """Bound on the relative error of a float32 sum of n terms in any order."""
    u = 2.0 ** -24
    return n * u / (1.0 - n * u)


def test_last_layers_gradients_elementwise_on_the_gpus_own_values():
    """Every element of the head's gradient and of the last convolution's
    weight gradient against FP64 sums of the GPU's own bfloat16 activations
    and output.  Bounds per element: a float32 sum of N terms in any order
    (|err| <= gamma_N * sum |terms|), the float32 rounding of the output
    gradient, and -- for the convolution, whose output gradient is rounded to
    bfloat16 -- one bfloat16 step at pixels whose exact value lies within
    float32 error of a rounding boundary (the same flips as in the forward
    layer test)."""
    torch = require_gpu()
    B, H, W = 2, 32, 48
    print("[gpu] surrogate last-layer gradients element by element", flush=True)
    p, K, U, h0, ht = _problem(2, B, H, W)
    net = _net(torch, B, H, W)
    net.set_params(p)
    args = [_dev(torch, a) for a in (K, U, h0, ht)]
    _, y = net.predict(*args[:3], want_y=True)
    net.sync()
    y = y.cpu().numpy().astype(np.float64)
    d0 = net.activation(20, B).astype(np.float64)   # last decoder output
    a0 = net.activation(19, B).astype(np.float64)   # its first convolution's output
    _, g = net.loss_grad(*args)
    g = g.cpu().numpy().astype(np.float64)
    layout, _ = S.param_layout()
    P = S.unpack(p.astype(np.float64))
    r = S.bf16_round
    mask = S.interior_mask(y.shape)
    n = mask.sum()
    t = S.target(ht, U)
    dy = np.where(mask, 2.0 * (y - t) / n, 0.0)
    # float32 error of the GPU's dy: a few roundings of y - t and the scaling.
    e_dy = np.where(mask, 8 * 2.0 ** -24 * (np.abs(y) + np.abs(t)) * 2.0 / n, 0.0)
    N = B * H * W
    # Head: weight gradient and bias gradient.
    ho = layout["head"][0]
    C0 = d0.shape[-1]
    ref_w = (d0 * dy[..., None]).sum(axis=(0, 1, 2))
    tol_w = (_gamma(N) * (np.abs(d0) * np.abs(dy)[..., None]).sum(axis=(0, 1, 2)) +
             (np.abs(d0) * e_dy[..., None]).sum(axis=(0, 1, 2)) + 1e-30)
    assert np.all(np.abs(g[ho:ho + C0] - ref_w) <= tol_w), \
        float(np.max(np.abs(g[ho:ho + C0] - ref_w) / tol_w))
    ref_b = dy.sum()
    tol_b = _gamma(N) * np.abs(dy).sum() + e_dy.sum()
    assert abs(g[ho + C0] - ref_b) <= tol_b, (g[ho + C0], ref_b, tol_b)
    # Last convolution (dec0b): output gradient gz = dy * w_head * [d0 > 0],
    # rounded to bfloat16, against its input a0.
    wh = r(P["head"][0])
    active = d0 > 0
    gz = dy[..., None] * wh[None, None, None, :] * active
    e_gz = (e_dy[..., None] * np.abs(wh)[None, None, None, :] + np.abs(gz) * 2.0 ** -23) * active
    gzr = r(gz)
    # A flip is possible where the exact value is within e_gz of a midpoint.
    lo, hi = r(gz - e_gz), r(gz + e_gz)
    flip = (lo != hi)
    step = np.where(flip, np.maximum(np.abs(hi - gzr), np.abs(lo - gzr)), 0.0)
    wname = "dec0b"
    off = layout[wname][0]
    cout, cin = gz.shape[-1], a0.shape[-1]
    nw = cout * 9 * cin
    ref_dw, _ = S.conv3x3_backward(a0, np.zeros((cout, 3, 3, cin)), gzr)
    abs_dw, _ = S.conv3x3_backward(np.abs(a0), np.zeros((cout, 3, 3, cin)), np.abs(gzr))
    flip_dw, _ = S.conv3x3_backward(np.abs(a0), np.zeros((cout, 3, 3, cin)), step)
    tol_dw = _gamma(N) * abs_dw + flip_dw + 1e-30
    got_dw = g[off:off + nw].reshape(cout, 3, 3, cin)
    ratio = np.abs(got_dw - ref_dw) / tol_dw
    assert np.all(ratio <= 1.0), float(ratio.max())
    # Its bias gradient: the sum of gz (float32, before rounding).
    ref_db = gz.sum(axis=(0, 1, 2))
    tol_db = _gamma(N) * np.abs(gz).sum(axis=(0, 1, 2)) + e_gz.sum(axis=(0, 1, 2))
    got_db = g[off + nw:off + nw + cout]
    assert np.all(np.abs(got_db - ref_db) <= tol_db), float(np.max(np.abs(got_db - ref_db) / tol_db))
    frac = float(flip[active].mean())
    print(f"[gpu] flip-prone output-gradient elements {frac:.2e}", flush=True)
    assert frac < 5e-2, frac
    net.close()
