"""The warm-start network's CPU reference against what pins it from outside:
SciPy's 2-D correlation, adjoint identities, finite differences of the FP64
loss, exact bfloat16 rounding, and Adam's closed form under a constant
gradient."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.signal
import torch

from oracle import surrogate as S


def _rng(seed):
    return np.random.default_rng(seed)


def test_layer_table_shapes():
    t = S.layer_table()
    assert len(t) == 14
    assert t[0] == ("enc0a", 32, 32) and t[7] == ("enc3b", 256, 256)
    assert dict((n, (ci, co)) for n, ci, co in t)["dec2a"] == (384, 128)
    assert dict((n, (ci, co)) for n, ci, co in t)["dec0a"] == (96, 32)
    _, total = S.param_layout()
    assert total == sum(co * 9 * ci + co for _, ci, co in t) + 33


def test_conv_matches_scipy_correlation():
    rng = _rng(1)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = S.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(scipy.signal.correlate2d(x[n, :, :, ci], w[co, :, :, ci], mode="same",
                                                       boundary="fill") for ci in range(3))
            assert np.allclose(got[n, :, :, co], ref, rtol=1e-13, atol=1e-13)


def test_conv_backward_is_the_adjoint():
    rng = _rng(2)
    x = rng.standard_normal((2, 6, 5, 4))
    w = rng.standard_normal((3, 3, 3, 4))
    dz = rng.standard_normal((2, 6, 5, 3))
    y = S.conv3x3(x, w, np.zeros(3))
    dw, dx = S.conv3x3_backward(x, w, dz)
    lhs = (y * dz).sum()
    assert np.isclose(lhs, (dw * w).sum(), rtol=1e-12)
    assert np.isclose(lhs, (dx * x).sum(), rtol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = _rng(3)
    x = rng.standard_normal((2, 8, 6, 3))
    g = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose((S.pool2(x) * g).sum(), (x * S.pool2_backward(g)).sum(), rtol=1e-12)
    gu = rng.standard_normal((2, 8, 6, 3))
    assert np.isclose((S.up2(g) * gu).sum(), (g * S.up2_backward(gu)).sum(), rtol=1e-12)
    assert np.array_equal(S.pool2(S.up2(g)), g)
    assert np.allclose(S.pool2(np.full((1, 4, 4, 2), 3.5)), 3.5)


def test_bf16_rounding_is_round_to_nearest_even():
    # Values exactly representable in float32: torch's float32 -> bfloat16
    # conversion rounds to nearest, ties to even.
    rng = _rng(4)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8,
                         -(1.0 + 2.0 ** -8), 255.5, 256.5, 2.0 ** -120]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(v.astype(np.float64)), ref)
    assert S.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert S.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert S.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -30) == 1.0 + 2.0 ** -7


def _tiny_problem(seed, H=16, W=16, B=1, scale=1.0):
    rng = _rng(seed)
    _, total = S.param_layout()
    p = np.zeros(total)
    layout, _ = S.param_layout()
    for name, cin, cout in S.layer_table():
        off = layout[name][0]
        nw = cout * 9 * cin
        fan = 9 * (3 if name == "enc0a" else cin)
        p[off:off + nw] = rng.standard_normal(nw) * np.sqrt(2.0 / fan) * scale
        p[off + nw:off + nw + cout] = rng.standard_normal(cout) * 0.05
    off = layout["head"][0]
    p[off:off + 32] = rng.standard_normal(32) * np.sqrt(1.0 / 32)
    p[off + 32] = 0.3
    K = 1e-5 * np.exp(0.5 * rng.standard_normal((B, H, W)))
    U = np.full((B, H, W), rng.uniform(1e-4, 2e-3))
    h0 = rng.random((B, H, W))
    ht = rng.random((B, H, W)) * 300.0
    return p, K, U, h0, ht


def test_gradient_matches_finite_differences():
    p, K, U, h0, ht = _tiny_problem(5)
    loss, g = S.loss_and_grad(p, K, U, h0, ht, bf16=False)
    assert np.isfinite(loss) and loss > 0
    layout, total = S.param_layout()
    rng = _rng(6)
    idx = []
    for name, cin, cout in S.layer_table():
        off = layout[name][0]
        nw = cout * 9 * cin
        real = [i for i in range(nw) if name != "enc0a" or (i % cin) < 3]
        idx += [off + int(i) for i in rng.choice(real, 3, replace=False)]
        idx.append(off + nw + int(rng.integers(cout)))
    idx += [layout["head"][0] + 5, layout["head"][0] + 32]
    for i in idx:
        e = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        fd = (S.loss_and_grad(pp, K, U, h0, ht, bf16=False)[0]
              - S.loss_and_grad(pm, K, U, h0, ht, bf16=False)[0]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(fd), 1e-4 * abs(loss)), (i, fd, g[i])
    # Padded input channels never see a nonzero input.
    off, cin = layout["enc0a"][0], 32
    w0 = g[off:off + 32 * 9 * cin].reshape(32, 3, 3, cin)
    assert np.all(w0[..., 3:] == 0.0)


def test_bf16_network_stays_close_to_the_exact_one():
    p, K, U, h0, ht = _tiny_problem(7)
    y_exact = S.forward(p, K, U, h0, bf16=False)["y"]
    y_bf16 = S.forward(p, K, U, h0, bf16=True)["y"]
    rel = np.linalg.norm(y_bf16 - y_exact) / np.linalg.norm(y_exact)
    assert 0 < rel < 5e-2


def test_adam_under_a_constant_gradient_moves_by_lr_times_sign():
    """With g constant the bias-corrected moments equal g and g^2 at every
    step, so each step is lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -1e-3, 2.0, -7.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-2
    for t in range(1, 8):
        q, m, v = S.adam(p, g, m, v, t, lr)
        assert np.allclose(p - q, lr * g / (np.abs(g) + S.ADAM_EPS), rtol=1e-9, atol=0)
        p = q
    q, _, _ = S.adam(p, np.zeros(4), np.zeros(4), np.zeros(4), 1, lr)
    assert np.array_equal(q, p)


@pytest.mark.parametrize("shape", [(16, 24), (8, 8)])
def test_heights_and_target_round_trip(shape):
    rng = _rng(8)
    U = np.full((2,) + shape, 7e-4)
    h = rng.random((2,) + shape) * 100
    h[:, 0, :] = h[:, -1, :] = h[:, :, 0] = h[:, :, -1] = 0.0
    assert np.allclose(S.heights(S.target(h, U), U), h, rtol=1e-15, atol=0)
