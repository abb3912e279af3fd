"""Pins of the FP64 reference of the warm-start network (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import unet as U


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(U.num_params())
    offs, hw, hb, _ = U.layout()
    for (cin, cout), (wo, bo) in zip(U.LAYERS, offs):
        p[wo:bo] = rng.normal(0, scale * np.sqrt(2.0 / (27 * cin)), bo - wo)
        p[bo:bo + cout] = rng.normal(0, 0.05, cout)
    p[hw:hw + 16] = rng.normal(0, 0.3, 16)
    p[hb] = 0.1
    return p


def test_param_count_by_hand():
    # 27*cin*cout + cout per convolution, summed by hand, plus the 1x1 head
    per_layer = [3472, 6928, 13856, 27680, 55360, 110656, 82976, 27680, 20752, 6928]
    assert U.num_params() == sum(per_layer) + 17 == 356305


def test_round_bf16_ties_to_even():
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + 2 * e, -1 - e, 3.0e-3, 1 + 1.01 * e])
    want = np.array([1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -1.0, None, 1 + 2 * e], dtype=object)
    got = U.round_bf16(vals)
    for g, w in zip(got, want):
        if w is not None:
            assert g == w
    # 8 significant bits: the error is at most half a unit in the last place, 2^-8 |x|
    x = np.random.default_rng(0).normal(size=1000) * 10.0 ** np.random.default_rng(1).integers(
        -5, 5, 1000)
    r = U.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))
    assert np.array_equal(U.from_bf16_bits(U.to_bf16_bits(x)), r)


def test_conv3_library_equals_direct_sum():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(3, 4, 5, 3))
    w = rng.normal(size=(4, 27, 3))
    b = rng.normal(size=4)
    assert np.allclose(U.conv3_cl(x, w, b), U.conv3_brute(x, w, b), rtol=0, atol=1e-12)
    # an impulse reproduces the mirrored kernel (tap order: x1 fastest)
    imp = np.zeros((3, 3, 3, 1))
    imp[1, 1, 1, 0] = 1.0
    w1 = np.arange(27.0).reshape(1, 27, 1)
    y = U.conv3_cl(imp, w1, None)[..., 0]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # y[1-dz, 1-dy, 1-dx] sees the impulse through tap (dz, dy, dx)
                assert y[1 - dz, 1 - dy, 1 - dx] == (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)


def test_first_layer_of_forward_uses_the_flat_layout():
    rng = np.random.default_rng(4)
    mask = (rng.random((4, 4, 8)) < 0.3).astype(np.uint8)
    p = _params(5)
    _, acts = U.forward(p, mask, 0.5, 1.0, return_acts=True)
    offs, _, _, _ = U.layout()
    wo, bo = offs[0]
    w = p[wo:bo].reshape(16, 27, 8)
    x = np.moveaxis(U.features(mask, 0.5, 1.0), 0, -1)
    ref = np.maximum(U.conv3_brute(x, w, p[bo:bo + 16]), 0.0)
    assert np.allclose(np.moveaxis(acts["a1"].numpy(), 0, -1), ref, atol=1e-12)


def test_pool_and_upsample():
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.normal(size=(3, 4, 6, 8)))
    assert torch.allclose(U.pool2(U.up2(x)), x, atol=0)
    c = torch.full((2, 4, 4, 4), 1.5, dtype=torch.float64)
    assert torch.all(U.pool2(c) == 1.5)
    # the block mean by hand
    assert float(U.pool2(x)[1, 0, 1, 2]) == pytest.approx(float(x[1, 0:2, 2:4, 4:6].mean()))


def test_output_masked_and_loss_over_water_only():
    rng = np.random.default_rng(7)
    mask = (rng.random((8, 4, 4)) < 0.3).astype(np.uint8)
    p = _params(8)
    y = U.forward(p, mask, 0.1, 2.0).numpy()
    assert np.all(y[mask == 1] == 0) and np.all((y[mask == 0] > 0) & (y[mask == 0] < 1))
    t = rng.random(mask.shape)
    l1 = U.loss_value(p, mask, t, 0.1, 2.0)
    t2 = t.copy()
    t2[mask == 1] = 5.0
    assert U.loss_value(p, mask, t2, 0.1, 2.0) == l1
    assert l1 == pytest.approx(np.mean((y - t)[mask == 0] ** 2), rel=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(9)
    mask = (rng.random((4, 4, 8)) < 0.25).astype(np.uint8)
    t = rng.random(mask.shape)
    p = _params(10)
    loss, g = U.loss_and_grad(p, mask, t, 0.3, 1.5)
    offs, hw, hb, n = U.layout()
    idx = [hw + 3, hb]
    for (wo, bo), (cin, cout) in zip(offs, U.LAYERS):
        idx += list(rng.integers(wo, bo, 3)) + [bo + int(rng.integers(0, cout))]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (U.loss_value(pp, mask, t, 0.3, 1.5) - U.loss_value(pm, mask, t, 0.3, 1.5)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
    # unused input channels 3..7 of the first convolution get no gradient
    w0 = g[offs[0][0]:offs[0][1]].reshape(16, 27, 8)
    assert np.all(w0[:, :, 3:] == 0)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(11)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    q, m, v = U.adam(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    # bias-corrected first moments: m_hat = g, v_hat = g^2
    assert np.allclose(q, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
