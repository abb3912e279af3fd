"""Warm-start network on the GPU (BF16 matrix cores) against the FP64 reference.

Bars, derived from the arithmetic: a convolution output is the FP32 sum of
K = 27 cin products of BF16-rounded operands, rounded once to BF16.  Against
the exact FP64 sum of the same rounded operands the error is at most
2^-8 |y| (the final rounding) + K 2^-24 S, where S is the same sum taken over
absolute values (FP32 accumulation).  Whole-network outputs compound such
roundings through ten layers; they are compared with the reference that
rounds at the same points, within bounds stated per test.
"""
import numpy as np
import pytest

import pf_inputs as pi
from oracle import unet as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402

DEV = "cuda:0"


def bits_to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(U.to_bf16_bits(a))).to(DEV)


def dev_to_f64(t):
    return U.from_bf16_bits(t.cpu().numpy())


def conv_bound(x, w, b, y_exact):
    """2^-8 |y| + K 2^-24 S per output element (see the module docstring)."""
    K = 27 * w.shape[2]
    S = U.conv3_cl(np.abs(x), np.abs(w), None if b is None else np.abs(b))
    return 2.0 ** -8 * np.abs(y_exact) + K * 2.0 ** -24 * S + 1e-30


def test_mfma_operand_layout():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(16, 32)).astype(np.float32)
    b = rng.normal(size=(32, 16)).astype(np.float32)
    c = pf.mfma_probe(torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)).cpu().numpy()
    ref = U.round_bf16(a) @ U.round_bf16(b)
    S = np.abs(U.round_bf16(a)) @ np.abs(U.round_bf16(b))
    assert np.all(np.abs(c - ref) <= 32 * 2.0 ** -24 * S + 1e-30)


CONV_CASES = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (48, 16),
              (16, 48), (32, 96)]


@pytest.mark.parametrize("cin,cout", CONV_CASES)
@pytest.mark.parametrize("shape", [(7, 10, 13), (4, 4, 4), (16, 8, 24), (32, 48, 48), (33, 41, 50)])
def test_conv_forward(cin, cout, shape):
    rng = np.random.default_rng(cin * 1000 + cout + shape[0])
    x = U.round_bf16(rng.normal(size=shape + (cin,)))
    w = rng.normal(0, np.sqrt(2.0 / (27 * cin)), size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    wb = U.round_bf16(w)
    for relu in (False, True):
        y = pf.conv3_bf16(bits_to_dev(x), torch.from_numpy(w).to(DEV),
                          torch.from_numpy(b).to(DEV), relu, cout)
        got = dev_to_f64(y)
        ex = U.conv3_cl(x, wb, b.astype(np.float64))
        if relu:
            ex = np.maximum(ex, 0.0)
        bound = conv_bound(x, wb, b.astype(np.float64), ex)
        assert np.all(np.abs(got - ex) <= bound), float(np.max(np.abs(got - ex) - bound))


@pytest.mark.parametrize("cin,cout", [(48, 16), (16, 16), (8, 16), (16, 32)])
def test_conv_forward_large_forms_ragged(cin, cout):
    """A grid large enough for the forms taken on full-resolution grids (the
    x-folded form for 16 output channels, with 14 outputs per row of 16
    positions; 8-plane tiles; register blocks for 16 -> 32), ragged in every
    direction for each of them: every voxel against the exact sum."""
    shape = (45, 62, 71)
    rng = np.random.default_rng(cin * 31 + cout)
    x = U.round_bf16(rng.normal(size=shape + (cin,)))
    w = rng.normal(0, np.sqrt(2.0 / (27 * cin)), size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    wb = U.round_bf16(w)
    ex = U.conv3_cl(x, wb, b.astype(np.float64))
    bound = conv_bound(x, wb, b.astype(np.float64), ex)
    for relu in (False, True):
        y = pf.conv3_bf16(bits_to_dev(x), torch.from_numpy(w).to(DEV),
                          torch.from_numpy(b).to(DEV), relu, cout)
        got = dev_to_f64(y)
        ref = np.maximum(ex, 0.0) if relu else ex
        assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) - bound))


@pytest.mark.parametrize("cin,cout", [(8, 16), (16, 16), (16, 32), (32, 64), (64, 64),
                                      (96, 32), (48, 16), (32, 32)])
@pytest.mark.parametrize("shape", [(7, 10, 13), (16, 8, 24), (21, 17, 70)])
def test_conv_backward(cin, cout, shape):
    """(21, 17, 70): twelve voxel ranges of the weight gradient, its 32 x 2 x 2
    blocks ragged in every direction."""
    rng = np.random.default_rng(7 * cin + cout + shape[0])
    x = U.round_bf16(rng.normal(size=shape + (cin,)))
    w = rng.normal(0, np.sqrt(2.0 / (27 * cin)), size=(cout, 27, cin)).astype(np.float32)
    dy = U.round_bf16(rng.normal(size=shape + (cout,)))
    want_dx = cin % 16 == 0
    dx, dw, db = pf.conv3_bf16_backward(bits_to_dev(x), torch.from_numpy(w).to(DEV),
                                        bits_to_dev(dy), want_dx)
    ref = U.conv3_cl_grads(x, U.round_bf16(w), dy)
    nvox = int(np.prod(shape))
    # weight gradient: FP32 sums over all voxels of BF16 products
    Sw = U.conv3_cl_grads(np.abs(x), np.abs(U.round_bf16(w)), np.abs(dy))["dw"]
    dwg = dw.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dwg - ref["dw"]) <= nvox * 2.0 ** -24 * Sw + 1e-30)
    Sb = np.abs(dy).reshape(-1, cout).sum(axis=0)
    assert np.all(np.abs(db.cpu().numpy() - ref["db"]) <= nvox * 2.0 ** -24 * Sb + 1e-30)
    if want_dx:
        gx = dev_to_f64(dx)
        Sx = U.conv3_cl_grads(np.abs(x), np.abs(U.round_bf16(w)), np.abs(dy))["dx"]
        bound = 2.0 ** -8 * np.abs(ref["dx"]) + 27 * cout * 2.0 ** -24 * Sx + 1e-30
        assert np.all(np.abs(gx - ref["dx"]) <= bound)


def _sample(shape, seed, glass=0.3):
    rng = np.random.default_rng(seed)
    mask = (rng.random(shape) < glass).astype(np.uint8)
    target = (rng.random(shape) < 0.6).astype(np.float32)
    target[mask == 1] = 0
    return mask, target


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


@pytest.mark.parametrize("variant", ["tiled", "direct", "reg"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 20, 24), (8, 36, 20), (32, 48, 48)])
def test_forward_matches_reference(shape, variant):
    net = pf.UNet(seed=3)
    net.set_conv_kernel(variant)
    p = net.get_params().astype(np.float64)
    mask, _ = _sample(shape, 1)
    for dT, ls in ((0.5, 0.0), (0.03, 2.7)):
        got = net.forward(_dev(mask, torch.uint8), dT, ls).cpu().numpy().astype(np.float64)
        ref_b = U.forward(p, mask, dT, ls, bf16=True).numpy()
        ref = U.forward(p, mask, dT, ls).numpy()
        assert np.all(got[mask == 1] == 0)
        # same rounding points: only FP32 accumulation order and the odd
        # one-ulp BF16 difference that it causes, propagated to the output
        assert np.abs(got - ref_b).max() <= 2e-2 and np.abs(got - ref_b).mean() <= 1e-3
        # against exact FP64: BF16 storage through ten layers (relative
        # 2^-8 per rounding, a few dozen roundings along any path)
        assert np.abs(got - ref).max() <= 5e-2 and np.abs(got - ref).mean() <= 5e-3


def routing_params(seed: int):
    """Parameters of a network whose every convolution copies one input channel
    at one tap (weight 1, bias 0): with the glass mask and the constant 1
    features as input, every activation is a multiple of 1/64 in [0, 1], so
    BF16 storage, FP32 accumulation and pooling are exact and the forward
    pass has one correct value per voxel.  The decoder convolutions take half
    of their outputs from the upsampled path and half from the skip."""
    rng = np.random.default_rng(seed)
    offs, hw, hb, n = U.layout()
    p = np.zeros(n, np.float32)
    for i, ((cin, cout), (wo, bo)) in enumerate(zip(U.LAYERS, offs)):
        w = np.zeros((cout, 27, cin), np.float32)
        for co in range(cout):
            if i == 0:  # mostly the glass mask, some constant features
                src = 0 if co % 4 else int(rng.integers(1, 3))
            elif i in (6, 8):                             # [upsampled, skip]
                n_up = cin - (32 if i == 6 else 16)
                src = int(rng.integers(0, n_up)) if co < cout // 2 else \
                    int(rng.integers(n_up, cin))
            else:
                src = int(rng.integers(0, cin))
            w[co, int(rng.integers(0, 27)), src] = 1.0
        p[wo:bo] = w.ravel()
    return p, hw, hb


@pytest.mark.parametrize("variant", ["tiled", "direct", "reg"])
@pytest.mark.parametrize("shape", [(12, 20, 24), (8, 8, 16), (32, 48, 48)])
def test_forward_exact_routing_network_every_voxel(shape, variant):
    """Element-wise check of the whole forward pass, glue included (pooling,
    upsampling, the concatenation halves, zero padding at the borders, the
    head and its masking): each of the 16 channels of the last convolution
    is read out through a one-hot head, and every voxel must equal the
    reference up to the sigmoid's FP32 rounding (no other rounding happens;
    the reference with and without BF16 storage agree exactly)."""
    _routing_check(shape, variant, range(16))


def test_forward_exact_routing_network_large_grid():
    """The same on a grid large enough for the full-resolution layers' large
    forms (16 x 4 x 8 LDS tiles for 16 output channels, the register blocks
    for 16 -> 32; four readouts: the FP64 reference takes seconds per forward
    pass here)."""
    _routing_check((84, 80, 80), "reg", (0, 5, 10, 15))


def _routing_check(shape, variant, readouts):
    net = pf.UNet(seed=1)
    net.set_conv_kernel(variant)
    mask, _ = _sample(shape, 5)
    dT, ls = 2.0, 3.0   # input features log10(dT/0.2) = 1 and (ls - 1.5)/1.5 = 1
    p, hw, hb = routing_params(11 + shape[0])
    md = _dev(mask, torch.uint8)
    distinct = set()
    for c in readouts:
        p[hw:hw + 16] = 0.0
        p[hw + c] = 1.0
        p[hb] = -0.25
        net.set_params(p)
        got = net.forward(md, dT, ls).cpu().numpy().astype(np.float64)
        ref_b = U.forward(p.astype(np.float64), mask, dT, ls, bf16=True).numpy()
        ref = U.forward(p.astype(np.float64), mask, dT, ls).numpy()
        assert np.array_equal(ref_b, ref)  # nothing is rounded on the way
        assert np.all(got[mask == 1] == 0)
        err = np.abs(got - ref)
        assert np.all(err <= 2.0 ** -21), (c, float(err.max()), np.argwhere(err > 2.0 ** -21)[:5])
        distinct.update(np.unique(np.round(ref[mask == 0], 9)).tolist())
    # the readouts see many different activation values (not a constant net)
    assert len(distinct) >= 8
    net.close()


def test_forward_deterministic():
    net = pf.UNet(seed=4)
    mask, _ = _sample((16, 16, 16), 2)
    m = _dev(mask, torch.uint8)
    a = net.forward(m, 0.2, 1.0).cpu().numpy()
    b = net.forward(m, 0.2, 1.0).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["tiled", "direct", "reg"])
def test_gradient_matches_reference(variant):
    shape = (16, 16, 16)
    net = pf.UNet(seed=5)
    net.set_conv_kernel(variant)
    p = net.get_params().astype(np.float64)
    mask, target = _sample(shape, 3)
    loss, g = net.grad(_dev(mask, torch.uint8), _dev(target, torch.float32), 0.4, 1.0)
    loss_r, g_r = U.loss_and_grad(p, mask, target, 0.4, 1.0)
    assert loss == pytest.approx(loss_r, rel=2e-2)
    offs, hw, hb, _ = U.layout()
    blocks = [(wo, bo) for wo, bo in offs] + [(bo, bo + c) for (wo, bo), (_, c) in
                                              zip(offs, U.LAYERS)] + [(hw, hb + 1)]
    for lo, hi in blocks:
        a, r = g[lo:hi].astype(np.float64), g_r[lo:hi]
        nr = np.linalg.norm(r)
        if nr == 0:
            assert np.all(a == 0)
            continue
        cos = float(a @ r / (np.linalg.norm(a) * nr))
        assert cos >= 0.995 and np.linalg.norm(a - r) / nr <= 0.1, (lo, hi, cos)
    # determinism of the fixed-order reductions
    loss2, g2 = net.grad(_dev(mask, torch.uint8), _dev(target, torch.float32), 0.4, 1.0)
    assert loss2 == loss and np.array_equal(g, g2)


def test_adam_step_matches_reference():
    shape = (8, 8, 16)
    net = pf.UNet(seed=6)
    p0 = net.get_params()
    mask, target = _sample(shape, 4)
    m, t = _dev(mask, torch.uint8), _dev(target, torch.float32)
    _, g = net.grad(m, t, 0.2, 0.5)
    net.train_step(m, t, 0.2, 0.5, lr=1e-3)
    p1 = net.get_params()
    want, _, _ = U.adam(p0.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    assert np.abs(p1 - want).max() <= 1e-6 * (1 + np.abs(p0).max())


def test_training_reduces_loss():
    shape = (16, 16, 16)
    net = pf.UNet(seed=7)
    mask, target = _sample(shape, 5)
    # a target with structure: ice on water cells above the middle plane
    target = np.zeros(shape, np.float32)
    target[8:] = 1.0
    target[mask == 1] = 0.0
    m, t = _dev(mask, torch.uint8), _dev(target, torch.float32)
    losses = [net.train_step(m, t, 0.5, 1.0, lr=1e-3) for _ in range(60)]
    assert np.mean(losses[-5:]) < 0.3 * losses[0], losses[::5]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_warmstart_writes_prediction(precision):
    c = pi.case_micro_32()
    s = pf.Solver(c.params, c.mask, precision, c.run)
    net = pf.UNet(seed=8)
    dT, ls = c.params["dT"], 0.0
    pred = net.forward(_dev(c.mask, torch.uint8), dT, ls).cpu().numpy()
    net.warmstart(s, dT, ls, mode="all")
    phi, _ = s.get_state()
    assert np.array_equal(phi.reshape(pred.shape), pred.astype(phi.dtype))
    # restricted to the water component(s) of the nucleus
    s.set_state(c.phi0.astype(phi.dtype))
    net.warmstart(s, dT, ls)
    phi2, _ = s.get_state()
    keep = U.nucleus_component(c.mask, c.phi0)
    assert np.array_equal(phi2[keep], pred[keep].astype(phi.dtype))
    assert np.all(phi2[~keep] == 0)
    # the baseline without the network: 1 on the nucleus's component
    s.set_state(c.phi0.astype(phi.dtype))
    net.warmstart(s, dT, ls, mode="flood")
    phi3, _ = s.get_state()
    assert np.array_equal(phi3, keep.astype(phi.dtype))
    s.close()


@pytest.mark.parametrize("seed", [20000, 20001])
def test_nucleus_component_on_bead_packs(seed):
    """Reachable water on a generated bead pack with sealed pockets, and on a
    grid where a glass wall cuts the box in two."""
    c = pi.warmstart_instance(seed, edge=48)
    mask = c.mask.copy()
    cx = c.meta["nucleus_centre"] % 48
    mask[:, :, (cx + 24) % 48] = 1  # a glass wall half a box away from the nucleus
    mask[:, :, (cx + 25) % 48] = 1
    s = pf.Solver(dict(c.params), mask, "fp32", c.run)
    phi0 = c.phi0.astype(np.float32)
    phi0[mask == 1] = 0
    s.set_state(phi0)
    net = pf.UNet(seed=2)
    net.warmstart(s, c.meta["dT"], 1.0)
    phi, _ = s.get_state()
    keep = U.nucleus_component(mask, phi0)
    assert keep.sum() > 0 and (~keep & (mask == 0)).sum() > 0
    assert np.all(phi[~keep] == 0) and np.all(phi[keep] > 0)
    s.close()


def test_errors():
    net = pf.UNet(seed=9)
    m = torch.zeros((6, 8, 8), dtype=torch.uint8, device=DEV)
    with pytest.raises(pf.PFError):
        net.forward(m, 0.5, 0.0)  # n3 = 6 is not a multiple of 4
    m = torch.zeros((8, 8, 8), dtype=torch.uint8, device=DEV)
    with pytest.raises(pf.PFError):
        net.forward(m, -1.0, 0.0)
    rc = pf.lib().pf_conv3_bf16(0, 8, 0, 0, 0, 0, 16, 4, 4, 4, 0)
    assert rc == pf.PF_EINVAL


def test_convolution_beyond_32bit_offsets_sampled():
    """A 512^3 grid of 16 channels: the input and the output each span 4 GiB,
    past the 32-bit byte offsets of the tiled forms, so the launcher takes the
    direct kernel (64-bit indexing); sampled voxels (the corners among them)
    against the direct sum."""
    edge, cin, cout = 512, 16, 16
    rng = np.random.default_rng(512)
    shape = (edge, edge, edge)
    g = torch.Generator(device=DEV)
    g.manual_seed(512)
    xb = torch.randint(-16000, 16000, shape + (cin,), dtype=torch.int16, device=DEV, generator=g)
    xb &= -32641  # sign and low mantissa bits; exponent set below
    xb |= 123 << 7
    w = rng.normal(0, 0.05, size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    y = pf.conv3_bf16(xb, torch.from_numpy(w).to(DEV), torch.from_numpy(b).to(DEV), False, cout)
    wb = U.round_bf16(w)
    pts = [(0, 0, 0), (edge - 1, edge - 1, edge - 1), (0, edge - 1, 0), (edge - 1, 0, edge - 1),
           (edge // 2, edge - 1, 3)] + [tuple(int(v) for v in rng.integers(0, edge, 3))
                                         for _ in range(60)]
    for z, yy, x in pts:
        z0, z1 = max(z - 1, 0), min(z + 2, edge)
        y0, y1 = max(yy - 1, 0), min(yy + 2, edge)
        x0, x1 = max(x - 1, 0), min(x + 2, edge)
        patch = dev_to_f64(xb[z0:z1, y0:y1, x0:x1].contiguous())
        ref = U.conv3_brute(patch, wb, b.astype(np.float64))[z - z0, yy - y0, x - x0]
        S = U.conv3_brute(np.abs(patch), np.abs(wb), np.abs(b).astype(np.float64))[
            z - z0, yy - y0, x - x0]
        got = dev_to_f64(y[z, yy, x].contiguous())
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 27 * cin * 2.0 ** -24 * S)
    del xb, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("edge", [96, 192])
@pytest.mark.parametrize("cin,cout", [(48, 16), (16, 16), (8, 16), (16, 32)])
def test_full_size_convolution_sampled(edge, cin, cout):
    """The full-resolution convolutions at the benchmark grids (the largest,
    48 -> 16 channels, and the other shapes of the large forms: 16 x 4 x 8
    LDS tiles for 16 output channels, register blocks for 16 -> 32); sampled
    voxels against the direct sum."""
    rng = np.random.default_rng(edge + cin)
    shape = (edge, edge, edge)
    xb = torch.randint(-16000, 16000, shape + (cin,), dtype=torch.int16, device=DEV)
    # keep the BF16 values moderate: sign, exponent in [-8, 1]
    xb = (xb & -32768) | ((torch.randint(119, 128, shape + (cin,), device=DEV) << 7)
                          .to(torch.int16)) | (xb & 127)
    w = rng.normal(0, 0.05, size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    y = pf.conv3_bf16(xb, torch.from_numpy(w).to(DEV), torch.from_numpy(b).to(DEV), False, cout)
    wb = U.round_bf16(w)
    pts = [(0, 0, 0), (edge - 1, edge - 1, edge - 1), (0, edge - 1, 5)] + [
        tuple(int(v) for v in rng.integers(0, edge, 3)) for _ in range(300)]
    for z, yy, x in pts:
        z0, z1 = max(z - 1, 0), min(z + 2, edge)
        y0, y1 = max(yy - 1, 0), min(yy + 2, edge)
        x0, x1 = max(x - 1, 0), min(x + 2, edge)
        patch = dev_to_f64(xb[z0:z1, y0:y1, x0:x1].contiguous())
        ref = U.conv3_brute(patch, wb, b.astype(np.float64))[z - z0, yy - y0, x - x0]
        S = U.conv3_brute(np.abs(patch), np.abs(wb), np.abs(b).astype(np.float64))[
            z - z0, yy - y0, x - x0]
        got = dev_to_f64(y[z, yy, x].contiguous())
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 27 * cin * 2.0 ** -24 * S)


def test_nucleus_component_through_a_serpentine():
    """A single one-cell-wide corridor that snakes along x, turns at the row
    ends, climbs from row to row and from layer to layer (hundreds of turns,
    crossing every reachability block many times), plus isolated water
    pockets: the warm start keeps exactly the corridor."""
    n = 40
    mask = np.ones((n, n, n), dtype=np.uint8)
    rows = [(z, y) for z in range(1, n - 1, 2) for y in range(1, n - 1, 2)]
    for k, (z, y) in enumerate(rows):
        mask[z, y, 1:n - 1] = 0
        if k + 1 < len(rows):
            z2, y2 = rows[k + 1]
            x = n - 2 if k % 2 == 0 else 1  # turn at alternating ends
            if z2 == z:
                mask[z, y:y2 + 1, x] = 0
            else:  # climb to the next layer
                mask[z:z2 + 1, y, x] = 0
                mask[z2, 1:y + 1, x] = 0
    # pockets sealed off from the corridor
    for (z, y, x) in ((0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5)):
        mask[z, y, x] = 0
    c = pi.warmstart_instance(20000, edge=48)
    p = dict(c.params, n1=n, n2=n, n3=n)
    phi0 = np.zeros((n, n, n), dtype=np.float32)
    phi0[1, 1, 1:4] = 1.0  # the nucleus: the corridor's first cells
    s = pf.Solver(p, mask, "fp32", c.run)
    s.set_state(phi0)
    net = pf.UNet(seed=2)
    net.warmstart(s, 0.5, 1.0)
    phi, _ = s.get_state()
    keep = U.nucleus_component(mask, phi0)
    assert keep.sum() == (mask == 0).sum() - 3  # the whole corridor, no pocket
    assert np.all(phi[~keep] == 0) and np.all(phi[keep] > 0)
    s.close()
