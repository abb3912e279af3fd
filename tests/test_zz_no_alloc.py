"""Allocation-free convolution entry point (pf_conv3_bf16_noalloc) against
the allocating one (pf_conv3_bf16): both run the same kernels on the same
BF16-rounded operands, so the outputs must agree bit for bit.  Two calls in a
row, the second on a smaller grid with fewer channels, show that the static
weight scratch keeps nothing of the previous call that matters; the outputs
are also held to the per-element bound against the FP64 reference (the bound
of the convolution tests: 2^-8 |y| + 27 cin 2^-24 sum|x||w|)."""
import numpy as np
import pytest

from oracle import unet as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402

DEV = "cuda:0"


def _case(rng, shape, cin, cout):
    x = U.round_bf16(rng.normal(size=shape + (cin,)))
    w = rng.normal(0, np.sqrt(2.0 / (27 * cin)), size=(cout, 27, cin)).astype(np.float32)
    b = rng.normal(0, 0.1, size=cout).astype(np.float32)
    return x, w, b


def _run_both(x, w, b, relu):
    cout = w.shape[0]
    xd = torch.from_numpy(np.ascontiguousarray(U.to_bf16_bits(x))).to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    bd = torch.from_numpy(b).to(DEV)
    ref = pf.conv3_bf16(xd, wd, bd, relu, cout)
    y = torch.full(tuple(x.shape[:3]) + (cout,), -1, dtype=torch.int16, device=DEV)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    pf.conv3_bf16_noalloc(xd, wd, bd, relu, y, stream=stream)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), y.cpu().numpy()


def _check_bound(x, w, b, relu, y_bits):
    wb = U.round_bf16(w)
    ex = U.conv3_cl(x, wb, b.astype(np.float64))
    if relu:
        ex = np.maximum(ex, 0.0)
    S = U.conv3_cl(np.abs(x), np.abs(wb), np.abs(b.astype(np.float64)))
    bound = 2.0 ** -8 * np.abs(ex) + 27 * w.shape[2] * 2.0 ** -24 * S + 1e-30
    got = U.from_bf16_bits(y_bits)
    assert np.all(np.abs(got - ex) <= bound), float(np.max(np.abs(got - ex) - bound))


def test_noalloc_matches_allocating_entry_point_twice():
    rng = np.random.default_rng(11)
    # first call: the largest channel counts the static scratch holds
    x1, w1, b1 = _case(rng, (12, 10, 20), 96, 96)
    ref1, got1 = _run_both(x1, w1, b1, True)
    assert np.array_equal(ref1, got1)
    _check_bound(x1, w1, b1, True, got1)
    # second call, right after: smaller grid, fewer channels, no ReLU
    x2, w2, b2 = _case(rng, (7, 5, 9), 16, 32)
    ref2, got2 = _run_both(x2, w2, b2, False)
    assert np.array_equal(ref2, got2)
    _check_bound(x2, w2, b2, False, got2)


def test_noalloc_rejects_channels_beyond_the_scratch():
    # rejected on the host before any device work
    rc = pf.lib().pf_conv3_bf16_noalloc(1, 104, 1, 0, 0, 1, 16, 4, 4, 4, 0)
    assert rc == pf.PF_EINVAL
    assert b"static weight scratch" in pf.lib().pf_last_error(None)
