"""What the trained warm-start network gains over the method without it, and
over a warm start without the network.

Held-out problems of the sweep generator (seeds outside the training range),
each run to max |d phi/dt| < 1e-6 on the GPU three times: from the sharp
nucleus (cold), from the network's prediction restricted to the nucleus's
water component (warm), and from the baseline without the network, phi = 1 on
that component (flood).  The equilibrium is judged by the plain method in
every run; the bar is the cold run's unfrozen water content within 1e-3
relative, reached in at least 3x less wall time on the freezing problems
(inference included).

The flood baseline is an exact equilibrium of the discrete system (phi = 1 is
a fixed point of the reaction term and has no Laplacian), so it costs no
attempts; it is right where the whole component freezes and wrong where the
nucleus melts back (UWC = 1).  The network tells the two apart.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402
from paper_2401_01672_amd import warmstart as W  # noqa: E402

PARAMS = os.path.join(os.path.dirname(pf.__file__), "data", "unet_warmstart_96.npz")


@pytest.fixture(scope="module")
def net():
    n = pf.UNet(seed=0)
    n.set_params(np.load(PARAMS)["params"])
    yield n
    n.close()


def _check(res, n_freeze, n_melt):
    for r in res:
        print(f"seed {r['seed']} at {r['edge']}^3: UWC cold {r['uwc_cold']:.5f}, warm "
              f"{r['uwc_warm']:.5f}, flood {r['uwc_flood']:.5f}; wall cold {r['cold_s']:.3f} s, "
              f"warm {r['warm_s']:.4f} s ({r['speedup']:.1f}x), flood {r['flood_s']:.4f} s "
              f"({r['flood_speedup']:.1f}x)")
        assert r["cold_status"] == 1 and r["warm_status"] == 1, r
        assert r["uwc_relerr"] <= 1e-3, r
    freezing = [r for r in res if r["uwc_cold"] < 0.5]
    melting = [r for r in res if r["uwc_cold"] == 1.0]
    assert len(freezing) == n_freeze and len(melting) == n_melt
    assert np.median([r["speedup"] for r in freezing]) >= 3.0, [r["speedup"] for r in res]
    # where the nucleus melts back, the baseline without the network settles
    # in the wrong equilibrium (all ice); the network's start does not
    for r in melting:
        assert r["flood_status"] == 1 and not r["flood_pass"] and r["pass"], r


def test_trained_network_warm_start(net):
    # 20000, 20002-20004 freeze (UWC ~ 1e-5); 20001 and 20009 melt back (UWC = 1)
    probs = W.generate([20000, 20001, 20002, 20003, 20004, 20009], 96, workers=1)
    res = W.evaluate(net, probs, budget=100000, log=lambda m: None)
    _check(res, 4, 2)


def test_trained_network_warm_start_192(net):
    """The fully convolutional network on grids twice the training size."""
    probs = W.generate([20000, 20003, 20009], 192, workers=3)
    res = W.evaluate(net, probs, budget=200000, log=lambda m: None)
    _check(res, 2, 1)
