"""What the trained warm-start network gains over the method without it.

Held-out problems of the sweep generator at 96^3 (seeds outside the
training range), each run to max |d phi/dt| < 1e-6 twice on the GPU: from
the sharp nucleus (cold) and from the network's prediction restricted to the
nucleus's water component (warm).  The equilibrium is judged by the plain
method in both runs; the bar is the same unfrozen water content within
1e-3 relative, reached in at least 3x less wall time on the freezing
problems (inference included).
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


def test_trained_network_warm_start(net):
    # 20000, 20002-20004 freeze (UWC ~ 1e-5); 20001 melts back (UWC = 1)
    probs = W.generate([20000, 20001, 20002, 20003, 20004], 96, workers=1)
    res = W.evaluate(net, probs, budget=100000, log=lambda m: None)
    for r in res:
        assert r["cold_status"] == 1 and r["warm_status"] == 1, r
        assert r["uwc_relerr"] <= 1e-3, r
    freezing = [r for r in res if r["uwc_cold"] < 0.5]
    assert len(freezing) == 4
    assert np.median([r["speedup"] for r in freezing]) >= 3.0, [r["speedup"] for r in res]
