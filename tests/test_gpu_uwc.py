"""Micro-scale UWC experiment (paper-mode vessel at the carbon-black scale):
the GPU run to a stationary state against the FP64 oracle run to the same
criterion, compared on the unfrozen water content of the bottom half (Sec.
3.3, eq. UWC-formula): the GPU's plane-range reduction against the oracle's
own bottom-half count."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2401_01672_amd import uwc_sweep as U  # noqa: E402


@pytest.mark.parametrize("dT", [2.0, 0.2])
def test_uwc_run_matches_oracle(dT):
    c = U.problem(0.12e-6, dT, n3=40)
    gpu = U.run_one(c, budget=200000)
    # the oracle runs the same two phases
    P = oracle.make_params(c.params)
    eq1 = max(U.EQ_TOL, 4.0 * c.run["lam_max"] * c.run["tol"])
    phi_o, _, st1 = oracle.integrate(P, c.G, oracle.make_ctl(tol=c.run["tol"]), 0.0,
                                     c.run["dt0"], c.phi0, None, max_steps=200000, eq_tol=eq1)
    phi_o, _, st = oracle.integrate(P, c.G, oracle.make_ctl(tol=c.run["tol_eq"]), st1["t"],
                                    st1["dt"], phi_o, None, max_steps=200000, eq_tol=U.EQ_TOL)
    ref = oracle.uwc_bottom_half(P, c.G, phi_o)
    # the ice set of eq. frozen-subdomain is every cell with phi > 1/2; the
    # counts take it among the water cells, the same set here because no
    # glass cell of the bottom half holds phi > 1/2
    half = c.G.shape[0] // 2
    assert not np.any((c.G[:half] >= 0.5) & (phi_o[:half] > 0.5))
    assert st["status"] == oracle.EQUILIBRIUM and gpu["status"] == 1
    assert gpu["water_cells"] == ref["water_cells"]
    assert gpu["ice_cells"] == ref["ice_cells"]
    # the step sequences agree up to the error estimate's roundoff
    n_o = st1["steps_accepted"] + st1["steps_rejected"] + st["steps_accepted"] + \
        st["steps_rejected"]
    assert abs(gpu["attempts"] - n_o) <= max(2, n_o // 1000)


def test_uwc_batch_equals_single_runs():
    """The sweep's batched form (the supercooling values of one material in one
    batch per phase, paper-mode glass fields) gives each problem exactly the
    run it gets alone: the same status, attempts, end time and bottom-half
    counts."""
    cases = [U.problem(0.12e-6, dT, n3=40) for dT in (5.0, 2.0, 0.2)]
    batch = U.run_batch(cases, budget=200000)
    for c, rb in zip(cases, batch):
        rs = U.run_one(c, budget=200000)
        for k in ("status", "attempts", "attempts_phase1", "t", "water_cells", "ice_cells"):
            assert rb[k] == rs[k], (k, rb[k], rs[k])
