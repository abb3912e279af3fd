"""The 64^3 crop of the 256^3 freeze-thaw case through the whole ramp: FP32
fields on the GPU against the FP64 oracle at t = 30 s (the bottom face
crosses 0 C), 45 s and 60 s (thawing; Sec. 2.2 eq. BC-temperature-cap with
the ramp -5 -> +5 C over 60 s).  The oracle's runs are stored in
tests/golden/crop_thaw_64.npz, written by tests/golden/make_crop_thaw.py.

The FP64 trajectory is robust: at tol 1e-6 the steps sit at the explicit
stability limit, and the oracle rerun at tol 1e-7 changes phi by 9e-9.
Two FP32 comparisons:
  * along the oracle's own steps: the GPU replays the accepted step sizes of
    the oracle's adaptive run one attempt at a time, so the two differ only
    by the FP32 storage of the fields;
  * the GPU's own adaptive FP32 run at the case's tol 1e-6.
Over 10^4 steps near moving fronts the FP32 storage alone moves phi by about
2e-3 (a front shift of about 0.01 cell): the 1e-4 bound on phi holds over
short horizons (tests/test_gpu_parity.py, 0.6 s) but not here, and these
tests assert the measured level with margin (1e-2 along the oracle's steps,
5e-2 adaptive) and print it.  The ice fraction stays within 1e-3 relative,
and theta within the latent-heat carry-over of the phi gap,
(Lv / min rho c) max(|d phi|, 1e-4).  At
tol 1e-6 the adaptive FP32 run also takes several times the oracle's
attempts: the FP32 rounding of the stage values, amplified by the latent
heat term, sits in the error estimate at about the tolerance."""
import os

import numpy as np
import pytest

import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crop_thaw_64.npz")


def _case():
    full = pi.case_coupled_256()
    return pi.crop_case(full), dict(full.run)


def _compare(g, k, s, st_ice):
    phi, th = s.get_state()
    ref = g["phi_q"][k].astype(np.float64) / float(g["qscale"])
    dphi = float(np.abs(phi.astype(np.float64) - ref).max())
    ice_ref = float(g["ice_fraction"][k])
    dice = abs(st_ice - ice_ref) / ice_ref
    dth = float(np.abs(th.ravel()[g["sample"]].astype(np.float64) - g["theta_sample"][k]).max())
    return dphi, dice, dth


def test_crop_freeze_thaw_fp32_along_oracle_steps():
    g = np.load(GOLD)
    c, run = _case()
    s = pf.Solver(c.params, c.mask, "fp32", dict(run, tol=0.0))
    s.set_state(c.phi0.astype(np.float32), (c.T0 - pi.T_STAR).astype(np.float32))
    lat = c.params["Lv"] / min(c.params["rhoc"])
    steps = g["accepted_dt"]
    ends = g["segment_end"]
    t, j = 0.0, 0
    for k, te in enumerate(g["times"]):
        while j < ends[k]:
            t, _, info = s.rkm_step(t, float(steps[j]))
            assert info["accepted"] == 1
            j += 1
        assert abs(t - te) <= 1e-9 * te, (t, te)
        st = s.diagnostics()
        dphi, dice, dth = _compare(g, k, s, st["ice_fraction"])
        print(f"crop 64^3 FP32 along the oracle's {ends[k]} steps, t = {te:g} s: "
              f"max|dphi| = {dphi:.2e}, ice fraction rel. error {dice:.2e}, "
              f"max|dtheta| at samples {dth:.2e} K")
        assert dphi <= 1e-2, (te, dphi)
        assert dice <= 1e-3, (te, dice)
        assert dth <= lat * max(dphi, 1e-4), (te, dth)
    s.close()


def test_crop_freeze_thaw_fp32_adaptive():
    g = np.load(GOLD)
    c, run = _case()
    s = pf.Solver(c.params, c.mask, "fp32", run)
    s.set_state(c.phi0.astype(np.float32), (c.T0 - pi.T_STAR).astype(np.float32))
    s.set_time(0.0, run["dt0"])
    lat = c.params["Lv"] / min(c.params["rhoc"])
    for k, te in enumerate(g["times"]):
        st = s.integrate(t_end=float(te))
        assert st["status"] == pf.PF_OK and st["t"] == te, st
        dphi, dice, dth = _compare(g, k, s, st["ice_fraction"])
        own = float(g["max_dphi_fine"][k])
        print(f"crop 64^3 FP32 adaptive, t = {te:g} s: max|dphi| = {dphi:.2e} (oracle tol 1e-6 "
              f"vs 1e-7: {own:.2e}), ice fraction rel. error {dice:.2e}, max|dtheta| at "
              f"samples {dth:.2e} K (oracle: {float(g['max_dtheta_fine'][k]):.2e} K), "
              f"attempts {st['steps_accepted'] + st['steps_rejected']} vs "
              f"{int(g['steps_accepted'][k] + g['steps_rejected'][k])}")
        assert dice <= 1e-3, (te, dice)
        assert dphi <= 5e-2, (te, dphi, own)
        assert dth <= lat * max(dphi, 1e-4), (te, dth)
    s.close()
