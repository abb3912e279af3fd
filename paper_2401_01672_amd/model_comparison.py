"""SigmaP1-P against GradP on the paper-mode vessel (Sec. 3.2, model comparison).

The paper reports that the GradP reaction term (eq. reaction-term-GradP) is
unstable for the larger attachment coefficients (smaller surface tension) and
produces phi > 1, while the SigmaP1-P term (eq. reaction-term-SigmaP1-P)
behaves in every setting.  This module runs the coupled model in paper mode
(``pf_inputs.case_paper``: smooth bead-bed glass field, cap, nucleation disk,
cooled cap face, Tab. 1 materials) with both reaction terms at the three
attachment coefficients of Tab. 2 ("large", "small" and "tiny" sigma), FP64
with adaptive Merson steps, and reports per run the range of phi over the
water cells, the ice fraction, and how the run ended (a step size collapsing
below dt_min is the instability).

The Temp model (Sec. 2.3: phi follows T through eq.
explicit-p-dependence-on-T) has no phase-field equation and no attachment
coefficient; the paper finds its ice volume insensitive to the transition
rate gamma (2 against 10) and to the mesh resolution.  ``run_temp`` runs it on
the same vessel and reports the ice fraction of the water volume and of the
whole box and the final temperature field, so that runs at two values of gamma
or two resolutions can be compared.  ``--sigma-n3`` runs the same resolution
study for SigmaP1-P (the paper's convergence check, Sec. 3.2).

Run ``python -m paper_2401_01672_amd.model_comparison --help``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import pf_inputs as pi  # noqa: E402

# Tab. 2: attachment coefficients of the "large", "small" and "tiny" surface tension
ALPHAS = {"large_sigma": 4.17e6, "small_sigma": 1.25e7, "tiny_sigma": 3.7e8}
DT_MIN = 1e-9


def run_one(c, reaction: str, t_end: float, budget: int) -> Dict:
    """One paper-mode run to t_end (or until the step size collapses)."""
    import paper_2401_01672_amd as pf
    p = dict(c.params, reaction=reaction)
    s = pf.Solver(p, None, "fp64", dict(c.run, dt_min=DT_MIN), glass_field=c.G)
    s.set_state(c.phi0, c.T0 - pi.T_STAR)
    s.set_time(0.0, 1e-3)
    t0 = time.perf_counter()
    st = s.integrate(t_end=t_end, max_steps=budget, raise_on_error=False)
    wall = time.perf_counter() - t0
    phi, _ = s.get_state()
    s.close()
    water = c.G < 0.5
    nwater = int(np.count_nonzero(water))
    return dict(reaction=reaction, status=int(st["status"]), t=float(st["t"]),
                attempts=int(st["steps_accepted"] + st["steps_rejected"]),
                phi_max=float(np.max(phi[water])), phi_min=float(np.min(phi[water])),
                ice_fraction=float(st["ice_fraction"]),
                ice_fraction_box=float(st["ice_fraction"]) * nwater / c.G.size, wall_s=wall)


def run_temp(n3: int, gamma: float, t_end: float, budget: int, seed: int = 5) -> Dict:
    """Temp model on the paper-mode vessel of height n3 cells to t_end."""
    import paper_2401_01672_amd as pf
    c = pi.case_paper(n3, seed=seed, model="temp")
    p = dict(c.params, gamma=gamma)
    s = pf.Solver(p, None, "fp64", dict(c.run, dt_min=DT_MIN), glass_field=c.G)
    s.set_state(None, c.T0 - pi.T_STAR)
    s.set_time(0.0, 1e-3)
    t0 = time.perf_counter()
    st = s.integrate(t_end=t_end, max_steps=budget, raise_on_error=False)
    wall = time.perf_counter() - t0
    _, theta = s.get_state()
    s.close()
    water = int(np.count_nonzero(c.G < 0.5))
    ice = float(st["ice_fraction"]) * water
    return dict(model="temp", n3=n3, gamma=gamma, status=int(st["status"]), t=float(st["t"]),
                attempts=int(st["steps_accepted"] + st["steps_rejected"]),
                ice_fraction=float(st["ice_fraction"]), ice_fraction_box=ice / c.G.size,
                theta_min=float(theta.min()), theta_max=float(theta.max()), wall_s=wall,
                theta=theta)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n3", type=int, default=100)
    ap.add_argument("--t-end", type=float, default=120.0, help="simulated time [s]")
    ap.add_argument("--budget", type=int, default=400000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default="")
    ap.add_argument("--temp-n3", default="",
                    help="comma-separated vessel heights for the Temp-model runs "
                         "(gamma 2 and 10 each); empty: the --n3 vessel")
    ap.add_argument("--sigma-n3", default="",
                    help="comma-separated vessel heights for a resolution study of "
                         "SigmaP1-P at the 'large sigma' coefficient (ice over the box)")
    a = ap.parse_args()
    cases = {k: pi.case_paper(a.n3, seed=a.seed, alpha=v) for k, v in ALPHAS.items()}
    import torch
    torch.cuda.set_device(0)
    res: List[Dict] = []
    for name, c in cases.items():
        for reaction in ("sigma", "gradp"):
            r = dict(setting=name, alpha=ALPHAS[name], **run_one(c, reaction, a.t_end, a.budget))
            res.append(r)
            print(json.dumps(r), flush=True)
    for n3 in [int(v) for v in a.sigma_n3.split(",") if v]:
        c = pi.case_paper(n3, seed=a.seed, alpha=ALPHAS["large_sigma"])
        r = dict(setting="large_sigma", n3=n3, **run_one(c, "sigma", a.t_end, a.budget))
        res.append(r)
        print(json.dumps(r), flush=True)
    temp_n3 = [int(v) for v in a.temp_n3.split(",") if v] or [a.n3]
    for n3 in temp_n3:
        th = {}
        for gamma in (2.0, 10.0):
            r = run_temp(n3, gamma, a.t_end, a.budget, a.seed)
            th[gamma] = r.pop("theta")
            res.append(r)
            print(json.dumps(r), flush=True)
        d = dict(model="temp", n3=n3, compare="gamma 2 vs 10",
                 max_abs_dtheta=float(np.max(np.abs(th[2.0] - th[10.0]))))
        res.append(d)
        print(json.dumps(d), flush=True)
    if a.out:
        json.dump(dict(results=res, args=vars(a)), open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
