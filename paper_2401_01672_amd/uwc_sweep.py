"""Unfrozen water content versus supercooling at the paper's micro scales.

The micro-scale experiment of Sec. 3.3: the vessel of Tab. 2 scaled so that
the bead radius r is that of a real powder (L3 = 20 r; the paper uses
polystyrene, r = 5 um, and graphitized carbon black, r = 0.12 um), the
micro-scale model of Sec. 2.4 (Allen-Cahn at constant supercooling dT) with
the realistic attachment coefficient of Tab. 1, ice growing from the
nucleation disk anchored in the glass cap until the state is stationary, and
the unfrozen water content of eq. UWC-formula evaluated over the bottom half
of the vessel (reduced on the GPU, pf_diagnostics_planes).  The geometry is the paper-mode vessel of
``pf_inputs.case_paper`` (smooth glass field, no phase-field face rule) on a
synthetic bead bed.

Every run goes through the library in FP64 (at the 0.12 um scale the
right-hand side's FP32 roundoff alone exceeds the 1e-6 s^-1 equilibrium
threshold): by default the supercooling values of one material run together
as one batch (pf_batch_integrate over pf_create_field handles, one batch per
phase), or one at a time (pf_integrate, --sequential).  Each phase has its
own attempt budget.

Run ``python -m paper_2401_01672_amd.uwc_sweep --help``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List


_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import pf_inputs as pi  # noqa: E402

MATERIALS = {"polystyrene": 5.0e-6, "carbon_black": 0.12e-6}
DT_LIST = [0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0, 25.0]
EQ_TOL = 1e-6


def problem(r_m: float, dT: float, n3: int = 100, seed: int = 5):
    """Paper-mode micro-scale problem.  Two tolerances: tol = 1e-6 while the
    ice front moves, then tol_eq, at which the stiffest mode held at its
    stability limit sits below half the equilibrium threshold (as for the
    sweep instances); first step at the explicit stability limit."""
    c = pi.case_paper(n3, seed=seed, model="ac", L3=20.0 * r_m, alpha=pi.ALPHA_REAL, dT=dT)
    h, a = c.params["h"], c.params["alpha"]
    lam_max = 12.0 / (a * h * h)
    c.run.update(tol=1e-6, tol_eq=min(1e-6, 0.5 * EQ_TOL / lam_max), dt0=1.0 / lam_max,
                 t_end=1e30, lam_max=lam_max)
    return c


def _eq1(c) -> float:
    return max(EQ_TOL, 4.0 * c.run["lam_max"] * c.run["tol"])


def _solver(c):
    import paper_2401_01672_amd as pf
    s = pf.Solver(c.params, None, "fp64", c.run, glass_field=c.G)
    s.set_state(c.phi0)
    s.set_time(0.0, c.run["dt0"])
    return s


def _result(s, st1, st2, wall, c) -> Dict:
    n1 = st1["steps_accepted"] + st1["steps_rejected"]
    st = st2 if st2 is not None else st1
    n2 = st2["steps_accepted"] + st2["steps_rejected"] if st2 is not None else 0
    out = dict(status=st["status"], attempts=n1 + n2, attempts_phase1=n1,
               t=st["t"], wall_s=wall, cells=c.ncells)
    out.update(s.uwc_bottom_half())  # eq. UWC-formula, reduced on the GPU
    return out


def run_one(c, budget: int) -> Dict:
    """Phase 1 at tol = 1e-6 until max water |d phi/dt| falls below the level
    that tolerance can resolve (4 lam_max tol); phase 2 at tol_eq down to the
    1e-6 s^-1 equilibrium threshold; each phase within `budget` attempts."""
    s = _solver(c)
    t0 = time.perf_counter()
    eq1 = _eq1(c)
    st1 = s.integrate(max_steps=budget, eq_tol=eq1, raise_on_error=False)
    st2 = None
    if st1["status"] == 1 and eq1 > EQ_TOL:
        s.set_tolerance(c.run["tol_eq"])
        st2 = s.integrate(max_steps=budget, eq_tol=EQ_TOL, raise_on_error=False)
    out = _result(s, st1, st2, time.perf_counter() - t0, c)
    s.close()
    return out


def run_batch(cases: List, budget: int) -> List[Dict]:
    """The same two phases for problems of one material (the same eq1) as
    batches: phase 1 over every problem, phase 2 over those that reached the
    phase-1 threshold.  wall_s: the whole batch's time."""
    import paper_2401_01672_amd as pf
    eq1 = _eq1(cases[0])
    assert all(_eq1(c) == eq1 for c in cases), "one material per batch"
    ss = [_solver(c) for c in cases]
    t0 = time.perf_counter()
    st1 = pf.batch_integrate(ss, max_steps=budget, eq_tol=eq1, raise_on_error=False)
    st2 = [None] * len(cases)
    if eq1 > EQ_TOL:
        again = [i for i, st in enumerate(st1) if st["status"] == 1]
        for i in again:
            ss[i].set_tolerance(cases[i].run["tol_eq"])
        if again:
            res2 = pf.batch_integrate([ss[i] for i in again], max_steps=budget, eq_tol=EQ_TOL,
                                      raise_on_error=False)
            for i, st in zip(again, res2):
                st2[i] = st
    wall = time.perf_counter() - t0
    out = [_result(s, a, b, wall, c) for s, a, b, c in zip(ss, st1, st2, cases)]
    for s in ss:
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n3", type=int, default=100)
    ap.add_argument("--materials", default="polystyrene,carbon_black")
    ap.add_argument("--dT", default=",".join(str(v) for v in DT_LIST))
    ap.add_argument("--budget", type=int, default=300000, help="attempts per phase")
    ap.add_argument("--sequential", action="store_true",
                    help="one problem at a time instead of one batch per material")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    res: List[Dict] = []
    wall = 0.0
    for mat in a.materials.split(","):
        dts = [float(v) for v in a.dT.split(",")]
        cases = [problem(MATERIALS[mat], dT, a.n3) for dT in dts]
        if a.sequential:
            rs = [run_one(c, a.budget) for c in cases]
            wall += sum(r["wall_s"] for r in rs)
        else:
            rs = run_batch(cases, a.budget)
            wall += rs[0]["wall_s"]
        for dT, c, r in zip(dts, cases, rs):
            r = dict(material=mat, r_m=MATERIALS[mat], dT=dT, h=c.params["h"], **r)
            res.append(r)
            print(json.dumps(r), flush=True)
    cells = sum(r["cells"] * r["attempts"] for r in res)
    summary = dict(runs=len(res), equilibrium=sum(r["status"] == 1 for r in res),
                   gcups=cells / wall / 1e9, wall_s=wall)
    print(json.dumps(summary), flush=True)
    if a.out:
        json.dump(dict(summary=summary, results=res, args=vars(a)), open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
