"""Writes sweep48.json: the FP64 oracle's runs to equilibrium of six 48^3
instances of the micro-scale parametric sweep (seeds 4005, 4009, 4017, 4027, 4035, 4036
of pf_inputs.sweep_instance; Sec. 2.4 model, each with its own supercooling
and surface-tension scale), from the sharp nucleus with the instance's
tolerance and first step, until max over water cells of |d phi/dt| < 1e-6.

Stored per instance: the run's status, accepted and rejected attempts, end
time, water and ice cell counts and the unfrozen water content of the box.
Only the oracle and the seeded input generator are called.

    python tests/golden/make_sweep48.py   (a few minutes on 8 host threads)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pf_inputs as pi  # noqa: E402

SEEDS = (4005, 4009, 4017, 4027, 4035, 4036)
EQ_TOL = 1e-6
BUDGET = 400000


def main(out=os.path.join(HERE, "sweep48.json")):
    recs = []
    for seed in SEEDS:
        c = pi.sweep_instance(seed)
        assert c.shape == (48, 48, 48)
        P = oracle.make_params(c.params)
        t0 = time.perf_counter()
        phi, _, st = oracle.integrate(P, c.mask, oracle.make_ctl(tol=c.run["tol"]), 0.0,
                                      c.run["dt0"], c.phi0, None, max_steps=BUDGET,
                                      eq_tol=EQ_TOL)
        wall = time.perf_counter() - t0
        d = oracle.diagnostics(P, c.mask, phi)
        r = dict(seed=seed, status=st["status"], steps_accepted=st["steps_accepted"],
                 steps_rejected=st["steps_rejected"], t=st["t"], water_cells=d["pore_count"],
                 ice_cells=d["ice_count"], uwc=d["uwc"], wall_s=round(wall, 2),
                 dT=c.params["dT"], alpha=c.params["alpha"], tol=c.run["tol"])
        print(json.dumps(r), flush=True)
        recs.append(r)
    json.dump(dict(eq_tol=EQ_TOL, budget=BUDGET, threads=oracle.num_threads(), runs=recs),
              open(out, "w"), indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
