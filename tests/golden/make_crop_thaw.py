"""Writes crop_thaw_64.npz: the FP64 oracle's runs of the 64^3 crop of the
256^3 freeze-thaw case (bottom face ramped linearly from -5 C to +5 C over
60 s, so it crosses 0 C at t = 30 s; Sec. 2.2 eq. BC-temperature-cap with the
ramp schedule), stopped at t = 30, 45 and 60 s (adaptive Merson steps, each
segment clipped to land on its end time).

Two oracle runs:
  * tol = 1e-6 (the case's tolerance), one attempt at a time, recording the
    step of every accepted attempt, so that another implementation can
    replay exactly this step sequence;
  * tol = 1e-7, to measure how far the method itself moves when only the
    tolerance changes (the time-integration error at tol = 1e-6).

Stored per end time, for the tol = 1e-6 run: phi in fixed point
(round(phi * 2^24) as int32, so the bulk cells at 0 and 1 compress), theta =
T - T* at 4096 seeded sample cells, the ice fraction (water cells with
phi > 1/2 among the water cells) and the attempt counts; the accepted steps
of each segment; for the tol = 1e-7 run: the ice fraction, the attempt
counts, max |phi(1e-7) - phi(1e-6)| and max |theta(1e-7) - theta(1e-6)| at
the sample cells.  Only the oracle and the seeded input generator are
called.

    python tests/golden/make_crop_thaw.py   (about 50 min on 8 host threads)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pf_inputs as pi  # noqa: E402

TIMES = (30.0, 45.0, 60.0)
NSAMPLE = 4096
QSCALE = float(1 << 24)
TOL_FINE = 1e-7


def main(out=os.path.join(HERE, "crop_thaw_64.npz")):
    full = pi.case_coupled_256()
    c = pi.crop_case(full)
    run = dict(full.run)
    P = oracle.make_params(c.params)
    tstar = c.params["t_star"]
    rng = np.random.default_rng(64)
    sample = np.sort(rng.choice(c.ncells, size=NSAMPLE, replace=False))
    rec = dict(times=np.array(TIMES), sample=sample.astype(np.int64), qscale=np.array(QSCALE),
               tol=np.array(run["tol"]), tol_fine=np.array(TOL_FINE),
               threads=np.array(oracle.num_threads()))

    # tol = 1e-6, attempt by attempt
    ctl = oracle.make_ctl(tol=run["tol"])
    phi, T = c.phi0, c.T0
    t, dt = 0.0, run["dt0"]
    phis, fields, thetas, ice, acc, rej, steps, seg = [], [], [], [], [], [], [], []
    t0 = time.perf_counter()
    for te in TIMES:
        na = nr = 0
        while t < te:
            phi, T, t, dt, info = oracle.rkm_step(P, c.mask, ctl, t, dt, phi, T, t_end=te)
            assert info["status"] >= 0, info
            if info["accepted"]:
                na += 1
                steps.append(info["dt_used"])
            else:
                nr += 1
        assert t == te, (t, te)
        d = oracle.diagnostics(P, c.mask, phi, T)
        phis.append(np.rint(phi * QSCALE).astype(np.int32))
        fields.append((phi.copy(), (T - tstar).ravel()[sample].copy()))
        thetas.append((T.ravel()[sample] - tstar).astype(np.float64))
        ice.append(d["ice_fraction"])
        acc.append(na)
        rej.append(nr)
        seg.append(len(steps))
        print(f"tol 1e-6, t = {te:g} s: ice fraction {d['ice_fraction']:.6f}, {na} accepted, "
              f"{nr} rejected, {time.perf_counter() - t0:.0f} s", flush=True)
    rec.update(phi_q=np.stack(phis), theta_sample=np.stack(thetas), ice_fraction=np.array(ice),
               steps_accepted=np.array(acc), steps_rejected=np.array(rej),
               accepted_dt=np.array(steps), segment_end=np.array(seg))

    # tol = 1e-7, the same segments
    ctl = oracle.make_ctl(tol=TOL_FINE)
    phi, T = c.phi0, c.T0
    t, dt = 0.0, run["dt0"]
    ice7, acc7, rej7, dphi7, dth7 = [], [], [], [], []
    for k, te in enumerate(TIMES):
        phi, T, st = oracle.integrate(P, c.mask, ctl, t, dt, phi, T, t_end=te)
        assert st["status"] == oracle.OK and st["t"] == te, st
        t, dt = st["t"], st["dt"]
        d = oracle.diagnostics(P, c.mask, phi, T)
        ice7.append(d["ice_fraction"])
        acc7.append(st["steps_accepted"])
        rej7.append(st["steps_rejected"])
        dphi7.append(float(np.abs(phi - fields[k][0]).max()))
        dth7.append(float(np.abs((T - tstar).ravel()[sample] - fields[k][1]).max()))
        print(f"tol 1e-7, t = {te:g} s: ice fraction {d['ice_fraction']:.6f}, "
              f"{st['steps_accepted']} accepted, {st['steps_rejected']} rejected, "
              f"max|phi - phi(1e-6)| = {dphi7[-1]:.3e}, {time.perf_counter() - t0:.0f} s",
              flush=True)
    rec.update(ice_fraction_fine=np.array(ice7), steps_accepted_fine=np.array(acc7),
               steps_rejected_fine=np.array(rej7), max_dphi_fine=np.array(dphi7),
               max_dtheta_fine=np.array(dth7))
    np.savez_compressed(out, **rec)
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    main()
