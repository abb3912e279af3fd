"""Learned warm start of micro-scale sweeps to equilibrium.

The network (pf_unet in the C ABI) predicts the equilibrium phase field of a
micro-scale problem (Sec. 2.4: Allen-Cahn at constant supercooling dT) from
its glass mask, dT and surface-tension scale s.  This module drives the whole
experiment through the library:

* ``make_dataset``: equilibria of generated problems, solved to
  max |d phi/dt| < 1e-6 by the batched solver from the usual sharp nucleus
  (cold start); the final phase fields are the training targets;
* ``train``: Adam on the masked squared error, one problem per step;
* ``evaluate``: per problem, wall time to equilibrium from the cold start and
  from the network's prediction (inference included), and the unfrozen water
  content (UWC) reached by each.

Run ``python -m paper_2401_01672_amd.warmstart --help`` for the command line.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time
from typing import Dict, List

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import pf_inputs as pi  # noqa: E402

EQ_TOL = 1e-6


def _gen(args):
    seed, edge = args
    c = pi.warmstart_instance(seed, edge=edge)
    return dict(seed=seed, mask=c.mask, phi0=c.phi0.astype(np.uint8), params=c.params,
                run=c.run, meta=c.meta)


def generate(seeds: List[int], edge: int, workers: int = 16) -> List[Dict]:
    """Problems of the sweep generator at a fixed edge (CPU, in parallel).
    Call before the GPU is initialised in this process."""
    jobs = [(int(s), int(edge)) for s in seeds]
    if workers <= 1 or len(jobs) < 4:
        return [_gen(j) for j in jobs]
    with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
        return pool.map(_gen, jobs, chunksize=1)


def log10_scale(prob: Dict) -> float:
    return math.log10(prob["meta"]["sigma_scale"])


def _solver(prob: Dict):
    """A solver whose tile depths are the library autotuner's for this grid
    shape; timed runs call _tune first, so that the measurement happens once
    per shape outside them and each handle only looks the choice up."""
    import paper_2401_01672_amd as pf
    return pf.Solver(prob["params"], prob["mask"], "fp32", prob["run"])


def _tune(probs: List[Dict]):
    """Run the autotuner once per grid shape (its choice is kept for the
    process and reused by every later handle of that shape)."""
    seen = set()
    for p in probs:
        key = tuple(p["mask"].shape)
        if key in seen:
            continue
        seen.add(key)
        s = _solver(p)
        s.set_state(p["phi0"].astype(np.float32))
        s.set_time(0.0, p["run"]["dt0"])
        s.integrate(max_steps=1, raise_on_error=False)
        s.close()


def make_dataset(probs: List[Dict], budget: int, batch: int = 64, log=print) -> List[Dict]:
    """Cold-start equilibria by the batched solver; returns one record per
    problem with device tensors mask (uint8) and target (FP32 phi)."""
    import torch
    import paper_2401_01672_amd as pf
    out = []
    for b0 in range(0, len(probs), batch):
        chunk = probs[b0:b0 + batch]
        ss = []
        for p in chunk:
            s = _solver(p)
            s.set_state(p["phi0"].astype(np.float32))
            s.set_time(0.0, p["run"]["dt0"])
            ss.append(s)
        t0 = time.perf_counter()
        st = pf.batch_integrate(ss, max_steps=budget, eq_tol=EQ_TOL, raise_on_error=False)
        wall = time.perf_counter() - t0
        for p, s, x in zip(chunk, ss, st):
            phi, _ = s.get_state(device=True)
            out.append(dict(seed=p["seed"], mask=torch.from_numpy(p["mask"]).cuda(),
                            target=phi.float().contiguous(), dT=p["meta"]["dT"],
                            log10_s=log10_scale(p), status=x["status"], uwc=x["uwc"],
                            attempts=x["steps_accepted"] + x["steps_rejected"]))
            s.close()
        log(f"dataset {b0 + len(chunk)}/{len(probs)}: batch wall {wall:.1f} s, "
            f"equilibrium {sum(x['status'] == 1 for x in st)}/{len(st)}")
    return out


def train(net, data: List[Dict], epochs: int, lr0: float = 2e-4, lr1: float = 2e-5,
          seed: int = 0, warmup: int = 100, log=print) -> List[float]:
    """Adam over the samples in a seeded random order; the learning rate rises
    linearly to lr0 over the first ``warmup`` steps, then decays to lr1 on a
    cosine.  (Adam's first steps move every weight by about lr in the
    direction of its gradient; on targets that are all ice or all water those
    directions agree across whole layers, so a large initial rate drives the
    sigmoid into saturation.)  Returns the mean loss of each epoch."""
    rng = np.random.default_rng(seed)
    usable = [d for d in data if d["status"] == 1]
    n = len(usable)
    total = epochs * n
    k = 0
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        losses = []
        t0 = time.perf_counter()
        for i in order:
            d = usable[i]
            if k < warmup:
                lr = lr0 * (k + 1) / warmup
            else:
                q = (k - warmup) / max(total - warmup - 1, 1)
                lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * q))
            n3, n2, n1 = d["mask"].shape
            loss = net.train_step(d["mask"], d["target"], d["dT"], d["log10_s"], lr,
                                  want_loss=True)
            losses.append(loss)
            k += 1
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.5f} "
            f"({time.perf_counter() - t0:.1f} s, {n} samples)")
    return hist


def _relerr(u, ref):
    return abs(u - ref) / ref if ref > 0 else (0.0 if u == ref else float("inf"))


def evaluate(net, probs: List[Dict], budget: int, log=print, flood: bool = True) -> List[Dict]:
    """Wall time to equilibrium, one problem at a time: cold (the sharp
    nucleus), warm (the network's prediction on the nucleus's water
    component) and, with flood, the baseline without the network (phi = 1 on
    that component)."""
    import torch
    _tune(probs)
    res = []
    for p in probs:
        cold = _solver(p)
        cold.set_state(p["phi0"].astype(np.float32))
        cold.set_time(0.0, p["run"]["dt0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sc = cold.integrate(max_steps=budget, eq_tol=EQ_TOL, raise_on_error=False)
        wc = time.perf_counter() - t0
        cold.close()
        warm = _solver(p)
        warm.set_state(p["phi0"].astype(np.float32))  # the nucleus: where ice may form
        warm.set_time(0.0, p["run"]["dt0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.warmstart(warm, p["meta"]["dT"], log10_scale(p))
        ti = time.perf_counter() - t0
        sw = warm.integrate(max_steps=budget, eq_tol=EQ_TOL, raise_on_error=False)
        ww = time.perf_counter() - t0
        warm.close()
        uc, uw = sc["uwc"], sw["uwc"]
        relerr = _relerr(uw, uc)
        fl = {}
        if flood:
            fs = _solver(p)
            fs.set_state(p["phi0"].astype(np.float32))
            fs.set_time(0.0, p["run"]["dt0"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net.warmstart(fs, p["meta"]["dT"], log10_scale(p), mode="flood")
            sf = fs.integrate(max_steps=budget, eq_tol=EQ_TOL, raise_on_error=False)
            wf = time.perf_counter() - t0
            fs.close()
            fl = dict(flood_status=sf["status"],
                      flood_attempts=sf["steps_accepted"] + sf["steps_rejected"],
                      flood_s=wf, uwc_flood=sf["uwc"], uwc_flood_relerr=_relerr(sf["uwc"], uc),
                      flood_speedup=wc / wf if wf > 0 else float("nan"))
            fl["flood_pass"] = bool(sc["status"] == 1 and sf["status"] == 1 and
                                    fl["uwc_flood_relerr"] <= 1e-3)
        r = dict(seed=p["seed"], edge=int(p["params"]["n1"]), dT=p["meta"]["dT"],
                 sigma_scale=p["meta"]["sigma_scale"],
                 cold_status=sc["status"], warm_status=sw["status"],
                 cold_attempts=sc["steps_accepted"] + sc["steps_rejected"],
                 warm_attempts=sw["steps_accepted"] + sw["steps_rejected"],
                 cold_s=wc, warm_s=ww, inference_s=ti, uwc_cold=uc, uwc_warm=uw,
                 uwc_relerr=relerr,
                 ice_cold=sc["ice_count"], ice_warm=sw["ice_count"],
                 speedup=wc / ww if ww > 0 else float("nan"))
        r["pass"] = bool(sc["status"] == 1 and sw["status"] == 1 and relerr <= 1e-3)
        r["pass_abs"] = bool(sc["status"] == 1 and sw["status"] == 1 and abs(uw - uc) <= 1e-3)
        r.update(fl)
        res.append(r)
        log(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}))
    return res


def summarize(res: List[Dict]) -> Dict:
    ok = [r for r in res if r["cold_status"] == 1]
    if not ok:
        return dict(problems=len(res), cold_equilibrium=0)
    sp = np.array([r["speedup"] for r in ok])
    passed = [r for r in ok if r["pass"]]
    # a problem whose warm result fails the UWC check keeps its cold result,
    # at the cost of both runs
    eff = np.array([r["cold_s"] / (r["warm_s"] if r["pass"] else r["warm_s"] + r["cold_s"])
                    for r in ok])
    return dict(problems=len(res), cold_equilibrium=len(ok), pass_rate=len(passed) / len(ok),
                pass_rate_abs=sum(r["pass_abs"] for r in ok) / len(ok),
                median_speedup=float(np.median(sp)),
                median_speedup_passing=float(np.median([r["speedup"] for r in passed]))
                if passed else None,
                median_effective_speedup=float(np.median(eff)),
                median_cold_s=float(np.median([r["cold_s"] for r in ok])),
                median_warm_s=float(np.median([r["warm_s"] for r in ok])),
                median_uwc_relerr=float(np.median([r["uwc_relerr"] for r in ok])),
                **_flood_summary(ok))


def _flood_summary(ok: List[Dict]) -> Dict:
    """The no-network baseline beside the network, over the problems whose
    cold run reached equilibrium."""
    if not ok or "flood_pass" not in ok[0]:
        return {}
    fp = [r for r in ok if r["flood_pass"]]
    both = [r for r in ok if r["flood_pass"] and r["pass"]]
    return dict(flood_pass_rate=len(fp) / len(ok),
                flood_median_speedup_passing=float(np.median([r["flood_speedup"] for r in fp]))
                if fp else None,
                network_only_passes=sum(r["pass"] and not r["flood_pass"] for r in ok),
                flood_only_passes=sum(r["flood_pass"] and not r["pass"] for r in ok),
                median_warm_over_flood_s=float(np.median([r["warm_s"] / r["flood_s"]
                                                          for r in both])) if both else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-seeds", default="10000:10512")
    ap.add_argument("--eval-seeds", default="20000:20064")
    ap.add_argument("--eval-seeds-large", default="20000:20016")
    ap.add_argument("--edge", type=int, default=96)
    ap.add_argument("--edge-large", type=int, default=192)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-4)
    ap.add_argument("--budget", type=int, default=100000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--net-seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--save-params", default="")
    ap.add_argument("--load-params", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args()

    def rng_of(s):
        lo, hi = (int(v) for v in s.split(":"))
        return list(range(lo, hi))

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    train_seeds = rng_of(a.train_seeds) if not a.load_params else []
    ev = rng_of(a.eval_seeds)
    evl = rng_of(a.eval_seeds_large) if a.eval_seeds_large else []
    probs_train = generate(train_seeds, a.edge, a.workers)
    probs_eval = generate(ev, a.edge, a.workers)
    probs_large = generate(evl, a.edge_large, a.workers)
    log(f"generated {len(probs_train)} + {len(probs_eval)} + {len(probs_large)} problems "
        f"in {time.perf_counter() - t0:.1f} s")

    import torch
    import paper_2401_01672_amd as pf
    torch.cuda.set_device(0)
    net = pf.UNet(seed=a.net_seed)
    report = dict(args=vars(a))
    if a.load_params:
        net.set_params(np.load(a.load_params)["params"])
    else:
        t1 = time.perf_counter()
        data = make_dataset(probs_train, a.budget, a.batch, log)
        report["dataset_s"] = time.perf_counter() - t1
        report["dataset_equilibrium"] = sum(d["status"] == 1 for d in data)
        t1 = time.perf_counter()
        report["loss_per_epoch"] = train(net, data, a.epochs, a.lr, a.lr * 0.1, log=log)
        report["train_s"] = time.perf_counter() - t1
        del data
        torch.cuda.empty_cache()
        if a.save_params:
            np.savez(a.save_params, params=net.get_params())
    for name, probs in (("eval", probs_eval), ("eval_large", probs_large)):
        if not probs:
            continue
        res = evaluate(net, probs, a.budget, log)
        report[name] = dict(summary=summarize(res), results=res)
        log(f"{name}: {json.dumps(report[name]['summary'])}")
    report["wall_s"] = time.perf_counter() - t0
    if a.out:
        json.dump(report, open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
