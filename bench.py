#!/usr/bin/env python3
"""Benchmark: GCUPS of the fused Runge-Kutta-Merson step on one MI355X.

Workload (default): the coupled heat + Allen-Cahn model on the 256^3
glass-bead grid (64 spheres of radius 28 voxels, ~35% solid; bottom face
ramped from -5 C to +5 C over 60 s, T0 = +1 C; tol 1e-6 adaptive steps), FP32
fields with FP64 error norm, time, step and diagnostic sums.  One benchmark
step is one adaptive Merson attempt over the whole grid: five fused stage
passes, the FP64 error-norm and diagnostic reductions and the on-device step
controller (a kernel of its own at this size).  GCUPS = cells x attempts / s / 1e9 (every cell counts, glass
included).  The 128^3 FP64 case and the other workloads run with --workload.

Prints ONE JSON line.  Inputs are synthetic (seeded random sequential addition
of spheres) and resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS of fused RKM step (FP64/FP32); time-to-equilibrium warm vs cold start"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per cell of each pass, per unknown: words read + written,
# plus the 1-byte neighbourhood code.
#  five-pass schedule, vector kernels (Y2 and Y4 formed at the stencil
#  points, never stored):
#                      S1 r y, w k1 | S2 r y k1, w Y3 | S3 r Y3, w k3
#                      | S4 r y k1 k3, w Y5 P C | S5 r Y5 P C, w y_new
#  five-pass schedule, one-cell kernels (every stage value stored):
#                      S1 r y, w Y2 k1 | S2 r Y2 k1, w Y3 | S3 r Y3 y k1, w Y4 k3
#                      | S4 r Y4 y k1 k3, w Y5 P C | S5 r Y5 P C, w y_new
#  paired schedule:    S1+S2 r y, w k1 Y3 | S3+S4 r Y3 y k1, w Y5 P C
#                      | S5 r Y5 P C, w y_new
PASS_WORDS = {"five": [2, 3, 2, 6, 4], "five_one_cell": [3, 3, 5, 7, 4], "paired": [3, 6, 4]}
PASS_NAMES = {"five": ["S1", "S2", "S3", "S4", "S5"], "paired": ["S1+S2", "S3+S4", "S5"]}
PASS_KERNELS = {"five": ["stage4_kernel<..,1>", "stage4_kernel<..,2>", "stage4_kernel<..,3>",
                         "stage4_kernel<..,4>", "stage4_kernel<..,5>"],
                "paired": ["pair_kernel<..,1,..>", "pair_kernel<..,3,..>",
                           "stage_kernel<..,5>"]}


def pass_bytes(schedule: str, nvar: int, esize: int):
    return [w * nvar * esize + 1 for w in PASS_WORDS[schedule]]


WORKLOADS = {
    "coupled_128_fp64": dict(
        case="case_coupled_128", precision="fp64",
        desc="coupled heat + Allen-Cahn (SigmaP1-P), FP64, 128^3, 64 spheres r=14, "
             "bottom Dirichlet -5 C, T0=+1 C, adaptive RKM tol 1e-6"),
    "coupled_256_fp32": dict(
        case="case_coupled_256", precision="fp32",
        desc="coupled heat + Allen-Cahn (SigmaP1-P), FP32 fields + FP64 reductions, 256^3, "
             "64 spheres r=28, bottom Dirichlet ramp -5 -> +5 C over 60 s, adaptive RKM tol 1e-6"),
    "warmstart_96": dict(
        case=None, precision="fp32",
        desc="learned warm start: trained 3D U-Net (16/32/64 channels, BF16 matrix-core "
             "convolutions) on held-out micro-scale problems at 96^3 (sweep generator, seeds "
             "20000+); per problem the wall time to max|dphi/dt| < 1e-6 from the sharp nucleus "
             "(cold) and from the network's prediction (warm, inference included); value = "
             "median cold/warm wall-time ratio over the problems whose cold run reaches "
             "equilibrium"),
    "temp_256_fp32": dict(
        case="case_coupled_256", precision="fp32", override=dict(model="temp", gamma=2.0),
        kernel="stage_kernel",
        desc="Temp model (Sec. 2.3: phi = varphi(T), apparent heat capacity), FP32 fields + "
             "FP64 reductions, 256^3 bead pack of the coupled case, bottom Dirichlet ramp "
             "-5 -> +5 C, adaptive RKM tol 1e-6, one-cell stage kernels"),
    "gradp_256_fp32": dict(
        case="case_coupled_256", precision="fp32", override=dict(reaction="gradp"),
        kernel="stage_kernel",
        desc="coupled heat + Allen-Cahn with the GradP reaction term, FP32 fields + FP64 "
             "reductions, 256^3 bead pack of the coupled case, bottom Dirichlet ramp "
             "-5 -> +5 C, adaptive RKM tol 1e-6, one-cell stage kernels"),
    "paper_200_fp32": dict(
        case="case_paper", case_args=dict(n3=200), precision="fp32", kernel="stage_kernel",
        desc="paper mode (Sec. 2.1, Tab. 2): coupled heat + Allen-Cahn on a 100x100x200 "
             "vessel, smooth glass field (RSA bead bed + glass cap), no phase-field face rule, "
             "nucleation disk anchored in the cap, cap face cooled to T*-25 K from T*+20 K, "
             "FP32 fields + FP64 reductions, adaptive RKM tol 1e-6, one-cell stage kernels"),
    "sweep48_fp32": dict(
        case=None, precision="fp32",
        desc="batched parametric sweep: 48 micro-scale Allen-Cahn instances (edges 48-96, "
             "bead radius 5-12 vox, 30-37% solid, dT 0.02-2 K, sigma scale 1-1000), FP32, "
             "per-instance adaptive RKM, each run to max|dphi/dt| < 1e-6 (attempt budget "
             "per instance), one batched launch per stage"),
}


def run_sweep(args):
    """All instances of the sweep to equilibrium in one batch; GCUPS counts the
    cell-updates actually performed (sum over instances of cells x attempts)."""
    import numpy as np
    import torch

    import paper_2401_01672_amd as pf
    import pf_inputs as pi

    torch.cuda.set_device(0)
    cases = pi.sweep_instances(48)
    ncell = sum(c.ncells for c in cases)

    def fresh():
        ss = []
        for c in cases:
            s = pf.Solver(c.params, c.mask, "fp32", c.run)
            s.set_state(c.phi0.astype(np.float32))
            s.set_time(0.0, c.run["dt0"])
            ss.append(s)
        return ss

    # early-phase step time (the instances still active): the bandwidth
    # figure, over EARLY batched attempts (one call, so its set-up -- item
    # table, graph capture -- is amortised over them)
    EARLY = 512
    ss = fresh()
    pf.batch_integrate(ss, max_steps=32, eq_tol=1e-6)  # warm-up (graph build, caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = pf.batch_integrate(ss, max_steps=EARLY, eq_tol=1e-6)
    torch.cuda.synchronize()
    early = time.perf_counter() - t0
    att_early = sum(x["steps_accepted"] + x["steps_rejected"] for x in st)
    cell_att_early = sum(c.ncells * (x["steps_accepted"] + x["steps_rejected"])
                         for c, x in zip(cases, st))
    for s in ss:
        s.close()
    ms_step = early / EARLY * 1e3
    # the full sweep to equilibrium
    ss = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = pf.batch_integrate(ss, max_steps=args.sweep_budget, eq_tol=1e-6,
                            raise_on_error=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    updates = sum(c.ncells * (x["steps_accepted"] + x["steps_rejected"])
                  for c, x in zip(cases, st))
    attempts = max(x["steps_accepted"] + x["steps_rejected"] for x in st)
    for s in ss:
        s.close()
    bpc = sum(PASS_WORDS["five"]) * 4 + 5  # AC model, FP32, five vector passes
    # bytes of the cell-updates actually performed (instances that reached
    # equilibrium within the early attempts stop counting)
    achieved = bpc * cell_att_early / early / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                kernel="one batched attempt of all 48 instances (5 stage launches + "
                       "controller, graph replay)",
                algorithmic_bytes_per_launch=int(round(bpc * cell_att_early / EARLY)))
    extra = dict(cells_total=ncell, early_ms_per_attempt=round(ms_step, 4),
                 early_attempts_check=att_early,
                 equilibrium=sum(x["status"] == 1 for x in st), instances=len(st),
                 max_attempts=attempts, budget=args.sweep_budget,
                 uwc=[round(x["uwc"], 4) for x in st])
    return updates / wall / 1e9, wall, roof, extra, attempts, ncell


MFMA_BF16_PEAK_TFLOPS = 2500.0


def run_warmstart(args, probs):
    """Trained network on held-out problems: warm vs cold time to equilibrium,
    and the convolutions against the dense BF16 matrix-core peak."""
    import numpy as np
    import torch

    import paper_2401_01672_amd as pf
    from paper_2401_01672_amd import warmstart as W

    torch.cuda.set_device(0)
    path = os.path.join(ROOT, "paper_2401_01672_amd", "data", "unet_warmstart_96.npz")
    net = pf.UNet(seed=0)
    net.set_params(np.load(path)["params"])
    edge = 96
    ms = net.time_layers((edge, edge, edge), reps=args.kernel_reps)
    nvox = edge ** 3
    layers = []
    for i, t in enumerate(ms):
        info = pf.unet_layer_info(i)
        nv = nvox // (8 ** info["level"])
        fl = 2 * 27 * info["cin"] * info["cout"] * nv
        layers.append(dict(layer=i, cin=info["cin"], cout=info["cout"], voxels=nv, ms=round(t, 5),
                           gflop=round(fl / 1e9, 3), tflops=round(fl / (t * 1e-3) / 1e12, 1)))
    dom = max(range(len(ms)), key=lambda i: ms[i])
    fl_dom = layers[dom]["gflop"] * 1e9
    achieved = fl_dom / (ms[dom] * 1e-3) / 1e12
    roof = dict(bound="mfma", achieved=round(achieved, 1), peak=MFMA_BF16_PEAK_TFLOPS,
                unit="TFLOP/s", frac=round(achieved / MFMA_BF16_PEAK_TFLOPS, 4), traffic=None,
                kernel=f"{'conv3_xfold_kernel' if layers[dom]['cout'] == 16 else 'conv3_tile_kernel'}, "
                       f"convolution {dom} ({layers[dom]['cin']} -> "
                       f"{layers[dom]['cout']} channels at {edge}^3), BF16 in, FP32 accumulate",
                algorithmic_flops_per_launch=fl_dom)
    res = W.evaluate(net, probs, args.ws_budget, log=lambda m: print(m, file=sys.stderr))
    summ = W.summarize(res)
    net.close()
    extra = dict(summary=summ, conv_layers=layers,
                 forward_ms=round(sum(ms), 4),
                 forward_tflops=round(sum(l["gflop"] for l in layers) / sum(ms), 1),
                 problems=[dict(seed=r["seed"], cold_s=round(r["cold_s"], 4),
                                warm_s=round(r["warm_s"], 4), uwc_cold=r["uwc_cold"],
                                uwc_warm=r["uwc_warm"], cold_attempts=r["cold_attempts"],
                                warm_attempts=r["warm_attempts"], passed=r["pass"])
                           for r in res])
    return summ, roof, extra, res


def kernel_source_hash() -> str:
    from paper_2401_01672_amd.profiling import source_hash
    return source_hash()


def read_traffic(workload: str, kernel: str, src_hash: str, z_chunk=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and (when it records one) at the
    depth this run's pass uses; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != src_hash:
        return None
    if d.get("z_chunk") is not None and z_chunk is not None and d["z_chunk"] != z_chunk:
        return None
    return d.get("bytes_per_launch")


def make_solver(wl):
    """(case, solver with its initial state set, model) of a stencil workload."""
    import numpy as np

    import paper_2401_01672_amd as pf
    import pf_inputs as pi

    case = getattr(pi, wl["case"])(**wl.get("case_args", {}))
    params = dict(case.params, **wl.get("override", {}))
    model = params.get("model", case.model)
    npdt = np.float64 if wl["precision"] == "fp64" else np.float32
    s = pf.Solver(params, case.mask, wl["precision"], dict(case.run), glass_field=case.G)
    th = None if case.T0 is None else (case.T0 - params["t_star"]).astype(npdt)
    if model == "temp":
        s.set_state(None, th)
    else:
        s.set_state(case.phi0.astype(npdt), th)
    return case, s, model


def poll_interval(steps: int, warmup: int, cap: int) -> int:
    """Attempts per host poll (and per captured graph): the largest value up to
    cap that divides the timed attempts and, if possible, the warm-up ones too,
    so that the graph is captured during the warm-up and the timed region
    issues exactly `steps` attempts as whole graphs."""
    cap = max(1, cap)
    both = [d for d in range(1, cap + 1) if steps % d == 0 and (warmup == 0 or warmup % d == 0)]
    if both and both[-1] >= 4:
        return both[-1]
    return max(d for d in range(1, cap + 1) if steps % d == 0)


def profile_check(workload: str, kernel_sig: str, event_us: float):
    """The dominant kernel's working average from the committed rocprofv3
    kernel-trace summary of this workload, beside the HIP-event mean, if the
    summary was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"stage_kernels_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"Kernel sources: `([0-9a-f]+)`", text)
    if not m or m.group(1) != kernel_source_hash():
        return dict(file=os.path.relpath(path, ROOT), current=False)
    for line in text.splitlines():
        if line.startswith("| `") and kernel_sig in line:
            cols = [c.strip() for c in line.strip("|").split("|")]
            prof_us = float(cols[4])
            return dict(file=os.path.relpath(path, ROOT), current=True, kernel=kernel_sig,
                        rocprof_working_avg_us=prof_us, event_avg_us=round(event_us, 2),
                        ratio=round(event_us / prof_us, 4))
    return dict(file=os.path.relpath(path, ROOT), current=True, kernel=kernel_sig)


def run_gpu(args, wl):
    import torch

    torch.cuda.set_device(0)
    prec = wl["precision"]
    case, s, model = make_solver(wl)
    run = dict(case.run)
    spp = poll_interval(args.steps, args.warmup, args.steps_per_poll)
    s.set_loop(spp, not args.no_graph)
    if args.schedule != "five":
        s.set_schedule(args.schedule)
    if args.z_chunk:
        s.set_tile(args.z_chunk)
    s.set_time(0.0, run["dt0"])
    torch.cuda.synchronize()
    # warmup (includes the tile autotuner on the first call)
    if args.warmup > 0:
        s.integrate(max_steps=args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.integrate(max_steps=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    attempts = st["steps_accepted"] + st["steps_rejected"]
    assert attempts == args.steps, st
    ncell = case.ncells
    gcups = ncell * attempts / wall / 1e9
    # per-kernel durations with HIP events on the library's stream
    ms = s.time_kernels(args.kernel_reps)
    cfg = s.get_config()
    sched = cfg["schedule"]
    esize = 8 if prec == "fp64" else 4
    nvar = 2 if model == "coupled" else 1
    sb = pass_bytes(sched if sched != "five" or cfg.get("vector", True) else "five_one_cell",
                    nvar, esize)
    if case.G is not None:  # paper mode also reads the glass field in every pass
        sb = [b + esize for b in sb]
    npass = len(sb)
    per_pass = []
    for i in range(npass):
        gbs = sb[i] * ncell / (ms[i] * 1e-3) / 1e9
        kl = PASS_KERNELS[sched][i]
        if not cfg.get("vector", True):
            kl = kl.replace("stage4_kernel", "stage_kernel")
        per_pass.append(dict(pass_=PASS_NAMES[sched][i], kernel=kl,
                             ms=round(ms[i], 5), bytes_per_cell=sb[i], gbs=round(gbs, 1)))
    # the dominant kernel: the pass that moves the most bytes (also the
    # longest one; choosing by bytes keeps the choice stable under a profiler,
    # which lengthens the first launch after each timing event)
    dom = max(range(npass), key=lambda i: (sb[i], ms[i]))
    step_ms = sum(ms[:npass]) + ms[5]
    src_hash = kernel_source_hash()
    kname = f"{sched}_pass{dom + 1}"
    zdom = list(cfg.get("stage_z_chunk", []))
    zdom = zdom[dom] if sched == "five" and len(zdom) == 5 else None
    traffic = read_traffic(args.workload, kname, src_hash, zdom)
    achieved = per_pass[dom]["gbs"]
    kl = per_pass[dom]["kernel"]
    ksig = (f"{kl.split('<')[0]}<{'float' if prec == 'fp32' else 'double'}, "
            f"{1 if model == 'coupled' else 0 if model == 'ac' else 2}, {dom + 1},")
    roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=f"{per_pass[dom]['kernel']} = {PASS_NAMES[sched][dom]} "
                       f"({prec}, {model}{', GradP' if 'gradp' in args.workload else ''})",
                algorithmic_bytes_per_launch=sb[dom] * ncell,
                timing="HIP events on the library's stream (pf_time_kernels)",
                profile_check=profile_check(args.workload, ksig, ms[dom] * 1e3))
    extra = dict(
        passes=per_pass,
        step_kernels_ms=round(step_ms, 5),
        step_algorithmic_bytes_per_cell=sum(sb),
        step_effective_gbs=round(sum(sb) * ncell / (step_ms * 1e-3) / 1e9, 1),
        controller_ms=round(ms[5], 5),
        accepted=st["steps_accepted"], rejected=st["steps_rejected"], t_sim=st["t"],
        ice_fraction=st["ice_fraction"], source_hash=src_hash, config=cfg,
        steps_per_poll=spp, attempts_timed=attempts,
    )
    s.close()
    return gcups, wall, roof, extra, case, prec


def cpu_baseline(wl, cell_updates: float):
    """The FP64 oracle (as it stands) on the same grid for a bounded number of
    adaptive attempts (about `cell_updates` cell-updates, at least 2 attempts),
    timed on this host's cores (all of them, and one: the single-thread rate
    from a tenth of the sample, at least one attempt, goes into the detail)."""
    import ctypes

    import oracle
    import pf_inputs as pi

    case = getattr(pi, wl["case"])(**wl.get("case_args", {}))
    params = dict(case.params, **wl.get("override", {}))
    P = oracle.make_params(params)
    T0 = case.T0
    phi0 = None if params.get("model") == "temp" else case.phi0
    G = case.mask if case.G is None else case.G

    def timed(steps):
        ctl = oracle.make_ctl(tol=case.run["tol"])
        t0 = time.perf_counter()
        _, _, st = oracle.integrate(P, G, ctl, 0.0, case.run["dt0"], phi0, T0, max_steps=steps)
        wall = time.perf_counter() - t0
        n = st["steps_accepted"] + st["steps_rejected"]
        return n, wall, case.ncells * n / wall / 1e9

    cores = oracle.num_threads()
    sample_steps = max(2, int(round(cell_updates / case.ncells)))
    n, wall, rate = timed(sample_steps)
    out = dict(value=round(rate, 5), unit="GCUPS", cores=cores, kind="oracle",
               sample=f"{n} adaptive RKM attempts of the same {case.shape[::-1]} grid in "
                      f"FP64 ({wall:.1f} s)")
    if cores > 1:
        try:  # the oracle's OpenMP runtime, already loaded by the oracle library
            gomp = ctypes.CDLL("libgomp.so.1")
        except OSError:
            gomp = None
        if gomp is not None:
            gomp.omp_set_num_threads(1)
            n1, wall1, rate1 = timed(max(1, sample_steps // 10))
            gomp.omp_set_num_threads(cores)
            out["single_thread"] = dict(value=round(rate1, 6), attempts=n1,
                                        wall_s=round(wall1, 2))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="coupled_256_fp32", choices=sorted(WORKLOADS))
    ap.add_argument("--steps-per-poll", type=int, default=16)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--z-chunk", type=int, default=0)
    ap.add_argument("--schedule", default="five", choices=["paired", "five"])
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-cell-updates", type=float, default=4.2e8,
                    help="size of the oracle's timed sample in cell-updates (about 10 s on "
                         "16 host threads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-budget", type=int, default=60000,
                    help="attempt budget per instance of the sweep workload")
    ap.add_argument("--ws-problems", type=int, default=16,
                    help="held-out problems of the warm-start workload")
    ap.add_argument("--ws-budget", type=int, default=100000,
                    help="attempt budget per run of the warm-start workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps(dict(error="the benchmark runs on one GPU only (the path is single-device); --gpus must be 1")))
        sys.exit(2)
    wl = WORKLOADS[args.workload]
    if args.workload.startswith("warmstart"):
        from paper_2401_01672_amd import warmstart as W
        # problem generation on the CPU, before the GPU is touched
        probs = W.generate(list(range(20000, 20000 + args.ws_problems)), 96, workers=16)
        summ, roof, extra, res = run_warmstart(args, probs)
        out = dict(
            metric=METRIC, value=round(summ["median_speedup"], 3),
            unit="x (median cold/warm wall time to equilibrium)", n_gpus=1, steps=len(res),
            warmup=0, ms_per_step=round(summ["median_warm_s"] * 1e3, 4),
            higher_is_better=True, scaling="weak", vs_baseline=None, dtype="bf16+f32",
            data="synthetic (seeded random sequential addition of glass spheres)",
            config=dict(workload=f"{args.workload}: {wl['desc']}", grid=[96, 96, 96],
                        parallelism="single GPU"),
            roofline=roof, cpu_baseline=None, detail=extra)
        print(json.dumps(out))
        return
    if args.workload.startswith("sweep"):
        gcups, wall, roof, extra, attempts, ncell = run_sweep(args)
        out = dict(
            metric=METRIC, value=round(gcups, 4), unit="GCUPS", n_gpus=1, steps=attempts,
            warmup=1, ms_per_step=round(wall / max(attempts, 1) * 1e3, 5),
            higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
            data="synthetic (seeded random sequential addition of glass spheres)",
            config=dict(workload=f"{args.workload}: {wl['desc']}", cells=ncell,
                        parallelism="single GPU"),
            roofline=roof, cpu_baseline=None, detail=extra)
        print(json.dumps(out))
        return
    gcups, wall, roof, extra, case, prec = run_gpu(args, wl)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_cell_updates)
    out = dict(
        metric=METRIC, value=round(gcups, 4), unit="GCUPS", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(wall / args.steps * 1e3, 5),
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if prec == "fp64" else "f32",
        data="synthetic (seeded random sequential addition of glass spheres)",
        config=dict(workload=f"{args.workload}: {wl['desc']}", cells=case.ncells,
                    grid=list(case.shape[::-1]), parallelism="single GPU"),
        roofline=roof, cpu_baseline=cpu, detail=extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
