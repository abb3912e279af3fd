"""HBM-traffic measurement helpers for the stage kernels.

Two modes, used around rocprofv3 counter runs:

  python -m paper_2401_01672_amd.profiling run --workload W --steps K
      runs K adaptive steps of workload W and then a device copy of a known
      size (the calibration kernel), so one ``rocprofv3 --pmc FETCH_SIZE``
      (or WRITE_SIZE) run sees both;

  python -m paper_2401_01672_amd.profiling summarize --workload W \
         --fetch DIR_FETCH --write DIR_WRITE --out profiles/
      reads the two counter CSVs, scales each counter by the reading of the
      calibration copy (bytes moved / counter value), and writes
      ``traffic_stage<N>_<W>.json`` with the HBM bytes per launch of every
      stage kernel and the hash of the kernel sources it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_01672_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def run(workload: str, steps: int):
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import bench
    import paper_2401_01672_amd as pf
    import pf_inputs as pi

    wl = bench.WORKLOADS[workload]
    case = getattr(pi, wl["case"])()
    prec = wl["precision"]
    npdt = np.float64 if prec == "fp64" else np.float32
    s = pf.Solver(case.params, case.mask, prec, case.run)
    # same loop and tile autotuning as the benchmark; with enough steps the
    # per-stage median comes from the stepping dispatches, not the tuner's
    s.set_loop(16, False)
    th = None if case.T0 is None else (case.T0 - case.params["t_star"]).astype(npdt)
    s.set_state(case.phi0.astype(npdt), th)
    s.set_time(0.0, case.run["dt0"])
    st = s.integrate(max_steps=steps)
    print(json.dumps(dict(steps=steps, accepted=st["steps_accepted"])), flush=True)
    s.close()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=COPY_BYTES)), flush=True)


def _read_counter(d: str, counter: str):
    """{kernel name: [values per dispatch]} from a rocprofv3 counter CSV."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = {}
    for f in files:
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name", counter) != counter:
                continue
            name = row.get("Kernel_Name", "")
            out.setdefault(name, []).append(float(row["Counter_Value"]))
    return out


def summarize(workload: str, fetch_dir: str, write_dir: str, out_dir: str):
    fetch = _read_counter(fetch_dir, "FETCH_SIZE")
    write = _read_counter(write_dir, "WRITE_SIZE")

    def calib(tab):
        vals = [v for k, vs in tab.items() if "copy" in k.lower() or "elementwise" in k.lower()
                for v in vs]
        big = max(vals) if vals else None
        return (COPY_BYTES / 1024.0) / big if big else None

    fr, wr = calib(fetch), calib(write)
    sh = source_hash()
    written = []
    for st in range(1, 6):
        key = f"stage_kernel<"
        fk = [v for k, vs in fetch.items() if key in k and k.rstrip(")").split(",")[-1].strip()
              .startswith(f"{st}>") for v in vs]
        wk = [v for k, vs in write.items() if key in k and k.rstrip(")").split(",")[-1].strip()
              .startswith(f"{st}>") for v in vs]
        if not fk or not wk:
            continue
        # KiB per dispatch (median of the dispatches) scaled by the calibration
        fk.sort()
        wk.sort()
        f_kib = fk[len(fk) // 2]
        w_kib = wk[len(wk) // 2]
        rec = dict(workload=workload, kernel=f"stage{st}", source_hash=sh,
                   fetch_kib_per_dispatch=f_kib, write_kib_per_dispatch=w_kib,
                   fetch_scale=fr, write_scale=wr,
                   bytes_per_launch=(f_kib * 1024 * (fr or 1.0) + w_kib * 1024 * (wr or 1.0)),
                   calibration=f"torch copy of {COPY_BYTES} bytes: "
                               f"FETCH x{fr and round(fr, 4)}, WRITE x{wr and round(wr, 4)}")
        path = os.path.join(out_dir, f"traffic_stage{st}_{workload}.json")
        json.dump(rec, open(path, "w"), indent=1)
        written.append(path)
    print("\n".join(written))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="coupled_256_fp32")
    r.add_argument("--steps", type=int, default=64)
    s = sub.add_parser("summarize")
    s.add_argument("--workload", default="coupled_256_fp32")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.steps)
    else:
        summarize(a.workload, a.fetch, a.write, a.out)


if __name__ == "__main__":
    main()
