"""HBM-traffic measurement helpers for the stencil passes.

Two modes, used around rocprofv3 counter runs:

  python -m paper_2401_01672_amd.profiling run --workload W --schedule S
      runs adaptive steps of workload W under stencil schedule S, then two
      calibration kernels of known size (a 1 GiB fill, which writes 1 GiB, and
      a 1 GiB float32 -> float64 conversion, which reads 1 GiB), so that one
      ``rocprofv3 --pmc FETCH_SIZE`` (or ``WRITE_SIZE``) run sees both;

  python -m paper_2401_01672_amd.profiling summarize --workload W --schedule S \
         --fetch DIR_FETCH --write DIR_WRITE --out DIR
      reads the two counter CSVs, scales each counter by its reading for the
      calibration kernel (bytes moved / counter value), and writes
      ``traffic_<S>_pass<N>_<W>.json``: HBM bytes per launch of every pass,
      with the hash of the kernel sources it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CAL_BYTES = 1 << 30


STENCIL_SOURCES = ("pf_internal.h", "pf_stencil.hip")
UNET_SOURCES = ("pf_unet_internal.h", "pf_unet.hip")


def source_hash(files=STENCIL_SOURCES) -> str:
    """Hash of kernel sources (by default the stencil kernels', on which the
    stencil traffic depends)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2401_01672_amd", "csrc")
    for f in files:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def run(workload: str, schedule: str, steps: int, stage_z=None):
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import bench
    import paper_2401_01672_amd as pf
    import pf_inputs as pi

    wl = bench.WORKLOADS[workload]
    case, s, _ = bench.make_solver(wl)
    s.set_loop(16, False)
    if schedule != "five":
        s.set_schedule(schedule)  # and the same tile autotuner as the benchmark
    if stage_z:
        s.set_stage_tiles(stage_z)  # fixed depths: the counters then match a known config
    s.set_time(0.0, case.run["dt0"])
    st = s.integrate(max_steps=steps)
    print(json.dumps(dict(steps=steps, accepted=st["steps_accepted"], config=s.get_config())),
          flush=True)
    s.close()
    a = torch.empty(CAL_BYTES // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)             # calibration: writes CAL_BYTES
    torch.cuda.synchronize()
    b = a.to(torch.float64)  # calibration: reads CAL_BYTES
    torch.cuda.synchronize()
    print(json.dumps(dict(calibration_bytes=CAL_BYTES, check=float(b[0]))), flush=True)


def _read_counter(d: str, counter: str):
    """[(kernel name, value)] per dispatch from a rocprofv3 counter CSV."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name", counter) != counter:
                continue
            out.append((row.get("Kernel_Name", ""), float(row["Counter_Value"])))
    return out


def _template_args(name: str):
    m = re.search(r"<([^<>]*)>", name)
    return [x.strip() for x in m.group(1).split(",")] if m else []


def pass_of(name: str, schedule: str):
    """1-based pass index of a kernel dispatch under the schedule, or None."""
    args = _template_args(name)
    if "pair_kernel<" in name and schedule == "paired" and len(args) >= 3:
        return 1 if args[2] == "1" else 2
    if ("stage_kernel<" in name or "stage4_kernel<" in name) and len(args) >= 3:
        st = int(args[2])
        if schedule == "five":
            return st if st >= 1 else None
        return 3 if st == 5 else None
    return None


def summarize(workload: str, schedule: str, fetch_dir: str, write_dir: str, out_dir: str,
              stage_z=None):
    fetch = _read_counter(fetch_dir, "FETCH_SIZE")
    write = _read_counter(write_dir, "WRITE_SIZE")
    # calibration: the conversion kernel reads CAL_BYTES (largest FETCH among
    # torch elementwise kernels); the fill kernel writes CAL_BYTES
    f_cal = max(v for k, v in fetch if "elementwise" in k or "copy" in k.lower())
    w_cal = max(v for k, v in write if "FillFunctor" in k)
    fr = (CAL_BYTES / 1024.0) / f_cal
    wr = (CAL_BYTES / 1024.0) / w_cal
    sh = source_hash()
    npass = 3 if schedule == "paired" else 5
    written = []
    for p in range(1, npass + 1):
        fk = sorted(v for k, v in fetch if pass_of(k, schedule) == p)
        wk = sorted(v for k, v in write if pass_of(k, schedule) == p)
        if not fk or not wk:
            continue
        f_kib, w_kib = fk[len(fk) // 2], wk[len(wk) // 2]  # median dispatch
        zarg = f" --stage-z {','.join(str(v) for v in stage_z)}" if stage_z else ""
        run_cmd = (f"python3 -m paper_2401_01672_amd.profiling run --workload {workload}"
                   + (f" --schedule {schedule}" if schedule != "five" else "") + zarg)
        rec = dict(workload=workload, schedule=schedule, kernel=f"{schedule}_pass{p}",
                   commands=[
                       "cd /tmp && export TMPDIR=/tmp && cd /root/repo",
                       f"rocprofv3 --pmc FETCH_SIZE -d {fetch_dir} -o run --output-format csv "
                       f"-- {run_cmd}",
                       f"rocprofv3 --pmc WRITE_SIZE -d {write_dir} -o run --output-format csv "
                       f"-- {run_cmd}",
                       f"python3 -m paper_2401_01672_amd.profiling summarize --workload {workload}"
                       f" --fetch {fetch_dir} --write {write_dir}{zarg}"],
                   source_hash=sh, dispatches=len(fk),
                   z_chunk=(int(stage_z[p - 1]) if stage_z and schedule == "five" else None),
                   fetch_kib_per_dispatch=f_kib, write_kib_per_dispatch=w_kib,
                   fetch_scale=fr, write_scale=wr,
                   bytes_per_launch=f_kib * 1024 * fr + w_kib * 1024 * wr,
                   calibration=f"{CAL_BYTES}-byte fill (WRITE_SIZE x{wr:.4f}) and "
                               f"{CAL_BYTES}-byte-read conversion (FETCH_SIZE x{fr:.4f})")
        path = os.path.join(out_dir, f"traffic_{schedule}_pass{p}_{workload}.json")
        json.dump(rec, open(path, "w"), indent=1)
        written.append(path)
    print("\n".join(written))


def kernel_stats(title: str, trace_dir: str, command: str, out: str, sources=STENCIL_SOURCES):
    """Markdown table of per-kernel durations from a rocprofv3 kernel trace.

    Besides the plain average over all dispatches it gives the average over
    working dispatches: a stencil pass launched after the step controller has
    already stopped (the tail of a captured batch of attempts) exits at once,
    and those few-microsecond dispatches are excluded there (duration below
    20% of the kernel's median)."""
    import statistics
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_trace.csv under {trace_dir}")
    by = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            by.setdefault(r["Kernel_Name"], []).append(d)
    total = sum(sum(v) for v in by.values())
    lines = [f"# rocprofv3 kernel statistics: {title}", "", "Command (repo root):", "", "```",
             command, "```", "", f"Kernel sources: `{source_hash(sources)}`", "",
             "| kernel | calls | avg us | working calls | working avg us | min us | max us | % time |",
             "|---|---|---|---|---|---|---|---|"]
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        med = statistics.median(v)
        w = [x for x in v if x >= 0.2 * med]
        lines.append(f"| `{k[:90]}` | {len(v)} | {sum(v) / len(v):.2f} | {len(w)} | "
                     f"{sum(w) / len(w):.2f} | {min(v):.2f} | {max(v):.2f} | "
                     f"{100 * sum(v) / total:.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")
    print(out)


def conv(edge: int, reps: int, variant: str):
    """The trained warm-start network's ten forward convolutions on an
    edge^3 grid (pf_unet_time_layers: reps launches of each, back to back)."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import paper_2401_01672_amd as pf
    torch.cuda.set_device(0)
    net = pf.UNet(seed=0)
    net.set_params(np.load(os.path.join(ROOT, "paper_2401_01672_amd", "data",
                                        "unet_warmstart_96.npz"))["params"])
    net.set_conv_kernel(variant)
    ms = net.time_layers((edge, edge, edge), reps=reps)
    out = []
    for i, t in enumerate(ms):
        info = pf.unet_layer_info(i)
        nv = edge ** 3 // (8 ** info["level"])
        fl = 2 * 27 * info["cin"] * info["cout"] * nv
        out.append(dict(layer=i, cin=info["cin"], cout=info["cout"], voxels=nv,
                        us=round(t * 1e3, 2), tflops=round(fl / (t * 1e-3) / 1e12, 1)))
    print(json.dumps(dict(edge=edge, variant=variant, layers=out)), flush=True)
    net.close()


def pmc_summary(title: str, dirs, commands, out: str, match: str = "",
                sources=STENCIL_SOURCES):
    """Markdown table of per-dispatch counter means per kernel, from one or
    more rocprofv3 --pmc runs (one counter set per run)."""
    vals = {}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise FileNotFoundError(f"no counter_collection.csv under {d}")
        for f in files:
            for row in csv.DictReader(open(f)):
                k = row.get("Kernel_Name", "")
                if match and match not in k:
                    continue
                key = (k, row.get("Dispatch_Id", ""))
                vals.setdefault(k, {}).setdefault(row["Counter_Name"], {}).setdefault(
                    key, 0.0)
                vals[k][row["Counter_Name"]][key] += float(row["Counter_Value"])
    lines = [f"# rocprofv3 counters: {title}", "", "Commands (repo root):", "", "```",
             *commands, "```", "", f"Kernel sources: `{source_hash(sources)}`", "",
             "Per-dispatch means (counters summed over the GPU's instances).", ""]
    for k in sorted(vals):
        lines += [f"## `{k[:100]}`", "", "| counter | dispatches | mean per dispatch |",
                  "|---|---|---|"]
        for cname in sorted(vals[k]):
            v = list(vals[k][cname].values())
            lines.append(f"| {cname} | {len(v)} | {sum(v) / len(v):.6g} |")
        lines.append("")
    open(out, "w").write("\n".join(lines) + "\n")
    print(out)


def _depths(text: str):
    if not text:
        return None
    z = [int(v) for v in text.split(",")]
    if len(z) != 5 or min(z) < 1:
        raise SystemExit("--stage-z takes five depths >= 1 (S1..S5)")
    return z


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    pm = sub.add_parser("pmcsum")
    pm.add_argument("--title", required=True)
    pm.add_argument("--dirs", nargs="+", required=True)
    pm.add_argument("--commands", nargs="+", required=True)
    pm.add_argument("--match", default="")
    pm.add_argument("--out", required=True)
    pm.add_argument("--unet", action="store_true", help="hash the network's kernel sources")
    cv = sub.add_parser("conv")
    cv.add_argument("--edge", type=int, default=96)
    cv.add_argument("--reps", type=int, default=5)
    cv.add_argument("--variant", default="reg", choices=["tiled", "direct", "reg"])
    k = sub.add_parser("stats")
    k.add_argument("--title", required=True)
    k.add_argument("--trace", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--unet", action="store_true", help="hash the network's kernel sources")
    r = sub.add_parser("run")
    r.add_argument("--workload", default="coupled_256_fp32")
    r.add_argument("--schedule", default="five", choices=["paired", "five"])
    r.add_argument("--steps", type=int, default=64)
    r.add_argument("--stage-z", default="", help="S1..S5 depths, e.g. 16,16,16,22,22 (default: autotune)")
    s = sub.add_parser("summarize")
    s.add_argument("--workload", default="coupled_256_fp32")
    s.add_argument("--schedule", default="five", choices=["paired", "five"])
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    s.add_argument("--stage-z", default="", help="the depths the counter runs used")
    a = ap.parse_args()
    if a.cmd == "pmcsum":
        pmc_summary(a.title, a.dirs, a.commands, a.out, a.match,
                    UNET_SOURCES if a.unet else STENCIL_SOURCES)
    elif a.cmd == "conv":
        conv(a.edge, a.reps, a.variant)
    elif a.cmd == "stats":
        kernel_stats(a.title, a.trace, a.command, a.out,
                     UNET_SOURCES if a.unet else STENCIL_SOURCES)
    elif a.cmd == "run":
        run(a.workload, a.schedule, a.steps, _depths(a.stage_z))
    else:
        summarize(a.workload, a.schedule, a.fetch, a.write, a.out, _depths(a.stage_z))


if __name__ == "__main__":
    main()
