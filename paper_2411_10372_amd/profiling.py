"""Summaries of rocprofv3 output for the files under ``profiles/``.

``trace``: per-kernel call counts and average durations from a
``rocprofv3 --kernel-trace --stats --output-format csv`` run.

``pmc``: HBM bytes per launch of one kernel from two ``rocprofv3 --pmc``
runs (``FETCH_SIZE``, then ``WRITE_SIZE``; KiB per dispatch), each scaled by
what the same counter reads for a plain device copy of known size (the
last three ``__amd_rocclr_copyBuffer`` dispatches of the run: ``bench.py
--copy-ref`` copies 256 MiB three times after everything it times).

``sq``: per-kernel sequencer counters (SQ_*, GRBM_GUI_ACTIVE) of one or
more ``rocprofv3 --pmc`` runs, summed over each kernel's dispatches, with
the ratios that say where a wave's time goes: wave-cycles issuing VALU,
scalar and LDS work, waiting for anything (memory, barriers, dependencies)
and waiting to be issued.  SQ_WAVE_CYCLES, SQ_WAIT_ANY and
SQ_WAIT_INST_ANY count quad-cycles, as do the SQ_ACTIVE_INST_* counters.

Usage (paths are the rocprofv3 output directories):
    python -m paper_2411_10372_amd.profiling trace DIR OUT.md "COMMAND"
    python -m paper_2411_10372_amd.profiling pmc FETCH_DIR WRITE_DIR KERNEL \
        WORKLOAD SOURCE_HASH COPY_BYTES OUT.json "COMMANDS" [DISPATCHES_PER_LAUNCH]
    python -m paper_2411_10372_amd.profiling sq OUT.md SOURCE_HASH "COMMANDS" DIR [DIR ...]
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _short(name: str) -> str:
    """Kernel name without its argument list and return type."""
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "")


def trace_summary(trace_dir: str, out_md: str, command: str, top: int = 12) -> list:
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "*kernel_stats.csv")))))
    lines = ["# Kernel trace summary", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    out = []
    for r in rows[:top]:
        name = _short(r["Name"])
        avg, mn, mx = (float(r[k]) / 1e3 for k in ("AverageNs", "MinNs", "MaxNs"))
        lines.append(f"| `{name}` | {r['Calls']} | {avg:.1f} | {mn:.1f} | {mx:.1f} | "
                     f"{float(r['Percentage']):.2f} % |")
        out.append({"kernel": name, "calls": int(r["Calls"]), "avg_us": avg})
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def _counter(dir_: str):
    return list(csv.DictReader(open(_one(os.path.join(dir_, "*counter_collection.csv")))))


def _mean_for(rows, pred):
    v = [float(r["Counter_Value"]) for r in rows if pred(r)]
    return (sum(v) / len(v), len(v)) if v else (None, 0)


def pmc_summary(fetch_dir: str, write_dir: str, kernel: str, workload: str, shash: str,
                copy_bytes: int, out_json: str, commands: str, per_launch: int = 1) -> dict:
    """HBM bytes of one launch of an operator: the mean over the dispatches
    whose name contains `kernel`, times `per_launch` dispatches per
    operator launch (an operator split over several kernels)."""
    fr, wr = _counter(fetch_dir), _counter(write_dir)

    def is_kernel(r):
        return kernel in r["Kernel_Name"]

    def big_copy(rows):
        # the reference copies are the run's last three copy dispatches
        # (bench.py --copy-ref makes them after everything it times); the
        # grid size alone does not single them out, other copies share it
        copies = sorted((r for r in rows if "copyBuffer" in r["Kernel_Name"]),
                        key=lambda r: int(r["Dispatch_Id"]))
        ids = {r["Dispatch_Id"] for r in copies[-3:]}
        return lambda r: "copyBuffer" in r["Kernel_Name"] and r["Dispatch_Id"] in ids

    fetch_kib, nf = _mean_for(fr, is_kernel)
    write_kib, nw = _mean_for(wr, is_kernel)
    cf, _ = _mean_for(fr, big_copy(fr))
    cw, _ = _mean_for(wr, big_copy(wr))
    half_kib = copy_bytes / 2 / 1024          # the copy reads and writes this much
    fs, ws = half_kib / cf, half_kib / cw
    d = {
        "kernel": kernel, "workload": workload, "source_hash": shash,
        "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib,
        "dispatches": [nf, nw],
        "copy_ref": {"bytes_read": copy_bytes // 2, "bytes_written": copy_bytes // 2,
                     "fetch_kib": cf, "write_kib": cw, "fetch_scale": fs, "write_scale": ws},
        "dispatches_per_launch": per_launch,
        "hbm_bytes_per_launch": (fetch_kib * fs + write_kib * ws) * 1024.0 * per_launch,
        "commands": commands,
    }
    with open(out_json, "w") as f:
        json.dump(d, f, indent=1)
    return d


def sq_summary(dirs, out_md: str, shash: str, commands: str) -> dict:
    """Sum every counter over each kernel's dispatches (all runs) and write
    the table of ratios per sweep kernel."""
    tot: dict = {}
    ndisp: dict = {}
    for d in dirs:
        for r in _counter(d):
            k = _short(r["Kernel_Name"])
            tot.setdefault(k, {}).setdefault(r["Counter_Name"], 0.0)
            tot[k][r["Counter_Name"]] += float(r["Counter_Value"])
            ndisp.setdefault(k, set()).add((d, r["Dispatch_Id"]))
    lines = ["# Sequencer counters", "", f"Source hash: `{shash}`", "", "Commands:", "", "```",
             commands, "```", "",
             "Per kernel, summed over its dispatches; shares of the waves' lifetime "
             "(SQ_WAVE_CYCLES):", "",
             "| kernel | dispatches | waves | VALU insts / wave | SALU insts / wave | "
             "issuing VALU | issuing SALU | issuing LDS | waiting (any) | waiting to issue |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    out = {}
    for k, c in sorted(tot.items()):
        if "sweep" not in k and "adj" not in k:
            continue
        wc = c.get("SQ_WAVE_CYCLES")
        w = c.get("SQ_WAVES")
        if not wc or not w:
            continue

        def share(n):
            v = c.get(n)
            return f"{100.0 * v / wc:.1f} %" if v is not None else "-"

        def per_wave(n):
            v = c.get(n)
            return f"{v / w:.0f}" if v is not None else "-"

        lines.append(f"| `{k}` | {len(ndisp[k]) // max(1, len(dirs))} | {w:.0f} | "
                     f"{per_wave('SQ_INSTS_VALU')} | {per_wave('SQ_INSTS_SALU')} | "
                     f"{share('SQ_ACTIVE_INST_VALU')} | {share('SQ_ACTIVE_INST_SCA')} | "
                     f"{share('SQ_ACTIVE_INST_LDS')} | {share('SQ_WAIT_ANY')} | "
                     f"{share('SQ_WAIT_INST_ANY')} |")
        out[k] = c
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


if __name__ == "__main__":
    a = sys.argv[1:]
    if a and a[0] == "trace":
        print(json.dumps(trace_summary(a[1], a[2], a[3]), indent=1))
    elif a and a[0] == "pmc":
        print(json.dumps(pmc_summary(a[1], a[2], a[3], a[4], a[5], int(a[6]), a[7], a[8],
                                     int(a[9]) if len(a) > 9 else 1), indent=1))
    elif a and a[0] == "sq":
        print(json.dumps(sq_summary(a[4:], a[1], a[2], a[3]), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
