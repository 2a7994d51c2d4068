"""Summaries of rocprofv3 output for the kernels of this package.

``kernel-stats``: a rocprofv3 ``--kernel-trace --stats`` run (csv output) ->
a short markdown table (calls, total and average duration per kernel).

``pmc``: two rocprofv3 ``--pmc`` runs of the same command, one with
FETCH_SIZE and one with WRITE_SIZE (KiB per dispatch, L2-to-memory traffic),
whose process also copied a buffer of known size once (``bench.py
--pmc-calibrate``) -> per kernel the mean counter values per dispatch, scaled
by (known copy bytes / what the counter read for that copy), written as JSON
(read by bench.py for the roofline's ``traffic``) and markdown.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
from collections import defaultdict

CALIBRATION_KERNEL_HINT = "copy"  # the calibration copy is torch's copy kernel


def _short(name: str) -> str:
    name = name.replace("void ", "").replace("kcore::", "")
    return name.split("(")[0] if name.startswith("k_") else name[:90]


def kernel_stats(stats_csv: str, command: str, title: str, out_md: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command (from the repository root; rocprofv3 writes `run_kernel_stats.csv`):", "",
             "```", command, "```", "",
             "| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _counter_means(counter_csv: str, counter: str) -> dict:
    acc = defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        if r.get("Counter_Name") != counter:
            continue
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def _calibration_kib(counter_csv: str, counter: str):
    """Kernel name and value of the largest copy dispatch (the calibration copy)."""
    best = None
    for r in csv.DictReader(open(counter_csv)):
        if r.get("Counter_Name") != counter or CALIBRATION_KERNEL_HINT not in r["Kernel_Name"].lower():
            continue
        if "kcore" in r["Kernel_Name"]:
            continue
        v = float(r["Counter_Value"])
        if best is None or v > best[1]:
            best = (r["Kernel_Name"], v)
    if best is None:
        raise SystemExit(f"no calibration copy dispatch in the {counter} run")
    return best


def pmc(fetch_csv: str, write_csv: str, copy_bytes: int, command_fetch: str, command_write: str, workload: str,
        source_hash: str, out_json: str, out_md: str) -> dict:
    fetch = _counter_means(fetch_csv, "FETCH_SIZE")
    write = _counter_means(write_csv, "WRITE_SIZE")
    ck, fk_cal = _calibration_kib(fetch_csv, "FETCH_SIZE")
    _, wk_cal = _calibration_kib(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (fk_cal * 1024)
    w_scale = copy_bytes / (wk_cal * 1024)
    kernels = {}
    for k, (fk, calls) in fetch.items():
        if "kcore" not in k:
            continue
        wk = write.get(k, (0.0, 0))[0]
        kernels[_short(k)] = {"dispatches": calls, "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                              "bytes_per_launch_scaled": int(fk * 1024 * f_scale + wk * 1024 * w_scale)}
    out = {"workload": workload, "source_hash": source_hash, "calibration_kernel": _short(ck),
           "calibration_bytes": copy_bytes, "calibration_fetch_kib": fk_cal, "calibration_write_kib": wk_cal,
           "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "commands": [command_fetch, command_write], "kernels": kernels}
    json.dump(out, open(out_json, "w"), indent=1)
    lines = [f"# HBM-side traffic per launch, {workload}", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two separate rocprofv3 runs), scaled by what the same",
             f"counters read for a plain copy of {copy_bytes} bytes in the same process "
             f"(fetch x{f_scale:.4f}, write x{w_scale:.4f}).", "", "Commands:", "", "```", command_fetch,
             command_write, "```", "", "| kernel | dispatches | FETCH KiB | WRITE KiB | scaled bytes/launch |",
             "|---|---:|---:|---:|---:|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch_scaled"] * kv[1]["dispatches"]):
        lines.append(f"| `{k}` | {v['dispatches']} | {v['fetch_kib']} | {v['write_kib']} | "
                     f"{v['bytes_per_launch_scaled']} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernel-stats")
    a.add_argument("stats_csv")
    a.add_argument("--command", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("--out", required=True)
    b = sub.add_parser("pmc")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--source-hash", required=True)
    b.add_argument("--out-json", required=True)
    b.add_argument("--out-md", required=True)
    args = ap.parse_args()
    if args.cmd == "kernel-stats":
        kernel_stats(args.stats_csv, args.command, args.title, args.out)
    else:
        pmc(args.fetch_csv, args.write_csv, args.copy_bytes, args.command_fetch, args.command_write, args.workload,
            args.source_hash, args.out_json, args.out_md)


if __name__ == "__main__":
    main()
