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
XCDS, CUS = 8, 256  # MI355X: accelerator complex dies and compute units


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


def _all_counter_means(counter_csv: str) -> dict:
    """kernel -> counter -> (mean value per dispatch, dispatches), and kernel -> list of per-dispatch rows
    in dispatch order (for picking out the calibration dispatches)."""
    acc = defaultdict(lambda: defaultdict(list))
    order = defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        order[r["Kernel_Name"]].append((int(r.get("Dispatch_Id", 0) or 0), r["Counter_Name"], float(r["Counter_Value"])))
    return acc, order


def counters(csvs, workload: str, commands, kernels, source_hash: str, out_json: str, out_md: str,
             read_calib_entries: int = 0) -> dict:
    """Per-kernel means per dispatch of every counter of several rocprofv3 --pmc runs (one counter group per
    run), with the derived figures: read bytes from the request-size counters, L2 hit rate, mean waves per
    compute unit, share of wave time waiting."""
    per = defaultdict(dict)
    calib = {}
    for path in csvs:
        acc, order = _all_counter_means(path)
        for k, cs in acc.items():
            short = _short(k)
            for c, vals in cs.items():
                if short.startswith("(anonymous namespace)::k_probe_gather") and read_calib_entries:
                    # the first dispatch is the sequential read calibration, the others the gather probe
                    first_id = min(d for d, cn, _ in order[k] if cn == c)
                    cal = [v for d, cn, v in order[k] if cn == c and d == first_id]
                    rest = [v for d, cn, v in order[k] if cn == c and d != first_id]
                    calib[c] = cal[0]
                    if rest:
                        per["k_probe_gather (the workload's adjacency)"][c] = (sum(rest) / len(rest), len(rest))
                    continue
                per[short][c] = (sum(vals) / len(vals), len(vals))
    rows = {}
    for k in kernels:
        if k not in per:
            continue
        c = {name: v for name, (v, _) in per[k].items()}
        d = {"dispatches": max(n for _, n in per[k].values()), "counters": {n: round(v, 1) for n, v in c.items()}}
        if all(x in c for x in ("TCC_EA0_RDREQ_32B", "TCC_EA0_RDREQ_64B", "TCC_EA0_RDREQ_128B")):
            d["read_bytes"] = int(32 * c["TCC_EA0_RDREQ_32B"] + 64 * c["TCC_EA0_RDREQ_64B"] +
                                  128 * c["TCC_EA0_RDREQ_128B"])
        if "TCC_EA0_WRREQ" in c and "TCC_EA0_WRREQ_64B" in c:
            d["write_bytes"] = int(32 * (c["TCC_EA0_WRREQ"] - c["TCC_EA0_WRREQ_64B"]) + 64 * c["TCC_EA0_WRREQ_64B"])
        if "TCC_HIT" in c and "TCC_MISS" in c and c["TCC_HIT"] + c["TCC_MISS"] > 0:
            d["l2_hit_rate"] = round(c["TCC_HIT"] / (c["TCC_HIT"] + c["TCC_MISS"]), 4)
        if "SQ_WAVE_CYCLES" in c and "GRBM_GUI_ACTIVE" in c and c["GRBM_GUI_ACTIVE"] > 0:
            # GRBM_GUI_ACTIVE adds up the busy cycles of the 8 XCDs (an eighth of it matches the kernel's
            # duration at 2.4 GHz); SQ_WAVE_CYCLES counts in units of 4 cycles
            d["mean_waves_per_cu"] = round(4 * c["SQ_WAVE_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / XCDS) / CUS, 2)
        if "SQ_WAIT_INST_ANY" in c and "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
            d["wait_inst_share"] = round(c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"], 4)
        if "SQ_WAIT_ANY" in c and "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
            d["wait_any_share"] = round(c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"], 4)
        if "SQ_ACTIVE_INST_VALU" in c and "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"] > 0:
            d["valu_share"] = round(c["SQ_ACTIVE_INST_VALU"] / c["SQ_WAVE_CYCLES"], 4)
        rows[k] = d
    out = {"workload": workload, "source_hash": source_hash, "commands": commands, "kernels": rows}
    if calib and read_calib_entries:
        known = 8 * read_calib_entries
        rb = 32 * calib.get("TCC_EA0_RDREQ_32B", 0) + 64 * calib.get("TCC_EA0_RDREQ_64B", 0) + \
            128 * calib.get("TCC_EA0_RDREQ_128B", 0)
        out["read_calibration"] = {"entries": read_calib_entries, "known_read_bytes": known,
                                   "request_size_bytes": int(rb) if rb else None,
                                   "FETCH_SIZE_bytes": int(calib["FETCH_SIZE"] * 1024) if "FETCH_SIZE" in calib else None}
    json.dump(out, open(out_json, "w"), indent=1)
    lines = [f"# Hardware counters per dispatch, {workload}", "",
             "Means per dispatch of rocprofv3 counters, one counter group per run (commands below; each pass is",
             "a separate process running the same bench command).  Derived: read bytes = 32, 64 and 128 times",
             "the L2-to-fabric read requests of each size; write bytes likewise; mean waves per compute unit =",
             "4 * SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8) / 256 (GRBM_GUI_ACTIVE adds up the 8 XCDs' busy cycles;",
             "an eighth of it matches the kernel's duration at 2.4 GHz); wait share = SQ_WAIT_INST_ANY /",
             "SQ_WAVE_CYCLES.", "",
             "Commands:", "", "```", *commands, "```", ""]
    if "read_calibration" in out:
        rc = out["read_calibration"]
        lines += [f"Read calibration: one sequential pass over {rc['entries']} indices and values "
                  f"({rc['known_read_bytes']} bytes read): request-size counters {rc['request_size_bytes']} bytes, "
                  f"FETCH_SIZE {rc['FETCH_SIZE_bytes']} bytes.", ""]
    keys = ["read_bytes", "write_bytes", "l2_hit_rate", "mean_waves_per_cu", "wait_inst_share", "wait_any_share",
            "valu_share"]
    lines += ["| kernel | dispatches | " + " | ".join(keys) + " |", "|---|---:|" + "---:|" * len(keys)]
    for k, d in rows.items():
        lines.append(f"| `{k}` | {d['dispatches']} | " + " | ".join(str(d.get(x, "")) for x in keys) + " |")
    lines += ["", "Raw counter means:", ""]
    for k, d in rows.items():
        lines.append(f"- `{k}`: " + ", ".join(f"{n} {v}" for n, v in sorted(d["counters"].items())))
    open(out_md, "w").write("\n".join(lines) + "\n")
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--workload", required=True)
    c.add_argument("--commands-file", required=True, help="text file, one command per line")
    c.add_argument("--kernels", required=True, help="comma list of short kernel names")
    c.add_argument("--source-hash", default="")
    c.add_argument("--read-calib-entries", type=int, default=0)
    c.add_argument("--out-json", required=True)
    c.add_argument("--out-md", required=True)
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
    if args.cmd == "counters":
        cmds = [line.rstrip("\n") for line in open(args.commands_file) if line.strip()]
        counters(args.csvs, args.workload, cmds, args.kernels.split(";"), args.source_hash, args.out_json,
                 args.out_md, args.read_calib_entries)
        return
    if args.cmd == "kernel-stats":
        kernel_stats(args.stats_csv, args.command, args.title, args.out)
    else:
        pmc(args.fetch_csv, args.write_csv, args.copy_bytes, args.command_fetch, args.command_write, args.workload,
            args.source_hash, args.out_json, args.out_md)


if __name__ == "__main__":
    main()
