"""Convergence of the estimates round by round.

The paper follows how far the estimates are from the coreness after each
round (mean absolute error per iteration, Fig. 4) and what share of the
vertices is active in each round (Fig. 5).  This tool measures both for the
GPU path on a graph resident in device memory: for r = 1, 2, ... it runs the
decomposition stopped after r rounds (``kcore_tuning.max_rounds``; the tail is
off so that every round is a separate launch), reads the estimates, and
compares them with a reference coreness supplied by the caller (the tests
supply the CPU oracle's; without one, the final result of a full run is used).
Active and changed counts per round come from one run launched round by round.
Each stopped run is a separate asynchronous schedule, so the error rows come
from different (equally valid) interleavings.

    python -m paper_2512_00233_amd.convergence --workload rmat24 [--max-rounds 80]
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def profile(row_ptr, col_idx, max_rounds: int = 200, reference=None):
    """Rows of (round, active vertices, changed vertices, mean |est - core|, max error, exact share).

    Active and changed counts come from one run recorded round by round
    (``kcore_decompose_rounds``); the errors after r rounds from a run stopped
    there (``max_rounds = r``), against ``reference`` (numpy int32 [n], the
    coreness) when given, else against the final result of the recorded run.
    """
    import paper_2512_00233_amd as kc
    import torch
    n = row_ptr.numel() - 1
    core_t, recs = kc.decompose_rounds(row_ptr, col_idx, tuning=kc.Tuning(tail_threshold=-1))
    core = core_t.cpu().numpy() if reference is None else np.asarray(reference, dtype=np.int64)
    total = len(recs)
    rows = []
    for rec in recs[:max_rounds]:
        r = rec["round"]
        est = kc.decompose(row_ptr, col_idx, tuning=kc.Tuning(max_rounds=r)).cpu().numpy()
        torch.cuda.synchronize()
        err = est.astype(np.int64) - core
        if (err < 0).any():
            raise RuntimeError(f"round {r}: an estimate fell below the coreness")
        rows.append({"round": r, "active": rec["vertex_updates"], "changed": rec["changes"],
                     "activations": rec["activations"], "edge_visits": rec["edge_visits"],
                     "active_share": rec["vertex_updates"] / max(n, 1), "ms": rec["ms"],
                     "mean_abs_err": float(err.mean()) if n else 0.0, "max_err": int(err.max()) if n else 0,
                     "exact_share": float((err == 0).mean()) if n else 1.0})
    return rows, total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat24")
    ap.add_argument("--max-rounds", type=int, default=200)
    ap.add_argument("--json", default="")
    args = ap.parse_args()
    import torch

    import graphgen as gg
    g = gg.workload(args.workload)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    rows, total = profile(rp, ci, args.max_rounds)
    print(f"# {args.workload}: n={g.n} nnz={g.nnz}, {total} rounds without the tail")
    print("| round | active | active % | changed | ms | mean abs err | max err | exact % |")
    print("|---:|---:|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        print(f"| {r['round']} | {r['active']} | {100 * r['active_share']:.3f} | {r['changed']} | {r['ms']:.3f} | "
              f"{r['mean_abs_err']:.4f} | {r['max_err']} | {100 * r['exact_share']:.3f} |")
    if args.json:
        json.dump({"workload": args.workload, "rounds": total, "rows": rows}, open(args.json, "w"), indent=1)


if __name__ == "__main__":
    main()
