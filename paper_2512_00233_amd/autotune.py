"""Persist the batch autotuner's choices as JSON (one entry per batch shape).

The library keeps tuned launch knobs in a process-wide cache keyed by the
number of graphs and the log2 buckets of the total vertex and entry counts;
this module saves that choice to a file and loads it back into a new process.
"""
from __future__ import annotations

import json
import os

from . import Tuning, autotune_batch, tuning_cache_set

FIELDS = [name for name, _ in Tuning._fields_ if name != "reserved"]


def tuning_to_dict(t: Tuning) -> dict:
    return {name: int(getattr(t, name)) for name in FIELDS}


def tuning_from_dict(d: dict) -> Tuning:
    t = Tuning()
    for name in FIELDS:
        setattr(t, name, int(d.get(name, 0)))
    return t


def key_of(num_graphs: int, total_vertices: int, total_entries: int) -> str:
    return f"G{num_graphs}_n{max(total_vertices, 1).bit_length() - 1}_e{max(total_entries, 1).bit_length() - 1}"


def load_file(path: str) -> int:
    """Load every stored tuning into the library cache; returns the number loaded."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        data = json.load(f)
    for entry in data.values():
        tuning_cache_set(entry["num_graphs"], entry["total_vertices"], entry["total_entries"],
                         tuning_from_dict(entry["tuning"]))
    return len(data)


def tune_and_save(graph_vtx_off, row_ptr, col_idx, path: str, reps: int = 3, out=None) -> dict:
    """Run the autotuner on a resident batch and record its choice in `path`."""
    best, ms = autotune_batch(graph_vtx_off, row_ptr, col_idx, out=out, reps=reps)
    G = graph_vtx_off.numel() - 1
    N = row_ptr.numel() - 1
    nnz = int(row_ptr[-1].item())
    entry = {"num_graphs": G, "total_vertices": N, "total_entries": nnz, "ms": ms, "tuning": tuning_to_dict(best)}
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key_of(G, N, nnz)] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return entry
