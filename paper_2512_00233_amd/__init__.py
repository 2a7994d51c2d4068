"""Exact k-core decomposition on MI355X (gfx950) -- Python binding of libkcore.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libkcore.so`` (built in-tree by ``build.py``).  PyTorch supplies
device memory and the stream.  There is no CPU fallback: if the library is
missing or no GPU is present, the calls raise.

The method is the iterative coreness computation of the paper (Sec. II-B,
Alg. 1; FastK, Sec. IV): estimates start at the degree and are lowered to the
h-index of the neighbours' estimates until nothing changes; the fixed point is
the coreness of Definition 1 (Sec. II), bit-exact.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["decompose", "update", "certify", "decompose_noalloc", "decompose_rounds", "decompose_batch", "autotune_batch", "tuning_cache_set", "tuning_cache_get", "Tuning",
           "Stats", "KcoreError", "Server", "ServeConfig", "Completion", "library_path", "load", "version"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libkcore.so")
_lib = None

STATUS = {
    0: "KCORE_OK", -1: "KCORE_E_INVALID", -2: "KCORE_E_NOMEM", -3: "KCORE_E_HIP", -4: "KCORE_E_TOO_LARGE",
    -5: "KCORE_E_AGAIN", -6: "KCORE_E_CANCELLED", -7: "KCORE_E_TIMEOUT",
}


class KcoreError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Tuning(ctypes.Structure):
    """Mirror of ``kcore_tuning`` (zero = library default)."""
    _fields_ = [
        ("thread_max_deg", ctypes.c_int32),
        ("group_max_deg", ctypes.c_int32),
        ("wave_max_deg", ctypes.c_int32),
        ("tail_threshold", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("big_grid_blocks", ctypes.c_int32),
        ("rounds_per_poll", ctypes.c_int32),
        ("activation", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("list_cap", ctypes.c_int32),
        ("no_prune", ctypes.c_int32),
        ("no_graph", ctypes.c_int32),
        ("max_rounds", ctypes.c_int32),
        ("relabel", ctypes.c_int32),
        ("deferred", ctypes.c_int32),
        ("tail_round_cap", ctypes.c_int32),
        ("tail_order", ctypes.c_int32),
        ("tail_big", ctypes.c_int32),
        ("round_renorm", ctypes.c_int32),
        ("big_wave", ctypes.c_int32),
        ("dense_sweep", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


KERNELS = ("big_first", "round_first", "big", "round", "compact", "defer")
# rocprofv3 names of the kernels of a single-graph run (int64 offsets), by KERNELS entry
KERNEL_SYMBOLS = {
    "big_first": "k_big<true, false, long>",
    "round_first": "k_round<256, true, false, long>",
    "big": "k_big<false, false, long>",
    "round": "k_round<256, false, false, long>",
    "compact": "k_compact<false, long>",
    "defer": "k_defer<long>",
}
# the class-3 wavefront pass of later rounds runs before k_big and counts its work with it
BIG_WAVE_SYMBOL = "k_big_wave<false, long>"


class KernelStats(ctypes.Structure):
    """Mirror of ``kcore_kernel_stats``."""
    _fields_ = [
        ("launches", ctypes.c_int64),
        ("vertex_updates", ctypes.c_int64),
        ("edge_visits", ctypes.c_int64),
        ("changes", ctypes.c_int64),
        ("activations", ctypes.c_int64),
        ("prune_writes", ctypes.c_int64),
        ("full_scans", ctypes.c_int64),
        ("max_full_scan", ctypes.c_int64),
        ("ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Stats(ctypes.Structure):
    """Mirror of ``kcore_stats``."""
    _fields_ = [
        ("rounds", ctypes.c_int64),
        ("tail_rounds", ctypes.c_int64),
        ("launches", ctypes.c_int64),
        ("dense_rounds", ctypes.c_int64),
        ("vertex_updates", ctypes.c_int64),
        ("edge_visits", ctypes.c_int64),
        ("changes", ctypes.c_int64),
        ("activations", ctypes.c_int64),
        ("prune_writes", ctypes.c_int64),
        ("full_scans", ctypes.c_int64),
        ("init_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("kernel", KernelStats * len(KERNELS)),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "kernel"}
        d["kernels"] = {k: self.kernel[i].as_dict() for i, k in enumerate(KERNELS)}
        return d


class RoundRecord(ctypes.Structure):
    """Mirror of ``kcore_round_record``."""
    _fields_ = [
        ("round", ctypes.c_int32),
        ("tail_rounds", ctypes.c_int32),
        ("vertex_updates", ctypes.c_int64),
        ("edge_visits", ctypes.c_int64),
        ("changes", ctypes.c_int64),
        ("activations", ctypes.c_int64),
        ("max_full_scan", ctypes.c_int64),
        ("ms", ctypes.c_double),
        ("big_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServeConfig(ctypes.Structure):
    """Mirror of ``kcore_serve_config`` (zero = library default)."""
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("max_queue", ctypes.c_int32),
        ("rounds_per_step", ctypes.c_int32),
        ("entries_per_vertex", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 5),
        ("tuning", Tuning),
    ]


class Completion(ctypes.Structure):
    """Mirror of ``kcore_completion``."""
    _fields_ = [
        ("req_id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("latency_us", ctypes.c_double),
        ("queue_us", ctypes.c_double),
    ]


class ServeReport(ctypes.Structure):
    """Mirror of ``kcore_serve_report``."""
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("cancelled", ctypes.c_int64),
        ("rejected", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("resident", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("bytes_budget", ctypes.c_int64),
        ("bytes_peak", ctypes.c_int64),
        ("p50_us", ctypes.c_double),
        ("p99_us", ctypes.c_double),
        ("max_us", ctypes.c_double),
        ("mean_us", ctypes.c_double),
        ("graphs_per_s", ctypes.c_double),
        ("rebases", ctypes.c_int64),
        ("reserved", ctypes.c_int64 * 3),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libkcore.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libkcore.so not built at {_LIB_PATH}; run python -m paper_2512_00233_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.kcore_decompose.restype = i32
    lib.kcore_decompose.argtypes = [i64, vp, vp, vp, vp]
    lib.kcore_decompose32.restype = i32
    lib.kcore_decompose32.argtypes = [i64, vp, vp, vp, vp]
    lib.kcore_decompose32_ex.restype = i32
    lib.kcore_decompose32_ex.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Tuning), ctypes.POINTER(Stats), vp]
    lib.kcore_decompose_ex.restype = i32
    lib.kcore_decompose_ex.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Tuning), ctypes.POINTER(Stats), vp]
    lib.kcore_decompose_noalloc.restype = i32
    lib.kcore_decompose_noalloc.argtypes = [i64, vp, vp, vp, vp]
    for name in ("kcore_certify", "kcore_certify32"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [i64, vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i64), vp]
    for name in ("kcore_update", "kcore_update32"):
        getattr(lib, name).restype = i32
        getattr(lib, name).argtypes = [i64, vp, vp, vp, i64, vp, i64, vp, vp, ctypes.POINTER(Tuning),
                                       ctypes.POINTER(Stats), vp]
    lib.kcore_decompose_rounds.restype = i32
    lib.kcore_decompose_rounds.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Tuning), ctypes.POINTER(RoundRecord), i32,
                                           ctypes.POINTER(i32), vp]
    lib.kcore_decompose_batch.restype = i32
    lib.kcore_decompose_batch.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(Tuning), ctypes.POINTER(Stats), vp]
    lib.kcore_autotune_batch.restype = i32
    lib.kcore_autotune_batch.argtypes = [i32, vp, vp, vp, vp, i32, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_float), vp]
    lib.kcore_tuning_cache_set.restype = i32
    lib.kcore_tuning_cache_set.argtypes = [i32, i64, i64, ctypes.POINTER(Tuning)]
    lib.kcore_tuning_cache_get.restype = i32
    lib.kcore_tuning_cache_get.argtypes = [i32, i64, i64, ctypes.POINTER(Tuning)]
    lib.kcore_last_error.restype = ctypes.c_char_p
    lib.kcore_last_error.argtypes = []
    lib.kcore_version.restype = ctypes.c_char_p
    lib.kcore_version.argtypes = []
    lib.kcore_release_workspace.restype = i32
    lib.kcore_release_workspace.argtypes = []
    lib.kcore_serve_create.restype = i32
    lib.kcore_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
    lib.kcore_serve_submit.restype = i32
    lib.kcore_serve_submit.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.kcore_serve_poll.restype = i32
    lib.kcore_serve_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)]
    lib.kcore_serve_wait.restype = i32
    lib.kcore_serve_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(Completion)]
    lib.kcore_serve_stats.restype = i32
    lib.kcore_serve_stats.argtypes = [vp, ctypes.POINTER(ServeReport)]
    lib.kcore_serve_destroy.restype = i32
    lib.kcore_serve_destroy.argtypes = [vp]
    lib.kcore_probe_gather.restype = i32
    lib.kcore_probe_gather.argtypes = [vp, i64, vp, i64, vp, vp]
    _lib = lib
    return lib


def version() -> str:
    return load().kcore_version().decode()


def _check(status: int):
    if status != 0:
        raise KcoreError(status, load().kcore_last_error().decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def decompose(row_ptr, col_idx, out=None, tuning: Tuning | None = None, stats: Stats | None = None,
              stream=None):
    """Coreness of every vertex of an undirected graph given as a symmetric CSR.

    row_ptr: int64 (or int32) CUDA tensor [n+1]; col_idx: int32 CUDA tensor [nnz].
    Returns ``out`` (int32 CUDA tensor [n], allocated when None).  The call
    returns once the result is final.  ``stats``, if given, is filled in.
    """
    import torch
    lib = load()
    if not (row_ptr.is_cuda and col_idx.is_cuda):
        raise ValueError("row_ptr and col_idx must be CUDA tensors")
    if col_idx.dtype != torch.int32:
        raise TypeError("col_idx must be int32")
    if row_ptr.dtype not in (torch.int64, torch.int32):
        raise TypeError("row_ptr must be int64 or int32")
    if not (row_ptr.is_contiguous() and col_idx.is_contiguous()):
        raise ValueError("row_ptr and col_idx must be contiguous")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must have at least one element")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    elif out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous int32 CUDA tensor of n elements")
    col_ptr = col_idx.data_ptr() if col_idx.numel() else out.data_ptr()  # any valid pointer when nnz == 0
    st = _stream_handle(stream)
    if row_ptr.dtype == torch.int32:
        if tuning is None and stats is None:
            _check(lib.kcore_decompose32(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(), st))
        else:
            _check(lib.kcore_decompose32_ex(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(),
                                            ctypes.byref(tuning) if tuning is not None else None,
                                            ctypes.byref(stats) if stats is not None else None, st))
    elif tuning is None and stats is None:
        _check(lib.kcore_decompose(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(), st))
    else:
        _check(lib.kcore_decompose_ex(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(),
                                      ctypes.byref(tuning) if tuning is not None else None,
                                      ctypes.byref(stats) if stats is not None else None, st))
    return out


def decompose_noalloc(row_ptr, col_idx, out, stream=None):
    """``kcore_decompose_noalloc``: like ``decompose`` (int64 row offsets, default tuning) into a caller-given
    ``out``, with the library allocating nothing (its workspace is a fixed device array)."""
    import torch
    lib = load()
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32 or not (row_ptr.is_cuda and col_idx.is_cuda):
        raise TypeError("row_ptr must be an int64 and col_idx an int32 CUDA tensor")
    n = row_ptr.numel() - 1
    if out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous int32 CUDA tensor of n elements")
    col_ptr = col_idx.data_ptr() if col_idx.numel() else out.data_ptr()
    _check(lib.kcore_decompose_noalloc(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(), _stream_handle(stream)))
    return out


CERTIFY_MESSAGES = {
    0: "ok",
    1: "core outside [0, degree]",
    2: "isolated vertex with a nonzero core, or a vertex with neighbours and core 0",
    3: "fewer than core(v) neighbours with core >= core(v)",
    4: "kmax(kmax+1)/2 exceeds the number of edges",
}


def certify(row_ptr, col_idx, core, stream=None):
    """``kcore_certify`` (``kcore_certify32`` for int32 row offsets): (code, vertex) of the local certificate of
    ``core`` on the device; code 0 = passes."""
    import torch
    lib = load()
    if row_ptr.dtype not in (torch.int64, torch.int32) or col_idx.dtype != torch.int32 or not (
            row_ptr.is_cuda and col_idx.is_cuda):
        raise TypeError("row_ptr must be an int64 or int32 and col_idx an int32 CUDA tensor")
    n = row_ptr.numel() - 1
    if core.dtype != torch.int32 or core.numel() != n or not core.is_cuda or not core.is_contiguous():
        raise ValueError("core must be a contiguous int32 CUDA tensor of n elements")
    code, vertex = ctypes.c_int32(), ctypes.c_int64()
    col_ptr = col_idx.data_ptr() if col_idx.numel() else core.data_ptr()
    fn = lib.kcore_certify if row_ptr.dtype == torch.int64 else lib.kcore_certify32
    _check(fn(n, row_ptr.data_ptr(), col_ptr, core.data_ptr(), ctypes.byref(code), ctypes.byref(vertex),
              _stream_handle(stream)))
    return int(code.value), int(vertex.value)


def update(row_ptr, col_idx, prev_core, removed=None, inserted=None, out=None, tuning: Tuning | None = None,
           stats: Stats | None = None, stream=None):
    """Coreness after edge changes (``kcore_update``).

    row_ptr / col_idx: the graph after the changes (int64 or int32 / int32 CUDA tensors; int32 offsets call
    ``kcore_update32``); prev_core: int32 CUDA tensor [n], the coreness before; removed / inserted: int32 CUDA
    tensors of shape [k, 2] (or None), the edges taken out and put in.  ``out`` may be ``prev_core`` itself.
    Returns ``out``.
    """
    import torch
    lib = load()
    if row_ptr.dtype not in (torch.int64, torch.int32) or col_idx.dtype != torch.int32 or not (
            row_ptr.is_cuda and col_idx.is_cuda):
        raise TypeError("row_ptr must be an int64 or int32 and col_idx an int32 CUDA tensor")
    n = row_ptr.numel() - 1
    if prev_core.dtype != torch.int32 or prev_core.numel() != n or not prev_core.is_cuda or not prev_core.is_contiguous():
        raise ValueError("prev_core must be a contiguous int32 CUDA tensor of n elements")
    edges = []
    for e, name in ((removed, "removed"), (inserted, "inserted")):
        if e is None or e.numel() == 0:
            edges.append((0, None))
            continue
        if e.dtype != torch.int32 or not e.is_cuda or not e.is_contiguous() or e.dim() != 2 or e.shape[1] != 2:
            raise ValueError(f"{name} must be a contiguous int32 CUDA tensor of shape [k, 2]")
        edges.append((e.shape[0], e.data_ptr()))
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    elif out.dtype != torch.int32 or out.numel() != n or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must be a contiguous int32 CUDA tensor of n elements")
    col_ptr = col_idx.data_ptr() if col_idx.numel() else out.data_ptr()
    fn = lib.kcore_update if row_ptr.dtype == torch.int64 else lib.kcore_update32
    _check(fn(n, row_ptr.data_ptr(), col_ptr, prev_core.data_ptr(), edges[0][0], edges[0][1], edges[1][0],
              edges[1][1], out.data_ptr(), ctypes.byref(tuning) if tuning is not None else None,
              ctypes.byref(stats) if stats is not None else None, _stream_handle(stream)))
    return out


def decompose_rounds(row_ptr, col_idx, out=None, tuning: Tuning | None = None, max_records: int = 1 << 16,
                     stream=None):
    """``decompose`` launching one round at a time; returns (out, list of per-round records)."""
    import torch
    lib = load()
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32 or not (row_ptr.is_cuda and col_idx.is_cuda):
        raise TypeError("row_ptr must be an int64 and col_idx an int32 CUDA tensor")
    n = row_ptr.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    recs = (RoundRecord * max_records)()
    got = ctypes.c_int32()
    col_ptr = col_idx.data_ptr() if col_idx.numel() else out.data_ptr()
    _check(lib.kcore_decompose_rounds(n, row_ptr.data_ptr(), col_ptr, out.data_ptr(),
                                      ctypes.byref(tuning) if tuning is not None else None, recs, max_records,
                                      ctypes.byref(got), _stream_handle(stream)))
    return out, [recs[i].as_dict() for i in range(got.value)]


def probe_gather(idx, vals, out_sum, stream=None):
    """Enqueue one pass of sum(vals[idx[j]]) into out_sum (int64 CUDA tensor of one element): the bare
    gather pattern of the neighbour scan, for measuring the device's random-gather rate (asynchronous)."""
    import torch
    for t, name in ((idx, "idx"), (vals, "vals")):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous int32 CUDA tensor")
    if not out_sum.is_cuda or out_sum.dtype != torch.int64 or out_sum.numel() != 1:
        raise ValueError("out_sum must be an int64 CUDA tensor of one element")
    m = idx.numel()
    _check(load().kcore_probe_gather(idx.data_ptr() if m else None, m, vals.data_ptr() if vals.numel() else None,
                                     vals.numel(), out_sum.data_ptr(), _stream_handle(stream)))


def _check_batch(graph_vtx_off, row_ptr, col_idx):
    import torch
    for t, name in ((graph_vtx_off, "graph_vtx_off"), (row_ptr, "row_ptr")):
        if not t.is_cuda or t.dtype != torch.int64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous int64 CUDA tensor")
    if not col_idx.is_cuda or col_idx.dtype != torch.int32 or not col_idx.is_contiguous():
        raise ValueError("col_idx must be a contiguous int32 CUDA tensor")
    return graph_vtx_off.numel() - 1, row_ptr.numel() - 1


def decompose_batch(graph_vtx_off, row_ptr, col_idx, out=None, tuning: Tuning | None = None,
                    stats: Stats | None = None, stream=None):
    """Coreness of many graphs at once (concatenated CSR, graph-local neighbour ids).

    graph_vtx_off: int64 CUDA tensor [G+1]; row_ptr: int64 [N+1] (global offsets);
    col_idx: int32 (local ids).  Returns out (int32 [N]).  With tuning None the
    autotuner's cached choice for this batch shape is used when there is one.
    """
    import torch
    lib = load()
    G, N = _check_batch(graph_vtx_off, row_ptr, col_idx)
    if out is None:
        out = torch.empty(N, dtype=torch.int32, device=row_ptr.device)
    col_ptr = col_idx.data_ptr() if col_idx.numel() else out.data_ptr()
    _check(lib.kcore_decompose_batch(G, graph_vtx_off.data_ptr(), row_ptr.data_ptr(), col_ptr, out.data_ptr(),
                                     ctypes.byref(tuning) if tuning is not None else None,
                                     ctypes.byref(stats) if stats is not None else None, _stream_handle(stream)))
    return out


def autotune_batch(graph_vtx_off, row_ptr, col_idx, out=None, reps: int = 3, stream=None):
    """Pick launch knobs for this batch shape by timing candidates; returns (Tuning, ms)."""
    import torch
    lib = load()
    G, N = _check_batch(graph_vtx_off, row_ptr, col_idx)
    if out is None:
        out = torch.empty(N, dtype=torch.int32, device=row_ptr.device)
    best, ms = Tuning(), ctypes.c_float()
    _check(lib.kcore_autotune_batch(G, graph_vtx_off.data_ptr(), row_ptr.data_ptr(), col_idx.data_ptr(),
                                    out.data_ptr(), reps, ctypes.byref(best), ctypes.byref(ms),
                                    _stream_handle(stream)))
    return best, float(ms.value)


def tuning_cache_set(num_graphs: int, total_vertices: int, total_entries: int, tuning: Tuning):
    _check(load().kcore_tuning_cache_set(num_graphs, total_vertices, total_entries, ctypes.byref(tuning)))


def tuning_cache_get(num_graphs: int, total_vertices: int, total_entries: int):
    t = Tuning()
    st = load().kcore_tuning_cache_get(num_graphs, total_vertices, total_entries, ctypes.byref(t))
    return t if st == 0 else None


def _host_ptr(x, dtype_name: str, name: str):
    """Address of a contiguous host array (numpy array or CPU torch tensor) of the given dtype."""
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):
        if x.is_cuda or str(x.dtype) != f"torch.{dtype_name}" or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous host {dtype_name} tensor")
        return x.data_ptr(), x.numel()
    import numpy as np
    if not isinstance(x, np.ndarray) or x.dtype != np.dtype(dtype_name) or not x.flags.c_contiguous:
        raise ValueError(f"{name} must be a C-contiguous numpy {dtype_name} array")
    return x.ctypes.data, x.size


class Server:
    """Continuous-batching decomposition server (``kcore_serve_*``).

    Graphs are submitted from host memory (numpy arrays or CPU torch tensors,
    pinned ones let copies overlap); results land in the caller's ``out``
    array.  The arrays are kept referenced here until the request's completion
    has been delivered by :meth:`poll` or :meth:`wait`.
    """

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, max_queue: int = 0, rounds_per_step: int = 0,
                 entries_per_vertex: int = 0, device: int = 0, tuning: Tuning | None = None):
        lib = load()
        cfg = ServeConfig(hbm_budget_bytes=hbm_budget_bytes, max_slots=max_slots, max_queue=max_queue,
                          rounds_per_step=rounds_per_step, entries_per_vertex=entries_per_vertex, device=device)
        if tuning is not None:
            cfg.tuning = tuning
        h = ctypes.c_void_p()
        _check(lib.kcore_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, row_ptr, col_idx, out) -> int:
        """Queue one graph (int64 row_ptr[n+1], int32 col_idx, int32 out[n]); returns the request id."""
        if self._h is None:
            raise RuntimeError("server closed")
        rp, nrp = _host_ptr(row_ptr, "int64", "row_ptr")
        ci, _ = _host_ptr(col_idx, "int32", "col_idx")
        op, nout = _host_ptr(out, "int32", "out")
        n = nrp - 1
        if n < 0 or nout != n:
            raise ValueError("row_ptr must have n+1 entries and out n entries")
        rid = ctypes.c_uint64()
        _check(load().kcore_serve_submit(self._h, n, rp, ci, op, ctypes.byref(rid)))
        self._keep[rid.value] = (row_ptr, col_idx, out)
        return rid.value

    def poll(self, max_items: int = 256) -> list:
        """Completions delivered since the last call (non-blocking)."""
        buf = (Completion * max_items)()
        got = ctypes.c_int32()
        _check(load().kcore_serve_poll(self._h, buf, max_items, ctypes.byref(got)))
        res = [buf[i] for i in range(got.value)]
        for c in res:
            self._keep.pop(c.req_id, None)
        return res

    def wait(self, req_id: int, timeout_s: float | None = None) -> Completion:
        """Block until req_id completes; raises KcoreError (KCORE_E_TIMEOUT) when the time runs out."""
        c = Completion()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        _check(load().kcore_serve_wait(self._h, req_id, us, ctypes.byref(c)))
        self._keep.pop(c.req_id, None)
        return c

    def stats(self) -> dict:
        r = ServeReport()
        _check(load().kcore_serve_stats(self._h, ctypes.byref(r)))
        return r.as_dict()

    def close(self):
        if self._h is not None:
            _check(load().kcore_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
