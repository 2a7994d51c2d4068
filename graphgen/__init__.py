"""Seeded synthetic graph inputs (CSR) shared by the CPU oracle and the GPU path.

Holds no coreness arithmetic: generators, the edge-list -> CSR builder and a
precondition validator only.  Every graph is a symmetric, loop-free,
duplicate-free CSR with rows sorted ascending: ``row_ptr`` int64 [n+1] and
``col_idx`` int32 [nnz].

The workloads stand in for the SNAP road / web / social graphs the paper
measures on (its Table I), which are not available here:

* ``er_small``   G(n=10,000, m=50,000), seed 1.
* ``road``       4096 x 4096 lattice, each lattice edge kept with p=0.6, each
                 vertex with probability 0.01 gets a chord to a vertex at
                 Manhattan distance 1..8, seed 2.
* ``rmat24``     R-MAT scale 24, edge factor 16 read as 16 directed entries per
                 vertex before deduplication (8 * 2^24 undirected samples),
                 (0.57, 0.19, 0.19, 0.05),
                 5% per-level noise, seeded relabel, seed 3.
* ``batch``      2048 graphs, n log-uniform in [1e3, 1e6], ER / Chung-Lu /
                 lattice, seed 4.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with g++ (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", _LIB_PATH + ".tmp",
               os.path.join(_HERE, "gen.cpp")]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, u64, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "gg_rand": (u64, [u64, u64, u64]),
        "gg_er": (vp, [i64, i64, u64]),
        "gg_lattice": (vp, [i64, i64, dbl, dbl, i32, u64]),
        "gg_rmat": (vp, [i32, i64, dbl, dbl, dbl, dbl, dbl, i32, u64]),
        "gg_chung_lu": (vp, [i64, dbl, dbl, u64]),
        "gg_from_edges": (vp, [i64, i64, vp, vp]),
        "gg_n": (i64, [vp]),
        "gg_nnz": (i64, [vp]),
        "gg_row_ptr": (vp, [vp]),
        "gg_col": (vp, [vp]),
        "gg_free": (None, [vp]),
        "gg_batch_spec": (None, [u64, i64, i64, i64, i32, vp, vp]),
        "gg_batch": (vp, [u64, i64, i32, i64, i64, i32]),
        "gg_batch_count": (i32, [vp]),
        "gg_batch_total_n": (i64, [vp]),
        "gg_batch_total_nnz": (i64, [vp]),
        "gg_batch_graph_vtx_off": (vp, [vp]),
        "gg_batch_row_ptr": (vp, [vp]),
        "gg_batch_col": (vp, [vp]),
        "gg_batch_kind": (vp, [vp]),
        "gg_batch_free": (None, [vp]),
        "gg_validate": (i32, [i64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _arr(ptr, count, dtype):
    if count == 0:
        return np.zeros(0, dtype=dtype)
    ctype = {np.int64: ctypes.c_int64, np.int32: ctypes.c_int32}[dtype]
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(count,)).copy()


@dataclass
class Graph:
    """Undirected graph as a symmetric CSR."""
    row_ptr: np.ndarray  # int64 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(h) -> Graph:
    lib = _load()
    n, nnz = lib.gg_n(h), lib.gg_nnz(h)
    g = Graph(_arr(lib.gg_row_ptr(h), n + 1, np.int64), _arr(lib.gg_col(h), nnz, np.int32))
    lib.gg_free(h)
    return g


def rand(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_rand(seed, stream, i))


def from_edges(n: int, src, dst) -> Graph:
    """Undirected edge list (loops and duplicates allowed) -> clean symmetric CSR."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    if src.size:
        assert src.min() >= 0 and dst.min() >= 0 and max(src.max(), dst.max()) < n
    h = _load().gg_from_edges(n, src.size, src.ctypes.data, dst.ctypes.data)
    return _take(h)


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    g = _take(_load().gg_er(n, m, seed))
    g.name, g.params = "er", dict(n=n, m=m, seed=seed)
    return g


def lattice(rows: int, cols: int, p: float = 0.6, chord_prob: float = 0.01, maxdist: int = 8,
            seed: int = 2) -> Graph:
    g = _take(_load().gg_lattice(rows, cols, p, chord_prob, maxdist, seed))
    g.name, g.params = "lattice", dict(rows=rows, cols=cols, p=p, chord_prob=chord_prob, maxdist=maxdist,
                                       seed=seed)
    return g


def rmat(scale: int, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05), noise: float = 0.05,
         relabel: bool = True, seed: int = 3) -> Graph:
    """R-MAT with ``edge_factor`` directed CSR entries per vertex before deduplication,
    i.e. ``edge_factor * 2^scale / 2`` undirected samples (each sample yields two entries)."""
    samples = (edge_factor << scale) // 2
    g = _take(_load().gg_rmat(scale, samples, *abcd, noise, int(relabel), seed))
    g.name, g.params = "rmat", dict(scale=scale, edge_factor=edge_factor, abcd=list(abcd), noise=noise,
                                    relabel=relabel, seed=seed)
    return g


def chung_lu(n: int, gamma: float, avg_deg: float, seed: int) -> Graph:
    g = _take(_load().gg_chung_lu(n, gamma, avg_deg, seed))
    g.name, g.params = "chung_lu", dict(n=n, gamma=gamma, avg_deg=avg_deg, seed=seed)
    return g


def validate(g: Graph) -> int:
    """0 if the CSR meets the preconditions, else the generator library's error code."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    return int(_load().gg_validate(g.n, rp.ctypes.data, ci.ctypes.data))


KIND_NAMES = ("er", "chung_lu", "lattice")


@dataclass
class Batch:
    """Concatenated CSR of several graphs with graph-local neighbour ids."""
    graph_vtx_off: np.ndarray  # int64 [G+1]
    row_ptr: np.ndarray        # int64 [N+1], global edge offsets
    col_idx: np.ndarray        # int32 [NNZ], graph-local ids
    kind: np.ndarray           # int32 [G]

    @property
    def num_graphs(self) -> int:
        return int(self.graph_vtx_off.shape[0] - 1)

    def graph(self, g: int) -> Graph:
        v0, v1 = int(self.graph_vtx_off[g]), int(self.graph_vtx_off[g + 1])
        e0, e1 = int(self.row_ptr[v0]), int(self.row_ptr[v1])
        return Graph(self.row_ptr[v0:v1 + 1] - e0, self.col_idx[e0:e1], KIND_NAMES[int(self.kind[g])])


def batch_spec(seed: int, g: int, nmin: int = 1000, nmax: int = 1_000_000, kinds_mask: int = 7):
    kind, n = ctypes.c_int32(), ctypes.c_int64()
    _load().gg_batch_spec(seed, g, nmin, nmax, kinds_mask, ctypes.byref(kind), ctypes.byref(n))
    return int(kind.value), int(n.value)


def batch(num_graphs: int, seed: int = 4, nmin: int = 1000, nmax: int = 1_000_000, kinds_mask: int = 7,
          first: int = 0) -> Batch:
    lib = _load()
    h = lib.gg_batch(seed, first, num_graphs, nmin, nmax, kinds_mask)
    G, N, NNZ = lib.gg_batch_count(h), lib.gg_batch_total_n(h), lib.gg_batch_total_nnz(h)
    b = Batch(_arr(lib.gg_batch_graph_vtx_off(h), G + 1, np.int64), _arr(lib.gg_batch_row_ptr(h), N + 1, np.int64),
              _arr(lib.gg_batch_col(h), NNZ, np.int32), _arr(lib.gg_batch_kind(h), G, np.int32))
    lib.gg_batch_free(h)
    return b


def concat(graphs) -> Batch:
    """Concatenate graphs into the batched layout."""
    G = len(graphs)
    vo = np.zeros(G + 1, np.int64)
    for i, g in enumerate(graphs):
        vo[i + 1] = vo[i] + g.n
    rows, cols, eo = [], [], 0
    for g in graphs:
        rows.append(g.row_ptr[:-1] + eo)
        cols.append(g.col_idx)
        eo += g.nnz
    rows.append(np.array([eo], np.int64))
    kinds = np.array([KIND_NAMES.index(g.name) if g.name in KIND_NAMES else 0 for g in graphs], np.int32)
    return Batch(vo, np.concatenate(rows).astype(np.int64),
                 np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32), kinds)


# ------------------------------------------------------------------ named workloads
WORKLOADS = {
    "er_small": dict(fn="erdos_renyi", kw=dict(n=10_000, m=50_000, seed=1)),
    "road": dict(fn="lattice", kw=dict(rows=4096, cols=4096, p=0.6, chord_prob=0.01, maxdist=8, seed=2)),
    "rmat24": dict(fn="rmat", kw=dict(scale=24, edge_factor=16, noise=0.05, relabel=True, seed=3)),
    # the same samples without the random relabel (R-MAT's own id order: low ids carry the high degrees)
    "rmat24_unpermuted": dict(fn="rmat", kw=dict(scale=24, edge_factor=16, noise=0.05, relabel=False, seed=3)),
    # scaled-down stand-ins of the same shapes, for fast tests
    "road_512": dict(fn="lattice", kw=dict(rows=512, cols=512, p=0.6, chord_prob=0.01, maxdist=8, seed=2)),
    "rmat16": dict(fn="rmat", kw=dict(scale=16, edge_factor=16, noise=0.05, relabel=True, seed=3)),
    "rmat20": dict(fn="rmat", kw=dict(scale=20, edge_factor=16, noise=0.05, relabel=True, seed=3)),
}


def cache_dir() -> str:
    d = os.environ.get("KCORE_GRAPH_CACHE") or os.path.join("/tmp", "kcore_graph_cache")
    os.makedirs(d, exist_ok=True)
    return d


def workload(name: str, cache: bool = True) -> Graph:
    """Generate (or load from the on-disk cache) a named workload."""
    spec = WORKLOADS[name]
    key = hashlib.sha1(repr((name, spec, "v2")).encode()).hexdigest()[:16]
    base = os.path.join(cache_dir(), f"{name}_{key}")
    if cache and os.path.exists(base + "_col.npy"):
        g = Graph(np.load(base + "_row.npy"), np.load(base + "_col.npy"), name, spec["kw"])
        return g
    g = globals()[spec["fn"]](**spec["kw"])
    g.name = name
    if cache:
        np.save(base + "_row.npy", g.row_ptr)
        np.save(base + "_col.npy", g.col_idx)
    return g
