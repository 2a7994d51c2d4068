"""CPU oracle for k-core decomposition -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package.  It shares no code with the GPU library
(``paper_2512_00233_amd``) and never imports it.

What it computes is the paper's Definition 1 (Sec. II) and the coreness
defined right after it: the k-core is the inclusion-maximal vertex set whose
induced subgraph has minimum degree >= k; coreness(v) is the largest such k
containing v, 0 for isolated vertices.  The iterative method (Sec. II-B,
Alg. 1; FastK in Sec. IV) is exact, not an approximation (Sec. V-C states it is
neither approximate nor heuristic), so the oracle is the definition:

* :func:`coreness`       the definition written out in C (level-by-level
                         repeated deletion of vertices with < k remaining
                         neighbours); the primary oracle.
* :func:`coreness_bz`    Batagelj-Zaversnik bucket peeling in C, the linear
                         sequential algorithm the paper cites (Sec. II); an
                         independent second implementation.
* :func:`brute_force`    pure Python, tiny graphs only: every k-core recomputed
                         from scratch by repeated pruning of the whole graph.
* :func:`check`          the local certificate (core <= deg, isolated <=> 0,
                         local support, kmax(kmax+1)/2 <= m).

Pins (see ``tests/test_oracle.py``): brute force on every labelled graph with
<= 6 vertices and on random graphs, closed forms derived from Definition 1,
agreement of the two C routines at full workload sizes, the certificate, and the
installed NetworkX ``core_number`` (the paper's own correctness baseline,
Sec. V-A) on medium graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O3)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O3", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-shared", "-fPIC", "-pthread",
               "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "kcore_oracle.c")]
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
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    for name in ("oracle_core_levels", "oracle_core_bz"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [i64, vp, vp, vp]
    lib.oracle_check.restype = ctypes.c_int
    lib.oracle_check.argtypes = [i64, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_core_batch.restype = ctypes.c_int
    lib.oracle_core_batch.argtypes = [i32, vp, vp, vp, vp, i32, i32]
    _lib = lib
    return lib


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)  # valid pointer for empty edge sets
    return rp, ci


def coreness(row_ptr, col_idx) -> np.ndarray:
    """Coreness of every vertex by the definition (primary oracle)."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.shape[0] - 1
    out = np.zeros(max(n, 0), np.int32)
    if n > 0 and _load().oracle_core_levels(n, rp.ctypes.data, ci.ctypes.data, out.ctypes.data) != 0:
        raise MemoryError("oracle_core_levels: allocation failed")
    return out


def coreness_bz(row_ptr, col_idx) -> np.ndarray:
    """Coreness of every vertex by Batagelj-Zaversnik peeling."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.shape[0] - 1
    out = np.zeros(max(n, 0), np.int32)
    if n > 0 and _load().oracle_core_bz(n, rp.ctypes.data, ci.ctypes.data, out.ctypes.data) != 0:
        raise MemoryError("oracle_core_bz: allocation failed")
    return out


def coreness_batch(graph_vtx_off, row_ptr, col_idx, method: str = "levels", threads: int = 0) -> np.ndarray:
    """Per-graph coreness of a concatenated batch (graph-local ids), graphs spread over threads."""
    vo = np.ascontiguousarray(graph_vtx_off, dtype=np.int64)
    rp, ci = _csr(row_ptr, col_idx)
    G = vo.shape[0] - 1
    out = np.zeros(int(vo[-1]) if G > 0 else 0, np.int32)
    threads = threads or os.cpu_count() or 1
    r = _load().oracle_core_batch(G, vo.ctypes.data, rp.ctypes.data, ci.ctypes.data, out.ctypes.data,
                                  0 if method == "levels" else 1, threads)
    if r != 0:
        raise MemoryError("oracle_core_batch: allocation failed")
    return out


CHECK_MESSAGES = {
    0: "ok",
    1: "core outside [0, deg]",
    2: "isolated vertex with core != 0, or non-isolated vertex with core 0",
    3: "local support violated: fewer than core(v) neighbours with core >= core(v)",
    4: "kmax(kmax+1)/2 exceeds the number of edges",
}


def check(row_ptr, col_idx, core):
    """Local certificate of a claimed coreness vector. Returns (code, first_bad_vertex)."""
    rp, ci = _csr(row_ptr, col_idx)
    c = np.ascontiguousarray(core, dtype=np.int32)
    n = rp.shape[0] - 1
    assert c.shape[0] == n
    bad = ctypes.c_int64(-1)
    code = _load().oracle_check(n, rp.ctypes.data, ci.ctypes.data, c.ctypes.data, ctypes.byref(bad))
    return int(code), int(bad.value)


def brute_force(n: int, edges) -> list:
    """Coreness from Definition 1 by brute force (tiny graphs only).

    For each k = 1, 2, ... the k-core is recomputed from the WHOLE graph by
    deleting vertices with fewer than k surviving neighbours until none is
    left; a vertex's coreness is the largest k for which it survives.
    """
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    core = [0] * n
    k = 1
    while True:
        alive = set(range(n))
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if len(adj[v] & alive) < k:
                    alive.discard(v)
                    changed = True
        if not alive:
            return core
        for v in alive:
            core[v] = k
        k += 1
