"""Builders for small named graphs (edge lists only; no coreness arithmetic).

Each builder returns ``(n, edges)`` with ``edges`` a list of (u, v) pairs.
"""
import itertools

import numpy as np


def complete(n):
    return n, list(itertools.combinations(range(n), 2))


def cycle(n):
    return n, [(i, (i + 1) % n) for i in range(n)]


def path(n):
    return n, [(i, i + 1) for i in range(n - 1)]


def star(leaves):
    return leaves + 1, [(0, i) for i in range(1, leaves + 1)]


def grid(a, b):
    e = []
    for r in range(a):
        for c in range(b):
            v = r * b + c
            if c + 1 < b:
                e.append((v, v + 1))
            if r + 1 < a:
                e.append((v, v + b))
    return a * b, e


def complete_bipartite(a, b):
    return a + b, [(i, a + j) for i in range(a) for j in range(b)]


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return 10, outer + spokes + inner


def hypercube(d):
    n = 1 << d
    return n, [(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)]


def wheel(rim):
    n, e = cycle(rim)
    e = [(u + 1, v + 1) for u, v in e] + [(0, i) for i in range(1, rim + 1)]
    return rim + 1, e


def complete_plus_pendant(n):
    _, e = complete(n)
    return n + 1, e + [(0, n)]


def random_tree(n, seed):
    rng = np.random.default_rng(seed)
    return n, [(i, int(rng.integers(0, i))) for i in range(1, n)]


def disjoint_union(*graphs):
    off, edges = 0, []
    for n, e in graphs:
        edges += [(u + off, v + off) for u, v in e]
        off += n
    return off, edges


def onion(sizes):
    """Cliques K_s for s in sizes, consecutive cliques joined by one edge."""
    off, edges, firsts = 0, [], []
    for s in sizes:
        edges += [(u + off, v + off) for u, v in itertools.combinations(range(s), 2)]
        firsts.append(off)
        off += s
    for a, b in zip(firsts, firsts[1:]):
        edges.append((a, b))
    return off, edges


def random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    return n, [(u, v) for u, v in itertools.combinations(range(n), 2) if rng.random() < p]


def to_csr(n, edges):
    """Symmetric, sorted, deduplicated CSR from an edge list (pure numpy)."""
    if edges:
        a = np.array(edges, dtype=np.int64)
        a = a[a[:, 0] != a[:, 1]]
        both = np.concatenate([a, a[:, ::-1]])
        both = np.unique(both, axis=0)
    else:
        both = np.zeros((0, 2), np.int64)
    deg = np.bincount(both[:, 0], minlength=n) if both.size else np.zeros(n, np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr, both[:, 1].astype(np.int32)
