"""Pins for the CPU oracle against what the paper's definition and mathematics fix.

The oracle computes coreness as defined in the paper (Sec. II, Definition 1 and
the coreness paragraph).  It is pinned here by things other than itself:

* brute force from the definition on every labelled graph with <= 6 vertices
  and on random graphs with <= 40 vertices;
* closed forms derived from Definition 1 (cliques, cycles, trees, grids,
  complete bipartite and regular graphs, wheels, onions, unions);
* the local certificate and the maximality it cannot see on its own;
* the installed NetworkX ``core_number`` (the paper's own correctness baseline,
  Sec. V-A) on medium graphs;
* mutated copies of the level algorithm (a dropped term, a wrong comparison, an
  off-by-one) that the pins above must reject.
"""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import small_graphs as sg


def both(n, edges):
    rp, ci = sg.to_csr(n, edges)
    a = oracle.coreness(rp, ci)
    b = oracle.coreness_bz(rp, ci)
    return a, b, rp, ci


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_every_labelled_graph_up_to_6_vertices(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        a, b, rp, ci = both(n, edges)
        ref = oracle.brute_force(n, edges)
        assert a.tolist() == ref, (n, edges)
        assert b.tolist() == ref, (n, edges)


def test_random_graphs_up_to_40_vertices():
    rng = np.random.default_rng(12345)
    for t in range(1500):
        n = int(rng.integers(1, 41))
        p = float(rng.choice([0.05, 0.1, 0.2, 0.35, 0.6, 0.9]))
        n, edges = sg.random_graph(n, p, int(rng.integers(1 << 30)))
        a, b, rp, ci = both(n, edges)
        ref = oracle.brute_force(n, edges)
        assert a.tolist() == ref
        assert b.tolist() == ref
        assert oracle.check(rp, ci, a)[0] == 0


# ---------------------------------------------------------------- closed forms
def closed_form_cases():
    cases = []
    for n in [1, 2, 3, 5, 8, 17]:
        cases.append((f"K{n}", sg.complete(n), [n - 1] * n))
    for n in [3, 4, 7, 100]:
        cases.append((f"C{n}", sg.cycle(n), [2] * n))
    for n in [2, 3, 10, 101]:
        cases.append((f"P{n}", sg.path(n), [1] * n))
    for k in [1, 5, 64]:
        cases.append((f"star{k}", sg.star(k), [1] * (k + 1)))
    for seed in range(4):
        cases.append((f"tree{seed}", sg.random_tree(60, seed), [1] * 60))
    for a, b in [(2, 2), (2, 7), (3, 3), (5, 9), (12, 12)]:
        cases.append((f"grid{a}x{b}", sg.grid(a, b), [2] * (a * b)))
    for a, b in [(1, 4), (2, 5), (3, 3), (4, 7)]:
        cases.append((f"K{a},{b}", sg.complete_bipartite(a, b), [min(a, b)] * (a + b)))
    cases.append(("petersen", sg.petersen(), [3] * 10))
    for d in [1, 2, 3, 4, 5]:
        cases.append((f"Q{d}", sg.hypercube(d), [d] * (1 << d)))
    for rim in [3, 4, 9]:
        cases.append((f"wheel{rim}", sg.wheel(rim), [3] * (rim + 1)))
    for n in [3, 4, 6]:
        cases.append((f"K{n}+pendant", sg.complete_plus_pendant(n), [n - 1] * n + [1]))
    sizes = [6, 3, 9, 4, 5]  # the s-1 closed form needs s >= 3 (a 2-clique linked twice is 2-core)
    cases.append(("onion", sg.onion(sizes), sum(([s - 1] * s for s in sizes), [])))
    u = sg.disjoint_union(sg.complete(5), sg.cycle(6), sg.path(4), (3, []))
    cases.append(("union", u, [4] * 5 + [2] * 6 + [1] * 4 + [0] * 3))
    cases.append(("isolated", (7, []), [0] * 7))
    return cases


@pytest.mark.parametrize("name,graph,expect", closed_form_cases(), ids=[c[0] for c in closed_form_cases()])
def test_closed_forms(name, graph, expect):
    n, edges = graph
    a, b, rp, ci = both(n, edges)
    assert a.tolist() == expect
    assert b.tolist() == expect
    if n <= 40:
        assert oracle.brute_force(n, edges) == expect
    assert oracle.check(rp, ci, a)[0] == 0


# ---------------------------------------------------------------- certificate
def test_certificate_rejects_planted_errors():
    n, edges = sg.onion([5, 4, 3])
    rp, ci = sg.to_csr(n, edges)
    good = oracle.coreness(rp, ci)
    assert oracle.check(rp, ci, good) == (0, -1)
    up = good.copy()
    up[0] += 1  # above the true value: support fails
    assert oracle.check(rp, ci, up)[0] in (1, 3)
    over = good.copy()
    over[5] = 99  # above the degree
    assert oracle.check(rp, ci, over)[0] == 1
    zero = good.copy()
    zero[3] = 0  # non-isolated with core 0 (also starves its clique neighbours of support)
    assert oracle.check(rp, ci, zero)[0] in (2, 3)
    leaf = np.zeros(2, np.int32)  # a single edge claimed to be 0-core
    assert oracle.check(*sg.to_csr(2, [(0, 1)]), leaf)[0] == 2


def test_certificate_is_not_maximality():
    # K4 with every value 2 satisfies the local certificate but is not the coreness:
    # maximality needs the peeling oracle, which gives 3.
    n, edges = sg.complete(4)
    rp, ci = sg.to_csr(n, edges)
    assert oracle.check(rp, ci, np.full(4, 2, np.int32))[0] == 0
    assert oracle.coreness(rp, ci).tolist() == [3, 3, 3, 3]


# ---------------------------------------------------------------- networkx
def _nx_core(g):
    nx = pytest.importorskip("networkx")
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    m = src < g.col_idx
    G.add_edges_from(zip(src[m].tolist(), g.col_idx[m].tolist()))
    c = nx.core_number(G)
    return np.array([c[i] for i in range(g.n)], np.int32)


@pytest.mark.parametrize("make", [
    lambda: gg.workload("er_small"),
    lambda: gg.lattice(200, 200, seed=7),
    lambda: gg.rmat(13, seed=11),
    lambda: gg.chung_lu(20000, 2.3, 12, seed=5),
], ids=["er_small", "lattice200", "rmat13", "chung_lu"])
def test_networkx_core_number(make):
    g = make()
    ref = _nx_core(g)
    assert np.array_equal(oracle.coreness(g.row_ptr, g.col_idx), ref)
    assert np.array_equal(oracle.coreness_bz(g.row_ptr, g.col_idx), ref)


# ---------------------------------------------------------------- medium sizes
@pytest.mark.parametrize("name", ["road_512", "rmat16", "rmat20"])
def test_levels_equal_bz_and_certificate(name):
    g = gg.workload(name)
    a = oracle.coreness(g.row_ptr, g.col_idx)
    b = oracle.coreness_bz(g.row_ptr, g.col_idx)
    assert np.array_equal(a, b)
    assert oracle.check(g.row_ptr, g.col_idx, a) == (0, -1)


def test_batch_oracle_matches_per_graph():
    b = gg.batch(24, seed=4, nmin=100, nmax=20000)
    core = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=4)
    core_bz = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, method="bz", threads=3)
    assert np.array_equal(core, core_bz)
    for g in range(b.num_graphs):
        sub = b.graph(g)
        v0, v1 = b.graph_vtx_off[g], b.graph_vtx_off[g + 1]
        assert np.array_equal(core[v0:v1], oracle.coreness(sub.row_ptr, sub.col_idx))


# ---------------------------------------------------------------- pins have teeth
def _levels_mutant(n, edges, mutation):
    """The level algorithm in Python with one planted mistake."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    deg = [len(a) for a in adj]
    alive = [True] * n
    core = [0] * n
    remaining = list(range(n))
    k = 1
    while remaining:
        thr = k + 1 if mutation == "le_instead_of_lt" else k
        queue = [v for v in remaining if deg[v] < thr]
        queued = set(queue)
        while queue:
            v = queue.pop()
            alive[v] = False
            core[v] = k if mutation == "off_by_one" else k - 1
            for u in adj[v]:
                if not alive[u]:
                    continue
                if mutation != "no_decrement":
                    deg[u] -= 1
                if deg[u] < thr and u not in queued:
                    queue.append(u)
                    queued.add(u)
        remaining = [v for v in remaining if alive[v]]
        k += 1
    return core


@pytest.mark.parametrize("mutation", ["le_instead_of_lt", "off_by_one", "no_decrement"])
def test_pins_reject_mutated_oracles(mutation):
    caught = False
    for name, (n, edges), expect in closed_form_cases():
        if _levels_mutant(n, edges, mutation) != expect:
            caught = True
            break
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        if caught:
            break
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        if _levels_mutant(5, edges, mutation) != oracle.brute_force(5, edges):
            caught = True
    assert caught
    assert _levels_mutant(*sg.onion([4, 3]), "none") == [3] * 4 + [2] * 3


# ---------------------------------------------------------------- golden fixture
def test_golden_small_graphs():
    from tests.golden.load import small_graphs
    seen = 0
    for name, n, edges, core in small_graphs():
        rp, ci = sg.to_csr(n, edges)
        assert oracle.coreness(rp, ci).tolist() == core, name
        assert oracle.brute_force(n, edges) == core, name
        seen += 1
    assert seen >= 10
