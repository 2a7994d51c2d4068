"""The update's start (bounds and frontier after edge changes) leads the round schedule to the
oracle's coreness of the changed graph; deliberately wrong starts are caught."""
import random

import numpy as np
import pytest

import oracle
from tests import schedule_model as sm
from tests import update_model as um


def csr(n, adj):
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(a) for a in adj])
    ci = np.array([v for a in adj for v in a], np.int32)
    return rp, ci


def random_change(rng, n, adj):
    """A random batch of removals and insertions; returns (new adjacency, removed, inserted)."""
    edges = {(u, v) for u in range(n) for v in adj[u] if u < v}
    non = [(u, v) for u in range(n) for v in range(u + 1, n) if (u, v) not in edges]
    k_rem = rng.randint(0, min(len(edges), 6))
    k_ins = rng.randint(0, min(len(non), 6))
    if k_rem + k_ins == 0:
        k_rem = min(1, len(edges))
    removed = rng.sample(sorted(edges), k_rem)
    inserted = rng.sample(non, k_ins)
    new = (edges - set(removed)) | set(inserted)
    nadj = [[] for _ in range(n)]
    for u, v in new:
        nadj[u].append(v)
        nadj[v].append(u)
    return [sorted(a) for a in nadj], removed, inserted


def run_cases(rule, cases, seed):
    rng = random.Random(seed)
    bad = 0
    for _ in range(cases):
        n, adj = sm.random_graph(rng, nmax=18)
        nadj, removed, inserted = random_change(rng, n, adj)
        prev = oracle.coreness(*csr(n, adj)).tolist()
        ref = oracle.coreness(*csr(n, nadj)).tolist()
        budget = rng.choice([None, None, 0, 1, 3])
        window_max = rng.choice([4, 4, 1, 0])  # 0: always the threshold rule
        est, frontier, slack = um.update_start(nadj, prev, removed, inserted, rule=rule, budget=budget,
                                               window_max=window_max)
        assert all(x >= c for x, c in zip(est, ref)) or rule != "gpu", "start is not an upper bound"
        got, _ = sm.run_model(n, nadj, rng, big_deg=rng.choice([3, 6, 100]), start=(est, frontier, slack),
                              defer=rng.random() < 0.5, big_first=rng.random() < 0.8)
        bad += got != ref
    return bad


def test_update_start_reaches_the_new_coreness():
    assert run_cases("gpu", 1500, seed=1) == 0


def star_change(rng, n, adj):
    """A vertex gets edges to several vertices it was not adjacent to (a vertex arriving, or growing)."""
    z = rng.randrange(n)
    non = [v for v in range(n) if v != z and v not in adj[z]]
    k = rng.randint(1, min(len(non), 7)) if non else 0
    inserted = [(min(z, v), max(z, v)) for v in rng.sample(non, k)]
    nadj = [list(a) for a in adj]
    for u, v in inserted:
        nadj[u].append(v)
        nadj[v].append(u)
    return [sorted(a) for a in nadj], [], inserted


def test_heavy_vertex_rule_on_vertex_arrivals():
    # insertions concentrated on one vertex: the heavy-vertex rule applies, the result is exact with searches
    # completed or given up, and its wrong forms are caught
    rng = random.Random(3)
    bad = {"z_no_neighbour_sources": 0, "z_rise_one": 0, "z_threshold_too_high": 0}
    used = 0
    for _ in range(1500):
        n, adj = sm.random_graph(rng, nmax=18)
        nadj, removed, inserted = star_change(rng, n, adj)
        if not inserted:
            continue
        prev = oracle.coreness(*csr(n, adj)).tolist()
        ref = oracle.coreness(*csr(n, nadj)).tolist()
        budget = rng.choice([None, 0, 1, 3])
        est, frontier, slack = um.update_start(nadj, prev, removed, inserted, budget=budget)
        assert all(x >= c for x, c in zip(est, ref))
        used += len(inserted) >= 2
        got, _ = sm.run_model(n, nadj, rng, big_deg=rng.choice([3, 6, 100]), start=(est, frontier, slack),
                              defer=rng.random() < 0.5)
        assert got == ref
        for rule in bad:
            e2, f2, s2 = um.update_start(nadj, prev, removed, inserted, rule=rule, budget=budget)
            g2, _ = sm.run_model(n, nadj, rng, big_deg=100, start=(e2, f2, s2))
            bad[rule] += g2 != ref
    assert used > 500
    assert all(v > 0 for v in bad.values()), bad


@pytest.mark.parametrize("rule", ["threshold_too_high", "rise_by_one", "cap_too_low", "no_removal_seed",
                                  "window_from_upper", "window_narrow", "final_with_removals", "endpoints_only",
                                  "clamp_to_degree", "no_neighbour_seed"])
def test_wrong_update_starts_are_caught(rule):
    assert run_cases(rule, 3000, seed=2) > 0, rule
