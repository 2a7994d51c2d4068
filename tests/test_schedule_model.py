"""The activation rules of the round kernels, checked on the host: under many
random interleavings of reads, writes and atomics the schedule model reaches
the oracle's coreness, and each deliberate mistake in the rules is caught."""
import random

import numpy as np
import pytest

import oracle
from tests.schedule_model import random_graph, run_model


def graphs(count, seed):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        n, adj = random_graph(rng)
        rp = np.zeros(n + 1, np.int64)
        for u in range(n):
            rp[u + 1] = rp[u] + len(adj[u])
        ci = np.array([v for a in adj for v in a], np.int32)
        out.append((n, adj, oracle.coreness(rp, ci).tolist()))
    return out


CASES = graphs(1500, seed=11)


@pytest.mark.parametrize("big_first,defer", [(True, True), (False, True), (True, False)])
def test_model_reaches_the_coreness_under_random_schedules(big_first, defer):
    rng = random.Random(5)
    for n, adj, ref in CASES:
        for big_deg in (rng.randint(1, 8), 1 << 30):
            got, _ = run_model(n, adj, rng, big_deg, big_first=big_first, defer=defer)
            assert got == ref, (n, adj, big_deg)


def test_model_with_hubs_out_of_the_first_round():
    # class-3 vertices above a degree bound skip the first round's recomputation: still exact, and
    # forgetting to queue them for the second round is caught
    rng = random.Random(13)
    wrong = 0
    for n, adj, ref in CASES:
        big_deg = rng.randint(1, 6)
        delay = rng.randint(big_deg, 10)
        got, _ = run_model(n, adj, rng, big_deg, delay_deg=delay, defer=rng.random() < 0.7)
        assert got == ref, (n, adj, big_deg)
        bad, _ = run_model(n, adj, rng, big_deg, delay_deg=delay, rule="delay_unqueued")
        wrong += bad != ref
    assert wrong > 0


@pytest.mark.parametrize("rule", ["no_frontier_clause", "no_kernel_order", "skip_in_class3_kernel", "defer_strict_level"])
def test_model_catches_broken_rules(rule):
    rng = random.Random(7)
    wrong = 0
    for n, adj, ref in CASES:
        got, _ = run_model(n, adj, rng, rng.randint(1, 8), rule=rule)
        wrong += got != ref
    assert wrong > 0
