"""Served form (kcore_serve_*): every result equals the oracle and the same
graph decomposed alone, whether it ran alone or joined a running mix; admission
by device footprint, queue limits, timeouts and shutdown."""
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import small_graphs as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def kc():
    import paper_2512_00233_amd as kc
    return kc


def mix_graphs():
    """Graphs that exercise every degree class, the tail and long round chains."""
    graphs = []
    for n, edges in [sg.complete(7), (1, []), (5, []), sg.cycle(50), sg.star(5000), sg.complete(600),
                     sg.complete(2500), sg.path(3000), sg.onion([3, 40, 7, 300, 5]), sg.grid(40, 70)]:
        rp, ci = sg.to_csr(n, edges)
        graphs.append(gg.Graph(rp, ci))
    graphs.append(gg.chung_lu(60_000, 2.1, 16, seed=21))
    graphs.append(gg.erdos_renyi(20_000, 160_000, seed=22))
    graphs.append(gg.lattice(150, 150, seed=23))
    b = gg.batch(12, seed=24, nmin=1000, nmax=80_000)
    graphs += [b.graph(i) for i in range(b.num_graphs)]
    return graphs


def run_all(server, graphs, gaps_s=None):
    """Submit every graph (optionally with pauses between submissions) and collect the results."""
    outs, ids = [], []
    for i, g in enumerate(graphs):
        out = np.full(g.n, -7, np.int32)
        ids.append(server.submit(g.row_ptr, g.col_idx, out))
        outs.append(out)
        if gaps_s is not None:
            time.sleep(gaps_s[i])
    for rid in ids:
        c = server.wait(rid, timeout_s=60)
        assert c.status == 0, c.status
    return outs


def test_single_request_matches_oracle():
    g = gg.workload("er_small")
    with kc().Server(hbm_budget_bytes=256 << 20) as s:
        out = np.zeros(g.n, np.int32)
        rid = s.submit(g.row_ptr, g.col_idx, out)
        c = s.wait(rid, timeout_s=60)
        assert c.status == 0 and c.req_id == rid and c.latency_us > 0
    assert np.array_equal(out, oracle.coreness(g.row_ptr, g.col_idx))


@pytest.mark.parametrize("tuning", [dict(), dict(list_cap=1, tail_threshold=-1), dict(tail_threshold=1 << 30),
                                    dict(no_graph=1), dict(thread_max_deg=1, group_max_deg=1, wave_max_deg=1)])
def test_same_result_alone_and_in_the_mix(tuning):
    graphs = mix_graphs()
    refs = [oracle.coreness(g.row_ptr, g.col_idx) for g in graphs]
    t = kc().Tuning(**tuning)
    with kc().Server(hbm_budget_bytes=1 << 30, tuning=t, rounds_per_step=4) as s:
        # alone: one request in the server at a time
        alone = []
        for i, g in enumerate(graphs):
            print(f"[serve] alone {i} n={g.n} nnz={g.nnz} {tuning}", flush=True)
            alone += run_all(s, [g])
        # in the mix: all submitted, staggered so that graphs join rounds already running
        rng = np.random.default_rng(5)
        order = rng.permutation(len(graphs))
        print(f"[serve] mix {tuning}", flush=True)
        mixed = run_all(s, [graphs[i] for i in order], gaps_s=rng.exponential(0.0005, len(graphs)))
        st = s.stats()
    for j, i in enumerate(order):
        assert np.array_equal(alone[i], refs[i]), i
        assert np.array_equal(mixed[j], refs[i]), i
    assert st["completed"] == 2 * len(graphs)
    assert st["p50_us"] <= st["p99_us"] <= st["max_us"]


def test_matches_plain_decompose_on_batch_members():
    b = gg.batch(24, seed=31, nmin=1000, nmax=200_000)
    graphs = [b.graph(i) for i in range(b.num_graphs)]
    dev = torch.device("cuda:0")
    with kc().Server(hbm_budget_bytes=2 << 30) as s:
        outs = run_all(s, graphs)
    for g, out in zip(graphs, outs):
        plain = kc().decompose(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev))
        assert np.array_equal(plain.cpu().numpy(), out)
        assert np.array_equal(oracle.coreness(g.row_ptr, g.col_idx), out)


@pytest.mark.parametrize("tuning", [dict(round_renorm=1024), dict(round_renorm=1024, tail_round_cap=50),
                                    dict(round_renorm=1024, tail_order=1, tail_big=1)])
def test_round_numbers_renumbered_while_serving(tuning):
    # long chains keep the server running thousands of rounds; with a low renumbering threshold the
    # stamps and activity words are renumbered many times while graphs join and leave
    graphs = []
    for n in (20_000, 7_000, 30_000):
        graphs.append(gg.from_edges(n, np.arange(n - 1), np.arange(1, n)))
    graphs += [gg.chung_lu(50_000, 2.3, 12, seed=71), gg.lattice(120, 120, seed=72)]
    sizes = [3 + (i % 9) for i in range(2000)]
    n, edges = sg.onion(sizes)
    graphs.append(gg.Graph(*sg.to_csr(n, edges)))
    graphs = graphs * 2
    refs = [oracle.coreness(g.row_ptr, g.col_idx) for g in graphs]
    with kc().Server(hbm_budget_bytes=1 << 30, tuning=kc().Tuning(**tuning), rounds_per_step=8) as s:
        rng = np.random.default_rng(9)
        outs = run_all(s, graphs, gaps_s=rng.exponential(0.002, len(graphs)))
        st = s.stats()
    print(f"[serve] rebases={st['rebases']} rounds={st['rounds']} steps={st['steps']}", flush=True)
    assert st["rebases"] >= 2
    for g, out, ref in zip(graphs, outs, refs):
        assert np.array_equal(out, ref)


def test_budget_binds_admission():
    # room for about three of these graphs at a time: the rest wait for space
    graphs = [gg.chung_lu(100_000, 2.5, 12, seed=40 + i) for i in range(10)]
    fp = max(45 * (g.n + 1) + 8 * g.nnz for g in graphs)
    budget = 3 * fp + (1 << 20)
    with kc().Server(hbm_budget_bytes=budget, entries_per_vertex=12) as s:
        outs = run_all(s, graphs)
        st = s.stats()
    for g, out in zip(graphs, outs):
        assert np.array_equal(out, oracle.coreness(g.row_ptr, g.col_idx))
    assert st["bytes_peak"] <= budget
    assert st["completed"] == 10


def test_errors_too_large_again_invalid():
    KcoreError = kc().KcoreError
    n = 200_000
    path = gg.from_edges(n, np.arange(n - 1), np.arange(1, n))
    fp = 45 * (n + 1) + 8 * path.nnz
    with kc().Server(hbm_budget_bytes=fp + fp // 2, entries_per_vertex=2, max_queue=2) as s:
        big = gg.erdos_renyi(400_000, 800_000, seed=3)
        with pytest.raises(KcoreError) as ei:
            s.submit(big.row_ptr, big.col_idx, np.zeros(big.n, np.int32))
        assert ei.value.status == -4
        # one path at a time fits; the queue holds two: a burst of submissions must hit E_AGAIN
        accepted, outs, again = [], [], 0
        for _ in range(6):
            out = np.zeros(n, np.int32)
            try:
                accepted.append(s.submit(path.row_ptr, path.col_idx, out))
                outs.append(out)
            except KcoreError as e:
                assert e.status == -5
                again += 1
        assert again >= 1 and len(accepted) >= 2
        bad_rp = path.row_ptr.copy()
        bad_rp[0] = 1
        with pytest.raises(KcoreError) as ei:
            s.submit(bad_rp, path.col_idx, np.zeros(n, np.int32))
        assert ei.value.status == -1
        with pytest.raises(KcoreError) as ei:
            s.wait(987654321)
        assert ei.value.status == -1
        for rid in accepted:
            assert s.wait(rid, timeout_s=120).status == 0
        assert s.stats()["rejected"] >= again + 2
    for out in outs:
        assert (out == 1).all()


def test_wait_timeout_then_complete_and_poll():
    n = 200_000
    path = gg.from_edges(n, np.arange(n - 1), np.arange(1, n))
    with kc().Server(hbm_budget_bytes=256 << 20) as s:
        out = np.zeros(n, np.int32)
        rid = s.submit(path.row_ptr, path.col_idx, out)
        with pytest.raises(kc().KcoreError) as ei:
            s.wait(rid, timeout_s=1e-6)
        assert ei.value.status == -7
        assert s.wait(rid, timeout_s=120).status == 0
        assert (out == 1).all()
        # poll delivers each completion once
        small = [sg.to_csr(*sg.complete(5)) for _ in range(8)]
        outs = [np.zeros(5, np.int32) for _ in small]
        ids = {s.submit(rp, ci, o) for (rp, ci), o in zip(small, outs)}
        seen = set()
        t0 = time.time()
        while len(seen) < len(ids) and time.time() - t0 < 60:
            for c in s.poll():
                assert c.req_id not in seen and c.status == 0
                seen.add(c.req_id)
            time.sleep(0.001)
        assert seen == ids
        assert all((o == 4).all() for o in outs)
        empty_id = s.submit(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
        assert s.wait(empty_id, timeout_s=10).status == 0


def test_validation_mode_rejects_bad_csr(monkeypatch):
    monkeypatch.setenv("KCORE_VALIDATE", "1")
    with kc().Server(hbm_budget_bytes=64 << 20) as s:
        with pytest.raises(kc().KcoreError, match="symmetric"):
            s.submit(np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32), np.zeros(3, np.int32))
        with pytest.raises(kc().KcoreError, match="range"):
            s.submit(np.array([0, 1, 2], np.int64), np.array([5, 0], np.int32), np.zeros(2, np.int32))
        rp, ci = sg.to_csr(*sg.petersen())
        out = np.zeros(10, np.int32)
        assert s.wait(s.submit(rp, ci, out), timeout_s=30).status == 0
        assert (out == 3).all()


def test_shutdown_with_work_in_flight():
    graphs = [gg.chung_lu(200_000, 2.2, 16, seed=60 + i) for i in range(6)]
    s = kc().Server(hbm_budget_bytes=1 << 30)
    outs = [np.zeros(g.n, np.int32) for g in graphs]
    for g, o in zip(graphs, outs):
        s.submit(g.row_ptr, g.col_idx, o)
    t0 = time.time()
    s.close()
    assert time.time() - t0 < 60
